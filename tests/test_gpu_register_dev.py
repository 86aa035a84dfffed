"""gicp_register_dev (device-resident initial pose and outputs, no host
synchronisation) through the C ABI: bitwise equal to gicp_register in every
accepted form, and captured in a HIP graph whose replays, from initial poses
written on the device between them, each match the eager call."""
import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu


def _say(*a):
    print("[case]", *a, flush=True)


@pytest.fixture(scope="module")
def env():
    import torch

    import paper_2403_12550_amd as g
    torch.cuda.set_device(0)
    ctx = g.Context(0)
    yield g, ctx
    ctx.close()


def _problem(g, ctx, seed):
    pr = synth.c1_problem(room_seed=seed, src_seed=seed + 1, tgt_seed=seed + 2, tf_seed=seed + 3)
    src, tgt = g.to_soa(pr.src), g.to_soa(pr.tgt)
    tcov = ctx.covariances(tgt, 20, reg_mode=1, eps=1e-3)
    return pr, src, ctx.map_build(tgt, tcov, cell=0.1)


def _buffers():
    import torch
    f64 = dict(dtype=torch.float64, device="cuda")
    return (torch.zeros(16, **f64), torch.zeros(16, **f64), torch.zeros(36, **f64), torch.zeros(6, **f64),
            torch.zeros(64, dtype=torch.uint8, device="cuda"))


def _check_equal(g, ctx, r, pose, H, b, stats):
    assert np.array_equal(pose.cpu().numpy().reshape(4, 4), r.pose)
    assert np.array_equal(H.cpu().numpy().reshape(6, 6), r.H)
    assert np.array_equal(b.cpu().numpy(), r.b)
    st = ctx.stats_from_bytes(stats.cpu().numpy())
    assert st["iters"] == r.iters and st["n_inliers"] == r.n_inliers and st["status"] == r.status
    assert st["cost"] == r.cost and bool(st["converged"]) == r.converged


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_register_dev_equals_register(env, seed):
    import torch
    g, ctx = env
    pr, src, gm = _problem(g, ctx, seed)
    init, pose, H, b, stats = _buffers()
    init.copy_(torch.from_numpy(pr.init.ravel()))
    for flags in (0, g.FLAG_MULTI_LAUNCH, g.FLAG_QUEUE):
        _say("register_dev", seed, flags)
        prm = g.params(max_it=30, conv_rot=1e-6, conv_trans=1e-6, flags=flags)
        ctx.register_dev(src, gm, init, pose, H, b, prm, stats=stats)
        r = ctx.register(src, gm, pr.init, prm)
        _check_equal(g, ctx, r, pose, H, b, stats)
    with pytest.raises(g.GicpError):
        ctx.register_dev(src, gm, init, pose, H, b, g.params(flags=g.FLAG_GRAPH))
    gm.close()


def test_register_dev_graph_capture(env):
    """One registration (source covariances included) captured in a graph;
    five replays from different device-written initial poses, each checked
    against an eager gicp_register run between the replays."""
    import torch
    g, ctx = env
    pr, src, gm = _problem(g, ctx, 4)
    init, pose, H, b, stats = _buffers()
    cell = ctx.estimate_cell(src, 20)
    prm = g.params(max_it=30, conv_rot=1e-6, conv_trans=1e-6, cell_src=cell)
    init.copy_(torch.from_numpy(np.eye(4).ravel()))
    ctx.register_dev(src, gm, init, pose, H, b, prm, stats=stats)   # sizes the workspaces
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    cs = torch.cuda.Stream()
    with torch.cuda.graph(graph, stream=cs):
        ctx.register_dev(src, gm, init, pose, H, b, prm, stats=stats)
    torch.cuda.synchronize()
    rng = np.random.default_rng(11)
    for k in range(5):
        T0 = synth.random_offset(rng, 2.0, 0.03)
        init.copy_(torch.from_numpy(T0.ravel()))
        graph.replay()
        torch.cuda.synchronize()
        got = (pose.clone(), H.clone(), b.clone(), stats.clone())
        r = ctx.register(src, gm, T0, prm)
        _say("replay", k, r.iters, r.status)
        _check_equal(g, ctx, r, *got)
    gm.close()
