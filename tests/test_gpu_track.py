"""gicp_track (sequential frame-to-map tracking with on-device pose
prediction) through the C ABI, on small sequences: against the oracle's
tracking loop, against per-frame gicp_register calls from the same initial
poses, graph-replayed against launched form, and its error paths."""
import numpy as np
import pytest

import synth
from oracle import covariance as oc
from oracle import se3
from oracle import tracking as ot

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


def _sequence(n_frames=8, seed=3):
    """A room map (6000 points, plane covariances) and frames that are
    independent noisy resamples of it seen from a smooth random walk."""
    room = synth.make_room(seed)
    mp, _ = synth.sample_surface(room, 6000, seed + 1, 0.001)
    mp = mp.astype(np.float32)
    mc = oc.covariances(mp, 20).astype(np.float32)
    rng = np.random.default_rng(seed + 2)
    poses = [np.eye(4)]
    for _ in range(n_frames - 1):
        poses.append(poses[-1] @ synth.random_offset(rng, 1.0, 0.01))
    frames = []
    for i, T in enumerate(poses):
        p, _ = synth.sample_surface(room, 3000, 100 * seed + i, 0.002)
        frames.append(((p - T[:3, 3]) @ T[:3, :3]).astype(np.float32))
    return mp, mc, frames, poses


PRM = dict(k=20, eps=1e-3, r_max=0.1, max_it=30, conv_rot=1e-6, conv_trans=1e-6, reg_mode=1)


@pytest.mark.parametrize("motion", [0, 1])
def test_track_vs_oracle(env, motion):
    g, ctx = env
    mp, mc, frames, poses = _sequence()
    gm = ctx.map_build(g.to_soa(mp), g.to_soa(mc), cell=0.1)
    _say("track vs oracle", motion)
    res = ctx.track([g.to_soa(f) for f in frames], gm, poses[0], motion=motion, prm=g.params(**PRM))
    est, _, ores = ot.track(frames, mp, mc, poses[0], motion=motion, max_it=30)
    for i, (r, E) in enumerate(zip(res, est)):
        dr, dt = se3.pose_error(r.pose, E)
        _say(f"  frame {i}: rot {dr:.2e} trans {dt:.2e} it {r.iters}/{ores[i].iters}")
        assert r.status == 0 and dr < 1e-5 and dt < 1e-5
    gm.close()


@pytest.mark.parametrize("motion", [0, 1])
def test_track_equals_register_from_same_inits(env, motion):
    """Every frame of the tracked sequence against gicp_register started from
    the pose the host predicts from the tracked estimates (the first frame
    bitwise); the iteration-slot (default), launched and graph-replayed forms
    bitwise equal."""
    g, ctx = env
    mp, mc, frames, poses = _sequence(seed=5)
    gm = ctx.map_build(g.to_soa(mp), g.to_soa(mc), cell=0.1)
    F = [g.to_soa(f) for f in frames]
    cell = ctx.estimate_cell(F[0], 20)
    prm = g.params(cell_src=cell, **PRM)
    res = ctx.track(F, gm, poses[0], motion=motion, prm=prm)
    res_l = ctx.track(F, gm, poses[0], motion=motion,
                      prm=g.params(cell_src=cell, flags=g.FLAG_MULTI_LAUNCH, **PRM))
    res_g = ctx.track(F, gm, poses[0], motion=motion, prm=g.params(cell_src=cell, flags=g.FLAG_GRAPH, **PRM))
    est = [r.pose for r in res]
    for i in range(len(F)):
        _say("track vs register", motion, i)
        for other in (res_l, res_g):
            assert np.array_equal(other[i].pose, res[i].pose) and np.array_equal(other[i].H, res[i].H)
            assert other[i].iters == res[i].iters and other[i].status == res[i].status
        r = ctx.register(F[i], gm, ot.predict(est, i, poses[0], motion), prm)
        if i == 0:
            assert np.array_equal(r.pose, res[0].pose) and np.array_equal(r.H, res[0].H)
        dr, dt = se3.pose_error(r.pose, res[i].pose)
        assert dr < 1e-5 and dt < 1e-5, (i, dr, dt)
    gm.close()


def test_track_failure_and_args(env):
    """A frame with no correspondence (moved 20 m away in its own frame)
    reports NO_CORR and keeps its initial pose; the frames after it keep
    tracking from the prediction.  Invalid motion models and forms are refused."""
    g, ctx = env
    mp, mc, frames, poses = _sequence(n_frames=5, seed=7)
    gm = ctx.map_build(g.to_soa(mp), g.to_soa(mc), cell=0.1)
    bad = frames[2] + np.float32(20.0)
    F = [g.to_soa(f) for f in frames[:2]] + [g.to_soa(bad)] + [g.to_soa(f) for f in frames[3:]]
    res = ctx.track(F, gm, poses[0], motion=0, prm=g.params(**PRM))
    assert [r.status for r in res] == [0, 0, 3, 0, 0]
    assert np.array_equal(res[2].pose, res[1].pose)
    dr, dt = se3.pose_error(res[4].pose, poses[4])
    assert dt < 5e-3
    with pytest.raises(g.GicpError):
        ctx.track(F, gm, poses[0], motion=7, prm=g.params(**PRM))
    with pytest.raises(g.GicpError):
        ctx.track(F, gm, poses[0], prm=g.params(flags=g.FLAG_QUEUE, **PRM))
    for flags in (g.FLAG_MULTI_LAUNCH, g.FLAG_GRAPH):
        other = ctx.track(F, gm, poses[0], motion=0, prm=g.params(flags=flags, **PRM))
        assert all(np.array_equal(a.pose, b.pose) and a.status == b.status for a, b in zip(res, other))
    gm.close()


def test_track_max_it_zero_and_single_frame(env):
    """max_it = 0: every frame keeps its predicted pose (the first its given
    pose); a one-frame sequence equals gicp_register."""
    g, ctx = env
    mp, mc, frames, poses = _sequence(n_frames=4, seed=9)
    gm = ctx.map_build(g.to_soa(mp), g.to_soa(mc), cell=0.1)
    F = [g.to_soa(f) for f in frames]
    res = ctx.track(F, gm, poses[1], motion=1, prm=g.params(**dict(PRM, max_it=0)))
    assert all(r.iters == 0 and r.status == 0 for r in res)
    # (constant velocity from two equal poses is the identity motion, up to FP64 rounding)
    assert np.array_equal(res[0].pose, poses[1]) and np.array_equal(res[1].pose, poses[1])
    assert all(np.allclose(r.pose, poses[1], atol=1e-12) for r in res)
    one = ctx.track(F[:1], gm, poses[0], motion=0, prm=g.params(**PRM))
    reg = ctx.register(F[0], gm, poses[0], g.params(**PRM))
    assert np.array_equal(one[0].pose, reg.pose) and np.array_equal(one[0].H, reg.H)
    gm.close()
