"""Parity at the full tracking sizes, through the C ABI: 60k-point frames
against a 1M-Gaussian map, and the 64-problem batch (sources 2k-200k points,
targets 0.1M-1M Gaussians).  The HIP path runs in the launch configuration the
benchmark times (50 frames per batched call with graph-replayed iterations; all
64 problems in one call); the oracle computes sampled outputs one by one.

Bars as at the small sizes: neighbour indices and FP32 keys bit-exact;
covariances within 1e-5 relative (Frobenius) where the normal is determined;
poses within 1e-5 rad and 1e-5 m of the FP64 oracle."""
import numpy as np
import pytest

import synth
from oracle import covariance as oc
from oracle import gicp as og
from oracle import knn as ok
from oracle import se3

import covcheck

pytestmark = pytest.mark.gpu

GAP_GATE = 0.02          # relative eigen-gap above which the normal is determined in FP32
BATCH = 50               # frames per batched call, as timed
ORACLE_FRAMES = (0, 23, 49)
R_MAX, MAX_IT, CONV = 0.1, 20, 1e-6


def _say(*a):
    print("[case]", *a, flush=True)


@pytest.fixture(scope="module")
def g():
    import paper_2403_12550_amd as g
    g.lib()
    return g


@pytest.fixture(scope="module")
def ctx(g):
    import torch
    torch.cuda.set_device(0)
    c = g.Context(0)
    yield c
    c.close()


@pytest.fixture(scope="module")
def c2(g, ctx):
    """The tracking sequence (1M-Gaussian map), its first BATCH frames on the
    device and the map built as the benchmark builds it."""
    import torch
    _say("c2 workload")
    # (the frames were rendered at collection time, before the GPU was initialised)
    seq = synth.c2_sequence(n_frames=100, map_size=1_000_000)
    frames = [g.to_soa(seq.frame(i)) for i in range(BATCH)]
    gm = ctx.map_build(g.to_soa(seq.map_means), g.to_soa(seq.map_cov_raw), cell=0.03, reg_mode=g.REG_PLANE,
                       eps=1e-3)
    torch.cuda.synchronize()
    yield seq, frames, gm
    gm.close()


def _init(seq, i):
    """Constant-velocity prediction from the two previous ground-truth poses."""
    if i == 0:
        return seq.poses[0].copy()
    if i == 1:
        return seq.poses[0].copy()
    a, b = seq.poses[i - 2], seq.poses[i - 1]
    ai = np.eye(4)
    ai[:3, :3] = a[:3, :3].T
    ai[:3, 3] = -a[:3, :3].T @ a[:3, 3]
    return b @ (ai @ b)


def _sample(n, m, seed):
    return np.sort(np.random.default_rng(seed).choice(n, size=min(n, m), replace=False))


def test_c2_frame_self_knn_sampled(g, ctx, c2):
    """k = 20 self-neighbours of a whole 60k frame; 3000 sampled rows against
    the oracle's exact (FP32 key, index) search."""
    seq, frames, _ = c2
    p = seq.frame(23)
    _say("c2 self knn", p.shape[0])
    idx, d2 = ctx.knn(frames[23], frames[23], 20)
    s = _sample(p.shape[0], 3000, 1)
    ei, ek = ok.knn_kdtree(p, p[s], 20)
    assert (idx.cpu().numpy()[s] == ei).all()
    assert (d2.cpu().numpy()[s].view(np.uint32) == ek.view(np.uint32)).all()


def test_c2_frame_to_map_nearest_sampled(g, ctx, c2):
    """Nearest map mean within r_max of every point of a frame at its true pose
    (the correspondence gate) against the 1M-point map; 5000 sampled rows."""
    seq, _, _ = c2
    p = seq.frame(49)
    T = seq.poses[49]
    q = (p.astype(np.float64) @ T[:3, :3].T + T[:3, 3]).astype(np.float32)
    _say("c2 frame-to-map nearest", q.shape[0])
    idx, d2 = ctx.knn(g.to_soa(seq.map_means), g.to_soa(q), 1, r_max=R_MAX)
    s = _sample(q.shape[0], 5000, 2)
    ei, ek = ok.knn_kdtree(seq.map_means, q[s], 1)
    gate = np.float32(np.float32(R_MAX) * np.float32(R_MAX))
    far = ek[:, 0] > gate
    ei[far, 0] = ok.INT_SENTINEL
    ek[far, 0] = np.inf
    assert far.mean() < 0.5
    assert (idx.cpu().numpy()[s] == ei).all()
    assert (d2.cpu().numpy()[s].view(np.uint32) == ek.view(np.uint32)).all()


@pytest.mark.parametrize("lanes", [2, 4])
@pytest.mark.parametrize("offset", [False, True])
def test_c2_map_nearest_sampled(g, ctx, c2, offset, lanes):
    """The registration's own correspondence search (gicp_map_nearest) for a
    whole frame against the 1M-Gaussian map handle, at the true pose and at a
    pose 5 cm / 2 deg off; 5000 sampled rows bit-exact against the oracle's
    gated (FP32 key, index) 1-NN, without and with hints; the certified radius
    of 2000 sampled rows holds under displacement."""
    import torch
    seq, _, gm = c2
    p = seq.frame(49)
    T = seq.poses[49]
    if offset:
        T = T @ synth.random_offset(np.random.default_rng(7), 2.0, 0.05, exact=True)
    q = (p.astype(np.float64) @ T[:3, :3].T + T[:3, 3]).astype(np.float32)
    _say("c2 map_nearest", q.shape[0], offset, lanes)
    Q = g.to_soa(q)
    idx, d2, rad = ctx.map_nearest(gm, Q, R_MAX, want_radius=True, lanes=lanes)
    s = _sample(q.shape[0], 5000, 4)
    ei, ek = ok.knn_kdtree(seq.map_means, q[s], 1)
    gate = np.float32(np.float32(R_MAX) * np.float32(R_MAX))
    far = ek[:, 0] > gate
    ei[far, 0] = ok.INT_SENTINEL
    ek[far, 0] = np.inf
    assert (idx.cpu().numpy()[s] == ei[:, 0]).all()
    assert (d2.cpu().numpy()[s].view(np.uint32) == ek[:, 0].view(np.uint32)).all()
    full = idx.cpu().numpy()
    rng = np.random.default_rng(8)
    for name, h in (("previous", np.where(full >= 0, full, -1)),
                    ("random", rng.integers(0, gm.m, q.shape[0])),
                    ("invalid", np.full(q.shape[0], gm.m + 1))):
        hi, hd, _ = ctx.map_nearest(gm, Q, R_MAX, hints=torch.from_numpy(h.astype(np.int32)).cuda(), lanes=lanes)
        assert (hi.cpu().numpy() == full).all(), name
        assert (hd.cpu().numpy().view(np.uint32) == d2.cpu().numpy().view(np.uint32)).all(), name
    r = rad.cpu().numpy()
    s2 = _sample(q.shape[0], 2000, 5)
    s2 = s2[r[s2] > 0]
    assert s2.size > 500
    d = rng.standard_normal((s2.size, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    qq = (q[s2].astype(np.float64) + d * (0.999 * r[s2, None].astype(np.float64))).astype(np.float32)
    mi, _ = ok.knn_kdtree(seq.map_means, qq, 1)
    assert (mi[:, 0] == full[s2]).all()


def test_c2_no_reuse_bitwise(g, ctx, c2):
    """50 frames in the timed (graph-replayed batched) form, with and without
    a fresh search for every point in every iteration: identical outputs."""
    seq, frames, gm = c2
    src_cell = ctx.estimate_cell(frames[0], 20)
    items = [(frames[i], None, gm, _init(seq, i)) for i in range(BATCH)]
    out = []
    for flags in (g.FLAG_GRAPH, g.FLAG_GRAPH | g.FLAG_NO_REUSE):
        _say("c2 no_reuse", flags)
        prm = g.params(k=20, eps=1e-3, r_max=R_MAX, max_it=MAX_IT, conv_rot=CONV, conv_trans=CONV,
                       reg_mode=g.REG_PLANE, cell_src=src_cell, flags=flags)
        out.append(ctx.register_batch(items, prm))
    for a, b in zip(*out):
        assert a.status == 0 and np.array_equal(a.pose, b.pose) and np.array_equal(a.H, b.H)
        assert np.array_equal(a.b, b.b) and a.iters == b.iters and a.n_inliers == b.n_inliers


@pytest.mark.parametrize("mode", [1, 2])
def test_c2_frame_covariances_sampled(g, ctx, c2, mode):
    """Plane- and ellipse-regularised k = 20 covariances of a whole frame; 3000
    sampled rows against the oracle's neighbourhood covariance and
    regularisation, every sampled row checked (tests/covcheck.py)."""
    seq, frames, _ = c2
    p = seq.frame(0)
    _say("c2 covariances", p.shape[0], mode)
    got = ctx.covariances(frames[0], 20, reg_mode=mode, eps=1e-3).cpu().numpy().T.astype(np.float64)
    s = _sample(p.shape[0], 3000, 3)
    nbr, _ = ok.knn_kdtree(p, p[s], 20)
    Craw = oc.neighbourhood_covariance(p, nbr)
    if mode == 1:
        stats = covcheck.check_plane(got[s], Craw)
        assert stats[1] > 0.9
    else:
        stats = covcheck.check_ellipse(got[s], Craw)
    _say("  ", stats)


def test_c2_batched_graph_poses_vs_oracle(g, ctx, c2):
    """50 frames in one batched call with graph-replayed iterations (the timed
    form); three of them registered by the oracle from the same initial poses."""
    seq, frames, gm = c2
    src_cell = ctx.estimate_cell(frames[0], 20)
    prm = g.params(k=20, eps=1e-3, r_max=R_MAX, max_it=MAX_IT, conv_rot=CONV, conv_trans=CONV,
                   reg_mode=g.REG_PLANE, cell_src=src_cell, flags=g.FLAG_GRAPH)
    _say("c2 batched graph", BATCH)
    res = ctx.register_batch([(frames[i], None, gm, _init(seq, i)) for i in range(BATCH)], prm)
    assert all(r.status == 0 and r.converged for r in res)
    map_cov = oc.regularise6(seq.map_cov_raw, oc.REG_PLANE, 1e-3)
    from scipy.spatial import cKDTree
    tree = cKDTree(seq.map_means.astype(np.float64))
    for i in ORACLE_FRAMES:
        src = seq.frame(i)
        cs = oc.covariances(src, 20, oc.REG_PLANE, 1e-3)
        o = og.register(src, cs, seq.map_means, map_cov, _init(seq, i), r_max=R_MAX, max_it=MAX_IT,
                        conv_rot=CONV, conv_trans=CONV, tree=tree)
        dr, dt = se3.pose_error(res[i].pose, o.pose)
        _say(f"  frame {i}: rot {dr:.2e} trans {dt:.2e} it {res[i].iters}/{o.iters} "
             f"inl {res[i].n_inliers}/{o.n_inliers}")
        assert dr < 1e-5 and dt < 1e-5
        assert abs(res[i].n_inliers - o.n_inliers) <= 3


@pytest.fixture(scope="module")
def c4(g, ctx):
    import torch
    _say("c4 workload")
    probs = synth.c4_batch(n_prob=64)
    maps = [ctx.map_build(g.to_soa(p.tgt), g.to_soa(p.tgt_cov_raw), cell=0.0, reg_mode=g.REG_PLANE)
            for p in probs]
    items = [(g.to_soa(p.src), None, gm, p.init) for p, gm in zip(probs, maps)]
    torch.cuda.synchronize()
    yield probs, items
    for gm in maps:
        gm.close()


@pytest.mark.parametrize("form", ["batched", "queue"])
def test_c4_batch_sampled_vs_oracle(g, ctx, c4, form):
    """All 64 problems in one call; the largest and the smallest source and
    the largest target registered by the oracle."""
    probs, items = c4
    flags = {"batched": 0, "queue": g.FLAG_QUEUE}[form]
    prm = g.params(k=20, eps=1e-3, r_max=0.1, max_it=30, conv_rot=CONV, conv_trans=CONV,
                   reg_mode=g.REG_PLANE, flags=flags)
    _say("c4", form)
    res = ctx.register_batch(items, prm)
    assert all(r.status == 0 for r in res)
    ns = [p.src.shape[0] for p in probs]
    ms = [p.tgt.shape[0] for p in probs]
    for i in sorted({int(np.argmax(ns)), int(np.argmin(ns)), int(np.argmax(ms))}):
        p = probs[i]
        o = _c4_oracle(p)
        dr, dt = se3.pose_error(res[i].pose, o.pose)
        _say(f"  problem {i} ({p.src.shape[0]} pts vs {p.tgt.shape[0]}): rot {dr:.2e} trans {dt:.2e} "
             f"it {res[i].iters}/{o.iters}")
        assert dr < 1e-5 and dt < 1e-5


_C4_ORACLE = {}


def _c4_oracle(p):
    key = p.seed
    if key not in _C4_ORACLE:
        cs = oc.covariances(p.src, 20, oc.REG_PLANE, 1e-3)
        ct = oc.regularise6(p.tgt_cov_raw, oc.REG_PLANE, 1e-3)
        _C4_ORACLE[key] = og.register(p.src, cs, p.tgt, ct, p.init, r_max=0.1, max_it=30, conv_rot=CONV,
                                      conv_trans=CONV)
    return _C4_ORACLE[key]


def test_c4_no_reuse_bitwise(g, ctx, c4):
    """All 64 problems in one batched call, with and without a fresh search
    for every point in every iteration: identical outputs."""
    _, items = c4
    out = []
    for flags in (0, g.FLAG_NO_REUSE):
        _say("c4 no_reuse", flags)
        prm = g.params(k=20, eps=1e-3, r_max=0.1, max_it=30, conv_rot=CONV, conv_trans=CONV,
                       reg_mode=g.REG_PLANE, flags=flags)
        out.append(ctx.register_batch(items, prm))
    for a, b in zip(*out):
        assert a.status == 0 and np.array_equal(a.pose, b.pose) and np.array_equal(a.H, b.H)
        assert np.array_equal(a.b, b.b) and a.iters == b.iters and a.n_inliers == b.n_inliers


@pytest.mark.parametrize("motion", [0, 1])
def test_c2_track_closed_loop_vs_oracle(g, ctx, c2, motion):
    """The first 12 frames tracked in one gicp_track call (iteration slots, the
    timed form), each frame from the pose predicted from its own previous
    estimates, against the oracle's tracking loop with the same motion model;
    the graph-replayed form bitwise equal (frames of 1,000+ work items: the
    slots' two-level hand-over of partials with groups of 30+ members)."""
    from scipy.spatial import cKDTree

    from oracle import tracking as ot
    seq, frames, gm = c2
    n = 12
    src_cell = ctx.estimate_cell(frames[0], 20)
    prm = g.params(k=20, eps=1e-3, r_max=R_MAX, max_it=MAX_IT, conv_rot=CONV, conv_trans=CONV,
                   reg_mode=g.REG_PLANE, cell_src=src_cell)
    _say("c2 track", motion)
    res = ctx.track(frames[:n], gm, seq.poses[0], motion=motion, prm=prm)
    assert all(r.status == 0 for r in res)
    prm.flags = g.FLAG_GRAPH
    res_g = ctx.track(frames[:n], gm, seq.poses[0], motion=motion, prm=prm)
    for a, b in zip(res, res_g):
        assert np.array_equal(a.pose, b.pose) and np.array_equal(a.H, b.H) and np.array_equal(a.b, b.b)
        assert a.iters == b.iters and a.status == b.status
    map_cov = oc.regularise6(seq.map_cov_raw, oc.REG_PLANE, 1e-3)
    tree = cKDTree(seq.map_means.astype(np.float64))
    est, _, ores = ot.track([seq.frame(i) for i in range(n)], seq.map_means, map_cov, seq.poses[0],
                            motion=motion, r_max=R_MAX, max_it=MAX_IT, conv=CONV, tree=tree)
    for i in range(n):
        dr, dt = se3.pose_error(res[i].pose, est[i])
        _say(f"  frame {i}: rot {dr:.2e} trans {dt:.2e} it {res[i].iters}/{ores[i].iters}")
        assert dr < 1e-5 and dt < 1e-5
