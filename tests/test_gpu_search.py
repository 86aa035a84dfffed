"""The registration's own correspondence search, checked at index level
through the C ABI (Sec. 3: correspondences come from nearest-neighbour
search; Eq. MLE_for_T pairs each source point with one map Gaussian).

* gicp_map_nearest runs the device search of the batched Gauss-Newton
  linearisation on arbitrary queries; its matches and FP32 keys must equal the
  oracle's exact (FP32 key, lower index) 1-NN with the r_max gate bit for bit,
  with or without a starting hint.
* The radius it certifies (the bound under which a registration keeps a
  match between iterations) must hold: a query moved by less than it keeps
  its nearest mean, by the oracle's exact search.
* GICP_FLAG_NO_REUSE (a fresh search for every point in every iteration)
  must leave every registration output bitwise unchanged."""
import numpy as np
import pytest

import synth
from oracle import covariance as oc
from oracle import gicp as og
from oracle import knn as ok
from oracle import se3

pytestmark = pytest.mark.gpu


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


def _soa(g, a):
    return g.to_soa(np.asarray(a, np.float32))


def _map(g, ctx, pts, cell, reg=1):
    cov = np.tile(np.array([1, 0, 0, 1, 0, 1e-3], np.float32), (pts.shape[0], 1))
    return ctx.map_build(_soa(g, pts), _soa(g, cov), cell=cell, reg_mode=reg)


def _hint_sets(rng, m, exact):
    nq = exact.shape[0]
    return {"answer": exact.astype(np.int32),
            "random": rng.integers(0, m, nq).astype(np.int32),
            "invalid": np.where(rng.random(nq) < 0.5, -1, m + 7).astype(np.int32)}


def _check_nearest(g, ctx, gm, mpts, q, r_max, seed=0, lanes=0):
    import torch
    ei, ek = ok.knn_bruteforce(mpts, q, 1, r_max=r_max)
    Q = _soa(g, q)
    idx, d2, rad = ctx.map_nearest(gm, Q, r_max, want_radius=True, lanes=lanes)
    assert (idx.cpu().numpy() == ei[:, 0]).all()
    assert (d2.cpu().numpy().view(np.uint32) == ek[:, 0].view(np.uint32)).all()
    rng = np.random.default_rng(seed)
    for name, h in _hint_sets(rng, mpts.shape[0], np.where(ei[:, 0] >= 0, ei[:, 0], 0)).items():
        hi, hd, _ = ctx.map_nearest(gm, Q, r_max, hints=torch.from_numpy(h).cuda(), lanes=lanes)
        assert (hi.cpu().numpy() == ei[:, 0]).all(), name
        assert (hd.cpu().numpy().view(np.uint32) == ek[:, 0].view(np.uint32)).all(), name
    return idx.cpu().numpy(), rad.cpu().numpy()


def _check_radius(mpts, q, idx, rad, seed, reps=4):
    """Queries moved by 0.999 of their certified radius keep their nearest
    mean (exact ungated FP32-key 1-NN over the whole map)."""
    sel = np.nonzero(rad > 0)[0]
    assert sel.size > 0
    rng = np.random.default_rng(seed)
    for _ in range(reps):
        d = rng.standard_normal((sel.size, 3))
        d /= np.linalg.norm(d, axis=1, keepdims=True)
        qq = (q[sel].astype(np.float64) + d * (0.999 * rad[sel, None].astype(np.float64))).astype(np.float32)
        ei, _ = ok.knn_bruteforce(mpts, qq, 1) if mpts.shape[0] * qq.shape[0] <= 4e8 else ok.knn_kdtree(mpts, qq, 1)
        assert (ei[:, 0] == idx[sel]).all()
    return sel.size


@pytest.mark.parametrize("lanes", [2, 4, 16])
@pytest.mark.parametrize("cell", [0.03, 0.1, 0.4])
def test_map_nearest_c1_bit_exact(g, ctx, cell, lanes):
    """C1 target as the map; the source at the identity and at the true pose
    (two lanes per query as in two-lane launches; four and sixteen as in the
    tracking launches)."""
    pr = synth.c1_problem()
    gm = _map(g, ctx, pr.tgt, cell)
    for k, T in enumerate((np.eye(4), pr.T_gt)):
        q = (pr.src.astype(np.float64) @ T[:3, :3].T + T[:3, 3]).astype(np.float32)
        _say("map_nearest_c1", cell, lanes, k)
        idx, rad = _check_nearest(g, ctx, gm, pr.tgt, q, 0.1, seed=k, lanes=lanes)
        assert 0.2 < (idx >= 0).mean() < 1.0
        _check_radius(pr.tgt, q, idx, rad, seed=10 + k)
    gm.close()


@pytest.mark.parametrize("r_max", [0.05, 0.2, 0.6])
def test_map_nearest_lattice_ties(g, ctx, r_max):
    """Map on an integer lattice with duplicates; queries on lattice points
    and midpoints (many exactly equal keys: the lower index wins)."""
    mp = synth.tiny_cloud(400, 3, duplicates=60, lattice=True)
    rng = np.random.default_rng(5)
    q = np.vstack([mp[rng.integers(0, mp.shape[0], 150)],
                   rng.integers(0, 12, (150, 3)).astype(np.float32) * np.float32(0.0625)]).astype(np.float32)
    for cell in (0.07, 0.125, 0.5):
        gm = _map(g, ctx, mp, cell, reg=0)
        for lanes in (2, 4, 8, 16):
            _say("map_nearest_ties", r_max, cell, lanes)
            _check_nearest(g, ctx, gm, mp, q, r_max, seed=int(100 * r_max), lanes=lanes)
        gm.close()


def test_map_nearest_far_and_empty(g, ctx):
    """Queries far outside the map (no match), a gate wider than the shells
    the search may visit (whole-map scan), and an empty query set."""
    pr = synth.c1_problem(n=3000)
    gm = _map(g, ctx, pr.tgt, 0.05)
    q = np.vstack([pr.src[:200], [[40, 0, 0], [0, -25, 3], [np.float32(1e3), 0, 0]]]).astype(np.float32)
    for lanes in (2, 4, 16):
        _say("map_nearest_far", lanes)
        _check_nearest(g, ctx, gm, pr.tgt, q, 0.1, lanes=lanes)
        _check_nearest(g, ctx, gm, pr.tgt, q, 5.0, lanes=lanes)
    with pytest.raises(g.GicpError):
        ctx.map_nearest(gm, _soa(g, q), 0.1, lanes=3)
    idx, d2, _ = ctx.map_nearest(gm, _soa(g, np.zeros((0, 3))), 0.1)
    assert idx.numel() == 0 and d2.numel() == 0
    gm.close()


def test_map_nearest_after_insert(g, ctx):
    """Indices of a grown map follow the insertion order; the hint table is
    rebuilt after an insertion."""
    import torch
    pr = synth.c1_problem(n=6000, room_seed=5)
    cov = np.tile(np.array([1, 0, 0, 1, 0, 1e-3], np.float32), (pr.tgt.shape[0], 1))
    gm = ctx.map_build(_soa(g, pr.tgt[:3500]), _soa(g, cov[:3500]), cell=0.1, reg_mode=1)
    q = pr.src
    ei, _ = ok.knn_bruteforce(pr.tgt[:3500], q, 1, r_max=0.1)
    h = torch.from_numpy(np.where(ei[:, 0] >= 0, ei[:, 0], 0).astype(np.int32)).cuda()
    a, _, _ = ctx.map_nearest(gm, _soa(g, q), 0.1, hints=h)
    assert (a.cpu().numpy() == ei[:, 0]).all()
    ctx.map_insert(gm, _soa(g, pr.tgt[3500:]), _soa(g, cov[3500:]))
    _check_nearest(g, ctx, gm, pr.tgt, q, 0.1)
    _check_nearest(g, ctx, gm, pr.tgt, q, 0.1, lanes=4)
    gm.close()


# ----------------------------------------------------------- no reuse: bitwise
def _same(a, b):
    return (np.array_equal(a.pose, b.pose) and np.array_equal(a.H, b.H) and np.array_equal(a.b, b.b)
            and a.iters == b.iters and a.n_inliers == b.n_inliers and a.cost == b.cost and a.status == b.status)


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_no_reuse_bitwise_c1(g, ctx, seed):
    pr = synth.c1_problem(room_seed=seed, src_seed=seed + 1, tgt_seed=seed + 2, tf_seed=seed + 3)
    src, tgt = _soa(g, pr.src), _soa(g, pr.tgt)
    tcov = ctx.covariances(tgt, 20, reg_mode=1, eps=1e-3)
    gm = ctx.map_build(tgt, tcov, cell=0.1)
    for lanes in (0, 4):
        for flags in (0, g.FLAG_MULTI_LAUNCH, g.FLAG_GRAPH, g.FLAG_QUEUE):
            _say("no_reuse_c1", seed, lanes, flags)
            a = ctx.register(src, gm, pr.init, g.params(max_it=30, flags=flags, lanes=lanes))
            b = ctx.register(src, gm, pr.init, g.params(max_it=30, flags=flags | g.FLAG_NO_REUSE, lanes=lanes))
            assert a.status == 0 and _same(a, b), (lanes, flags)
    gm.close()


def test_no_reuse_flag_changes_nothing_but_work(g, ctx):
    """The same registration with early exit (tracking parameters): equal
    outputs, and equal to the oracle within the pose bar."""
    pr = synth.c1_problem()
    src, tgt = _soa(g, pr.src), _soa(g, pr.tgt)
    tcov = ctx.covariances(tgt, 20, reg_mode=1, eps=1e-3)
    gm = ctx.map_build(tgt, tcov, cell=0.1)
    prm = dict(max_it=30, conv_rot=1e-6, conv_trans=1e-6)
    a = ctx.register(src, gm, pr.init, g.params(**prm))
    b = ctx.register(src, gm, pr.init, g.params(flags=g.FLAG_NO_REUSE, **prm))
    assert _same(a, b)
    o = og.register(pr.src, oc.covariances(pr.src, 20), pr.tgt, oc.covariances(pr.tgt, 20), pr.init, r_max=0.1,
                    max_it=30, conv_rot=1e-6, conv_trans=1e-6)
    dr, dt = se3.pose_error(a.pose, o.pose)
    assert dr < 1e-5 and dt < 1e-5
    gm.close()


def test_covariance_k_range(g, ctx):
    """k below 3 is rejected for covariances (rank 0 or 1); searches accept k = 1."""
    P = _soa(g, synth.tiny_cloud(50, 1))
    for k in (1, 2):
        with pytest.raises(g.GicpError):
            ctx.covariances(P, k)
    pr = synth.c1_problem(n=300)
    gm = _map(g, ctx, pr.tgt, 0.1)
    with pytest.raises(g.GicpError):
        ctx.register(_soa(g, pr.src), gm, np.eye(4), g.params(k=2))
    gm.close()
    idx, _ = ctx.knn(P, P, 1)
    assert (idx.cpu().numpy()[:, 0] >= 0).all()
