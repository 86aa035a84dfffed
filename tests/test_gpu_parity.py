"""GPU parity of the HIP path against the FP64 oracle, through the C ABI.

Bars: neighbour indices and FP32 keys bit-exact; covariances within 1e-5
relative (Frobenius) where the normal is determined; poses within 1e-5 rad and
1e-5 m."""
import numpy as np
import pytest

import synth
from oracle import covariance as oc
from oracle import gicp as og
from oracle import knn as ok
from oracle import se3

import covcheck

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


# ----------------------------------------------------------------------------- k-NN
@pytest.mark.parametrize("cell", [0.0, 0.08, 0.35, 1.5])
def test_self_knn_c1_bit_exact(g, ctx, cell):
    _say("self_knn_c1", cell)
    p = synth.c1_problem().src
    P = _soa(g, p)
    idx, d2 = ctx.knn(P, P, 20, cell=cell)
    ei, ek = ok.knn_bruteforce(p, p, 20)
    assert (idx.cpu().numpy() == ei).all()
    assert (d2.cpu().numpy().view(np.uint32) == ek.view(np.uint32)).all()


@pytest.mark.parametrize("seed,lattice,dups,n,k", [
    (0, False, 0, 40, 7), (1, True, 0, 64, 20), (2, False, 13, 50, 20), (3, True, 40, 120, 20),
    (4, True, 0, 200, 5), (5, False, 0, 23, 20), (6, True, 64, 64, 64), (7, False, 3, 300, 33)])
def test_knn_ties_and_duplicates(g, ctx, seed, lattice, dups, n, k):
    _say("knn_ties", seed, lattice, dups, n, k)
    p = synth.tiny_cloud(n, seed, duplicates=dups, lattice=lattice)
    P = _soa(g, p)
    for cell in (0.0, 0.05, 0.3):
        idx, d2 = ctx.knn(P, P, k, cell=cell)
        ei, ek = ok.knn_bruteforce(p, p, k)
        assert (idx.cpu().numpy() == ei).all(), cell
        assert (d2.cpu().numpy().view(np.uint32) == ek.view(np.uint32)).all(), cell


@pytest.mark.parametrize("n", [1, 2, 19, 20, 255, 256, 257, 4095, 4096, 4097, 9000])
def test_knn_ragged_sizes(g, ctx, n):
    _say("knn_ragged", n)
    rng = np.random.default_rng(n)
    p = rng.uniform(-2, 2, (n, 3)).astype(np.float32)
    q = rng.uniform(-2.5, 2.5, (min(n, 700) + 3, 3)).astype(np.float32)
    k = min(20, n)
    idx, d2 = ctx.knn(_soa(g, p), _soa(g, q), k, cell=0.0)
    ei, ek = ok.knn_bruteforce(p, q, k)
    assert (idx.cpu().numpy() == ei).all()
    assert (d2.cpu().numpy().view(np.uint32) == ek.view(np.uint32)).all()


def test_knn_far_queries_full_scan(g, ctx):
    """Queries far outside the cloud exhaust the grid shells and fall back to
    the full scan, which must still be exact."""
    _say("knn_far")
    rng = np.random.default_rng(9)
    p = rng.uniform(0, 1, (3000, 3)).astype(np.float32)
    q = np.array([[5, 5, 5], [-3, 0.5, 0.5], [0.5, 0.5, 40.0], [0.2, 0.3, 0.4]], np.float32)
    idx, d2 = ctx.knn(_soa(g, p), _soa(g, q), 10, cell=0.05)
    ei, ek = ok.knn_bruteforce(p, q, 10)
    assert (idx.cpu().numpy() == ei).all()
    assert (d2.cpu().numpy().view(np.uint32) == ek.view(np.uint32)).all()


@pytest.mark.parametrize("r_max", [0.05, 0.1, 0.3])
def test_knn_gate(g, ctx, r_max):
    _say("knn_gate", r_max)
    pr = synth.c1_problem()
    p, q = pr.tgt, pr.src[:1500]
    idx, d2 = ctx.knn(_soa(g, p), _soa(g, q), 8, cell=0.0, r_max=r_max)
    ei, ek = ok.knn_bruteforce(p, q, 8, r_max=r_max)
    assert (idx.cpu().numpy() == ei).all()
    got = d2.cpu().numpy()
    assert (got.view(np.uint32) == ek.view(np.uint32)).all()


def test_knn_arg_errors(g, ctx):
    import torch
    P = _soa(g, np.zeros((10, 3)))
    with pytest.raises(g.GicpError):
        ctx.knn(P, P, 0)
    with pytest.raises(g.GicpError):
        ctx.knn(P, P, 65)
    with pytest.raises(ValueError):
        ctx.knn(P.double(), P, 3)
    del torch


# ----------------------------------------------------------------------- covariances
def _rel_frob(A6, B6):
    A, B = oc.from6(A6), oc.from6(B6)
    return np.linalg.norm(A - B, axis=(1, 2)) / np.linalg.norm(B, axis=(1, 2))


# Relative eigen-gap above which the normal is well determined in FP32 (see
# the derivation of the covariance tolerance): covariance entries carry an
# absolute error of order 20 * 2^-24 * |C|, which tilts the normal by that
# over the gap; at a gap of 0.02 this stays below 1e-5.
GAP_GATE = 0.02


@pytest.mark.parametrize("seed", [0, 1])
@pytest.mark.parametrize("mode", [0, 1, 2])
def test_covariances_c1(g, ctx, mode, seed):
    """Every point checked: raw covariances within 1e-5; plane forms within
    1e-5 where the normal is determined and with a normal in the near-null
    space elsewhere; ellipse forms within their derived per-point bound
    (tests/covcheck.py)."""
    _say("cov_c1", mode, seed)
    p = synth.c1_problem(src_seed=1 + 10 * seed).src
    got = ctx.covariances(_soa(g, p), 20, cell=0.0, reg_mode=mode, eps=1e-3).cpu().numpy().T.astype(np.float64)
    exp, Craw, _ = oc.covariances(p, 20, mode, 1e-3, return_raw=True)
    if mode == oc.REG_NONE:
        err = _rel_frob(got, exp)
        assert err.max() < 1e-5, err.max()
    elif mode == oc.REG_PLANE:
        _say("  plane", covcheck.check_plane(got, Craw))
    else:
        _say("  ellipse", covcheck.check_ellipse(got, Craw))
    lam = np.linalg.eigvalsh(oc.from6(got))
    assert lam.min() > -1e-6 * np.abs(lam).max()


def test_covariances_ellipse_degenerate_fixture(g, ctx):
    """Collinear, coincident and needle-shaped neighbourhoods (the hand-derived
    fixture of the ellipse form's clamp): every point of each cloud has the
    whole cloud as its neighbourhood."""
    import json
    import os
    d = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "cov_ellipse_degenerate.json")))
    for name in ("collinear", "coincident", "thin_needle"):
        case = d[name]
        pts = np.asarray(case["points"], np.float32)
        got = ctx.covariances(_soa(g, pts), case["k"], cell=0.0, reg_mode=2).cpu().numpy().T.astype(np.float64)
        exp = np.asarray(case["expected_cov6_ellipse_each"], np.float64)
        scale = max(1.0, np.abs(exp).max())
        _say("ellipse fixture", name, np.abs(got - exp).max() / scale)
        assert np.abs(got - exp).max() <= 1e-5 * scale, name


@pytest.mark.parametrize("cell", [0.05, 0.2, 0.6])
def test_covariances_cell_independent(g, ctx, cell):
    """Exactness of the neighbour sets does not depend on the grid cell size."""
    _say("cov_cells", cell)
    p = synth.c1_problem(n=3000).src
    P = _soa(g, p)
    a = ctx.covariances(P, 20, cell=cell, reg_mode=0).cpu().numpy()
    b = ctx.covariances(P, 20, cell=0.0, reg_mode=0).cpu().numpy()
    assert (a.view(np.uint32) == b.view(np.uint32)).all()


def test_covariances_isolated_points_overflow(g, ctx):
    """A few points far from a dense patch: their 20-NN radius exceeds the
    searched grid shells, so they are finished by the overflow pass (a
    workgroup-wide full scan); indices stay bit-exact and covariances match."""
    _say("cov_overflow")
    p, _ = synth.planar_patch(3000, 4, normal=(0.2, 0.1, 1.0))
    rng = np.random.default_rng(4)
    far = np.array([0.5, -0.3, 2.0]) + rng.uniform(1.5, 2.5, (6, 3))
    pts = np.vstack([p, far]).astype(np.float32)
    P = _soa(g, pts)
    idx, d2 = ctx.knn(P, P, 20, cell=0.02)
    ei, ek = ok.knn_bruteforce(pts, pts, 20)
    assert (idx.cpu().numpy() == ei).all()
    assert (d2.cpu().numpy().view(np.uint32) == ek.view(np.uint32)).all()
    got = ctx.covariances(P, 20, cell=0.02, reg_mode=0).cpu().numpy().T
    exp = oc.covariances(pts, 20, oc.REG_NONE)
    assert _rel_frob(got, exp).max() < 1e-5


def test_covariances_planar_patch(g, ctx):
    _say("cov_planar")
    p, n = synth.planar_patch(2000, 3, normal=(0, 0, 1))
    got = ctx.covariances(_soa(g, p), 20, reg_mode=1, eps=1e-3).cpu().numpy().T
    expect = oc.to6(np.eye(3) - (1 - 1e-3) * np.outer(n, n))
    assert np.abs(got - expect).max() < 1e-6


def test_covariances_arg_errors(g, ctx):
    P = _soa(g, np.zeros((10, 3)))
    with pytest.raises(g.GicpError):
        ctx.covariances(P, 11)
    with pytest.raises(g.GicpError):
        ctx.covariances(P, 5, reg_mode=7)


def test_nonfinite_flag(g, ctx):
    _say("nonfinite")
    p = synth.tiny_cloud(100, 1)
    p[17, 1] = np.nan
    ctx.covariances(_soa(g, p), 8, reg_mode=0)
    assert ctx.sync_status() == 2
    assert ctx.sync_status() == 0


# -------------------------------------------------------------------- registration
def _register_pair(g, ctx, pr, max_it=30, r_max=0.1, map_cell=0.1, acc=0):
    src, tgt = _soa(g, pr.src), _soa(g, pr.tgt)
    tcov = ctx.covariances(tgt, 20, reg_mode=1, eps=1e-3)
    gm = ctx.map_build(tgt, tcov, cell=map_cell)
    prm = g.params(k=20, eps=1e-3, r_max=r_max, max_it=max_it, reg_mode=1, precision=acc)
    import torch
    scov = torch.empty((6, pr.src.shape[0]), dtype=torch.float32, device="cuda")
    r = ctx.register(src, gm, pr.init, prm, src_covs_out=scov)
    gm.close()
    return r, scov.cpu().numpy().T, tcov.cpu().numpy().T


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_register_c1_parity(g, ctx, seed):
    _say("register_c1", seed)
    pr = synth.c1_problem(room_seed=seed, src_seed=seed + 1, tgt_seed=seed + 2, tf_seed=seed + 3)
    r, _, _ = _register_pair(g, ctx, pr)
    cs, ct = oc.covariances(pr.src, 20), oc.covariances(pr.tgt, 20)
    o = og.register(pr.src, cs, pr.tgt, ct, pr.init, r_max=0.1, max_it=30)
    dr, dt = se3.pose_error(r.pose, o.pose)
    _say(f"  rot {dr:.2e} trans {dt:.2e} inl {r.n_inliers}/{o.n_inliers} it {r.iters}")
    assert r.status == 0 and r.iters == 30
    assert dr < 1e-5 and dt < 1e-5
    assert abs(r.n_inliers - o.n_inliers) <= 2
    # H, b of the last linearisation: same sums up to FP32 per-point rounding
    assert np.abs(r.H - o.H).max() < 1e-3 * np.abs(o.H).max()
    assert np.allclose(r.H, r.H.T)


@pytest.mark.parametrize("seed", [0, 3])
def test_register_pair_c1_parity(g, ctx, seed):
    """The problem-statement form gicp_register_pair(src, map_means, map_covs,
    init): map covariances used as given (here the oracle's plane-regularised
    ones in FP32), source covariances computed by the call."""
    _say("register_pair", seed)
    pr = synth.c1_problem(room_seed=seed, src_seed=seed + 1, tgt_seed=seed + 2, tf_seed=seed + 3)
    ct = oc.covariances(pr.tgt, 20).astype(np.float32)
    prm = g.params(k=20, eps=1e-3, r_max=0.1, max_it=30, reg_mode=1)
    r = ctx.register_pair(_soa(g, pr.src), _soa(g, pr.tgt), _soa(g, ct), pr.init, prm, map_cell=0.0)
    o = og.register(pr.src, oc.covariances(pr.src, 20), pr.tgt, ct, pr.init, r_max=0.1, max_it=30)
    dr, dt = se3.pose_error(r.pose, o.pose)
    _say(f"  rot {dr:.2e} trans {dt:.2e} inl {r.n_inliers}/{o.n_inliers}")
    assert r.status == 0 and r.iters == 30
    assert dr < 1e-5 and dt < 1e-5
    assert np.abs(r.H - o.H).max() < 1e-3 * np.abs(o.H).max()


def test_register_exact_recovery(g, ctx):
    _say("register_exact")
    room = synth.make_room(0)
    p, _ = synth.sample_surface(room, 20000, 1, 0.0)
    src = p.astype(np.float32)
    T = synth.random_offset(np.random.default_rng(100), 2.0, 0.02, exact=True)
    tgt = (src.astype(np.float64) @ T[:3, :3].T + T[:3, 3]).astype(np.float32)
    pr = synth.Problem(src, tgt, T, np.eye(4))
    r, _, _ = _register_pair(g, ctx, pr, max_it=40)
    dr, dt = se3.pose_error(r.pose, T)
    assert dr < 2e-6 and dt < 2e-6, (dr, dt)


@pytest.mark.parametrize("acc", [0, 1, 2])
def test_register_precision_modes(g, ctx, acc):
    _say("register_acc", acc)
    pr = synth.c1_problem()
    r, _, _ = _register_pair(g, ctx, pr, acc=acc)
    cs, ct = oc.covariances(pr.src, 20), oc.covariances(pr.tgt, 20)
    o = og.register(pr.src, cs, pr.tgt, ct, pr.init, r_max=0.1, max_it=30)
    dr, dt = se3.pose_error(r.pose, o.pose)
    _say(f"  acc {acc}: rot {dr:.2e} trans {dt:.2e}")
    assert dr < 1e-5 and dt < 1e-5


def test_register_deterministic(g, ctx):
    _say("register_determinism")
    pr = synth.c1_problem()
    a, _, _ = _register_pair(g, ctx, pr)
    b, _, _ = _register_pair(g, ctx, pr)
    assert (a.pose == b.pose).all() and (a.H == b.H).all() and (a.b == b.b).all()


def test_register_no_corr_and_degenerate(g, ctx):
    _say("register_errors")
    pr = synth.c1_problem(n=500)
    far = np.eye(4)
    far[:3, 3] = [20, 0, 0]
    r, _, _ = _register_pair(g, ctx, synth.Problem(pr.src, pr.tgt, pr.T_gt, far))
    assert r.status == 3 and r.iters == 1
    assert np.allclose(r.pose, far)
    z = np.linspace(-1, 1, 40)
    line = np.stack([np.zeros(40), np.zeros(40), z], 1).astype(np.float32)
    src = _soa(g, line)
    cov = _soa(g, np.tile([1, 0, 0, 1, 0, 0.001], (40, 1)))
    gm = ctx.map_build(src, cov, cell=0.1)
    rr = ctx.register(src, gm, np.eye(4), g.params(max_it=5), src_covs=cov)
    assert rr.status == 4


def test_register_max_it_zero(g, ctx):
    pr = synth.c1_problem(n=300)
    r, _, _ = _register_pair(g, ctx, pr, max_it=0)
    assert r.status == 0 and r.iters == 0 and np.allclose(r.pose, np.eye(4))
