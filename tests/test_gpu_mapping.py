"""Depth-to-points, keyframe Gaussians and incremental map update on the GPU
against the oracles (oracle/depth.py, oracle/mapping.py, oracle/gicp.py)."""
import numpy as np
import pytest

import synth
from oracle import covariance as oc
from oracle import depth as od
from oracle import gicp as og
from oracle import mapping as omap
from oracle import se3

pytestmark = pytest.mark.gpu

K = synth.camera.C2_INTRINSICS


@pytest.fixture(scope="module")
def env():
    import torch

    import paper_2403_12550_amd as g
    torch.cuda.set_device(0)
    ctx = g.Context(0)
    yield g, ctx
    ctx.close()


def _say(*a):
    print("[case]", *a, flush=True)


def _depth_case(g, ctx, d, voxel=0.02, max_depth=1e4):
    import torch
    got = ctx.depth_to_points(torch.from_numpy(d).cuda(), K.fx, K.fy, K.cx, K.cy, voxel, max_depth)
    dd = d.copy()
    dd[~(dd <= max_depth)] = 0
    exp, _ = od.depth_to_points(dd, K.fx, K.fy, K.cx, K.cy, voxel)
    return got.cpu().numpy().T, exp


@pytest.mark.parametrize("frame", [0, 37])
def test_depth_to_points_c2_frame(env, frame):
    g, ctx = env
    _say("depth", frame)
    seq = synth.C2Sequence(n_frames=40, map_size=1000)
    got, exp = _depth_case(g, ctx, seq.depth(frame))
    assert got.shape == exp.shape and 40000 < len(exp) < 120000
    # same voxels in the same order: every centroid within one FP32 rounding of the oracle's
    ulp = np.spacing(np.abs(exp).astype(np.float32))
    assert (np.abs(got - exp) <= ulp).all()


def test_depth_to_points_edge_cases(env):
    g, ctx = env
    _say("depth_edges")
    z = np.zeros((7, 9), np.float32)
    got, exp = _depth_case(g, ctx, z)
    assert got.shape == (0, 3) and exp.shape == (0, 3)
    z[3, 4] = 1.5
    got, exp = _depth_case(g, ctx, z)
    assert got.shape == (1, 3) and np.array_equal(got, exp)
    rng = np.random.default_rng(0)
    d = rng.uniform(0.3, 8.0, (31, 45)).astype(np.float32)
    d[rng.random(d.shape) < 0.2] = np.nan
    got, exp = _depth_case(g, ctx, d, voxel=0.05, max_depth=5.0)
    assert got.shape == exp.shape
    assert (np.abs(got - exp) <= np.spacing(np.abs(exp).astype(np.float32))).all()


def test_keyframe_policy_matches_oracle(env):
    g, ctx = env
    rng = np.random.default_rng(1)
    for _ in range(200):
        r, a, b = float(rng.random()), int(rng.integers(0, 40)), int(rng.integers(0, 15))
        assert ctx.keyframe_policy(r, a, b, 0.8, 30, 10) == omap.keyframe_policy(r, a, b, 0.8, 30, 10)


def test_keyframe_gaussians_parity(env):
    g, ctx = env
    _say("keyframe_gaussians")
    pr = synth.c1_problem(n=4000)
    # the source in a camera frame 1 m below the room (every depth z >= ~1 m)
    src = (pr.src + np.array([0.0, 0.0, 1.0])).astype(np.float32)
    lift = np.eye(4)
    lift[2, 3] = -1.0
    pose = pr.T_gt @ lift
    cs = oc.covariances(src, 20, oc.REG_ELLIPSE).astype(np.float32)
    # map: the target cloud with a hole (points near x < 1 removed) so that some source points overlap and some not
    tgt = pr.tgt[pr.tgt[:, 0] > 1.0]
    tcov = oc.covariances(tgt, 20, oc.REG_PLANE).astype(np.float32)
    gm = ctx.map_build(g.to_soa(tgt), g.to_soa(tcov), cell=0.1)
    means, covs, ratio = ctx.keyframe_gaussians(g.to_soa(src), g.to_soa(cs), gm, pose, 0.1, 1.5)
    gm.close()
    r_o, m_o, c_o = omap.keyframe_gaussians(src.astype(np.float64), cs.astype(np.float64), pose,
                                            tgt.astype(np.float64), 0.1, 1.5)
    # overlap decisions may differ only for points whose distance is within FP32 rounding of r
    flags = omap.overlap_flags(src.astype(np.float64), pose, tgt.astype(np.float64), 0.1)
    assert 0.2 < r_o < 0.95
    assert abs(ratio - r_o) * len(src) <= 2
    mg, cg = means.cpu().numpy().T.astype(np.float64), covs.cpu().numpy().T.astype(np.float64)
    # a point at the overlap boundary may be decided differently (FP32 test):
    # the kept sets are matched by position, and every matched Gaussian's mean
    # and covariance compared; at most two points may be unmatched per side
    from scipy.spatial import cKDTree
    d, j = cKDTree(m_o).query(mg)
    matched = d < 1e-5
    assert matched.sum() >= len(mg) - 2 and matched.sum() >= len(m_o) - 2
    if len(mg) == len(m_o):
        assert matched.all() and (j == np.arange(len(m_o))).all()
    assert np.abs(mg[matched] - m_o[j[matched]]).max() <= 1e-6 * max(1.0, np.abs(m_o).max())
    rel = np.linalg.norm(cg[matched] - c_o[j[matched]], axis=1) / np.linalg.norm(c_o[j[matched]], axis=1)
    _say("  kept", len(mg), len(m_o), "max rel cov", rel.max())
    assert rel.max() < 1e-5


def test_map_insert_equals_build(env):
    g, ctx = env
    _say("map_insert")
    pr = synth.c1_problem(n=6000, room_seed=5)
    tgt = pr.tgt
    tcov = oc.covariances(tgt, 20, oc.REG_NONE).astype(np.float32)
    parts = [slice(0, 2500), slice(2500, 4000), slice(4000, 4100), slice(4100, 6000)]
    gm = ctx.map_build(g.to_soa(tgt[parts[0]]), g.to_soa(tcov[parts[0]]), cell=0.1, reg_mode=g.REG_PLANE)
    for sl in parts[1:]:
        ctx.map_insert(gm, g.to_soa(tgt[sl]), g.to_soa(tcov[sl]))
    assert gm.m == 6000
    ref = ctx.map_build(g.to_soa(tgt), g.to_soa(tcov), cell=0.1, reg_mode=g.REG_PLANE)
    src = g.to_soa(pr.src)
    scov = g.to_soa(oc.covariances(pr.src, 20, oc.REG_PLANE).astype(np.float32))
    prm = g.params(max_it=30)
    a = ctx.register(src, gm, np.eye(4), prm, src_covs=scov)
    b = ctx.register(src, ref, np.eye(4), prm, src_covs=scov)
    assert np.array_equal(a.pose, b.pose) and np.array_equal(a.H, b.H) and a.n_inliers == b.n_inliers
    # and against the oracle on the union map
    tc = oc.regularise6(tcov.astype(np.float64), oc.REG_PLANE, 1e-3).astype(np.float32)
    o = og.register(pr.src, oc.covariances(pr.src, 20, oc.REG_PLANE).astype(np.float32), tgt, tc, np.eye(4),
                    r_max=0.1, max_it=30)
    dr, dt = se3.pose_error(a.pose, o.pose)
    assert dr < 1e-5 and dt < 1e-5
    gm.close()
    ref.close()
