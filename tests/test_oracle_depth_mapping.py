"""Pins of the depth-to-points and keyframe oracles (oracle/depth.py,
oracle/mapping.py): closed forms, loops over tiny inputs, invariants."""
import numpy as np

from oracle import covariance as oc
from oracle import depth as od
from oracle import mapping as om


def test_backproject_constant_depth_closed_form():
    H, W, z = 5, 7, 2.0
    fx, fy, cx, cy = 600.0, 500.0, 3.0, 2.0
    p = od.backproject(np.full((H, W), z, np.float32), fx, fy, cx, cy)
    assert p.shape == (H * W, 3)
    v, u = np.divmod(np.arange(H * W), W)
    assert np.allclose(p[:, 0], (u - cx) * z / fx, rtol=1e-6, atol=1e-9)
    assert np.allclose(p[:, 1], (v - cy) * z / fy, rtol=1e-6, atol=1e-9)
    assert (p[:, 2] == z).all()


def test_backproject_drops_invalid_pixels():
    d = np.array([[1.0, 0.0, -1.0], [np.nan, np.inf, 2.0]], np.float32)
    p = od.backproject(d, 1.0, 1.0, 0.0, 0.0)
    assert p.shape == (2, 3) and list(p[:, 2]) == [1.0, 2.0]


def _loop_voxels(points, s):
    groups = {}
    for q in points:
        key = tuple(int(np.floor(np.float32(c) / np.float32(s))) for c in q)
        groups.setdefault(key, []).append([float(c) for c in q])
    keys = sorted(groups)
    return [np.mean(groups[k], axis=0) for k in keys], [len(groups[k]) for k in keys]


def test_voxel_centroids_match_loops():
    rng = np.random.default_rng(0)
    p = rng.uniform(-0.1, 0.1, (300, 3)).astype(np.float32)
    cen, cnt = od.voxel_centroids(p, 0.05)
    lc, ln = _loop_voxels(p, 0.05)
    assert list(cnt) == ln
    assert np.allclose(cen, np.array(lc), rtol=0, atol=1e-7)
    assert cnt.sum() == len(p)


def test_voxel_centroids_invariants():
    rng = np.random.default_rng(1)
    p = rng.uniform(-1, 1, (2000, 3)).astype(np.float32)
    s = 0.1
    cen, cnt = od.voxel_centroids(p, s)
    cen2, cnt2 = od.voxel_centroids(p[rng.permutation(len(p))], s)
    assert np.array_equal(cnt, cnt2) and np.allclose(cen, cen2, atol=1e-7)
    # a centroid lies in its voxel's box (convex hull of its points)
    ids = od.voxel_ids(cen, s)
    lo, hi = ids * s - 1e-6, (ids + 1) * s + 1e-6
    assert ((cen >= lo) & (cen <= hi)).all()
    # sorted lexicographically, no repeats
    keys = [tuple(r) for r in ids]
    assert keys == sorted(set(keys))


def test_scale_align_closed_form():
    C = oc.to6(np.diag([4.0, 1.0, 0.25])[None])
    out = om.scale_align(C, np.array([2.0]), 1.5)
    lam = np.linalg.eigvalsh(oc.from6(out)[0])
    # scales (2, 1, 0.5) divided by z^p = 2^1.5, squared
    assert np.allclose(sorted(lam), sorted(np.array([2.0, 1.0, 0.5]) ** 2 / 2 ** 3), rtol=1e-12)


def test_overlap_flags_brute_force():
    rng = np.random.default_rng(2)
    src = rng.uniform(0, 1, (50, 3))
    mp = rng.uniform(0, 1, (80, 3))
    T = np.eye(4)
    T[:3, 3] = [0.05, -0.02, 0.01]
    f = om.overlap_flags(src, T, mp, 0.1)
    q = src + T[:3, 3]
    d = np.sqrt(((q[:, None, :] - mp[None]) ** 2).sum(-1)).min(axis=1)
    assert np.array_equal(f, d <= 0.1)


def test_keyframe_gaussians_transform():
    rng = np.random.default_rng(3)
    src = rng.uniform(0.5, 2.0, (40, 3))
    covs = oc.to6(np.tile(np.diag([1e-4, 4e-4, 1e-6]), (40, 1, 1)))
    th = np.pi / 2
    T = np.eye(4)
    T[:3, :3] = [[np.cos(th), -np.sin(th), 0], [np.sin(th), np.cos(th), 0], [0, 0, 1]]
    T[:3, 3] = [1.0, 2.0, 3.0]
    far_map = np.array([[100.0, 100.0, 100.0]])
    ratio, means, out = om.keyframe_gaussians(src, covs, T, far_map, 0.1, 1.5)
    assert ratio == 0.0 and len(means) == 40
    assert np.allclose(means, src @ T[:3, :3].T + T[:3, 3])
    # rotation about z by 90 degrees swaps the xx and yy entries; every entry scaled by z^-3
    z3 = src[:, 2] ** 3
    assert np.allclose(out[:, 0], 4e-4 / z3) and np.allclose(out[:, 3], 1e-4 / z3)
    assert np.allclose(out[:, 5], 1e-6 / z3)
    # a map containing every transformed point: nothing is added
    ratio, means, _ = om.keyframe_gaussians(src, covs, T, src @ T[:3, :3].T + T[:3, 3], 0.1, 1.5)
    assert ratio == 1.0 and len(means) == 0


def test_keyframe_policy_cases():
    K, M = om.KEYFRAME, om.MAPPING_ONLY
    assert om.keyframe_policy(0.5, 1, 1, 0.8) == K
    assert om.keyframe_policy(0.9, 30, 3, 0.8) == K
    assert om.keyframe_policy(0.9, 12, 10, 0.8) == M
    assert om.keyframe_policy(0.9, 5, 5, 0.8) == 0
