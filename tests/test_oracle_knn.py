"""Pins of the oracle's k-NN (Sec. 3: covariance from the k nearest neighbours;
correspondences by nearest-neighbour search) against brute force written as
plain scalar loops, hand-derived ties, and library kd-trees."""
import json
import os

import numpy as np
import pytest
from scipy.spatial import cKDTree

import synth
from oracle import knn as oknn

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _scalar_knn(points, q, k):
    """Brute force as scalar float32 arithmetic and a Python sort."""
    f = np.float32
    rows = []
    for j, p in enumerate(points):
        dx = f(q[0]) - f(p[0])
        dy = f(q[1]) - f(p[1])
        dz = f(q[2]) - f(p[2])
        key = f(f(f(dx * dx) + f(dy * dy)) + f(dz * dz))
        rows.append((float(key), j))
    rows.sort()
    return [j for _, j in rows[:k]], [kk for kk, _ in rows[:k]]


def test_golden_ties():
    g = json.load(open(os.path.join(GOLD, "knn_ties.json")))
    pts = np.array(g["points"], np.float32)
    idx, key = oknn.knn_bruteforce(pts, pts[g["query_index"]:g["query_index"] + 1], g["k"])
    assert idx[0].tolist() == g["expected_idx"]
    assert np.allclose(key[0], g["expected_key"], rtol=0, atol=0)


@pytest.mark.parametrize("seed,lattice,dups", [(0, False, 0), (1, True, 0), (2, False, 7), (3, True, 9)])
def test_bruteforce_matches_scalar_loops(seed, lattice, dups):
    pts = synth.tiny_cloud(40, seed, duplicates=dups, lattice=lattice)
    k = 7
    idx, key = oknn.knn_bruteforce(pts, pts, k)
    for i in range(pts.shape[0]):
        ei, ek = _scalar_knn(pts, pts[i], k)
        assert idx[i].tolist() == ei
        assert key[i].tolist() == ek


def test_self_is_first_neighbour_without_duplicates():
    pts = synth.tiny_cloud(200, 5)
    idx, key = oknn.knn_bruteforce(pts, pts, 5)
    assert (idx[:, 0] == np.arange(200)).all()
    assert (key[:, 0] == 0).all()


def test_duplicates_rank_by_lower_index():
    pts = synth.tiny_cloud(30, 6, duplicates=30)
    idx, key = oknn.knn_bruteforce(pts, pts, 2)
    # every point has an exact copy; the copy with the lower index comes first
    for i in range(pts.shape[0]):
        same = np.nonzero((pts == pts[i]).all(axis=1))[0]
        assert idx[i, 0] == same.min()
        assert key[i, 0] == 0


def test_key_close_to_exact_distance():
    rng = np.random.default_rng(0)
    q = rng.uniform(-5, 5, (1000, 3)).astype(np.float32)
    p = rng.uniform(-5, 5, (1000, 3)).astype(np.float32)
    key = oknn.fp32_key(q, p).astype(np.float64)
    exact = ((q.astype(np.float64) - p.astype(np.float64)) ** 2).sum(1)
    assert np.all(np.abs(key - exact) <= 4e-7 * exact + 1e-30)


def test_fewer_points_than_k_and_gate():
    pts = np.array([[0, 0, 0], [0.3, 0, 0], [0, 0.05, 0]], np.float32)
    idx, key = oknn.knn_bruteforce(pts, pts[:1], 5)
    assert idx[0].tolist() == [0, 2, 1, -1, -1]
    assert np.isinf(key[0, 3:]).all()
    idx, key = oknn.knn_bruteforce(pts, pts[:1], 5, r_max=0.1)
    assert idx[0].tolist() == [0, 2, -1, -1, -1]


def test_empty_inputs():
    idx, key = oknn.knn_bruteforce(np.zeros((0, 3), np.float32), np.zeros((3, 3), np.float32), 4)
    assert (idx == -1).all()
    idx, key = oknn.knn_bruteforce(np.zeros((5, 3), np.float32), np.zeros((0, 3), np.float32), 4)
    assert idx.shape == (0, 4)


@pytest.mark.parametrize("seed", [0, 1])
def test_kdtree_path_equals_bruteforce(seed):
    room = synth.make_room(seed)
    p, _ = synth.sample_surface(room, 3000, seed + 10, 0.002)
    p = p.astype(np.float32)
    # add exact duplicates and a lattice patch to create ties
    p = np.vstack([p, p[:50], synth.tiny_cloud(64, seed, lattice=True) + np.float32(5.0)])
    bi, bk = oknn.knn_bruteforce(p, p, 20)
    ki, kk = oknn.knn_kdtree(p, p, 20)
    assert (bi == ki).all()
    assert (bk == kk).all()


def test_nearest_fp64_against_library_and_gate():
    rng = np.random.default_rng(3)
    tgt = rng.uniform(0, 1, (2000, 3))
    q = rng.uniform(0, 1, (500, 3))
    idx, d2 = oknn.nearest_fp64(tgt, q, r_max=0.05)
    d, j = cKDTree(tgt).query(q, k=1)
    inside = d <= 0.05
    assert (idx[inside] == j[inside]).all()
    assert (idx[~inside] == -1).all()
    assert np.allclose(d2[inside], d[inside] ** 2, rtol=1e-12)


def test_nearest_fp64_tie_lower_index():
    tgt = np.array([[1.0, 0, 0], [-1.0, 0, 0], [0, 1.0, 0], [0, -1.0, 0], [0, 0, 1.0], [0, 0, -1.0]])
    idx, _ = oknn.nearest_fp64(tgt, np.zeros((1, 3)), r_max=2.0)
    assert idx[0] == 0
    idx, _ = oknn.nearest_fp64(tgt[::-1].copy(), np.zeros((1, 3)), r_max=2.0)
    assert idx[0] == 0
