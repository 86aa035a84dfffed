"""Pins of the oracle's covariances (Sec. 3: covariance of the k nearest
neighbours; Sec. 3.1.1: C = R Lambda^2 R^T, plane and ellipse regularisation)."""
import json
import os

import numpy as np
import pytest
from scipy.spatial.transform import Rotation

import synth
from oracle import covariance as oc

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def test_golden_line():
    g = json.load(open(os.path.join(GOLD, "cov_line.json")))
    pts = np.array(g["points"], np.float32)
    c = oc.covariances(pts, g["k"], oc.REG_NONE)
    for row in c:
        assert np.allclose(row, g["expected_cov6_raw_each"], rtol=0, atol=1e-15)


def test_golden_rectangle():
    g = json.load(open(os.path.join(GOLD, "cov_rectangle.json")))
    pts = np.array(g["points"], np.float32)
    for mode, key in [(oc.REG_NONE, "expected_raw"), (oc.REG_PLANE, "expected_plane"),
                      (oc.REG_ELLIPSE, "expected_ellipse")]:
        c = oc.covariances(pts, g["k"], mode, g["eps"])
        for row in c:
            assert np.allclose(row, g[key], rtol=0, atol=1e-12), (mode, row)


def test_cube_vertices_isotropic():
    a = 0.5
    pts = np.array([[sx * a, sy * a, sz * a] for sx in (-1, 1) for sy in (-1, 1) for sz in (-1, 1)], np.float32)
    c = oc.covariances(pts, 8, oc.REG_NONE)
    assert np.allclose(oc.from6(c), a * a * np.eye(3), atol=1e-15)


@pytest.mark.parametrize("normal", [(0, 0, 1), (1, 2, 3), (-0.3, 0.9, 0.1)])
def test_planar_patch_closed_form(normal):
    """Noise-free points on a plane with normal n: lambda0 = 0 and
    C_plane = I - (1 - eps) n n^T (computed on FP64 points, exact neighbour sets)."""
    p, n = synth.planar_patch(300, 7, normal=normal)
    eps = 1e-3
    from oracle.knn import knn_bruteforce
    idx, _ = knn_bruteforce(p.astype(np.float32), p.astype(np.float32), 20)
    C = oc.neighbourhood_covariance(p, idx)              # FP64 points, exactly planar
    lam = np.linalg.eigvalsh(C)
    assert np.all(np.abs(lam[:, 0]) < 1e-15)
    Cp = oc.regularise(C, oc.REG_PLANE, eps)
    expect = np.eye(3) - (1 - eps) * np.outer(n, n)
    assert np.abs(Cp - expect).max() < 1e-12


def test_rigid_equivariance():
    rng = np.random.default_rng(1)
    P = rng.normal(size=(400, 3)) * [0.5, 0.2, 0.01]
    idx = np.stack([rng.permutation(400)[:20] for _ in range(400)])
    R = Rotation.from_rotvec([0.3, -1.1, 0.4]).as_matrix()
    t = np.array([1.0, -2.0, 3.0])
    C = oc.neighbourhood_covariance(P, idx)
    C2 = oc.neighbourhood_covariance(P @ R.T + t, idx)
    assert np.abs(C2 - R @ C @ R.T).max() < 1e-13
    for mode in (oc.REG_PLANE, oc.REG_ELLIPSE):
        A = oc.regularise(C, mode)
        B = oc.regularise(C2, mode)
        assert np.abs(B - R @ A @ R.T).max() < 1e-9


def test_neighbour_order_invariance():
    rng = np.random.default_rng(2)
    P = rng.normal(size=(100, 3))
    idx = np.stack([rng.permutation(100)[:20] for _ in range(100)])
    perm = idx[:, rng.permutation(20)]
    assert np.abs(oc.neighbourhood_covariance(P, idx) - oc.neighbourhood_covariance(P, perm)).max() < 1e-14


def test_plane_form_properties_on_room():
    p = synth.c1_problem().src
    c, C, _ = oc.covariances(p, 20, oc.REG_PLANE, 1e-3, return_raw=True)
    Cp = oc.from6(c)
    lam = np.linalg.eigvalsh(Cp)
    assert np.allclose(lam, [1e-3, 1, 1], atol=1e-12)        # eigenvalues exactly (eps, 1, 1)
    assert np.allclose(np.trace(Cp, axis1=1, axis2=2), 2.001, atol=1e-12)
    # the plane normal is the raw covariance's smallest-eigenvalue direction
    w, V = np.linalg.eigh(C)
    n = V[:, :, 0]
    assert np.allclose(np.einsum("nij,nj->ni", Cp, n), 1e-3 * n, atol=1e-10)


def test_ellipse_middle_eigenvalue_is_one():
    p = synth.c1_problem().src
    c = oc.covariances(p, 20, oc.REG_ELLIPSE)
    lam = np.linalg.eigvalsh(oc.from6(c))
    assert np.allclose(lam[:, 1], 1.0, rtol=1e-10)
    assert np.all(lam[:, 0] <= 1 + 1e-12) and np.all(lam[:, 2] >= 1 - 1e-12)


def test_sum_decomposition_reconstructs():
    rng = np.random.default_rng(3)
    A = rng.normal(size=(50, 3, 3))
    C = A @ A.transpose(0, 2, 1)
    lam, V = np.linalg.eigh(C)
    assert np.abs(np.einsum("nij,nj,nkj->nik", V, lam, V) - C).max() < 1e-12


@pytest.mark.parametrize("case", ["collinear", "coincident", "thin_needle"])
def test_golden_ellipse_degenerate(case):
    """The ellipse form where the middle eigenvalue vanishes (collinear or
    coincident neighbours), and at the clamp's edge."""
    g = json.load(open(os.path.join(GOLD, "cov_ellipse_degenerate.json")))[case]
    pts = np.array(g["points"], np.float64)
    idx = np.tile(np.arange(len(pts)), (len(pts), 1))
    C = oc.neighbourhood_covariance(pts, idx)
    got = oc.to6(oc.regularise(C, oc.REG_ELLIPSE))
    exp = np.array(g["expected_cov6_ellipse_each"])
    for row in got:
        assert np.allclose(row, exp, rtol=1e-9, atol=1e-9), (case, row)
