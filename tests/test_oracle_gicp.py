"""Pins of the oracle's Gauss-Newton G-ICP (Sec. 3, Eq. MLE_for_T): hand-derived
single steps, exact recovery of known rigid transforms, the Kabsch/Umeyama
special case, finite-difference Jacobians and gradients, and the error paths."""
import json
import os

import numpy as np
import pytest
from scipy.spatial.transform import Rotation

import synth
from oracle import covariance as oc
from oracle import gicp as og
from oracle import se3

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _gold():
    return json.load(open(os.path.join(GOLD, "gn_one_step.json")))


def _apply(T, p):
    return p @ T[:3, :3].T + T[:3, 3]


def test_golden_translation_step():
    g = _gold()
    src = np.array(g["source"], float)
    cov = np.tile(np.array(g["cov"]), (6, 1))
    c = g["translation_case"]
    tgt = src + np.array(c["target_offset"])
    H, b, e, n, j = og.linearise(np.eye(4), src, oc.from6(cov), tgt, oc.from6(cov), g["r_max"])
    assert n == 6 and (j == np.arange(6)).all()
    assert np.abs(H - np.diag(c["expected_H_diag"])).max() < 1e-14
    assert np.abs(b - np.array(c["expected_b"])).max() < 1e-14
    assert abs(e - c["expected_cost"]) < 1e-15
    step = -og.cholesky_solve(H, b)
    assert np.abs(step - np.array(c["expected_step"])).max() < 1e-15
    # register() reads FP32 inputs: 1 + 0.1 is not exact in FP32, so compare with
    # the offset the rounded target actually carries (the mean of tgt - src)
    r = og.register(src, cov, tgt, cov, np.eye(4), r_max=g["r_max"], max_it=1)
    t32 = (tgt.astype(np.float32).astype(np.float64) - src).mean(0)
    assert np.abs(r.pose[:3, 3] - t32).max() < 1e-15


def test_golden_rotation_step():
    g = _gold()
    src = np.array(g["source"], float)
    cov = np.tile(np.array(g["cov"]), (6, 1))
    a = g["rotation_case"]["alpha"]
    R = Rotation.from_rotvec([0, 0, a]).as_matrix()
    tgt = src @ R.T
    H, b, e, n, j = og.linearise(np.eye(4), src, oc.from6(cov), tgt, oc.from6(cov), g["r_max"])
    assert n == 6
    assert abs(b[2] - (-4 * np.sin(a))) < 1e-14
    assert np.abs(np.delete(b, 2)).max() < 1e-14
    assert abs(e - 8 * (1 - np.cos(a))) < 1e-14
    step = -og.cholesky_solve(H, b)
    assert abs(step[2] - np.sin(a)) < 1e-14
    assert np.abs(np.delete(step, 2)).max() < 1e-14


def _dense_room(n=20000, seed=0):
    room = synth.make_room(seed)
    p, _ = synth.sample_surface(room, n, seed + 1, 0.0)
    return p.astype(np.float32)


@pytest.mark.parametrize("deg,m,seed", [(2.0, 0.02, 0), (3.0, 0.03, 1)])
def test_exact_recovery_noise_free(deg, m, seed):
    """Noise-free target = T_gt * (the same points): T_gt is a fixed point with
    zero residuals, and GN from identity converges to it."""
    src = _dense_room(20000, seed)
    T = synth.random_offset(np.random.default_rng(seed + 100), deg, m, exact=True)
    tgt = _apply(T, src.astype(np.float64)).astype(np.float32)
    cs = oc.covariances(src, 20)
    ct = oc.covariances(tgt, 20)
    r = og.register(src, cs, tgt, ct, np.eye(4), r_max=0.1, max_it=40)
    dr, dt = se3.pose_error(r.pose, T)
    # target coordinates are FP32-rounded images, so recovery is exact up to that rounding
    assert dr < 1e-7 and dt < 1e-7, (dr, dt)
    assert r.n_inliers == src.shape[0]


def test_kabsch_special_case():
    """With M = I (both covariances I/2) and correspondences that cannot change
    (points 1 m apart, noise 1 cm), the GN fixed point is the least-squares rigid
    fit, which the SVD (Kabsch/Umeyama) gives in closed form."""
    rng = np.random.default_rng(4)
    src = rng.uniform(-3, 3, (60, 3))
    src = src[np.argsort(src[:, 0])]
    # spread points so that nearest neighbours are unambiguous
    src = np.array([[i % 4, (i // 4) % 4, i // 16] for i in range(60)], float) * 1.0 + rng.normal(0, 0.02, (60, 3))
    T = synth.random_offset(np.random.default_rng(5), 3.0, 0.05, exact=True)
    tgt = _apply(T, src) + rng.normal(0, 0.01, (60, 3))
    src = src.astype(np.float32).astype(np.float64)
    tgt = tgt.astype(np.float32).astype(np.float64)
    cov = np.tile([0.5, 0, 0, 0.5, 0, 0.5], (60, 1))
    r = og.register(src, cov, tgt, cov, np.eye(4), r_max=0.45, max_it=30)
    assert r.n_inliers == 60
    # closed form
    ms, mt = src.mean(0), tgt.mean(0)
    U, S, Vt = np.linalg.svd((tgt - mt).T @ (src - ms))
    D = np.diag([1, 1, np.sign(np.linalg.det(U @ Vt))])
    R = U @ D @ Vt
    t = mt - R @ ms
    K = np.eye(4)
    K[:3, :3], K[:3, 3] = R, t
    dr, dt = se3.pose_error(r.pose, K)
    assert dr < 1e-10 and dt < 1e-10, (dr, dt)


def _frozen_problem(seed=0):
    p = synth.c1_problem(n=2000, room_seed=seed)
    src = p.src.astype(np.float64)
    tgt = p.tgt.astype(np.float64)
    Cs = oc.from6(oc.covariances(p.src, 20))
    Ct = oc.from6(oc.covariances(p.tgt, 20))
    T = p.T_gt @ se3.exp_se3(np.array([0.01, -0.02, 0.015, 0.01, 0.02, -0.01]))
    return T, src, Cs, tgt, Ct


def test_jacobian_finite_difference():
    """J_i = [[q]x, -I] is the derivative of d_i(xi) = mu_i - Exp(xi) T x_i at xi = 0."""
    T, src, _, tgt, _ = _frozen_problem()
    x = src[:50]
    mu = tgt[:50]
    q = _apply(T, x)
    J = np.concatenate([og.skew(q), np.broadcast_to(-np.eye(3), (50, 3, 3))], axis=2)
    h = 1e-6
    for k in range(6):
        e = np.zeros(6)
        e[k] = h
        dp = mu - _apply(se3.exp_se3(e) @ T, x)
        dm = mu - _apply(se3.exp_se3(-e) @ T, x)
        assert np.abs((dp - dm) / (2 * h) - J[:, :, k]).max() < 1e-8


def test_gradient_and_hessian_finite_difference():
    """With correspondences and M frozen, E(xi) = sum d_i(xi)^T M_i d_i(xi) has
    gradient 2b at xi = 0 and Gauss-Newton Hessian 2H (exact for the linearised
    residual)."""
    T, src, Cs, tgt, Ct = _frozen_problem()
    H, b, e, n, j = og.linearise(T, src, Cs, tgt, Ct, 0.1)
    ok = j >= 0
    R = T[:3, :3]
    M = np.linalg.inv(Ct[j[ok]] + R @ Cs[ok] @ R.T)
    x, mu = src[ok], tgt[j[ok]]

    def E(xi):
        d = mu - _apply(se3.exp_se3(xi) @ T, x)
        return float(np.einsum("ni,nij,nj->", d, M, d))

    assert abs(E(np.zeros(6)) - e) < 1e-9 * e
    h = 1e-6
    g = np.array([(E(h * np.eye(6)[k]) - E(-h * np.eye(6)[k])) / (2 * h) for k in range(6)])
    assert np.abs(g - 2 * b).max() < 1e-5 * np.abs(2 * b).max() + 1e-6
    # H symmetric positive semi-definite
    assert np.abs(H - H.T).max() < 1e-9 * np.abs(H).max()
    assert np.linalg.eigvalsh(H).min() > -1e-9 * np.abs(H).max()


def test_inliers_monotone_in_rmax():
    T, src, Cs, tgt, Ct = _frozen_problem()
    counts = [og.linearise(T, src, Cs, tgt, Ct, r)[3] for r in (0.02, 0.05, 0.1, 0.2)]
    assert counts == sorted(counts)


def test_b_vanishes_at_convergence():
    p = synth.c1_problem(n=3000)
    cs, ct = oc.covariances(p.src, 20), oc.covariances(p.tgt, 20)
    r = og.register(p.src, cs, p.tgt, ct, np.eye(4), r_max=0.1, max_it=30)
    # register() reads covariances as FP32, so linearise at the same values
    c32 = lambda c: oc.from6(c.astype(np.float32).astype(np.float64))
    H, b, e, n, _ = og.linearise(r.pose, p.src.astype(np.float64), c32(cs),
                                 p.tgt.astype(np.float64), c32(ct), 0.1)
    step = og.cholesky_solve(H, b)
    assert np.abs(step).max() < 1e-13


def test_no_correspondences():
    p = synth.c1_problem(n=500)
    cs, ct = oc.covariances(p.src, 20), oc.covariances(p.tgt, 20)
    far = np.eye(4)
    far[:3, 3] = [20.0, 0, 0]
    r = og.register(p.src, cs, p.tgt, ct, far, r_max=0.1, max_it=5)
    assert r.status == og.E_NO_CORR and r.iters == 1


def test_degenerate_collinear():
    """Source and target on the z axis: rotation about z leaves every residual
    unchanged, so H has an exactly zero row and column and Cholesky fails."""
    z = np.linspace(-1, 1, 40)
    src = np.stack([np.zeros(40), np.zeros(40), z], 1).astype(np.float32)
    cov = np.tile([1, 0, 0, 1, 0, 0.001], (40, 1)).astype(np.float32)
    r = og.register(src, cov, src.copy(), cov, np.eye(4), r_max=0.1, max_it=5)
    assert r.status == og.E_DEGENERATE


def test_c1_converges_near_truth():
    p = synth.c1_problem()
    cs, ct = oc.covariances(p.src, 20), oc.covariances(p.tgt, 20)
    r = og.register(p.src, cs, p.tgt, ct, np.eye(4), r_max=0.1, max_it=30)
    dr, dt = se3.pose_error(r.pose, p.T_gt)
    # resampled, noisy clouds: a sanity bound, not an exactness claim
    assert dr < 2e-3 and dt < 2e-3


# ------------------------------------------------------------------ tracking loop
def test_track_motion_models_on_exact_motion():
    """On a sequence that moves by exactly the same relative motion every
    frame, the constant-velocity prediction of frame i from the true poses of
    frames i-2 and i-1 is the true pose of frame i (closed form), and the
    previous-pose prediction is the pose of frame i-1."""
    from oracle import se3
    from oracle import tracking as ot
    step = se3.exp_se3(np.array([0.01, -0.02, 0.015, 0.02, 0.0, -0.01]))
    poses = [np.eye(4)]
    for _ in range(5):
        poses.append(poses[-1] @ step)
    for i in range(2, 6):
        cv = ot.predict(poses, i, np.eye(4), ot.CONSTANT_VELOCITY)
        assert np.allclose(cv, poses[i], atol=1e-13)
        assert np.array_equal(ot.predict(poses, i, np.eye(4), ot.PREVIOUS), poses[i - 1])
    assert np.array_equal(ot.predict(poses, 1, np.eye(4), ot.CONSTANT_VELOCITY), poses[0])
    T0 = se3.exp_se3(np.array([0.1, 0, 0, 1, 2, 3]))
    assert np.array_equal(ot.predict([], 0, T0, ot.PREVIOUS), T0)
    assert np.allclose(ot.rigid_inverse(T0) @ T0, np.eye(4), atol=1e-15)


def test_track_exact_sequence_recovers_poses():
    """Noise-free frames that are the map seen from known poses: tracking from
    the first pose recovers every pose (both motion models)."""
    import synth
    from oracle import tracking as ot
    room = synth.make_room(3)
    mp, _ = synth.sample_surface(room, 6000, 5, 0.0)
    mp = mp.astype(np.float32)
    mc = oc.covariances(mp, 20)
    rng = np.random.default_rng(4)
    poses = [np.eye(4)]
    for _ in range(4):
        poses.append(poses[-1] @ synth.random_offset(rng, 1.0, 0.01))
    frames = [((mp.astype(np.float64) - T[:3, 3]) @ T[:3, :3]).astype(np.float32) for T in poses]
    for motion in (ot.PREVIOUS, ot.CONSTANT_VELOCITY):
        est, _, res = ot.track(frames, mp, mc, poses[0], motion=motion, max_it=40, conv=1e-9)
        for T, E in zip(poses, est):
            dr, dt = se3.pose_error(E, T)
            assert dr < 1e-6 and dt < 1e-6, (motion, dr, dt)
