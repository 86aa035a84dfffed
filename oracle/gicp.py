"""Oracle: G-ICP registration by Gauss-Newton (test infrastructure only).

Paper, Sec. 3: with correspondences x^s_i <-> x^t_i from nearest-neighbour
search, the residual d_i = x^t_i - T x^s_i is Gaussian with covariance
C^t_i + T C^s_i T^T, and the maximum-likelihood pose is
    T* = argmin_T  sum_i d_i^T (C^B_i + T C^A_i T^T)^{-1} d_i      (Eq. MLE_for_T)
where C^B is the target (map) covariance and C^A the source covariance.

Readings (the paper names no optimiser and mixes notations):
* only the rotation acts on a covariance: Sigma_i = C^t_i + R C^s_i R^T;
* Gauss-Newton with a left perturbation T <- Exp(xi) T, xi = [omega; v];
  d_i(xi) = mu_i - (q_i + omega x q_i + v) with q_i = R x_i + t, hence the
  Jacobian J_i = [ [q_i]x , -I ];  M_i = Sigma_i^{-1} is evaluated at the
  current rotation and held fixed while differentiating;
* H = sum J^T M J, b = sum J^T M d, e = sum d^T M d (sums, not means);
  the step is xi = -H^{-1} b by Cholesky, then T <- Exp(xi) T;
* correspondences are recomputed at every iteration: the exact nearest map
  mean of q_i, accepted iff within r_max (ties to the lower index);
* fewer than 6 inliers -> NO_CORR; a failed Cholesky -> DEGENERATE, where the
  factorisation fails when a pivot is not above PIVOT_TOL * max(diag H)
  (an exactly or numerically rank-deficient system);
* stop when |omega| < conv_rot and |v| < conv_trans, or after max_it;
* the returned H, b are those of the last linearisation (the one that
  produced the final step).
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np
import scipy.linalg
from scipy.spatial import cKDTree

from .covariance import from6
from .knn import nearest_fp64
from .se3 import exp_se3

OK, E_NO_CORR, E_DEGENERATE = 0, 3, 4
PIVOT_TOL = 1e-12


def cholesky_solve(H: np.ndarray, b: np.ndarray):
    """Solve H x = b for symmetric positive definite H by the textbook
    Cholesky factorisation H = L L^T; returns None if a pivot is not above
    PIVOT_TOL * max(diag H)."""
    n = H.shape[0]
    L = np.zeros_like(H)
    floor = PIVOT_TOL * max(float(np.max(np.diag(H))), 0.0)
    for j in range(n):
        s = H[j, j] - L[j, :j] @ L[j, :j]
        if not (s > floor) or not np.isfinite(s):
            return None
        L[j, j] = np.sqrt(s)
        for i in range(j + 1, n):
            L[i, j] = (H[i, j] - L[i, :j] @ L[j, :j]) / L[j, j]
    y = scipy.linalg.solve_triangular(L, b, lower=True)
    return scipy.linalg.solve_triangular(L.T, y, lower=False)


@dataclass
class Result:
    pose: np.ndarray
    H: np.ndarray
    b: np.ndarray
    cost: float
    n_inliers: int
    iters: int
    converged: bool
    status: int = OK
    history: list = field(default_factory=list)


def skew(q: np.ndarray) -> np.ndarray:
    """Batched [q]x for q [n,3]."""
    Z = np.zeros(q.shape[0])
    return np.stack([np.stack([Z, -q[:, 2], q[:, 1]], -1),
                     np.stack([q[:, 2], Z, -q[:, 0]], -1),
                     np.stack([-q[:, 1], q[:, 0], Z], -1)], axis=1)


def linearise(T, src, src_cov, tgt, tgt_cov, r_max, tree=None):
    """One linearisation of Eq. MLE_for_T at pose T.

    src [n,3], src_cov [n,3,3], tgt [m,3], tgt_cov [m,3,3] (FP64).
    Returns (H[6,6], b[6], e, n_inliers, corr[n])."""
    R, t = T[:3, :3], T[:3, 3]
    q = src @ R.T + t
    j, _ = nearest_fp64(tgt, q, r_max, tree)
    ok = j >= 0
    n_in = int(ok.sum())
    H = np.zeros((6, 6))
    b = np.zeros(6)
    if n_in == 0:
        return H, b, 0.0, 0, j
    qi = q[ok]
    mu = tgt[j[ok]]
    d = mu - qi
    Sigma = tgt_cov[j[ok]] + R @ src_cov[ok] @ R.T
    M = np.linalg.inv(Sigma)
    J = np.concatenate([skew(qi), np.broadcast_to(-np.eye(3), (n_in, 3, 3))], axis=2)   # [n,3,6]
    MJ = M @ J
    H = np.einsum("nki,nkj->ij", J, MJ)
    Md = np.einsum("nij,nj->ni", M, d)
    b = np.einsum("nki,nk->i", J, Md)
    e = float(np.einsum("ni,ni->", d, Md))
    return H, b, e, n_in, j


def register(src, src_cov6, tgt, tgt_cov6, init, r_max=0.1, max_it=30,
             conv_rot=0.0, conv_trans=0.0, keep_history=False, tree=None) -> Result:
    """Gauss-Newton G-ICP.  Inputs are the FP32 arrays the GPU sees, read
    exactly into FP64; covariances in the [n,6] layout.  ``tree`` optionally
    supplies a prebuilt kd-tree of ``tgt`` (for repeated registrations against
    one map)."""
    src = np.asarray(src, np.float32).astype(np.float64)
    tgt = np.asarray(tgt, np.float32).astype(np.float64)
    Cs = from6(np.asarray(src_cov6, np.float32).astype(np.float64))
    Ct = from6(np.asarray(tgt_cov6, np.float32).astype(np.float64))
    if tree is None:
        tree = cKDTree(tgt)
    T = np.array(init, np.float64)
    H = np.zeros((6, 6))
    b = np.zeros(6)
    e, n_in = 0.0, 0
    hist = []
    for it in range(max_it):
        H, b, e, n_in, _ = linearise(T, src, Cs, tgt, Ct, r_max, tree)
        if n_in < 6:
            return Result(T, H, b, e, n_in, it + 1, False, E_NO_CORR, hist)
        sol = cholesky_solve(H, b)
        if sol is None:
            return Result(T, H, b, e, n_in, it + 1, False, E_DEGENERATE, hist)
        xi = -sol
        T = exp_se3(xi) @ T
        if keep_history:
            hist.append(T.copy())
        if np.linalg.norm(xi[:3]) < conv_rot and np.linalg.norm(xi[3:]) < conv_trans:
            return Result(T, H, b, e, n_in, it + 1, True, OK, hist)
    return Result(T, H, b, e, n_in, max_it, False, OK, hist)
