"""Oracle: per-point covariances and scale regularisation (test infrastructure only).

Paper, Sec. 3: the covariance C of a point x is the covariance matrix of its k
nearest neighbours.  Sec. 3.1.1 (Scale Regularization): C = R Lambda^2 R^T with
Lambda = diag(s2, s1, s0), s2 > s1 > s0 (for a symmetric PSD matrix the SVD is
its eigendecomposition, so ``numpy.linalg.eigh`` is used); the plane
regularisation replaces the scales by (1, 1, eps) so that each Gaussian is a
plane-like distribution; the ellipse regularisation divides the scales by
their median.

Readings (the paper is silent on these):
* the k neighbours include the point itself; the centre is the neighbourhood
  mean and the normalisation is 1/k;
* "eigenvalues (1,1,eps)" of the regularised covariance (the plane form used by
  the workloads): C_plane = v1 v1^T + v2 v2^T + eps v0 v0^T, v0 the eigenvector
  of the smallest eigenvalue;
* ellipse: the median of the three scales is the middle one, s1, so the
  covariance is divided by s1^2 = lambda1.

Layout: covariances are returned as [n,6] in the order xx, xy, xz, yy, yz, zz.
"""
from __future__ import annotations

import numpy as np

from .knn import knn

REG_NONE, REG_PLANE, REG_ELLIPSE = 0, 1, 2


def to6(C: np.ndarray) -> np.ndarray:
    return np.stack([C[..., 0, 0], C[..., 0, 1], C[..., 0, 2], C[..., 1, 1], C[..., 1, 2], C[..., 2, 2]], axis=-1)


def from6(c6: np.ndarray) -> np.ndarray:
    c6 = np.asarray(c6, np.float64)
    C = np.empty(c6.shape[:-1] + (3, 3))
    C[..., 0, 0] = c6[..., 0]
    C[..., 0, 1] = C[..., 1, 0] = c6[..., 1]
    C[..., 0, 2] = C[..., 2, 0] = c6[..., 2]
    C[..., 1, 1] = c6[..., 3]
    C[..., 1, 2] = C[..., 2, 1] = c6[..., 4]
    C[..., 2, 2] = c6[..., 5]
    return C


def neighbourhood_covariance(points: np.ndarray, nbr_idx: np.ndarray) -> np.ndarray:
    """C_i = (1/k) sum_j (p_j - mu_i)(p_j - mu_i)^T over the k neighbours j of
    point i, mu_i their mean.  points [n,3] (read exactly into FP64)."""
    P = np.asarray(points, np.float64)[nbr_idx]            # [n,k,3]
    mu = P.mean(axis=1, keepdims=True)
    D = P - mu
    return np.einsum("nki,nkj->nij", D, D) / nbr_idx.shape[1]


def regularise(C: np.ndarray, mode: int, eps: float = 1e-3) -> np.ndarray:
    """Scale regularisation of covariances C [n,3,3] (Sec. 3.1.1)."""
    if mode == REG_NONE:
        return C.copy()
    lam, V = np.linalg.eigh(C)                              # ascending: lam0 <= lam1 <= lam2
    if mode == REG_PLANE:
        scales2 = np.broadcast_to(np.array([eps, 1.0, 1.0]), lam.shape)
    elif mode == REG_ELLIPSE:
        # the median scale squared is the middle eigenvalue; where it vanishes
        # (all neighbours collinear) the paper's division is undefined: it is
        # clamped at 1e-6 of the largest eigenvalue, and an all-zero
        # covariance (all neighbours coincide) stays zero
        den = np.maximum(lam[:, 1:2], 1e-6 * lam[:, 2:3])
        with np.errstate(invalid="ignore", divide="ignore"):
            scales2 = np.where(den > 0, lam / np.where(den > 0, den, 1.0), 0.0)
    else:
        raise ValueError(f"unknown regularisation mode {mode}")
    return np.einsum("nij,nj,nkj->nik", V, scales2, V)


def covariances(points: np.ndarray, k: int, mode: int = REG_PLANE, eps: float = 1e-3,
                return_raw: bool = False):
    """Per-point regularised covariances [n,6] (FP64) of an FP32 cloud [n,3]."""
    points = np.asarray(points, np.float32)
    idx, _ = knn(points, points, k)
    C = neighbourhood_covariance(points, idx)
    out = to6(regularise(C, mode, eps))
    if return_raw:
        return out, C, idx
    return out


def eigen_gap(C: np.ndarray) -> np.ndarray:
    """(lambda1 - lambda0) / lambda2 of raw covariances [n,3,3]: how well the
    normal (smallest-eigenvalue direction) is determined."""
    lam = np.linalg.eigvalsh(C)
    with np.errstate(invalid="ignore", divide="ignore"):
        return np.where(lam[:, 2] > 0, (lam[:, 1] - lam[:, 0]) / lam[:, 2], 0.0)


def regularise6(c6: np.ndarray, mode: int, eps: float = 1e-3) -> np.ndarray:
    """``regularise`` on covariances in the [n,6] layout (used for map Gaussians
    that arrive with their own covariances, Sec. 3.1.1)."""
    return to6(regularise(from6(c6), mode, eps))
