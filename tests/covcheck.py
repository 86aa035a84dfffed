"""Validity checks of GPU covariances against the oracle's FP64 neighbourhood
covariances (shared by the C1 and full-size parity tests).

Tolerances (derived from the FP32 arithmetic of the kernels): the raw moments
of k = 20 shifted neighbours carry an absolute error of at most about
120 u lambda_max (u = 2^-24: 20 rounded products and sums of terms bounded by
about 6 lambda_max), i.e. GAMMA lambda_max.
* PLANE, I - (1 - eps) n n^T: the normal tilts by that error over the eigen-
  gap, so points with a relative gap >= 0.02 are held to 1e-5; below the gate
  several normals are correct, and the GPU's must lie in the near-null space
  of the exact covariance: n^T C n <= lambda_1 + 1e-4 lambda_2.
* ELLIPSE, C / max(lambda_mid, 1e-6 lambda_max): the divisor's relative
  error is GAMMA lambda_max / lambda_mid, so every point is held to
  1e-5 + GAMMA lambda_max / den, and points with lambda_mid >= 0.1 lambda_max
  to the plain 1e-5."""
import numpy as np

from oracle import covariance as oc

U = 2.0 ** -24
GAMMA = 120 * U
GAP_GATE = 0.02


def rel_frob(A6, B6):
    A, B = oc.from6(np.asarray(A6, np.float64)), oc.from6(np.asarray(B6, np.float64))
    nb = np.linalg.norm(B, axis=(1, 2))
    na = np.linalg.norm(A - B, axis=(1, 2))
    return np.where(nb > 0, na / np.where(nb > 0, nb, 1.0), na)


def check_plane(got6, Craw, eps=1e-3):
    """Returns (max error of gated points, fraction gated, max excess of n^T C n)."""
    exp = oc.to6(oc.regularise(Craw, oc.REG_PLANE, eps))
    err = rel_frob(got6, exp)
    well = oc.eigen_gap(Craw) >= GAP_GATE
    assert err[well].max() < 1e-5, err[well].max()
    G = oc.from6(np.asarray(got6, np.float64))
    lam_g, V = np.linalg.eigh(G)
    assert np.allclose(lam_g, [eps, 1, 1], atol=2e-6)
    n = V[:, :, 0]
    nCn = np.einsum("ni,nij,nj->n", n, Craw, n)
    lam = np.linalg.eigvalsh(Craw)
    excess = (nCn - lam[:, 1]) / lam[:, 2]
    assert (excess <= 1e-4).all(), excess.max()
    return float(err[well].max()), float(well.mean()), float(excess.max())


def check_ellipse(got6, Craw):
    """Returns (max error where lambda_mid >= 0.1 lambda_max, max error / bound overall)."""
    exp = oc.to6(oc.regularise(Craw, oc.REG_ELLIPSE))
    err = rel_frob(got6, exp)
    lam = np.linalg.eigvalsh(Craw)
    den = np.maximum(lam[:, 1], 1e-6 * lam[:, 2])
    with np.errstate(divide="ignore", invalid="ignore"):
        bound = 1e-5 + GAMMA * np.where(den > 0, lam[:, 2] / np.where(den > 0, den, 1.0), 0.0)
    assert (err <= bound).all(), (err / bound).max()
    good = lam[:, 1] >= 0.1 * lam[:, 2]
    assert good.mean() > 0.5
    assert err[good].max() < 1e-5, err[good].max()
    return float(err[good].max()), float((err / bound).max())
