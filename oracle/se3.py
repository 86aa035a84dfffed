"""Oracle: SE(3) exponential and SO(3) logarithm (test infrastructure only).

The pose update of the Gauss-Newton iteration is the left perturbation
T <- Exp(xi) T with xi = [omega; v] (rotation first).  The paper states only
the objective (Sec. 3, Eq. MLE_for_T); the closed forms below are the standard
Rodrigues / left-Jacobian expressions, with Taylor expansions for small angles.
"""
from __future__ import annotations

import numpy as np


def hat(w: np.ndarray) -> np.ndarray:
    """Skew matrix [w]x with [w]x u = w x u."""
    return np.array([[0.0, -w[2], w[1]], [w[2], 0.0, -w[0]], [-w[1], w[0], 0.0]])


def exp_se3(xi: np.ndarray) -> np.ndarray:
    """4x4 exponential of the twist xi = [omega; v]:
    R = I + A W + B W^2,  t = (I + B W + C W^2) v,  W = [omega]x, theta = |omega|,
    A = sin(theta)/theta, B = (1 - cos(theta))/theta^2, C = (theta - sin(theta))/theta^3."""
    xi = np.asarray(xi, np.float64)
    w, v = xi[:3], xi[3:]
    th2 = float(w @ w)
    th = np.sqrt(th2)
    if th < 1e-4:
        A = 1.0 - th2 / 6.0 + th2 * th2 / 120.0
        B = 0.5 - th2 / 24.0 + th2 * th2 / 720.0
        C = 1.0 / 6.0 - th2 / 120.0 + th2 * th2 / 5040.0
    else:
        A = np.sin(th) / th
        B = (1.0 - np.cos(th)) / th2
        C = (th - np.sin(th)) / (th2 * th)
    W = hat(w)
    W2 = W @ W
    T = np.eye(4)
    T[:3, :3] = np.eye(3) + A * W + B * W2
    T[:3, 3] = (np.eye(3) + B * W + C * W2) @ v
    return T


def log_so3(R: np.ndarray) -> np.ndarray:
    """Rotation vector of R (angle in [0, pi])."""
    c = np.clip((np.trace(R) - 1.0) / 2.0, -1.0, 1.0)
    th = np.arccos(c)
    wv = np.array([R[2, 1] - R[1, 2], R[0, 2] - R[2, 0], R[1, 0] - R[0, 1]])
    if th < 1e-7:
        return 0.5 * wv
    if np.pi - th < 1e-6:
        # near pi: axis from the symmetric part
        M = (R + np.eye(3)) / 2.0
        a = int(np.argmax(np.diag(M)))
        axis = M[:, a] / np.sqrt(M[a, a])
        return axis * th
    return th / (2.0 * np.sin(th)) * wv


def inv(T: np.ndarray) -> np.ndarray:
    Ti = np.eye(4)
    Ti[:3, :3] = T[:3, :3].T
    Ti[:3, 3] = -T[:3, :3].T @ T[:3, 3]
    return Ti


def pose_error(Ta: np.ndarray, Tb: np.ndarray):
    """(rotation error [rad], translation error [m]) between two poses:
    |Log(Ra^T Rb)| and |ta - tb|."""
    dr = float(np.linalg.norm(log_so3(Ta[:3, :3].T @ Tb[:3, :3])))
    dt = float(np.linalg.norm(Ta[:3, 3] - Tb[:3, 3]))
    return dr, dt
