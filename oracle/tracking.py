"""Oracle: frame-to-map tracking of a sequence (test infrastructure only).

Paper, Sec. 3 and Fig. 2: tracking registers every incoming frame against the
map by G-ICP (Eq. MLE_for_T), frame after frame.  The paper does not say where
each registration starts; the motion models here are readings:

* PREVIOUS: frame i starts from the estimate of frame i-1;
* CONSTANT_VELOCITY: frame i starts from T_{i-1} T_{i-2}^-1 T_{i-1} (the last
  estimated relative motion applied once more); frame 1 from frame 0's
  estimate.

Frame 0 starts from the given pose.  Each registration is ``gicp.register``.
"""
from __future__ import annotations

import numpy as np

from . import covariance as oc
from . import gicp as og

PREVIOUS, CONSTANT_VELOCITY = 0, 1


def rigid_inverse(T: np.ndarray) -> np.ndarray:
    Ti = np.eye(4)
    Ti[:3, :3] = T[:3, :3].T
    Ti[:3, 3] = -T[:3, :3].T @ T[:3, 3]
    return Ti


def predict(estimates, i: int, init: np.ndarray, motion: int) -> np.ndarray:
    """Initial pose of frame i from the estimates of frames 0..i-1."""
    if i == 0:
        return np.array(init, np.float64)
    b = estimates[i - 1]
    if motion == CONSTANT_VELOCITY and i >= 2:
        a = estimates[i - 2]
        return b @ (rigid_inverse(a) @ b)
    return np.array(b, np.float64)


def track(frames, map_means, map_covs6, init, motion=PREVIOUS, k=20, reg_mode=oc.REG_PLANE, eps=1e-3,
          r_max=0.1, max_it=20, conv=1e-6, tree=None, frame_covs=None):
    """Registers frames[0..] in order; returns (estimates, inits, results)."""
    from scipy.spatial import cKDTree
    if tree is None:
        tree = cKDTree(np.asarray(map_means, np.float32).astype(np.float64))
    est, inits, res = [], [], []
    for i, src in enumerate(frames):
        T0 = predict(est, i, init, motion)
        cs = frame_covs[i] if frame_covs is not None else oc.covariances(src, k, reg_mode, eps)
        r = og.register(src, cs, map_means, map_covs6, T0, r_max=r_max, max_it=max_it, conv_rot=conv,
                        conv_trans=conv, tree=tree)
        est.append(r.pose)
        inits.append(T0)
        res.append(r)
    return est, inits, res
