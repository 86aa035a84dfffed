"""Oracle: keyframe decision, scale aligning and the Gaussians a keyframe adds
to the map (test infrastructure only).

Paper, Sec. 3.1.2 (Keyframe Selection): the proportion of source points that
have a correspondence in the map (a map Gaussian within the distance
threshold at the estimated pose, a by-product of G-ICP) decides keyframes: a
frame whose proportion falls below a threshold is a keyframe.  Only the
frame's Gaussians that do not overlap the existing map are added to it.

Paper, Sec. 3.2.1 (Scale Aligning): before insertion the scales of a frame's
Gaussians are normalised by depth, Lambda'' = Lambda' / z^p, where Lambda' is
the ellipse-regularised scale (Sec. 3.1.1); the ablation (Table: scale
aligning) selects p = 1.5.  With C = R Lambda^2 R^T this divides the
covariance by z^(2p).

Paper, Sec. 3.2.2 (Additional Keyframe Selection for Mapping): besides the
tracking keyframes, mapping-only keyframes are taken at a shorter interval,
and a tracking keyframe is forced when none was selected for a longer one
(the text uses 10 and 30 frames).

Readings: z is the point's depth in the camera frame (the distance along the
optical axis; a point with z <= 0 keeps its covariance); a correspondence is the exact nearest map mean within the
threshold, distances in FP64; the inserted Gaussians keep the frame's point
order; a frame that is a tracking keyframe is not also counted as a
mapping-only keyframe.
"""
from __future__ import annotations

import numpy as np
from scipy.spatial import cKDTree

from . import covariance as oc

KEYFRAME = 1
MAPPING_ONLY = 2


def scale_align(covs6, z, p=1.5):
    """C'' = C' / z^(2p) for covariances [n, 6] and depths z [n] (a point
    with z <= 0, which no depth image produces, keeps its covariance)."""
    z = np.asarray(z, np.float64)
    f = np.ones_like(z)
    pos = z > 0
    f[pos] = z[pos] ** (-2.0 * p)
    return np.asarray(covs6, np.float64) * f[:, None]


def overlap_flags(src, pose, map_means, r):
    """True where R x + t has a map mean within distance r (inclusive)."""
    T = np.asarray(pose, np.float64)
    q = np.asarray(src, np.float64) @ T[:3, :3].T + T[:3, 3]
    d, _ = cKDTree(np.asarray(map_means, np.float64)).query(q, k=1)
    return d <= r


def keyframe_gaussians(src, src_covs6, pose, map_means, r, p=1.5):
    """(inlier ratio, means [m, 3], covariances [m, 6]) of the Gaussians a
    keyframe adds: the points without a correspondence, scale aligned in the
    camera frame, then moved into the map frame (mu = R x + t, C = R C R^T)."""
    src = np.asarray(src, np.float64)
    flags = overlap_flags(src, pose, map_means, r)
    ratio = float(flags.mean()) if len(flags) else 0.0
    keep = ~flags
    T = np.asarray(pose, np.float64)
    R, t = T[:3, :3], T[:3, 3]
    C = oc.from6(scale_align(np.asarray(src_covs6)[keep], src[keep, 2], p))
    Cw = np.einsum("ij,njk,lk->nil", R, C, R)
    return ratio, src[keep] @ R.T + t, oc.to6(Cw)


def keyframe_policy(ratio, since_keyframe, since_mapping, threshold, max_gap=30, mapping_gap=10):
    """Bit flags of a frame: KEYFRAME when the correspondence ratio is below
    the threshold or max_gap frames passed since the last keyframe;
    MAPPING_ONLY when mapping_gap frames passed since the last keyframe of
    either kind and the frame is not a keyframe."""
    if ratio < threshold or since_keyframe >= max_gap:
        return KEYFRAME
    if since_mapping >= mapping_gap:
        return MAPPING_ONLY
    return 0
