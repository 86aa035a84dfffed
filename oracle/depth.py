"""Oracle: depth image -> point cloud -> voxel downsampling (test
infrastructure only).

The paper's system overview (Sec. 3, Fig. 2) generates the tracking point
cloud by reprojecting the current depth image and downsampling it.  It names
neither the camera model nor the downsampling rule; the readings here are:

* pinhole back-projection of pixel (u, v) with depth z > 0:
      x = (u - cx) * z / fx,   y = (v - cy) * z / fy,   z = z
  evaluated in FP32 in exactly this order, left to right, each operation
  rounded (the voxel a point falls into is an integer decided by floating
  point, so both implementations take it in the same precision);
  pixels with z <= 0 or non-finite z are invalid;
* voxel downsampling: voxel (floor(x / s), floor(y / s), floor(z / s)) with
  FP32 division and floor; each occupied voxel yields the centroid of its
  points (FP64 mean, rounded to FP32 once);
* output order: voxels sorted by (ix, iy, iz) lexicographically.
"""
from __future__ import annotations

import numpy as np


def backproject(depth, fx, fy, cx, cy):
    """depth [H, W] -> valid points [n, 3] float32 in row-major pixel order."""
    d = np.asarray(depth, np.float32)
    H, W = d.shape
    v, u = np.meshgrid(np.arange(H, dtype=np.float32), np.arange(W, dtype=np.float32), indexing="ij")
    f32 = np.float32
    x = ((u - f32(cx)) * d) / f32(fx)
    y = ((v - f32(cy)) * d) / f32(fy)
    ok = np.isfinite(d) & (d > 0)
    return np.stack([x[ok], y[ok], d[ok]], axis=1).astype(np.float32)


def voxel_ids(points, voxel):
    p = np.asarray(points, np.float32)
    return np.floor(p / np.float32(voxel)).astype(np.int64)


def voxel_centroids(points, voxel):
    """Centroids [m, 3] float32 of the occupied voxels, sorted by (ix, iy, iz),
    and the number of points of each."""
    p = np.asarray(points, np.float32)
    if len(p) == 0:
        return np.zeros((0, 3), np.float32), np.zeros(0, np.int64)
    ids = voxel_ids(p, voxel)
    order = np.lexsort((ids[:, 2], ids[:, 1], ids[:, 0]))
    ids, q = ids[order], p[order].astype(np.float64)
    start = np.ones(len(ids), bool)
    start[1:] = np.any(ids[1:] != ids[:-1], axis=1)
    seg = np.cumsum(start) - 1
    m = int(seg[-1]) + 1
    cnt = np.bincount(seg, minlength=m)
    sums = np.stack([np.bincount(seg, weights=q[:, a], minlength=m) for a in range(3)], axis=1)
    return (sums / cnt[:, None]).astype(np.float32), cnt


def depth_to_points(depth, fx, fy, cx, cy, voxel):
    return voxel_centroids(backproject(depth, fx, fy, cx, cy), voxel)
