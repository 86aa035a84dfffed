"""Pinhole depth rendering of procedural scenes, back-projection and voxel
downsampling (the frame generator of the frame-to-map tracking workload).

Camera convention: x right, y down, z forward; a pose T_wc maps camera
coordinates into the world (p_w = R p_c + t).  Depth is the z coordinate in
the camera frame (not the range along the ray).
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from .scene import Scene


@dataclass(frozen=True)
class Intrinsics:
    width: int
    height: int
    fx: float
    fy: float
    cx: float
    cy: float


C2_INTRINSICS = Intrinsics(1200, 680, 600.0, 600.0, 599.5, 339.5)


def _pixel_rays(K: Intrinsics):
    u = np.arange(K.width, dtype=np.float64)
    v = np.arange(K.height, dtype=np.float64)
    uu, vv = np.meshgrid(u, v)
    # ray with unit z so that the ray parameter equals the depth
    return np.stack([(uu - K.cx) / K.fx, (vv - K.cy) / K.fy, np.ones_like(uu)], axis=-1)


def _project_bounds(K, c_cam, r):
    """Conservative pixel rectangle covering a sphere (centre c_cam in the camera
    frame, radius r).  None if entirely behind the camera."""
    x, y, z = c_cam
    if z + r <= 1e-3:
        return None
    if z - r <= 1e-3:
        return 0, K.width, 0, K.height
    us = [K.fx * (x + sx * r) / (z + sz * r) + K.cx for sx in (-1, 1) for sz in (-1, 1)]
    vs = [K.fy * (y + sy * r) / (z + sz * r) + K.cy for sy in (-1, 1) for sz in (-1, 1)]
    u0 = max(int(np.floor(min(us))) - 1, 0)
    u1 = min(int(np.ceil(max(us))) + 2, K.width)
    v0 = max(int(np.floor(min(vs))) - 1, 0)
    v1 = min(int(np.ceil(max(vs))) + 2, K.height)
    if u0 >= u1 or v0 >= v1:
        return None
    return u0, u1, v0, v1


def render_depth(scene: Scene, T_wc: np.ndarray, K: Intrinsics = C2_INTRINSICS):
    """Ray-cast depth image (float64 metres, 0 where nothing is hit).

    Every rectangle of the procedural scenes is axis-aligned, which keeps the
    ray-plane test to a division and two range checks per pixel."""
    R = T_wc[:3, :3]
    t = T_wc[:3, 3]
    Rt = R.T
    rays_c = _pixel_rays(K)
    d_all = rays_c @ Rt                          # world directions [H,W,3]
    with np.errstate(divide="ignore"):
        inv_all = 1.0 / d_all
    depth = np.full((K.height, K.width), np.inf)

    for i in range(scene.rect_o.shape[0]):
        o, u, v = scene.rect_o[i], scene.rect_u[i], scene.rect_v[i]
        n = np.cross(u, v)
        a = int(np.argmax(np.abs(n)))
        if np.count_nonzero(np.abs(n) > 1e-12) != 1:
            raise ValueError("render_depth handles axis-aligned rectangles only")
        lo = np.minimum(o, o + u + v)
        hi = np.maximum(o, o + u + v)
        centre = 0.5 * (lo + hi)
        rad = 0.5 * np.linalg.norm(hi - lo)
        b = _project_bounds(K, Rt @ (centre - t), rad)
        if b is None:
            continue
        u0, u1, v0, v1 = b
        d = d_all[v0:v1, u0:u1]
        s = (o[a] - t[a]) * inv_all[v0:v1, u0:u1, a]
        ok = s > 1e-6
        for ax in range(3):
            if ax == a:
                continue
            h = t[ax] + s * d[..., ax]
            ok &= (h >= lo[ax]) & (h <= hi[ax])
        sub = depth[v0:v1, u0:u1]
        upd = ok & (s < sub)
        sub[upd] = s[upd]

    for i in range(scene.sph_c.shape[0]):
        c, r = scene.sph_c[i], scene.sph_r[i]
        b = _project_bounds(K, Rt @ (c - t), r)
        if b is None:
            continue
        u0, u1, v0, v1 = b
        d = d_all[v0:v1, u0:u1]
        oc = t - c
        A = np.einsum("...k,...k->...", d, d)
        B = d @ oc
        Cc = oc @ oc - r * r
        disc = B * B - A * Cc
        ok = disc > 0
        sq = np.sqrt(np.where(ok, disc, 0.0))
        s0 = (-B - sq) / A
        s1 = (-B + sq) / A
        s = np.where(s0 > 1e-6, s0, s1)
        ok &= s > 1e-6
        sub = depth[v0:v1, u0:u1]
        upd = ok & (s < sub)
        sub[upd] = s[upd]

    depth[~np.isfinite(depth)] = 0.0
    return depth


def corrupt_depth(depth: np.ndarray, noise_seed: int, invalid_seed: int,
                  sigma_coeff: float = 0.001, invalid_frac: float = 0.01):
    """Axial noise sigma = sigma_coeff * z^2 and a random fraction of invalid (0) pixels."""
    rng = np.random.default_rng(noise_seed)
    z = depth.copy()
    valid = z > 0
    z[valid] += rng.standard_normal(valid.sum()) * sigma_coeff * z[valid] ** 2
    rng2 = np.random.default_rng(invalid_seed)
    kill = rng2.random(z.shape) < invalid_frac
    z[kill] = 0.0
    z[z < 0] = 0.0
    return z


def depth_to_points(depth: np.ndarray, K: Intrinsics = C2_INTRINSICS):
    """Back-project valid pixels to camera-frame points [n,3] float64."""
    vv, uu = np.nonzero(depth > 0)
    z = depth[vv, uu]
    x = (uu - K.cx) / K.fx * z
    y = (vv - K.cy) / K.fy * z
    return np.stack([x, y, z], axis=1)


def voxel_downsample(points: np.ndarray, voxel: float):
    """Centroid of the points falling in each voxel of a grid anchored at the
    origin; output sorted by voxel key (x fastest)."""
    ijk = np.floor(points / voxel).astype(np.int64)
    ijk -= ijk.min(axis=0)
    dims = ijk.max(axis=0) + 1
    key = ijk[:, 0] + dims[0] * (ijk[:, 1] + dims[1] * ijk[:, 2])
    uniq, inv = np.unique(key, return_inverse=True)
    cnt = np.bincount(inv).astype(np.float64)
    out = np.empty((uniq.size, 3))
    for a in range(3):
        out[:, a] = np.bincount(inv, weights=points[:, a]) / cnt
    return out
