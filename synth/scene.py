"""Procedural indoor scenes made of rectangles and spheres.

A scene is a union of planar rectangles (room walls, box faces) and spheres.
It can be sampled area-uniformly (point clouds, map Gaussians) and ray-cast
(depth frames, see ``camera``).
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np


@dataclass
class Scene:
    # rectangles: corner o, edges u and v (3-vectors); the surface is o + a*u + b*v, a,b in [0,1]
    rect_o: np.ndarray = field(default_factory=lambda: np.zeros((0, 3)))
    rect_u: np.ndarray = field(default_factory=lambda: np.zeros((0, 3)))
    rect_v: np.ndarray = field(default_factory=lambda: np.zeros((0, 3)))
    # spheres: centre and radius
    sph_c: np.ndarray = field(default_factory=lambda: np.zeros((0, 3)))
    sph_r: np.ndarray = field(default_factory=lambda: np.zeros((0,)))
    extent: tuple = (4.0, 4.0, 3.0)

    def add_rect(self, o, u, v):
        self.rect_o = np.vstack([self.rect_o, np.asarray(o, float)[None]])
        self.rect_u = np.vstack([self.rect_u, np.asarray(u, float)[None]])
        self.rect_v = np.vstack([self.rect_v, np.asarray(v, float)[None]])

    def add_sphere(self, c, r):
        self.sph_c = np.vstack([self.sph_c, np.asarray(c, float)[None]])
        self.sph_r = np.append(self.sph_r, float(r))

    def add_box(self, lo, hi):
        lo = np.asarray(lo, float)
        hi = np.asarray(hi, float)
        d = hi - lo
        ex, ey, ez = np.diag(d)
        # six faces; edge order does not matter for sampling or ray casting
        self.add_rect(lo, ey, ez)
        self.add_rect(lo + ex, ey, ez)
        self.add_rect(lo, ex, ez)
        self.add_rect(lo + ey, ex, ez)
        self.add_rect(lo, ex, ey)
        self.add_rect(lo + ez, ex, ey)

    @property
    def rect_normal(self):
        n = np.cross(self.rect_u, self.rect_v)
        return n / np.linalg.norm(n, axis=1, keepdims=True)

    def areas(self):
        ra = np.linalg.norm(np.cross(self.rect_u, self.rect_v), axis=1)
        sa = 4.0 * np.pi * self.sph_r ** 2
        return ra, sa

    def total_area(self):
        ra, sa = self.areas()
        return float(ra.sum() + sa.sum())


def _room_walls(scene: Scene, ex: float, ey: float, ez: float):
    X = np.array([ex, 0, 0.0])
    Y = np.array([0, ey, 0.0])
    Z = np.array([0, 0, ez])
    o = np.zeros(3)
    scene.add_rect(o, X, Y)          # floor
    scene.add_rect(o + Z, X, Y)      # ceiling
    scene.add_rect(o, X, Z)          # wall y=0
    scene.add_rect(o + Y, X, Z)      # wall y=ey
    scene.add_rect(o, Y, Z)          # wall x=0
    scene.add_rect(o + X, Y, Z)      # wall x=ex


def make_room(seed: int, extent=(4.0, 4.0, 3.0), n_spheres: int = 3,
              r_range=(0.3, 0.6), centred: bool = True) -> Scene:
    """Axis-aligned room of the given extent plus spheres whose centres are drawn
    uniformly in the room shrunk by r+0.1 (so no sphere touches a wall).

    With ``centred`` the room is [-ex/2,ex/2]x[-ey/2,ey/2]x[-ez/2,ez/2], so that a
    rigid transform's rotation acts about the room centre; otherwise it is
    [0,ex]x[0,ey]x[0,ez]."""
    rng = np.random.default_rng(seed)
    ex, ey, ez = extent
    s = Scene(extent=tuple(extent))
    _room_walls(s, ex, ey, ez)
    for _ in range(n_spheres):
        r = rng.uniform(*r_range)
        m = r + 0.1
        c = rng.uniform([m, m, m], [ex - m, ey - m, ez - m])
        s.add_sphere(c, r)
    if centred:
        off = -0.5 * np.array([ex, ey, ez])
        s.rect_o = s.rect_o + off
        s.sph_c = s.sph_c + off
    return s


def _near_wall(rng, ex, ey, half, band):
    """(x, y) of an object's centre within ``band`` of a random vertical wall
    (its half-size ``half`` [2] keeps it inside the room)."""
    w = rng.integers(0, 4)
    off = rng.uniform(0.02, band)
    if w < 2:
        x = rng.uniform(half[0] + 0.05, ex - half[0] - 0.05)
        y = half[1] + off if w == 0 else ey - half[1] - off
    else:
        y = rng.uniform(half[1] + 0.05, ey - half[1] - 0.05)
        x = half[0] + off if w == 2 else ex - half[0] - off
    return x, y


def make_cluttered_room(seed: int, keep_clear: np.ndarray, extent=(4.0, 4.0, 3.0),
                        n_boxes: int = 20, n_spheres: int = 20, clearance: float = 0.3,
                        wall_band: float | None = None) -> Scene:
    """Room with axis-aligned boxes (sides U(0.1,0.6) m) and spheres (r U(0.1,0.4) m),
    each kept at least ``clearance`` from every point of ``keep_clear`` (the camera path).
    Objects are placed uniformly in the room, or, with ``wall_band``, within that
    distance of a random vertical wall (like furniture along the walls)."""
    rng = np.random.default_rng(seed)
    ex, ey, ez = extent
    s = Scene(extent=tuple(extent))
    _room_walls(s, ex, ey, ez)
    keep = np.asarray(keep_clear, float).reshape(-1, 3)
    placed = 0
    while placed < n_boxes:
        side = rng.uniform(0.1, 0.6, size=3)
        lo = rng.uniform([0.05, 0.05, 0.0], [ex - side[0] - 0.05, ey - side[1] - 0.05, ez - side[2] - 0.05])
        if wall_band is not None:
            x, y = _near_wall(rng, ex, ey, side[:2] / 2, wall_band)
            lo[:2] = [x - side[0] / 2, y - side[1] / 2]
        hi = lo + side
        # distance from camera path to the box
        d = np.linalg.norm(np.maximum(np.maximum(lo - keep, keep - hi), 0.0), axis=1)
        if d.min() < clearance:
            continue
        s.add_box(lo, hi)
        placed += 1
    placed = 0
    while placed < n_spheres:
        r = rng.uniform(0.1, 0.4)
        m = r + 0.05
        c = rng.uniform([m, m, m], [ex - m, ey - m, ez - m])
        if wall_band is not None:
            c[:2] = _near_wall(rng, ex, ey, np.array([r, r]), wall_band)
        d = np.linalg.norm(keep - c, axis=1) - r
        if d.min() < clearance:
            continue
        s.add_sphere(c, r)
        placed += 1
    return s


def sample_surface(scene: Scene, n: int, seed: int, noise_sigma: float = 0.0):
    """Area-uniform samples of the union of the scene's surfaces.

    Returns (points[n,3] float64, normals[n,3] float64).  Gaussian noise of
    ``noise_sigma`` metres is added independently to each coordinate."""
    rng = np.random.default_rng(seed)
    ra, sa = scene.areas()
    w = np.concatenate([ra, sa])
    which = rng.choice(len(w), size=n, p=w / w.sum())
    pts = np.empty((n, 3))
    nrm = np.empty((n, 3))
    nr = len(ra)
    is_rect = which < nr
    ir = which[is_rect]
    a = rng.random(ir.size)[:, None]
    b = rng.random(ir.size)[:, None]
    pts[is_rect] = scene.rect_o[ir] + a * scene.rect_u[ir] + b * scene.rect_v[ir]
    nrm[is_rect] = scene.rect_normal[ir]
    isp = which[~is_rect] - nr
    g = rng.standard_normal((isp.size, 3))
    g /= np.linalg.norm(g, axis=1, keepdims=True)
    pts[~is_rect] = scene.sph_c[isp] + scene.sph_r[isp, None] * g
    nrm[~is_rect] = g
    if noise_sigma > 0:
        pts += rng.normal(0.0, noise_sigma, size=pts.shape)
    return pts, nrm


def disc_covariances(normals: np.ndarray, seed: int, in_plane=(0.005, 0.015), normal_scale=0.001):
    """Flat, anisotropic Gaussians lying in the surface (the shape a trained
    Gaussian-splat map holds): random in-plane scales and orientation, a small
    scale along the surface normal.  Returns covariances [n,6] (xx,xy,xz,yy,yz,zz)."""
    rng = np.random.default_rng(seed)
    n = normals / np.linalg.norm(normals, axis=1, keepdims=True)
    helper = np.where(np.abs(n[:, 0:1]) < 0.9, np.array([[1.0, 0, 0]]), np.array([[0, 1.0, 0]]))
    t1 = np.cross(n, helper)
    t1 /= np.linalg.norm(t1, axis=1, keepdims=True)
    t2 = np.cross(n, t1)
    ang = rng.uniform(0, 2 * np.pi, size=(n.shape[0], 1))
    e1 = np.cos(ang) * t1 + np.sin(ang) * t2
    e2 = np.cross(n, e1)
    s1 = rng.uniform(*in_plane, size=(n.shape[0], 1))
    s2 = rng.uniform(*in_plane, size=(n.shape[0], 1))
    s3 = normal_scale
    C = (s1 ** 2)[:, :, None] * e1[:, :, None] * e1[:, None, :] \
        + (s2 ** 2)[:, :, None] * e2[:, :, None] * e2[:, None, :] \
        + (s3 ** 2) * n[:, :, None] * n[:, None, :]
    return np.stack([C[:, 0, 0], C[:, 0, 1], C[:, 0, 2], C[:, 1, 1], C[:, 1, 2], C[:, 2, 2]], axis=1)
