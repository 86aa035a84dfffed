"""The registration workloads, as seeded synthetic inputs.

* ``c1_problem``  — single registration: 5,000-point source and target resampled
  from a procedural room (6 planes, 3 spheres), sigma = 2 mm, target under a
  known rigid transform (5 deg about a random axis, 5 cm translation).
* ``c2_sequence`` — frame-to-map tracking: 1200x680 depth frames rendered along
  a 100-frame smooth trajectory in a room with 40 boxes and spheres, 1 % invalid
  pixels, sigma_z = 1 mm * z^2, voxel-downsampled at 2 cm (about 60k points);
  a 1M-Gaussian map of the same scene.
* ``c4_batch``    — 64 independent problems, source sizes log-uniform in
  [2k, 200k], targets log-uniform in [0.1M, 1M], initial offsets up to 10 cm and
  5 deg.
* ``c5_pairs``    — frame pairs along random trajectories (<= 8 cm, <= 4 deg per
  frame) for the learned warm start.

Every array the method consumes is FP32, structure-of-arrays friendly
(``[n,3]`` here; the bindings transpose to ``[3,n]``).
"""
from __future__ import annotations

from dataclasses import dataclass
from functools import lru_cache

import numpy as np

from .camera import C2_INTRINSICS, corrupt_depth, depth_to_points, render_depth, voxel_downsample
from .scene import disc_covariances, make_cluttered_room, make_room, sample_surface
from .trajectory import random_offset, smooth_trajectory


def _apply(T, p):
    return p @ T[:3, :3].T + T[:3, 3]


def _inv(T):
    Ti = np.eye(4)
    Ti[:3, :3] = T[:3, :3].T
    Ti[:3, 3] = -T[:3, :3].T @ T[:3, 3]
    return Ti


@dataclass
class Problem:
    """One registration: find T (source frame -> target frame), q = R x + t."""
    src: np.ndarray            # [n,3] float32, source frame
    tgt: np.ndarray            # [m,3] float32, target frame
    T_gt: np.ndarray           # [4,4] float64
    init: np.ndarray           # [4,4] float64
    tgt_cov_raw: np.ndarray | None = None   # [m,6] float32 map Gaussians (None: compute from kNN)
    seed: int = 0


def c1_problem(n: int = 5000, room_seed: int = 0, src_seed: int = 1, tgt_seed: int = 2,
               tf_seed: int = 3, noise: float = 0.002, deg: float = 5.0, metres: float = 0.05) -> Problem:
    room = make_room(room_seed)
    src, _ = sample_surface(room, n, src_seed, noise)
    tgt_w, _ = sample_surface(room, n, tgt_seed, noise)
    T = random_offset(np.random.default_rng(tf_seed), deg, metres, exact=True)
    tgt = _apply(T, tgt_w)
    return Problem(src.astype(np.float32), tgt.astype(np.float32), T, np.eye(4), None, room_seed)


class C2Sequence:
    """Frame-to-map tracking workload.  Frames are rendered lazily and cached."""

    def __init__(self, n_frames=100, scene_seed=10, traj_seed=14, map_seed=12,
                 map_size=1_000_000, voxel=0.02, K=C2_INTRINSICS, extent=(5.5, 5.0, 3.0), inward=False,
                 wall_band=None):
        self.K = K
        self.voxel = voxel
        self.poses = smooth_trajectory(traj_seed, n_frames, extent=extent, inward=inward)
        self.scene = make_cluttered_room(scene_seed, self.poses[:, :3, 3], extent=extent, wall_band=wall_band)
        mp, mn = sample_surface(self.scene, map_size, map_seed, noise_sigma=0.001)
        self.map_means = mp.astype(np.float32)
        self.map_cov_raw = disc_covariances(mn, map_seed + 1).astype(np.float32)
        self._frames = {}

    def __len__(self):
        return self.poses.shape[0]

    def frame(self, i: int) -> np.ndarray:
        """Camera-frame points [n,3] float32 of frame i (voxel centroids, sorted by voxel key)."""
        if i not in self._frames:
            d = render_depth(self.scene, self.poses[i], self.K)
            d = corrupt_depth(d, 100 + i, 200 + i)
            pts = voxel_downsample(depth_to_points(d, self.K), self.voxel)
            self._frames[i] = pts.astype(np.float32)
        return self._frames[i]

    def depth(self, i: int) -> np.ndarray:
        """Depth image [H, W] float32 of frame i (noise and invalid pixels applied)."""
        d = render_depth(self.scene, self.poses[i], self.K)
        return corrupt_depth(d, 100 + i, 200 + i).astype(np.float32)

    def prefetch(self, indices, workers: int = 8):
        """Render several frames in parallel worker processes (fork).  Call it
        before the process initialises the GPU runtime: a forked copy of a
        process with an initialised GPU runtime is not safe to run."""
        import concurrent.futures as cf
        import multiprocessing as mp
        todo = [i for i in indices if i not in self._frames]
        if not todo:
            return
        ctx = mp.get_context("fork")
        with cf.ProcessPoolExecutor(max_workers=max(1, min(workers, len(todo))), mp_context=ctx) as ex:
            for i, pts in zip(todo, ex.map(self.frame, todo)):
                self._frames[i] = pts

    def cv_init(self, est_poses, i: int) -> np.ndarray:
        """Constant-velocity initial pose from the previous two estimates
        (frame 0: ground truth; frame 1: the previous estimate)."""
        if i == 0:
            return self.poses[0].copy()
        if i == 1:
            return est_poses[0].copy()
        a, b = est_poses[i - 2], est_poses[i - 1]
        return b @ (_inv(a) @ b)


@lru_cache(maxsize=2)
def c2_sequence(n_frames=100, map_size=1_000_000) -> C2Sequence:
    return C2Sequence(n_frames=n_frames, map_size=map_size)


def c4_batch(n_prob: int = 64, seed0: int = 4000, ns_range=(2_000, 200_000),
             m_range=(100_000, 1_000_000), max_deg=5.0, max_m=0.10, sizes_only=False):
    """Batch of independent problems.  Target Gaussians: area-uniform room samples
    (sigma 1 mm) with flat disc covariances; source: an independent resample
    (sigma 2 mm) expressed in a frame offset by T_gt."""
    out = []
    for i in range(n_prob):
        rng = np.random.default_rng(seed0 + i)
        ns = int(np.exp(rng.uniform(np.log(ns_range[0]), np.log(ns_range[1]))))
        m = int(np.exp(rng.uniform(np.log(m_range[0]), np.log(m_range[1]))))
        if sizes_only:
            out.append((ns, m))
            continue
        room = make_room(seed0 + i)
        tp, tn = sample_surface(room, m, seed0 + i + 100_000, 0.001)
        sp, _ = sample_surface(room, ns, seed0 + i + 200_000, 0.002)
        T = random_offset(rng, max_deg, max_m)
        src = _apply(_inv(T), sp)
        out.append(Problem(src.astype(np.float32), tp.astype(np.float32), T, np.eye(4),
                           disc_covariances(tn, seed0 + i + 300_000).astype(np.float32), seed0 + i))
    return out


def c5_trajectory(seed: int, n_frames: int = 101, n_points: int = 5000,
                  max_m: float = 0.08, max_deg: float = 4.0):
    """Frames of one learned-warm-start trajectory: each frame is an independent
    resample of a room (sigma 2 mm) expressed in the body frame T_k^-1.  The
    motion is a smoothed random walk with steps bounded by max_m / max_deg.
    Returns (frames [n_frames,n_points,3] float32, poses [n_frames,4,4])."""
    from scipy.spatial.transform import Rotation
    rng = np.random.default_rng(seed)
    room = make_room(seed)
    poses = [np.eye(4)]
    v = rng.uniform(-1, 1, 3) * max_m * 0.5
    w = rng.uniform(-1, 1, 3) * np.radians(max_deg) * 0.5
    for _ in range(n_frames - 1):
        v = 0.8 * v + 0.2 * rng.uniform(-1, 1, 3) * max_m
        w = 0.8 * w + 0.2 * rng.uniform(-1, 1, 3) * np.radians(max_deg)
        vn, wn = np.linalg.norm(v), np.linalg.norm(w)
        if vn > max_m:
            v *= max_m / vn
        if wn > np.radians(max_deg):
            w *= np.radians(max_deg) / wn
        step = np.eye(4)
        step[:3, :3] = Rotation.from_rotvec(w).as_matrix()
        step[:3, 3] = v
        poses.append(poses[-1] @ step)
    frames = np.empty((n_frames, n_points, 3), np.float32)
    for k in range(n_frames):
        p, _ = sample_surface(room, n_points, seed * 1000 + k, 0.002)
        frames[k] = _apply(_inv(poses[k]), p).astype(np.float32)
    return frames, np.stack(poses)


def c5_pairs(seed: int, n_frames: int = 101, n_points: int = 5000):
    """Consecutive frame pairs of one trajectory: pair k registers frame k+1
    (source) against frame k (target); ground-truth relative pose T_k^-1 T_{k+1}."""
    frames, poses = c5_trajectory(seed, n_frames, n_points)
    rel = np.stack([_inv(poses[k]) @ poses[k + 1] for k in range(n_frames - 1)])
    return frames, rel


def tiny_cloud(n: int, seed: int, duplicates: int = 0, lattice: bool = False):
    """Small clouds for exhaustive kNN checks: uniform in a 1 m cube, optionally
    on an integer lattice scaled to 0.1 m (many exactly equal distances), with
    ``duplicates`` exact copies of existing points appended."""
    rng = np.random.default_rng(seed)
    if lattice:
        p = rng.integers(0, 6, size=(n, 3)).astype(np.float64) * 0.125
    else:
        p = rng.random((n, 3))
    if duplicates:
        idx = rng.integers(0, n, size=duplicates)
        p = np.vstack([p, p[idx]])
    return p.astype(np.float32)


def planar_patch(n: int, seed: int, normal=(0.0, 0.0, 1.0), centre=(0.5, -0.3, 2.0), size=0.3):
    """Noise-free points on a plane through ``centre`` with the given normal."""
    rng = np.random.default_rng(seed)
    nrm = np.asarray(normal, float)
    nrm /= np.linalg.norm(nrm)
    helper = np.array([1.0, 0, 0]) if abs(nrm[0]) < 0.9 else np.array([0, 1.0, 0])
    t1 = np.cross(nrm, helper)
    t1 /= np.linalg.norm(t1)
    t2 = np.cross(nrm, t1)
    ab = rng.uniform(-size, size, size=(n, 2))
    p = np.asarray(centre, float) + ab[:, :1] * t1 + ab[:, 1:] * t2
    return p, nrm
