"""Smooth camera trajectories and random rigid offsets."""
from __future__ import annotations

import numpy as np
from scipy.interpolate import CubicSpline
from scipy.spatial.transform import Rotation


def _look_rotation(yaw, pitch):
    """World-from-camera rotation for a camera looking along (yaw, pitch), world z up,
    camera x right, y down, z forward."""
    f = np.array([np.cos(yaw) * np.cos(pitch), np.sin(yaw) * np.cos(pitch), np.sin(pitch)])
    right = np.cross(f, [0.0, 0.0, 1.0])
    right /= np.linalg.norm(right)
    down = np.cross(f, right)
    return np.stack([right, down, f], axis=1)


def smooth_trajectory(seed: int, n_frames: int = 100, extent=(4.0, 4.0, 3.0),
                      max_step_m: float = 0.02, max_step_deg: float = 1.0, n_ctrl: int = 8,
                      inward: bool = False, ring: float = 1.5):
    """Camera poses T_wc [n,4,4] along a periodic cubic spline through random control
    points (position, yaw, pitch), re-timed so that no frame-to-frame step exceeds
    ``max_step_m`` of translation or ``max_step_deg`` of rotation.

    Default: control points within 0.75 m of the room centre, the view turning
    outward (yaw advancing around the loop).  ``inward``: control points on a
    ring of radius ``ring`` (+-0.2 m) around the centre, the camera facing the
    centre (+-0.35 rad of yaw wobble), so that every view holds the clutter of
    the room's middle in front of the far wall."""
    rng = np.random.default_rng(seed)
    ex, ey, ez = extent
    c = np.array([ex / 2, ey / 2, 1.5])
    if inward:
        phi = rng.uniform(0, 2 * np.pi) + 2 * np.pi * np.arange(n_ctrl) / n_ctrl
        rad = ring + rng.uniform(-0.2, 0.2, size=n_ctrl)
        P = c + np.stack([rad * np.cos(phi), rad * np.sin(phi), rng.uniform(-0.3, 0.3, size=n_ctrl)], 1)
    else:
        P = c + rng.uniform([-0.75, -0.75, -0.3], [0.75, 0.75, 0.3], size=(n_ctrl, 3))
    yaw0 = rng.uniform(0, 2 * np.pi)
    yaw_rate = 2 * np.pi / n_ctrl * rng.uniform(0.5, 1.0)
    wobble = np.append(rng.uniform(-0.35, 0.35, size=n_ctrl) if inward else rng.uniform(-0.4, 0.4, size=n_ctrl), 0.0)
    wobble[-1] = wobble[0]
    pitch = np.append(rng.uniform(-0.25, 0.1, size=n_ctrl), 0.0)
    pitch[-1] = pitch[0]
    s_ctrl = np.arange(n_ctrl + 1, dtype=float)
    P = np.vstack([P, P[:1]])
    sp = CubicSpline(s_ctrl, P, bc_type="periodic")
    sy = CubicSpline(s_ctrl, wobble, bc_type="periodic")
    sq = CubicSpline(s_ctrl, pitch, bc_type="periodic")

    def pose(s):
        T = np.eye(4)
        p = sp(s)
        if inward:
            yaw = np.arctan2(c[1] - p[1], c[0] - p[0]) + sy(s)
        else:
            yaw = yaw0 + yaw_rate * s + sy(s)
        T[:3, :3] = _look_rotation(yaw, sq(s))
        T[:3, 3] = p
        return T

    # re-time: walk along the periodic spline in small increments and emit a
    # frame whenever the next increment would break the per-frame bound (with a
    # 10% margin); the walk wraps around the loop as often as needed
    ds = n_ctrl / 20000.0
    poses = [pose(0.0)]
    last = poses[0]
    prev_T = last
    s_cur = 0.0
    while len(poses) < n_frames:
        s_cur += ds
        T = pose(s_cur % n_ctrl)
        dt = np.linalg.norm(T[:3, 3] - last[:3, 3])
        dr = np.degrees(Rotation.from_matrix(last[:3, :3].T @ T[:3, :3]).magnitude())
        if dt > 0.9 * max_step_m or dr > 0.9 * max_step_deg:
            poses.append(prev_T)
            last = prev_T
        prev_T = T
    return np.stack(poses)


def random_offset(rng: np.random.Generator, max_deg: float, max_m: float, exact: bool = False):
    """Rigid transform: rotation about a uniform random axis by an angle U(0,max_deg)
    (exactly max_deg if ``exact``), translation in a uniform random direction of
    magnitude U(0,max_m) (exactly max_m if ``exact``)."""
    axis = rng.standard_normal(3)
    axis /= np.linalg.norm(axis)
    ang = np.radians(max_deg if exact else rng.uniform(0, max_deg))
    dirn = rng.standard_normal(3)
    dirn /= np.linalg.norm(dirn)
    mag = max_m if exact else rng.uniform(0, max_m)
    T = np.eye(4)
    T[:3, :3] = Rotation.from_rotvec(axis * ang).as_matrix()
    T[:3, 3] = dirn * mag
    return T
