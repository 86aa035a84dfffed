"""Seeded synthetic workloads for the G-ICP tracking path.

This package generates inputs only: procedural indoor scenes, surface samples,
rendered depth frames, camera trajectories and batches of registration
problems.  It contains none of the registration method's arithmetic (no
neighbour search, no covariance estimation, no Gauss-Newton), so that the GPU
path and the CPU oracle can both consume its output without sharing any of
the computation they are compared on.

All generators are numpy, seeded, FP64 internally, and return FP32 arrays
where the method consumes them.
"""
from .scene import Scene, make_room, make_cluttered_room, sample_surface, disc_covariances
from .camera import Intrinsics, C2_INTRINSICS, render_depth, depth_to_points, voxel_downsample
from .trajectory import smooth_trajectory, random_offset
from .workloads import (
    Problem, C2Sequence, c1_problem, c2_sequence, c4_batch, c5_pairs, c5_trajectory,
    tiny_cloud, planar_patch,
)

__all__ = [
    "Scene", "make_room", "make_cluttered_room", "sample_surface", "disc_covariances",
    "Intrinsics", "C2_INTRINSICS", "render_depth", "depth_to_points", "voxel_downsample",
    "smooth_trajectory", "random_offset",
    "Problem", "C2Sequence", "c1_problem", "c2_sequence", "c4_batch", "c5_pairs",
    "c5_trajectory", "tiny_cloud", "planar_patch",
]
