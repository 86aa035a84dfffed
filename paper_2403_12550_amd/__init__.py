"""MI355X (gfx950) G-ICP tracking: thin Python binding of libgicp.so.

Every step of the tracking path runs in the HIP kernels of libgicp.so; this
module only marshals arguments.  PyTorch supplies device memory and the
current stream.  Arrays use the library's structure-of-arrays layouts:
points [3, n] float32, covariances [6, n] float32 (xx, xy, xz, yy, yz, zz).
There is no CPU fallback: if the library is missing, every call raises.
"""
from __future__ import annotations

import ctypes as C
from dataclasses import dataclass

import numpy as np

from . import _abi
from ._abi import (ACC_FP32, ACC_FP64, ACC_TWOSUM, FLAG_GRAPH, FLAG_MULTI_LAUNCH, FLAG_NO_REUSE, FLAG_QUEUE,
                   MOTION_CONSTANT_VELOCITY, MOTION_PREVIOUS, REG_ELLIPSE, REG_NONE, REG_PLANE, GICP_OK, Frame, Params,
                   Problem, Stats)

__all__ = ["Context", "Map", "Params", "Stats", "Problem", "RegisterResult", "GicpError", "params",
           "REG_NONE", "REG_PLANE", "REG_ELLIPSE", "ACC_TWOSUM", "ACC_FP32", "ACC_FP64", "FLAG_MULTI_LAUNCH", "FLAG_QUEUE", "FLAG_GRAPH",
           "FLAG_NO_REUSE", "MOTION_PREVIOUS", "MOTION_CONSTANT_VELOCITY",
           "to_soa", "lib"]


class GicpError(RuntimeError):
    def __init__(self, status: int, what: str = ""):
        self.status = status
        msg = lib().gicp_strerror(status).decode()
        super().__init__(f"{what}: {msg} (status {status})" if what else msg)


def lib():
    return _abi.load()


def params(**kw) -> Params:
    """gicp_params with the library defaults, overridden by keyword."""
    p = Params()
    lib().gicp_params_default(C.byref(p))
    for k, v in kw.items():
        if not hasattr(p, k):
            raise AttributeError(k)
        setattr(p, k, v)
    return p


# numpy views of the batched call's C structs (same field order, sizes and
# alignment as gicp_problem and gicp_stats), filled column by column
_PROBLEM_DT = np.dtype([("src", np.uint64), ("src_covs", np.uint64), ("n", np.int64), ("map", np.uint64),
                        ("init_pose", np.float64, (16,))])
_STATS_DT = np.dtype([("iters", np.int32), ("n_inliers", np.int32), ("cost", np.float64), ("converged", np.int32),
                      ("status", np.int32), ("hip_error", np.int32), ("reserved", np.int32)])
assert _PROBLEM_DT.itemsize == C.sizeof(Problem) and _STATS_DT.itemsize == C.sizeof(Stats)


def _ptr(t) -> int:
    return 0 if t is None else int(t.data_ptr())


def _check_f32_cuda(t, rows: int, name: str):
    import torch
    if t.dtype != torch.float32 or not t.is_cuda or not t.is_contiguous() or t.dim() != 2 or t.shape[0] != rows:
        raise ValueError(f"{name} must be a contiguous float32 CUDA tensor of shape [{rows}, n]")


def to_soa(pts, device="cuda"):
    """[n,3] (numpy or torch) -> contiguous float32 [3,n] on the device."""
    import torch
    t = torch.as_tensor(pts, dtype=torch.float32)
    return t.t().contiguous().to(device)


def _stream():
    import torch
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


@dataclass
class RegisterResult:
    pose: np.ndarray
    H: np.ndarray
    b: np.ndarray
    iters: int
    n_inliers: int
    cost: float
    converged: bool
    status: int


class Map:
    """Cell-sorted map Gaussians and their hash table (owned by the library)."""

    def __init__(self, handle: C.c_void_p, m: int, cell: float):
        self.handle = handle
        self.m = m
        self.cell = cell

    def close(self):
        if self.handle:
            lib().gicp_map_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Context:
    def __init__(self, device: int = 0):
        self.device = device
        h = C.c_void_p()
        st = lib().gicp_create(C.byref(h), device)
        if st != GICP_OK:
            raise GicpError(st, "gicp_create")
        self.handle = h

    def close(self):
        if getattr(self, "handle", None):
            lib().gicp_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def profile(self, enable: bool = True):
        """Enable (and reset) or disable the library's HIP-event kernel timing."""
        st = lib().gicp_profile(self.handle, int(enable))
        if st != GICP_OK:
            raise GicpError(st, "gicp_profile")

    def profile_read(self, group: int):
        """(launches that did work, summed milliseconds, work units) of a kernel group."""
        n = C.c_int64()
        ms = C.c_double()
        u = C.c_double()
        st = lib().gicp_profile_read(self.handle, group, C.byref(n), C.byref(ms), C.byref(u))
        if st != GICP_OK:
            raise GicpError(st, "gicp_profile_read")
        return int(n.value), float(ms.value), float(u.value)

    def sync_status(self) -> int:
        return lib().gicp_sync_status(self.handle, _stream())

    def estimate_cell(self, pts, k: int) -> float:
        _check_f32_cuda(pts, 3, "pts")
        c = C.c_float()
        st = lib().gicp_estimate_cell(self.handle, _ptr(pts), pts.shape[1], k, C.byref(c), _stream())
        if st != GICP_OK:
            raise GicpError(st, "gicp_estimate_cell")
        return float(c.value)

    def knn(self, pts, queries, k: int, cell: float = 0.0, r_max: float = 0.0, out=None):
        import torch
        _check_f32_cuda(pts, 3, "pts")
        _check_f32_cuda(queries, 3, "queries")
        nq = queries.shape[1]
        if out is None:
            idx = torch.empty((nq, k), dtype=torch.int32, device=pts.device)
            d2 = torch.empty((nq, k), dtype=torch.float32, device=pts.device)
        else:
            idx, d2 = out
        st = lib().gicp_knn(self.handle, _ptr(pts), pts.shape[1], _ptr(queries), nq, k, cell, r_max,
                            _ptr(idx), _ptr(d2), _stream())
        if st != GICP_OK:
            raise GicpError(st, "gicp_knn")
        return idx, d2

    def covariances(self, pts, k: int = 20, cell: float = 0.0, reg_mode: int = REG_PLANE, eps: float = 1e-3,
                    out=None):
        import torch
        _check_f32_cuda(pts, 3, "pts")
        n = pts.shape[1]
        covs = torch.empty((6, n), dtype=torch.float32, device=pts.device) if out is None else out
        st = lib().gicp_covariances(self.handle, _ptr(pts), n, k, cell, reg_mode, eps, _ptr(covs), _stream())
        if st != GICP_OK:
            raise GicpError(st, "gicp_covariances")
        return covs

    def covariances_noalloc(self, pts, k: int = 20, cell: float = 0.0, reg_mode: int = REG_PLANE,
                            eps: float = 1e-3, out=None):
        """covariances() through the entry point that allocates nothing (fixed
        per-GPU workspace, at most NOALLOC_MAX_POINTS points)."""
        import torch
        _check_f32_cuda(pts, 3, "pts")
        n = pts.shape[1]
        covs = torch.empty((6, n), dtype=torch.float32, device=pts.device) if out is None else out
        st = lib().gicp_covariances_noalloc(self.handle, _ptr(pts), n, k, cell, reg_mode, eps, _ptr(covs),
                                            _stream())
        if st != GICP_OK:
            raise GicpError(st, "gicp_covariances_noalloc")
        return covs

    def map_build(self, means, covs, cell: float = 0.0, reg_mode: int = REG_NONE, eps: float = 1e-3) -> Map:
        _check_f32_cuda(means, 3, "means")
        _check_f32_cuda(covs, 6, "covs")
        h = C.c_void_p()
        st = lib().gicp_map_build(self.handle, _ptr(means), _ptr(covs), means.shape[1], cell, reg_mode, eps,
                                  C.byref(h), _stream())
        if st != GICP_OK:
            raise GicpError(st, "gicp_map_build")
        m = C.c_int64()
        c = C.c_float()
        lib().gicp_map_info(h, C.byref(m), C.byref(c))
        return Map(h, int(m.value), float(c.value))

    def map_nearest(self, gmap: Map, queries, r_max: float, hints=None, want_radius: bool = False,
                    lanes: int = 0):
        """Nearest map mean of each query [3, nq] (map frame) within r_max by the
        registration's own search (lanes per query: 0 or 2 as two-lane
        launches, 4, 8 or 16 as four-lane ones such as tracking): (idx int32 [nq],
        d2 float32 [nq], radius or None)."""
        import torch
        _check_f32_cuda(queries, 3, "queries")
        nq = queries.shape[1]
        if hints is not None and (hints.dtype != torch.int32 or not hints.is_cuda or hints.numel() != nq
                                  or not hints.is_contiguous()):
            raise ValueError("hints must be a contiguous int32 CUDA tensor of nq entries")
        idx = torch.empty(nq, dtype=torch.int32, device=queries.device)
        d2 = torch.empty(nq, dtype=torch.float32, device=queries.device)
        rad = torch.empty(nq, dtype=torch.float32, device=queries.device) if want_radius else None
        st = lib().gicp_map_nearest(self.handle, gmap.handle, _ptr(queries), nq, r_max, _ptr(hints), _ptr(idx),
                                    _ptr(d2), _ptr(rad), int(lanes), _stream())
        if st != GICP_OK:
            raise GicpError(st, "gicp_map_nearest")
        return idx, d2, rad

    def register(self, src, gmap: Map, init_pose, prm: Params | None = None, src_covs=None,
                 src_covs_out=None, raise_on_error: bool = False) -> RegisterResult:
        _check_f32_cuda(src, 3, "src")
        if src_covs is not None:
            _check_f32_cuda(src_covs, 6, "src_covs")
        if src_covs_out is not None:
            _check_f32_cuda(src_covs_out, 6, "src_covs_out")
        prm = prm or params()
        init = _abi.D16(*np.asarray(init_pose, np.float64).reshape(16))
        pose, H, b = _abi.D16(), _abi.D36(), _abi.D6()
        stats = Stats()
        st = lib().gicp_register(self.handle, _ptr(src), _ptr(src_covs), src.shape[1], gmap.handle, init,
                                 C.byref(prm), pose, H, b, _ptr(src_covs_out), C.byref(stats), _stream())
        if st == _abi.GICP_E_ARG or st in (_abi.GICP_E_HIP, _abi.GICP_E_OOM) or (raise_on_error and st != GICP_OK):
            raise GicpError(st, "gicp_register")
        return RegisterResult(np.array(pose[:]).reshape(4, 4), np.array(H[:]).reshape(6, 6), np.array(b[:]),
                              stats.iters, stats.n_inliers, stats.cost, bool(stats.converged), st)

    def register_dev(self, src, gmap: Map, init_pose, pose, H, b, prm: Params | None = None, src_covs=None,
                     src_covs_out=None, stats=None):
        """gicp_register_dev: init_pose [16] float64, pose [16], H [36], b [6]
        float64 and stats (a uint8 tensor of sizeof(gicp_stats) bytes, or
        None) are CUDA tensors; nothing is synchronised or copied to the host."""
        import torch
        _check_f32_cuda(src, 3, "src")
        for t, k, name in ((init_pose, 16, "init_pose"), (pose, 16, "pose"), (H, 36, "H"), (b, 6, "b")):
            if t.dtype != torch.float64 or not t.is_cuda or t.numel() != k or not t.is_contiguous():
                raise ValueError(f"{name} must be a contiguous float64 CUDA tensor of {k} values")
        if stats is not None and (not stats.is_cuda or stats.numel() * stats.element_size() < C.sizeof(Stats)):
            raise ValueError("stats must be a CUDA tensor of at least sizeof(gicp_stats) bytes")
        prm = prm or params()
        st = lib().gicp_register_dev(self.handle, _ptr(src), _ptr(src_covs), src.shape[1], gmap.handle,
                                     _ptr(init_pose), C.byref(prm), _ptr(pose), _ptr(H), _ptr(b),
                                     _ptr(src_covs_out), _ptr(stats), _stream())
        if st != GICP_OK:
            raise GicpError(st, "gicp_register_dev")

    @staticmethod
    def stats_from_bytes(raw) -> dict:
        """Decodes a gicp_stats read back from the device (numpy uint8)."""
        a = np.frombuffer(np.asarray(raw, np.uint8).tobytes()[:_STATS_DT.itemsize], _STATS_DT)[0]
        return {k: a[k].item() for k in _STATS_DT.names}

    def register_pair(self, src, map_means, map_covs, init_pose, prm: Params | None = None, src_covs=None,
                      map_cell: float = 0.0) -> RegisterResult:
        """The problem-statement form: registers src against Gaussians (means
        [3, m], covs [6, m], used as given) through a transient map."""
        _check_f32_cuda(src, 3, "src")
        _check_f32_cuda(map_means, 3, "map_means")
        _check_f32_cuda(map_covs, 6, "map_covs")
        if src_covs is not None:
            _check_f32_cuda(src_covs, 6, "src_covs")
        prm = prm or params()
        init = _abi.D16(*np.asarray(init_pose, np.float64).reshape(16))
        pose, H, b = _abi.D16(), _abi.D36(), _abi.D6()
        stats = Stats()
        st = lib().gicp_register_pair(self.handle, _ptr(src), _ptr(src_covs), src.shape[1], _ptr(map_means),
                                      _ptr(map_covs), map_means.shape[1], map_cell, init, C.byref(prm), pose, H, b,
                                      C.byref(stats), _stream())
        if st in (_abi.GICP_E_ARG, _abi.GICP_E_HIP, _abi.GICP_E_OOM):
            raise GicpError(st, "gicp_register_pair")
        return RegisterResult(np.array(pose[:]).reshape(4, 4), np.array(H[:]).reshape(6, 6), np.array(b[:]),
                              stats.iters, stats.n_inliers, stats.cost, bool(stats.converged), st)

    def depth_to_points(self, depth, fx, fy, cx, cy, voxel=0.02, max_depth=1e4):
        """depth: [H, W] float32 CUDA tensor (metres) -> voxel centroids [3, n] (camera frame)."""
        import torch
        if depth.dtype != torch.float32 or not depth.is_cuda or depth.dim() != 2 or not depth.is_contiguous():
            raise ValueError("depth must be a contiguous float32 CUDA tensor [H, W]")
        H, W = depth.shape
        buf = torch.empty(3 * H * W, dtype=torch.float32, device=depth.device)
        n = C.c_int64()
        st = lib().gicp_depth_to_points(self.handle, _ptr(depth), W, H, fx, fy, cx, cy, voxel, max_depth, _ptr(buf),
                                        H * W, C.byref(n), _stream())
        if st != GICP_OK:
            raise GicpError(st, "gicp_depth_to_points")
        return buf[:3 * n.value].view(3, n.value)

    def keyframe_gaussians(self, src, src_covs, gmap: Map, pose, r_overlap=0.1, p=1.5):
        """Gaussians a keyframe adds (non-overlapping points, scale aligned, in
        the map frame): (means [3, m], covs [6, m], inlier ratio)."""
        import torch
        _check_f32_cuda(src, 3, "src")
        _check_f32_cuda(src_covs, 6, "src_covs")
        n = src.shape[1]
        means = torch.empty((3, n), dtype=torch.float32, device=src.device)
        covs = torch.empty((6, n), dtype=torch.float32, device=src.device)
        m = C.c_int64()
        ratio = C.c_double()
        T = _abi.D16(*np.asarray(pose, np.float64).reshape(16))
        st = lib().gicp_keyframe_gaussians(self.handle, _ptr(src), _ptr(src_covs), n, gmap.handle, T, r_overlap, p,
                                           _ptr(means), _ptr(covs), C.byref(m), C.byref(ratio), _stream())
        if st != GICP_OK:
            raise GicpError(st, "gicp_keyframe_gaussians")
        k = m.value
        # the outputs use stride n; return compact [3, k] / [6, k] views' copies
        return means[:, :k].contiguous(), covs[:, :k].contiguous(), ratio.value

    def map_insert(self, gmap: Map, means, covs):
        _check_f32_cuda(means, 3, "means")
        _check_f32_cuda(covs, 6, "covs")
        st = lib().gicp_map_insert(self.handle, gmap.handle, _ptr(means), _ptr(covs), means.shape[1], _stream())
        if st != GICP_OK:
            raise GicpError(st, "gicp_map_insert")
        m = C.c_int64()
        c = C.c_float()
        lib().gicp_map_info(gmap.handle, C.byref(m), C.byref(c))
        gmap.m = int(m.value)
        return gmap

    @staticmethod
    def keyframe_policy(ratio, since_keyframe, since_mapping, threshold, max_gap=30, mapping_gap=10):
        return int(lib().gicp_keyframe_policy(ratio, since_keyframe, since_mapping, threshold, max_gap, mapping_gap))

    def track(self, frames, gmap: Map, init_pose, motion: int = MOTION_PREVIOUS, prm: Params | None = None,
              covs=None):
        """Tracks a sequence: frames [3, n_i] registered in order against gmap,
        frame 0 from init_pose and every later frame from the pose predicted
        on the device from the previous estimates.  covs: optional list of
        [6, n_i] (None entries are computed).  Returns a list of RegisterResult."""
        prm = prm or params()
        k = len(frames)
        arr = (Frame * max(k, 1))()
        for i, f in enumerate(frames):
            _check_f32_cuda(f, 3, "frame")
            cv = None if covs is None else covs[i]
            if cv is not None:
                _check_f32_cuda(cv, 6, "covs")
            arr[i].src = f.data_ptr()
            arr[i].src_covs = 0 if cv is None else cv.data_ptr()
            arr[i].n = f.shape[1]
        init = _abi.D16(*np.asarray(init_pose, np.float64).reshape(16))
        poses = np.zeros((k, 4, 4))
        Hs = np.zeros((k, 6, 6))
        bs = np.zeros((k, 6))
        stats = np.zeros(k, _STATS_DT)
        st = lib().gicp_track(self.handle, k, arr, gmap.handle, init, motion, C.byref(prm), poses.ctypes.data,
                              Hs.ctypes.data, bs.ctypes.data, C.cast(stats.ctypes.data, C.POINTER(Stats)), _stream())
        if st in (_abi.GICP_E_ARG, _abi.GICP_E_HIP, _abi.GICP_E_OOM):
            raise GicpError(st, "gicp_track")
        return [RegisterResult(poses[i], Hs[i], bs[i], it, ni, cost, bool(cv), status)
                for i, (it, ni, cost, cv, status, _, _) in enumerate(stats.tolist())]

    def register_batch(self, problems, prm: Params | None = None):
        """problems: sequence of (src [3,n], src_covs [6,n] or None, Map, init_pose 4x4).
        Returns a list of RegisterResult (one per problem)."""
        prm = prm or params()
        k = len(problems)
        arr = np.zeros(k, _PROBLEM_DT)
        srcs, scovs, maps, inits = zip(*problems) if k else ((), (), (), ())
        for src, scov in zip(srcs, scovs):
            _check_f32_cuda(src, 3, "src")
            if scov is not None:
                _check_f32_cuda(scov, 6, "src_covs")
        arr["src"] = [t.data_ptr() for t in srcs]
        arr["src_covs"] = [0 if t is None else t.data_ptr() for t in scovs]
        arr["n"] = [t.shape[1] for t in srcs]
        arr["map"] = [m.handle.value or 0 for m in maps]
        if k:
            arr["init_pose"] = np.asarray(inits, np.float64).reshape(k, 16)
        poses = np.zeros((k, 4, 4))
        Hs = np.zeros((k, 6, 6))
        bs = np.zeros((k, 6))
        stats = np.zeros(k, _STATS_DT)
        st = lib().gicp_register_batch(self.handle, k, C.cast(arr.ctypes.data, C.POINTER(Problem)), C.byref(prm),
                                       poses.ctypes.data, Hs.ctypes.data, bs.ctypes.data,
                                       C.cast(stats.ctypes.data, C.POINTER(Stats)), _stream())
        if st in (_abi.GICP_E_ARG, _abi.GICP_E_HIP, _abi.GICP_E_OOM):
            raise GicpError(st, "gicp_register_batch")
        return [RegisterResult(poses[i], Hs[i], bs[i], it, ni, cost, bool(cv), status)
                for i, (it, ni, cost, cv, status, _, _) in enumerate(stats.tolist())]
