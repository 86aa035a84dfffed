"""Binding of the learned warm-start network (gicp_mlp_* in include/gicp.h).

Argument marshalling only: packing, the forward and backward passes and the
Adam update all run in libgicp.so.  Buffers are torch tensors on the device.
"""
from __future__ import annotations

import ctypes as C

import numpy as np

from . import _abi
from ._abi import MLP_BF16, MLP_CACHE, MLP_MAX_BATCH, MLP_PARAMS, MLP_POINTS, MlpPair


def _lib():
    return _abi.load()


def _ptr(t) -> int:
    return 0 if t is None else int(t.data_ptr())


def _stream():
    import torch
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ok(st, what):
    if st != _abi.GICP_OK:
        from . import GicpError
        raise GicpError(st, what)


class WarmStartNet:
    """Parameters (FP32), Adam moments and the bf16 weight fragments of one
    network, owned by the caller as torch tensors."""

    def __init__(self, ctx, seed: int = 0, device: str = "cuda"):
        import torch
        self.ctx = ctx
        self.params = torch.empty(MLP_PARAMS, dtype=torch.float32, device=device)
        self.m = torch.empty_like(self.params)
        self.v = torch.empty_like(self.params)
        self.wbf16 = torch.empty(MLP_BF16, dtype=torch.int16, device=device)
        self.grad = torch.empty_like(self.params)
        self.loss = torch.empty(1, dtype=torch.float32, device=device)
        self.step_count = 0
        _ok(_lib().gicp_mlp_init(ctx.handle, seed, _ptr(self.params), _ptr(self.m), _ptr(self.v), _ptr(self.wbf16),
                                 _stream()), "gicp_mlp_init")

    def load(self, params):
        """Replace the parameters (FP32, MLP_PARAMS values) and reset Adam."""
        import torch
        self.params.copy_(torch.as_tensor(params, dtype=torch.float32))
        self.m.zero_()
        self.v.zero_()
        self.step_count = 0
        _ok(_lib().gicp_mlp_sync_weights(self.ctx.handle, _ptr(self.params), _ptr(self.wbf16), _stream()),
            "gicp_mlp_sync_weights")

    def pack(self, pairs, X=None, centres=None):
        """pairs: sequence of (src [3,n], tgt [3,m], src_idx int32 [4096], tgt_idx int32 [4096]) device tensors.
        Returns X (int16 bf16 bits [B, 4096, 6]) and centres (float64 [B, 3])."""
        import torch
        B = len(pairs)
        if not 1 <= B <= MLP_MAX_BATCH:
            raise ValueError("batch size out of range")
        arr = (MlpPair * B)()
        for i, (src, tgt, si, ti) in enumerate(pairs):
            for t, name in ((si, "src_idx"), (ti, "tgt_idx")):
                if t.dtype != torch.int32 or not t.is_cuda or t.numel() != MLP_POINTS or not t.is_contiguous():
                    raise ValueError(f"{name} must be a contiguous int32 CUDA tensor of {MLP_POINTS} entries")
            for t, name in ((src, "src"), (tgt, "tgt")):
                if t.dtype != torch.float32 or not t.is_cuda or t.dim() != 2 or t.shape[0] != 3 or \
                        not t.is_contiguous():
                    raise ValueError(f"{name} must be a contiguous float32 CUDA tensor [3, n]")
            arr[i].src, arr[i].n_src = _ptr(src), src.shape[1]
            arr[i].tgt, arr[i].n_tgt = _ptr(tgt), tgt.shape[1]
            arr[i].src_idx, arr[i].tgt_idx = _ptr(si), _ptr(ti)
        dev = pairs[0][0].device
        if X is None:
            X = torch.empty((B, MLP_POINTS, 6), dtype=torch.int16, device=dev)
        if centres is None:
            centres = torch.empty((B, 3), dtype=torch.float64, device=dev)
        _ok(_lib().gicp_mlp_pack(self.ctx.handle, B, arr, _ptr(X), _ptr(centres), _stream()), "gicp_mlp_pack")
        return X, centres

    def forward(self, X, centres=None, want_cache=False, want_poses=False):
        """Returns (y [B,6] float32, cache or None, poses [B,4,4] float64 or None)."""
        import torch
        B = X.shape[0]
        y = torch.empty((B, 6), dtype=torch.float32, device=X.device)
        cache = torch.empty((B, MLP_CACHE), dtype=torch.float32, device=X.device) if want_cache else None
        poses = torch.empty((B, 4, 4), dtype=torch.float64, device=X.device) if want_poses else None
        _ok(_lib().gicp_mlp_forward(self.ctx.handle, B, _ptr(X), _ptr(self.params), _ptr(self.wbf16), _ptr(centres),
                                    _ptr(y), _ptr(cache), _ptr(poses), _stream()), "gicp_mlp_forward")
        return y, cache, poses

    def backward(self, X, cache, y, ystar):
        """Gradient (into self.grad) and loss (self.loss) against ystar [B,6]."""
        B = X.shape[0]
        _ok(_lib().gicp_mlp_backward(self.ctx.handle, B, _ptr(X), _ptr(self.params), _ptr(cache), _ptr(y),
                                     _ptr(ystar), _ptr(self.grad), _ptr(self.loss), _stream()), "gicp_mlp_backward")
        return self.grad, self.loss

    def adam_step(self, lr: float = 1e-3, grad=None):
        self.step_count += 1
        g = self.grad if grad is None else grad
        _ok(_lib().gicp_mlp_adam_step(self.ctx.handle, _ptr(self.params), _ptr(self.m), _ptr(self.v), _ptr(g),
                                      self.step_count, lr, _ptr(self.wbf16), _stream()), "gicp_mlp_adam_step")

    def train_step(self, X, ystar, lr: float = 1e-3):
        y, cache, _ = self.forward(X, want_cache=True)
        self.backward(X, cache, y, ystar)
        self.adam_step(lr)
        return self.loss

    def predict_poses(self, X, centres):
        """Relative poses (source -> target) [B,4,4] float64 on the device."""
        return self.forward(X, centres, want_poses=True)[2]


def subsample_indices(n: int, seed: int, count: int = MLP_POINTS) -> np.ndarray:
    """Seeded choice of `count` row indices of an n-point cloud (a permutation
    prefix; repeated draws when n < count)."""
    rng = np.random.default_rng(seed)
    if n >= count:
        return rng.permutation(n)[:count].astype(np.int32)
    return rng.integers(0, n, size=count).astype(np.int32)
