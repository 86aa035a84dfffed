"""Oracle: nearest-neighbour search (test infrastructure only).

Paper: Sec. 3 — the covariance of a point is the covariance of its k nearest
neighbours, and source-target correspondences are "determined by nearest
neighbor search".  The paper fixes no distance precision or tie rule; the
readings used here are:

* Ranking key for k-NN (covariance neighbourhoods and the standalone k-NN
  query): the FP32 squared distance evaluated as
  ``fl(fl(fl(dx*dx) + fl(dy*dy)) + fl(dz*dz))`` with ``dx = fl(q.x - p.x)``,
  round-to-nearest and no fused multiply-add, so that an index list can be
  compared bit for bit; ties go to the lower original index.  The query point
  itself is one of its own neighbours (distance 0).
* Correspondence 1-NN inside Gauss-Newton: the exact (FP64) Euclidean nearest
  map mean, accepted iff its squared distance is <= r_max^2; ties to the lower
  index.
"""
from __future__ import annotations

import numpy as np
from scipy.spatial import cKDTree

INT_SENTINEL = -1


def fp32_key(q: np.ndarray, p: np.ndarray) -> np.ndarray:
    """FP32 squared-distance ranking key between query rows q[...,3] and points
    p[...,3] (broadcasting), evaluated op by op in float32."""
    q = np.asarray(q, np.float32)
    p = np.asarray(p, np.float32)
    dx = np.subtract(q[..., 0], p[..., 0], dtype=np.float32)
    dy = np.subtract(q[..., 1], p[..., 1], dtype=np.float32)
    dz = np.subtract(q[..., 2], p[..., 2], dtype=np.float32)
    s = np.add(np.multiply(dx, dx, dtype=np.float32), np.multiply(dy, dy, dtype=np.float32), dtype=np.float32)
    return np.add(s, np.multiply(dz, dz, dtype=np.float32), dtype=np.float32)


def _lex(key32: np.ndarray, idx: np.ndarray) -> np.ndarray:
    """64-bit value whose integer order is the (key, index) lexicographic order
    (keys are non-negative floats, whose bit patterns order like integers)."""
    kb = np.ascontiguousarray(key32, np.float32).view(np.uint32).astype(np.uint64)
    return (kb << np.uint64(32)) | idx.astype(np.uint64)


def knn_bruteforce(points: np.ndarray, queries: np.ndarray, k: int, r_max: float | None = None,
                   chunk: int = 256):
    """Exact k-NN by evaluating the key against every point.

    Returns (idx[nq,k] int32, key[nq,k] float32).  Slots beyond the available
    neighbours (fewer than k points, or beyond the r_max gate: key >
    fl32(r_max*r_max)) hold index -1 and key +inf."""
    points = np.asarray(points, np.float32)
    queries = np.asarray(queries, np.float32)
    n, nq = points.shape[0], queries.shape[0]
    idx_out = np.full((nq, k), INT_SENTINEL, np.int32)
    key_out = np.full((nq, k), np.inf, np.float32)
    if n == 0 or nq == 0:
        return idx_out, key_out
    gate = None if r_max is None else np.float32(np.float32(r_max) * np.float32(r_max))
    ar = np.arange(n, dtype=np.int64)
    kk = min(k, n)
    for s in range(0, nq, chunk):
        qc = queries[s:s + chunk]
        key = fp32_key(qc[:, None, :], points[None, :, :])          # [c,n]
        lex = _lex(key, np.broadcast_to(ar, key.shape))
        part = np.partition(lex, kk - 1, axis=1)[:, :kk] if kk < n else lex
        part = np.sort(part, axis=1)
        sel_idx = (part & np.uint64(0xFFFFFFFF)).astype(np.int64)
        sel_key = (part >> np.uint64(32)).astype(np.uint32).view(np.float32)
        if gate is not None:
            bad = sel_key > gate
            sel_idx = np.where(bad, INT_SENTINEL, sel_idx)
            sel_key = np.where(bad, np.float32(np.inf), sel_key)
        idx_out[s:s + chunk, :kk] = sel_idx
        key_out[s:s + chunk, :kk] = sel_key
    return idx_out, key_out


def knn_kdtree(points: np.ndarray, queries: np.ndarray, k: int, extra: int = 8, workers: int = -1):
    """Exact k-NN for large inputs: an exact FP64 kd-tree proposes k+extra
    candidates, which are re-ranked by (FP32 key, index).  The result is the
    brute-force result whenever every point outside the candidate set is
    provably farther (in FP32 key) than the k-th chosen one; queries where that
    cannot be shown are redone by brute force."""
    points = np.asarray(points, np.float32)
    queries = np.asarray(queries, np.float32)
    n, nq = points.shape[0], queries.shape[0]
    kk = min(k + extra, n)
    tree = cKDTree(points.astype(np.float64))
    d64, cand = tree.query(queries.astype(np.float64), k=kk, workers=workers)
    if kk == 1:
        d64, cand = d64[:, None], cand[:, None]
    key = fp32_key(queries[:, None, :], points[cand])
    lex = np.sort(_lex(key, cand), axis=1)
    kr = min(k, n)
    sel = lex[:, :kr]
    idx = (sel & np.uint64(0xFFFFFFFF)).astype(np.int32)
    keyk = (sel >> np.uint64(32)).astype(np.uint32).view(np.float32)
    # safety: every non-candidate has FP64 squared distance >= d64[:, -1]^2; the
    # FP32 key of a point differs from its FP64 squared distance by a relative
    # error below 1e-6 (plus a tiny absolute term), so a margin settles it.
    if kk < n:
        far = d64[:, -1] ** 2
        kth = keyk[:, -1].astype(np.float64)
        unsafe = np.nonzero(far * (1 - 1e-6) - 1e-30 <= kth * (1 + 1e-6))[0]
        if unsafe.size:
            bi, bk = knn_bruteforce(points, queries[unsafe], k)
            idx[unsafe] = bi[:, :kr]
            keyk[unsafe] = bk[:, :kr]
    out_i = np.full((nq, k), INT_SENTINEL, np.int32)
    out_k = np.full((nq, k), np.inf, np.float32)
    out_i[:, :kr] = idx
    out_k[:, :kr] = keyk
    return out_i, out_k


def knn(points, queries, k, r_max=None):
    """k-NN with the (FP32 key, lower index) rule; picks brute force for small
    problems and the re-ranked kd-tree otherwise.  r_max gates by FP32 key."""
    points = np.asarray(points, np.float32)
    queries = np.asarray(queries, np.float32)
    if points.shape[0] * queries.shape[0] <= 4e7 or r_max is not None:
        return knn_bruteforce(points, queries, k, r_max)
    return knn_kdtree(points, queries, k)


def nearest_fp64(points: np.ndarray, queries: np.ndarray, r_max: float, tree: cKDTree | None = None):
    """Correspondence search: exact FP64 nearest neighbour of each query among
    ``points``; returns (idx[nq] int64 with -1 = none, d2[nq] float64).  A match
    is accepted iff d^2 <= r_max^2; ties go to the lower index."""
    points = np.asarray(points, np.float64)
    queries = np.asarray(queries, np.float64)
    if tree is None:
        tree = cKDTree(points)
    kq = min(4, points.shape[0])
    d, j = tree.query(queries, k=kq, distance_upper_bound=r_max * (1 + 1e-9) + 1e-12, workers=-1)
    if kq == 1:
        d, j = d[:, None], j[:, None]
    nq = queries.shape[0]
    idx = np.full(nq, -1, np.int64)
    d2 = np.full(nq, np.inf)
    have = np.isfinite(d[:, 0])
    if not have.any():
        return idx, d2
    jj = j[have]
    # exact squared distances of the candidates, recomputed in FP64
    diff = queries[have][:, None, :] - points[np.minimum(jj, points.shape[0] - 1)]
    dd = np.einsum("ijk,ijk->ij", diff, diff)
    dd = np.where(jj < points.shape[0], dd, np.inf)
    best = dd.min(axis=1)
    # lowest index among exact ties
    cand = np.where(dd == best[:, None], jj, np.iinfo(np.int64).max)
    choice = cand.min(axis=1)
    # if all kq candidates tie, a lower-index tied point could lie outside: brute force those
    full_tie = (dd == best[:, None]).all(axis=1) & (kq < points.shape[0])
    if full_tie.any():
        hq = np.nonzero(have)[0][full_tie]
        for r in hq:
            dr = points - queries[r]
            e = np.einsum("ij,ij->i", dr, dr)
            m = e.min()
            choice[np.searchsorted(np.nonzero(have)[0], r)] = int(np.nonzero(e == m)[0][0])
    ok = best <= r_max * r_max
    hi = np.nonzero(have)[0]
    idx[hi[ok]] = choice[ok]
    d2[hi[ok]] = best[ok]
    return idx, d2
