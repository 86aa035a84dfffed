"""Autotuner for the launch-shape parameters of the tracking path.

Exactness never depends on these choices (every search proves its result or
hands the query to the overflow pass); only speed does.  Tuned here:

* the source grid cell, as a factor of the estimated k-NN radius
  (``gicp_estimate_cell``), timed on the fused k-NN covariance;
* the map grid cell in metres, timed on a two-iteration registration;
* the number of frames per ``gicp_register_batch`` call;
* the form of a ``gicp_register_batch`` call (batched launches or the work
  queue) and the lanes per source point of its linearisation;
* the lanes per source point of ``gicp_track``.

Results are cached as JSON keyed by the device name and a size bucket, in
``$GICP_TUNE_CACHE`` (default: ``~/.cache/gicp_tune.json``).
"""
from __future__ import annotations

import json
import math
import os

CACHE = os.environ.get("GICP_TUNE_CACHE", os.path.join(os.path.expanduser("~"), ".cache", "gicp_tune.json"))

SRC_FACTORS = (0.6, 0.75, 0.9, 1.0, 1.2, 1.5)
MAP_CELLS = (0.02, 0.03, 0.04, 0.045, 0.05, 0.055, 0.06)
BATCHES = (1, 4, 8, 16, 32)


def _time_ms(fn, reps=3):
    import torch
    fn()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        fn()
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps


def _key(kind, *sizes):
    import torch
    name = torch.cuda.get_device_name(0).replace(" ", "_")
    buckets = "_".join(str(int(2 ** round(math.log2(max(int(s), 1))))) for s in sizes)
    return f"{name}:{kind}:{buckets}"


def _load():
    try:
        with open(CACHE) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def _store(d):
    try:
        os.makedirs(os.path.dirname(CACHE), exist_ok=True)
        with open(CACHE, "w") as f:
            json.dump(d, f, indent=1)
    except OSError:
        pass


def tune_source_cell(ctx, pts, k=20, reg_mode=1, use_cache=True):
    """Best source cell [m] for `pts` ([3, n] CUDA tensor): the estimated k-NN
    radius times the fastest factor of SRC_FACTORS."""
    import torch
    base = ctx.estimate_cell(pts, k)
    key = _key("src", pts.shape[1], k)
    cache = _load() if use_cache else {}
    if key in cache:
        return base * cache[key]["factor"], cache[key]
    out = torch.empty((6, pts.shape[1]), dtype=torch.float32, device=pts.device)
    times = {f: _time_ms(lambda: ctx.covariances(pts, k, cell=base * f, reg_mode=reg_mode, out=out))
             for f in SRC_FACTORS}
    best = min(times, key=times.get)
    rec = {"factor": best, "ms": {str(f): round(t, 4) for f, t in times.items()}}
    if use_cache:
        cache[key] = rec
        _store(cache)
    return base * best, rec


def tune_map_cell(ctx, means, covs, frame, init, prm, reg_mode=1, use_cache=True):
    """Best map cell [m] for a map ([3, m] means, [6, m] covariances), timed on
    a two-iteration registration of `frame` from `init`."""
    import paper_2403_12550_amd as g
    key = _key("map", means.shape[1], frame.shape[1])
    cache = _load() if use_cache else {}
    if key in cache:
        return cache[key]["cell"], cache[key]
    times = {}
    p2 = g.params(k=prm.k, eps=prm.eps, r_max=prm.r_max, max_it=2, conv_rot=0.0, conv_trans=0.0,
                  reg_mode=prm.reg_mode, cell_src=prm.cell_src)
    scov = ctx.covariances(frame, prm.k, cell=prm.cell_src, reg_mode=prm.reg_mode)
    for cell in MAP_CELLS:
        gm = ctx.map_build(means, covs, cell=cell, reg_mode=reg_mode)
        times[cell] = _time_ms(lambda: ctx.register(frame, gm, init, p2, src_covs=scov))
        gm.close()
    best = min(times, key=times.get)
    rec = {"cell": best, "ms": {str(c): round(t, 4) for c, t in times.items()}}
    if use_cache:
        cache[key] = rec
        _store(cache)
    return best, rec


def tune_batch(ctx, gmap, frames, inits, prm, use_cache=True):
    """Frames per gicp_register_batch call with the best frames/s."""
    key = _key("batch", frames[0].shape[1], len(frames))
    cache = _load() if use_cache else {}
    if key in cache:
        return cache[key]["batch"], cache[key]
    rate = {}
    for b in BATCHES:
        if b > len(frames):
            continue
        items = [(frames[i], None, gmap, inits[i]) for i in range(b)]
        if b == 1:
            t = _time_ms(lambda: ctx.register(frames[0], gmap, inits[0], prm), reps=2)
        else:
            t = _time_ms(lambda: ctx.register_batch(items, prm), reps=2)
        rate[b] = b / t
    best = max(rate, key=rate.get)
    rec = {"batch": best, "frames_per_ms": {str(b): round(r, 4) for b, r in rate.items()}}
    if use_cache:
        cache[key] = rec
        _store(cache)
    return best, rec


FORMS = (("batched", 0, 2), ("batched", 0, 4), ("queue", 2, 2), ("queue", 2, 4))   # (name, flags, lanes)
TRACK_LANES = (2, 4)


def _with(prm, **kw):
    import paper_2403_12550_amd as g
    p = g.Params()
    for name, _ in g.Params._fields_:
        setattr(p, name, getattr(prm, name))
    for k, v in kw.items():
        setattr(p, k, v)
    return p


def tune_form(ctx, items, prm, use_cache=True, reps=2):
    """Fastest (flags, lanes) for ``ctx.register_batch(items, prm)`` among
    FORMS; prm's own form flags and lanes are replaced.  Returns
    ((flags, lanes), record)."""
    npts = sum(int(it[0].shape[1]) for it in items)
    key = _key("form", len(items), npts)
    cache = _load() if use_cache else {}
    if key in cache:
        return (cache[key]["flags"], cache[key]["lanes"]), cache[key]
    times = {}
    for name, flags, lanes in FORMS:
        base = prm.flags & ~(1 | 2 | 4)   # keep NO_REUSE, drop the form flags
        p = _with(prm, flags=base | flags, lanes=lanes)
        times[(name, flags, lanes)] = _time_ms(lambda: ctx.register_batch(items, p), reps=reps)
    best = min(times, key=times.get)
    rec = {"form": best[0], "flags": best[1], "lanes": best[2],
           "ms": {f"{n}/lanes{ln}": round(t, 4) for (n, _, ln), t in times.items()}}
    if use_cache:
        cache[key] = rec
        _store(cache)
    return (best[1], best[2]), rec


def tune_track_lanes(ctx, frames, gmap, init_pose, motion, prm, use_cache=True, reps=2):
    """Fastest lanes per source point for ``ctx.track(frames, ...)`` among
    TRACK_LANES.  Returns (lanes, record)."""
    npts = sum(int(f.shape[1]) for f in frames)
    key = _key("track", len(frames), npts)
    cache = _load() if use_cache else {}
    if key in cache:
        return cache[key]["lanes"], cache[key]
    times = {}
    for lanes in TRACK_LANES:
        p = _with(prm, lanes=lanes)
        times[lanes] = _time_ms(lambda: ctx.track(frames, gmap, init_pose, motion, p), reps=reps)
    best = min(times, key=times.get)
    rec = {"lanes": best, "ms": {str(k): round(t, 4) for k, t in times.items()}}
    if use_cache:
        cache[key] = rec
        _store(cache)
    return best, rec


def clear_cache():
    try:
        os.remove(CACHE)
    except OSError:
        pass


__all__ = ["tune_source_cell", "tune_map_cell", "tune_batch", "tune_form", "tune_track_lanes", "clear_cache", "CACHE"]
