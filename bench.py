#!/usr/bin/env python3
"""Frame-to-map G-ICP tracking benchmark on one MI355X.

Workload: synthetic 1200x680 depth frames (pinhole fx=fy=600) rendered along a
100-frame smooth trajectory in a procedural room with 40 boxes and spheres,
1 % invalid pixels, sigma_z = 1 mm * z^2, voxel-downsampled at 2 cm (about 68k
points per frame), tracked against a 1M-Gaussian map of the same scene;
k = 20 plane-regularised frame covariances, r_max = 0.1 m, at most 20
Gauss-Newton iterations per frame (stop below 1e-6 rad / 1e-6 m).

The headline is closed-loop tracking: the frames are registered in order, each
starting from the previous frame's estimate (predicted on the device, so that
the whole sequence is one gicp_track call with no host round trip between
frames).  A step is one frame: its share of the batched covariance launches and
all of its Gauss-Newton iterations.  Frames and the map are resident in HBM
before the timed region; the map is built once (timed separately).

    python bench.py [--gpus 1] [--steps K] [--warmup W]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# algorithmic bytes per unit of work: what the step must read and write, not
# what a particular search touches
BYTES_PER_UNIT = {
    0: 72.0,   # linearisation: src xyz 12 + src cov 24 + map mean 12 + map cov 24, per point per iteration
    1: 36.0,   # k-NN covariance: xyz 12 in + cov 24 out, per point
    2: 20.0,   # grid build: xyz 12 in + key/index 8 out, per point (compulsory part)
    3: 232.0,  # solve: 29 FP64 partials per ... (negligible)
}
GROUP_NAMES = {0: "k_gn_linearize", 1: "k_knn_cov", 2: "grid build (keys, radix sort, table)", 3: "k_gn_solve"}
# In the tracking form one launch is a whole iteration (group 0): the
# linearisation, the hand-over of the partials and the solve.
TRACK_NAMES = {**GROUP_NAMES, 0: "k_slot_iterate"}
# Calibrated HBM bytes per unit from rocprofv3 FETCH_SIZE / WRITE_SIZE runs of
# the tracking form on this workload
# (profiles/hbm_traffic__k_slot_iterate__c2_track_pmc.md): per point and
# iteration over the launches that did work.
# Valid for the kernels as they were when the counters were taken (None: not
# taken for the current kernels).
TRAFFIC_BYTES_PER_UNIT = {0: 297.2}
# Wavefront VALU instructions per unit from rocprofv3 SQ_INSTS_VALU on the same
# runs (profiles/hbm_traffic__k_slot_iterate__c2_track_pmc.md), and the chip's VALU issue peak: 256 CUs x 4 SIMDs, one wave64
# instruction per SIMD every 4 cycles (16 lanes a cycle) at 2.4 GHz.
VALU_INSTS_PER_UNIT = {0: 93.9}
VALU_PEAK_INSTS = 256 * 4 * 2.4e9 / 4
MOTION_NAMES = {0: "previous", 1: "constant_velocity"}


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def pose_delta(Ta, Tb):
    """(rotation angle of Ra^T Rb [rad], |ta - tb| [m]); the angle from atan2 of
    the skew and symmetric parts stays accurate for tiny rotations."""
    R = Ta[:3, :3].T @ Tb[:3, :3]
    s = 0.5 * np.linalg.norm([R[2, 1] - R[1, 2], R[0, 2] - R[2, 0], R[1, 0] - R[0, 1]])
    c = 0.5 * (np.trace(R) - 1.0)
    return float(np.arctan2(s, c)), float(np.linalg.norm(Ta[:3, 3] - Tb[:3, 3]))


def run_oracle_track(seq, n_frames, motion, r_max, max_it, conv):
    """The FP64 oracle's tracking loop on the first n_frames frames (its own
    estimates feed its own predictions); returns (poses, seconds per frame,
    setup seconds)."""
    from scipy.spatial import cKDTree

    from oracle import covariance as oc
    from oracle import gicp as og
    from oracle import tracking as ot

    t0 = time.perf_counter()
    map_cov = oc.regularise6(seq.map_cov_raw, oc.REG_PLANE, 1e-3).astype(np.float32)
    tree = cKDTree(seq.map_means.astype(np.float64))
    setup = time.perf_counter() - t0
    est, secs = [], []
    for i in range(n_frames):
        t1 = time.perf_counter()
        T0 = ot.predict(est, i, seq.poses[0], motion)
        src = seq.frame(i)
        cs = oc.covariances(src, 20, oc.REG_PLANE, 1e-3)
        r = og.register(src, cs, seq.map_means, map_cov, T0, r_max=r_max, max_it=max_it,
                        conv_rot=conv, conv_trans=conv, tree=tree)
        secs.append(time.perf_counter() - t1)
        est.append(r.pose)
    return est, secs, setup


def rigid_inverse(T):
    Ti = np.eye(4)
    Ti[:3, :3] = T[:3, :3].T
    Ti[:3, 3] = -T[:3, :3].T @ T[:3, 3]
    return Ti


def predict(est, i, T0, motion):
    """Initial pose of frame i for the host-driven forms (the motion models of
    gicp_track): frame 0 from T0, then the previous estimate (motion 0) or
    constant velocity T_{i-1} T_{i-2}^-1 T_{i-1} (motion 1, from frame 2)."""
    if i == 0:
        return np.array(T0, np.float64)
    if motion == 1 and i >= 2:
        return est[i - 1] @ (rigid_inverse(est[i - 2]) @ est[i - 1])
    return np.array(est[i - 1], np.float64)


def timed(fn):
    import torch
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    out = fn()
    torch.cuda.synchronize()
    return time.perf_counter() - t0, out


def copy_calibration(mib):
    """A plain copy of `mib` MiB: under a counter profiler its FETCH_SIZE and
    WRITE_SIZE per dispatch give the counter's reading for a known byte count."""
    import torch
    n = mib * (1 << 20) // 4
    a = torch.arange(n, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    for _ in range(5):
        b.copy_(a)
    torch.cuda.synchronize()
    log(f"copied {mib} MiB five times")


def kernel_table(prof, frames, names=GROUP_NAMES):
    out = {}
    for gid, (n, ms, units) in prof.items():
        if n == 0:
            continue
        out[names[gid]] = {"launches": n, "avg_us": 1e3 * ms / n, "total_ms_per_frame": ms / frames,
                           "units_per_launch": units / n}
    return out


def roofline_of(prof, gid, names=GROUP_NAMES):
    n, ms, units = prof[gid]
    achieved = BYTES_PER_UNIT[gid] * units / (ms * 1e-3) / 1e9
    traffic = TRAFFIC_BYTES_PER_UNIT.get(gid)
    r = {"kernel": names[gid], "bound": "hbm", "achieved": round(achieved, 2), "peak": HBM_PEAK_GBS,
         "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 5),
         "traffic": None if traffic is None else round(traffic * units / n),
         "traffic_unit": "bytes per launch (calibrated FETCH_SIZE + WRITE_SIZE)",
         "bytes_per_unit": BYTES_PER_UNIT[gid], "units_per_launch": units / n, "avg_launch_us": 1e3 * ms / n}
    valu = VALU_INSTS_PER_UNIT.get(gid)
    if valu is not None:
        rate = valu * units / (ms * 1e-3)
        r["alu"] = {"bound": "valu_issue", "achieved": round(rate / 1e9, 2), "peak": VALU_PEAK_INSTS / 1e9,
                    "unit": "G wave64 VALU instructions/s", "frac": round(rate / VALU_PEAK_INSTS, 4),
                    "insts_per_unit": valu}
    return r


def _render_depths(seq, idx, workers):
    import multiprocessing as mp
    if workers <= 1:
        return [seq.depth(i) for i in idx]
    with mp.get_context("fork").Pool(min(workers, len(idx))) as pool:
        return pool.map(seq.depth, idx)


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100, help="timed frames (the first STEPS frames, tracked in order)")
    ap.add_argument("--warmup", type=int, default=100,
                    help="frames tracked untimed before the timed sequence (as many as are timed: the first "
                         "call of a size grows the library's workspaces)")
    ap.add_argument("--frames", type=int, default=100)
    ap.add_argument("--map-size", type=int, default=1_000_000)
    ap.add_argument("--map-cell", type=float, default=0.05,
                    help="map grid cell [m] (0.05: the fastest tracking on this map of 0.045-0.07; measured)")
    ap.add_argument("--motion", choices=("previous", "cv"), default="previous",
                    help="initial pose of each frame: the previous estimate, or constant velocity")
    ap.add_argument("--batch", type=int, default=50, help="frames per call of the batched (independent) form")
    ap.add_argument("--cpu-frames", type=int, default=20, help="frames the CPU oracle tracks")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-c4", action="store_true", help="skip the 64-problem batch workload")
    ap.add_argument("--no-frontend", action="store_true",
                    help="skip the depth-to-points and keyframe-insertion timings")
    ap.add_argument("--regularisation-study", type=int, default=0, metavar="FRAMES",
                    help="closed-loop tracking of the first FRAMES frames with no / plane / ellipse "
                         "regularisation of map and frame covariances; reports the trajectory error of each")
    ap.add_argument("--tracking-only", action="store_true",
                    help="run only the warm-up and the timed tracking call, and print their work units (point "
                         "iterations) with the timing; for counter profiles of the tracking kernels")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run a plain device copy of MIB MiB five times (the reference kernel that scales "
                         "the HBM byte counters) and exit")
    args = ap.parse_args()
    if args.copy_calibration:
        copy_calibration(args.copy_calibration)
        return

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU: the library has no multi-GPU path (a batch of registrations "
              "shards with no communication between problems). Run with --gpus 1.", file=sys.stderr)
        sys.exit(2)

    import synth

    # every input is generated before the GPU runtime is initialised: the
    # renderers use pools of forked workers, and a forked copy of a process
    # with an initialised GPU runtime is not safe to run
    t0 = time.perf_counter()
    nf = args.frames
    K = min(args.steps, nf)
    seq = synth.C2Sequence(n_frames=nf, map_size=args.map_size)
    workers = max(1, min(16, len(os.sched_getaffinity(0))))
    seq.prefetch(range(nf), workers=workers)
    depths_np = None if args.no_frontend else _render_depths(seq, list(range(10)), workers)
    npts = np.array([seq.frame(i).shape[0] for i in range(nf)])
    log(f"workload generated in {time.perf_counter() - t0:.1f} s: {nf} frames, "
        f"{npts.mean():.0f} pts/frame (min {npts.min()}, max {npts.max()}), map {args.map_size}")

    import torch

    import paper_2403_12550_amd as g

    g.lib()
    torch.cuda.set_device(0)
    ctx = g.Context(0)
    means = g.to_soa(seq.map_means)
    covs = g.to_soa(seq.map_cov_raw)
    frames = [g.to_soa(seq.frame(i)) for i in range(nf)]
    torch.cuda.synchronize()

    # map: built once (static map), timed on its own
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record()
    gmap = ctx.map_build(means, covs, cell=args.map_cell, reg_mode=g.REG_PLANE, eps=1e-3)
    ev1.record()
    torch.cuda.synchronize()
    map_ms = ev0.elapsed_time(ev1)
    src_cell = ctx.estimate_cell(frames[0], 20)
    log(f"map built in {map_ms:.2f} ms (cell {gmap.cell * 100:.2f} cm); source cell {src_cell * 100:.2f} cm")

    r_max, max_it, conv = 0.1, 20, 1e-6
    motion = g.MOTION_PREVIOUS if args.motion == "previous" else g.MOTION_CONSTANT_VELOCITY

    def prm(flags=0):
        return g.params(k=20, eps=1e-3, r_max=r_max, max_it=max_it, conv_rot=conv, conv_trans=conv,
                        reg_mode=g.REG_PLANE, cell_src=src_cell, flags=flags)

    T0 = seq.poses[0]
    # lanes per source point of the tracking launches, chosen by the autotuner
    # (cached per device and workload size)
    from paper_2403_12550_amd import autotune
    lanes, lanes_rec = autotune.tune_track_lanes(ctx, frames[:K], gmap, T0, motion, prm(0))
    log(f"tracking lanes per point (autotuned): {lanes_rec}")

    def prm(flags=0, lanes=lanes):
        return g.params(k=20, eps=1e-3, r_max=r_max, max_it=max_it, conv_rot=conv, conv_trans=conv,
                        reg_mode=g.REG_PLANE, cell_src=src_cell, flags=flags, lanes=lanes)

    # --- headline: closed-loop tracking, one gicp_track call for the K frames
    # in its default form (iteration slots: each frame costs its own
    # iterations, the device moves on to the next frame itself)
    tw = ctx.track(frames[:max(1, args.warmup)], gmap, T0, motion, prm(0))
    elapsed, tr = timed(lambda: ctx.track(frames[:K], gmap, T0, motion, prm(0)))
    fps = K / elapsed
    statuses = sorted(set(int(r.status) for r in tr))
    iters = [r.iters for r in tr]
    log(f"tracking form ({K} frames, one call): {fps:.1f} frames/s, mean iterations {np.mean(iters):.2f}, "
        f"statuses {statuses}")
    if args.tracking_only:
        def units(res):
            return int(sum(int(npts[i]) * r.iters for i, r in enumerate(res)))
        print(json.dumps({"tracking_only": True, "frames": K, "value": round(fps, 3), "units_timed": units(tr),
                          "units_warmup": units(tw), "slots_timed": int(sum(iters)),
                          "slots_warmup": int(sum(r.iters for r in tw))}), flush=True)
        gmap.close()
        ctx.close()
        return
    # the other two forms of the same call (max_it launch pairs per frame,
    # launched or replayed from a graph): equal poses
    el_launch, tr_l = timed(lambda: ctx.track(frames[:K], gmap, T0, motion, prm(g.FLAG_MULTI_LAUNCH)))
    ctx.track(frames[:max(1, args.warmup)], gmap, T0, motion, prm(g.FLAG_GRAPH))
    el_graph, tr_g = timed(lambda: ctx.track(frames[:K], gmap, T0, motion, prm(g.FLAG_GRAPH)))
    same = all(np.array_equal(a.pose, b.pose) and np.array_equal(a.pose, c.pose) for a, b, c in zip(tr, tr_l, tr_g))
    # kernel timing of the headline form (HIP events around every launch)
    ctx.profile(True)
    el_ev, _ = timed(lambda: ctx.track(frames[:K], gmap, T0, motion, prm(0)))
    prof = {gid: ctx.profile_read(gid) for gid in range(4)}
    ctx.profile(False)
    kernels = kernel_table(prof, K, TRACK_NAMES)
    roofline = roofline_of(prof, 0, TRACK_NAMES)

    # --- secondary forms on the same frames
    # per-frame form: one gicp_register call per frame, closed on the previous estimate
    def per_frame():
        est = []
        for i in range(K):
            est.append(ctx.register(frames[i], gmap, predict(est, i, T0, motion), prm(lanes=0)).pose)
        return est
    per_frame()
    el_pf, _ = timed(per_frame)
    # independent registrations in batched calls (each frame from the previous
    # ground-truth pose: open loop; throughput of independent problems)
    inits = [seq.poses[max(i - 1, 0)] for i in range(nf)]

    def batched():
        out = []
        for s0 in range(0, K, args.batch):
            idx = list(range(s0, min(K, s0 + args.batch)))
            out += ctx.register_batch([(frames[i], None, gmap, inits[i]) for i in idx], prm(g.FLAG_GRAPH, lanes=0))
        return out
    batched()
    el_b, _ = timed(batched)
    log(f"per-frame form {K / el_pf:.1f} frames/s; batched independent form {K / el_b:.1f} frames/s")

    gt = np.array([pose_delta(r.pose, seq.poses[i]) for i, r in enumerate(tr)])
    c4 = None if args.no_c4 else run_c4(ctx, g)
    frontend = None if args.no_frontend else run_frontend(ctx, g, seq, means, covs, args.map_cell, depths_np)
    regst = run_regularisation_study(ctx, g, seq, means, args.map_cell, args.regularisation_study, motion) \
        if args.regularisation_study else None

    cpu = None
    err_vs_oracle = None
    if not args.no_cpu_baseline and args.cpu_frames > 0:
        nc = min(args.cpu_frames, K)
        opos, secs, setup = run_oracle_track(seq, nc, motion, r_max, max_it, conv)
        errs = np.array([pose_delta(tr[i].pose, op) for i, op in enumerate(opos)])
        err_vs_oracle = {"frames": nc, "max_rad": float(errs[:, 0].max()), "max_m": float(errs[:, 1].max()),
                         "within_1e-4_m": bool(errs[:, 1].max() <= 1e-4),
                         "form": "both closed loop: each side tracks from its own previous estimates"}
        cores = len(os.sched_getaffinity(0))
        cpu = {"value": round(nc / sum(secs), 4), "unit": "frames/s", "cores": cores, "kind": "oracle",
               "sample": f"the oracle's tracking loop over the first {nc} frames of the same sequence, FP64 "
                         f"numpy/scipy, cKDTree workers=-1; per-frame time excludes the one-off map preparation "
                         f"({setup:.1f} s: eigh of 1M covariances + kd-tree)"}
        log(f"cpu oracle: {cpu['value']} frames/s over {nc} frames; GPU vs oracle max "
            f"{err_vs_oracle['max_rad']:.2e} rad {err_vs_oracle['max_m']:.2e} m")

    out = {
        "metric": "G-ICP frames/s (60k pts vs 1M-Gaussian map) at pose err <=1e-4 vs FP64",
        "value": round(fps, 3),
        "unit": "frames/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": args.warmup,
        "ms_per_step": round(1e3 * elapsed / K, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "closed-loop frame-to-map tracking: 1200x680 depth frames voxelised at 2 cm "
                               f"(mean {npts.mean():.0f} pts) vs a {args.map_size}-Gaussian map, {K} frames of a "
                               f"{nf}-frame trajectory, k=20, plane eps=1e-3, r_max=0.1 m, <=20 GN it",
                   "frames": K, "map_gaussians": args.map_size, "mean_points": float(npts[:K].mean()),
                   "form": f"gicp_track: one call for the {K} frames; frame covariances in batched launches, "
                           "then one launch per Gauss-Newton iteration (linearisation, device-side hand-over "
                           "of the partials, solve) whose frame the device picks: a frame's last solve predicts "
                           "the next frame's pose from the estimates and moves on to it; a step is one frame",
                   "motion": MOTION_NAMES[motion], "init": "frame 0 from its ground-truth pose"},
        "tracking": {"statuses": statuses, "mean_gn_iterations": float(np.mean(iters)),
                     "lanes_per_point": lanes, "lanes_autotune": lanes_rec,
                     "value_with_kernel_events": round(K / el_ev, 3),
                     "per_frame_launch_pairs_form": {"value": round(K / el_launch, 3),
                                                     "form": "max_it (linearise, solve) launch pairs per frame"},
                     "graph_form": {"value": round(K / el_graph, 3),
                                    "form": "each frame's max_it launch pairs replayed from a HIP graph"},
                     "poses_equal_across_forms": bool(same),
                     "ate_rmse_m": float(np.sqrt(np.mean(gt[:, 1] ** 2))), "max_trans_err_m": float(gt[:, 1].max())},
        "per_frame_form": {"value": round(K / el_pf, 3), "unit": "frames/s", "ms_per_frame": round(1e3 * el_pf / K, 4),
                           "form": "one gicp_register call per frame, closed loop (host-side prediction)"},
        "batched_independent_form": {"value": round(K / el_b, 3), "unit": "frames/s",
                                     "form": f"{args.batch} frames per gicp_register_batch call (graph-replayed "
                                             "iterations), each from the previous ground-truth pose: independent "
                                             "registrations, not tracking"},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "pose_err_vs_oracle": err_vs_oracle,
        "map_build_ms": round(map_ms, 3),
        "kernels": kernels,
        "c4_batch": c4,
        "frontend": frontend,
        "regularisation_study": regst,
    }
    print(json.dumps(out), flush=True)
    gmap.close()
    ctx.close()


def run_c4(ctx, g, n_prob=64):
    """The batched-registration workload: 64 problems (sources 2k-200k points,
    targets 0.1M-1M Gaussians), one gicp_register_batch call."""
    import torch

    import synth
    t0 = time.perf_counter()
    probs = synth.c4_batch(n_prob=n_prob)
    items, maps = [], []
    for p in probs:
        gm = ctx.map_build(g.to_soa(p.tgt), g.to_soa(p.tgt_cov_raw), cell=0.0, reg_mode=g.REG_PLANE)
        maps.append(gm)
        items.append((g.to_soa(p.src), None, gm, p.init))
    torch.cuda.synchronize()
    log(f"c4: {n_prob} problems generated and maps built in {time.perf_counter() - t0:.1f} s")
    from paper_2403_12550_amd import autotune
    prm = g.params(k=20, eps=1e-3, r_max=0.1, max_it=30, conv_rot=1e-6, conv_trans=1e-6, reg_mode=g.REG_PLANE)
    (t_flags, t_lanes), trec = autotune.tune_form(ctx, items, prm)
    log(f"c4 autotuned form: {trec}")
    out = {"autotune": trec}
    for name, flags, lanes in (("batched", 0, 0), ("queue", g.FLAG_QUEUE, 0), ("per_problem", g.FLAG_MULTI_LAUNCH, 0),
                               ("tuned", t_flags, t_lanes)):
        p2 = g.params(k=20, eps=1e-3, r_max=0.1, max_it=30, conv_rot=1e-6, conv_trans=1e-6, reg_mode=g.REG_PLANE,
                      flags=flags, lanes=lanes)
        ctx.register_batch(items, p2)
        torch.cuda.synchronize()
        t = time.perf_counter()
        res = ctx.register_batch(items, p2)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t
        # kernel times from a second, evented call (events around every launch)
        ctx.profile(True)
        ctx.register_batch(items, p2)
        torch.cuda.synchronize()
        n, ms, u = ctx.profile_read(0)
        groups = {GROUP_NAMES[gid]: round(ctx.profile_read(gid)[1], 3) for gid in range(4)}
        ctx.profile(False)
        terr = max(float(np.linalg.norm(r.pose[:3, 3] - p.T_gt[:3, 3])) for r, p in zip(res, probs))
        out[name] = {"problems_per_s": round(n_prob / dt, 2), "ms": round(1e3 * dt, 3), "lanes": lanes or None,
                     "mean_iterations": float(np.mean([r.iters for r in res])),
                     "statuses": sorted(set(int(r.status) for r in res)),
                     "linearize_GBps": round(72.0 * u / (ms * 1e-3) / 1e9, 2) if ms > 0 else None,
                     "kernel_ms": groups,
                     "max_trans_err_vs_truth_m": terr}
        log(f"c4 {name}: {out[name]}")
    for gm in maps:
        gm.close()
    out["source_points"] = int(sum(p.src.shape[0] for p in probs))
    out["target_gaussians"] = int(sum(p.tgt.shape[0] for p in probs))
    del prm
    return out


def run_frontend(ctx, g, seq, means, covs, map_cell, depths_np):
    """Depth image -> voxelised cloud on the GPU (1200x680 frames, 2 cm
    voxels; the images were rendered before the GPU was initialised), and the
    keyframe insertion of one frame into the 1M map (overlap test, scale
    aligning, transform, merge into the map)."""
    import torch
    depths = [torch.from_numpy(d).cuda() for d in depths_np]
    K = seq.K
    ctx.depth_to_points(depths[0], K.fx, K.fy, K.cx, K.cy, seq.voxel)
    torch.cuda.synchronize()
    t = time.perf_counter()
    npts = []
    for d in depths:
        npts.append(ctx.depth_to_points(d, K.fx, K.fy, K.cx, K.cy, seq.voxel).shape[1])
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t) / len(depths)
    out = {"depth_to_points": {"frames_per_s": round(1.0 / dt, 1), "ms_per_frame": round(1e3 * dt, 3),
                               "mean_points": float(np.mean(npts)), "pixels": int(depths[0].numel()),
                               "note": "includes two host synchronisations per frame (bounding box, count)"}}
    # keyframe insertion: frame 0 at its ground-truth pose into a fresh copy of the map
    gm = ctx.map_build(means, covs, cell=map_cell, reg_mode=g.REG_PLANE, eps=1e-3)
    src = g.to_soa(seq.frame(0))
    scov = ctx.covariances(src, 20, reg_mode=g.REG_ELLIPSE)
    ctx.keyframe_gaussians(src, scov, gm, seq.poses[0], 0.02, 1.5)
    torch.cuda.synchronize()
    reps = 5
    t = time.perf_counter()
    for _ in range(reps):
        m_new, c_new, ratio = ctx.keyframe_gaussians(src, scov, gm, seq.poses[0], 0.02, 1.5)
    torch.cuda.synchronize()
    t_kf = (time.perf_counter() - t) / reps
    t = time.perf_counter()
    ctx.map_insert(gm, m_new, c_new)
    torch.cuda.synchronize()
    t_first = time.perf_counter() - t
    # later inserts (the spare arrays exist): the same Gaussians five more times
    t = time.perf_counter()
    for _ in range(reps):
        ctx.map_insert(gm, m_new, c_new)
    torch.cuda.synchronize()
    t_ins = (time.perf_counter() - t) / reps
    out["keyframe_insert"] = {"frame_points": int(src.shape[1]), "inserted": int(m_new.shape[1]),
                              "correspondence_ratio": round(ratio, 4), "keyframe_gaussians_ms": round(1e3 * t_kf, 3),
                              "map_insert_ms": round(1e3 * t_ins, 3), "first_map_insert_ms": round(1e3 * t_first, 3),
                              "map_size_after": gm.m,
                              "note": "r_overlap 2 cm, p = 1.5; map_insert_ms: mean of five inserts after the "
                                      "first, which allocates the map's spare arrays"}
    gm.close()
    log(f"frontend: {out}")
    return out


def run_regularisation_study(ctx, g, seq, means, map_cell, n_frames, motion):
    """The regularisation of map and frame covariances (none / plane /
    ellipse) compared on tracking error: closed-loop tracking of the first
    n_frames frames (one gicp_track call with the given motion model), and
    per-frame registration from the previous ground-truth pose over the whole
    sequence."""
    out = {"closed_loop_frames": n_frames, "open_loop_frames": len(seq), "motion": MOTION_NAMES[motion]}
    frames = [g.to_soa(seq.frame(i)) for i in range(len(seq))]
    for name, mode in (("none", g.REG_NONE), ("plane", g.REG_PLANE), ("ellipse", g.REG_ELLIPSE)):
        gm = ctx.map_build(means, g.to_soa(seq.map_cov_raw), cell=map_cell, reg_mode=mode, eps=1e-3)
        prm = g.params(k=20, eps=1e-3, r_max=0.1, max_it=20, conv_rot=1e-6, conv_trans=1e-6, reg_mode=mode)
        res = ctx.track(frames[:n_frames], gm, seq.poses[0], motion, prm)
        e = np.array([pose_delta(r.pose, seq.poses[i]) for i, r in enumerate(res)])
        out_m = {"closed_loop_ate_rmse_m": float(np.sqrt(np.mean(e[:, 1] ** 2))),
                 "closed_loop_max_trans_err_m": float(e[:, 1].max()),
                 "closed_loop_failed_frames": int(sum(r.status != 0 for r in res)),
                 "closed_loop_mean_iterations": float(np.mean([r.iters for r in res]))}
        e2 = np.array([pose_delta(ctx.register(frames[i], gm, seq.poses[max(i - 1, 0)], prm).pose, seq.poses[i])
                       for i in range(len(seq))])
        out_m.update({"open_loop_rmse_m": float(np.sqrt(np.mean(e2[:, 1] ** 2))),
                      "open_loop_max_trans_err_m": float(e2[:, 1].max()),
                      "open_loop_mean_rot_err_rad": float(e2[:, 0].mean())})
        out[name] = out_m
        gm.close()
        log(f"regularisation {name}: {out_m}")
    return out


if __name__ == "__main__":
    main()
