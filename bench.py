#!/usr/bin/env python3
"""Frame-to-map G-ICP tracking benchmark on one MI355X.

Workload: synthetic 1200x680 depth frames (pinhole fx=fy=600) rendered along a
100-frame smooth trajectory in a procedural room with 40 boxes and spheres,
1 % invalid pixels, sigma_z = 1 mm * z^2, voxel-downsampled at 2 cm (about 60k
points per frame), registered against a 1M-Gaussian map of the same scene;
k = 20 plane-regularised source covariances, r_max = 0.1 m, at most 20
Gauss-Newton iterations per frame (stop below 1e-6 rad / 1e-6 m), constant-
velocity initial poses.

A step is one frame: the source grid build, the fused k-NN covariance, and
every Gauss-Newton iteration (correspondences, linearisation, FP64 solve and
update).  Frames and the map are resident in HBM before the timed region;
the map is built once (timed separately).

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
# Calibrated HBM bytes per unit from rocprofv3 FETCH_SIZE / WRITE_SIZE runs on
# this workload (profiles/hbm_traffic__c2_60k_vs_1M_pmc.md): covariance group
# per point; linearisation per point and iteration, over the launches that did
# work.  Valid for the kernels as they were when the counters were taken.
TRAFFIC_BYTES_PER_UNIT = {1: 448.9, 0: 300.3}
# Wavefront VALU instructions per unit from rocprofv3 SQ_INSTS_VALU on the same
# runs (profiles/valu_issue__c2_60k_vs_1M_pmc.md), and the chip's VALU issue
# peak: 256 CUs x 4 SIMDs, one wave64 instruction per SIMD every 4 cycles
# (16 lanes a cycle) at 2.4 GHz.
VALU_INSTS_PER_UNIT = {1: 258.0, 0: 82.6}
VALU_PEAK_INSTS = 256 * 4 * 2.4e9 / 4


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def pose_delta(Ta, Tb):
    """(rotation angle of Ra^T Rb [rad], |ta - tb| [m]); the angle from atan2 of
    the skew and symmetric parts stays accurate for tiny rotations."""
    R = Ta[:3, :3].T @ Tb[:3, :3]
    s = 0.5 * np.linalg.norm([R[2, 1] - R[1, 2], R[0, 2] - R[2, 0], R[1, 0] - R[0, 1]])
    c = 0.5 * (np.trace(R) - 1.0)
    return float(np.arctan2(s, c)), float(np.linalg.norm(Ta[:3, 3] - Tb[:3, 3]))


def cv_init(seq, est, i):
    """Constant-velocity prediction from the two previous poses of `est`
    (frame 0: ground truth; frame 1: the previous pose)."""
    if i == 0:
        return seq.poses[0].copy()
    if i == 1:
        return est[0].copy()
    a, b = est[i - 2], est[i - 1]
    ai = np.eye(4)
    ai[:3, :3] = a[:3, :3].T
    ai[:3, 3] = -a[:3, :3].T @ a[:3, 3]
    return b @ (ai @ b)


def run_oracle(seq, n_frames, r_max, max_it, conv, closed_loop=False):
    """The FP64 oracle on the first n_frames frames with its own constant-velocity
    recursion; returns (poses, seconds spent per frame, setup seconds)."""
    from scipy.spatial import cKDTree

    from oracle import covariance as oc
    from oracle import gicp as og

    t0 = time.perf_counter()
    map_cov = oc.regularise6(seq.map_cov_raw, oc.REG_PLANE, 1e-3).astype(np.float32)
    tree = cKDTree(seq.map_means.astype(np.float64))
    setup = time.perf_counter() - t0
    est, secs = [], []
    for i in range(n_frames):
        init = cv_init(seq, est if closed_loop else seq.poses, i)
        t1 = time.perf_counter()
        src = seq.frame(i)
        cs = oc.covariances(src, 20, oc.REG_PLANE, 1e-3)
        r = og.register(src, cs, seq.map_means, map_cov, init, r_max=r_max, max_it=max_it,
                        conv_rot=conv, conv_trans=conv, tree=tree)
        secs.append(time.perf_counter() - t1)
        est.append(r.pose)
    return est, secs, setup


def time_frames(ctx, gmap, frames, inits, prm, order, batch, prof=False):
    """Registers the frames listed in `order` in groups of `batch` from the
    initial poses `inits` (one per frame, prepared beforehand like the frames);
    returns (seconds, poses by frame, iterations, statuses)."""
    import torch
    poses, iters, statuses = {}, [], []
    if prof:
        ctx.profile(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for s0 in range(0, len(order), batch):
        idx = order[s0:s0 + batch]
        if batch == 1:
            i = idx[0]
            rs = [ctx.register(frames[i], gmap, inits[i], prm)]
        else:
            rs = ctx.register_batch([(frames[i], None, gmap, inits[i]) for i in idx], prm)
        for i, r in zip(idx, rs):
            poses[i] = r.pose
            iters.append(r.iters)
            statuses.append(r.status)
    torch.cuda.synchronize()
    return time.perf_counter() - t0, poses, iters, statuses


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


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100, help="timed frames")
    ap.add_argument("--warmup", type=int, default=20, help="untimed frames before the timed ones")
    ap.add_argument("--batch", type=int, default=50, help="frames per gicp_register_batch call")
    ap.add_argument("--frames", type=int, default=100)
    ap.add_argument("--map-size", type=int, default=1_000_000)
    ap.add_argument("--map-cell", type=float, default=0.03)
    ap.add_argument("--cpu-frames", type=int, default=20, help="frames the CPU oracle baseline registers")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--c4", action="store_true", help="also time the 64-problem batch workload")
    ap.add_argument("--no-frontend", action="store_true",
                    help="skip the depth-to-points and keyframe-insertion timings")
    ap.add_argument("--regularisation-study", type=int, default=0, metavar="FRAMES",
                    help="closed-loop tracking of the first FRAMES frames with no / plane / ellipse "
                         "regularisation of map and frame covariances; reports the trajectory error of each")
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

    import torch

    import paper_2403_12550_amd as g
    import synth

    g.lib()
    torch.cuda.set_device(0)
    t0 = time.perf_counter()
    seq = synth.C2Sequence(n_frames=args.frames, map_size=args.map_size)
    workers = max(1, min(16, len(os.sched_getaffinity(0))))
    seq.prefetch(range(args.frames), workers=workers)
    npts = np.array([seq.frame(i).shape[0] for i in range(args.frames)])
    log(f"workload generated in {time.perf_counter() - t0:.1f} s: {args.frames} frames, "
        f"{npts.mean():.0f} pts/frame (min {npts.min()}, max {npts.max()}), map {args.map_size}")

    ctx = g.Context(0)
    means = g.to_soa(seq.map_means)
    covs = g.to_soa(seq.map_cov_raw)
    frames = [g.to_soa(seq.frame(i)) for i in range(args.frames)]
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
    prm = g.params(k=20, eps=1e-3, r_max=r_max, max_it=max_it, conv_rot=conv, conv_trans=conv,
                   reg_mode=g.REG_PLANE, cell_src=src_cell)
    nf = args.frames
    warm = [i % nf for i in range(args.warmup)]
    # the batched forms warm up on a whole batch, so that the timed calls find
    # their workspaces sized
    warm_batch = [i % nf for i in range(max(args.warmup, args.batch))]
    order = [(args.warmup + i) % nf for i in range(args.steps)]
    # constant-velocity initial poses from the ground-truth trajectory (open
    # loop): inputs of the timed work, prepared with the frames
    inits = [cv_init(seq, seq.poses, i) for i in range(nf)]

    # plain per-frame form (one gicp_register call per frame)
    time_frames(ctx, gmap, frames, inits, prm, warm, 1)
    t_plain, _, _, _ = time_frames(ctx, gmap, frames, inits, prm, order, 1)
    log(f"per-frame form timed: {args.steps / t_plain:.1f} frames/s")
    # batched form (the headline): `batch` frames per call
    time_frames(ctx, gmap, frames, inits, prm, warm_batch, args.batch)
    elapsed, poses, iters, statuses = time_frames(ctx, gmap, frames, inits, prm, order, args.batch)
    log(f"batched form timed: {args.steps / elapsed:.1f} frames/s")
    # the batched form with its iterations replayed from a HIP graph
    prm_graph = g.params(k=20, eps=1e-3, r_max=r_max, max_it=max_it, conv_rot=conv, conv_trans=conv,
                         reg_mode=g.REG_PLANE, cell_src=src_cell, flags=g.FLAG_GRAPH)
    time_frames(ctx, gmap, frames, inits, prm_graph, warm_batch, args.batch)
    elapsed_graph, poses_graph, _, _ = time_frames(ctx, gmap, frames, inits, prm_graph, order, args.batch)
    same = all(np.array_equal(poses_graph[i], poses[i]) for i in poses)
    # the same frames again with the library's kernel timing (HIP events around
    # every kernel group) for the per-kernel table and the roofline
    elapsed_ev, _, _, _ = time_frames(ctx, gmap, frames, inits, prm, order, args.batch, prof=True)
    prof = {gid: ctx.profile_read(gid) for gid in range(4)}
    ctx.profile(False)
    fps_launch = args.steps / elapsed
    fps_graph = args.steps / elapsed_graph
    # the headline is the graph-replayed batched form (same kernels and, as
    # checked above, the same poses as the batched launches)
    fps = fps_graph if same else fps_launch
    elapsed_value = elapsed_graph if same else elapsed
    fps_plain = args.steps / t_plain
    log(f"graph form {args.steps / elapsed_graph:.1f} frames/s (poses equal: {same})")
    log(f"timed {args.steps} frames: batched ({args.batch}/call) {fps_launch:.1f} frames/s "
        f"({args.steps / elapsed_ev:.1f} with kernel events), per-frame {fps_plain:.1f} "
        f"frames/s; mean iterations {np.mean(iters):.2f}, statuses {sorted(set(statuses))}")

    # ground-truth error (information only: the synthetic frames are noisy resamples)
    gt_err = np.array([pose_delta(p, seq.poses[i]) for i, p in poses.items()])

    kernels = {}
    for gid, (n, ms, units) in prof.items():
        if n == 0:
            continue
        kernels[GROUP_NAMES[gid]] = {"launches": n, "avg_us": 1e3 * ms / n, "total_ms_per_frame": ms / args.steps,
                                     "units_per_launch": units / n}
    dom = max((gid for gid in prof if prof[gid][0] > 0 and gid in (0, 1)), key=lambda gid: prof[gid][1])
    n, ms, units = prof[dom]
    achieved = BYTES_PER_UNIT[dom] * units / (ms * 1e-3) / 1e9
    traffic = TRAFFIC_BYTES_PER_UNIT.get(dom)
    roofline = {"kernel": GROUP_NAMES[dom], "bound": "hbm", "achieved": round(achieved, 2), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 5),
                "traffic": None if traffic is None else round(traffic * units / n),
                "traffic_unit": "bytes per launch (calibrated FETCH_SIZE + WRITE_SIZE)",
                "bytes_per_unit": BYTES_PER_UNIT[dom], "units_per_launch": units / n,
                "avg_launch_us": 1e3 * ms / n}
    valu = VALU_INSTS_PER_UNIT.get(dom)
    if valu is not None:
        # the roof the kernel actually meets: vector-ALU instruction issue
        rate = valu * units / (ms * 1e-3)
        roofline["alu"] = {"bound": "valu_issue", "achieved": round(rate / 1e9, 2), "peak": VALU_PEAK_INSTS / 1e9,
                           "unit": "G wave64 VALU instructions/s", "frac": round(rate / VALU_PEAK_INSTS, 4),
                           "insts_per_unit": valu}

    c4 = run_c4(ctx, g) if args.c4 else None
    frontend = None if args.no_frontend else run_frontend(ctx, g, seq, means, covs, args.map_cell)
    regst = run_regularisation_study(ctx, g, seq, means, args.map_cell, args.regularisation_study) \
        if args.regularisation_study else None

    cpu = None
    err_vs_oracle = None
    if not args.no_cpu_baseline and args.cpu_frames > 0:
        nc = min(args.cpu_frames, nf)
        opos, secs, setup = run_oracle(seq, nc, r_max, max_it, conv)
        # the GPU poses of the same frames, from the same initial poses
        _, gp, _, _ = time_frames(ctx, gmap, frames, inits, prm, list(range(nc)), args.batch)
        errs = np.array([pose_delta(gp[i], op) for i, op in enumerate(opos)])
        err_vs_oracle = {"frames": nc, "max_rad": float(errs[:, 0].max()), "max_m": float(errs[:, 1].max())}
        cores = len(os.sched_getaffinity(0))
        cpu = {"value": round(nc / sum(secs), 4), "unit": "frames/s", "cores": cores, "kind": "oracle",
               "sample": f"first {nc} frames of the same workload and initial poses, FP64 numpy/scipy, "
                         f"cKDTree workers=-1; per-frame time excludes the one-off map preparation "
                         f"({setup:.1f} s: eigh of 1M covariances + kd-tree)"}
        log(f"cpu oracle: {cpu['value']} frames/s over {nc} frames; GPU vs oracle max "
            f"{err_vs_oracle['max_rad']:.2e} rad {err_vs_oracle['max_m']:.2e} m")

    out = {
        "metric": "G-ICP frames/s (60k pts vs 1M-Gaussian map) at pose err <=1e-4 vs FP64",
        "value": round(fps, 3),
        "unit": "frames/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(1e3 * elapsed_value / args.steps, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "frame-to-map tracking: 1200x680 depth frames voxelised at 2 cm "
                               f"(mean {npts.mean():.0f} pts) vs a {args.map_size}-Gaussian map, "
                               f"{nf}-frame trajectory, k=20, plane eps=1e-3, r_max=0.1 m, <=20 GN it",
                   "frames": nf, "map_gaussians": args.map_size, "mean_points": float(npts.mean()),
                   "form": f"batched: {args.batch} frames per gicp_register_batch call, Gauss-Newton iterations "
                           "replayed from a HIP graph (GICP_FLAG_GRAPH); a step is one frame",
                   "init": "constant-velocity prediction from the previous two ground-truth poses, "
                           "prepared with the frames before the timed region"},
        "per_frame_form": {"value": round(fps_plain, 3), "unit": "frames/s",
                           "ms_per_frame": round(1e3 * t_plain / args.steps, 4),
                           "form": "one gicp_register call per frame"},
        "batched_over_per_frame": round(fps / fps_plain, 3),
        "batched_launch_form": {"value": round(fps_launch, 3), "unit": "frames/s",
                                "form": "batched, one launch per kernel and iteration",
                                "graph_poses_equal": bool(same),
                                "value_with_kernel_events": round(args.steps / elapsed_ev, 3)},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "pose_err_vs_oracle": err_vs_oracle,
        "pose_err_vs_ground_truth": {"mean_rad": float(gt_err[:, 0].mean()), "mean_m": float(gt_err[:, 1].mean())},
        "mean_gn_iterations": float(np.mean(iters)),
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
    prm = g.params(k=20, eps=1e-3, r_max=0.1, max_it=30, conv_rot=1e-6, conv_trans=1e-6, reg_mode=g.REG_PLANE)
    out = {}
    for name, flags in (("batched", 0), ("queue", g.FLAG_QUEUE), ("per_problem", g.FLAG_MULTI_LAUNCH)):
        p2 = g.params(k=20, eps=1e-3, r_max=0.1, max_it=30, conv_rot=1e-6, conv_trans=1e-6, reg_mode=g.REG_PLANE,
                      flags=flags)
        ctx.register_batch(items, p2)
        torch.cuda.synchronize()
        ctx.profile(True)
        t = time.perf_counter()
        res = ctx.register_batch(items, p2)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t
        n, ms, u = ctx.profile_read(0)
        groups = {GROUP_NAMES[gid]: round(ctx.profile_read(gid)[1], 3) for gid in range(4)}
        ctx.profile(False)
        terr = max(float(np.linalg.norm(r.pose[:3, 3] - p.T_gt[:3, 3])) for r, p in zip(res, probs))
        out[name] = {"problems_per_s": round(n_prob / dt, 2), "ms": round(1e3 * dt, 3),
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


def _render_depths(seq, idx, workers):
    import multiprocessing as mp
    if workers <= 1:
        return [seq.depth(i) for i in idx]
    with mp.get_context("fork").Pool(min(workers, len(idx))) as pool:
        return pool.map(seq.depth, idx)


def run_frontend(ctx, g, seq, means, covs, map_cell, n_depth=10):
    """Depth image -> voxelised cloud on the GPU (1200x680 frames, 2 cm
    voxels), and the keyframe insertion of one frame into the 1M map
    (overlap test, scale aligning, transform, merge into the map)."""
    import torch
    idx = list(range(n_depth))
    workers = max(1, min(16, len(os.sched_getaffinity(0))))
    depths = [torch.from_numpy(d).cuda() for d in _render_depths(seq, idx, workers)]
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
    t_ins = time.perf_counter() - t
    out["keyframe_insert"] = {"frame_points": int(src.shape[1]), "inserted": int(m_new.shape[1]),
                              "correspondence_ratio": round(ratio, 4), "keyframe_gaussians_ms": round(1e3 * t_kf, 3),
                              "map_insert_ms": round(1e3 * t_ins, 3), "map_size_after": gm.m,
                              "note": "r_overlap 2 cm, p = 1.5; the first insert allocates the map's spare arrays"}
    gm.close()
    log(f"frontend: {out}")
    return out


def run_regularisation_study(ctx, g, seq, means, map_cell, n_frames):
    """The regularisation of map and frame covariances (none / plane /
    ellipse) compared on tracking error: closed-loop tracking (constant-
    velocity prediction from the estimated poses) of the first n_frames
    frames, and per-frame registration from the prediction of the ground-
    truth poses over the whole sequence."""
    out = {"closed_loop_frames": n_frames, "open_loop_frames": len(seq)}
    frames = [g.to_soa(seq.frame(i)) for i in range(len(seq))]
    for name, mode in (("none", g.REG_NONE), ("plane", g.REG_PLANE), ("ellipse", g.REG_ELLIPSE)):
        gm = ctx.map_build(means, g.to_soa(seq.map_cov_raw), cell=map_cell, reg_mode=mode, eps=1e-3)
        prm = g.params(k=20, eps=1e-3, r_max=0.1, max_it=20, conv_rot=1e-6, conv_trans=1e-6, reg_mode=mode)
        est, errs, iters, lost = [], [], [], 0
        for i in range(n_frames):
            r = ctx.register(frames[i], gm, cv_init(seq, est, i), prm)
            est.append(r.pose)
            iters.append(r.iters)
            lost += int(r.status != 0)
            errs.append(pose_delta(r.pose, seq.poses[i]))
        e = np.array(errs)
        res = {"closed_loop_ate_rmse_m": float(np.sqrt(np.mean(e[:, 1] ** 2))),
               "closed_loop_max_trans_err_m": float(e[:, 1].max()), "closed_loop_failed_frames": lost,
               "closed_loop_mean_iterations": float(np.mean(iters))}
        e2 = np.array([pose_delta(ctx.register(frames[i], gm, cv_init(seq, seq.poses, i), prm).pose, seq.poses[i])
                       for i in range(len(seq))])
        res.update({"open_loop_rmse_m": float(np.sqrt(np.mean(e2[:, 1] ** 2))),
                    "open_loop_max_trans_err_m": float(e2[:, 1].max()),
                    "open_loop_mean_rot_err_rad": float(e2[:, 0].mean())})
        out[name] = res
        gm.close()
        log(f"regularisation {name}: {res}")
    return out


if __name__ == "__main__":
    main()
