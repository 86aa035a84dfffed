"""Training and evaluation of the learned warm start on synthetic frame pairs.

Pairs come from seeded trajectories through procedural rooms (each frame an
independent 5000-point surface resample in the body frame; inter-frame motion
at most 8 cm and 4 degrees).  Labels are the relative poses the G-ICP path of
this library converges to from the ground-truth relative pose.  Inputs are
4096 points of each frame chosen by a seeded permutation and packed on the
device.  The comparison against the constant-velocity initialisation
registers every pair of held-out trajectories from each initial pose and
reports Gauss-Newton iterations, convergence, errors and throughput.

    python -m paper_2403_12550_amd.warmstart_train --train 2000 --test 100
"""
from __future__ import annotations

import argparse
import json
import multiprocessing as mp
import os
import sys
import time

import numpy as np

from . import warmstart as ws

TRAIN_SEED0 = 10000
TEST_SEED0 = 20000
N_FRAMES = 101
R_MAX = 0.1
MAX_IT = 30


def _log(*a):
    print("[warmstart]", *a, file=sys.stderr, flush=True)


def _trajectory(seed):
    import synth
    return synth.workloads.c5_trajectory(seed, n_frames=N_FRAMES)


def generate(seeds, workers):
    """Frames and poses of the given trajectory seeds (fork pool)."""
    if workers <= 1 or len(seeds) == 1:
        return [_trajectory(s) for s in seeds]
    with mp.get_context("fork").Pool(workers) as pool:
        return pool.map(_trajectory, seeds)


def _inv(T):
    R, t = T[:3, :3], T[:3, 3]
    out = np.eye(4)
    out[:3, :3] = R.T
    out[:3, 3] = -R.T @ t
    return out


def _rotvec(R):
    c = np.clip((np.trace(R) - 1.0) / 2.0, -1.0, 1.0)
    th = np.arccos(c)
    v = np.array([R[2, 1] - R[1, 2], R[0, 2] - R[2, 0], R[1, 0] - R[0, 1]])
    return 0.5 * v if th < 1e-9 else th / (2.0 * np.sin(th)) * v


def pose_error(Ta, Tb):
    """(rotation angle [rad], translation distance [m]) between two poses."""
    dR = Ta[:3, :3].T @ Tb[:3, :3]
    return float(np.linalg.norm(_rotvec(dR))), float(np.linalg.norm(Ta[:3, 3] - Tb[:3, 3]))


class Trajectory:
    """Device copies, covariances and maps of one trajectory's frames."""

    def __init__(self, g, ctx, frames, poses):
        self.frames = [g.to_soa(f) for f in frames]
        self.covs = [ctx.covariances(f, 20, reg_mode=g.REG_PLANE, eps=1e-3) for f in self.frames]
        self.maps = [ctx.map_build(self.frames[k], self.covs[k], cell=R_MAX) for k in range(len(frames) - 1)]
        self.gt = [_inv(poses[k]) @ poses[k + 1] for k in range(len(frames) - 1)]

    def items(self, inits):
        return [(self.frames[k + 1], self.covs[k + 1], self.maps[k], inits[k]) for k in range(len(self.maps))]

    def close(self):
        for m in self.maps:
            m.close()


def _prm(g):
    return g.params(k=20, eps=1e-3, r_max=R_MAX, max_it=MAX_IT, conv_rot=1e-6, conv_trans=1e-6,
                    reg_mode=g.REG_PLANE)


def pair_indices(seed, k, n_src, n_tgt):
    return (ws.subsample_indices(n_src, seed * 1000 + 2 * k), ws.subsample_indices(n_tgt, seed * 1000 + 2 * k + 1))


def pack_trajectory(net, tr, seed):
    import torch
    pairs = []
    for k in range(len(tr.maps)):
        si, ti = pair_indices(seed, k, tr.frames[k + 1].shape[1], tr.frames[k].shape[1])
        pairs.append((tr.frames[k + 1], tr.frames[k], torch.from_numpy(si).cuda(), torch.from_numpy(ti).cuda()))
    return net.pack(pairs)


def targets(T_rel, centres):
    """Network targets [rotation vector ; t + (R - I) c] of relative poses."""
    out = np.empty((len(T_rel), 6))
    for i, (T, c) in enumerate(zip(T_rel, centres)):
        R = T[:3, :3]
        out[i, :3] = _rotvec(R)
        out[i, 3:] = T[:3, 3] + (R - np.eye(3)) @ c
    return out


def build_dataset(g, ctx, net, seeds, workers, chunk=64):
    """Packed inputs (device int16 [P, 4096, 6]) and G-ICP targets (device float32 [P, 6])."""
    import torch
    Xs, Ys = [], []
    prm = _prm(g)
    for c0 in range(0, len(seeds), chunk):
        part = seeds[c0:c0 + chunk]
        for seed, (frames, poses) in zip(part, generate(part, workers)):
            tr = Trajectory(g, ctx, frames, poses)
            res = ctx.register_batch(tr.items(tr.gt), prm)
            X, cen = pack_trajectory(net, tr, seed)
            Y = targets([r.pose for r in res], cen.cpu().numpy())
            Xs.append(X)
            Ys.append(torch.from_numpy(Y.astype(np.float32)).cuda())
            tr.close()
        _log(f"dataset: {min(c0 + chunk, len(seeds))}/{len(seeds)} trajectories")
    return torch.cat(Xs), torch.cat(Ys)


def train(net, X, Y, epochs, batch, lr, seed=0):
    import torch
    P = X.shape[0]
    rng = np.random.default_rng(seed)
    hist = []
    for ep in range(epochs):
        perm = torch.from_numpy(rng.permutation(P)).cuda()
        for b0 in range(0, P - batch + 1, batch):
            idx = perm[b0:b0 + batch]
            loss = net.train_step(X.index_select(0, idx), Y.index_select(0, idx), lr)
        hist.append(float(loss.item()))
        _log(f"epoch {ep + 1}/{epochs}: last batch loss {hist[-1]:.3e}")
    return hist


def evaluate(g, ctx, net, seeds, workers):
    """Registers every pair of the held-out trajectories from the constant-
    velocity initial pose and from the network's, with the fallback."""
    import torch
    prm = _prm(g)
    rows = {"cv": [], "net": [], "net_fallback": []}
    init_err = {"cv": [], "net": []}
    t_cv = t_net = t_net_batched = 0.0
    n_pairs = 0
    for seed, (frames, poses) in zip(seeds, generate(list(seeds), workers)):
        tr = Trajectory(g, ctx, frames, poses)
        labels = [r.pose for r in ctx.register_batch(tr.items(tr.gt), prm)]
        n = len(tr.maps)
        n_pairs += n
        # constant velocity: pair k starts from the estimate of pair k-1 (identity for k = 0)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        cv_res, prev = [], np.eye(4)
        for k in range(n):
            init = prev
            r = ctx.register(tr.frames[k + 1], tr.maps[k], init, prm, src_covs=tr.covs[k + 1])
            cv_res.append((init, r))
            prev = r.pose
        torch.cuda.synchronize()
        t_cv += time.perf_counter() - t0
        # network, one pair at a time (the streaming form)
        t0 = time.perf_counter()
        net_res = []
        for k in range(n):
            si, ti = pair_indices(seed, k, tr.frames[k + 1].shape[1], tr.frames[k].shape[1])
            X, cen = net.pack([(tr.frames[k + 1], tr.frames[k], torch.from_numpy(si).cuda(),
                                torch.from_numpy(ti).cuda())])
            init = net.predict_poses(X, cen)[0].cpu().numpy()
            r = ctx.register(tr.frames[k + 1], tr.maps[k], init, prm, src_covs=tr.covs[k + 1])
            net_res.append((init, r))
        torch.cuda.synchronize()
        t_net += time.perf_counter() - t0
        # network, whole trajectory at once (no pair depends on another)
        t0 = time.perf_counter()
        X, cen = pack_trajectory(net, tr, seed)
        inits = net.predict_poses(X, cen).cpu().numpy()
        ctx.register_batch(tr.items(list(inits)), prm)
        torch.cuda.synchronize()
        t_net_batched += time.perf_counter() - t0
        for k in range(n):
            ic, rc = cv_res[k]
            inn, rn = net_res[k]
            init_err["cv"].append(pose_error(ic, labels[k]))
            init_err["net"].append(pose_error(inn, labels[k]))
            rows["cv"].append((rc.iters, rc.converged and rc.status == 0, *pose_error(rc.pose, labels[k])))
            rows["net"].append((rn.iters, rn.converged and rn.status == 0, *pose_error(rn.pose, labels[k])))
            # fallback: a registration from the network's pose that does not converge is redone from CV
            if rn.converged and rn.status == 0:
                rows["net_fallback"].append(rows["net"][-1])
            else:
                rf = ctx.register(tr.frames[k + 1], tr.maps[k], ic, prm, src_covs=tr.covs[k + 1])
                rows["net_fallback"].append((rn.iters + rf.iters, rf.converged and rf.status == 0,
                                             *pose_error(rf.pose, labels[k])))
        tr.close()
    out = {}
    for name, r in rows.items():
        a = np.array(r, dtype=np.float64)
        out[name] = {"mean_iterations": float(a[:, 0].mean()), "converged_frac": float(a[:, 1].mean()),
                     "mean_rot_err_rad": float(a[:, 2].mean()), "mean_trans_err_m": float(a[:, 3].mean()),
                     "max_trans_err_m": float(a[:, 3].max())}
    for name, e in init_err.items():
        a = np.array(e)
        out[name]["init_mean_rot_err_rad"] = float(a[:, 0].mean())
        out[name]["init_mean_trans_err_m"] = float(a[:, 1].mean())
    out["cv"]["pairs_per_s"] = n_pairs / t_cv
    out["net"]["pairs_per_s"] = n_pairs / t_net
    out["net_batched_pairs_per_s"] = n_pairs / t_net_batched
    out["pairs"] = n_pairs
    return out


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--train", type=int, default=2000, help="training trajectories (100 pairs each)")
    ap.add_argument("--test", type=int, default=100, help="held-out trajectories")
    ap.add_argument("--epochs", type=int, default=8)
    ap.add_argument("--batch", type=int, default=64)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--save", default="", help="write the trained FP32 parameters (.npy)")
    args = ap.parse_args(argv)

    import torch

    import paper_2403_12550_amd as g
    torch.cuda.set_device(0)
    workers = max(1, min(16, len(os.sched_getaffinity(0))))
    ctx = g.Context(0)
    net = ws.WarmStartNet(ctx, args.seed)
    t0 = time.perf_counter()
    X, Y = build_dataset(g, ctx, net, list(range(TRAIN_SEED0, TRAIN_SEED0 + args.train)), workers)
    t_data = time.perf_counter() - t0
    _log(f"dataset: {X.shape[0]} pairs in {t_data:.1f} s")
    t0 = time.perf_counter()
    hist = train(net, X, Y, args.epochs, args.batch, args.lr, args.seed)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    steps = args.epochs * (X.shape[0] // args.batch)
    _log(f"trained {steps} steps in {t_train:.1f} s")
    if args.save:
        np.save(args.save, net.params.cpu().numpy())
    del X, Y
    ev = evaluate(g, ctx, net, list(range(TEST_SEED0, TEST_SEED0 + args.test)), workers)
    out = {"train_pairs": args.train * (N_FRAMES - 1), "test_pairs": ev.pop("pairs"), "epochs": args.epochs,
           "batch": args.batch, "lr": args.lr, "train_steps": steps, "dataset_s": round(t_data, 1),
           "train_s": round(t_train, 2), "train_steps_per_s": round(steps / t_train, 1), "loss_history": hist,
           "eval": ev}
    print(json.dumps(out), flush=True)
    ctx.close()
    return out


if __name__ == "__main__":
    main()
