"""Learned initial guess for the conservative-to-primitive recovery: training set, training and evaluation.

The training states are seeded primitive states (workloads.c2p_states); the library maps them to conserved
variables and to the targets (log W, log(z/D)) with its own prim->cons kernel, computes the network's input
features, and trains the network with its own forward/backward kernels (bfloat16 matrix cores, FP32
accumulate) and Adam.  Evaluation runs the point c2p of the library three ways on the same conserved states:
cold start, warm start from perturbed true primitives, and the network's guess, and reports failures,
Newton iterations, agreement of the recovered primitives and throughput.

    python -m paper_2406_11669_amd.learned [--train 10000000] [--epochs 8] [--block 256]
"""
import argparse
import json
import math
import os
import sys
import time

import numpy as np
import torch

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

from paper_2406_11669_amd import asterx as ax  # noqa: E402
from paper_2406_11669_amd import workloads as W  # noqa: E402

C2P_PARAMS = W.default_params()


def _dev(a, dtype=torch.float64):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda", dtype)


def device_states(states):
    """Upload a c2p_states / c2p_block_states dict; flat metric built on the device when absent."""
    prim = _dev(states["prim"])
    n = prim.shape[1]
    if "metric" in states:
        metric = _dev(states["metric"])
    else:
        metric = torch.zeros((10, n), dtype=torch.float64, device="cuda")
        metric[0] = 1.0
        metric[4] = metric[7] = metric[9] = 1.0
    gam = states["gam"]
    gam = _dev(gam) if isinstance(gam, np.ndarray) else float(gam)
    return dict(prim=prim, Bt=_dev(states["Bt"]), metric=metric, gam=gam, n=n)


def conserved(d, with_targets=False):
    cons = torch.empty((5, d["n"]), dtype=torch.float64, device="cuda")
    tgt = torch.empty((2, d["n"]), dtype=torch.float64, device="cuda") if with_targets else None
    ax.prim2con_points(d["gam"], d["metric"], d["Bt"], d["prim"], cons, tgt)
    return cons, tgt


def features(d, cons):
    feat = torch.empty((8, d["n"]), dtype=torch.float32, device="cuda")
    ax.mlp_features(d["gam"], d["metric"], d["Bt"], cons, feat)
    return feat


def training_set(n, seed=0):
    d = device_states(W.c2p_states(seed, n))
    cons, tgt = conserved(d, with_targets=True)
    feat = features(d, cons)
    return feat, tgt.to(torch.float32)


def standardization(feat, tgt):
    fm, fs = feat.double().mean(1), feat.double().std(1)
    tm, ts = tgt.double().mean(1), tgt.double().std(1)
    return dict(in_shift=fm.cpu().numpy(), in_scale=(1.0 / torch.clamp(fs, min=1e-6)).cpu().numpy(),
                out_shift=tm.cpu().numpy(), out_scale=torch.clamp(ts, min=1e-6).cpu().numpy())


def init_params(seed):
    """Seeded initial parameters (uniform, fan-in scaled; zero biases), packed as the library expects."""
    rng = np.random.default_rng([int(seed), 65521])
    parts = [rng.uniform(-1, 1, 64 * 8) / math.sqrt(8), np.zeros(64), rng.uniform(-1, 1, 64 * 64) / 8.0, np.zeros(64),
             rng.uniform(-1, 1, 2 * 64) / 8.0, np.zeros(2)]
    return np.concatenate(parts).astype(np.float32)


def train(feat, tgt, stdz, epochs=8, batch=16384, lr=3e-3, lr_min=1e-4, seed=0, log=None):
    """Adam on the library's loss gradient; cosine learning-rate decay.  Returns (params, losses per epoch)."""
    n = feat.shape[1]
    params = _dev(init_params(seed), torch.float32)
    m = torch.zeros_like(params)
    v = torch.zeros_like(params)
    grad = torch.zeros(ax.MLP_NPARAMS + 1, dtype=torch.float32, device="cuda")
    ws = torch.empty(ax.mlp_grad_workspace_size(batch) // 4 + 1, dtype=torch.float32, device="cuda")
    mlp = ax.make_mlp(params, stdz)
    gen = torch.Generator(device="cuda")
    gen.manual_seed(int(seed))
    steps_per_epoch = max(1, n // batch)
    total = epochs * steps_per_epoch
    step = 0
    losses = []
    for ep in range(epochs):
        perm = torch.randperm(n, device="cuda", generator=gen)
        acc = torch.zeros((), dtype=torch.float64, device="cuda")
        for b in range(steps_per_epoch):
            idx = perm[b * batch:(b + 1) * batch]
            fb = feat.index_select(1, idx).contiguous()
            tb = tgt.index_select(1, idx).contiguous()
            ax.mlp_grad(mlp, fb, tb, grad, ws)
            acc += grad[ax.MLP_NPARAMS].double()
            step += 1
            rate = lr_min + 0.5 * (lr - lr_min) * (1.0 + math.cos(math.pi * step / total))
            ax.mlp_adam(params, grad, m, v, rate, 0.9, 0.999, 1e-8, step)
        losses.append(float(acc.item()) / steps_per_epoch)
        if log:
            log("epoch %d: mean loss %.4e" % (ep, losses[-1]))
    return params, losses


def c2p_run(d, cons0, mode, mlp=None, guess=None, repeat=3):
    """Point c2p of copies of cons0; mode 'cold', 'warm' (guess) or 'learned' (mlp).  Returns prims, flags,
    iterations, stats and the best time of `repeat` runs in ms."""
    n = d["n"]
    prim = torch.empty((5, n), dtype=torch.float64, device="cuda")
    flags = torch.empty(n, dtype=torch.uint8, device="cuda")
    iters = torch.empty(n, dtype=torch.int32, device="cuda")
    best = None
    for r in range(repeat):
        cons = cons0.clone()
        stats = torch.zeros(7, dtype=torch.int64, device="cuda")
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        ax.c2p_points(C2P_PARAMS, d["gam"], d["metric"], d["Bt"], cons, prim, guess=guess if mode == "warm" else None,
                      mlp=mlp if mode == "learned" else None, flags=flags, iters=iters, stats=stats)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1)
        best = ms if best is None else min(best, ms)
    return prim, flags, iters, stats.cpu().numpy(), best


def _errs(prim, ref, cons):
    """|d rho| / rho and |d p| / (p + tau~) per point."""
    er = (prim[0] - ref[0]).abs() / ref[0].abs()
    ep = (prim[1] - ref[1]).abs() / (ref[1].abs() + cons[4].abs())
    return er, ep


def evaluate(d, mlp, warm_noise=1e-2, seed=0):
    """c2p of the states of d three ways; errors are relative to the cold-start result."""
    cons0, _ = conserved(d)
    g = torch.Generator(device="cuda")
    g.manual_seed(int(seed) + 17)
    warm = d["prim"] * (1.0 + warm_noise * (2.0 * torch.rand(d["prim"].shape, generator=g, device="cuda",
                                                             dtype=torch.float64) - 1.0))
    out = {}
    ref = None
    for mode in ("cold", "warm", "learned"):
        prim, flags, iters, st, ms = c2p_run(d, cons0, mode, mlp=mlp, guess=warm)
        fl = flags.to(torch.int32)
        r = {"noble_failed_frac": float(((fl & 1) != 0).double().mean()),
             "palenzuela_fallback_frac": float(((fl & 2) != 0).double().mean()),
             "hard_fail_frac": float(((fl & 8) != 0).double().mean()),
             "atmosphere_frac": float(((fl & 4) != 0).double().mean()),
             "iters_mean": float(iters.double().mean()), "iters_p99": float(torch.quantile(
                 iters[:min(d["n"], 1 << 24)].double(), 0.99)), "iters_max": int(iters.max()),
             "ms": round(ms, 3), "cells_per_s": d["n"] / (ms * 1e-3)}
        if mode == "learned":
            r["learned_guess_not_converged_frac"] = float(((fl & 32) != 0).double().mean())
        # rho relative to rho; p relative to p + tau (the energy scale: recovering p from tau cancels)
        if ref is None:
            ref = prim
            # accuracy of the recovery itself: cold start against the primitives the states were made from
            er, ep = _errs(prim, d["prim"], cons0)
            r["rho_rel_err_vs_input_max"], r["p_err_vs_input_max"] = float(er.max()), float(ep.max())
            r["rho_rel_err_vs_input_median"] = float(torch.quantile(er[:1 << 24], 0.5))
        else:
            er, ep = _errs(prim, ref, cons0)
            r["rho_rel_diff_vs_cold_max"], r["p_diff_vs_cold_max"] = float(er.max()), float(ep.max())
            r["rho_rel_diff_vs_cold_median"] = float(torch.quantile(er[:1 << 24], 0.5))
        out[mode] = r
    return out


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--train", type=int, default=10_000_000)
    ap.add_argument("--epochs", type=int, default=20)
    ap.add_argument("--batch", type=int, default=16384)
    ap.add_argument("--heldout", type=int, default=1_000_000)
    ap.add_argument("--block", type=int, default=256)
    args = ap.parse_args()
    log = lambda s: print("learned: " + s, file=sys.stderr, flush=True)
    t0 = time.time()
    feat, tgt = training_set(args.train, seed=0)
    torch.cuda.synchronize()
    log("training set of %d states in %.1f s" % (args.train, time.time() - t0))
    stdz = standardization(feat, tgt)
    t0 = time.time()
    params, losses = train(feat, tgt, stdz, epochs=args.epochs, batch=args.batch, log=log)
    torch.cuda.synchronize()
    t_train = time.time() - t0
    mlp = ax.make_mlp(params, stdz)
    del feat, tgt
    held = device_states(W.c2p_states(1, args.heldout))
    res_held = evaluate(held, mlp)
    log("held-out: %s" % json.dumps(res_held))
    del held
    blk = device_states(W.c2p_block_states(2, args.block))
    res_blk = evaluate(blk, mlp)
    log("block: %s" % json.dumps(res_blk))
    print(json.dumps({"train_states": args.train, "epochs": args.epochs, "batch": args.batch,
                      "train_seconds": round(t_train, 2), "loss_per_epoch": losses,
                      "heldout_%d" % args.heldout: res_held, "block_%d^3" % args.block: res_blk}), flush=True)


if __name__ == "__main__":
    main()
