"""Gradient check of the differentiation workload on the GPU.

Workload: the periodic Riemann box, 64^3, PPM, HLLE, RK2 at CFL 0.25, 20 steps, Gamma = 5/3, loss
L = (sum over owned cells of rho^2 dV)^(1/2) at the final time; parameters: the initial velocity field
(3 x 64^3 values) and Gamma.  The gradient comes from the hand-written adjoint with per-stage
checkpoints (one forward + one reverse pass).  It is checked against
  * central finite differences of the GPU forward (step h, default 1e-6) along seeded unit directions;
  * the CPU oracle's dual-number directional derivatives stored in tests/golden (when the file exists).
Prints one JSON line with the timings and the error statistics.

At the Riemann problem's rest state (v_amp = 0) every cell sits on a limiter tie, where the loss is not
differentiable in v; the default base point adds a seeded smooth velocity field (v_amp = 0.1).
"""
import argparse
import json
import os
import sys
import time

import numpy as np
import torch

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

from paper_2406_11669_amd import adjoint as adj  # noqa: E402
from paper_2406_11669_amd import workloads as W  # noqa: E402

GOLDEN = os.path.join(ROOT, "tests", "golden", "periodic_riemann64_jvp.json")


def gradient(runner, prim_np, gamma, nsteps):
    prim = torch.from_numpy(prim_np.copy()).cuda().requires_grad_(True)
    gam = torch.tensor(gamma, dtype=torch.float64, device="cuda", requires_grad=True)
    t0, t1, t2 = (torch.cuda.Event(enable_timing=True) for _ in range(3))
    t0.record()
    loss = adj.density_loss_run(runner, prim, gam, nsteps)
    t1.record()
    loss.backward()
    t2.record()
    torch.cuda.synchronize()
    return (float(loss.item()), prim.grad.detach().cpu().numpy(), float(gam.grad.item()),
            t0.elapsed_time(t1), t1.elapsed_time(t2))


def directional(L, g, gg, d, dg):
    terms = L.owned(g)[2:5] * L.owned(d)[2:5]
    return float(np.sum(terms)) + gg * dg, float(np.sum(np.abs(terms))) + abs(gg * dg)


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--n", type=int, default=64)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--dirs", type=int, default=200)
    ap.add_argument("--h", type=float, default=1e-6)
    ap.add_argument("--v-amp", type=float, default=0.1)
    args = ap.parse_args()
    torch.cuda.set_device(0)
    w = W.periodic_riemann_box(seed=0, n=args.n, nsteps=args.steps, v_amp=args.v_amp)
    L = w.layout
    g0 = w.params["gamma"]
    runner = adj.Runner(w)
    gradient(runner, w.prim, g0, 1)  # warm-up (code objects, allocator)
    loss, g, gg, ms_fwd, ms_bwd = gradient(runner, w.prim, g0, args.steps)
    print("gradcheck: loss %.15e, forward %.1f ms, reverse %.1f ms, dL/dGamma %.6e" % (loss, ms_fwd, ms_bwd, gg),
          file=sys.stderr, flush=True)
    prim0 = torch.from_numpy(w.prim).cuda()
    rel, nrm = [], []
    t0 = time.perf_counter()
    for s in range(args.dirs):
        d, dg = W.gradient_direction(L, s)
        dt = torch.from_numpy(d).cuda()
        lp = adj.density_loss_value(runner, prim0 + args.h * dt, g0 + args.h * dg, args.steps)
        lm = adj.density_loss_value(runner, prim0 - args.h * dt, g0 - args.h * dg, args.steps)
        fd = (lp - lm) / (2.0 * args.h)
        mine, scale = directional(L, g, gg, d, dg)
        rel.append(abs(fd - mine) / abs(mine))
        nrm.append(abs(fd - mine) / scale)
        if s % 25 == 0:
            print("gradcheck: direction %d fd %.10e adjoint %.10e rel %.2e" % (s, fd, mine, rel[-1]),
                  file=sys.stderr, flush=True)
    t_fd = time.perf_counter() - t0
    rel, nrm = np.array(rel), np.array(nrm)
    out = {"workload": "periodic_riemann%d-ppm-rk2, %d steps, v_amp %g" % (args.n, args.steps, args.v_amp),
           "loss": loss, "dL_dGamma": gg, "grad_v_norm": float(np.sqrt(np.sum(L.owned(g)[2:5] ** 2))),
           "adjoint_ms": {"forward_with_checkpoints": round(ms_fwd, 2), "reverse": round(ms_bwd, 2)},
           "fd": {"h": args.h, "directions": args.dirs, "seconds": round(t_fd, 1),
                  "rel_err_median": float(np.median(rel)), "rel_err_p95": float(np.percentile(rel, 95)),
                  "frac_rel_err_le_1e-5": float(np.mean(rel <= 1e-5)),
                  "scaled_err_median": float(np.median(nrm)), "scaled_err_max": float(np.max(nrm))}}
    if os.path.exists(GOLDEN) and args.n == 64 and args.steps == 20:
        with open(GOLDEN) as f:
            gold = json.load(f)
        rows = []
        for c in gold["cases"]:
            if abs(c["v_amp"] - args.v_amp) > 0:
                continue
            if c["dir_seed"] is None:
                d, dg = L.zeros(5), 1.0
            else:
                d, dg = W.gradient_direction(L, c["dir_seed"], c["with_gamma"])
            mine, scale = directional(L, g, gg, d, dg)
            rows.append({"dir_seed": c["dir_seed"], "with_gamma": c["with_gamma"], "oracle_jvp": c["jvp"],
                         "adjoint": mine, "rel_err": abs(mine - c["jvp"]) / abs(c["jvp"]),
                         "scaled_err": abs(mine - c["jvp"]) / scale,
                         "loss_rel_err": abs(loss - c["loss"]) / c["loss"]})
        out["vs_oracle_jvp"] = rows
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
