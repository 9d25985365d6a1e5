"""Benchmark of the batched form: 512 AMR-like patches (sides 16/24/32/48 + 3 ghosts, 3 levels, Riemann
problems, MINMOD, HLLE, RK2), all advanced per phase by one persistent launch and captured in a HIP graph,
with the schedule picked by the autotuner; against the per-patch launch loop (eager and graph-captured).

python -m paper_2406_11669_amd.bench_batched [--npatches 512] [--steps 3]
Prints one JSON line (zone-updates per RK stage per second for each form)."""
import argparse
import json
import sys

import torch

from . import asterx, autotune
from . import workloads as W


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--npatches", type=int, default=512)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--no-tune", action="store_true")
    args = ap.parse_args()
    log = lambda m: print(m, file=sys.stderr, flush=True)
    wls = W.patch_set(seed=0, npatches=args.npatches)
    cells = sum(w.layout.n[0] * w.layout.n[1] * w.layout.n[2] for w in wls)
    zs = cells * 2  # RK2: two stages per step
    log("patch set: %d patches, %d interior cells" % (len(wls), cells))
    if args.no_tune:
        best, table = (4, 1), []
    else:
        best, table = autotune.tune(wls, log=log)
    bt = asterx.Batch(wls, tuning=best)
    ms_batched = autotune.time_batch(bt, steps=args.steps, graph=True)
    del bt
    torch.cuda.empty_cache()
    log("batched (graph): %.3f ms/step" % ms_batched)

    class Loop:
        def __init__(self):
            self.blocks = [asterx.Block(w) for w in wls]

        def step(self):
            for b in self.blocks:
                b.step()

    loop = Loop()
    ms_loop_eager = autotune.time_batch(loop, steps=args.steps, graph=False)
    log("per-patch loop (eager): %.3f ms/step" % ms_loop_eager)
    ms_loop_graph = autotune.time_batch(loop, steps=args.steps, graph=True)
    log("per-patch loop (graph): %.3f ms/step" % ms_loop_graph)
    out = {"metric": "zone-updates/s per RK stage, 512 AMR-like patches", "unit": "zone-updates/s",
           "interior_cells": cells, "npatches": len(wls),
           "batched_graph": zs / (ms_batched * 1e-3), "per_patch_loop_eager": zs / (ms_loop_eager * 1e-3),
           "per_patch_loop_graph": zs / (ms_loop_graph * 1e-3),
           "ms_per_step": {"batched_graph": ms_batched, "loop_eager": ms_loop_eager, "loop_graph": ms_loop_graph},
           "tuning": {"best": list(best), "table": [[list(t), ms] for t, ms in table]}}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
