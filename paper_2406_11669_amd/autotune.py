"""Autotuner of the batched persistent launches: times whole RK2 steps of a patch set for every candidate
schedule (workgroups per compute unit x work-list order) and returns the fastest."""
import itertools
import json
import time

import torch

from . import asterx

CANDIDATES = list(itertools.product((1, 2, 4, 8), (0, 1, 2)))


def time_batch(batch, steps=2, graph=True):
    """Milliseconds per step of `batch` (graph replay by default), after one warm-up step."""
    step = batch.step
    if graph:
        side = torch.cuda.Stream()
        side.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(side):
            batch.step()
        torch.cuda.current_stream().wait_stream(side)
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            batch.step()
        step = g.replay
    step()
    torch.cuda.synchronize()
    a = torch.cuda.Event(enable_timing=True)
    b = torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(steps):
        step()
    b.record()
    torch.cuda.synchronize()
    return a.elapsed_time(b) / steps


def tune(workloads, candidates=CANDIDATES, steps=2, log=None):
    """Returns (best tuning, table of (tuning, ms/step))."""
    table = []
    for tun in candidates:
        bt = asterx.Batch(workloads, tuning=tun)
        ms = time_batch(bt, steps=steps)
        table.append((tun, ms))
        if log:
            log("autotune blocks_per_cu=%d order=%d: %.3f ms/step" % (tun[0], tun[1], ms))
        del bt
        torch.cuda.empty_cache()
    best = min(table, key=lambda t: t[1])[0]
    return best, table


def save(path, best, table):
    with open(path, "w") as f:
        json.dump({"best": list(best), "table": [[list(t), ms] for t, ms in table], "time": time.time()}, f)
