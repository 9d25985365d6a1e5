#!/usr/bin/env python3
"""Benchmark of the FP64 GRMHD right-hand side on one MI355X.

Workload: the 128^3 periodic block in a static curved 3+1 metric (seeded low-k mode sums), Gamma = 2, PPM
reconstruction, HLLE, quartic characteristic speeds, Noble c2p, RK4 at CFL 0.25.  A step is one whole RK4
step (4 stages: c2p, primitive ghost fill, right-hand side, combine, state ghost fill), replayed from a
captured HIP graph, with all inputs resident in HBM.

Prints one JSON line: zone-updates/s per RK stage (interior cells x stages / wall time of the timed steps); the
roofline of the dominant kernel and per-kernel figures of the face kernels, the recovery with sources and the
divergence kernel (per-kernel HIP events recorded live on the launch stream); the whole-stage HBM and FP64
rooflines; the same block with the other reconstruction, batched patches against a per-patch loop, the learned
recovery guess against the plain one, one adjoint gradient, forward and reverse, and the paper's own single-GPU
benchmark (its Setup A, a magnetized TOV star at 240^3) in the paper's zone-cycles/s beside the paper's figure
(comparison keys); and the CPU oracle timed on the host (serial on a bounded sample, all cores on the full block).
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "zone-updates/s per RK stage (FP64, 128^3) and % of HBM roofline"
HBM_PEAK_GBS = 8000.0        # MI355X HBM3E, GB/s
FP64_VECTOR_PEAK_TFLOPS = 78.6   # MI355X FP64 vector (256 CUs x 128 FLOP/clk x 2.4 GHz)

# A-priori estimates of the work per unit, made before any implementation existed (and +-50%): about 1.4 kFLOP
# per face (reconstruction, prim->cons and fluxes of both sides, quartic Newton, HLLE; the face metric is counted
# with the metric interpolation) and about 6.4 kFLOP per zone-stage in all; 514 B per zone-stage of RK4.
SURVEY_FLOPS_PER_FACE = 1400.0
SURVEY_FLOPS_PER_ZONE_STAGE = 6400.0
# Algorithmic FP64 operations per face of the face kernel (reconstruction of 7 variables on both sides,
# 16-point face metric of 10 components, prim->cons, fluxes, quartic speeds, HLLE or LxF), counted by running
# the plain serial implementation on an operation-counting scalar (+, -, *, /, sqrt, pow = 1 each) over the
# 3 x 129^3 faces of the 128^3 block of this workload (same seed and recipe; limiter branches make the count
# data dependent).
FACE_FLOPS = {"ppm": 2603.1, "wenoz": 3955.0, "minmod": 2022.6, "mp5": 2480.3, "ppm+lxf": 2581.1,
              "ppm+hlle+uct": 2620.8}
# The same count per owned cell of the cell kernel (centre metric values and derivatives, curvature values,
# sources, flux divergence) and of the recovery (centre metric values, centre field, geometry, warm-started
# Noble iteration) on that block.
CELL_FLOPS = 4716.0
C2P_FLOPS = 1795.0
# The benchmark's stage evaluates the sources in the recovery kernel (asterx_c2p_src) and leaves the flux
# divergence, div B and the stage outputs to a streaming kernel (asterx_rhs_rk_src).  Counted per cell: the
# divergence 5 components x (3 differences, 3 divisions by the spacing, 3 additions, 1 source addition) = 50, and
# div B 6 face curls x 5 (the counter's face_B) + 3 differences + 3 divisions + 2 additions = 38; the recovery
# with sources is the recovery plus the cell count without these, less the ten centre metric values the two
# counts both contain (10 x 147, the counter's centre_value), which the fused kernel interpolates once.
DIV_FLOPS = 50.0 + 38.0
C2P_SRC_FLOPS = C2P_FLOPS + CELL_FLOPS - DIV_FLOPS - 10 * 147.0
# Algorithmic bytes per face: read 5 primitives + 2 centre fields + 10 face-metric components + 2 potential
# components, write 7 face fluxes (each value once, stencil reuse served on chip).
FACE_BYTES = 8.0 * (5 + 2 + 10 + 2 + 7)
# Per owned cell of the cell kernel: metric and curvature (16), primitives (5), centre field (3) and the 15 hydro
# face fluxes read once; RK4 stage outputs of the 5 hydro fields averaged over the four stages (1.5 states read,
# 1.75 written).
CELL_BYTES_RK4 = 8.0 * (16 + 5 + 3 + 15 + 1.5 * 5 + 1.75 * 5)
# Per owned cell of the recovery: conserved (5), potential (3), metric (10), previous primitives (5) read,
# primitives (5) written.
C2P_BYTES = 8.0 * (5 + 3 + 10 + 5 + 5)
# Per owned cell of the recovery with sources: the recovery's and the curvature (6) read; the primitives (5), the
# densitized sources (4) and the metric at the cell's lower x face (10, handed to the x-face kernel) written.
C2P_SRC_BYTES = 8.0 * (5 + 3 + 10 + 6 + 5 + 5 + 4 + 10)
# Per owned cell of the divergence kernel: the 15 hydro face fluxes, the 4 sources and the potential (3, for
# div B) read once; RK4 stage outputs of the 5 hydro fields as for the cell kernel.
DIV_BYTES_RK4 = 8.0 * (15 + 4 + 3 + 1.5 * 5 + 1.75 * 5)
# Whole-stage algorithmic HBM bytes per zone-stage, RK4 averaged over its four stages: reads of the stage
# state (9), metric and curvature (16), previous primitives (5), RK base state and accumulator (9 + 9 when
# used); writes of primitives (5), next state (9) and accumulator (9 when used).
STAGE_BYTES_RK4 = 514.0
# Whole-stage algorithmic FP64 operations per zone-stage at 128^3 (same counting scalar, over one
# right-hand side and one c2p of the 128^3 block of this workload; for PPM: centre field 41, faces of
# the three directions 7994, cell sources and divergence 4716, constrained transport and gauge 139, c2p
# 1795; the RK combine's 2 operations per field are not counted).
STAGE_FLOPS = {"ppm": 14684.9, "wenoz": 18836.6, "minmod": 12902.4, "mp5": 14307.9, "ppm+lxf": 14617.3,
               "ppm+hlle+uct": 16669.8}  # upwind CT: 129 x 133^2 faces per direction, edge field 1561
RIDGE = FP64_VECTOR_PEAK_TFLOPS * 1e3 / HBM_PEAK_GBS   # FLOP/B where the FP64 and HBM roofs meet


def library_source_sha():
    """First 16 hex digits of the sha256 of the HIP sources the library is built from and of the flags that
    decide its code."""
    import hashlib
    from paper_2406_11669_amd.build import CODEGEN_FLAGS
    csrc = os.path.join(ROOT, "paper_2406_11669_amd", "csrc")
    h = hashlib.sha256()
    for name in ("asterx.hip", "grmhd_device.h"):
        with open(os.path.join(csrc, name), "rb") as f:
            h.update(f.read())
    h.update(" ".join(CODEGEN_FLAGS).encode())
    return h.hexdigest()[:16]


def measured_face_traffic(recon, n):
    """HBM bytes per face-kernel launch from the committed rocprofv3 counter summary (FETCH_SIZE and WRITE_SIZE
    scaled by a plain copy), or None when no summary exists for this workload or it was taken on other sources."""
    path = os.path.join(ROOT, "profiles", "face_curved%d_%s_hbm_traffic.md" % (n, recon))
    if not os.path.exists(path):
        return None
    value, sha = None, None
    with open(path) as f:
        for line in f:
            if line.startswith("face kernel, average of the three directions: traffic bytes per launch:"):
                value = float(line.rsplit(":", 1)[1])
            elif line.startswith("library source sha256"):
                sha = line.rsplit(":", 1)[1].strip()
    return value if (value is not None and sha == library_source_sha()) else None


def parse():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--n", type=int, default=128)
    ap.add_argument("--recon", default="ppm", choices=["ppm", "wenoz", "minmod", "mp5"])
    ap.add_argument("--riemann", default="hlle", choices=["hlle", "lxf"])
    ap.add_argument("--ct", default="fct", choices=["fct", "uct"],
                    help="edge electric field: flux CT or upwind CT (4 ghost layers)")
    ap.add_argument("--no-graph", action="store_true", help="launch eagerly instead of replaying a HIP graph")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the comparison keys (other scheme, batched patches, learned guess, T_munu, inter-level)")
    ap.add_argument("--cpu-n", type=int, default=88, help="edge of the block the CPU oracle times")
    ap.add_argument("--learned-c2p", action="store_true",
                    help="seed every c2p with the learned guess (network trained first, outside the timed region)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run three plain device copies of 256 MiB (reference for the HBM byte counters)")
    return ap.parse_args()


def copy_calibration():
    """Three device-to-device copies of 256 MiB each: a kernel whose HBM traffic is known exactly (256 MiB read
    and 256 MiB written per launch), so that FETCH_SIZE / WRITE_SIZE per dispatch can be scaled to bytes."""
    import torch
    n = 256 * 1024 * 1024 // 8
    a = torch.ones(n, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    torch.cuda.synchronize()
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_calibration_bytes_per_launch": n * 8, "launches": 3}), flush=True)


def host_cpu():
    """CPU model, logical CPUs of the machine and CPUs this process may run on."""
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        usable = len(os.sched_getaffinity(0))
    except AttributeError:
        usable = os.cpu_count()
    return {"cpu_model": model, "nproc": os.cpu_count(), "usable_cpus": usable}


def cpu_baseline(recon, riemann, ct, n_cpu, w_full=None):
    """The oracle, as it stands, on the same workload recipe: the serial build on one RK4 step of an n_cpu^3 block
    (about 10 s on one core), and the OpenMP build of the same source (k-planes over threads, bitwise the same
    results) on one RK4 step of the full block w_full with every usable CPU (capped by OMP_NUM_THREADS)."""
    from oracle import oracle as O
    from paper_2406_11669_amd import workloads as W
    O.build(force=False)

    def one_step(w, lib_=None):
        w.params["riemann"] = riemann
        w.params["ct"] = ct
        L = w.layout
        cons = O.prim2con(L, w.params, w.metric, w.A, w.prim)
        O.fill_ghosts(L, cons, w.bc_cell)
        state = w.state(cons)
        prim = w.prim.copy()
        t0 = time.perf_counter()
        O.run(L, w.params, w.metric, w.curv, state, prim, w.dt, 1, 4, w.bc_cell, w.bc_A, lib_=lib_)
        return time.perf_counter() - t0

    host = host_cpu()
    w = W.curved_block(seed=0, n=n_cpu, recon=recon, nsteps=1, ng=4 if ct == "uct" else 3)
    dt = one_step(w)
    out = {"value": n_cpu ** 3 * 4 / dt, "unit": "zone-updates/s", "cores": 1, "kind": "oracle",
           "sample": "one RK4 step (4 stages) of the %d^3 block of the same workload recipe, serial FP64 oracle "
                     "(g++ -O2 -ffp-contract=off), %.1f s" % (n_cpu, dt), "host": host}
    if w_full is not None:
        threads = host["usable_cpus"]
        if os.environ.get("OMP_NUM_THREADS", "").isdigit():
            threads = min(threads, int(os.environ["OMP_NUM_THREADS"]))
        lo, used = O.lib_omp(threads)
        n = w_full.layout.n
        dt = one_step(w_full, lib_=lo)
        out["all_cores"] = {"value": n[0] * n[1] * n[2] * 4 / dt, "unit": "zone-updates/s", "cores": used,
                            "kind": "oracle",
                            "sample": "one RK4 step of the full %dx%dx%d block, the same oracle source built with "
                                      "-fopenmp (k-planes over %d threads), %.1f s" % (n[0], n[1], n[2], used, dt)}
    return out


def time_inter_level(asterx, torch, n, reps=10):
    """Factor-2 inter-level operators on the 9 state fields (5 conserved: cell; A_x, A_y, A_z: edges; Psi: vertex):
    prolongation of every point of an n^3 fine block with 3 ghost layers from a coarse block, then restriction of
    the coarse cells its owned cells cover.  HIP events around reps repetitions.  Algorithmic bytes: each fine
    point written once and each coarse value read once (prolongation); each fine value read once and each coarse
    point written once (restriction)."""
    from paper_2406_11669_amd.workloads import Layout
    nc = n // 2 + 8
    coarse, fine = Layout((nc,) * 3, 3), Layout((n,) * 3, 3)
    c0 = (4, 4, 4)
    f64 = dict(dtype=torch.float64, device="cuda")
    gen = torch.Generator(device="cuda")
    gen.manual_seed(5)
    cf = torch.rand((9,) + coarse.shape3, generator=gen, **f64)
    ff = torch.zeros((9,) + fine.shape3, **f64)
    back = torch.zeros_like(cf)
    flo, fhi = (-3, -3, -3), (n + 2,) * 3
    clo, chi = c0, tuple(c + n // 2 - 1 for c in c0)
    parts = [(slice(0, 5), "cell"), (slice(5, 6), "xedge"), (slice(6, 7), "yedge"), (slice(7, 8), "zedge"),
             (slice(8, 9), "vertex")]

    def prolong_all():
        for sl, st in parts:
            asterx.prolong(coarse, fine, c0, st, cf[sl], ff[sl], flo, fhi)

    def restrict_all():
        for sl, st in parts:
            asterx.restrict(coarse, fine, c0, st, ff[sl], back[sl], clo, chi)

    out = {}
    for name, fn in (("prolong", prolong_all), ("restrict", restrict_all)):
        fn()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / reps
        if name == "prolong":
            pts = 9 * (n + 6) ** 3
            nbytes = 8.0 * (pts + 9 * (n // 2 + 5) ** 3)
        else:
            pts = 9 * (n // 2) ** 3
            nbytes = 8.0 * (pts * 8 + pts)
        gbs = nbytes / (ms * 1e-3) / 1e9
        out[name] = {"ms": round(ms, 4), "points_per_s": pts / (ms * 1e-3), "algorithmic_GBs": round(gbs, 1),
                     "hbm_frac": round(gbs / HBM_PEAK_GBS, 4)}
    return out


def time_tmunu(asterx, torch, blk, n, reps=20):
    """T_{mu nu} at the (n+1)^3 vertices of the block's current state (asterx_tmunu), HIP events around reps
    launches on the current stream.  Algorithmic bytes per vertex: 5 primitives, 3 potential components and 10
    metric components read once, 10 components written (224 B)."""
    out = torch.empty((10,) + blk.L.shape3, dtype=torch.float64, device="cuda")
    args = (blk.L, blk.params, blk.metric, blk.prim, blk.state[5:8], out)
    asterx.tmunu(*args)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        asterx.tmunu(*args)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    nv = (n + 1) ** 3
    gbs = 224.0 * nv / (ms * 1e-3) / 1e9
    return {"ms": round(ms, 4), "vertices_per_s": nv / (ms * 1e-3), "algorithmic_GBs": round(gbs, 1),
            "hbm_frac": round(gbs / HBM_PEAK_GBS, 4)}


def graph_steps(torch, blk, steps, warmup, graph=True):
    """Time `steps` whole steps of blk (after `warmup`), replayed from one captured HIP graph unless graph is
    False.  Returns ms for all steps (HIP events on the current stream, synchronized on both sides)."""
    step = blk.step
    if graph:
        side = torch.cuda.Stream()
        side.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(side):
            blk.step()  # first step eagerly on the capture stream
        torch.cuda.current_stream().wait_stream(side)
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            blk.step()
        step = g.replay
    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    t0.record()
    for _ in range(steps):
        step()
    t1.record()
    torch.cuda.synchronize()
    return t0.elapsed_time(t1)


def kernel_rooflines(kt, stages, n, scheme, ct):
    """Per-kernel figures from the live HIP-event durations kt (one eager step): the face kernel (three direction
    launches per stage, averaged), the recovery with sources (timed under "c2p") and the divergence kernel (timed
    under "cell"), each against both roofs.  Achieved figures are algorithmic work per launch (per-unit figure x
    units per launch) over the average launch duration."""
    cells = n ** 3
    faces = (n + 1) ** 3 if ct == "fct" else (n + 1) * (n + 5) ** 2
    face_keys = ("face_x", "face_y", "face_z")
    face_ms = sum(kt[k][0] for k in face_keys) / max(1, sum(kt[k][1] for k in face_keys))
    rows = {
        "face": dict(ms=face_ms, launches_per_stage=3, units="faces", units_per_launch=faces,
                     flops={"estimate": SURVEY_FLOPS_PER_FACE, "oracle_count": FACE_FLOPS.get(scheme)},
                     bytes=FACE_BYTES),
        "c2p_src": dict(ms=kt["c2p"][0] / max(1, kt["c2p"][1]), launches_per_stage=1, units="cells",
                        units_per_launch=cells, flops={"oracle_count": C2P_SRC_FLOPS}, bytes=C2P_SRC_BYTES),
        "divergence": dict(ms=kt["cell"][0] / max(1, kt["cell"][1]), launches_per_stage=1, units="cells",
                           units_per_launch=cells, flops={"oracle_count": DIV_FLOPS}, bytes=DIV_BYTES_RK4),
    }
    out = {}
    for name, r in rows.items():
        sec = r["ms"] * 1e-3
        gbs = r["bytes"] * r["units_per_launch"] / sec / 1e9
        e = {"ms_per_launch": round(r["ms"], 4), "launches_per_stage": r["launches_per_stage"],
             "units": r["units"], "units_per_launch": r["units_per_launch"], "bytes_per_unit": r["bytes"],
             "algorithmic_GBs": round(gbs, 1), "hbm_frac": round(gbs / HBM_PEAK_GBS, 4),
             "flops_per_unit": r["flops"]}
        for src, f in r["flops"].items():
            if f:
                tf = f * r["units_per_launch"] / sec / 1e12
                e["fp64_TFLOPs_" + src] = round(tf, 3)
                e["fp64_frac_" + src] = round(tf / FP64_VECTOR_PEAK_TFLOPS, 4)
        out[name] = e
    return out


def headline_roofline(kr, kt, stages, scheme, n):
    """The roofline of the dominant kernel: the kernel function with the largest total time per stage (the face
    kernel's three direction launches are one kernel).  Its bound follows from the arithmetic intensity of the
    a-priori per-unit figures (FLOP/B against the ridge of the two roofs)."""
    per_stage = {"face": kr["face"]["ms_per_launch"] * 3, "divergence": kr["divergence"]["ms_per_launch"],
                 "c2p_src": kr["c2p_src"]["ms_per_launch"]}
    for k, v in kt.items():
        if k not in ("face_x", "face_y", "face_z", "cell", "c2p") and v[1] > 0:
            per_stage[k] = v[0] / stages
    dom = max(per_stage, key=per_stage.get)
    largest_launch = max(((k, v[0] / max(1, v[1])) for k, v in kt.items() if v[1] > 0), key=lambda kv: kv[1])[0]
    e = kr.get(dom, kr["face"])
    if dom not in kr:
        dom = "face"
    est = e["flops_per_unit"].get("estimate") or e["flops_per_unit"].get("oracle_count")
    intensity = est / e["bytes_per_unit"]
    bound = "hbm" if intensity < RIDGE else "alu"
    if bound == "hbm":
        achieved, peak, unit = e["algorithmic_GBs"], HBM_PEAK_GBS, "GB/s"
    else:
        achieved = est * e["units_per_launch"] / (e["ms_per_launch"] * 1e-3) / 1e12
        peak, unit = FP64_VECTOR_PEAK_TFLOPS, "TFLOP/s"
    return {"kernel": dom + (" (x, y, z launches averaged)" if dom == "face" else ""),
            "dominant_by": "kernel time per stage (%s)" % ", ".join("%s %.3f ms" % kv for kv in sorted(
                per_stage.items(), key=lambda kv: -kv[1])[:4]),
            "largest_single_launch": largest_launch, "bound": bound, "achieved": round(achieved, 3), "peak": peak,
            "unit": unit, "frac": round(achieved / peak, 4),
            "traffic": measured_face_traffic(scheme, n) if dom == "face" else None,
            "avg_launch_ms": e["ms_per_launch"], "units_per_launch": e["units_per_launch"],
            "flops_per_unit": e["flops_per_unit"], "bytes_per_unit": e["bytes_per_unit"],
            "intensity_flop_per_byte": round(intensity, 2), "ridge_flop_per_byte": round(RIDGE, 2),
            "fp64_frac_estimate": e.get("fp64_frac_estimate"), "fp64_frac_oracle_count": e.get("fp64_frac_oracle_count")}


def extra_scheme(torch, asterx, w, recon, steps):
    """The same block and inputs with another reconstruction: graph-replayed RK4 steps."""
    import copy
    w2 = copy.copy(w)
    w2.params = dict(w.params, recon=recon)
    blk = asterx.Block(w2)
    ms = graph_steps(torch, blk, steps, 1)
    n = w.layout.n
    del blk
    torch.cuda.empty_cache()
    return {"value": n[0] * n[1] * n[2] * 4 * steps / (ms * 1e-3), "unit": "zone-updates/s",
            "ms_per_step": round(ms / steps, 4)}


def extra_batched(torch, asterx, W, npatches=128, steps=3):
    """A reduced set of the AMR-like patches (sides 16/24/32/48 + 3 ghosts, 3 levels, Riemann problems, MINMOD,
    HLLE, RK2): the persistent batch (graph) against the per-patch launch loop (graph) and against one block of
    about the same cell count with the same scheme."""
    from paper_2406_11669_amd import autotune
    wls = W.patch_set(seed=0, npatches=npatches)
    cells = sum(w.layout.n[0] * w.layout.n[1] * w.layout.n[2] for w in wls)
    bt = asterx.Batch(wls, tuning=(8, 0))
    ms_b = autotune.time_batch(bt, steps=steps, graph=True)
    del bt

    class Loop:
        def __init__(self):
            self.blocks = [asterx.Block(w) for w in wls]

        def step(self):
            for b in self.blocks:
                b.step()

    loop = Loop()
    ms_l = autotune.time_batch(loop, steps=steps, graph=True)
    del loop
    side = int(round(cells ** (1.0 / 3.0)))
    one = asterx.Block(W.riemann_block(seed=0, n=side, nsteps=steps))
    ms_1 = graph_steps(torch, one, steps, 1)
    del one
    torch.cuda.empty_cache()
    zs = 2.0 * cells  # per step (time_batch returns milliseconds per step)
    return {"npatches": npatches, "interior_cells": cells, "unit": "zone-updates/s",
            "batched_graph": zs / (ms_b * 1e-3), "per_patch_loop_graph": zs / (ms_l * 1e-3),
            "single_block_%d^3" % side: 2.0 * side ** 3 * steps / (ms_1 * 1e-3), "tuning": [8, 0]}


def extra_learned(torch, asterx, blk, steps, n_points=256, n_train=10_000_000, epochs=20):
    """The learned initial guess of the recovery: a network trained by the library's kernels (n_train states,
    `epochs` epochs, outside the timed regions), then (a) point recoveries of an n_points^3 block of per-cell
    states (Riemann-problem ranges, W ~ U[1, 10]) from the plain cold start and from the network, (b) the benchmark
    block stepped with the network in every recovery against the plain warm start."""
    from paper_2406_11669_amd import learned
    from paper_2406_11669_amd import workloads as W
    t0 = time.perf_counter()
    feat, tgt = learned.training_set(n_train, seed=0)
    stdz = learned.standardization(feat, tgt)
    params, losses = learned.train(feat, tgt, stdz, epochs=epochs, batch=16384, seed=0)
    del feat, tgt
    mlp = asterx.make_mlp(params, stdz)
    torch.cuda.synchronize()
    setup = time.perf_counter() - t0
    d = learned.device_states(W.c2p_block_states(2, n_points))
    res = learned.evaluate(d, mlp)
    del d
    torch.cuda.empty_cache()
    pts = {m: {k: res[m][k] for k in ("cells_per_s", "iters_mean", "noble_failed_frac", "hard_fail_frac")}
           for m in ("cold", "learned")}
    n = blk.L.n
    plain_ms = graph_steps(torch, blk, steps, 1)
    blk.mlp = mlp
    blk._mlp_params = params
    learned_ms = graph_steps(torch, blk, steps, 1)
    blk.mlp = None
    zs = n[0] * n[1] * n[2] * 4 * steps
    return {"train_states": n_train, "epochs": epochs, "final_loss": round(losses[-1], 5),
            "setup_seconds": round(setup, 1), "points_%d^3" % n_points: pts,
            "pipeline": {"plain_warm_start": zs / (plain_ms * 1e-3), "learned": zs / (learned_ms * 1e-3),
                         "unit": "zone-updates/s"}}


def extra_adjoint(torch, W, reps=3):
    """One gradient of the differentiation workload (64^3 periodic Riemann box, PPM, 20 RK2 steps, loss = the L2
    norm of the final density) with respect to the initial primitives and Gamma: the forward pass with per-stage
    checkpoints and the reverse pass timed apart, wall clock with the device synchronized (the last of reps runs;
    the first one also initialises)."""
    from paper_2406_11669_amd import adjoint as adj
    w = W.periodic_riemann_box(seed=0, n=64, nsteps=20, v_amp=0.1)
    runner = adj.Runner(w)
    for _ in range(reps):
        prim = torch.from_numpy(w.prim.copy()).cuda().requires_grad_(True)
        gam = torch.tensor(w.params["gamma"], dtype=torch.float64, device="cuda", requires_grad=True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        loss = adj.density_loss_run(runner, prim, gam, 20)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        loss.backward()
        torch.cuda.synchronize()
        t2 = time.perf_counter()
    del runner
    torch.cuda.empty_cache()
    return {"workload": "periodic_riemann64-ppm-rk2, 20 steps", "forward_ms": round(1e3 * (t1 - t0), 2),
            "reverse_ms": round(1e3 * (t2 - t1), 2), "reverse_over_forward": round((t2 - t1) / (t1 - t0), 2)}


# The paper's single-GPU benchmark (its Setup A): a magnetized TOV star in a static (Cowling) spacetime on a
# uniform 240^3 grid, PPM + HLLE, RK4, Neumann (copy) boundaries, 3 ghosts: 0.27e8 zone-cycles/s on one MI250X
# GCD, a zone-cycle being one cell advanced one whole RK4 step.
PAPER_SETUP_A_ZCS = 0.27e8


def extra_setup_a(torch, asterx, W, steps, n=240, extent=40.0):
    """The paper's Setup A on this GPU: the K = 100, Gamma = 2 polytrope with central density 1.28e-3 in its
    fixed isotropic metric, the field of A_phi = A_b varpi^2 max(p - 0.04 p_max, 0)^2 with A_b giving a largest
    field of about 1e14 G, rho_atm = 1e-7 rho_c, on [-20, 20]^3 (the extent of the finest level of the
    paper's TOV runs; the benchmark's own extent is not printed) with 240^3 cells: graph-replayed RK4 steps."""
    w = W.magnetized_star_block(n=n, extent=extent)
    blk = asterx.Block(w)
    ms = graph_steps(torch, blk, steps, 1)
    value = n ** 3 * 4 * steps / (ms * 1e-3)
    stats = [int(v) for v in blk.stats.cpu().tolist()]
    del blk
    torch.cuda.empty_cache()
    return {"workload": "magnetized TOV star, Cowling, %d^3 on [-%g, %g]^3, PPM, HLLE, RK4, copy boundaries"
                        % (n, 0.5 * extent, 0.5 * extent),
            "value": value, "unit": "zone-updates/s", "ms_per_step": round(ms / steps, 4),
            "zone_cycles_per_s": value / 4, "paper_zone_cycles_per_s_one_mi250x_gcd": PAPER_SETUP_A_ZCS,
            "ratio_to_paper": round(value / 4 / PAPER_SETUP_A_ZCS, 2), "c2p_stats": stats}


def main():
    args = parse()
    if args.copy_calibration:
        copy_calibration()
        return
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one block on one GPU; a run on more than one GPU would need the domain "
              "decomposition with halo exchange, which is not implemented", file=sys.stderr)
        sys.exit(2)
    import torch

    from paper_2406_11669_amd import asterx
    from paper_2406_11669_amd import workloads as W

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    n = args.n
    w = W.curved_block(seed=0, n=n, recon=args.recon, nsteps=args.steps, ng=4 if args.ct == "uct" else 3)
    w.params["riemann"] = args.riemann
    w.params["ct"] = args.ct
    scheme = args.recon
    if args.riemann != "hlle" or args.ct != "fct":
        scheme += "+" + args.riemann
    if args.ct != "fct":
        scheme += "+" + args.ct
    blk = asterx.Block(w)
    learned_info = None
    if args.learned_c2p:
        from paper_2406_11669_amd import learned
        t0 = time.perf_counter()
        feat, tgt = learned.training_set(2_000_000, seed=0)
        stdz = learned.standardization(feat, tgt)
        params, losses = learned.train(feat, tgt, stdz, epochs=10, batch=16384, seed=0)
        del feat, tgt
        blk.mlp = asterx.make_mlp(params, stdz)
        blk._mlp_params = params  # keep the parameters alive
        torch.cuda.synchronize()
        learned_info = {"train_states": 2_000_000, "epochs": 10, "final_loss": losses[-1],
                        "setup_seconds": round(time.perf_counter() - t0, 1)}
    torch.cuda.synchronize()
    print("bench: %s n=%d recon=%s, block resident (%.2f GB device memory)" % (
        w.name, n, args.recon, torch.cuda.memory_allocated() / 1e9), file=sys.stderr, flush=True)

    ms = graph_steps(torch, blk, args.steps, args.warmup, graph=not args.no_graph)
    stages = blk.stages_per_step
    zone_stages = n ** 3 * stages * args.steps
    value = zone_stages / (ms * 1e-3)
    print("bench: %d steps in %.3f ms" % (args.steps, ms), file=sys.stderr, flush=True)

    # per-kernel durations, live, from HIP events bracketing each launch on its stream (one eager step)
    asterx.timing_reset()
    asterx.timing_enable(True)
    blk.step()
    torch.cuda.synchronize()
    kt = asterx.timing_read()
    asterx.timing_enable(False)
    # the library times the recovery with sources as "c2p" and the divergence kernel as "cell"
    names = {"c2p": "c2p_src", "cell": "divergence"}
    per_stage = {names.get(k, k): round(v[0] / stages, 4) for k, v in kt.items() if v[1] > 0}
    kr = kernel_rooflines(kt, stages, n, scheme, args.ct)
    roofline = headline_roofline(kr, kt, stages, scheme, n)
    stage_gbs = STAGE_BYTES_RK4 * value / 1e9
    hbm = {"bytes_per_zone_stage": STAGE_BYTES_RK4, "achieved": round(stage_gbs, 1), "peak": HBM_PEAK_GBS,
           "unit": "GB/s", "frac": round(stage_gbs / HBM_PEAK_GBS, 4)}
    stage_flops = STAGE_FLOPS.get(scheme) if n == 128 else None
    fp64 = {"unit": "TFLOP/s", "peak": FP64_VECTOR_PEAK_TFLOPS}
    for src, f in (("estimate", SURVEY_FLOPS_PER_ZONE_STAGE), ("oracle_count", stage_flops)):
        if f:
            fp64["flops_per_zone_stage_" + src] = f
            fp64["frac_" + src] = round(f * value / 1e12 / FP64_VECTOR_PEAK_TFLOPS, 4)
    out = {"metric": METRIC, "value": value, "unit": "zone-updates/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": ms / args.steps, "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "f64", "data": "synthetic",
           "config": {"workload": "curved%d-%s-rk4" % (n, scheme.replace("+", "-")), "n": n, "ng": w.layout.ng,
                      "recon": args.recon, "riemann": args.riemann, "ct": args.ct, "rk": 4,
                      "stages_per_step": stages, "cfl": 0.25, "gamma": 2.0, "speeds": "quartic",
                      "graph": not args.no_graph, "c2p_guess": "learned" if args.learned_c2p else "warm"},
           "roofline": roofline, "hbm_roofline_stage": hbm, "fp64_roofline_stage": fp64,
           "kernels": kr, "kernel_ms_per_stage": per_stage,
           "c2p_stats": [int(v) for v in blk.stats.cpu().tolist()]}
    if learned_info:
        out["learned_c2p"] = learned_info
    if args.ct == "fct" and not args.no_extras:
        out["tmunu_vertices"] = time_tmunu(asterx, torch, blk, n)
        out["inter_level_9_fields"] = time_inter_level(asterx, torch, n)
    if not args.no_extras and args.ct == "fct" and args.riemann == "hlle" and not args.learned_c2p:
        other = "wenoz" if args.recon != "wenoz" else "ppm"
        print("bench: %s on the same block" % other, file=sys.stderr, flush=True)
        out["same_block_" + other] = extra_scheme(torch, asterx, w, other, args.steps)
        print("bench: batched patches against the per-patch loop", file=sys.stderr, flush=True)
        out["batched_vs_loop"] = extra_batched(torch, asterx, W)
        print("bench: learned initial guess against the plain recovery", file=sys.stderr, flush=True)
        out["learned_vs_plain"] = extra_learned(torch, asterx, blk, args.steps)
        print("bench: adjoint gradient (forward with checkpoints, reverse pass)", file=sys.stderr, flush=True)
        out["adjoint_gradient"] = extra_adjoint(torch, W)
        print("bench: the paper's Setup A (magnetized TOV star, Cowling, 240^3)", file=sys.stderr, flush=True)
        out["paper_setup_a"] = extra_setup_a(torch, asterx, W, args.steps)
    if not args.no_cpu_baseline:
        print("bench: timing the CPU oracle (serial on a %d^3 sample, all cores on the full block)" % args.cpu_n,
              file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(args.recon, args.riemann, args.ct, args.cpu_n, w_full=w)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
