#!/usr/bin/env python3
"""Benchmark of the FP64 GRMHD right-hand side on one MI355X.

Workload: the 128^3 periodic block in a static curved 3+1 metric (seeded low-k mode sums), Gamma = 2, PPM
reconstruction, HLLE, quartic characteristic speeds, Noble c2p, RK4 at CFL 0.25.  A step is one whole RK4
step (4 stages: c2p, primitive ghost fill, right-hand side, combine, state ghost fill), replayed from a
captured HIP graph, with all inputs resident in HBM.

Prints one JSON line: zone-updates/s per RK stage (interior cells x stages / wall time of the timed steps),
the roofline of the dominant kernel (per-kernel HIP events recorded live on the launch stream), the
whole-stage HBM roofline, and the serial CPU oracle timed on a bounded sample of the same workload.
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

# Algorithmic FP64 operations per face of the face kernel (reconstruction of 7 variables on both sides,
# 16-point face metric of 10 components, prim->cons, fluxes, quartic speeds, HLLE or LxF), counted by running
# the plain serial implementation on an operation-counting scalar (+, -, *, /, sqrt, pow = 1 each) over the
# 3 x 129^3 faces of the 128^3 block of this workload (same seed and recipe; limiter branches make the count
# data dependent).
FACE_FLOPS = {"ppm": 2603.1, "wenoz": 3955.0, "minmod": 2022.6, "mp5": 2480.3, "ppm+lxf": 2581.1,
              "ppm+hlle+uct": 2620.8}
# Algorithmic bytes per face: read 5 primitives + 2 centre fields + 10 face-metric components + 2 potential
# components, write 7 face fluxes (each value once, stencil reuse served on chip).
FACE_BYTES = 8.0 * (5 + 2 + 10 + 2 + 7)
# Whole-stage algorithmic HBM bytes per zone-stage, RK4 averaged over its four stages: reads of the stage
# state (9), metric and curvature (16), previous primitives (5), RK base state and accumulator (9 + 9 when
# used); writes of primitives (5), next state (9) and accumulator (9 when used).
STAGE_BYTES_RK4 = 514.0
# Whole-stage algorithmic FP64 operations per zone-stage at 128^3 (same counting scalar, over one
# right-hand side and one c2p of the 128^3 block of this workload; for PPM: centre field 41, faces of
# the three directions 7994, cell sources and divergence 5598, constrained transport and gauge 139, c2p
# 3265; the RK combine's 2 operations per field are not counted).
STAGE_FLOPS = {"ppm": 17036.9, "wenoz": 21188.6, "minmod": 15254.4, "mp5": 16659.9, "ppm+lxf": 16969.3,
               "ppm+hlle+uct": 19021.8}  # upwind CT: 129 x 133^2 faces per direction, edge field 1561


def library_source_sha():
    """First 16 hex digits of the sha256 of the HIP sources the library is built from."""
    import hashlib
    csrc = os.path.join(ROOT, "paper_2406_11669_amd", "csrc")
    h = hashlib.sha256()
    for name in ("asterx.hip", "grmhd_device.h"):
        with open(os.path.join(csrc, name), "rb") as f:
            h.update(f.read())
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


def cpu_baseline(recon, riemann, ct, n_cpu):
    """The serial oracle, as it stands, on an n_cpu^3 block of the same workload: one RK4 step."""
    from oracle import oracle as O
    from paper_2406_11669_amd import workloads as W
    O.build(force=False)
    w = W.curved_block(seed=0, n=n_cpu, recon=recon, nsteps=1, ng=4 if ct == "uct" else 3)
    w.params["riemann"] = riemann
    w.params["ct"] = ct
    L = w.layout
    cons = O.prim2con(L, w.params, w.metric, w.A, w.prim)
    O.fill_ghosts(L, cons, w.bc_cell)
    state = w.state(cons)
    prim = w.prim.copy()
    t0 = time.perf_counter()
    O.run(L, w.params, w.metric, w.curv, state, prim, w.dt, 1, 4, w.bc_cell, w.bc_A)
    dt = time.perf_counter() - t0
    zs = n_cpu ** 3 * 4
    return {"value": zs / dt, "unit": "zone-updates/s", "cores": 1, "kind": "oracle",
            "sample": "one RK4 step (4 stages) of the %d^3 block of the same workload recipe, serial FP64 oracle "
                      "(g++ -O2 -ffp-contract=off), %.1f s" % (n_cpu, dt)}


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

    step = blk.step
    graph = None
    if not args.no_graph:
        side = torch.cuda.Stream()
        side.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(side):
            blk.step()  # first step eagerly on the capture stream
        torch.cuda.current_stream().wait_stream(side)
        torch.cuda.synchronize()
        graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(graph):
            blk.step()
        step = graph.replay
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    t0.record()
    for _ in range(args.steps):
        step()
    t1.record()
    torch.cuda.synchronize()
    ms = t0.elapsed_time(t1)
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
    per_stage = {k: round(v[0] / stages, 4) for k, v in kt.items() if v[1] > 0}
    face_ms = sum(kt[k][0] for k in ("face_x", "face_y", "face_z"))
    face_launches = sum(kt[k][1] for k in ("face_x", "face_y", "face_z"))
    dominant = max(((k, v[0]) for k, v in kt.items()), key=lambda kv: kv[1])[0]
    faces_per_launch = (n + 1) ** 3 if args.ct == "fct" else (n + 1) * (n + 5) ** 2
    avg_face_s = face_ms * 1e-3 / face_launches
    face_flops = FACE_FLOPS.get(scheme)
    achieved = face_flops * faces_per_launch / avg_face_s / 1e12 if face_flops else None
    roofline = {"kernel": "face (x, y, z launches averaged)", "dominant_by_time": dominant,
                "bound": "alu", "achieved": None if achieved is None else round(achieved, 3),
                "peak": FP64_VECTOR_PEAK_TFLOPS, "unit": "TFLOP/s",
                "frac": None if achieved is None else round(achieved / FP64_VECTOR_PEAK_TFLOPS, 4),
                "traffic": measured_face_traffic(scheme, n),
                "avg_launch_ms": round(avg_face_s * 1e3, 4),
                "flops_per_face": face_flops, "faces_per_launch": faces_per_launch,
                "algorithmic_GBs": round(FACE_BYTES * faces_per_launch / avg_face_s / 1e9, 1)}
    stage_gbs = STAGE_BYTES_RK4 * value / 1e9
    hbm = {"bytes_per_zone_stage": STAGE_BYTES_RK4, "achieved": round(stage_gbs, 1), "peak": HBM_PEAK_GBS,
           "unit": "GB/s", "frac": round(stage_gbs / HBM_PEAK_GBS, 4)}
    stage_flops = STAGE_FLOPS.get(scheme) if n == 128 else None
    stage_tf = stage_flops * value / 1e12 if stage_flops else None
    fp64 = {"flops_per_zone_stage": stage_flops,
            "achieved": None if stage_tf is None else round(stage_tf, 3), "peak": FP64_VECTOR_PEAK_TFLOPS,
            "unit": "TFLOP/s", "frac": None if stage_tf is None else round(stage_tf / FP64_VECTOR_PEAK_TFLOPS, 4)}
    out = {"metric": METRIC, "value": value, "unit": "zone-updates/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": ms / args.steps, "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "f64", "data": "synthetic",
           "config": {"workload": "curved%d-%s-rk4" % (n, scheme.replace("+", "-")), "n": n, "ng": w.layout.ng,
                      "recon": args.recon, "riemann": args.riemann, "ct": args.ct, "rk": 4, "stages_per_step": stages, "cfl": 0.25, "gamma": 2.0,
                      "speeds": "quartic", "graph": graph is not None,
                      "c2p_guess": "learned" if args.learned_c2p else "warm"},
           "roofline": roofline, "hbm_roofline_stage": hbm, "fp64_roofline_stage": fp64,
           "kernel_ms_per_stage": per_stage,
           "c2p_stats": [int(v) for v in blk.stats.cpu().tolist()]}
    if learned_info:
        out["learned_c2p"] = learned_info
    if args.ct == "fct":
        out["tmunu_vertices"] = time_tmunu(asterx, torch, blk, n)
        out["inter_level_9_fields"] = time_inter_level(asterx, torch, n)
    if not args.no_cpu_baseline:
        print("bench: timing the CPU oracle on a %d^3 sample" % args.cpu_n, file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(args.recon, args.riemann, args.ct, args.cpu_n)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
