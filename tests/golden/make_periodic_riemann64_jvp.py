"""Writes periodic_riemann64_jvp.json: the CPU oracle's loss and its forward-mode (dual-number) directional
derivatives for the differentiation workload: the periodic Riemann box, 64^3, PPM, HLLE, RK2 at CFL 0.25,
20 steps, Gamma = 5/3, loss (sum over owned cells of rho^2 dV)^(1/2) at the final time, directions from
workloads.gradient_direction (seeded unit vectors in (initial velocity field, Gamma)).

Calls only the oracle and the seeded input generators.  Run: python tests/golden/make_periodic_riemann64_jvp.py
(about 2.5 minutes of one CPU core per direction)."""
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import oracle as orc  # noqa: E402
from paper_2406_11669_amd import workloads as W  # noqa: E402

CASES = [  # (v_amp, direction seed, with Gamma)
    (0.1, 0, True), (0.1, 1, True), (0.1, 2, False), (0.1, None, True),
    (0.0, 0, True), (0.0, None, True),
]


def main():
    out = {"workload": "periodic_riemann_box(seed=0, n=64, nsteps=20, v_amp=...)", "nsteps": 20, "cases": []}
    for v_amp, seed, with_g in CASES:
        w = W.periodic_riemann_box(seed=0, n=64, nsteps=20, v_amp=v_amp)
        L = w.layout
        if seed is None:
            d, dg = L.zeros(5), 1.0
        else:
            d, dg = W.gradient_direction(L, seed, with_g)
        t0 = time.time()
        loss, jvp, stats = orc.loss_jvp(L, w.params, w.metric, w.curv, w.prim, w.A, w.psi, w.dt, 20, w.rk,
                                        w.bc_cell, w.bc_A, dprim0=d, dgamma=dg, A_shift=w.A_shift)
        case = {"v_amp": v_amp, "dir_seed": seed, "with_gamma": with_g, "loss": loss, "jvp": jvp,
                "c2p_stats": [int(v) for v in stats], "seconds": round(time.time() - t0, 1)}
        print(json.dumps(case), flush=True)
        out["cases"].append(case)
    with open(os.path.join(HERE, "periodic_riemann64_jvp.json"), "w") as f:
        json.dump(out, f, indent=1)


if __name__ == "__main__":
    main()
