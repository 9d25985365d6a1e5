"""The all-core build of the oracle (the same source with -fopenmp over k-planes) gives bitwise the same steps as
the serial build: cells are independent and the reductions are integer sums and maxima."""
import numpy as np

from paper_2406_11669_amd import workloads as W


def test_openmp_build_bitwise_equals_serial(orc):
    lo, nthreads = orc.lib_omp(4)
    assert nthreads == 4
    w = W.curved_block(seed=3, n=(12, 10, 9), recon="wenoz", nsteps=2)
    L = w.layout
    res = []
    for lib_ in (None, lo):
        cons = orc.prim2con(L, w.params, w.metric, w.A, w.prim)
        orc.fill_ghosts(L, cons, w.bc_cell)
        state = w.state(cons)
        prim = w.prim.copy()
        flags, stats, red = orc.run(L, w.params, w.metric, w.curv, state, prim, w.dt, 2, 4, w.bc_cell, w.bc_A,
                                    lib_=lib_)
        res.append((state, prim, flags, stats, red))
    for a, b in zip(res[0], res[1]):
        assert np.array_equal(a, b)
