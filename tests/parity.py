"""Comparison helpers for GPU-vs-oracle parity tests."""
import numpy as np


def field_errors(gpu, cpu, owned_view=None):
    """Per-field max of |gpu - cpu| / max(|cpu|, s_f), s_f = max over the block of |cpu| for that field
    (cancellation-aware relative error)."""
    gpu = np.asarray(gpu)
    cpu = np.asarray(cpu)
    if owned_view is not None:
        gpu = owned_view(gpu)
        cpu = owned_view(cpu)
    out = []
    for f in range(cpu.shape[0]):
        c = cpu[f]
        g = gpu[f]
        sf = np.max(np.abs(c))
        den = np.maximum(np.abs(c), sf if sf > 0 else 1.0)
        out.append(float(np.max(np.abs(g - c) / den)))
    return np.array(out)


def assert_fields_close(gpu, cpu, tol, owned_view=None, names=None):
    e = field_errors(gpu, cpu, owned_view)
    bad = [(names[i] if names else i, e[i]) for i in range(len(e)) if not (e[i] <= tol)]
    assert not bad, "fields over tolerance %g: %s (all: %s)" % (tol, bad, e)
    return e
