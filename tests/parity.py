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


def cell_relative_errors(gpu, cpu, owned_view=None, floor=1e-6):
    """Per field: the largest per-cell relative error |gpu - cpu| / |cpu| over the cells with |cpu| >= floor * s_f
    (s_f = max |cpu| of the field), and the fraction of cells that bound excludes.  Unlike field_errors it sees
    small-magnitude cells, so it is meaningful for fields bounded away from zero (density, energy); for fields that
    cross zero it reports cancellation, not error."""
    gpu = np.asarray(gpu)
    cpu = np.asarray(cpu)
    if owned_view is not None:
        gpu = owned_view(gpu)
        cpu = owned_view(cpu)
    out = []
    for f in range(cpu.shape[0]):
        c = cpu[f]
        sf = np.max(np.abs(c))
        keep = np.abs(c) >= floor * sf if sf > 0 else np.zeros(c.shape, bool)
        rel = np.abs(gpu[f][keep] - c[keep]) / np.abs(c[keep]) if keep.any() else np.zeros(1)
        out.append((float(np.max(rel)), float(1.0 - keep.mean())))
    return out
