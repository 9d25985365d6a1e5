"""Pins of the CPU reference of the learned c2p guess's network: bfloat16 rounding against exactly known
values, the backward pass against central differences of the forward pass (float64, no rounding), and the
sampler of training states against the oracle's own fluid quantities (W and the magnetisation)."""
import numpy as np
import pytest

from oracle import mlp_ref as M
from paper_2406_11669_amd import workloads as W


def test_bf16_rounding_known_values():
    # bfloat16 keeps 7 mantissa bits: spacing 2^-7 on [1, 2)
    x = np.array([1.0, 1.0 + 2.0 ** -8, 1.0 + 3 * 2.0 ** -8, 1.0 + 2.0 ** -7 + 2.0 ** -9, -2.5, 1.0 + 2.0 ** -8 + 2.0 ** -20],
                 dtype=np.float32)
    # ties go to the even mantissa: 1 + 2^-8 -> 1, 1 + 3 * 2^-8 -> 1 + 2^-6; below/above a tie round to nearest
    expect = np.array([1.0, 1.0, 1.0 + 2.0 ** -6, 1.0 + 2.0 ** -7, -2.5, 1.0 + 2.0 ** -7], dtype=np.float32)
    assert np.array_equal(M.bf16(x), expect)


def _stdz():
    return dict(in_shift=np.linspace(-1, 1, 8), in_scale=np.linspace(0.5, 2, 8), out_shift=np.array([0.3, 1.2]),
                out_scale=np.array([0.7, 1.9]))


def test_precise_gradient_matches_central_differences():
    rng = np.random.default_rng(0)
    p = M.init_params(1).astype(np.float64)
    p[M.NH * M.NI:M.NH * M.NI + M.NH] = rng.normal(size=M.NH) * 0.1
    feat = rng.normal(size=(8, 37))
    tgt = rng.normal(size=(2, 37))
    loss, g = M.loss_grad(p, feat, tgt, _stdz(), precise=True)
    idx = rng.choice(M.NP, 60, replace=False)
    h = 1e-6
    for i in idx:
        e = np.zeros(M.NP)
        e[i] = h
        fd = (M.loss_grad(p + e, feat, tgt, _stdz(), precise=True)[0] -
              M.loss_grad(p - e, feat, tgt, _stdz(), precise=True)[0]) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(1e-3, np.max(np.abs(g))), (i, fd, g[i])


def test_rounded_forward_close_to_precise():
    rng = np.random.default_rng(1)
    p = M.init_params(2)
    feat = rng.normal(size=(8, 50))
    a, _ = M.forward(p, feat, _stdz())
    b, _ = M.forward(p.astype(np.float64), feat, _stdz(), precise=True)
    assert np.max(np.abs(a - b)) <= 0.05 * np.max(np.abs(b))  # bfloat16 operands: a few parts in 1e3 per layer


def test_adam_first_step_is_signed_lr():
    g = np.array([0.3, -2.0, 1e-3], np.float32)
    p0 = np.zeros(3, np.float32)
    p, m, v = M.adam(p0, g, np.zeros(3, np.float32), np.zeros(3, np.float32), 0.01, 0.9, 0.999, 1e-12, 1)
    assert np.allclose(p, -0.01 * np.sign(g), rtol=1e-5)


def test_c2p_state_sampler_hits_W_and_sigma(orc):
    s = W.c2p_states(3, 200)
    rng = np.random.default_rng([3, 8191])
    rng.uniform(-8.0, 0.0, 200)
    Wt = rng.uniform(1.0, 10.0, 200)
    sig = np.exp(rng.uniform(np.log(1e-3), np.log(10.0), 200))
    for i in range(0, 200, 7):
        f = orc.pt_fluid(s["metric"][:, i], s["prim"][:, i], s["Bt"][:, i], s["gam"][i])
        assert abs(f["W"] - Wt[i]) <= 1e-12 * Wt[i]
        assert abs(f["bsq"] / s["prim"][0, i] - sig[i]) <= 1e-10 * sig[i]


def test_rounded_network_exact_on_dyadic_network():
    """On a network whose every rounded value is exactly representable (tests/mlp_exact.py), the bfloat16 forward
    and gradient equal the plain float64 network's bit for bit -- a pin of the rounded mode that does not restate
    where it rounds.  A transposed hidden matrix or dropped bias changes the result."""
    from tests import mlp_exact as X
    p, st, feat, off = X.network(3)
    out_p, _ = M.forward(p, feat, st, precise=True)
    out_b, _ = M.forward(p, feat, st)
    assert np.array_equal(out_b.astype(np.float64), out_p)
    tgt = (out_p - off).astype(np.float32)
    assert np.array_equal(tgt.astype(np.float64), out_p - off)
    lp, gp = M.loss_grad(p, feat, tgt, st, precise=True)
    lb, gb = M.loss_grad(p, feat, tgt, st)
    assert lb == lp and np.array_equal(np.asarray(gb, np.float64), np.asarray(gp, np.float64))
    assert np.count_nonzero(gp) > 200
    W1, b1, W2, b2, W3, b3 = M.unpack(p)
    for q in (M.pack(W1, b1, W2.T.copy(), b2, W3, b3), M.pack(W1, b1, W2, 0.0 * b2 + 0.25, W3, b3)):
        assert not np.array_equal(M.forward(q.astype(np.float32), feat, st)[0].astype(np.float64), out_p)
