"""TEST INFRASTRUCTURE -- plain CPU reference of the learned c2p guess's network (numpy).

Only tests/, the entry-point smoke check and the benchmark's CPU baseline may import this module;
the library never does.

The network: 8 -> 64 -> 64 -> 2, ReLU hidden activations, parameters packed as W1[64][8], b1[64],
W2[64][64], b2[64], W3[2][64], b3[2] (4866 floats).  The library's arithmetic is restated here
step by step: inputs standardised in float32, then every matrix product takes bfloat16 operands
(round to nearest even) -- weights, layer inputs, activations and the backward cotangents -- with
the products accumulated exactly (float64 here; the matrix cores accumulate in float32, so the two
differ by float32 rounding), biases and activations in float32.

precise=True drops every bfloat16 rounding and works in float64: the plain network, whose gradient
the tests pin against central differences.
"""
import numpy as np

NI, NH, NO = 8, 64, 2
NP = NH * NI + NH + NH * NH + NH + NO * NH + NO


def unpack(p):
    p = np.asarray(p)
    o = 0
    W1 = p[o:o + NH * NI].reshape(NH, NI); o += NH * NI
    b1 = p[o:o + NH]; o += NH
    W2 = p[o:o + NH * NH].reshape(NH, NH); o += NH * NH
    b2 = p[o:o + NH]; o += NH
    W3 = p[o:o + NO * NH].reshape(NO, NH); o += NO * NH
    b3 = p[o:o + NO]
    return W1, b1, W2, b2, W3, b3


def pack(W1, b1, W2, b2, W3, b3):
    return np.concatenate([W1.ravel(), b1, W2.ravel(), b2, W3.ravel(), b3])


def bf16(x):
    """Round float32 values to bfloat16 (nearest, ties to even); returned as float32."""
    u = np.ascontiguousarray(x, dtype=np.float32).view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32)


def act(x, precise=False):
    """ReLU."""
    if precise:
        return np.maximum(x, 0.0)
    return np.maximum(np.asarray(x, dtype=np.float32), np.float32(0.0))


def dact(t):
    """ReLU' from the activation's value (1 where it is positive)."""
    return (t > 0).astype(t.dtype)


def init_params(seed):
    """Seeded initial parameters (uniform, fan-in scaled; zero biases)."""
    rng = np.random.default_rng([int(seed), 65521])
    W1 = rng.uniform(-1, 1, (NH, NI)) / np.sqrt(NI)
    W2 = rng.uniform(-1, 1, (NH, NH)) / np.sqrt(NH)
    W3 = rng.uniform(-1, 1, (NO, NH)) / np.sqrt(NH)
    return pack(W1, np.zeros(NH), W2, np.zeros(NH), W3, np.zeros(NO)).astype(np.float32)


def _r(x, precise):
    return np.asarray(x, dtype=np.float64) if precise else bf16(x).astype(np.float64)


def forward(params, feat, stdz, precise=False):
    """Outputs (2, n) de-standardised, and the intermediate values for backward."""
    W1, b1, W2, b2, W3, b3 = unpack(params)
    dt = np.float64 if precise else np.float32
    ish, isc, osh, osc = (np.asarray(stdz[k], dtype=dt) for k in ("in_shift", "in_scale", "out_shift", "out_scale"))
    X = ((np.asarray(feat, dtype=dt) - ish[:, None]) * isc[:, None]).astype(dt)
    x1 = _r(X, precise)
    h1 = (_r(W1, precise) @ x1 + np.asarray(b1, np.float64)[:, None]).astype(dt)
    t1 = act(h1, precise)
    x2 = _r(t1, precise)
    h2 = (_r(W2, precise) @ x2 + np.asarray(b2, np.float64)[:, None]).astype(dt)
    t2 = act(h2, precise)
    x3 = _r(t2, precise)
    y = (_r(W3, precise) @ x3 + np.asarray(b3, np.float64)[:, None]).astype(dt)
    out = osh[:, None] + y * osc[:, None]
    return out, dict(x1=x1, t1=t1, x2=x2, t2=t2, x3=x3, y=y, osh=osh, osc=osc, dt=dt)


def loss_grad(params, feat, target, stdz, precise=False):
    """(loss, gradient (NP,)) of (1/n) sum |y - t|^2 / 2 with t = (target - out_shift) / out_scale."""
    W1, b1, W2, b2, W3, b3 = unpack(params)
    _, c = forward(params, feat, stdz, precise)
    dt = c["dt"]
    n = feat.shape[1]
    t = ((np.asarray(target, dtype=dt) - c["osh"][:, None]) / c["osc"][:, None]).astype(dt)
    e = (c["y"] - t).astype(dt)
    loss = float(np.sum(0.5 * e.astype(np.float64) ** 2) / n)
    d3 = (e / dt(n)).astype(dt)
    gW3 = _r(d3, precise) @ c["x3"].T
    gb3 = d3.astype(np.float64).sum(1)
    g2 = (_r(W3, precise).T @ _r(d3, precise)).astype(dt)
    d2 = (g2 * dact(c["t2"])).astype(dt)
    gW2 = _r(d2, precise) @ c["x2"].T
    gb2 = d2.astype(np.float64).sum(1)
    g1 = (_r(W2, precise).T @ _r(d2, precise)).astype(dt)
    d1 = (g1 * dact(c["t1"])).astype(dt)
    gW1 = _r(d1, precise) @ c["x1"].T
    gb1 = d1.astype(np.float64).sum(1)
    return loss, pack(gW1, gb1, gW2, gb2, gW3, gb3)


def adam(params, grad, m, v, lr, b1, b2, eps, step):
    """One bias-corrected Adam step in float32; returns (params, m, v)."""
    f = np.float32
    g = np.asarray(grad, f)
    m = (f(b1) * m + (f(1) - f(b1)) * g).astype(f)
    v = (f(b2) * v + (f(1) - f(b2)) * g * g).astype(f)
    c1 = f(1) - f(b1) ** f(step)
    c2 = f(1) - f(b2) ** f(step)
    p = (params - f(lr) * (m / c1) / (np.sqrt(v / c2) + f(eps))).astype(f)
    return p, m, v
