"""A network on which bfloat16 operands and float32 accumulation are exact (test fixture).

Weights, biases, inputs and targets are small dyadic numbers chosen so that every value the rounded network
forms -- standardised inputs, layer inputs and activations, output errors and backward cotangents -- has at
most 8 significant bits, and every sum (over 8 or 64 inputs, and over the 1024 samples of a gradient) fits in
float32's 24: the rounded network then equals the plain one bit for bit.  Layout as in oracle/mlp_ref.py
(8 -> 64 -> 64 -> 2, ReLU).
  W1 in {-1/4, 0, 1/4}, b1 in quarter steps of [-1, 1], inputs integers in [-2, 2]: |h1| <= 5 in quarters;
  W2 two entries of +-1/4 per row and per column (i, i) and (i, i+1 mod 64), b2 quarters in [-1, 1]:
    |h2| <= 3.5 in sixteenths, and the backward sums W2^T d2 have two terms;
  W3 four entries of +-1/2 per row in distinct columns, b3 in 1/32 steps of [-1, 1];
  targets y - k/32 with |k| <= 63, n = 1024 samples, so d3 = (y - t)/n = k 2^-15.
Standardisation is the identity (shift 0, scale 1)."""
import numpy as np

N_SAMPLES = 1024


def network(seed):
    rng = np.random.default_rng(seed)
    W1 = rng.integers(-1, 2, size=(64, 8)) * 0.25
    b1 = rng.integers(-4, 5, size=64) * 0.25
    W2 = np.zeros((64, 64))
    for i in range(64):
        W2[i, i] = rng.choice([-0.25, 0.25])
        W2[i, (i + 1) % 64] = rng.choice([-0.25, 0.25])
    b2 = rng.integers(-4, 5, size=64) * 0.25
    W3 = np.zeros((2, 64))
    cols = rng.permutation(64)[:8]
    W3[0, cols[:4]] = rng.choice([-0.5, 0.5], size=4)
    W3[1, cols[4:]] = rng.choice([-0.5, 0.5], size=4)
    b3 = rng.integers(-32, 33, size=2) / 32.0
    params = np.concatenate([W1.ravel(), b1, W2.ravel(), b2, W3.ravel(), b3]).astype(np.float32)
    stdz = {"in_shift": np.zeros(8, np.float32), "in_scale": np.ones(8, np.float32),
            "out_shift": np.zeros(2, np.float32), "out_scale": np.ones(2, np.float32)}
    feat = rng.integers(-2, 3, size=(8, N_SAMPLES)).astype(np.float32)
    offsets = rng.integers(-63, 64, size=(2, N_SAMPLES)) / 32.0
    return params, stdz, feat, offsets
