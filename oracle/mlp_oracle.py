"""FP64 reference of the learned-majorant network and its training step.

TEST INFRASTRUCTURE.  Only tests, the smoke check and the benchmark's CPU
baseline may import this module; the HIP path shares no code with it.

Network: 6 -> 64 -> 64 -> 1 with ReLU after both hidden layers; parameters
in the flat order W1[64][6], b1[64], W2[64][64], b2[64], w3[64], b3 (4673
values).  Output y is a prediction of log2 of the largest relative speed in
a cell.

Loss: the expectile (asymmetric least squares) loss of Newey & Powell
(Econometrica 1987), L = mean_s |tau - 1[r_s < 0]| r_s^2 with r = label - y;
tau > 1/2 penalises under-prediction more, so the fit sits above the
conditional mean, which is what a majorant wants.  Rows whose label is not
finite are ignored.

Optimiser: Adam (Kingma & Ba, ICLR 2015) with bias-corrected moments.
"""
import numpy as np

N_IN, N_H = 6, 64
NPARAM = N_H * N_IN + N_H + N_H * N_H + N_H + N_H + 1  # 4673


def unpack(p):
    p = np.asarray(p, dtype=np.float64)
    o = 0
    W1 = p[o:o + N_H * N_IN].reshape(N_H, N_IN); o += N_H * N_IN
    b1 = p[o:o + N_H]; o += N_H
    W2 = p[o:o + N_H * N_H].reshape(N_H, N_H); o += N_H * N_H
    b2 = p[o:o + N_H]; o += N_H
    w3 = p[o:o + N_H]; o += N_H
    b3 = p[o]
    return W1, b1, W2, b2, w3, b3


def pack(W1, b1, W2, b2, w3, b3):
    return np.concatenate([W1.ravel(), b1, W2.ravel(), b2, w3, [b3]]).astype(np.float64)


def forward(p, x):
    """y for inputs x [n, 6] (FP64)."""
    W1, b1, W2, b2, w3, b3 = unpack(p)
    x = np.asarray(x, dtype=np.float64)
    z1 = x @ W1.T + b1
    h1 = np.maximum(z1, 0.0)
    z2 = h1 @ W2.T + b2
    h2 = np.maximum(z2, 0.0)
    return h2 @ w3 + b3


def loss_grad(p, x, label, tau):
    """(loss, gradient [4673]) of the mean expectile loss (FP64, analytic)."""
    W1, b1, W2, b2, w3, b3 = unpack(p)
    x = np.asarray(x, dtype=np.float64)
    label = np.asarray(label, dtype=np.float64)
    ok = np.isfinite(label)
    x, label = x[ok], label[ok]
    n = len(label)
    if n == 0:
        return 0.0, np.zeros(NPARAM)
    z1 = x @ W1.T + b1
    h1 = np.maximum(z1, 0.0)
    z2 = h1 @ W2.T + b2
    h2 = np.maximum(z2, 0.0)
    y = h2 @ w3 + b3
    r = label - y
    wgt = np.where(r < 0.0, 1.0 - tau, tau)
    loss = np.mean(wgt * r * r)
    dy = -2.0 * wgt * r / n            # dL/dy per sample
    dw3 = h2.T @ dy
    db3 = dy.sum()
    d2 = np.outer(dy, w3) * (z2 > 0.0)  # dL/dz2
    dW2 = d2.T @ h1
    db2 = d2.sum(0)
    d1 = (d2 @ W2) * (z1 > 0.0)         # dL/dz1
    dW1 = d1.T @ x
    db1 = d1.sum(0)
    return loss, pack(dW1, db1, dW2, db2, dw3, db3)


def adam(p, g, m, v, t, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update; returns (p, m, v) as new arrays (t is 1-based)."""
    m = b1 * m + (1.0 - b1) * g
    v = b2 * v + (1.0 - b2) * g * g
    mh = m / (1.0 - b1 ** t)
    vh = v / (1.0 - b2 ** t)
    return p - lr * mh / (np.sqrt(vh) + eps), m, v


def init_params(seed=0):
    """He-style initialisation (weights ~ N(0, 2/fan_in)), zero biases."""
    rng = np.random.default_rng(seed)
    W1 = rng.standard_normal((N_H, N_IN)) * np.sqrt(2.0 / N_IN)
    W2 = rng.standard_normal((N_H, N_H)) * np.sqrt(2.0 / N_H)
    w3 = rng.standard_normal(N_H) * np.sqrt(2.0 / N_H)
    return pack(W1, np.zeros(N_H), W2, np.zeros(N_H), w3, 0.0)


def to_bf16(p):
    """Round FP32 values to bfloat16 (round to nearest, ties to even); uint16 bits."""
    f = np.asarray(p, dtype=np.float32).view(np.uint32).astype(np.uint64)
    rounding = 0x7FFF + ((f >> 16) & 1)
    return ((f + rounding) >> 16).astype(np.uint16)


def from_bf16(bits):
    return (np.asarray(bits, dtype=np.uint16).astype(np.uint32) << 16).view(np.float32)
