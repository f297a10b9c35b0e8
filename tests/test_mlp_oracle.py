"""Pins of the FP64 network reference (oracle/mlp_oracle.py) and of the
oracle's FP32 forward pass: finite differences, closed forms of the
expectile loss and of Adam's first step, and library bfloat16 rounding."""
import math

import numpy as np
import pytest

import oracle
from oracle import mlp_oracle as M


def _data(n=64, seed=0):
    rng = np.random.default_rng(seed)
    x = rng.standard_normal((n, 6))
    label = rng.standard_normal(n) + 2.0
    return x, label


def test_gradient_matches_central_differences():
    p = M.init_params(3)
    x, label = _data(48, 1)
    loss, g = M.loss_grad(p, x, label, 0.95)
    rng = np.random.default_rng(2)
    idx = rng.choice(M.NPARAM, 200, replace=False)
    h = 1e-6
    for k in idx:
        e = np.zeros(M.NPARAM)
        e[k] = h
        lp, _ = M.loss_grad(p + e, x, label, 0.95)
        lm, _ = M.loss_grad(p - e, x, label, 0.95)
        fd = (lp - lm) / (2 * h)
        assert abs(fd - g[k]) <= 1e-6 * max(1.0, abs(g[k])) + 1e-8, (k, fd, g[k])


def test_expectile_stationary_point_of_a_constant_model():
    # with zero hidden weights the network is the constant b3; the gradient in
    # b3 vanishes exactly at the tau-expectile of the labels, found here by
    # bisection of its defining equation sum |tau - 1[l < e]| (l - e) = 0
    x, label = _data(500, 4)
    tau = 0.9
    def g_of(e):
        r = label - e
        return np.sum(np.where(r < 0, 1 - tau, tau) * r)
    lo, hi = label.min(), label.max()
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        if g_of(mid) > 0:
            lo = mid
        else:
            hi = mid
    p = np.zeros(M.NPARAM)
    p[-1] = 0.5 * (lo + hi)
    _, g = M.loss_grad(p, x, label, tau)
    assert abs(g[-1]) < 1e-10
    # tau = 1/2 is half the squared error: d/db3 = -mean(label - b3)
    p[-1] = 0.3
    _, g = M.loss_grad(p, x, label, 0.5)
    assert abs(g[-1] + np.mean(label - 0.3)) < 1e-12


def test_nonfinite_labels_are_ignored():
    p = M.init_params(1)
    x, label = _data(40, 5)
    l2 = label.copy()
    l2[::3] = -np.inf
    keep = np.isfinite(l2)
    a = M.loss_grad(p, x, l2, 0.95)
    b = M.loss_grad(p, x[keep], label[keep], 0.95)
    assert a[0] == b[0] and np.array_equal(a[1], b[1])


def test_adam_first_step_closed_form():
    rng = np.random.default_rng(0)
    p = rng.standard_normal(50)
    g = rng.standard_normal(50)
    p1, m, v = M.adam(p, g, np.zeros(50), np.zeros(50), 1, lr=1e-3)
    # bias-corrected first step is lr * g / (|g| + eps)
    assert np.allclose(p1, p - 1e-3 * g / (np.abs(g) + 1e-8), rtol=0, atol=1e-15)


def test_bf16_rounding_matches_torch():
    import torch
    rng = np.random.default_rng(3)
    v = np.concatenate([rng.standard_normal(5000).astype(np.float32) * 10,
                        np.array([1.0, 1 + 2 ** -8, 1 + 3 * 2 ** -9, -2.5, 0.0], dtype=np.float32)])
    ref = torch.from_numpy(v).to(torch.bfloat16).view(torch.int16).numpy().view(np.uint16)
    assert np.array_equal(M.to_bf16(v), ref)
    assert np.array_equal(M.from_bf16(M.to_bf16(v)), torch.from_numpy(v).to(torch.bfloat16).float().numpy())


def test_oracle_fp32_forward_agrees_with_fp64_reference():
    p = M.init_params(7)
    pf = p.astype(np.float32)
    x, _ = _data(100, 8)
    xf = x.astype(np.float32)
    y64 = M.forward(pf.astype(np.float64), xf.astype(np.float64))
    y32 = np.array([oracle.mlp_forward_f32(pf, xf[s]) for s in range(len(xf))])
    assert np.abs(y32 - y64).max() <= 2e-5 * max(1.0, np.abs(y64).max())
