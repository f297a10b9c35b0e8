"""Pins of the oracle's importance-weight re-estimation (weighted runs).

The re-estimation replaces a cell's weight deviations W - 1 by their
least-squares projection onto the span of the 13 velocity functions the cell
samples (1, c, c_d c_e, c_d |c|^2).  Checked against facts that do not come
from the oracle: numpy's SVD least-squares solution written in another basis
of the same span, exact invariants (every sampled weighted moment is kept,
unit weights stay exactly 1, projections are idempotent and reproduce a
function of the span), and run-level statistics (weights stay finite where
they diverge without it; the weighted and plain estimators agree; the
weighted one is less noisy near equilibrium).  CPU only."""
import math
from multiprocessing import Pool

import numpy as np
import pytest

import oracle
from paper_2301_05985_amd import workloads as W


def sampled_functions(c):
    """The 13 functions whose sums a cell samples, of the raw velocity:
    1, c_x, c_y, c_z, c_x^2, c_y^2, c_z^2, c_x c_y, c_x c_z, c_y c_z,
    c_x |c|^2, c_y |c|^2, c_z |c|^2 (columns)."""
    x, y, z = c
    s = x * x + y * y + z * z
    return np.stack([np.ones_like(x), x, y, z, x * x, y * y, z * z, x * y, x * z, y * z,
                     x * s, y * s, z * s], axis=1)


def _cell(rng, n, spread=0.3):
    c = rng.standard_normal((3, n)) * rng.uniform(0.7, 1.5) + rng.standard_normal((3, 1)) * 0.3
    w = 1.0 + spread * rng.standard_normal(n) * (1 + 0.3 * (c ** 2).sum(0))
    return c, w


@pytest.mark.parametrize("T0", [1.0, 1.5, 40.0])
def test_reestimation_is_the_least_squares_projection(T0):
    # numpy's SVD least squares in the raw-velocity basis of the same span
    rng = np.random.default_rng(31)
    for _ in range(60):
        n = int(rng.integers(26, 400))
        c, w = _cell(rng, n)
        c = c * math.sqrt(T0)
        w2, ok = oracle.vr_reconstruct(*c, w, T0)
        assert ok
        Phi = sampled_functions(c)
        a, *_ = np.linalg.lstsq(Phi, w - 1.0, rcond=None)
        ref = 1.0 + Phi @ a
        assert np.abs(w2 - ref).max() <= 1e-9 * (1 + np.abs(w - 1).max())


def test_reestimation_keeps_every_sampled_weighted_moment():
    rng = np.random.default_rng(32)
    for _ in range(60):
        n = int(rng.integers(26, 300))
        c, w = _cell(rng, n, spread=1.0)
        w2, ok = oracle.vr_reconstruct(*c, w, 1.0)
        assert ok
        Q = sampled_functions(c)
        before, after = (1 - w) @ Q, (1 - w2) @ Q
        scale = np.abs(1 - w) @ np.abs(Q)
        assert (np.abs(after - before) <= 1e-11 * scale).all()
        # and it does change the weights (a smoothing, not the identity)
        assert np.abs(w2 - w).max() > 1e-3


@pytest.mark.parametrize("dtype", [np.float64, np.float32])
def test_reestimation_fixed_points(dtype):
    rng = np.random.default_rng(33)
    for _ in range(40):
        n = int(rng.integers(26, 300))
        c, _ = _cell(rng, n)
        # unit weights stay exactly 1 (the right-hand side is exactly zero)
        w2, ok = oracle.vr_reconstruct(*c, np.ones(n), 1.0, dtype=dtype)
        assert ok and (w2 == 1.0).all()
        # a deviation that already lies in the span is reproduced
        cw = c.astype(dtype).astype(np.float64)
        coef = rng.standard_normal(13) * 0.05
        w = (1.0 + sampled_functions(cw) @ coef).astype(dtype)
        w2, _ = oracle.vr_reconstruct(*cw, w, 1.0, dtype=dtype)
        tol = 1e-12 if dtype == np.float64 else 4e-7
        assert np.abs(w2.astype(np.float64) - w).max() <= tol * (1 + np.abs(w).max())
    # idempotent
    c, w = _cell(rng, 150)
    w1, _ = oracle.vr_reconstruct(*c, w, 1.0)
    w2, _ = oracle.vr_reconstruct(*c, w1, 1.0)
    assert np.abs(w2 - w1).max() <= 1e-12 * (1 + np.abs(w1).max())


def test_reestimation_leaves_small_or_degenerate_cells_alone():
    rng = np.random.default_rng(34)
    c, w = _cell(rng, 25)
    w2, ok = oracle.vr_reconstruct(*c, w, 1.0)
    assert not ok and np.array_equal(w2, w)
    # all particles with one velocity: the functions are linearly dependent
    c = np.repeat(rng.standard_normal((3, 1)), 60, axis=1)
    w = 1 + 0.1 * rng.standard_normal(60)
    w2, ok = oracle.vr_reconstruct(*c, w, 1.0)
    assert not ok and np.array_equal(w2, w)


def test_reestimation_keeps_the_cavity_weights_finite():
    # the lid-driven cavity at the full-size benchmark's resolution per cell
    # (16 x 16 cells of 100, mean free path 2.56 cells, about 0.13
    # collisions per particle and step): without re-estimation the weighted
    # sums turn non-finite within 100 steps; with it (every step) the weights
    # stay within a few percent of 1 for 400 steps
    out = {}
    for K in (0, 1):
        p, parts = W.cavity(nx=16, ny=16, per_cell=100, Kn=0.16, real="f32")
        p["vr_reconstruct"] = K
        o = oracle.Oracle(p, parts, np.float32)
        o.run(100)
        n100 = int(o.diag.vr_nonfinite)
        if K:
            o.run(300)
        w = o.w.astype(np.float64)
        out[K] = (n100, int(o.diag.vr_nonfinite), np.sqrt(np.mean((w - 1) ** 2)), np.abs(w - 1).max())
    assert out[0][0] > 0, out
    assert out[1][1] == 0 and out[1][2] < 0.01 and out[1][3] < 0.5, out


def _fourier_member(args):
    K, seed = args
    nc, steps = 16, 2400
    p, parts = W.fourier(n_cells=nc, per_cell=150, Kn=0.1, T_left=1.45, T_right=1.55, T0=1.5,
                         dt=1e-3, real="f64", seed=seed, init_seed=seed)
    p["vr_reconstruct"] = K
    o = oracle.Oracle(p, parts)
    o.run(steps // 4)
    o.reset_samples()
    o.run(steps - steps // 4)
    ns = steps - steps // 4
    V = 1.0 / nc
    pl = oracle.estimators(o.sums, ns, 1.0, V)
    vr = oracle.estimators(o.sums, ns, 1.0, V, vr=True, vr_n0=p["vr_n0"], vr_T0=1.5)
    return (int(o.diag.vr_nonfinite), pl["T"], vr["T"], pl["q"][:, 0], vr["q"][:, 0])


def test_reestimated_weights_give_unbiased_lower_variance_estimates():
    # Fourier flow near equilibrium (walls at 1.45 and 1.55, reference 1.5),
    # 8 independent members (initial state and random stream), re-estimation
    # every step, 1800 sampled steps: six times longer than the weights
    # survive without it.  The weighted and plain temperature profiles agree
    # within their combined standard error (the members differ in the
    # initial sample, whose energy the weighted estimator inherits), and the
    # weighted profile's member-to-member scatter is well below the plain one.
    with Pool(8) as pool:
        res = pool.map(_fourier_member, [(1, s) for s in range(1, 9)])
    assert all(r[0] == 0 for r in res)
    plT = np.array([r[1] for r in res])
    vrT = np.array([r[2] for r in res])
    d = vrT - plT
    z = d.mean(0) / (d.std(0, ddof=1) / math.sqrt(len(res)))
    # 16 cells, t with 7 degrees of freedom: a few |z| > 2.4 by chance at most
    assert np.abs(z).max() < 5.5 and np.mean(np.abs(z) > 2.4) < 0.25, z
    # domain-mean temperature difference within 3 combined standard errors
    dm = d.mean(1)
    assert abs(dm.mean()) < 3 * dm.std(ddof=1) / math.sqrt(len(dm)) + 1e-4
    assert vrT.std(0, ddof=1).mean() < 0.35 * plT.std(0, ddof=1).mean()
    plq = np.array([r[3] for r in res]).mean(1)
    vrq = np.array([r[4] for r in res]).mean(1)
    assert vrq.std(ddof=1) < 0.5 * plq.std(ddof=1)
    assert abs(vrq.mean() - plq.mean()) < 3 * math.hypot(vrq.std(ddof=1), plq.std(ddof=1)) / math.sqrt(8)
