"""Pins of the CPU oracle against facts that do not come from the oracle itself:
published known-answer vectors, closed forms, conservation laws, exact
invariants and brute force on small inputs.  CPU only."""
import math
import os

import numpy as np
import pytest
from scipy import stats

import oracle
from oracle.philox_ref import philox4x32_10 as py_philox
from paper_2301_05985_amd import workloads as W

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# ------------------------------------------------------------------ Philox
def _kat():
    rows = []
    for line in open(os.path.join(GOLDEN, "philox4x32_10_kat.txt")):
        if line.startswith("#") or not line.strip():
            continue
        v = [int(t, 16) for t in line.split()]
        rows.append((v[0:4], v[4:6], v[6:10]))
    return rows


@pytest.mark.parametrize("row", _kat())
def test_philox_known_answers(row):
    ctr, key, out = row
    assert py_philox(ctr, key) == out
    assert list(oracle.philox(ctr, key)) == out


def test_philox_c_matches_python_definition():
    rng = np.random.default_rng(7)
    for _ in range(300):
        ctr = rng.integers(0, 2**32, 4, dtype=np.uint64)
        key = rng.integers(0, 2**32, 2, dtype=np.uint64)
        assert list(oracle.philox(ctr, key)) == py_philox([int(v) for v in ctr], [int(v) for v in key])


def test_philox_uniformity_chi2():
    # byte histogram of 4 * 20000 output words on consecutive counters
    words = np.array([oracle.philox([k, 2 << 24, 5, 9], [0, 0]) for k in range(20000)]).ravel()
    b = words.view(np.uint8)
    hist = np.bincount(b, minlength=256)
    chi2 = ((hist - b.size / 256) ** 2 / (b.size / 256)).sum()
    assert stats.chi2.sf(chi2, 255) > 1e-4


# ------------------------------------------------------- pair selection
@pytest.mark.parametrize("n", [2, 3, 5, 8])
def test_pair_draw_uniform_over_ordered_distinct_pairs(n):
    key = oracle.seed_key(3)
    cnt = np.zeros((n, n))
    draws = 4000 * n * (n - 1)
    for k in range(draws):
        i, j, U = oracle.pair(key, k, 11, 4, n)
        assert 0 <= i < n and 0 <= j < n and i != j
        assert 0.0 <= U < 1.0
        cnt[i, j] += 1
    obs = cnt[~np.eye(n, dtype=bool)]
    exp = draws / (n * (n - 1))
    chi2 = ((obs - exp) ** 2 / exp).sum()
    assert stats.chi2.sf(chi2, obs.size - 1) > 1e-4


def test_pair_index_map_brute_force_small_n():
    # the multiply-shift map sends r to floor(r n / 2^32): every index gets
    # floor(2^32/n) or ceil(2^32/n) preimages; verified at the preimage
    # boundaries with exact integer arithmetic for n <= 8
    key = oracle.seed_key(0)
    for n in range(2, 9):
        for k in range(200):
            r = oracle.philox([k, 2 << 24, 1, 2], key)
            i, j, _ = oracle.pair(key, k, 1, 2, n)
            lo_i = -(-(i << 32) // n)          # smallest r with floor(r n / 2^32) == i
            hi_i = -(-((i + 1) << 32) // n)    # first r of the next index
            assert lo_i <= int(r[0]) < hi_i
            jj = j - 1 if j > i else j
            lo_j = -(-(jj << 32) // (n - 1))
            hi_j = -(-((jj + 1) << 32) // (n - 1))
            assert lo_j <= int(r[1]) < hi_j


# ------------------------------------------------------------ scattering
@pytest.mark.parametrize("dtype,tol", [(np.float64, 2e-15), (np.float32, 2e-6)])
def test_direction_is_unit_and_isotropic(dtype, tol):
    key = oracle.seed_key(1)
    v = np.array([oracle.direction(key, k, 3, 7, dtype) for k in range(20000)], dtype=np.float64)
    assert np.abs(np.linalg.norm(v, axis=1) - 1.0).max() < tol
    # Archimedes: each component of a uniform unit vector is uniform on [-1, 1]
    for d in range(3):
        assert stats.kstest(v[:, d], "uniform", args=(-1, 2)).pvalue > 1e-4
    assert np.abs(v.mean(0)).max() < 4 * math.sqrt(1 / 3 / len(v))
    cov = v.T @ v / len(v)
    assert np.abs(cov - np.eye(3) / 3).max() < 0.02


@pytest.mark.parametrize("dtype,tol", [(np.float64, 1e-14), (np.float32, 1e-6)])
def test_scatter_conserves_momentum_energy_and_speed(dtype, tol):
    rng = np.random.default_rng(5)
    key = oracle.seed_key(2)
    for k in range(500):
        ci = rng.standard_normal(3) * 2
        cj = rng.standard_normal(3) * 2
        n = oracle.direction(key, k, 0, 0, dtype)
        a, b = oracle.scatter(ci.astype(dtype), cj.astype(dtype), n, dtype)
        ci64, cj64 = ci.astype(dtype).astype(np.float64), cj.astype(dtype).astype(np.float64)
        a, b = a.astype(np.float64), b.astype(np.float64)
        scale = np.abs(ci64).sum() + np.abs(cj64).sum()
        assert np.abs((a + b) - (ci64 + cj64)).max() < tol * scale
        e0 = (ci64 ** 2).sum() + (cj64 ** 2).sum()
        assert abs((a ** 2).sum() + (b ** 2).sum() - e0) < 4 * tol * e0
        assert abs(np.linalg.norm(a - b) - np.linalg.norm(ci64 - cj64)) < 4 * tol * scale
        # post-collision relative velocity is along the drawn direction
        g = a - b
        assert np.abs(g / np.linalg.norm(g) - n.astype(np.float64)).max() < 10 * tol * scale


# ------------------------------------------------------- exact majorant
def test_exact_bound_brackets_the_diameter():
    rng = np.random.default_rng(9)
    for trial in range(200):
        n = int(rng.integers(2, 60))
        c = rng.standard_normal((3, n)) * rng.uniform(0.1, 3) + rng.standard_normal((3, 1))
        for dtype in (np.float64, np.float32):
            b = oracle.exact_bound(*c, dtype=dtype)
            d = oracle.diameter(*c, dtype=dtype)
            assert b >= d
            # every radius about the box midpoint is at most half the box
            # diagonal, itself at most sqrt(3) times the largest extent
            assert b <= math.sqrt(3.0) * d * (1 + 1e-6) + 1e-300


def test_exact_bound_is_order_independent():
    rng = np.random.default_rng(4)
    c = rng.standard_normal((3, 300))
    o = rng.permutation(300)
    assert oracle.exact_bound(*c) == oracle.exact_bound(*c[:, o])


def _random_cells(rng, trials):
    """Random velocity sets, some with repeated velocities and some tiny."""
    for t in range(trials):
        n = int(rng.choice([0, 1, 2, 3, int(rng.integers(4, 90))]))
        c = rng.standard_normal((3, n)) * rng.uniform(0.2, 2.5) + rng.standard_normal((3, 1))
        if n >= 4 and t % 3 == 0:
            # duplicated particles (same velocity twice or more)
            k = int(rng.integers(1, n // 2 + 1))
            c[:, n - k:] = c[:, :k]
        yield c


@pytest.mark.parametrize("dtype", [np.float64, np.float32])
def test_diameter_is_the_largest_pairwise_distance(dtype):
    # brute force by scipy's pairwise distances (a library routine, in a
    # different summation and root order) over random cells with duplicates
    from scipy.spatial.distance import pdist
    rng = np.random.default_rng(21)
    for c in _random_cells(rng, 300):
        cw = c.astype(dtype)
        d = oracle.diameter(*cw, dtype=dtype)
        n = c.shape[1]
        if n < 2:
            assert d == 0.0
            continue
        ref = pdist(cw.T.astype(np.float64)).max()
        assert abs(d - ref) <= 1e-15 * max(ref, 1e-300), (n, d, ref)
        # the value is attained by some pair (not a bound)
        assert d <= ref * (1 + 1e-15)


@pytest.mark.parametrize("dtype", [np.float64, np.float32])
def test_features_are_the_cell_moments(dtype):
    # the six network inputs recomputed from their definitions with numpy's
    # mean, variance and covariance routines: log2 of the number density,
    # mean velocity over sqrt(T), log2 T (T = the mean of the three velocity
    # variances), P_xx / p - 1 and P_xy / p with p = n T
    rng = np.random.default_rng(22)
    for c in _random_cells(rng, 300):
        n = c.shape[1]
        if n < 2:
            continue
        cw = c.astype(dtype)
        FNum, V = float(rng.uniform(0.5, 40.0)), float(rng.uniform(0.01, 3.0))
        f = oracle.features(*cw, FNum, V, dtype=dtype).astype(np.float64)
        v = cw.astype(np.float64)
        u = v.mean(axis=1)
        var = v.var(axis=1)                 # population variances
        T = var.mean()
        if not T > 1e-12:
            continue                        # all velocities equal
        dens = n * FNum / V
        cov_xy = np.cov(v[0], v[1], bias=True)[0, 1]
        ref = np.array([math.log2(dens), u[0] / math.sqrt(T), u[1] / math.sqrt(T), math.log2(T),
                        var[0] / T - 1.0, cov_xy / T])
        # features are FP64 values rounded once to float: agreement to float
        # rounding plus the FP64 cancellation of the moment differences
        scale = 1.0 + np.abs(v).max() ** 2 / T
        tol = 2.0 ** -23 * np.abs(ref) + 1e-13 * scale
        assert (np.abs(f - ref) <= tol).all(), (n, f, ref)


def test_features_pin_detects_planted_slips():
    # the pin's reference distinguishes the plausible slips (P_xy over the
    # pressure instead of p = n T, a natural logarithm, a missing -1)
    rng = np.random.default_rng(23)
    c = rng.standard_normal((3, 50)) * 1.3 + np.array([[0.4], [-0.2], [0.1]])
    f = oracle.features(*c, 2.0, 0.5).astype(np.float64)
    T = c.var(axis=1).mean()
    pxy = np.cov(c[0], c[1], bias=True)[0, 1]
    assert abs(f[5] - pxy / T) < 1e-6 and abs(f[5] - pxy / (T * 100 * 2.0 / 0.5)) > 1e-3
    assert abs(f[3] - math.log2(T)) < 1e-6 and abs(f[3] - math.log(T)) > 1e-3
    assert abs(f[4] - (c[0].var() / T - 1.0)) < 1e-6 and abs(f[4] - c[0].var() / T) > 0.5


# ------------------------------------------------------- variance reduction
def test_vr_update_martingale_and_equilibrium_invariance():
    rng = np.random.default_rng(11)
    for _ in range(2000):
        p = rng.uniform(0.0, 0.999)
        wi, wj = rng.uniform(0.2, 3.0, 2)
        acc_i, _ = oracle.vr_update(True, p, wi, wj)
        rej_i, rej_j = oracle.vr_update(False, p, wi, wj)
        # expected weight after the candidate equals the weight before
        assert abs(p * acc_i + (1 - p) * rej_i - wi) < 1e-12 * max(1.0, wi * wj / (1 - p))
        assert abs(p * acc_i + (1 - p) * rej_j - wj) < 1e-12 * max(1.0, wi * wj / (1 - p))
        # unit weights are a fixed point in exact IEEE arithmetic
        for dt in (np.float64, np.float32):
            assert oracle.vr_update(True, p, 1.0, 1.0, dt) == (1.0, 1.0)
            assert oracle.vr_update(False, p, 1.0, 1.0, dt) == (1.0, 1.0)


# --------------------------------------------------------------- walls
@pytest.mark.parametrize("dtype", [np.float64, np.float32])
def test_diffuse_wall_sampler_moments(dtype):
    key = oracle.seed_key(6)
    Tw = 1.7
    n = 60000
    d = np.array([oracle.wall_draw(key, h % 8, h // 8, 3, Tw, dtype) for h in range(n)], dtype=np.float64)
    cn, t1, t2 = d.T
    assert (cn >= 0).all()
    se = lambda v: math.sqrt(v / n)
    # flux-Maxwellian normal speed: <c_n> = sqrt(pi Tw / 2), <c_n^2> = 2 Tw (Var = (2 - pi/2) Tw)
    assert abs(cn.mean() - math.sqrt(math.pi * Tw / 2)) < 5 * se((2 - math.pi / 2) * Tw)
    assert abs((cn ** 2).mean() - 2 * Tw) < 5 * se(4 * Tw * Tw)
    for t in (t1, t2):
        assert abs(t.mean()) < 5 * se(Tw)
        assert abs(t.var() - Tw) < 5 * se(2 * Tw * Tw)
    # Rayleigh law of c_n: P(c_n > s) = exp(-s^2 / 2 Tw)
    assert stats.kstest(cn, lambda s: 1 - np.exp(-s ** 2 / (2 * Tw))).pvalue > 1e-4


def test_wall_weight_ratio_has_unit_mean_under_the_wall_flux():
    key = oracle.seed_key(8)
    Tw, T0 = 2.0, 1.5
    uw = np.array([0.3, 0.0, 0.0])
    r = []
    for h in range(40000):
        cn, t1, t2 = oracle.wall_draw(key, h % 8, h // 8, 1, Tw)
        c = np.array([t1 + uw[0], cn, t2])  # a y-wall: normal is y, tangential x and z
        r.append(oracle.wall_ratio(c, Tw, uw, T0))
    r = np.array(r)
    assert abs(r.mean() - 1.0) < 5 * r.std() / math.sqrt(len(r))
    # equal temperatures at rest: the ratio is exactly one
    assert oracle.wall_ratio(np.array([0.3, 1.2, -0.7]), 1.5, np.zeros(3), 1.5) == 1.0


# ------------------------------------------------------------ full runs
@pytest.mark.parametrize("real,tol", [("f64", 1e-13), ("f32", 1e-6)])
def test_homogeneous_run_conserves_momentum_and_energy(real, tol):
    dtype = np.float64 if real == "f64" else np.float32
    p, parts = W.batched(n_inst=16, nmin=50, nmax=600, steps=20, real=real, dt=0.2)
    o = oracle.Oracle(p, parts, dtype)
    off = p["inst_offset"]
    def mom_en():
        c = np.stack([o.cx, o.cy, o.cz]).astype(np.float64)
        P = np.add.reduceat(c, off[:-1], axis=1)
        E = np.add.reduceat((c ** 2).sum(0), off[:-1])
        return P, E
    P0, E0 = mom_en()
    for _ in range(20):
        o.run(1)
        P1, E1 = mom_en()
        N = np.diff(off)
        T = E1 / (3 * N)
        assert (np.abs(P1 - P0).max(0) / (N * np.sqrt(T))).max() < tol
        assert (np.abs(E1 - E0) / E0).max() < tol
    assert o.counters[:, 1].sum() > 1000


def test_candidate_count_is_floor_of_mreal_plus_uniform():
    # M = floor(M_real + U0): the only values are floor(M_real) and
    # floor(M_real) + 1, and the mean is M_real (stateless NTC count)
    N, n_inst = 200, 400
    p, parts = W.bkw(N=N, n_inst=n_inst, K0=1.0, dt=0.037, steps=1)
    o = oracle.Oracle(p, parts)
    o.run(1)
    Mreal = 0.5 * N * (N - 1) * 1.0 * 1.0 * 0.037 / N
    M = o.counters[:, 0].astype(np.float64)
    assert set(np.unique(M)) <= {math.floor(Mreal), math.floor(Mreal) + 1}
    f = Mreal - math.floor(Mreal)
    assert abs(M.mean() - Mreal) < 5 * math.sqrt(f * (1 - f) / n_inst)
    assert (o.counters[:, 1] == o.counters[:, 0]).all()  # Maxwell molecules accept all


def test_candidate_count_limit():
    # at most 2^24 candidates per cell and step; one more is a capacity error
    # (Maxwell molecules: M_real = 1/2 (N - 1) dt exactly here)
    N = 200
    for M_real, ok in ((2.0 ** 24 - 2.0, True), (2.0 ** 24 + 1.5, False)):
        p, parts = W.bkw(N=N, n_inst=1, K0=1.0, dt=M_real / (0.5 * (N - 1)), steps=1)
        o = oracle.Oracle(p, parts)
        if ok:
            o.run(1)
            assert o.counters[0, 0] in (2 ** 24 - 2, 2 ** 24 - 1)
        else:
            with pytest.raises(RuntimeError, match="status -6"):
                o.run(1)


def test_hard_sphere_acceptance_rate_matches_exact_mean_relative_speed():
    # Given the state, each candidate is accepted with probability g / g_max for
    # a uniformly drawn ordered pair: E[accepted] = E[M] * mean_pairs(g) / g_max.
    # Many instances of the same equilibrium state, one short step each.
    N, n_inst = 120, 3000
    rng = np.random.default_rng(12)
    c = rng.standard_normal((3, N))
    cc = np.tile(c, n_inst)
    off = np.arange(n_inst + 1, dtype=np.int64) * N
    dt = 0.004
    p = dict(dims=0, n_cells=(n_inst, 1), dt=dt, sigma=1.0, FN=1.0, molecule=0, seed=5,
             inst_offset=off, cell_volume=np.ones(n_inst))
    o = oracle.Oracle(p, dict(cx=cc[0], cy=cc[1], cz=cc[2]))
    o.run(1)
    d = c[:, :, None] - c[:, None, :]
    g = np.sqrt((d ** 2).sum(0))
    gbar = g[~np.eye(N, dtype=bool)].mean()
    gmax = oracle.exact_bound(*c)
    Mreal = 0.5 * N * (N - 1) * dt * gmax
    cand = o.counters[:, 0].astype(float)
    acc = o.counters[:, 1].astype(float)
    assert abs(cand.mean() - Mreal) < 5 * 0.5 / math.sqrt(n_inst)
    pacc = gbar / gmax
    exp_acc = Mreal * pacc
    # binomial-with-random-M spread; a small in-step drift is far below this
    se = math.sqrt((Mreal * pacc * (1 - pacc) + 0.25 * pacc * pacc) / n_inst)
    assert abs(acc.mean() - exp_acc) < 5 * se


def _central_xx(o, off):
    c = np.stack([o.cx, o.cy, o.cz]).astype(np.float64)
    N = np.diff(off)
    u = np.add.reduceat(c, off[:-1], axis=1) / N
    m2 = np.add.reduceat(c ** 2, off[:-1], axis=1) / N
    T = (m2.sum(0) - (u ** 2).sum(0)) / 3.0
    return m2[0] - u[0] ** 2 - T


def test_maxwell_molecules_anisotropy_decay_closed_form():
    # Maxwell molecules, isotropic scattering: each collision multiplies the
    # expected x-anisotropy D = <c_x^2> - u_x^2 - T by (1 - 1/(N-1)) (pair
    # average over the empirical distribution), and the per-step count M is
    # floor(M_real + U), so E[D_s] = D_0 (E[a^M])^s exactly.
    N, n_inst, dt, steps = 300, 96, 0.05, 40
    p, parts = W.relaxation(N=N * n_inst, molecule=W.MAXWELL, steps=steps, dt=dt)
    # split into n_inst instances of N particles, each with the bimodal state
    c = np.stack([parts["cx"], parts["cy"], parts["cz"]])
    rng = np.random.default_rng(3)
    c = rng.standard_normal((3, N * n_inst))
    for b in range(n_inst):
        s = b * N
        c[0, s:s + N // 2] += 1.5
        c[0, s + N // 2:s + N] -= 1.5
    off = np.arange(n_inst + 1, dtype=np.int64) * N
    p = dict(dims=0, n_cells=(n_inst, 1), dt=dt, sigma=1.0, FN=1.0, molecule=W.MAXWELL, seed=2,
             inst_offset=off, cell_volume=np.full(n_inst, float(N)))
    o = oracle.Oracle(p, dict(cx=c[0], cy=c[1], cz=c[2]))
    D0 = _central_xx(o, off)
    a = 1.0 - 1.0 / (N - 1)
    Mr = 0.5 * N * (N - 1) * dt / N
    m, f = math.floor(Mr), Mr - math.floor(Mr)
    EaM = (1 - f) * a ** m + f * a ** (m + 1)
    ratios = []
    for s in range(1, steps + 1):
        o.run(1)
        if s % 10 == 0:
            D = _central_xx(o, off)
            pred = EaM ** s
            obs = (D / D0).mean()
            se = (D / D0).std() / math.sqrt(n_inst)
            ratios.append((obs, pred, se))
            assert abs(obs - pred) < 5 * se + 1e-3, (s, obs, pred, se)
    # the decay is visible (not a trivial pass)
    assert ratios[-1][1] < 0.4


@pytest.mark.slow
def test_bkw_fourth_and_sixth_moments():
    # BKW similarity solution for Maxwell molecules with isotropic scattering:
    # K(t) = 1 - (1 - K0) exp(-t/6) at nu = 1; <|c|^4> = 15 K (2 - K),
    # <|c|^6> = 105 K^2 (3 - 2K).  Finite-N corrections are O(1/N).
    N, n_inst, K0, dt = 2000, 24, 0.6, 0.05
    p, parts = W.bkw(N=N, n_inst=n_inst, K0=K0, dt=dt, seed=4)
    o = oracle.Oracle(p, parts)
    off = p["inst_offset"]
    def moms():
        c2 = (np.stack([o.cx, o.cy, o.cz]) ** 2).sum(0)
        return (np.add.reduceat(c2 ** 2, off[:-1]) / N, np.add.reduceat(c2 ** 3, off[:-1]) / N)
    t = 0.0
    for target in (1.0, 3.0, 6.0):
        nst = int(round((target - t) / dt))
        o.run(nst)
        t += nst * dt
        K = 1 - (1 - K0) * math.exp(-t / 6)
        m4, m6 = moms()
        e4, e6 = 15 * K * (2 - K), 105 * K * K * (3 - 2 * K)
        assert abs(m4.mean() - e4) < 5 * m4.std() / math.sqrt(n_inst) + 0.01 * e4, (t, m4.mean(), e4)
        assert abs(m6.mean() - e6) < 5 * m6.std() / math.sqrt(n_inst) + 0.02 * e6, (t, m6.mean(), e6)


def test_hard_sphere_relaxes_to_the_maxwellian():
    p, parts = W.relaxation(N=6000, steps=300)
    o = oracle.Oracle(p, parts)
    Teq = p["T_eq"]
    c = np.stack([o.cx, o.cy, o.cz])
    u = c.mean(1)
    assert abs(((c - u[:, None]) ** 2).sum(0).mean() / 3 - Teq) < 0.05
    o.run(300)  # 15 equilibrium collision times
    c = np.stack([o.cx, o.cy, o.cz])
    u = c.mean(1)
    cc = c - u[:, None]
    T = (cc ** 2).sum(0).mean() / 3
    kx = (cc[0] ** 4).mean() / (cc[0] ** 2).mean() ** 2
    assert abs(kx - 3.0) < 0.25  # started at 2.04 (bimodal)
    m4 = ((cc ** 2).sum(0) ** 2).mean()
    assert abs(m4 / (15 * T * T) - 1) < 0.08
    for d in range(3):
        assert stats.kstest(cc[d] / math.sqrt(T), "norm").pvalue > 1e-3


def test_results_do_not_depend_on_storage_order():
    # the initial sequence orders each cell by particle id, later sequences
    # follow from it by stable grouping, and every draw is keyed by (step,
    # cell, candidate) or (step, particle, hit): permuting the storage order
    # must give the same bits per particle
    p, parts = W.cavity(nx=4, ny=4, per_cell=12, Kn=0.05, steps=6, real="f64")
    a = oracle.Oracle(p, parts)
    b = oracle.Oracle(p, W.shuffle_storage(parts, seed=3))
    a.run(6)
    b.run(6)
    sa, sb = a.state(), b.state()
    for k in ("x", "y", "cx", "cy", "cz", "w"):
        assert np.array_equal(sa[k], sb[k]), k
    assert np.array_equal(a.counters, b.counters)


def test_checkpoint_resume_is_bit_exact():
    p, parts = W.fourier(n_cells=10, per_cell=30, Kn=0.05, steps=10, real="f64")
    a = oracle.Oracle(p, parts)
    a.run(10)
    b = oracle.Oracle(p, parts)
    b.run(5)
    snap = b.sequence_state()
    c = oracle.Oracle(p, snap, layout="storage")
    c.step = 5
    c.run(5)
    sa, sc = a.state(), c.state()
    for k in ("x", "cx", "cy", "cz", "w"):
        assert np.array_equal(sa[k], sc[k]), k


def test_vr_weights_stay_exactly_one_between_walls_at_the_reference_temperature():
    p, parts = W.fourier(n_cells=10, per_cell=40, Kn=0.05, T_left=1.5, T_right=1.5, T0=1.5,
                         steps=50, real="f32")
    o = oracle.Oracle(p, parts, np.float32)
    o.run(50)
    assert o.diag.wall_hits > 0 and o.counters[:, 1].sum() > 0
    assert (o.w == 1.0).all()
    assert np.abs(o.sums[:, 13:]).max() == 0.0


def test_free_molecular_heat_flux_closed_form():
    # No collisions between diffuse walls at T1, T2: the left- and right-moving
    # populations are half-range Maxwellians with densities n1 sqrt(T1) =
    # n2 sqrt(T2); number flux Gamma = n sqrt(2/pi) sqrt(T1 T2)/(sqrt T1 + sqrt T2)
    # and heat flux q_x = 2 Gamma (T1 - T2).
    T1, T2 = 1.0, 2.0
    p, parts = W.fourier(n_cells=10, per_cell=600, Kn=0.0, sigma=0.0, T_left=T1, T_right=T2,
                         steps=1, dt=0.01, real="f64", vr=0)
    o = oracle.Oracle(p, parts)
    o.run(400)
    o.reset_samples()
    ns = 800
    o.run(ns)
    n = 6000.0
    est = oracle.estimators(o.sums, ns, 1.0, 0.1)
    G = n * math.sqrt(2 / math.pi) * math.sqrt(T1 * T2) / (math.sqrt(T1) + math.sqrt(T2))
    q = 2 * G * (T1 - T2)
    assert np.abs(est["n"] / n - 1).max() < 0.03
    assert abs(est["q"][:, 0].mean() / q - 1) < 0.03, (est["q"][:, 0].mean(), q)
    assert np.abs(est["u"][:, 0]).max() < 0.05


@pytest.mark.parametrize("real", ["f64", "f32"])
def test_fourier_vr_and_plain_estimators_agree(real):
    # Near equilibrium the variance-reduced estimator and the plain one
    # estimate the same profile; runs are kept short (a few collision times)
    # because the raw weights' variance grows without reconstruction.
    dtype = np.float64 if real == "f64" else np.float32
    p, parts = W.fourier(n_cells=8, per_cell=300, Kn=0.1, T_left=1.45, T_right=1.55, T0=1.5,
                         dt=2e-3, steps=1, real=real)
    o = oracle.Oracle(p, parts, dtype)
    o.run(20)
    o.reset_samples()
    ns = 60
    o.run(ns)
    assert o.diag.vr_nonfinite == 0
    V = 1.0 / 8
    plain = oracle.estimators(o.sums, ns, 1.0, V)
    vr = oracle.estimators(o.sums, ns, 1.0, V, vr=True, vr_n0=p["vr_n0"], vr_T0=1.5)
    # domain-averaged temperature: plain-estimator noise ~ 1.5 sqrt(2/3/N_eff)
    assert abs(plain["T"].mean() - vr["T"].mean()) < 0.05
    assert abs(plain["n"].mean() / vr["n"].mean() - 1) < 0.02
    # the weighted estimator is far less noisy near equilibrium
    assert np.std(vr["T"] - 1.5) < np.std(plain["T"] - 1.5)


def test_vr_weight_divergence_is_a_diagnostic_not_an_error():
    # Without weight reconstruction the weight variance grows exponentially in
    # collision times; the motion never depends on the weights, so the run
    # continues and the plain sums stay finite.
    p, parts = W.fourier(n_cells=8, per_cell=150, Kn=0.1, T_left=1.4, T_right=1.6, T0=1.5,
                         dt=2e-3, steps=1, real="f64")
    o = oracle.Oracle(p, parts)
    o.run(400)
    assert np.isfinite(o.sums[:, :13]).all()
    assert o.diag.vr_nonfinite > 0


def _cells_np(p, x, y):
    nx = p["n_cells"][0]
    ix = np.clip(np.floor(np.asarray(x, dtype=np.float64) * nx), 0, nx - 1).astype(np.int64)
    if p["dims"] < 2:
        return ix
    ny = p["n_cells"][1]
    iy = np.clip(np.floor(np.asarray(y, dtype=np.float64) * ny), 0, ny - 1).astype(np.int64)
    return iy * nx + ix


@pytest.mark.parametrize("kind", ["cavity", "fourier"])
def test_particle_sequence_is_a_stable_grouping_by_cell(kind):
    # the initial sequence is (cell, id) in lexicographic order; after every
    # step the sequence is the previous one regrouped by the new cells with
    # the relative order kept (checked against numpy's stable argsort)
    if kind == "cavity":
        p, parts = W.cavity(nx=6, ny=5, per_cell=20, Kn=0.05, steps=4, real="f64", dt=0.05)
    else:
        p, parts = W.fourier(n_cells=7, per_cell=25, Kn=0.05, steps=4, real="f64", dt=0.02)
    parts = W.shuffle_storage(parts, seed=5)
    o = oracle.Oracle(p, parts)
    cell0 = _cells_np(p, o.x, o.y)
    want = np.lexsort((o.id, cell0))
    assert np.array_equal(o.layout, want)
    moved = 0
    for _ in range(4):
        prev = o.layout.copy()
        c_prev = _cells_np(p, o.x, o.y)
        o.run(1)
        c_new = _cells_np(p, o.x, o.y)
        moved += int((c_prev != c_new).sum())
        want = prev[np.argsort(c_new[prev], kind="stable")]
        assert np.array_equal(o.layout, want)
    assert moved > 20


# ------------------------------------------------------ VHS molecules
def test_vhs_power_matches_the_power_function():
    # the fixed-sequence x^a of the VHS acceptance against numpy's power, and
    # its exact special values
    rng = np.random.default_rng(21)
    x = np.concatenate([rng.random(3000), 10.0 ** rng.uniform(-300, 0, 1000), [1e-308, 0.5, 0.999999, 1.2]])
    a = rng.uniform(0.0, 1.0, len(x))
    got = np.array([oracle.vhs_pow(u, v) for u, v in zip(x, a)])
    want = np.power(x, a)
    # 2^(a log2 x): the exponent's own rounding (~ulp(|y|)) is the error floor
    y = np.abs(a * np.log2(x))
    assert (np.abs(got - want) / want / (8.0 + y)).max() < 2e-16
    for u in (0.3, 1e-10, 0.999):
        tol = 2e-16 * (8.0 + abs(math.log2(u)))
        assert oracle.vhs_pow(u, 0.0) == 1.0
        assert abs(oracle.vhs_pow(u, 1.0) / u - 1) < tol
        assert abs(oracle.vhs_pow(u, 0.5) / math.sqrt(u) - 1) < tol
    for v in (0.0, 0.19, 0.5, 1.0):
        assert oracle.vhs_pow(1.0, v) == 1.0
    assert oracle.vhs_pow(0.0, 0.3) == 0.0


@pytest.mark.parametrize("real", ["f64", "f32"])
def test_vhs_at_omega_one_is_maxwell_molecules_bit_for_bit(real):
    # omega = 1: sigma_T g is constant, (g / g_max)^0 = 1 accepts every
    # candidate and the majorant factor is 1, exactly the Maxwell-molecule run
    dtype = np.float64 if real == "f64" else np.float32
    p, parts = W.bkw(N=400, n_inst=6, dt=0.05, seed=3, real=real)
    a = oracle.Oracle(p, parts, dtype)
    b = oracle.Oracle(dict(p, molecule=W.VHS, omega=1.0), parts, dtype)
    a.run(12)
    b.run(12)
    for k in ("cx", "cy", "cz"):
        assert np.array_equal(getattr(a, k), getattr(b, k)), k
    assert np.array_equal(a.counters, b.counters)


def test_vhs_acceptance_rate_matches_exact_pair_mean():
    # VHS (omega = 0.81, argon-like): a candidate is accepted with probability
    # (g / g_max)^(2 - 2 omega), so E[accepted] = E[M] mean_pairs(g^(2-2w)) /
    # g_max^(2-2w), with M_real = 1/2 N (N-1) sigma g_max^(2-2w) dt
    N, n_inst, dt, om = 120, 3000, 0.004, 0.81
    rng = np.random.default_rng(13)
    c = rng.standard_normal((3, N))
    cc = np.tile(c, n_inst)
    off = np.arange(n_inst + 1, dtype=np.int64) * N
    p = dict(dims=0, n_cells=(n_inst, 1), dt=dt, sigma=1.0, FN=1.0, molecule=W.VHS, omega=om, seed=6,
             inst_offset=off, cell_volume=np.ones(n_inst))
    o = oracle.Oracle(p, dict(cx=cc[0], cy=cc[1], cz=cc[2]))
    o.run(1)
    d = c[:, :, None] - c[:, None, :]
    g = np.sqrt((d ** 2).sum(0))
    e = 2.0 - 2.0 * om
    gbar = (g[~np.eye(N, dtype=bool)] ** e).mean()
    gmax = oracle.exact_bound(*c)
    Mreal = 0.5 * N * (N - 1) * dt * gmax ** e
    cand = o.counters[:, 0].astype(float)
    acc = o.counters[:, 1].astype(float)
    assert abs(cand.mean() - Mreal) < 5 * 0.5 / math.sqrt(n_inst)
    pacc = gbar / gmax ** e
    se = math.sqrt((Mreal * pacc * (1 - pacc) + 0.25 * pacc * pacc) / n_inst)
    assert abs(acc.mean() - Mreal * pacc) < 5 * se
    # a softer cross-section accepts more often than hard spheres would
    assert pacc > (g[~np.eye(N, dtype=bool)]).mean() / gmax


def test_vhs_relaxes_to_the_maxwellian_and_conserves():
    p, parts = W.relaxation(N=6000, steps=300)
    p = dict(p, molecule=W.VHS, omega=0.81)
    o = oracle.Oracle(p, parts)
    c0 = np.stack([o.cx, o.cy, o.cz])
    P0, E0 = c0.sum(1), (c0 ** 2).sum()
    o.run(300)
    c = np.stack([o.cx, o.cy, o.cz])
    assert np.abs(c.sum(1) - P0).max() < 1e-9 * len(o.cx)
    assert abs((c ** 2).sum() / E0 - 1) < 1e-12
    u = c.mean(1)
    cc = c - u[:, None]
    T = (cc ** 2).sum(0).mean() / 3
    kx = (cc[0] ** 4).mean() / (cc[0] ** 2).mean() ** 2
    assert abs(kx - 3.0) < 0.25  # started at 2.04 (bimodal)
    for d in range(3):
        assert stats.kstest(cc[d] / math.sqrt(T), "norm").pvalue > 1e-3


# ------------------------------------------------------ VSS molecules
def _sphere(rng, n):
    v = rng.standard_normal((n, 3))
    return v / np.linalg.norm(v, axis=1)[:, None]


def _vss_batch(alpha, n, seed, degenerate=False):
    rng = np.random.default_rng(seed)
    ci = rng.standard_normal((n, 3)) * 1.3 + 0.2
    cj = rng.standard_normal((n, 3)) * 0.8 - 0.1
    if degenerate:  # relative velocity along the x axis: the second frame
        cj[:, 1:] = ci[:, 1:]
    nn = _sphere(rng, n)
    out_i, out_j = np.empty_like(ci), np.empty_like(cj)
    for k in range(n):
        out_i[k], out_j[k] = oracle.scatter_vss(ci[k], cj[k], nn[k], alpha)
    return ci, cj, out_i, out_j


@pytest.mark.parametrize("degenerate", [False, True])
def test_vss_collision_conserves_momentum_and_energy(degenerate):
    for alpha in (1.0, 1.4, 2.0):
        ci, cj, ai, aj = _vss_batch(alpha, 400, 31, degenerate)
        assert np.abs((ai + aj) - (ci + cj)).max() < 1e-14
        g, gp = ci - cj, ai - aj
        e0 = (ci ** 2).sum(1) + (cj ** 2).sum(1)
        e1 = (ai ** 2).sum(1) + (aj ** 2).sum(1)
        assert np.abs(e1 / e0 - 1).max() < 1e-14
        # |g'| = |g| up to the rounding of the velocities themselves
        scale = np.linalg.norm(ci, axis=1) + np.linalg.norm(cj, axis=1)
        assert (np.abs(np.linalg.norm(gp, axis=1) - np.linalg.norm(g, axis=1)) / scale).max() < 1e-14


@pytest.mark.parametrize("alpha", [1.0, 1.4, 2.0])
def test_vss_deflection_law(alpha):
    # cos chi = 2 B^(1/alpha) - 1 with B uniform: ((1 + cos chi)/2)^alpha is
    # uniform; E[cos chi] = (alpha - 1)/(alpha + 1) and the viscosity factor
    # E[sin^2 chi] = 4 alpha / ((alpha + 1)(alpha + 2)); the azimuth about g,
    # measured in a frame that is not the one used to build g', is uniform
    n = 20000
    ci, cj, ai, aj = _vss_batch(alpha, n, 41)
    g, gp = ci - cj, ai - aj
    gn = g / np.linalg.norm(g, axis=1)[:, None]
    cchi = (gp * gn).sum(1) / np.linalg.norm(gp, axis=1)
    assert stats.kstest(((1 + cchi) / 2) ** alpha, "uniform").pvalue > 1e-3
    m1 = (alpha - 1) / (alpha + 1)
    assert abs(cchi.mean() - m1) < 5 * cchi.std() / math.sqrt(n)
    s2 = 1 - cchi ** 2
    assert abs(s2.mean() - 4 * alpha / ((alpha + 1) * (alpha + 2))) < 5 * s2.std() / math.sqrt(n)
    perp = gp - (gp * gn).sum(1)[:, None] * gn
    e1 = np.cross(gn, np.array([0.3, -0.5, 0.81]))
    e1 /= np.linalg.norm(e1, axis=1)[:, None]
    e2 = np.cross(gn, e1)
    phi = np.arctan2((perp * e2).sum(1), (perp * e1).sum(1))
    assert stats.kstest(phi, "uniform", args=(-math.pi, 2 * math.pi)).pvalue > 1e-3


def test_vss_maxwell_group_momentum_decay_closed_form():
    # Maxwell molecules (omega = 1: every candidate accepted) with VSS
    # scattering.  One collision moves each partner's velocity by (g' - g)/2,
    # whose mean over the scattering law is -(1 - E[cos chi]) g / 2 =
    # -g / (alpha + 1).  For a uniform ordered pair of an N-particle cell, the
    # momentum of a marked half, taken relative to its share of the total,
    # D = S_+ - (N_+ / N) S, therefore shrinks in expectation by the factor
    # r = 1 - 2 / ((alpha + 1)(N - 1)) per candidate: E[D_end] = D_0 r^M for
    # M candidates, whatever the velocity distribution.
    N, n_inst, alpha, steps = 100, 400, 2.0, 10
    dt = 15.0 / (0.5 * N * (N - 1))  # about 15 candidates per step
    rng = np.random.default_rng(17)
    c = rng.standard_normal((3, N * n_inst))
    c[0] += np.where((np.arange(N * n_inst) % N) < N // 2, 1.5, -1.5)
    off = np.arange(n_inst + 1, dtype=np.int64) * N
    p = dict(dims=0, n_cells=(n_inst, 1), dt=dt, sigma=1.0, FN=1.0, molecule=W.VSS, omega=1.0,
             alpha=alpha, seed=8, inst_offset=off, cell_volume=np.ones(n_inst))
    o = oracle.Oracle(p, dict(cx=c[0].copy(), cy=c[1].copy(), cz=c[2].copy()))
    o.run(steps)
    assert (o.counters[:, 0] == o.counters[:, 1]).all()
    M = o.counters[:, 0].astype(float)

    def D(cx):
        v = cx.reshape(n_inst, N)
        return v[:, : N // 2].sum(1) - 0.5 * v.sum(1)

    d0, d1 = D(c[0]), D(o.cx)
    def ratio(a):
        return d1 / (d0 * (1 - 2 / ((a + 1) * (N - 1))) ** M)
    q = ratio(alpha)
    se = q.std() / math.sqrt(n_inst)
    assert abs(q.mean() - 1) < 5 * se
    # isotropic scattering (alpha = 1) would predict a faster decay
    assert abs(ratio(1.0).mean() - 1) > 10 * se


def test_vss_run_conserves_and_keeps_vhs_collision_counts_on_first_step():
    # the scattering law does not enter the majorant or the acceptance: the
    # first step's candidate counts equal the VHS run's, and the collisions
    # conserve momentum and energy
    p, parts = W.relaxation(N=3000, steps=1)
    a = oracle.Oracle(dict(p, molecule=W.VHS, omega=0.81), parts)
    b = oracle.Oracle(dict(p, molecule=W.VSS, omega=0.81, alpha=1.6), parts)
    c0 = np.stack([b.cx, b.cy, b.cz])
    a.run(1)
    b.run(1)
    assert np.array_equal(a.counters[:, 0], b.counters[:, 0])
    c = np.stack([b.cx, b.cy, b.cz])
    assert np.abs(c.sum(1) - c0.sum(1)).max() < 1e-10
    assert abs((c ** 2).sum() / (c0 ** 2).sum() - 1) < 1e-13
    assert not np.array_equal(c, np.stack([a.cx, a.cy, a.cz]))
