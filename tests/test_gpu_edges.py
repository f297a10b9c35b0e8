"""Edge cases of the GPU path against the oracle: empty runs, cells and
instances; every particle in one cell; particles exactly on cell edges and
walls; one and two particles."""
import numpy as np
import pytest

import oracle
from paper_2301_05985_amd import workloads as W
from tests.sums_check import assert_sums_close

pytestmark = pytest.mark.gpu


def _announce(name):
    print("[gpu case] %s" % name, flush=True)


def _both(p, parts, steps, real="f64"):
    from paper_2301_05985_amd.binding import Simulation
    p = dict(p, real=real)
    dtype = np.float64 if real == "f64" else np.float32
    sim = Simulation(p, parts)
    orc = oracle.Oracle(p, parts, dtype)
    sim.step(steps)
    orc.run(steps)
    sums, cnt, ns = sim.sample()
    g = sim.particles()
    seq = sim.sequence()["id"] if p["dims"] >= 1 and len(parts["cx"]) else None
    d = sim.diagnostics()
    sim.close()
    return g, sums, cnt, ns, seq, d, orc


def _check(g, sums, cnt, seq, d, orc, fields=("x", "y", "cx", "cy", "cz", "w")):
    assert d["status"] == 0, d
    o = orc.state()
    assert np.array_equal(g["id"], o["id"])
    if seq is not None:
        assert np.array_equal(seq, orc.sequence_state()["id"])
    assert np.array_equal(cnt, orc.counters)
    for k in fields:
        if g[k] is None or len(g[k]) == 0:
            continue
        assert np.array_equal(g[k], o[k]), k
    assert_sums_close(sums, orc.sums, 1e-11)


def _spec(p):
    return dict(p, wall_kind=(W.WALL_SPECULAR,) * 4)


@pytest.mark.parametrize("dims", [1, 2])
def test_no_particles(gpu, dims):
    _announce("no particles dims=%d" % dims)
    if dims == 2:
        p, _ = W.cavity(nx=6, ny=5, per_cell=1, Kn=0.05, dt=0.01)
    else:
        p, _ = W.fourier(n_cells=7, per_cell=1, Kn=0.05, dt=0.01)
    e = np.zeros(0)
    parts = dict(x=e, y=e, cx=e, cy=e, cz=e, w=e, id=np.zeros(0, dtype=np.uint32))
    g, sums, cnt, ns, seq, d, orc = _both(p, parts, 9)
    assert ns == 9 and not sums.any() and not cnt.any()
    _check(g, sums, cnt, seq, d, orc)


def test_homogeneous_instances_empty_and_single(gpu):
    _announce("homogeneous empty/single instances")
    counts = [0, 1, 0, 2, 1, 0]
    off = np.concatenate([[0], np.cumsum(counts)]).astype(np.int64)
    rng = np.random.default_rng(4)
    c = rng.standard_normal((3, int(off[-1])))
    p = dict(dims=0, n_cells=(len(counts), 1), dt=0.5, sigma=0.5, FN=1.0, molecule=0, seed=3,
             inst_offset=off, cell_volume=np.ones(len(counts)))
    g, sums, cnt, ns, seq, d, orc = _both(p, dict(cx=c[0], cy=c[1], cz=c[2], id=np.arange(len(c[0]), dtype=np.uint32)), 7)
    assert cnt[3, 0] > 0  # the pair collides
    _check(g, sums, cnt, seq, d, orc, fields=("cx", "cy", "cz"))


@pytest.mark.parametrize("real", ["f64", "f32"])
def test_every_particle_in_one_cell(gpu, real):
    # 2,500 particles start in one corner cell of a 5 x 5 grid (above the LDS
    # capacity: global-memory gather and collisions) and spread out
    _announce("one crowded cell %s" % real)
    p, _ = W.cavity(nx=5, ny=5, per_cell=1, Kn=0.05, dt=0.02)
    p = _spec(p)
    n = 2500
    rng = np.random.default_rng(6)
    parts = dict(x=rng.random(n) * 0.2, y=rng.random(n) * 0.2, cx=rng.standard_normal(n),
                 cy=rng.standard_normal(n), cz=rng.standard_normal(n), w=np.ones(n),
                 id=rng.permutation(n).astype(np.uint32))
    p["sigma"] = 2e-4
    g, sums, cnt, ns, seq, d, orc = _both(p, parts, 6, real)
    assert d["big_cells"] > 0 and cnt[:, 1].sum() > 100
    _check(g, sums, cnt, seq, d, orc)


def test_particles_on_cell_edges_and_walls(gpu):
    # positions exactly on cell edges k/n and on the walls 0 and 1, at rest
    # and moving, with specular and periodic walls
    _announce("edges and walls")
    p, _ = W.cavity(nx=8, ny=4, per_cell=1, Kn=0.05, dt=0.01)
    p["wall_kind"] = (W.WALL_PERIODIC, W.WALL_PERIODIC, W.WALL_SPECULAR, W.WALL_SPECULAR)
    xs = np.array([0.0, 1.0, 0.125, 0.25, 0.5, 0.875, 1.0 - 2 ** -40, 0.375])
    ys = np.array([0.0, 1.0, 0.25, 0.5, 0.75, 0.25, 1.0, 0.0])
    X, Y = np.meshgrid(xs, ys)
    x, y = X.ravel(), Y.ravel()
    n = len(x)
    rng = np.random.default_rng(8)
    c = rng.standard_normal((3, n))
    c[:, :8] = 0.0  # some at rest on an edge
    parts = dict(x=x, y=y, cx=c[0], cy=c[1], cz=c[2], w=np.ones(n), id=np.arange(n, dtype=np.uint32))
    p["sigma"] = 0.02
    g, sums, cnt, ns, seq, d, orc = _both(p, parts, 12)
    _check(g, sums, cnt, seq, d, orc)


@pytest.mark.parametrize("n", [1, 2])
def test_one_and_two_particles(gpu, n):
    _announce("%d particle(s)" % n)
    p, _ = W.fourier(n_cells=3, per_cell=1, Kn=0.05, dt=0.05)
    p["wall_kind"] = (W.WALL_SPECULAR, W.WALL_SPECULAR, 0, 0)
    p["sigma"] = 5.0
    parts = dict(x=np.array([0.1, 0.15])[:n], cx=np.array([0.7, -0.3])[:n], cy=np.array([0.2, 0.1])[:n],
                 cz=np.array([-0.4, 0.9])[:n], w=np.ones(n), id=np.arange(n, dtype=np.uint32))
    g, sums, cnt, ns, seq, d, orc = _both(p, parts, 20)
    _check(g, sums, cnt, seq, d, orc)


def _lds_fit(real, packed=False):
    # the largest multiple of 32 particles whose LDS staging fits 64 KiB
    # (homogeneous runs without weights keep no separate owner array)
    rb = 8 if real == "f64" else 4
    return (65472 // (4 * rb + (0 if packed else 4))) // 32 * 32


@pytest.mark.parametrize("real", ["f64", "f32"])
def test_instances_at_lds_capacity_and_one_above(gpu, real):
    # the largest instance that is staged in LDS and the smallest one that
    # is not (global-memory kernel), side by side
    cap = _lds_fit(real, packed=True)
    _announce("instances at capacity %s (%d)" % (real, cap))
    counts = [cap, cap + 1, 50]
    off = np.concatenate([[0], np.cumsum(counts)]).astype(np.int64)
    rng = np.random.default_rng(14)
    c = rng.standard_normal((3, int(off[-1])))
    c[0, :cap // 2] += 1.0
    p = dict(dims=0, n_cells=(len(counts), 1), dt=0.05, sigma=3e-4, FN=1.0, molecule=0, seed=9,
             inst_offset=off, cell_volume=np.ones(len(counts)))
    steps = 3
    g, sums, cnt, ns, seq, d, orc = _both(p, dict(cx=c[0], cy=c[1], cz=c[2], id=np.arange(len(c[0]), dtype=np.uint32)),
                                          steps, real)
    assert d["big_cells"] == steps  # only the instance above capacity
    assert cnt[0, 1] > 100 and cnt[1, 1] > 100
    _check(g, sums, cnt, seq, d, orc, fields=("cx", "cy", "cz"))


@pytest.mark.parametrize("vr", [1, 0])
@pytest.mark.parametrize("extra", [0, 1])
def test_walled_cell_at_lds_capacity_and_one_above(gpu, extra, vr):
    # 160 particles in 8 cells: the FP32 per-cell capacity is 2.5 x 20 + 64
    # with weights, 2 x 20 + 64 without, both rounded up to 128; cell 0 holds 128
    # (staged in LDS) or 129 (global memory).  A tiny time step keeps every
    # particle in its cell.
    _announce("walled cell at capacity + %d, weights %d" % (extra, vr))
    p, _ = W.fourier(n_cells=8, per_cell=1, Kn=0.05, dt=1e-7, vr=vr)
    p["wall_kind"] = (W.WALL_SPECULAR, W.WALL_SPECULAR, 0, 0)
    p["sigma"] = 1300.0
    n, n0 = 160, 128 + extra
    rng = np.random.default_rng(12)
    x = np.concatenate([rng.uniform(0.01, 0.115, n0), rng.uniform(0.135, 0.99, n - n0)])
    c = rng.standard_normal((3, n))
    parts = dict(x=x, cx=c[0], cy=c[1], cz=c[2], w=np.ones(n), id=rng.permutation(n).astype(np.uint32))
    g, sums, cnt, ns, seq, d, orc = _both(p, parts, 4, "f32")
    assert (d["big_cells"] > 0) == bool(extra)
    assert cnt[0, 1] > 20
    _check(g, sums, cnt, seq, d, orc)


def test_setup_rejects_a_cell_above_the_ordering_bound(gpu):
    # 140,000 particles in one cell of a 2 x 2 grid: above the 131,072 that
    # the set-up's per-cell ordering by id accepts, so dsmc_init returns
    # DSMC_ECAPACITY (at once, before any ordering kernel runs)
    _announce("set-up cell above the ordering bound")
    from paper_2301_05985_amd.binding import DsmcError, Simulation
    p, _ = W.cavity(nx=2, ny=2, per_cell=1, Kn=0.05, dt=0.01)
    p = dict(_spec(p), real="f32", sigma=0.0)
    n = 140_000
    rng = np.random.default_rng(21)
    parts = dict(x=rng.uniform(0.05, 0.45, n), y=rng.uniform(0.05, 0.45, n), cx=rng.standard_normal(n),
                 cy=rng.standard_normal(n), cz=rng.standard_normal(n), w=np.ones(n),
                 id=np.arange(n, dtype=np.uint32))
    with pytest.raises(DsmcError) as e:
        Simulation(p, parts)
    assert e.value.code == -6  # DSMC_ECAPACITY


def test_overflow_merge_above_its_work_bound_reports_capacity(gpu):
    # 20,000 particles cross from cell 1 into cell 0 of a two-cell slab in one
    # step: 19,744 of them beyond the 256 mover slots, and 20,000 x 19,744 is
    # above the merge's work bound (2^28), so the step ends at once with
    # DSMC_ECAPACITY instead of ranking the entries (no collisions: sigma 0)
    _announce("overflow merge above its work bound")
    from paper_2301_05985_amd.binding import Simulation
    p, _ = W.fourier(n_cells=2, per_cell=1, Kn=0.05, dt=0.01, vr=0, real="f32")
    p = dict(p, wall_kind=(W.WALL_SPECULAR, W.WALL_SPECULAR, 0, 0), sigma=0.0)
    n = 20_000
    rng = np.random.default_rng(22)
    parts = dict(x=rng.uniform(0.55, 0.95, n), cx=np.full(n, -50.0), cy=np.zeros(n), cz=np.zeros(n),
                 w=np.ones(n), id=rng.permutation(n).astype(np.uint32))
    sim = Simulation(p, parts)
    assert sim.diagnostics()["status"] == 0
    sim.step(1)
    d = sim.diagnostics()
    sim.close()
    assert d["status"] == -6  # DSMC_ECAPACITY
