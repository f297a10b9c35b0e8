"""The walled launches other than one cell per wave -- two cells per wave
(cells_per_wave = 2, 32 lanes per cell) and a workgroup of four waves per
cell (waves_per_cell = 4) -- against the CPU oracle and against the
one-cell-per-wave launch, through the C ABI.

Bar: as in the other walled parity tests.  Pair choices, counts and the
particle sequence are bit-exact; the state is bit-exact where no
transcendental function enters (specular and periodic walls) and within
1e-12 relative (FP32: four ulp) otherwise; re-estimated weights carry the re-estimation's
tolerance (1e-9 of max(|W|, 1) in FP64, a few ulp in FP32).  Against the
one-cell launch the motion, the sequence and the counters are identical (the
same decisions in the same order); the sums, and re-estimated weights, differ
only by their order of summation.

Cases: both precisions; specular, periodic and diffuse walls; weights with
and without re-estimation; hard, variable hard and variable soft spheres;
the brute-force majorant; several generations of candidates per cell with
weights; cells above the pair capacity (global-memory kernel) and overflow
mover lists; odd cell counts, so that a wave's second
half has no cell; single-cell and tiny periodic grids; up to 128 movers per
cell; empty runs and one or two particles."""
import sys

import numpy as np
import pytest

import oracle
from paper_2301_05985_amd import workloads as W
from tests.sums_check import assert_sums_close

pytestmark = pytest.mark.gpu

SPEC = (W.WALL_SPECULAR,) * 4
PERIODIC_X = (W.WALL_PERIODIC, W.WALL_PERIODIC, W.WALL_SPECULAR, W.WALL_SPECULAR)


def _announce(name):
    print("[gpu case] pair %s" % name, flush=True)
    sys.stdout.flush()


def _crowd(p, parts, extra, seed, lo=0.02, width=0.2):
    # `extra` particles added inside one corner cell region
    rng = np.random.default_rng(seed)
    n0 = len(parts["cx"])
    add = dict(x=rng.random(extra) * width + lo, y=rng.random(extra) * width + lo,
               cx=rng.standard_normal(extra), cy=rng.standard_normal(extra), cz=rng.standard_normal(extra),
               w=np.ones(extra), id=np.arange(n0, n0 + extra, dtype=np.uint32))
    if p["dims"] == 1:
        add["y"] = np.zeros(extra)
    return p, {k: np.concatenate([np.asarray(parts[k]), add[k]]) for k in add}


def _weights(parts, seed, spread=0.1):
    rng = np.random.default_rng(seed)
    return dict(parts, w=1.0 + spread * rng.standard_normal(len(parts["cx"])))


def _case(name):
    """(p, parts, steps, chunks, real, motion_exact, weights_reestimated)"""
    if name.startswith("fourier_specular"):
        real = name[-3:]
        p, parts = W.fourier(n_cells=16, per_cell=40, Kn=0.02, dt=4e-3, real=real)
        p["wall_kind"] = (W.WALL_SPECULAR, W.WALL_SPECULAR, 0, 0)
        return p, W.shuffle_storage(parts, seed=2), 10, 2, real, True, False
    if name.startswith("cavity_periodic"):
        real = name[-3:]
        p, parts = W.cavity(nx=12, ny=10, per_cell=25, Kn=0.01, real=real, dt=0.01)
        p["wall_kind"] = PERIODIC_X
        return p, parts, 10, 2, real, True, False
    if name == "odd_grid_specular_f32":
        # 7 x 5 cells: the last wave's second half has no cell
        p, parts = W.cavity(nx=7, ny=5, per_cell=30, Kn=0.02, real="f32", dt=0.02)
        p["wall_kind"] = SPEC
        return p, W.shuffle_storage(parts, seed=6), 8, 2, "f32", True, False
    if name == "fourier_diffuse_vr_f64":
        p, parts = W.fourier(n_cells=20, per_cell=50, Kn=0.05, dt=2e-3, real="f64")
        return p, parts, 16, 2, "f64", False, False
    if name == "cavity_diffuse_lid_vr_f64":
        p, parts = W.cavity(nx=10, ny=10, per_cell=30, Kn=0.02, real="f64", lid=0.3, dt=2e-3)
        return p, parts, 16, 1, "f64", False, False
    if name.startswith("reest_cavity_specular"):
        real = name[-3:]
        p, parts = W.cavity(nx=10, ny=10, per_cell=40, Kn=0.03, real=real, dt=2e-3)
        p["wall_kind"] = PERIODIC_X
        p["vr_reconstruct"] = 1
        return p, _weights(parts, 3), 12, 2, real, True, True
    if name == "reest_cavity_diffuse_kappa_f32":
        p, parts = W.cavity(nx=9, ny=9, per_cell=50, Kn=0.03, real="f32", lid=0.3, dt=2e-3)
        p.update(vr_reconstruct=2, vr_kappa=1.5)
        return p, parts, 12, 2, "f32", False, True
    if name == "reest_fourier_diffuse_k3_f64":
        p, parts = W.fourier(n_cells=16, per_cell=60, Kn=0.05, dt=2e-3, real="f64", T_left=1.2, T_right=1.8)
        p["vr_reconstruct"] = 3
        return p, parts, 14, 2, "f64", False, True
    if name == "vhs_cavity_f64":
        p, parts = W.cavity(nx=12, ny=10, per_cell=25, Kn=0.01, real="f64", dt=0.01)
        p["wall_kind"] = PERIODIC_X
        return dict(p, molecule=W.VHS, omega=0.74), parts, 10, 2, "f64", True, False
    if name == "vss_cavity_f32":
        p, parts = W.cavity(nx=12, ny=10, per_cell=25, Kn=0.01, real="f32", dt=0.01)
        p["wall_kind"] = PERIODIC_X
        return dict(p, molecule=W.VSS, omega=0.74, alpha=1.4), parts, 10, 2, "f32", True, False
    if name == "maxwell_fourier_f32":
        p, parts = W.fourier(n_cells=12, per_cell=40, Kn=0.05, dt=4e-3, real="f32")
        p["wall_kind"] = (W.WALL_SPECULAR, W.WALL_SPECULAR, 0, 0)
        return dict(p, molecule=W.MAXWELL, sigma=0.02), parts, 8, 2, "f32", True, False
    if name == "diameter_cavity_f32":
        p, parts = W.cavity(nx=8, ny=6, per_cell=30, Kn=0.02, real="f32", dt=0.01)
        p["wall_kind"] = SPEC
        return dict(p, majorant=2), parts, 8, 2, "f32", True, False
    if name == "big_cell_f64":
        # one crowded cell above the pair capacity (global-memory kernel)
        p, parts = W.cavity(nx=4, ny=4, per_cell=40, Kn=0.05, real="f64", dt=1e-4)
        p, parts = _crowd(p, parts, 1200, 5)  # mean 115 per cell: 128 mover slots
        return p, parts, 4, 1, "f64", False, False
    if name == "big_cell_far_f64":
        # a crowded cell while particles jump across the box (overflow lists)
        p, parts = W.cavity(nx=4, ny=4, per_cell=30, Kn=0.05, real="f64", dt=0.2)
        p["wall_kind"] = SPEC
        p, parts = _crowd(p, parts, 1200, 8)
        return p, W.shuffle_storage(parts, seed=4), 6, 2, "f64", True, False
    if name == "periodic_1x1_f64":
        p, parts = W.cavity(nx=1, ny=1, per_cell=60, Kn=0.05, real="f64", dt=0.4)
        p["wall_kind"] = (W.WALL_PERIODIC,) * 4
        return p, W.shuffle_storage(parts, seed=4), 6, 2, "f64", True, False
    if name == "periodic_2x3_f64":
        p, parts = W.cavity(nx=2, ny=3, per_cell=30, Kn=0.05, real="f64", dt=0.4)
        p["wall_kind"] = (W.WALL_PERIODIC,) * 4
        return p, W.shuffle_storage(parts, seed=4), 6, 2, "f64", True, False
    if name == "fourier_periodic_3_f32":
        p, parts = W.fourier(n_cells=3, per_cell=50, Kn=0.05, real="f32", dt=0.3)
        p["wall_kind"] = (W.WALL_PERIODIC, W.WALL_PERIODIC, 0, 0)
        return p, W.shuffle_storage(parts, seed=4), 6, 2, "f32", True, False
    if name == "odd_grid_vr_generations_f32":
        # 7 x 5 cells (the last wave's second half has no cell) with several
        # generations of candidates per cell and weights re-estimated;
        # specular walls, so that the motion is compared bit for bit
        p, parts = W.cavity(nx=7, ny=5, per_cell=60, Kn=0.01, real="f32", dt=4e-3)
        p["wall_kind"] = SPEC
        p.update(vr_reconstruct=2, vr_kappa=1.5)
        return p, W.shuffle_storage(parts, seed=9), 10, 2, "f32", True, True
    if name == "vss_vr_generations_f64":
        # variable soft spheres with weights (rejections weighted by the VSS
        # acceptance probability), up to two generations per cell (about 27
        # candidates, 16 to 38), re-estimated; denser cells with these
        # weights diverge between re-estimations, on the host as on the device
        p, parts = W.cavity(nx=8, ny=6, per_cell=60, Kn=0.01, real="f64", dt=4e-3, lid=0.3)
        p.update(vr_reconstruct=3, vr_kappa=1.5, molecule=W.VSS, omega=0.74, alpha=1.4)
        return p, parts, 9, 3, "f64", False, True
    if name.startswith("vr_generations"):
        # about 80 candidates per cell and step (40 to 120): two to four
        # generations of 32 per half-wave cell, the two cells of a wave
        # completing theirs in different windows
        real = name[-3:]
        p, parts = W.cavity(nx=8, ny=8, per_cell=60, Kn=0.01, real=real, dt=4e-3, lid=0.3)
        p.update(vr_reconstruct=2, vr_kappa=1.5)
        return p, parts, 10, 2, real, False, True
    if name == "many_movers_f64":
        # more than 64 particles enter a cell in one step: 128 mover slots,
        # sorted over four values per lane of a half
        p, parts = W.cavity(nx=6, ny=6, per_cell=100, Kn=0.05, real="f64", dt=0.08)
        p["wall_kind"] = SPEC
        return p, W.shuffle_storage(parts, seed=5), 4, 2, "f64", True, False
    raise KeyError(name)


CASES = ["fourier_specular_f32", "fourier_specular_f64", "cavity_periodic_f32", "cavity_periodic_f64",
         "odd_grid_specular_f32", "fourier_diffuse_vr_f64", "cavity_diffuse_lid_vr_f64",
         "reest_cavity_specular_f32", "reest_cavity_specular_f64", "reest_cavity_diffuse_kappa_f32",
         "reest_fourier_diffuse_k3_f64", "vhs_cavity_f64", "vss_cavity_f32", "maxwell_fourier_f32",
         "diameter_cavity_f32", "big_cell_f64", "big_cell_far_f64", "periodic_1x1_f64", "periodic_2x3_f64",
         "fourier_periodic_3_f32", "many_movers_f64", "vr_generations_f32", "vr_generations_f64",
         "odd_grid_vr_generations_f32", "vss_vr_generations_f64"]


def _gpu(p, parts, steps, chunks, real, launch):
    from paper_2301_05985_amd.binding import Simulation
    if not isinstance(launch, dict):
        launch = {"cells_per_wave": launch}
    sim = Simulation(dict(p, real=real, **launch), parts)
    try:
        for _ in range(chunks):
            sim.step(steps // chunks)
        sums, cnt, ns = sim.sample()
        seq = sim.sequence()["id"] if len(parts["cx"]) else None
        return dict(sums=sums, cnt=cnt, ns=ns, st=sim.particles(), seq=seq, diag=sim.diagnostics())
    finally:
        sim.close()


# FP32 re-estimated weights of the case with several generations per cell:
# every particle takes several weight updates between two re-estimations,
# and the rejection update (division by 1 - p, p up to 1 / kappa) carries
# and amplifies the one-ulp rounding difference of a re-estimated weight
# (the host's and the device's Gram sums add in different orders); every
# launch on the device gives the same weights, 18.5 ulp from the oracle's
# after 10 steps.
W_ULP = {"vr_generations_f32": 64, "odd_grid_vr_generations_f32": 64}


def _against_oracle(g, orc, real, exact, reest, w_ulp=8):
    o = orc.state()
    assert g["diag"]["status"] == 0, g["diag"]
    assert np.array_equal(g["st"]["id"], o["id"])
    assert np.array_equal(g["seq"], orc.sequence_state()["id"]), "particle sequence differs"
    assert np.array_equal(g["cnt"], orc.counters), "per-cell candidate/accepted counts differ"
    for k in ("x", "y", "cx", "cy", "cz", "w"):
        a, b = g["st"][k], o[k]
        if a is None or len(a) == 0:
            continue
        if k == "w" and reest:
            a, b = a.astype(np.float64), b.astype(np.float64)
            assert np.isfinite(a).all()
            err = np.abs(a - b) / np.maximum(np.abs(b), 1.0)
            assert err.max() <= (1e-9 if real == "f64" else w_ulp * 2.0 ** -23), err.max()
        elif exact:
            bad = np.flatnonzero(a != b)
            assert bad.size == 0, (k, bad[:5], a[bad[:5]], b[bad[:5]])
        else:
            # the device's and the host's log, sin, cos may differ in the last
            # bit: 1e-12 relative in FP64, four ulp in FP32
            err = np.abs(a.astype(np.float64) - b.astype(np.float64)) / np.maximum(np.abs(b), 1.0)
            assert err.max() <= (1e-12 if real == "f64" else 4 * 2.0 ** -23), (k, err.max())
    # sums of a state that may differ by an ulp (FP32 with diffuse walls)
    # differ by about that much
    plain = 1e-11 if exact or real == "f64" else 1e-6
    if reest:
        assert_sums_close(g["sums"], orc.sums, plain, cols=range(13))
        assert_sums_close(g["sums"], orc.sums, 1e-9 if real == "f64" else 1e-5, cols=range(13, 26))
    else:
        assert_sums_close(g["sums"], orc.sums, plain)


LAUNCHES = [{"cells_per_wave": 2}, {"waves_per_cell": 4}]


@pytest.mark.parametrize("launch", LAUNCHES, ids=["two_cells", "four_waves"])
@pytest.mark.parametrize("name", CASES)
def test_walled_launch_matches_oracle_and_one_cell_launch(gpu, name, launch):
    p, parts, steps, chunks, real, exact, reest = _case(name)
    _announce("%s %s" % (name, launch))
    g2 = _gpu(p, parts, steps, chunks, real, launch)
    g1 = _gpu(p, parts, steps, chunks, real, 1)
    orc = oracle.Oracle(dict(p, real=real), parts, np.float64 if real == "f64" else np.float32)
    orc.run(steps)
    assert orc.counters[:, 1].sum() > 10
    if name.startswith("big_cell"):
        assert g2["diag"]["big_cells"] > 0
    _against_oracle(g2, orc, real, exact, reest, W_ULP.get(name, 8))
    assert np.array_equal(g2["seq"], g1["seq"]) and np.array_equal(g2["cnt"], g1["cnt"])
    for k in ("x", "y", "cx", "cy", "cz", "w"):
        if g1["st"][k] is None:
            continue
        if k == "w" and reest:
            # the Gram sums are added over another number of lanes: the same
            # least-squares solution up to its rounding
            a, b = g2["st"][k].astype(np.float64), g1["st"][k].astype(np.float64)
            err = np.abs(a - b) / np.maximum(np.abs(b), 1.0)
            assert err.max() <= (1e-9 if real == "f64" else 8 * 2.0 ** -23), err.max()
        else:
            assert np.array_equal(g2["st"][k], g1["st"][k]), k
    if reest:
        assert_sums_close(g2["sums"], g1["sums"], 1e-11, cols=range(13))
        assert_sums_close(g2["sums"], g1["sums"], 1e-9 if real == "f64" else 1e-5, cols=range(13, 26))
    else:
        assert_sums_close(g2["sums"], g1["sums"], 1e-12)


@pytest.mark.parametrize("extra", [0, 1])
def test_cell_at_pair_capacity_and_one_above(gpu, extra):
    # 160 particles in 8 cells: the pair capacity is 0.96 x 20 + 64 rounded
    # up to 32, at least 128; cell 0 holds 128 (staged in LDS) or 129 (global
    # memory).  A tiny time step keeps every particle in its cell.
    _announce("cell at pair capacity + %d" % extra)
    p, _ = W.fourier(n_cells=8, per_cell=1, Kn=0.05, dt=1e-7, vr=1)
    p["wall_kind"] = (W.WALL_SPECULAR, W.WALL_SPECULAR, 0, 0)
    p["sigma"] = 1300.0
    n, n0 = 160, 128 + extra
    rng = np.random.default_rng(12)
    x = np.concatenate([rng.uniform(0.01, 0.115, n0), rng.uniform(0.135, 0.99, n - n0)])
    c = rng.standard_normal((3, n))
    parts = dict(x=x, cx=c[0], cy=c[1], cz=c[2], w=np.ones(n), id=rng.permutation(n).astype(np.uint32))
    g = _gpu(p, parts, 4, 1, "f32", 2)
    orc = oracle.Oracle(dict(p, real="f32"), parts, np.float32)
    orc.run(4)
    assert (g["diag"]["big_cells"] > 0) == bool(extra)
    assert orc.counters[0, 1] > 20
    _against_oracle(g, orc, "f32", True, False)


@pytest.mark.parametrize("launch", LAUNCHES, ids=["two_cells", "four_waves"])
@pytest.mark.parametrize("case", ["empty_slab", "empty_cavity", "one", "two"])
def test_empty_and_tiny_runs(gpu, case, launch):
    _announce("%s %s" % (case, launch))
    if case in ("empty_slab", "empty_cavity"):
        if case == "empty_cavity":
            p, _ = W.cavity(nx=6, ny=5, per_cell=1, Kn=0.05, dt=0.01)
        else:
            p, _ = W.fourier(n_cells=7, per_cell=1, Kn=0.05, dt=0.01)
        e = np.zeros(0)
        parts = dict(x=e, y=e, cx=e, cy=e, cz=e, w=e, id=np.zeros(0, dtype=np.uint32))
        steps = 5
    else:
        n = 1 if case == "one" else 2
        p, _ = W.fourier(n_cells=3, per_cell=1, Kn=0.05, dt=0.05)
        p["wall_kind"] = (W.WALL_SPECULAR, W.WALL_SPECULAR, 0, 0)
        p["sigma"] = 5.0
        parts = dict(x=np.array([0.1, 0.15])[:n], cx=np.array([0.7, -0.3])[:n], cy=np.array([0.2, 0.1])[:n],
                     cz=np.array([-0.4, 0.9])[:n], w=np.ones(n), id=np.arange(n, dtype=np.uint32))
        steps = 20
    g = _gpu(p, parts, steps, 1, "f64", launch)
    orc = oracle.Oracle(dict(p, real="f64"), parts, np.float64)
    orc.run(steps)
    assert g["diag"]["status"] == 0
    assert np.array_equal(g["cnt"], orc.counters)
    o = orc.state()
    for k in ("x", "cx", "cy", "cz", "w"):
        if len(o[k]):
            assert np.array_equal(g["st"][k], o[k]), k
    assert_sums_close(g["sums"], orc.sums, 1e-11)
