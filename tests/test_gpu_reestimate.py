"""GPU parity of the importance-weight re-estimation and of the majorant
factor of weighted runs, through the C ABI, against the CPU oracle.

Bar: the motion never depends on the weights, so positions, velocities,
pair choices and counts keep the parity bar of the other tests (bit-exact in
FP32 without transcendental functions, 1e-12 relative in FP64).  The
re-estimated weights solve the same least-squares problem in another order
of summation and elimination (Gauss-Jordan on the GPU, Cholesky in the
oracle): in FP64 they agree within 1e-9 of max(|W|, 1) after a few steps
(the differences are a few times the solve's rounding, cond(G) x 1e-16,
carried along by later collisions); in FP32 almost every weight rounds to
the same float and none differs by more than a few ulp.  The weighted sums
are compared relative to the scale of their terms.
"""
import sys

import numpy as np
import pytest

import oracle
from paper_2301_05985_amd import workloads as W
from tests.sums_check import assert_sums_close

pytestmark = pytest.mark.gpu


def _announce(name):
    print("[gpu case] %s" % name, flush=True)
    sys.stdout.flush()


def _run(p, parts, steps, real, chunks=1):
    from paper_2301_05985_amd.binding import Simulation
    p = dict(p, real=real)
    dtype = np.float64 if real == "f64" else np.float32
    sim = Simulation(p, parts)
    orc = oracle.Oracle(p, parts, dtype)
    for _ in range(chunks):
        sim.step(steps // chunks)
        orc.run(steps // chunks)
    sums, cnt, ns = sim.sample()
    out = dict(sums=sums, cnt=cnt, st=sim.particles(), diag=sim.diagnostics())
    if orc.layout is not None:
        out["seq"] = sim.sequence()["id"]
    sim.close()
    return out, orc


def _check(g, orc, real, motion_exact):
    o = orc.state()
    assert g["diag"]["status"] == 0, g["diag"]
    assert np.array_equal(g["st"]["id"], o["id"])
    if orc.layout is not None:
        assert np.array_equal(g["seq"], orc.sequence_state()["id"]), "particle sequence differs"
    assert np.array_equal(g["cnt"], orc.counters), "per-cell candidate/accepted counts differ"
    for k in ("x", "y", "cx", "cy", "cz"):
        a, b = g["st"][k], o[k]
        if motion_exact:
            assert np.array_equal(a, b), k
        else:
            err = np.abs(a.astype(np.float64) - b) / np.maximum(np.abs(b), 1.0)
            assert err.max() <= 1e-12, (k, err.max())
    a, b = g["st"]["w"].astype(np.float64), o["w"].astype(np.float64)
    assert np.isfinite(a).all() and np.isfinite(b).all()
    err = np.abs(a - b) / np.maximum(np.abs(b), 1.0)
    if real == "f64":
        assert err.max() <= 1e-9, err.max()
    else:
        assert err.max() <= 8 * 2.0 ** -23, err.max()
        assert np.mean(a == b) >= 0.99
    # sums: plain ones as in the other parity tests; weighted ones carry the
    # weights' tolerance, against the same per-cell scale
    assert_sums_close(g["sums"], orc.sums, 1e-11, cols=range(13))
    assert_sums_close(g["sums"], orc.sums, 1e-9 if real == "f64" else 1e-5, cols=range(13, 26))


def _weights(n, seed, spread=0.05):
    rng = np.random.default_rng(seed)
    return 1.0 + spread * rng.standard_normal(n)


def test_reestimate_cavity_diffuse_lid_f64(gpu):
    # one-wave cells staged in LDS; a fast lid makes the weights deviate
    _announce("re-estimation cavity diffuse f64")
    p, parts = W.cavity(nx=10, ny=10, per_cell=40, Kn=0.03, real="f64", lid=0.3, dt=2e-3)
    p["vr_reconstruct"] = 1
    g, orc = _run(p, parts, 12, "f64", chunks=2)
    assert orc.diag.wall_hits > 0 and orc.counters[:, 1].sum() > 100
    assert np.abs(orc.state()["w"] - 1).max() > 1e-3  # the weights did move
    _check(g, orc, "f64", motion_exact=False)


@pytest.mark.parametrize("real", ["f64", "f32"])
def test_reestimate_cavity_specular_perturbed_weights(gpu, real):
    # walls without transcendental functions (periodic in x, specular in y),
    # so the motion is bit-exact in both precisions; the weights start
    # perturbed
    _announce("re-estimation cavity specular %s" % real)
    p, parts = W.cavity(nx=10, ny=10, per_cell=40, Kn=0.03, real=real, dt=2e-3)
    p["wall_kind"] = (W.WALL_PERIODIC, W.WALL_PERIODIC, W.WALL_SPECULAR, W.WALL_SPECULAR)
    p["vr_reconstruct"] = 1
    parts = dict(parts, w=_weights(len(parts["cx"]), 3, spread=0.1))
    g, orc = _run(p, parts, 12, real, chunks=2)
    assert orc.counters[:, 1].sum() > 100
    _check(g, orc, real, motion_exact=True)


def test_reestimate_fourier_diffuse_every_third_step_f64(gpu):
    _announce("re-estimation fourier K=3 f64")
    p, parts = W.fourier(n_cells=16, per_cell=60, Kn=0.05, dt=2e-3, real="f64", T_left=1.2, T_right=1.8)
    p["vr_reconstruct"] = 3
    g, orc = _run(p, parts, 14, "f64", chunks=2)
    _check(g, orc, "f64", motion_exact=False)


def test_reestimate_fourier_specular_every_third_step_f32(gpu):
    _announce("re-estimation fourier K=3 specular f32")
    p, parts = W.fourier(n_cells=16, per_cell=60, Kn=0.05, dt=2e-3, real="f32")
    p["wall_kind"] = (W.WALL_SPECULAR, W.WALL_SPECULAR, 0, 0)
    p["vr_reconstruct"] = 3
    parts = dict(parts, w=_weights(len(parts["cx"]), 8, spread=0.1))
    g, orc = _run(p, parts, 14, "f32", chunks=2)
    _check(g, orc, "f32", motion_exact=True)


@pytest.mark.parametrize("real", ["f64", "f32"])
def test_reestimate_homogeneous_wave_workgroup_and_global_cells(gpu, real):
    # one-wave cells, four-wave workgroup cells (above 1024 particles) and a
    # cell above the LDS capacity (global-memory kernel); below 26 particles
    # a cell keeps its weights
    _announce("re-estimation homogeneous %s" % real)
    counts = [70, 1300, 25, 26, 2, 600, 1100, 4500]
    rng = np.random.default_rng(4)
    off = np.zeros(len(counts) + 1, dtype=np.int64)
    off[1:] = np.cumsum(counts)
    c = rng.standard_normal((3, int(off[-1])))
    c[0, ::2] += 1.0
    # volumes proportional to the counts: about 0.4 candidates per particle
    # and step in every cell
    p = dict(dims=0, n_cells=(len(counts), 1), dt=0.05, sigma=0.002, FN=1.0, seed=23, inst_offset=off,
             cell_volume=np.array(counts, dtype=np.float64) / 1000.0 + 1e-3, vr=1, vr_T0=1.0,
             vr_reconstruct=1)
    parts = dict(cx=c[0], cy=c[1], cz=c[2], id=np.arange(int(off[-1]), dtype=np.uint32),
                 w=_weights(int(off[-1]), 5))
    g, orc = _run(p, parts, 6, real, chunks=2)
    assert g["diag"]["big_cells"] > 0
    _check(g, orc, real, motion_exact=True)


@pytest.mark.parametrize("real", ["f64", "f32"])
def test_majorant_factor_bit_exact(gpu, real):
    # weighted runs with the majorant scaled by 1.5: the candidate counts
    # grow, acceptance probabilities shrink; state exact where no
    # transcendental function enters (specular walls)
    _announce("majorant factor %s" % real)
    p, parts = W.fourier(n_cells=16, per_cell=40, Kn=0.02, dt=4e-3, real=real)
    p["wall_kind"] = (W.WALL_SPECULAR, W.WALL_SPECULAR, 0, 0)
    parts = dict(parts, w=_weights(len(parts["cx"]), 9))
    p["vr_kappa"] = 1.5
    g, orc = _run(p, parts, 8, real, chunks=2)
    assert g["cnt"][:, 0].sum() > 0
    o = orc.state()
    assert np.array_equal(g["cnt"], orc.counters)
    for k in ("x", "cx", "cy", "cz", "w"):
        assert np.array_equal(g["st"][k], o[k]), k


def test_reestimated_cavity_weights_stay_finite(gpu):
    # the cavity at the full-size benchmark's resolution per cell (64 x 64
    # cells of 100, mean free path 2.56 cells, about 0.13 collisions per
    # particle and step): without re-estimation the weighted sums turn
    # non-finite within 300 steps; with it the weights stay within a few
    # percent of 1 over 3000 steps
    from paper_2301_05985_amd.binding import Simulation
    _announce("re-estimation cavity 64x64 3000 steps")
    res = {}
    for K, steps in ((0, 300), (1, 3000)):
        p, parts = W.cavity(nx=64, ny=64, per_cell=100, Kn=0.04, real="f32")
        p["vr_reconstruct"] = K
        sim = Simulation(p, parts)
        sim.step(steps)
        d = sim.diagnostics()
        w = sim.particles()["w"].astype(np.float64)
        res[K] = (d["vr_nonfinite"], float(np.sqrt(np.mean((w - 1) ** 2))), d["status"])
        sim.close()
    assert res[0][0] > 0, res
    assert res[1][0] == 0 and res[1][1] < 0.01 and res[1][2] == 0, res


@pytest.mark.parametrize("real", ["f32", "f64"])
def test_learned_majorant_walled_weights_reestimated(gpu, real):
    # walled cells with the learned majorant (verified proposal or exact
    # fallback), weights re-estimated every second step and the majorant
    # factor 1.5; a crowded corner cell runs on the global-memory learned
    # kernel; walls without transcendental functions keep the motion
    # bit-exact
    from oracle import mlp_oracle as M
    from paper_2301_05985_amd.binding import Simulation
    _announce("learned majorant, walled, weights re-estimated %s" % real)
    dtype = np.float64 if real == "f64" else np.float32
    p, parts = W.cavity(nx=10, ny=10, per_cell=40, Kn=0.03, real=real, dt=2e-3)
    p["wall_kind"] = (W.WALL_PERIODIC, W.WALL_PERIODIC, W.WALL_SPECULAR, W.WALL_SPECULAR)
    p.update(vr_reconstruct=2, vr_kappa=1.5)
    n = len(parts["cx"])
    x, y = parts["x"].copy(), parts["y"].copy()
    x[:230] *= 0.1  # 230 more particles in cell (0, 0): above its LDS capacity
    y[:230] *= 0.1
    parts = dict(parts, x=x, y=y, w=_weights(n, 5, spread=0.1))
    net = M.init_params(7) * 0.05
    net[-1] = 2.5  # log2 of a typical cell's largest pair speed
    bits = M.to_bf16(net.astype(np.float32))
    delta = 0.01
    orc = oracle.Oracle(dict(p, majorant=1, mlp=M.from_bf16(bits).astype(np.float32), mlp_delta=delta), parts,
                        dtype)
    log = orc.run(8, learned_log=True)
    assert (log == 1).any() and (log == -1).any() and (log == 0).any(), np.unique(log, return_counts=True)
    sim = Simulation(dict(p, majorant=1), parts)
    sim.set_majorant_model(bits, delta, 0)
    sim.step(8)
    sums, cnt, _ = sim.sample()
    g = dict(sums=sums, cnt=cnt, st=sim.particles(), diag=sim.diagnostics(), seq=sim.sequence()["id"])
    sim.close()
    assert g["diag"]["big_cells"] > 0
    assert g["diag"]["learned_used"] == (log == 1).sum()
    assert g["diag"]["fallback"] == (log == -1).sum()
    assert g["diag"]["learned_skip"] == (log == 0).sum()
    _check(g, orc, real, motion_exact=True)
