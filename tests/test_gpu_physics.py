"""Physics of the GPU path at a size the oracle cannot reach in a test: the
hard-sphere thermal conductivity of a near-continuum Fourier flow against the
Chapman-Enskog value (second Sonine approximation, Chapman & Cowling), with
the cell-size correction of Alexander, Garcia & Alder (1998).  Parity with
the oracle is tested elsewhere; this pins the law the kernels produce."""
import math

import numpy as np
import pytest

import oracle
from paper_2301_05985_amd import workloads as W

pytestmark = pytest.mark.gpu


def test_fourier_conductivity_matches_chapman_enskog(gpu):
    print("[gpu case] fourier conductivity", flush=True)
    from paper_2301_05985_amd.binding import Simulation
    n_cells, per_cell, Kn, dt = 400, 100, 0.01, 5e-4
    burn, nsamp = 48000, 40000
    # walls at T = 1 and 2, no weights; lambda = 0.01 at the mean density,
    # cells of lambda / 4, about 0.1 mean collision times per step
    p, parts = W.fourier(n_cells=n_cells, per_cell=per_cell, Kn=Kn, dt=dt, real="f32", vr=0)
    sigma = p["sigma"]
    sim = Simulation(p, parts)
    sim.step(burn)
    sim.sample(reset=True)
    sim.step(nsamp)
    sums, cnt, ns = sim.sample()
    d = sim.diagnostics()
    sim.close()
    assert d["status"] == 0 and ns == nsamp
    dx = 1.0 / n_cells
    est = oracle.estimators(sums, ns, p["FN"], dx)
    T, q, n = est["T"], est["q"][:, 0], est["n"]
    x = (np.arange(n_cells) + 0.5) * dx
    inner = slice(n_cells // 5, 4 * n_cells // 5)  # away from the Knudsen layers
    # steady 1-D conduction: q is uniform, and with k = k0 sqrt(T),
    # q = -(2/3) k0 d(T^1.5)/dx
    qm = q[inner].mean()
    slope = np.polyfit(x[inner], T[inner] ** 1.5, 1)[0]
    k0_meas = -1.5 * qm / slope
    # Chapman-Enskog, hard spheres of cross-section sigma = pi d^2 (k = m = 1):
    # k = 1.025 (75/64) (1/d^2) sqrt(T/pi) = 1.025 (75/64) sqrt(pi) sqrt(T) / sigma
    k0_ce = 1.025 * (75.0 / 64.0) * math.sqrt(math.pi) / sigma
    # finite cells: k(dx) = k (1 + (32/225) (dx/lambda)^2), local lambda
    lam = 1.0 / (math.sqrt(2.0) * n[inner] * sigma)
    corr = 1.0 + (32.0 / 225.0) * float(((dx / lam) ** 2).mean())
    ratio = k0_meas / (k0_ce * corr)
    print("[gpu case] conductivity ratio %.4f (cell correction %.4f, q %.1f)" % (ratio, corr, qm), flush=True)
    assert qm < 0.0  # heat flows from the hot wall (x = 1) to the cold one
    # about 0.98 over seeds, 25-400 particles per cell, precisions and time
    # steps (slow thermal modes make single runs scatter by 0.4-2%): the
    # bound is a 5% check of the law, not a convergence study
    assert abs(ratio - 1.0) < 0.05
