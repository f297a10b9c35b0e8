"""Write the oracle ensemble statistics used by the ensemble tests.

Calls only the CPU oracle (its double-precision build) and the seeded input
generator.  Every member starts from the same initial state (input seed 0)
and differs in the Philox key (seeds 1..R).  Each ensemble file holds, per
cell (or instance) and estimator, the ensemble mean and standard deviation
(ddof = 1) and R.

  cavity32     reduced lid-driven cavity: 32 x 32 cells, 50 particles per
               cell, Kn = 0.05, lid speed 0.2, no importance weights; after
               BURN steps the plain cell estimators (density, u_x, u_y,
               temperature, P_xy, q_x, q_y) of SAMPLE steps
  cavity32vr   32 x 32 cells of 100, Kn = 0.1, lid 0.05, importance weights
               re-estimated every 4 steps, majorant factor 1.5 (without it the
               rare rejections with p near 1 give the weighted estimators
               heavy tails that a 3-sigma test cannot describe); the
               weighted (variance-reduced) estimators of the same seven
               quantities
  batched256   256 homogeneous cells, N uniform in [50, 400], bimodal
               initial states (shift in [0.5, 2]), exact majorant; over the
               first SAMPLE_B steps the time-averaged P_xx / p - 1,
               (P_yy - P_zz) / p, P_xy / p and q_x / p^(3/2) of each cell
               (density, velocity and temperature are conserved exactly)

Usage: python tests/golden/make_ensemble.py [R]
"""
import os
import sys
from multiprocessing import Pool

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_2301_05985_amd import workloads as W  # noqa: E402

NX = 32
PER = 50
KN = 0.05
LID = 0.2
BURN = 100
SAMPLE = 200
# weighted cavity
PER_VR = 100
KN_VR = 0.1
LID_VR = 0.05
KAPPA_VR = 1.5  # majorant factor: 1 / (1 - p) <= 3 in the weight update
REEST_VR = 4    # weights re-estimated every 4 steps (the full-size benchmark's setting)
# batched homogeneous cells
NB = 256
NMIN, NMAX = 50, 400
SAMPLE_B = 200


def params(seed):
    return W.cavity(nx=NX, ny=NX, per_cell=PER, Kn=KN, lid=LID, real="f32", vr=0, seed=seed, init_seed=0)


def params_vr(seed):
    p, parts = W.cavity(nx=NX, ny=NX, per_cell=PER_VR, Kn=KN_VR, lid=LID_VR, real="f32", vr=1, seed=seed,
                        init_seed=0)
    p["vr_reconstruct"] = REEST_VR
    p["vr_kappa"] = KAPPA_VR
    return p, parts


def params_batched(seed):
    return W.batched(n_inst=NB, nmin=NMIN, nmax=NMAX, real="f32", seed=seed, init_seed=0)


def _seven(e):
    return np.stack([e["n"], e["u"][:, 0], e["u"][:, 1], e["T"], e["P"][:, 0, 1], e["q"][:, 0], e["q"][:, 1]], 1)


def estimates(sums, n_samples):
    return _seven(oracle.estimators(sums, n_samples, 1.0, 1.0 / (NX * NX)))


def estimates_vr(sums, n_samples, p):
    return _seven(oracle.estimators(sums, n_samples, 1.0, 1.0 / (NX * NX), vr=True, vr_n0=p["vr_n0"],
                                    vr_T0=p["vr_T0"]))


def estimates_batched(sums, n_samples):
    e = oracle.estimators(sums, n_samples, 1.0, 1.0)
    P = e["P"]
    pr = e["n"] * e["T"]
    return np.stack([P[:, 0, 0] / pr - 1.0, (P[:, 1, 1] - P[:, 2, 2]) / pr, P[:, 0, 1] / pr,
                     e["q"][:, 0] / pr ** 1.5], 1)


def member(seed):
    p, parts = params(seed)
    o = oracle.Oracle(p, parts, np.float64)
    o.run(BURN)
    o.reset_samples()
    o.run(SAMPLE)
    return estimates(o.sums, SAMPLE)


def member_vr(seed):
    p, parts = params_vr(seed)
    o = oracle.Oracle(p, parts, np.float64)
    o.run(BURN)
    o.reset_samples()
    o.run(SAMPLE)
    assert o.diag.vr_nonfinite == 0
    return estimates_vr(o.sums, SAMPLE, p)


def member_batched(seed):
    p, parts = params_batched(seed)
    o = oracle.Oracle(p, parts, np.float64)
    o.run(SAMPLE_B)
    return estimates_batched(o.sums, SAMPLE_B)


def _write(name, res, **meta):
    out = os.path.join(HERE, "ensemble_%s_f64.npz" % name)
    m = np.stack(res).astype(np.float64)
    np.savez_compressed(out, mean=m.mean(0), std=m.std(0, ddof=1), R=m.shape[0], **meta)
    print("wrote", out, m.shape, flush=True)


def main():
    R = int(sys.argv[1]) if len(sys.argv) > 1 else 32
    with Pool(min(8, os.cpu_count() or 1)) as pool:
        _write("cavity32", pool.map(member, range(1, R + 1)), nx=NX, per=PER, kn=KN, lid=LID, burn=BURN,
               sample=SAMPLE)
        _write("cavity32vr", pool.map(member_vr, range(1, R + 1)), nx=NX, per=PER_VR, kn=KN_VR, lid=LID_VR,
               kappa=KAPPA_VR, reest=REEST_VR, burn=BURN, sample=SAMPLE)
        _write("batched256", pool.map(member_batched, range(1, R + 1)), n=NB, nmin=NMIN, nmax=NMAX,
               sample=SAMPLE_B)


if __name__ == "__main__":
    main()
