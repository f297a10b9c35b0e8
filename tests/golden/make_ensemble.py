"""Write the oracle ensemble statistics used by the FP32 ensemble test.

Calls only the CPU oracle (and the seeded input generator).  Reduced lid-driven
cavity: 32 x 32 cells, 50 particles per cell, Kn = 0.05, lid speed 0.2, no
importance weights, FP32 oracle build; all members start from the same
initial state (input seed 0) and differ in the Philox key (seeds 1..R).
After BURN steps, moments are sampled for SAMPLE steps and reduced to the
plain cell estimators (density, u_x, u_y, temperature, P_xy, q_x, q_y).
Output: ensemble_cavity32.npz with the ensemble mean and standard deviation
(ddof = 1) of each estimator in each cell, and R.

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


def params(seed):
    p, parts = W.cavity(nx=NX, ny=NX, per_cell=PER, Kn=KN, lid=LID, real="f32", vr=0, seed=seed, init_seed=0)
    return p, parts


def estimates(sums, n_samples):
    V = 1.0 / (NX * NX)
    e = oracle.estimators(sums, n_samples, 1.0, V)
    return np.stack([e["n"], e["u"][:, 0], e["u"][:, 1], e["T"], e["P"][:, 0, 1], e["q"][:, 0], e["q"][:, 1]], 1)


def member(seed):
    p, parts = params(seed)
    o = oracle.Oracle(p, parts, np.float32)
    o.run(BURN)
    o.reset_samples()
    o.run(SAMPLE)
    return estimates(o.sums, SAMPLE)


def main():
    R = int(sys.argv[1]) if len(sys.argv) > 1 else 32
    with Pool(min(8, os.cpu_count() or 1)) as pool:
        res = pool.map(member, range(1, R + 1))
    out = os.path.join(HERE, "ensemble_cavity32.npz")
    m = np.stack(res).astype(np.float64)
    np.savez_compressed(out, mean=m.mean(0), std=m.std(0, ddof=1), R=R, nx=NX, per=PER, kn=KN, lid=LID,
                        burn=BURN, sample=SAMPLE)
    print("wrote", out, m.shape)


if __name__ == "__main__":
    main()
