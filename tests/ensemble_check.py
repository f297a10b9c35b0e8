"""Ensemble agreement test for stochastic results (used by CPU and GPU tests).

Given R independent oracle realisations of a cell estimator (mean m, sample
standard deviation s) and one more realisation x from the path under test,
z = (x - m) / (s sqrt(1 + 1/R)) follows Student's t with R - 1 degrees of
freedom when x comes from the same distribution (Gaussian estimators).
The test passes when the fraction of |z| > 3 is at most its expectation
p3 = 2 P(t > 3) plus four binomial standard deviations, and the largest |z|
is below the Bonferroni bound of the t distribution at family level 1e-3.
"""
import numpy as np
from scipy import stats

ROOT_GOLDEN = "golden"


def ensemble_z(x, mean, std, R):
    return (x - mean) / (std * np.sqrt(1.0 + 1.0 / R))


def ensemble_verdict(x, mean, std, R, level=1e-3):
    z = ensemble_z(x, mean, std, R).ravel()
    z = z[np.isfinite(z)]
    M = z.size
    p3 = 2.0 * stats.t.sf(3.0, R - 1)
    frac = float(np.mean(np.abs(z) > 3.0))
    frac_bound = p3 + 4.0 * np.sqrt(p3 * (1 - p3) / M)
    zmax = float(np.abs(z).max())
    zmax_bound = float(stats.t.isf(level / (2.0 * M), R - 1))
    ok = frac <= frac_bound and zmax <= zmax_bound
    return ok, dict(frac=frac, frac_bound=frac_bound, zmax=zmax, zmax_bound=zmax_bound, M=M)
