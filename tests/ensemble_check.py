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


def ensemble_mean_shift(x, mean, std, R, k_sigma=4.0):
    """Aggregate check for independent cells: the mean of z over the cells,
    per estimator (columns of x), has expectation 0 and standard error
    sqrt(((R - 1) / (R - 3)) / M) (the variance of Student's t with R - 1
    degrees of freedom over M cells).  Passes when every column's mean is
    within k_sigma standard errors; sensitive to a small shift common to all
    cells, which the per-cell 3-sigma fraction does not see."""
    z = ensemble_z(x, mean, std, R)
    z = z.reshape(z.shape[0], -1)
    out = []
    for k in range(z.shape[1]):
        zk = z[:, k][np.isfinite(z[:, k])]
        se = np.sqrt((R - 1.0) / (R - 3.0) / zk.size)
        out.append(float(zk.mean() / se))
    return all(abs(v) <= k_sigma for v in out), out

