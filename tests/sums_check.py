"""Comparison of running moment sums taken in different summation orders.

Per cell: the particle count (sum 0) is an integer and must match exactly;
every other sum may differ by rounding, which is bounded by the number of
terms times the largest term, both at most the largest sum of the same cell
(the count, the energy sums or the third moments).  So each sum is compared
against rtol times (that cell's largest |sum| + 1): for a small or nearly
empty cell this is far tighter than a scale shared by all cells."""
import numpy as np


def assert_sums_close(s_gpu, s_ref, rtol=1e-11, cols=None, scale_cols=None):
    """s_*: [n_cells][26] FP64 running sums.  cols: the sums compared (all by
    default); scale_cols: the sums whose largest magnitude per cell sets the
    scale (the plain moments 0-12 by default)."""
    s_gpu = np.asarray(s_gpu, dtype=np.float64)
    s_ref = np.asarray(s_ref, dtype=np.float64)
    ok = np.isfinite(s_ref)
    assert np.array_equal(ok, np.isfinite(s_gpu)), "non-finite sums differ"
    s_gpu = np.where(ok, s_gpu, 0.0)
    s_ref = np.where(ok, s_ref, 0.0)
    cols = list(range(s_ref.shape[1])) if cols is None else list(cols)
    scale_cols = list(range(min(13, s_ref.shape[1]))) if scale_cols is None else list(scale_cols)
    if 0 in cols:
        bad = np.flatnonzero(s_gpu[:, 0] != s_ref[:, 0])
        assert bad.size == 0, ("particle counts differ", bad[:5])
    scale = np.abs(s_ref[:, scale_cols]).max(axis=1, keepdims=True) + 1.0
    err = np.abs(s_gpu[:, cols] - s_ref[:, cols]) / scale
    worst = np.unravel_index(int(np.argmax(err)), err.shape) if err.size else None
    assert err.size == 0 or err.max() < rtol, ("sums differ", float(err.max()), worst)
