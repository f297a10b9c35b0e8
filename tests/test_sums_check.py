"""The per-cell comparison of running sums (tests/sums_check.py) catches an
error in a small cell that a scale shared by all cells would hide, and
accepts rounding-level differences.  CPU only."""
import numpy as np
import pytest

from tests.sums_check import assert_sums_close


def _sums(rng, ncell=50):
    s = np.zeros((ncell, 26))
    n = rng.integers(0, 400, ncell).astype(np.float64)
    n[:5] = [0, 1, 2, 3, 4]  # empty and tiny cells
    s[:, 0] = n
    s[:, 1:13] = rng.standard_normal((ncell, 12)) * n[:, None]
    s[:, 13:] = rng.standard_normal((ncell, 13)) * 0.01 * n[:, None]
    return s


def test_rounding_level_differences_pass():
    rng = np.random.default_rng(1)
    s = _sums(rng)
    t = s * (1.0 + 1e-14 * rng.standard_normal(s.shape))
    t[:, 0] = s[:, 0]
    assert_sums_close(t, s, 1e-11)


def test_error_in_a_small_cell_is_caught():
    rng = np.random.default_rng(2)
    s = _sums(rng)
    t = s.copy()
    t[3, 4] += 1e-8  # a cell of 3 particles: negligible against the largest cell
    col_scale = np.abs(s).max(axis=0) + 1.0
    assert abs(t[3, 4] - s[3, 4]) / col_scale[4] < 1e-10  # a shared scale would pass it
    with pytest.raises(AssertionError):
        assert_sums_close(t, s, 1e-11)


def test_counts_must_match_exactly():
    rng = np.random.default_rng(3)
    s = _sums(rng)
    t = s.copy()
    t[10, 0] += 1.0
    with pytest.raises(AssertionError):
        assert_sums_close(t, s, 1e-3)
