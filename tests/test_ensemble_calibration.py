"""The ensemble test is calibrated (an independent oracle member passes) and
has power (an oracle member with a planted mistake fails), for each of the
FP64-oracle ensembles in tests/golden.  CPU only."""
import os
import sys

import numpy as np
import pytest

import oracle
from tests.ensemble_check import ensemble_mean_shift, ensemble_verdict

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.join(HERE, "golden"))
import make_ensemble as E  # noqa: E402


def golden(name):
    d = np.load(os.path.join(HERE, "golden", "ensemble_%s_f64.npz" % name))
    return d["mean"], d["std"], int(d["R"])


def _cavity(seed, **over):
    p, parts = E.params(seed)
    p.update(over)
    o = oracle.Oracle(p, parts, np.float64)
    o.run(E.BURN)
    o.reset_samples()
    o.run(E.SAMPLE)
    return E.estimates(o.sums, E.SAMPLE)


def _cavity_vr(seed, **over):
    p, parts = E.params_vr(seed)
    p.update(over)
    o = oracle.Oracle(p, parts, np.float64)
    o.run(E.BURN)
    o.reset_samples()
    o.run(E.SAMPLE)
    return E.estimates_vr(o.sums, E.SAMPLE, p)


def _batched(seed, dtype=np.float64, **over):
    p, parts = E.params_batched(seed)
    p.update(over)
    o = oracle.Oracle(p, parts, dtype)
    o.run(E.SAMPLE_B)
    return E.estimates_batched(o.sums, E.SAMPLE_B)


def test_independent_oracle_member_passes():
    mean, std, R = golden("cavity32")
    ok, info = ensemble_verdict(_cavity(1000), mean, std, R)
    assert ok, info


@pytest.mark.parametrize("over", [dict(wall_u=((0, 0, 0), (0, 0, 0), (0, 0, 0), (0.3, 0, 0))),
                                  dict(wall_T=(1.0, 1.0, 1.0, 1.08))])
def test_planted_mistake_fails(over):
    # lid 50% too fast, or the lid 8% too hot: the ensemble test must notice
    mean, std, R = golden("cavity32")
    ok, info = ensemble_verdict(_cavity(1001, **over), mean, std, R)
    assert not ok, info


def test_weighted_estimators_independent_member_passes_and_mistake_fails():
    mean, std, R = golden("cavity32vr")
    ok, info = ensemble_verdict(_cavity_vr(1002), mean, std, R)
    assert ok, info
    # the lid 40% too fast: a 0.02 velocity change the weighted estimators
    # resolve
    ok, info = ensemble_verdict(_cavity_vr(1003, wall_u=((0, 0, 0),) * 3 + ((0.07, 0, 0),)), mean, std, R)
    assert not ok, info


def test_batched_independent_members_pass_and_wrong_rate_fails():
    mean, std, R = golden("batched256")
    for dtype in (np.float64, np.float32):
        x = _batched(1004, dtype)
        ok, info = ensemble_verdict(x, mean, std, R)
        assert ok, (dtype, info)
        ok, shift = ensemble_mean_shift(x, mean, std, R)
        assert ok, (dtype, shift)
    # a cross-section 30% too large relaxes the anisotropy too fast: each
    # cell moves by less than its own scatter, the mean over the cells by
    # many standard errors
    p, _ = E.params_batched(0)
    ok, shift = ensemble_mean_shift(_batched(1005, sigma=p["sigma"] * 1.3), mean, std, R)
    assert not ok, shift
