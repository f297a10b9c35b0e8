"""The ensemble test is calibrated (an independent oracle member passes) and
has power (an oracle member with a planted mistake fails).  CPU only."""
import os
import sys

import numpy as np
import pytest

import oracle
from tests.ensemble_check import ensemble_verdict

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.join(HERE, "golden"))
import make_ensemble as E  # noqa: E402


def _golden():
    d = np.load(os.path.join(HERE, "golden", "ensemble_cavity32.npz"))
    return d["mean"], d["std"], int(d["R"])


def _member(seed, **over):
    p, parts = E.params(seed)
    p.update(over)
    o = oracle.Oracle(p, parts, np.float32)
    o.run(E.BURN)
    o.reset_samples()
    o.run(E.SAMPLE)
    return E.estimates(o.sums, E.SAMPLE)


def test_independent_oracle_member_passes():
    mean, std, R = _golden()
    ok, info = ensemble_verdict(_member(1000), mean, std, R)
    assert ok, info


@pytest.mark.parametrize("over", [dict(wall_u=((0, 0, 0), (0, 0, 0), (0, 0, 0), (0.3, 0, 0))),
                                  dict(wall_T=(1.0, 1.0, 1.0, 1.08))])
def test_planted_mistake_fails(over):
    # lid 50% too fast, or the lid 8% too hot: the ensemble test must notice
    mean, std, R = _golden()
    ok, info = ensemble_verdict(_member(1001, **over), mean, std, R)
    assert not ok, info
