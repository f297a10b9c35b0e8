"""Pins of the oracle's learned-majorant path: a proposal that is not below
the exact bound, or that fails verification, leaves the run bit-identical to
the exact-majorant run; a verified proposal always bounds every pair."""
import math

import numpy as np
import pytest

import oracle
from oracle import mlp_oracle as M
from paper_2301_05985_amd import workloads as W


def const_net(value):
    """Network whose output is the constant `value` (log2 units)."""
    p = np.zeros(M.NPARAM, dtype=np.float32)
    p[-1] = value
    return p


def _pair(p, parts, mlp, steps=6, dtype=np.float32):
    a = oracle.Oracle(p, parts, dtype)
    q = dict(p, majorant=1, mlp=mlp, mlp_delta=0.0)
    b = oracle.Oracle(q, parts, dtype)
    a.run(steps)
    log = b.run(steps, learned_log=True)
    return a, b, log


@pytest.mark.parametrize("value,flag", [(20.0, 0), (-20.0, -1)])
def test_unusable_proposal_reproduces_exact_run(value, flag):
    p, parts = W.batched(n_inst=12, nmin=40, nmax=400, real="f32", steps=6)
    a, b, log = _pair(p, parts, const_net(value))
    assert (log == flag).all()
    for k in ("cx", "cy", "cz"):
        assert np.array_equal(getattr(a, k), getattr(b, k))
    assert np.array_equal(a.counters, b.counters)


def test_verified_proposal_bounds_every_pair_and_cuts_candidates():
    # proposal just above each cell's largest pair speed: the lattice value
    # 2^(k/64) lies within a factor 2^(1/64) above log2(diameter) + delta
    p, parts = W.batched(n_inst=16, nmin=60, nmax=300, real="f64", steps=1)
    off = p["inst_offset"]
    c = np.stack([parts["cx"], parts["cy"], parts["cz"]])
    used = 0
    fewer = 0
    for b in range(16):
        s, e = off[b], off[b + 1]
        d = oracle.diameter(*c[:, s:e])
        q = dict(dims=0, n_cells=(1, 1), dt=0.05, sigma=2e-2, FN=1.0, seed=3,
                 inst_offset=np.array([0, e - s], dtype=np.int64), cell_volume=np.ones(1))
        cell = dict(cx=c[0, s:e], cy=c[1, s:e], cz=c[2, s:e])
        o = oracle.Oracle(dict(q, majorant=1, mlp=const_net(math.log2(d) + 1e-3), mlp_delta=0.0), cell)
        log = o.run(1, learned_log=True)
        x = oracle.Oracle(q, cell)  # the same cell with the exact bound
        x.run(1)
        if log[0, 0] == 1:
            used += 1
            # the proposal in use is >= the diameter: no pre-collision overshoot
            assert o.diag.overshoot == 0
            # the candidate count floor(M_real + U0) shares U0 with the exact
            # run and M_real is proportional to the majorant: never more
            # candidates, and fewer wherever the tighter majorant moves the floor
            assert o.counters[0, 0] <= x.counters[0, 0]
            fewer += int(o.counters[0, 0] < x.counters[0, 0])
        else:
            assert log[0, 0] in (0, -1)
            assert np.array_equal(o.counters, x.counters)
    assert used >= 12
    assert fewer >= used // 2


def test_learned_run_has_same_collision_rate_law():
    # Two majorants that both bound every pair give the same acceptance law:
    # candidates scale with g_max, accepted collisions do not (statistically).
    # 400 copies of one cell state, each with its own random stream.
    N, n_inst = 200, 400
    rng = np.random.default_rng(6)
    c = rng.standard_normal((3, N))
    cc = np.tile(c, n_inst)
    off = np.arange(n_inst + 1, dtype=np.int64) * N
    p = dict(dims=0, n_cells=(n_inst, 1), dt=0.02, sigma=1e-2, FN=1.0, seed=9, inst_offset=off,
             cell_volume=np.ones(n_inst))
    parts = dict(cx=cc[0], cy=cc[1], cz=cc[2])
    diam = oracle.diameter(*c)
    assert diam < oracle.exact_bound(*c)
    a = oracle.Oracle(p, parts)
    b = oracle.Oracle(dict(p, majorant=1, mlp=const_net(math.log2(diam) + 0.01), mlp_delta=0.0), parts)
    a.run(1)
    log = b.run(1, learned_log=True)
    ca, cb = a.counters.sum(0).astype(float), b.counters.sum(0).astype(float)
    assert (log == 1).all()
    assert cb[0] < ca[0]                       # fewer candidates with the tighter majorant
    se = math.sqrt(ca[1] + cb[1])
    assert abs(ca[1] - cb[1]) < 5 * se          # same expected number of collisions


def test_size_gate_reproduces_exact_run_for_small_cells():
    # cells below the gate take the exact bound without the network: with
    # the gate above every cell the run is the exact run bit for bit; with a
    # gate inside the sizes only the cells at or above it use the proposal
    p, parts = W.batched(n_inst=16, nmin=40, nmax=400, real="f32", steps=4)
    sizes = np.diff(p["inst_offset"])
    net = const_net(float(np.log2(6.0)))
    a, b, log = _pair(dict(p, mlp_min_n=0), parts, net, steps=4)
    q = dict(p, majorant=1, mlp=net, mlp_delta=0.0, mlp_min_n=10 ** 6)
    c = oracle.Oracle(q, parts, np.float32)
    logc = c.run(4, learned_log=True)
    assert (logc == 0).all()
    for k in ("cx", "cy", "cz"):
        assert np.array_equal(getattr(a, k), getattr(c, k))
    gate = int(np.median(sizes))
    d = oracle.Oracle(dict(q, mlp_min_n=gate), parts, np.float32)
    logd = d.run(4, learned_log=True)
    small = sizes < gate
    assert (logd[:, small] == 0).all()
    assert np.array_equal(logd[:, ~small], log[:, ~small])

