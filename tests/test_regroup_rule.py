"""The regrouping rule of the walled step, checked on the CPU: for a
sequence grouped by cell, the particles of new cell t taken as (movers from
cells before t in ascending position) + (the particles that stayed in t, in
position order) + (movers from cells after t in ascending position) are
exactly the stable counting sort of the sequence by new cell, whatever order
the movers were listed in.  This is the argument the collision kernel's
selection rests on; the kernel itself is compared with the oracle on the GPU."""
import numpy as np


def _stable_by_rule(old_cell, new_cell, ncell, rng):
    n = len(old_cell)
    start = np.searchsorted(old_cell, np.arange(ncell + 1))
    out = []
    for t in range(ncell):
        b, e = start[t], start[t + 1]
        pos = np.arange(n)
        movers = pos[(new_cell == t) & (old_cell != t)]
        movers = rng.permutation(movers)          # listed in arbitrary order
        movers = np.sort(movers)                  # the wave's sort
        stays = pos[b:e][new_cell[b:e] == t]      # code bytes of t's own range
        low = movers[movers < b]
        high = movers[movers >= e]
        assert len(low) + len(high) == len(movers)
        out.append(np.concatenate([low, stays, high]))
    return np.concatenate(out) if out else np.zeros(0, dtype=np.int64)


def test_rule_equals_stable_counting_sort():
    rng = np.random.default_rng(11)
    for trial in range(60):
        ncell = int(rng.integers(1, 40))
        n = int(rng.integers(0, 400))
        old_cell = np.sort(rng.integers(0, ncell, n))
        # most particles stay, some move to a neighbour, a few anywhere
        step = rng.choice([-1, 0, 0, 0, 1], n)
        far = rng.random(n) < 0.05
        new_cell = np.where(far, rng.integers(0, ncell, n), np.clip(old_cell + step, 0, ncell - 1))
        got = _stable_by_rule(old_cell, new_cell, ncell, rng)
        want = np.argsort(new_cell, kind="stable")
        assert np.array_equal(got, want), trial
