"""GPU tests of the learned majorant: training kernels against the FP64
oracle, feature collection against the oracle, the learned collision path
bit for bit against the oracle, forced fallback, and what training gains."""
import math
import sys

import numpy as np
import pytest

import oracle
from oracle import mlp_oracle as M
from paper_2301_05985_amd import workloads as W

pytestmark = pytest.mark.gpu


def _announce(name):
    print("[gpu case] %s" % name, flush=True)


def _rand_data(n, seed):
    rng = np.random.default_rng(seed)
    x = rng.standard_normal((n, 6)).astype(np.float32)
    x[:, 0] += 10.0
    y = (rng.standard_normal(n) * 0.3 + 2.5).astype(np.float32)
    y[::17] = -np.inf  # cells with fewer than two particles carry no label
    return x, y


def test_mlp_forward_matches_oracle(gpu):
    _announce("mlp forward")
    import torch
    from paper_2301_05985_amd import learned
    p = M.init_params(4).astype(np.float32)
    x, _ = _rand_data(3000, 1)
    yg = learned.forward(torch.from_numpy(p).cuda(), torch.from_numpy(x).cuda()).cpu().numpy()
    yo = M.forward(p.astype(np.float64), x.astype(np.float64))
    assert np.abs(yg - yo).max() <= 1e-4 * max(1.0, np.abs(yo).max())


@pytest.mark.parametrize("tau", [0.5, 0.95])
def test_mlp_gradients_match_oracle(gpu, tau):
    _announce("mlp gradients tau=%g" % tau)
    import torch
    from paper_2301_05985_amd import learned
    p = M.init_params(5).astype(np.float32)
    x, y = _rand_data(4096, 2)
    tr = learned.Trainer(torch.from_numpy(p).cuda(), batch=4096, tau=tau)
    g, loss = tr.loss_grad(torch.from_numpy(x).cuda(), torch.from_numpy(y).cuda())
    g = g.cpu().numpy().astype(np.float64)
    lo, go = M.loss_grad(p.astype(np.float64), x.astype(np.float64), y.astype(np.float64), tau)
    assert abs(float(loss.item()) - lo) <= 1e-4 * abs(lo)
    W1, b1, W2, b2, w3, b3 = M.unpack(g)
    O = M.unpack(go)
    for a, b in zip((W1, b1, W2, b2, w3, np.array([b3])), (O[0], O[1], O[2], O[3], O[4], np.array([O[5]]))):
        assert np.linalg.norm(a - b) <= 1e-4 * np.linalg.norm(b) + 1e-12


def test_adam_matches_oracle(gpu):
    _announce("adam")
    import torch
    from paper_2301_05985_amd import learned
    p = M.init_params(6).astype(np.float32)
    x, y = _rand_data(4096, 3)
    tr = learned.Trainer(torch.from_numpy(p.copy()).cuda(), batch=4096, lr=1e-3)
    xg, yg = torch.from_numpy(x).cuda(), torch.from_numpy(y).cuda()
    po, m, v = p.astype(np.float64), np.zeros(M.NPARAM), np.zeros(M.NPARAM)
    for t in range(1, 4):
        # both sides step from the same gradient (the GPU one), so only Adam is compared
        g, _ = tr.loss_grad(xg, yg)
        gnp = g.cpu().numpy().astype(np.float64)
        tr.t += 1
        from paper_2301_05985_amd import binding
        binding.check(tr.L.dsmc_mlp_adam(learned._ptr(tr.p), learned._ptr(tr.g), learned._ptr(tr.m),
                                         learned._ptr(tr.v), M.NPARAM, tr.t, 1e-3, 0.9, 0.999, 1e-8, tr.stream),
                      "adam")
        po, m, v = M.adam(po, gnp, m, v, t)
    pg = tr.p.cpu().numpy().astype(np.float64)
    assert np.abs(pg - po).max() <= 1e-6


def test_collected_features_and_labels_match_oracle(gpu):
    _announce("collect features")
    from paper_2301_05985_amd import learned
    from paper_2301_05985_amd.binding import Simulation
    p, parts = W.batched(n_inst=64, nmin=1, nmax=400, real="f32", steps=1)
    sim = Simulation(p, parts)
    f, y = learned.collect(sim)
    f, y = f.cpu().numpy(), y.cpu().numpy()
    off = p["inst_offset"]
    c = [np.asarray(parts[k], dtype=np.float32) for k in ("cx", "cy", "cz")]
    for b in range(64):
        s, e = off[b], off[b + 1]
        if e - s < 2:
            assert y[b] == -np.inf
            continue
        fo = oracle.features(c[0][s:e], c[1][s:e], c[2][s:e], 1.0, 1.0, dtype=np.float32)
        assert np.abs(f[b] - fo).max() <= 1e-6 * max(1.0, np.abs(fo).max()), (b, f[b], fo)
        d = oracle.diameter(c[0][s:e], c[1][s:e], c[2][s:e], dtype=np.float32)
        assert abs(y[b] - math.log2(d)) <= 1e-6
    sim.close()


def _synthetic_net(seed, center):
    """A random small network whose output scatters around `center` (log2 units)."""
    rng = np.random.default_rng(seed)
    p = M.init_params(seed) * 0.05
    p[-1] = center
    return M.from_bf16(M.to_bf16(p.astype(np.float32)))


@pytest.mark.parametrize("real,sizes,mol", [("f32", (48, 30, 600), "hs"), ("f64", (48, 30, 600), "hs"),
                                            ("f32", (12, 900, 1600), "hs"), ("f32", (48, 30, 600), "vss"),
                                            ("f64", (8, 1500, 2400), "hs")])
def test_learned_collisions_bit_exact_against_oracle(gpu, real, sizes, mol):
    # the third case has instances above 1024 particles (workgroup cells);
    # the fourth runs variable soft spheres; the last has FP64 instances
    # above the LDS capacity (global-memory workgroups)
    _announce("learned collide %s %s %s" % (real, sizes, mol))
    from paper_2301_05985_amd.binding import Simulation
    n_inst, nmin, nmax = sizes
    p, parts = W.batched(n_inst=n_inst, nmin=nmin, nmax=nmax, real=real, steps=6, dt=0.2)
    if mol == "vss":
        p = dict(p, molecule=W.VSS, omega=0.81, alpha=1.5)
    dtype = np.float32 if real == "f32" else np.float64
    off = p["inst_offset"]
    c = [np.asarray(parts[k], dtype=dtype) for k in ("cx", "cy", "cz")]
    d = [oracle.diameter(c[0][off[b]:off[b + 1]], c[1][off[b]:off[b + 1]], c[2][off[b]:off[b + 1]], dtype)
         for b in range(n_inst)]
    net = _synthetic_net(7, math.log2(np.median(d)))
    delta = 0.01
    q = dict(p, majorant=1, mlp=net, mlp_delta=delta)
    orc = oracle.Oracle(q, parts, dtype)
    log = orc.run(6, learned_log=True)
    if nmax <= 600:
        assert (log == 1).any() and (log == 0).any() and (log == -1).any(), np.unique(log, return_counts=True)
    else:
        assert (np.diff(off) > 1024).any()
    if real == "f64" and nmax > 2016:
        assert (np.diff(off) > 2016).any()  # FP64 LDS capacity without weights
    sim = Simulation(dict(p, majorant=1), parts)
    sim.set_majorant_model(M.to_bf16(net), delta)
    sim.step(6)
    st, so = sim.particles(), orc.state()
    _, cnt, _ = sim.sample()
    dg = sim.diagnostics()
    assert dg["learned_used"] == (log == 1).sum()
    assert dg["fallback"] == (log == -1).sum()
    assert dg["learned_skip"] == (log == 0).sum()
    assert np.array_equal(cnt, orc.counters)
    for k in ("cx", "cy", "cz"):
        assert np.array_equal(st[k], so[k]), k
    sim.close()


def test_forced_fallback_reproduces_exact_run(gpu):
    _announce("forced fallback")
    from paper_2301_05985_amd.binding import Simulation
    p, parts = W.batched(n_inst=64, nmin=50, nmax=800, real="f32", steps=5)
    a = Simulation(p, parts)
    a.step(5)
    sa = a.particles()
    low = np.zeros(M.NPARAM, dtype=np.float32)
    low[-1] = -30.0  # proposal far below every cell's speeds: always rejected
    b = Simulation(dict(p, majorant=1), parts)
    b.set_majorant_model(M.to_bf16(low), 0.0)
    b.step(5)
    sb = b.particles()
    assert b.diagnostics()["fallback"] == 64 * 5
    for k in ("cx", "cy", "cz"):
        assert np.array_equal(sa[k], sb[k]), k
    assert np.array_equal(a.sample()[1], b.sample()[1])


def test_training_reduces_candidates_at_equal_collision_rate(gpu):
    # Train on short exact-majorant runs, then compare on a held-out run: the
    # learned proposal must be used in a large fraction of cells, cut the
    # number of NTC candidates, and leave the accepted-collision rate (a
    # property of the law, not of the majorant) unchanged within noise.
    _announce("training gain")
    from paper_2301_05985_amd import learned
    from paper_2301_05985_amd.binding import Simulation
    model = learned.train_model(n_epochs=6, seeds=(1, 2), val_seed=3, steps=64, every=4, n_inst=1024,
                                log=lambda s: print(s, flush=True))
    assert model["loss_history"][-1] < model["loss_history"][0]
    p, parts = W.batched(n_inst=1024, real="f32", seed=0)
    a = Simulation(p, parts)
    b = learned.simulation_with_model(p, parts, model)
    a.step(40)
    b.step(40)
    ca = a.sample()[1].sum(0).astype(float)
    cb = b.sample()[1].sum(0).astype(float)
    db = b.diagnostics()
    used = db["learned_used"] / (1024 * 40)
    print("learned used %.3f fallback %.4f skip %.3f; candidates exact %d learned %d; accepted %d vs %d" % (
        used, db["fallback"] / (1024 * 40), db["learned_skip"] / (1024 * 40), ca[0], cb[0], ca[1], cb[1]),
        flush=True)
    assert used > 0.05
    assert cb[0] < ca[0]
    assert abs(ca[1] - cb[1]) < 5 * math.sqrt(ca[1] + cb[1])
