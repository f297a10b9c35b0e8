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
    f, y, bd, sl = (t.cpu().numpy() for t in learned.collect(sim, with_bound=True))
    off = p["inst_offset"]
    c = [np.asarray(parts[k], dtype=np.float32) for k in ("cx", "cy", "cz")]
    big = 0
    for b in range(64):
        s, e = off[b], off[b + 1]
        if e - s < 2:
            assert y[b] == -np.inf and bd[b] == -np.inf and sl[b] == -np.inf
            continue
        fo = oracle.features(c[0][s:e], c[1][s:e], c[2][s:e], 1.0, 1.0, dtype=np.float32)
        assert np.abs(f[b] - fo).max() <= 1e-6 * max(1.0, np.abs(fo).max()), (b, f[b], fo)
        d = oracle.diameter(c[0][s:e], c[1][s:e], c[2][s:e], dtype=np.float32)
        assert abs(y[b] - math.log2(d)) <= 1e-6
        assert abs(bd[b] - math.log2(oracle.exact_bound(c[0][s:e], c[1][s:e], c[2][s:e], np.float32))) <= 1e-6
        # the |S| <= 64 threshold: the 65th largest r_p + r_(1) (numpy)
        v = np.stack([c[k][s:e].astype(np.float64) for k in range(3)])
        mid = 0.5 * (v.max(1) + v.min(1))
        r = np.sqrt(((v - mid[:, None]) ** 2).sum(0))
        t = np.sort(r + r.max())[::-1]
        if e - s <= 64:
            assert sl[b] == -np.inf
        else:
            big += 1
            assert abs(sl[b] - math.log2(t[64])) <= 1e-6, (b, sl[b], math.log2(t[64]))
    assert big > 10
    sim.close()


def test_standardize_fold_and_bf16_export(gpu):
    # statistics against numpy, the fold against the network on standardised
    # inputs, the bfloat16 rounding against torch's conversion
    _announce("standardize, fold, bf16")
    import torch
    from paper_2301_05985_amd import learned
    rng = np.random.default_rng(8)
    n = 5000
    x = (rng.standard_normal((n, 6)) * [1, 2, 0.5, 3, 0.1, 0.2] + [8, -1, 0.3, 1, 0.05, 0]).astype(np.float32)
    y = rng.standard_normal(n).astype(np.float32)
    y[::13] = -np.inf
    xg, yg = torch.from_numpy(x).cuda(), torch.from_numpy(y).cuda()
    xs, stats_dev, stats = learned.standardize(xg, yg)
    ok = np.isfinite(y)
    xd = x[ok].astype(np.float64)
    assert np.allclose(stats[:6], xd.mean(0), rtol=1e-12, atol=1e-12)
    assert np.allclose(stats[6:12], xd.std(0, ddof=1), rtol=1e-10)
    assert abs(stats[12] - y[ok].astype(np.float64).mean()) < 1e-12 and stats[13] == ok.sum()
    ref = ((x.astype(np.float64) - stats[:6]) / stats[6:12]).astype(np.float32)
    assert np.array_equal(xs.cpu().numpy(), ref)
    p = torch.from_numpy((M.init_params(3) * 0.3).astype(np.float32)).cuda()
    before = learned.forward(p, xs).cpu().numpy()
    bits_dev, bits = learned.export_bf16(p, stats_dev)
    after = learned.forward(p, xg).cpu().numpy()
    assert np.abs(after - before).max() <= 1e-4 * (1 + np.abs(before).max())
    assert np.array_equal(bits, p.to(torch.bfloat16).view(torch.int16).cpu().numpy().view(np.uint16))


def test_calibration_table_matches_its_definition(gpu):
    # the library's table against the definition evaluated with numpy on the
    # same network outputs, for several margins
    _announce("calibration table")
    import torch
    from paper_2301_05985_amd import binding, learned
    xv, yv, bv, sv = learned.generate(seeds=(7,), steps=8, every=4, n_inst=512, nmin=20, nmax=1200, with_bound=True)
    net = _synthetic_net(5, float(np.nanmedian(yv.cpu().numpy()[np.isfinite(yv.cpu().numpy())])))
    bits_dev = torch.from_numpy(M.to_bf16(net).view(np.int16)).cuda()
    sigma, dt = 0.01, 0.05
    costs = dict(cost_network=3.0, cost_member=0.01, cost_verify=5.0)
    delta, min_n, table = learned.calibrate(bits_dev, xv, yv, bv, sv, sigma, dt, costs=costs)
    ypred = learned.forward(bits_dev.view(torch.bfloat16).float(), xv).cpu().numpy().astype(np.float64)
    x, lab, bnd, slm = (t.cpu().numpy().astype(np.float64) for t in (xv, yv, bv, sv))
    N = np.rint(np.exp2(x[:, 0]))
    keep = np.isfinite(lab) & (N >= 2)
    edges = 64.0 * 2.0 ** np.arange(binding.CALIB_NBINS - 1)
    bins = np.searchsorted(edges, N, side="right")
    for j in (0, 40, 64, 90, 127):
        d = -0.64 + 0.01 * j
        k = np.clip(np.ceil(64.0 * (ypred + d)), -4096, 4096)
        gp = k / 64.0
        ver = keep & (gp < bnd)
        gv = gp + math.log2(1.0 - 2.0 ** -20)
        used = ver & (gv >= lab) & (gv >= slm)
        gain = np.where(used, 0.5 * sigma * dt * N * (N - 1) * (np.exp2(bnd) - np.exp2(gp)), 0.0)
        cost = np.where(keep, costs["cost_network"] + np.where(ver, N * costs["cost_member"] + costs["cost_verify"], 0),
                        0)
        for b in range(binding.CALIB_NBINS):
            m = bins == b
            assert table[j, b, 2] == (used & m).sum() and table[j, b, 3] == (ver & ~used & m).sum(), (j, b)
            assert abs(table[j, b, 0] - gain[m].sum()) <= 1e-3 * (1 + m.sum())
            assert abs(table[j, b, 1] - cost[m].sum()) <= 1e-3 * (1 + m.sum())
    # the returned margin and gate maximise the net saving over the table
    net_gain = np.cumsum((table[:, :, 0] - table[:, :, 1])[:, ::-1], axis=1)[:, ::-1]
    if net_gain.max() > 0:
        jb, gb = np.unravel_index(np.argmax(net_gain), net_gain.shape)
        assert abs(delta - (-0.64 + 0.01 * jb)) < 1e-12 and min_n == (0 if gb == 0 else 32 << gb)
    else:
        assert min_n == 2 ** 31 - 1


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
    # a size gate in the middle of the sizes: small cells skip the network
    gate = int(np.median(np.diff(off))) if real == "f32" and mol == "hs" else 0
    q = dict(p, majorant=1, mlp=net, mlp_delta=delta, mlp_min_n=gate)
    orc = oracle.Oracle(q, parts, dtype)
    log = orc.run(6, learned_log=True)
    if nmax <= 600:
        assert (log == 1).any() and (log == 0).any() and (log == -1).any(), np.unique(log, return_counts=True)
    else:
        assert (np.diff(off) > 1024).any()
    if real == "f64" and nmax > 2016:
        assert (np.diff(off) > 2016).any()  # FP64 LDS capacity without weights
    sim = Simulation(dict(p, majorant=1), parts)
    sim.set_majorant_model(M.to_bf16(net), delta, gate)
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
    print("calibrated margin %.2f, size gate %d" % (model["delta"], model["min_n"]), flush=True)
    # the network's effect on the candidates, with every cell using it (the
    # size gate weighs that effect against the network's cost)
    model = dict(model, min_n=0)
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
