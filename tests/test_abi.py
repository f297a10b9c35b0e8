"""Host-side checks of the C ABI: the library loads, exports every entry point
the header declares, and rejects invalid configurations before any launch.
No GPU is touched (dsmc_workspace_size is pure host validation)."""
import ctypes
import os
import re

import numpy as np
import pytest

from paper_2301_05985_amd import binding, workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    text = open(os.path.join(ROOT, "include", "dsmc.h")).read()
    return sorted(set(re.findall(r"^(?:dsmc_status|const char \*|int64_t)\s*(dsmc_[a-z0-9_]+)\s*\(", text, re.M)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(binding.lib_path()):
        from paper_2301_05985_amd import build
        build.build()
    return binding.load()


def test_every_declared_symbol_is_exported(lib):
    syms = declared_symbols()
    assert len(syms) >= 15
    for s in syms:
        assert hasattr(lib, s), s


def test_status_strings(lib):
    for code in range(0, -8, -1):
        assert lib.dsmc_status_string(code)


def _ws(lib, cfg):
    n = ctypes.c_size_t()
    return lib.dsmc_workspace_size(ctypes.byref(cfg), ctypes.byref(n)), n.value


def test_workspace_size_valid_configs(lib):
    for p, parts in (W.cavity(nx=8, ny=8, per_cell=10), W.fourier(n_cells=10, per_cell=10),
                     W.batched(n_inst=8, nmin=10, nmax=20)):
        cfg = binding.make_config(p, len(parts["cx"]))
        keep = []
        if p["dims"] == 0:
            off = np.ascontiguousarray(p["inst_offset"], dtype=np.int64)
            keep.append(off)
            cfg.inst_offset = off.ctypes.data
        rc, n = _ws(lib, cfg)
        assert rc == 0 and n > 0


@pytest.mark.parametrize("field,value,code", [
    ("abi_version", 99, -7), ("dims", 3, -1), ("real_bytes", 2, -1), ("dt", 0.0, -1),
    ("FN", -1.0, -1), ("molecule", 5, -1), ("majorant", 7, -1), ("n_particles", -5, -1),
    ("schedule", 2, -1), ("persistent_waves", -1, -1), ("chunk_work", -3, -1),
    ("vr_reconstruct", -1, -1), ("vr_kappa", 0.5, -1), ("vr_kappa", 17.0, -1), ("wide_min", 32, -1),
    ("wide_min", -1, -1), ("occupancy", 4, -1), ("occupancy", 7, -1), ("cells_per_wave", 3, -1),
    ("cells_per_wave", -1, -1), ("waves_per_cell", 2, -1), ("waves_per_cell", -1, -1),
])
def test_workspace_size_rejects_invalid(lib, field, value, code):
    p, parts = W.cavity(nx=4, ny=4, per_cell=5)
    cfg = binding.make_config(p, len(parts["cx"]))
    setattr(cfg, field, value)
    rc, _ = _ws(lib, cfg)
    assert rc == code


def test_rejects_unpaired_periodic_wall_and_bad_offsets(lib):
    p, parts = W.cavity(nx=4, ny=4, per_cell=5)
    cfg = binding.make_config(p, len(parts["cx"]))
    cfg.wall_kind[0] = 2
    assert _ws(lib, cfg)[0] == -1
    p, parts = W.batched(n_inst=4, nmin=10, nmax=20)
    cfg = binding.make_config(p, len(parts["cx"]))
    bad = np.ascontiguousarray(p["inst_offset"], dtype=np.int64).copy()
    bad[-1] += 1  # does not end at n_particles
    cfg.inst_offset = bad.ctypes.data
    assert _ws(lib, cfg)[0] == -1
    cfg.inst_offset = None
    assert _ws(lib, cfg)[0] == -1


def test_vhs_needs_a_viscosity_index_in_range(lib):
    p, parts = W.cavity(nx=4, ny=4, per_cell=5)
    for omega, code in ((0.81, 0), (0.5, 0), (1.0, 0), (0.3, -1), (1.2, -1)):
        cfg = binding.make_config(dict(p, molecule=W.VHS, omega=omega), len(parts["cx"]))
        assert _ws(lib, cfg)[0] == code, omega


def test_vss_needs_omega_and_alpha_in_range(lib):
    p, parts = W.cavity(nx=4, ny=4, per_cell=5)
    for omega, alpha, code in ((0.81, 1.6, 0), (0.5, 1.0, 0), (1.0, 2.0, 0), (0.3, 1.5, -1),
                               (0.81, 0.9, -1), (0.81, 2.5, -1), (0.81, float("nan"), -1)):
        cfg = binding.make_config(dict(p, molecule=W.VSS, omega=omega, alpha=alpha), len(parts["cx"]))
        assert _ws(lib, cfg)[0] == code, (omega, alpha)


def test_autotune_signature_separates_workloads():
    # the cache key changes with everything that changes the collision cost
    from paper_2301_05985_amd import autotune
    p, _ = W.batched(n_inst=64, nmin=10, nmax=200)
    sig = autotune.signature(p)
    assert sig == autotune.signature(dict(p))
    assert sig != autotune.signature(dict(p, vr=1))
    assert sig != autotune.signature(dict(p, majorant=1))
    assert sig != autotune.signature(dict(p, real="f64"))
    assert sig != autotune.signature(dict(p, sigma=p["sigma"] * 10))  # another collision rate
    q, _ = W.batched(n_inst=64, nmin=10, nmax=200, seed=1)
    assert sig != autotune.signature(q)  # other instance sizes
    assert all(c["schedule"] in (0, 1) for c in autotune.CANDIDATES)


def test_init_rejects_misaligned_particle_arrays(lib):
    # validation happens before any device call: the addresses below are
    # never dereferenced
    p, parts = W.cavity(nx=4, ny=4, per_cell=5, real="f32")
    n = len(parts["cx"])
    cfg = binding.make_config(p, n)
    ctx = ctypes.c_void_p()
    fake = 1 << 40
    names = ("x", "y", "cx", "cy", "cz", "w", "id")
    for field in ("x", "y", "cx", "cy", "cz", "id"):
        soa = binding.Soa(*(fake + k * (1 << 20) + (4 if f == field else 0) for k, f in enumerate(names)))
        rc = lib.dsmc_init(ctypes.byref(cfg), ctypes.byref(soa), ctypes.c_void_p(fake + (1 << 30)),
                           ctypes.c_size_t(1 << 40), None, ctypes.byref(ctx))
        assert rc == -1, field
        assert not ctx.value


def test_mlp_scratch_size_and_batch_limit(lib):
    # per-sample records (260 floats) plus the FP64 sums of every chunk of
    # 128 samples (4,675 parameters + loss + valid count, two floats each)
    for n in (1, 127, 128, 129, 4096, 100000):
        chunks = -(-n // 128)
        assert lib.dsmc_mlp_scratch_floats(n) == n * 260 + 2 * chunks * (4673 + 2), n
    assert lib.dsmc_mlp_scratch_floats(-1) == 0
    # a batch needing more than 65,535 chunks is refused before any launch
    # (the addresses are never dereferenced)
    fake = ctypes.c_void_p(1 << 40)
    big = 65535 * 128 + 1
    rc = lib.dsmc_mlp_loss_grad(fake, fake, fake, big, 0.95, fake, fake, fake, None)
    assert rc == -1
    rc = lib.dsmc_mlp_loss_grad(fake, fake, fake, 0, 0.95, fake, fake, fake, None)
    assert rc == -1
    rc = lib.dsmc_mlp_loss_grad(fake, fake, fake, 16, 1.5, fake, fake, fake, None)
    assert rc == -1


@pytest.mark.parametrize("vr", [False, True])
def test_estimators_match_the_oracle(lib, vr):
    # host arithmetic of the library against the oracle's numpy estimators
    import oracle
    rng = np.random.default_rng(12)
    nc, ns = 40, 37
    c = rng.standard_normal((nc, 200, 3)) * 1.3 + rng.standard_normal((nc, 1, 3)) * 0.4
    w = 1.0 + 0.05 * rng.standard_normal((nc, 200))
    x, y, z = c[..., 0], c[..., 1], c[..., 2]
    s2 = x * x + y * y + z * z
    q = np.stack([np.ones_like(x), x, y, z, x * x, y * y, z * z, x * y, x * z, y * z, x * s2, y * s2, z * s2], -1)
    sums = np.concatenate([q.sum(1), ((1 - w)[..., None] * q).sum(1)], 1) * ns
    V = rng.uniform(0.5, 2.0, nc)
    ref = oracle.estimators(sums, ns, 2.0, V, vr=vr, vr_n0=300.0, vr_T0=1.2)
    out = binding.estimators(sums, ns, 2.0, volume=V, vr=vr, vr_n0=300.0, vr_T0=1.2)
    P = ref["P"]
    want = np.concatenate([ref["n"][:, None], ref["u"], ref["T"][:, None],
                           np.stack([P[:, 0, 0], P[:, 1, 1], P[:, 2, 2], P[:, 0, 1], P[:, 0, 2], P[:, 1, 2]], 1),
                           ref["q"]], 1)
    assert np.allclose(out, want, rtol=1e-12, atol=1e-9 * np.abs(want).max())
    assert lib.dsmc_estimators(None, nc, ns, 2.0, None, 1.0, 0, 0.0, 1.0, None) == -1



def test_grid_kernel_parameters_accepted(lib):
    p, parts = W.batched(n_inst=8, nmin=10, nmax=20)
    off = np.ascontiguousarray(p["inst_offset"], dtype=np.int64)
    for over in (dict(wide_min=64), dict(wide_min=5000), dict(occupancy=5), dict(occupancy=6),
                 dict(vr_kappa=16.0), dict(vr_reconstruct=4)):
        cfg = binding.make_config(dict(p, **over), len(parts["cx"]))
        cfg.inst_offset = off.ctypes.data
        assert _ws(lib, cfg)[0] == 0, over


def test_four_waves_per_cell_accepted_only_where_it_applies(lib):
    p, parts = W.fourier(n_cells=8, per_cell=300)
    n = len(parts["cx"])
    for over, code in ((dict(waves_per_cell=4), 0), (dict(waves_per_cell=4, majorant=2), 0),
                       (dict(waves_per_cell=4, majorant=1), -1), (dict(waves_per_cell=4, cells_per_wave=2), -1),
                       (dict(waves_per_cell=1), 0)):
        assert _ws(lib, binding.make_config(dict(p, **over), n))[0] == code, over
    pb, partsb = W.batched(n_inst=8, nmin=10, nmax=20)
    cfg = binding.make_config(dict(pb, waves_per_cell=4), len(partsb["cx"]))
    off = np.ascontiguousarray(pb["inst_offset"], dtype=np.int64)
    cfg.inst_offset = off.ctypes.data
    assert _ws(lib, cfg)[0] == -1


def test_autotune_walled_signature_and_pair_rule():
    from paper_2301_05985_amd import autotune
    p, parts = W.cavity(nx=8, ny=8, per_cell=20)
    n = len(parts["cx"])
    sig = autotune.signature(p, n)
    assert sig == autotune.signature(dict(p), n)
    for q in (dict(p, vr=1 - p.get("vr", 0)), dict(p, vr_reconstruct=4), dict(p, vr_kappa=1.5),
              dict(p, real="f64"), dict(p, molecule=W.VHS), dict(p, n_cells=(8, 4)), dict(p, sigma=p["sigma"] * 10),
              dict(p, dt=p["dt"] * 2)):
        assert autotune.signature(q, n) != sig
    assert autotune.signature(p, n + 1) != sig
    assert autotune.pair_allowed(p, n) and autotune.pair_allowed(dict(p, majorant=2), n)
    assert not autotune.pair_allowed(dict(p, majorant=1), n)
    assert autotune.pair_allowed(p, 128 * 64) and not autotune.pair_allowed(p, 128 * 64 + 1)
    pb, partsb = W.batched(n_inst=8, nmin=10, nmax=20)
    assert not autotune.pair_allowed(pb, len(partsb["cx"]))
    assert "cells_per_wave" in autotune.LAUNCH_KEYS and "waves_per_cell" in autotune.LAUNCH_KEYS
    assert autotune.walled_candidates(p, n) == autotune.WALLED
    assert autotune.walled_candidates(dict(p, majorant=1), n) == [autotune.WALLED[0]]
    assert autotune.walled_candidates(p, 128 * 64 + 1) == [autotune.WALLED[0], autotune.WALLED[2]]
    assert autotune.walled_candidates(pb, len(partsb["cx"])) == []


def test_two_cells_per_wave_accepted_only_where_it_applies(lib):
    # walled runs with the exact or brute-force majorant and a mean cell
    # population of at most 128 (128 mover slots)
    for p, parts in (W.cavity(nx=4, ny=4, per_cell=5), W.fourier(n_cells=8, per_cell=128, real="f64")):
        for maj, code in ((0, 0), (2, 0), (1, -1)):
            cfg = binding.make_config(dict(p, cells_per_wave=2, majorant=maj), len(parts["cx"]))
            assert _ws(lib, cfg)[0] == code, (maj, p["dims"])
    p, parts = W.fourier(n_cells=8, per_cell=129)
    assert _ws(lib, binding.make_config(dict(p, cells_per_wave=2), len(parts["cx"])))[0] == -1
    assert _ws(lib, binding.make_config(dict(p, cells_per_wave=1), len(parts["cx"])))[0] == 0
    p, parts = W.batched(n_inst=8, nmin=10, nmax=20)
    off = np.ascontiguousarray(p["inst_offset"], dtype=np.int64)
    for cpw, code in ((0, 0), (1, 0), (2, -1)):
        cfg = binding.make_config(dict(p, cells_per_wave=cpw), len(parts["cx"]))
        cfg.inst_offset = off.ctypes.data
        assert _ws(lib, cfg)[0] == code, cpw


def test_autotune_refines_only_the_grid_schedule():
    from paper_2301_05985_amd import autotune
    p, _ = W.batched(n_inst=64, nmin=10, nmax=200)
    assert autotune.refinements(p, {"schedule": 1, "persistent_waves": 1024, "chunk_work": 0}) == []
    assert [a for a, _ in autotune.refinements(p, dict(autotune.GRID))] == ["wide_min"]
    assert [a for a, _ in autotune.refinements(dict(p, vr=1), dict(autotune.GRID))] == ["wide_min", "occupancy"]
    for a, values in autotune.refinements(dict(p, vr=1), dict(autotune.GRID)):
        assert a in autotune.LAUNCH_KEYS and len(values) > 0
