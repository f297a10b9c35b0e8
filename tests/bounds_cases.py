"""Workloads run on the bounds-checking build of the library (and on the
release build, for comparison) by tests/test_gpu_bounds.py.

Every kernel of the path takes part: walled cells staged in LDS, one or two
per wave or one per four-wave workgroup (with the gather, diffuse walls,
weights and their re-estimation),
walled cells above the LDS capacity (global-memory kernel) with overflow
mover lists,
homogeneous instances on one wave, on four-wave workgroups and above the LDS
capacity, the persistent schedule, the learned majorant, FP32 and FP64.

Run as a module (python -m tests.bounds_cases) it prints one JSON line with,
per case, the failed index checks, whether the loaded library checks indices
at all, and a digest of the run's final state, counters and sums."""
import hashlib
import json
import sys

import numpy as np

from paper_2301_05985_amd import workloads as W


def _net():
    from oracle import mlp_oracle as M
    net = M.init_params(7) * 0.05
    net[-1] = 2.9
    return M.to_bf16(M.from_bf16(M.to_bf16(net.astype(np.float32))).astype(np.float32))


def _crowded_slab(real):
    # every particle starts in the first of 8 cells: that cell is above the
    # LDS capacity, and with a long step more of its particles move into the
    # next cell than that cell has mover slots (overflow lists)
    p, parts = W.fourier(n_cells=8, per_cell=30, Kn=0.05, dt=0.08, real=real, vr=1, seed=3)
    parts = dict(parts, x=parts["x"] / 8.0)
    return dict(p, vr_reconstruct=1, vr_kappa=1.5), parts


def cases():
    out = []
    p, parts = W.cavity(nx=16, ny=16, per_cell=30, Kn=0.05, lid=0.2, real="f32", vr=1, seed=1)
    out.append(("cavity_f32_vr_reest", dict(p, vr_reconstruct=2, vr_kappa=1.5), parts, 10, None))
    out.append(("cavity_f32_vr_reest_pair", dict(p, vr_reconstruct=2, vr_kappa=1.5, cells_per_wave=2), parts, 10,
                None))
    out.append(("cavity_f32_vr_reest_wide4", dict(p, vr_reconstruct=2, vr_kappa=1.5, waves_per_cell=4), parts, 10,
                None))
    p, parts = W.fourier(n_cells=20, per_cell=50, Kn=0.1, dt=2e-3, real="f64", vr=1, seed=2)
    out.append(("fourier_f64_vr_reest", dict(p, vr_reconstruct=1, vr_kappa=1.5), parts, 10, None))
    out.append(("fourier_f64_vr_reest_pair", dict(p, vr_reconstruct=1, vr_kappa=1.5, cells_per_wave=2), parts, 10,
                None))
    p, parts = _crowded_slab("f32")
    out.append(("slab_above_capacity_f32", p, parts, 8, None))
    out.append(("slab_above_capacity_f32_pair", dict(p, cells_per_wave=2), parts, 8, None))
    out.append(("slab_above_capacity_f32_wide4", dict(p, waves_per_cell=4), parts, 8, None))
    p, parts = W.batched(n_inst=40, nmin=20, nmax=6000, real="f32", seed=4)
    out.append(("batched_grid_f32", dict(p, schedule=0), parts, 5, None))
    out.append(("batched_persistent_f32", dict(p, schedule=1, persistent_waves=256, chunk_work=2000), parts, 5, None))
    out.append(("batched_learned_f32", dict(p, majorant=1), parts, 5, _net()))
    p, parts = W.batched(n_inst=24, nmin=10, nmax=3000, real="f64", seed=5)
    rng = np.random.default_rng(5)
    parts = dict(parts, w=1.0 + 0.05 * rng.standard_normal(len(parts["cx"])))
    out.append(("batched_f64_vr_reest_wide", dict(p, vr=1, vr_reconstruct=1, vr_kappa=1.5, wide_min=64,
                                                   occupancy=6), parts, 4, None))
    return out


def run_case(name, p, parts, steps, net):
    from paper_2301_05985_amd.binding import Simulation
    sim = Simulation(p, parts)
    try:
        if net is not None:
            sim.set_majorant_model(net, 0.02)
        sim.step(steps)
        sums, cnt, _ = sim.sample()
        st = sim.particles()
        d = sim.diagnostics()
    finally:
        sim.close()
    h = hashlib.sha1()
    for k in ("x", "y", "cx", "cy", "cz", "w", "id"):
        if st.get(k) is not None:
            h.update(np.ascontiguousarray(st[k]).tobytes())
    h.update(np.ascontiguousarray(cnt).tobytes())
    h.update(np.ascontiguousarray(sums).tobytes())
    return {"bounds_violations": int(d["bounds_violations"]), "bounds_checked": int(d["bounds_checked"]),
            "status": int(d["status"]), "digest": h.hexdigest()}


def main():
    res = {}
    for name, p, parts, steps, net in cases():
        print("[bounds case] %s" % name, file=sys.stderr, flush=True)
        res[name] = run_case(name, p, parts, steps, net)
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
