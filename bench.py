#!/usr/bin/env python3
"""Benchmark of the DSMC hot path on one MI355X.

Default (no flags): the 2-D lid-driven cavity at its full size -- 256 x 256
cells, 100 particles per cell (6,553,600 particles), Kn = 0.01, diffuse walls,
importance weights re-estimated every 4 steps with the relative-speed
majorant scaled by 1.5, FP32 state with FP64 moment sums
-- W untimed warm-up steps, then exactly K timed steps (one step = free
flight with walls, the stable regrouping by cell, per-cell majorant + NTC
collisions + weight update + weight re-estimation, moment sampling).  Rank 0
prints one JSON line.

Also reported in the same line: per-kernel durations measured live with HIP
events on the run's stream (roofline of the dominant kernel), the CPU oracle
timed on a bounded sample of the same workload, and secondary workloads
(1-D Fourier, batched homogeneous cells with the exact and, when a trained
network is available, the learned majorant, and the single-cell relaxation).
"""
import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, 8 TB/s
METRIC = "accepted collisions/s + particle-steps/s on 1 MI355X; learned vs exact majorant"

# algorithmic bytes per particle and launch, FP32 2-D with weights, 100
# particles per cell
ALGO_BYTES = {
    "stream": 17.0,    # read x, y, cx, cy; write one code byte (the gather advances the positions)
    # gather-collide: read the 28 B state (x, y, cx, cy, cz, w, id) and one
    # code byte, write the 28 B state into the new sequence, read and
    # write the cell's 26 FP64 running sums (416 B per cell of 100)
    "collide": 28.0 + 1.0 + 28.0 + 4.16,
}
VALU_PEAK_TOPS = 256 * 4 * 16 * 2.4e9 / 1e12  # 32-bit VALU lane operations per second (no FMA doubling)
PROFILE_DIR = os.path.join(ROOT, "profiles")
# weighted cavity runs: weights re-estimated every 4 steps, relative-speed
# majorant scaled by 1.5 (the weight update's 1 / (1 - p) at most 3)
VR_SETTINGS = {"vr_reconstruct": 4, "vr_kappa": 1.5}


def source_digest():
    """SHA-1 of the HIP sources: counter figures taken from a committed
    profile are used only while the kernels are unchanged."""
    import hashlib
    h = hashlib.sha1()
    csrc = os.path.join(ROOT, "paper_2301_05985_amd", "csrc")
    for f in sorted(os.listdir(csrc)):
        if f.endswith((".h", ".hip")):
            h.update(f.encode())
            h.update(open(os.path.join(csrc, f), "rb").read())
    return h.hexdigest()


def committed_counters(kernel, digest):
    """Per-launch counter figures of `kernel` from the committed rocprofv3
    summaries (lines `pmc: kernel=... key=value ... source_sha1=...`), or {}
    when none was taken with the current sources."""
    out = {}
    if not os.path.isdir(PROFILE_DIR):
        return out
    for f in sorted(os.listdir(PROFILE_DIR)):
        if not f.endswith(".md"):
            continue
        for line in open(os.path.join(PROFILE_DIR, f)):
            line = line.strip()
            if not line.startswith("pmc:"):
                continue
            kv = dict(t.split("=", 1) for t in line[4:].split() if "=" in t)
            if kv.get("kernel") == kernel and kv.get("source_sha1") == digest:
                out.update({k: float(v) for k, v in kv.items() if k not in ("kernel", "source_sha1")})
    return out


def _timed_steps(sim, torch, steps, warmup):
    sim.step(warmup)
    torch.cuda.synchronize()
    s = sim.stream
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    _, cnt0, _ = sim.sample()
    t0 = time.perf_counter()
    e0.record(s)
    sim.step(steps)
    e1.record(s)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms = e0.elapsed_time(e1)
    _, cnt1, _ = sim.sample()
    d = (cnt1.astype(np.int64) - cnt0.astype(np.int64)).sum(0)
    return ms, wall, int(d[0]), int(d[1])


def copy_rate(torch, nbytes=512 * 1024 * 1024, reps=4):
    """Bytes read plus written per second of a plain device-to-device copy
    between two already-touched buffers: the HBM rate a streaming kernel
    can reach on this device, beside the datasheet peak."""
    src = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        dst.copy_(src)
    e1.record()
    e1.synchronize()
    gbs = 2.0 * nbytes * reps / (e0.elapsed_time(e1) * 1e-3) / 1e9
    del src, dst
    torch.cuda.empty_cache()
    return gbs


def run_workload(name, p, parts, steps, warmup, torch):
    from paper_2301_05985_amd.binding import Simulation
    sim = Simulation(p, parts)
    ms, wall, cand, acc = _timed_steps(sim, torch, steps, warmup)
    diag = sim.diagnostics()
    n = len(parts["cx"])
    out = {
        "workload": name, "particles": n, "steps": steps, "ms_per_step": ms / steps,
        "overshoot_per_candidate": diag["overshoot"] / max(cand, 1),
        "particle_steps_per_s": n * steps / (ms * 1e-3),
        "collisions_per_s": acc / (ms * 1e-3), "candidates_per_s": cand / (ms * 1e-3),
        "acceptance": acc / max(cand, 1), "dtype": p.get("real", "f64"),
        "wall_clock_s": wall,
    }
    for k in ("learned_used", "fallback", "learned_skip", "overshoot", "vr_nonfinite", "big_cells"):
        out[k] = diag[k]
    sim.close()
    return out


def kernel_profile(sim, torch, steps, period=1):
    """Per-kernel durations (ms) from HIP events around every launch.  Each
    profile_step advances two steps and times the second; `extra` more steps
    between calls make the timed step index advance by a stride prime to
    `period` (the weight re-estimation interval), so over a multiple of
    `period` calls every residue of the step index modulo the period is
    timed equally often and the averages are those of consecutive steps."""
    acc = {}
    extra = 0
    if period > 1:
        steps = -(-steps // period) * period
        while math.gcd(2 + extra, period) != 1:
            extra += 1
    for i in range(steps):
        if extra and i > 0:
            sim.step(extra)
        for name, ms in sim.profile_step():
            acc.setdefault(name, []).append(ms)
    return {k: float(np.mean(v)) for k, v in acc.items()}


def host_cpu():
    """Model name and logical CPU count of the host (from /proc/cpuinfo)."""
    model, n = None, 0
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                n += 1
                model = model or line.split(":", 1)[1].strip()
    except OSError:
        pass
    return {"model": model, "logical_cpus": n or os.cpu_count()}


def _oracle_rate(p, parts, n_steps, dtype):
    import oracle
    orc = oracle.Oracle(p, parts, dtype)
    orc.run(1)  # the first step streams from the unsorted initial state, like the GPU warm-up
    acc0 = int(orc.counters[:, 1].sum())
    t0 = time.perf_counter()
    orc.run(n_steps)
    dt = time.perf_counter() - t0
    n = len(parts["cx"])
    acc = int(orc.counters[:, 1].sum()) - acc0  # accepted in the timed steps only
    return n * n_steps / dt, acc / dt, dt


def cpu_baseline(p, parts, n_steps, n_steps64):
    """The oracle on one host core: its double-precision build (the plain
    FP64 reference) and its single-precision build (the decisions of the
    FP32 path), each on a bounded number of steps of the same workload."""
    v64, c64, t64 = _oracle_rate(p, parts, n_steps64, np.float64)
    v32, c32, t32 = _oracle_rate(p, parts, n_steps, np.float32)
    return {"value": v64, "unit": "particle-steps/s", "cores": 1, "kind": "oracle",
            "sample": "%d steps of the same workload after 1 untimed step, FP64 oracle build, single-threaded "
                      "(%.1f s)" % (n_steps64, t64),
            "collisions_per_s": c64, "host": host_cpu(),
            "fp32_build": {"value": v32, "collisions_per_s": c32, "steps": n_steps, "seconds": t32}}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--kn", type=float, default=0.01)
    ap.add_argument("--no-secondary", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--cpu-steps", type=int, default=10)
    ap.add_argument("--cpu-steps64", type=int, default=6)
    ap.add_argument("--profile-steps", type=int, default=12)
    ap.add_argument("--launch", default=None,
                    help="headline launch parameters as JSON (e.g. '{\"cells_per_wave\": 2}') instead of "
                         "timing the candidates, so that a profiled run launches only the timed kernels")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="also run one plain 512 MiB device-to-device copy (reference for HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on exactly one GPU: there is no multi-GPU path "
              "(the slab decomposition with particle migration is a design note only)", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2301_05985_amd import workloads as W
    from paper_2301_05985_amd.binding import Simulation

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    torch.cuda.set_device(0)

    if args.calibrate_copy:
        src = torch.ones(128 * 1024 * 1024, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        print("[bench] calibration copy: 536870912 bytes read, 536870912 bytes written", file=sys.stderr, flush=True)
        del src, dst
        torch.cuda.empty_cache()
    copy_gbs = copy_rate(torch)
    print("[bench] plain device copy (warm, 512 MiB): %.0f GB/s read + written" % copy_gbs, file=sys.stderr,
          flush=True)

    # ---------------- headline: full-size cavity
    from paper_2301_05985_amd import autotune
    tlog = lambda s: print("[bench] " + s, file=sys.stderr, flush=True)
    p, parts = W.cavity(Kn=args.kn, real="f32")
    p.update(VR_SETTINGS)
    name = "cavity 256x256 cells x 100 particles (6,553,600), Kn=%g, diffuse walls, lid 0.01*sqrt(2), " \
           "VR weights re-estimated every 4 steps, majorant factor 1.5, FP32 state / FP64 sums" % args.kn
    print("[bench] headline: %s" % name, file=sys.stderr, flush=True)
    # launch of the collision step (one or two cells per wave, or four waves
    # per cell; identical decisions either way), picked by timing them
    if args.launch:
        launch, launch_times = json.loads(args.launch), {}
    else:
        launch, launch_times = autotune.tune(p, parts, log=tlog)
    p.update(launch)
    sim = Simulation(p, parts)
    ms, wall, cand, acc = _timed_steps(sim, torch, args.steps, args.warmup)
    n = len(parts["cx"])
    value = n * args.steps / (ms * 1e-3)
    print("[bench] timed %d steps: %.3f ms/step" % (args.steps, ms / args.steps), file=sys.stderr, flush=True)
    prof = kernel_profile(sim, torch, args.profile_steps, period=max(int(p.get("vr_reconstruct", 0)), 1))
    diag = sim.diagnostics()
    sim.close()
    del sim
    torch.cuda.empty_cache()
    # dominant kernel and its roofline (HBM bound)
    kname = max(prof, key=prof.get)
    digest = source_digest()
    pmc = committed_counters(kname, digest)
    per_kernel = {}
    for k, v in prof.items():
        gbs = ALGO_BYTES[k] * n / (v * 1e-3) / 1e9 if k in ALGO_BYTES else None
        per_kernel[k] = {"ms": v, "algo_GBps": gbs, "frac": (gbs / HBM_PEAK_GBS) if gbs else None,
                         "frac_of_copy": (gbs / copy_gbs) if gbs else None}
    achieved = per_kernel[kname]["algo_GBps"]
    # HBM bytes per launch from the committed FETCH_SIZE / WRITE_SIZE passes
    # (already scaled by the plain-copy calibration), while the kernels match
    traffic = pmc.get("hbm_bytes")
    roof = {"bound": "hbm", "kernel": kname, "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS if achieved else None, "traffic": traffic,
            "copy_GBps": copy_gbs,
            "traffic_GBps": (traffic / (prof[kname] * 1e-3) / 1e9) if traffic else None,
            "per_kernel": per_kernel, "source_sha1": digest}
    if pmc.get("valu_insts"):
        # the collision kernel is limited by vector-ALU issue, not HBM: the
        # executed VALU lane operations per launch (committed SQ_INSTS_VALU
        # x 64) over the live duration, against the 32-bit VALU issue peak
        ops = pmc["valu_insts"] * 64.0
        roof["valu"] = {"achieved": ops / (prof[kname] * 1e-3) / 1e12, "peak": VALU_PEAK_TOPS, "unit": "TOP/s",
                        "frac": ops / (prof[kname] * 1e-3) / 1e12 / VALU_PEAK_TOPS,
                        "insts_per_cell": pmc["valu_insts"] / 65536.0, "kind": "executed, not algorithmic"}

    line = {
        "metric": METRIC, "value": value, "unit": "particle-steps/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms / args.steps,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": name, "particles": n, "cells": 65536, "Kn": args.kn, "dt": p["dt"],
                   "launch": launch, "parallelism": "single GPU"},
        "launch_candidates_ms_per_step": launch_times,
        "collisions_per_s": acc / (ms * 1e-3), "candidates_per_s": cand / (ms * 1e-3),
        "acceptance": acc / max(cand, 1),
        "diagnostics": {k: diag[k] for k in ("steps", "overshoot", "wall_hits", "vr_nonfinite", "big_cells")},
        "roofline": roof,
    }

    if not args.no_secondary:
        sec = []
        print("[bench] secondary workloads", file=sys.stderr, flush=True)

        def walled(label, q, qparts, steps, warm):
            # the walled launch (one or two cells per wave, four waves per
            # cell) picked by timing the candidates
            best, times = autotune.tune(q, qparts, log=tlog)
            r = run_workload(label, dict(q, **best), qparts, steps, warm, torch)
            r["launch"], r["launch_candidates_ms_per_step"] = best, times
            return r

        p2, parts2 = W.fourier(real="f32")
        p2.update(vr_reconstruct=1, vr_kappa=1.5)
        sec.append(walled("fourier 200 cells x 200 (40,000), Kn=0.1, VR re-estimated every step, majorant "
                          "factor 1.5, FP32", p2, parts2, 2000, 100))
        p3, parts3 = W.batched(real="f32")
        # launch parameters of the collision step picked by the autotuner
        # (grid vs persistent work queue; identical results either way)
        best3, times3 = autotune.tune(p3, parts3, steps=20, warmup=8, log=tlog)
        r3 = run_workload("batched 4096 cells, N uniform in [50,2000], exact majorant, FP32",
                          dict(p3, **best3), parts3, 200, 20, torch)
        r3["launch"], r3["launch_candidates_ms_per_step"] = best3, times3
        sec.append(r3)
        p3d = dict(p3, majorant=2)
        sec.append(run_workload("batched 4096 cells, largest-pair-speed majorant (O(N^2)), FP32", p3d, parts3,
                                20, 2, torch))
        # learned majorant: train on exact-majorant runs (seeds 1-4, held-out seed 5), then time it
        from paper_2301_05985_amd import learned
        t0 = time.perf_counter()
        model = learned.train_model(log=lambda s: print("[bench] " + s, file=sys.stderr, flush=True))
        t_train = time.perf_counter() - t0
        p5 = dict(p3, majorant=1)
        n3 = len(parts3["cx"])
        cells = 4096 * 220
        # the calibration's table: per cell-size bin, at the chosen margin,
        # the candidates a verified proposal saves and what the network and
        # the verification cost (candidate-equivalents per step of 4096 cells)
        tab = model["calibration"]
        j = int(round((model["delta"] + 0.64) / 0.01))
        edges = [2] + [64 << b for b in range(7)]
        breakeven = [{"cells_from_N": edges[b], "saved": float(tab[j, b, 0]), "cost": float(tab[j, b, 1]),
                      "used": int(tab[j, b, 2]), "fallback": int(tab[j, b, 3])} for b in range(tab.shape[1])]
        for label, gate in (("calibrated size gate", model["min_n"]), ("every cell", 0)):
            m5 = dict(model, min_n=gate)
            best5, times5 = autotune.tune(p5, parts3, steps=20, warmup=8, model=(m5["bits"], m5["delta"], gate),
                                          log=tlog)
            sim5 = learned.simulation_with_model(dict(p5, **best5), parts3, m5)
            ms5, wall5, cand5, acc5 = _timed_steps(sim5, torch, 200, 20)
            d5 = sim5.diagnostics()
            sim5.close()
            sec.append({"workload": "batched 4096 cells, learned majorant (verified, exact-bound fallback), %s, "
                                    "FP32" % label,
                        "particles": n3, "steps": 200, "min_n": gate,
                        "ms_per_step": ms5 / 200, "particle_steps_per_s": n3 * 200 / (ms5 * 1e-3),
                        "collisions_per_s": acc5 / (ms5 * 1e-3), "candidates_per_s": cand5 / (ms5 * 1e-3),
                        "acceptance": acc5 / max(cand5, 1), "learned_used_frac": d5["learned_used"] / cells,
                        "fallback_frac": d5["fallback"] / cells, "skip_frac": d5["learned_skip"] / cells,
                        "overshoot": d5["overshoot"], "overshoot_per_candidate": d5["overshoot"] / max(cand5, 1),
                        "delta": model["delta"], "train_samples": model["n_train"],
                        "launch": best5, "launch_candidates_ms_per_step": times5,
                        "train_loss": model["loss_history"], "train_seconds": t_train,
                        "calibration_at_delta": breakeven})
        p6 = dict(p3, molecule=W.VHS, omega=0.81)
        sec.append(run_workload("batched 4096 cells, variable hard spheres (omega 0.81), exact majorant, FP32",
                                dict(p6, **best3), parts3, 200, 20, torch))
        p6s = dict(p3, molecule=W.VSS, omega=0.81, alpha=1.4)
        sec.append(run_workload("batched 4096 cells, variable soft spheres (omega 0.81, alpha 1.4), exact majorant, "
                                "FP32", dict(p6s, **best3), parts3, 200, 20, torch))
        p7, parts7 = W.cavity(Kn=args.kn, real="f32")
        p7 = dict(p7, molecule=W.VHS, omega=0.74, **VR_SETTINGS)
        sec.append(walled("cavity 256x256 x 100, variable hard spheres (omega 0.74), VR, FP32", p7, parts7, 100, 10))
        p7s = dict(p7, molecule=W.VSS, alpha=1.4)
        sec.append(walled("cavity 256x256 x 100, variable soft spheres (omega 0.74, alpha 1.4), VR, FP32", p7s,
                          parts7, 100, 10))
        # the rest of the cavity's Knudsen sweep
        for kn in (0.1, 1.0):
            if kn == args.kn:
                continue
            pk, partsk = W.cavity(Kn=kn, real="f32")
            pk.update(VR_SETTINGS)
            sec.append(walled("cavity 256x256 x 100, Kn=%g, VR, FP32" % kn, pk, partsk, 100, 10))
        # the same cavity without importance weights (plain DSMC estimators)
        p8, parts8 = W.cavity(Kn=args.kn, real="f32", vr=0)
        sec.append(walled("cavity 256x256 x 100, Kn=%g, no weights, FP32" % args.kn, p8, parts8, 100, 10))
        p1, parts1 = W.relaxation()
        sec.append(run_workload("relaxation 10,000 particles one cell FP64", p1, parts1, 200, 0, torch))
        line["secondary"] = sec

    if not args.no_cpu:
        print("[bench] cpu baseline (oracle)", file=sys.stderr, flush=True)
        line["cpu_baseline"] = cpu_baseline(p, parts, args.cpu_steps, args.cpu_steps64)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
