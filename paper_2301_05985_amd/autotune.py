"""Launch-parameter autotuner.

The collision step of many independent homogeneous cells can run as one
workgroup per instance (``schedule=0``, grid launch in longest-first order)
or as a persistent grid of ``persistent_waves`` single-wave workgroups that
take work units from per-XCD device queues (``schedule=1``); a unit groups
consecutive small instances of the longest-first order while they hold
fewer than ``chunk_work`` particles.  The choice changes only the order in which
instances are processed, never their arithmetic (every draw is keyed by
instance, step and candidate), so all candidates give identical results and
the tuner may pick purely on time.

When the grid schedule wins, two of its kernel parameters are refined one at
a time (coordinate descent from the defaults): ``wide_min``, the size above
which an instance runs on a four-wave workgroup instead of one wave, and, for
weighted runs, ``occupancy``, the waves per SIMD the one-wave kernel is
compiled for (5, or 6 with a few register spills).  Neither changes a bit of
the result either.

Walled workloads (dims 1, 2) choose between one cell per wave, two cells
per wave (``cells_per_wave``, 32 lanes per cell; mean cell population at
most 128) and a workgroup of four waves per cell (``waves_per_cell``), the
last two with the exact or brute-force majorant, again without changing a
decision of the method.

The tuner times each candidate on a scratch simulation built from a copy of
the caller's initial state and caches the winner in a JSON file keyed by the
GPU architecture and a signature of the workload (kind, precision, weights,
majorant, and the instance-size histogram or the grid).
"""
import hashlib
import json
import os

import numpy as np

GRID = {"schedule": 0}
CANDIDATES = [GRID] + [
    {"schedule": 1, "persistent_waves": w, "chunk_work": c}
    for w in (1024, 2048, 4096) for c in (0, 256, 1024)
]
LAUNCH_KEYS = ("schedule", "persistent_waves", "chunk_work", "wide_min", "occupancy", "cells_per_wave",
               "waves_per_cell")
WALLED = [{"cells_per_wave": 1}, {"cells_per_wave": 2}, {"waves_per_cell": 4}]
# refinements of the grid schedule, each tried against the best so far
WIDE_MIN = (128, 256, 384, 512, 768, 2048)
OCCUPANCY = (6,)


def cache_path():
    base = os.environ.get("DSMC_AUTOTUNE_CACHE")
    if base:
        return base
    return os.path.join(os.path.expanduser("~"), ".cache", "dsmc_hip", "autotune.json")


def pair_allowed(params, n_particles):
    """Whether a walled workload may run two cells per wave."""
    if params.get("dims", 0) == 0 or params.get("majorant", 0) == 1:
        return False
    nc = int(np.prod(params["n_cells"][:params["dims"]]))
    return n_particles <= 128 * nc


def walled_candidates(params, n_particles):
    """Launches a walled workload may take (the first is the default)."""
    if params.get("dims", 0) == 0:
        return []
    out = [dict(WALLED[0])]
    if pair_allowed(params, n_particles):
        out.append(dict(WALLED[1]))
    if params.get("majorant", 0) != 1:
        out.append(dict(WALLED[2]))
    return out


def signature(params, n_particles=0):
    """Key of a workload: everything that changes the collision kernel's cost."""
    # the collision rate (sigma, dt) sets the candidates per cell
    rate = "s%.6g_t%.6g" % (params.get("sigma", 0.0), params.get("dt", 0.0))
    if params.get("dims", 0) != 0:
        return "d%d_%s_vr%d_re%d_ka%g_m%d_mol%d_c%s_n%d_%s" % (
            params["dims"], params.get("real", "f64"), params.get("vr", 0), params.get("vr_reconstruct", 0),
            params.get("vr_kappa", 1.0), params.get("majorant", 0), params.get("molecule", 0),
            "x".join(str(int(c)) for c in params["n_cells"][:params["dims"]]), n_particles, rate)
    off = np.asarray(params["inst_offset"], dtype=np.int64)
    n = np.diff(off)
    hist = np.bincount(np.minimum(n // 64, 255), minlength=256)
    h = hashlib.sha1(hist.astype(np.int64).tobytes()).hexdigest()[:16]
    return "d%d_%s_vr%d_m%d_mol%d_k%d_n%d_%s_%s" % (
        params.get("dims", 0), params.get("real", "f64"), params.get("vr", 0),
        params.get("majorant", 0), params.get("molecule", 0), len(n), int(off[-1]), h, rate)


def _arch():
    import torch
    return torch.cuda.get_device_properties(0).gcnArchName.split(":")[0]


def _load_cache(path):
    try:
        with open(path) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def _store_cache(path, table):
    os.makedirs(os.path.dirname(path) or ".", exist_ok=True)
    tmp = path + ".tmp%d" % os.getpid()
    with open(tmp, "w") as f:
        json.dump(table, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def time_candidate(params, particles, cand, steps=8, warmup=8, model=None):
    """Milliseconds per step of one launch candidate on a scratch simulation."""
    import torch
    from .binding import Simulation
    sim = Simulation(dict(params, **cand), particles)
    try:
        if model is not None:
            sim.set_majorant_model(*model)
        sim.step(warmup)
        torch.cuda.synchronize()
        t0, t1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        t0.record()
        sim.step(steps)
        t1.record()
        t1.synchronize()
        return t0.elapsed_time(t1) / steps
    finally:
        sim.close()


def refinements(params, best):
    """Axes (key, values) of the second stage for a first-stage winner."""
    if best.get("schedule", 0) != 0:
        return []
    axes = [("wide_min", WIDE_MIN)]
    if params.get("vr", 0):
        axes.append(("occupancy", OCCUPANCY))
    return axes


def tune(params, particles, candidates=None, steps=8, warmup=8, model=None, use_cache=True, log=None,
         refine=None):
    """Return (best launch parameters, {candidate label: ms per step}).

    Walled workloads time the launches of ``walled_candidates`` (one cell
    per wave untimed where it is the only one).
    ``model`` is ``(bf16_weights, delta, min_n)`` for learned-majorant runs.
    ``refine`` (default: only when ``candidates`` is not given) adds the
    coordinate-descent stage over the grid schedule's kernel parameters."""
    walled = params.get("dims", 0) != 0
    n_particles = len(particles["cx"])
    if walled:
        allowed = walled_candidates(params, n_particles)
        if len(allowed) == 1:
            return allowed[0], {}
        candidates = candidates or allowed
        refine = False
        steps = max(steps, 24)  # every phase of a re-estimation interval, several times
    key = "%s/%s" % (_arch(), signature(params, n_particles))
    path = cache_path()
    if use_cache:
        hit = _load_cache(path).get(key)
        if hit is not None:
            return {k: hit["best"][k] for k in hit["best"] if k in LAUNCH_KEYS}, hit.get("times", {})
    if refine is None:
        refine = candidates is None
    times = {}
    best, best_t = None, float("inf")

    def run(cands):
        nonlocal best, best_t
        for cand in cands:
            label = json.dumps(cand, sort_keys=True)
            t = time_candidate(params, particles, cand, steps, warmup, model)
            times[label] = t
            if log:
                log("autotune %s: %.4f ms/step" % (label, t))
            if t < best_t:
                best, best_t = dict(cand), t

    run(candidates or CANDIDATES)
    if refine:
        for axis, values in refinements(params, best):
            run([dict(best, **{axis: v}) for v in values])
    if use_cache:
        table = _load_cache(path)
        table[key] = {"best": best, "times": times}
        _store_cache(path, table)
    return best, times
