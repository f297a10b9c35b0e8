"""Seeded synthetic workloads: run parameters and initial particle states.

This module holds no step of the method.  It only draws initial states with
numpy's own generator (PCG64, seeded) and states the physical parameters of
each workload, so that the GPU path and the CPU oracle start from identical
bits.  Units: Boltzmann constant and molecular mass are 1, so temperatures are
squared speeds and the reference temperature is 1.

Workloads (sizes as run by the benchmark and the full-size tests):
  relaxation  one homogeneous cell, two shifted Maxwellians relaxing to one
  fourier     1-D heat transfer between diffuse walls at T=1 and T=2
  batched     thousands of independent homogeneous cells of uneven size
  cavity      2-D lid-driven cavity with diffuse walls
  bkw         homogeneous Maxwell-molecule cell started on the BKW solution
Every builder takes size arguments so the tests can run reduced versions.
"""
import math

import numpy as np

WALL_DIFFUSE, WALL_SPECULAR, WALL_PERIODIC = 0, 1, 2
HARD_SPHERE, MAXWELL, VHS, VSS = 0, 1, 2, 3


def _maxwellian(rng, n, T):
    return rng.standard_normal((3, n)) * math.sqrt(T)


def _base(**kw):
    p = dict(dims=0, n_cells=(1, 1), length=(1.0, 1.0), dt=0.05, sigma=1.0, FN=1.0,
             molecule=HARD_SPHERE, vr=0, vr_T0=1.0, vr_n0=0.0, wall_kind=(0, 0, 0, 0),
             wall_T=(1.0, 1.0, 1.0, 1.0), wall_u=((0.0, 0.0, 0.0),) * 4, seed=0,
             majorant=0, real="f64", max_wall_hits=64)
    p.update(kw)
    return p


def relaxation(N=10000, steps=200, seed=0, shift=1.5, molecule=HARD_SPHERE, real="f64",
               dt=0.05, init_seed=None):
    """One homogeneous cell: two equal-weight Maxwellians (T=1) shifted by +-shift
    along x.  The first ceil(N/2) particles take +shift.  The volume makes the
    equilibrium mean collision time 1 for hard spheres of unit cross-section
    at the equilibrium temperature T_eq = 1 + shift^2 / 3."""
    rng = np.random.default_rng(seed if init_seed is None else init_seed)
    c = _maxwellian(rng, N, 1.0)
    h = (N + 1) // 2
    c[0, :h] += shift
    c[0, h:] -= shift
    Teq = 1.0 + shift * shift / 3.0
    if molecule == HARD_SPHERE:
        V = N * 1.0 * 4.0 * math.sqrt(Teq / math.pi)  # n sigma <g> = 1
        sigma = 1.0
    else:
        V = float(N)   # Maxwell molecules: sigma g = K = 1, nu = n K = 1
        sigma = 1.0
    p = _base(dims=0, n_cells=(1, 1), dt=dt, sigma=sigma, FN=1.0, molecule=molecule,
              seed=seed, real=real, steps=steps, cell_volume=np.array([V]),
              inst_offset=np.array([0, N], dtype=np.int64), T_eq=Teq,
              workload="relaxation N=%d" % N)
    parts = dict(cx=c[0], cy=c[1], cz=c[2], id=np.arange(N, dtype=np.uint32))
    return p, parts


def bkw(N=2000, n_inst=1, K0=0.6, seed=0, dt=0.02, steps=100, real="f64", init_seed=None):
    """Maxwell molecules (sigma g = K = 1, unit density so nu = 1) started on the
    BKW similarity solution at T = 1 with scale K0 (3/5 <= K0 <= 1): with weight
    A = (5 K0 - 3) / (2 K0) a Gaussian of variance K0, otherwise a 5-dof
    chi radius scaled by sqrt(K0) in a uniform direction."""
    rng = np.random.default_rng(seed if init_seed is None else init_seed)
    tot = N * n_inst
    A = (5.0 * K0 - 3.0) / (2.0 * K0)
    c = rng.standard_normal((3, tot)) * math.sqrt(K0)
    second = rng.random(tot) >= A
    m = int(second.sum())
    r = np.sqrt(rng.chisquare(5, m) * K0)
    d = rng.standard_normal((3, m))
    d /= np.linalg.norm(d, axis=0)
    c[:, second] = d * r
    off = np.arange(n_inst + 1, dtype=np.int64) * N
    p = _base(dims=0, n_cells=(n_inst, 1), dt=dt, sigma=1.0, FN=1.0, molecule=MAXWELL,
              seed=seed, real=real, steps=steps, cell_volume=np.full(n_inst, float(N)),
              inst_offset=off, K0=K0, workload="bkw N=%d x %d" % (N, n_inst))
    return p, dict(cx=c[0], cy=c[1], cz=c[2], id=np.arange(tot, dtype=np.uint32))


def batched(n_inst=4096, nmin=50, nmax=2000, seed=0, steps=500, real="f32", dt=0.05,
            sigma=None, init_seed=None):
    """Independent homogeneous cells (unit volume) with particle counts uniform on
    [nmin, nmax] and bimodal initial states: Maxwellians at T=1 shifted by
    +-a along x, a uniform on [0.5, 2].  The cross-section makes
    n sigma <g> = 1 at the mean count and T = 1."""
    rng = np.random.default_rng(seed if init_seed is None else init_seed)
    counts = rng.integers(nmin, nmax + 1, size=n_inst)
    shift = rng.uniform(0.5, 2.0, size=n_inst)
    off = np.zeros(n_inst + 1, dtype=np.int64)
    off[1:] = np.cumsum(counts)
    tot = int(off[-1])
    c = _maxwellian(rng, tot, 1.0)
    for b in range(n_inst):
        s, e = off[b], off[b + 1]
        h = (e - s + 1) // 2
        c[0, s:s + h] += shift[b]
        c[0, s + h:e] -= shift[b]
    nbar = 0.5 * (nmin + nmax)
    if sigma is None:
        sigma = math.sqrt(math.pi) / (4.0 * nbar)
    p = _base(dims=0, n_cells=(n_inst, 1), dt=dt, sigma=sigma, FN=1.0, seed=seed, real=real,
              steps=steps, cell_volume=np.ones(n_inst), inst_offset=off, shifts=shift,
              workload="batched %d cells N in [%d,%d]" % (n_inst, nmin, nmax))
    return p, dict(cx=c[0], cy=c[1], cz=c[2], id=np.arange(tot, dtype=np.uint32))


def fourier(n_cells=200, per_cell=200, Kn=0.1, T_left=1.0, T_right=2.0, T0=1.5, dt=1e-3,
            steps=20000, seed=0, vr=1, real="f32", sigma=None, init_seed=None):
    """1-D slab 0 <= x <= 1 between diffuse walls at T_left and T_right, uniform
    initial positions, Maxwellian T0 at rest, weights 1.  Hard spheres with
    mean free path Kn * L at the mean density (unit area, F_N = 1)."""
    rng = np.random.default_rng(seed if init_seed is None else init_seed)
    N = n_cells * per_cell
    x = rng.random(N)
    c = _maxwellian(rng, N, T0)
    n = float(N)  # number density over unit length and area
    if sigma is None:
        sigma = 1.0 / (math.sqrt(2.0) * n * Kn) if Kn > 0 else 0.0
    p = _base(dims=1, n_cells=(n_cells, 1), length=(1.0, 1.0), dt=dt, sigma=sigma, FN=1.0,
              vr=vr, vr_T0=T0, vr_n0=n, wall_kind=(WALL_DIFFUSE, WALL_DIFFUSE, 0, 0),
              wall_T=(T_left, T_right, 1.0, 1.0), seed=seed, real=real, steps=steps,
              burn_in=steps // 4, workload="fourier %d cells x %d, Kn=%g" % (n_cells, per_cell, Kn))
    return p, dict(x=x, cx=c[0], cy=c[1], cz=c[2], w=np.ones(N), id=np.arange(N, dtype=np.uint32))


def cavity(nx=256, ny=256, per_cell=100, Kn=0.01, lid=0.01 * math.sqrt(2.0), T=1.0, steps=10000,
           seed=0, vr=1, real="f32", dt=None, sigma=None, init_seed=None):
    """Unit square with diffuse walls at T; the lid y = 1 moves along +x at
    `lid` (default 1% of the most probable speed sqrt(2T)).  Hard spheres with
    mean free path Kn at the mean density; dt = 0.3 dx / sqrt(2)."""
    rng = np.random.default_rng(seed if init_seed is None else init_seed)
    N = nx * ny * per_cell
    pos = rng.random((2, N))
    c = _maxwellian(rng, N, T)
    n = float(N)
    if sigma is None:
        sigma = 1.0 / (math.sqrt(2.0) * n * Kn)
    if dt is None:
        dt = 0.3 * (1.0 / nx) / math.sqrt(2.0)
    p = _base(dims=2, n_cells=(nx, ny), length=(1.0, 1.0), dt=dt, sigma=sigma, FN=1.0, vr=vr,
              vr_T0=T, vr_n0=n, wall_kind=(WALL_DIFFUSE,) * 4, wall_T=(T,) * 4,
              wall_u=((0.0, 0.0, 0.0), (0.0, 0.0, 0.0), (0.0, 0.0, 0.0), (lid, 0.0, 0.0)),
              seed=seed, real=real, steps=steps, burn_in=steps // 2,
              workload="cavity %dx%d x %d, Kn=%g" % (nx, ny, per_cell, Kn))
    return p, dict(x=pos[0], y=pos[1], cx=c[0], cy=c[1], cz=c[2], w=np.ones(N),
                   id=np.arange(N, dtype=np.uint32))


def shuffle_storage(parts, seed=1):
    """Permute the storage order of a walled workload (ids travel with particles)."""
    rng = np.random.default_rng(seed)
    n = len(parts["cx"])
    o = rng.permutation(n)
    return {k: (np.asarray(v)[o] if v is not None else None) for k, v in parts.items()}
