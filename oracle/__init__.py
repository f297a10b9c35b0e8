"""CPU oracle of the DSMC hot path (ctypes wrapper around dsmc_oracle.c).

TEST INFRASTRUCTURE.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this package.  The product
path (``paper_2301_05985_amd``) never imports it and shares no code with it.

The C source is compiled here with gcc (``-O2 -ffp-contract=off``), twice:
once in double precision (functions suffixed ``_f64``) and once in single
precision (``_f32``).  ``build()`` is idempotent and is also called by the
package build step, so that the checker exists wherever the product is built.
"""
import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "dsmc_oracle.c")
_LIB = os.path.join(_HERE, "_build", "liboracle_dsmc.so")

NSUM = 26
MLP_NPARAM = 64 * 6 + 64 + 64 * 64 + 64 + 64 + 1  # 4673

WALL_DIFFUSE, WALL_SPECULAR, WALL_PERIODIC = 0, 1, 2
HARD_SPHERE, MAXWELL, VHS, VSS = 0, 1, 2, 3


def build(force=False):
    """Compile the oracle shared library with gcc; returns its path."""
    os.makedirs(os.path.dirname(_LIB), exist_ok=True)
    if (not force and os.path.exists(_LIB)
            and os.path.getmtime(_LIB) >= os.path.getmtime(_SRC)):
        return _LIB
    objs = []
    flags = ["-O2", "-fPIC", "-ffp-contract=off", "-fno-fast-math", "-std=c11", "-Wall"]
    for real, sfx, extra in (("double", "_f64", ["-DORC_PRIMARY"]), ("float", "_f32", [])):
        obj = os.path.join(os.path.dirname(_LIB), "oracle%s.o" % sfx)
        subprocess.check_call(["gcc", *flags, "-DREAL=" + real, "-DSFX=" + sfx, *extra,
                               "-c", _SRC, "-o", obj])
        objs.append(obj)
    tmp = _LIB + ".tmp%d" % os.getpid()
    subprocess.check_call(["gcc", "-shared", "-o", tmp, *objs, "-lm"])
    os.replace(tmp, _LIB)
    return _LIB


class OrcCfg(ctypes.Structure):
    _fields_ = [
        ("dims", ctypes.c_int32), ("nx", ctypes.c_int32), ("ny", ctypes.c_int32),
        ("molecule", ctypes.c_int32),
        ("vr", ctypes.c_int32), ("majorant", ctypes.c_int32), ("n_inst", ctypes.c_int32),
        ("max_wall_hits", ctypes.c_int32),
        ("Lx", ctypes.c_double), ("Ly", ctypes.c_double), ("dt", ctypes.c_double),
        ("sigma", ctypes.c_double), ("FN", ctypes.c_double), ("vr_T0", ctypes.c_double),
        ("wall_kind", ctypes.c_int32 * 4),
        ("wall_T", ctypes.c_double * 4),
        ("wall_u", ctypes.c_double * 12),
        ("key", ctypes.c_uint32 * 2),
        ("cell_volume", ctypes.c_void_p),
        ("inst_offset", ctypes.c_void_p),
        ("mlp", ctypes.c_void_p),
        ("mlp_delta", ctypes.c_double),
        ("cell_ids", ctypes.c_void_p),
        ("only_cells", ctypes.c_void_p),
        ("n_only", ctypes.c_int64),
        ("omega", ctypes.c_double),
        ("alpha", ctypes.c_double),
        ("vr_reconstruct", ctypes.c_int32),
        ("pad_", ctypes.c_int32),
        ("vr_kappa", ctypes.c_double),
        ("mlp_min_n", ctypes.c_int64),
    ]


class OrcDiag(ctypes.Structure):
    _fields_ = [("overshoot", ctypes.c_uint64), ("wall_hits", ctypes.c_uint64),
                ("learned_used", ctypes.c_uint64), ("fallback", ctypes.c_uint64),
                ("learned_skip", ctypes.c_uint64), ("vr_nonfinite", ctypes.c_uint64),
                ("error", ctypes.c_int64)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        _lib = ctypes.CDLL(build())
        P = ctypes.c_void_p
        for sfx in ("_f64", "_f32"):
            f = getattr(_lib, "orc_run" + sfx)
            f.restype = ctypes.c_int
            f.argtypes = [P, ctypes.c_int64, P, P, P, P, P, P, P, P, ctypes.c_int64, ctypes.c_int32,
                          P, P, P, P]
            g = getattr(_lib, "orc_initial_layout" + sfx)
            g.restype = None
            g.argtypes = [P, ctypes.c_int64, P, P, P, P]
            for name in ("orc_exact_bound", "orc_diameter"):
                g = getattr(_lib, name + sfx)
                g.restype = ctypes.c_double
                g.argtypes = [P, P, P, P, ctypes.c_int64]
            g = getattr(_lib, "orc_direction" + sfx)
            g.restype = None
            g.argtypes = [P, ctypes.c_uint32, ctypes.c_uint32, ctypes.c_uint32, P]
            g = getattr(_lib, "orc_wall_draw" + sfx)
            g.restype = None
            g.argtypes = [P, ctypes.c_uint32, ctypes.c_uint32, ctypes.c_uint32, ctypes.c_double, P]
            g = getattr(_lib, "orc_wall_ratio" + sfx)
            g.restype = ctypes.c_double
            g.argtypes = [P, ctypes.c_double, P, ctypes.c_double]
            g = getattr(_lib, "orc_vr_update" + sfx)
            g.restype = None
            g.argtypes = [ctypes.c_int, ctypes.c_double, P, P]
            g = getattr(_lib, "orc_scatter" + sfx)
            g.restype = None
            g.argtypes = [P, P, ctypes.c_double if sfx == "_f64" else ctypes.c_float, P]
            g = getattr(_lib, "orc_scatter_vss" + sfx)
            g.restype = None
            g.argtypes = [P, P, P, ctypes.c_double]
            g = getattr(_lib, "orc_pair" + sfx)
            g.restype = None
            g.argtypes = [P, ctypes.c_uint32, ctypes.c_uint32, ctypes.c_uint32, ctypes.c_uint32,
                          P, P, P]
            g = getattr(_lib, "orc_mlp_forward_f32" + sfx)
            g.restype = ctypes.c_float
            g.argtypes = [P, P]
            g = getattr(_lib, "orc_features" + sfx)
            g.restype = None
            g.argtypes = [P, P, P, P, ctypes.c_int64, ctypes.c_double, ctypes.c_double, P]
            g = getattr(_lib, "orc_vr_reconstruct" + sfx)
            g.restype = ctypes.c_int
            g.argtypes = [P, P, P, P, P, ctypes.c_int64, ctypes.c_double]
            g = getattr(_lib, "orc_cell_of" + sfx)
            g.restype = ctypes.c_int64
            if sfx == "_f64":
                g.argtypes = [P, ctypes.c_double, ctypes.c_double]
            else:
                g.argtypes = [P, ctypes.c_float, ctypes.c_float]
        _lib.orc_vhs_pow.restype = ctypes.c_double
        _lib.orc_vhs_pow.argtypes = [ctypes.c_double, ctypes.c_double]
        _lib.orc_philox4x32_10.restype = None
        _lib.orc_philox4x32_10.argtypes = [P, P, P]
    return _lib


def _ptr(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _sfx(dtype):
    return "_f64" if np.dtype(dtype) == np.float64 else "_f32"


def philox(ctr, key):
    c = np.ascontiguousarray(ctr, dtype=np.uint32)
    k = np.ascontiguousarray(key, dtype=np.uint32)
    out = np.zeros(4, dtype=np.uint32)
    lib().orc_philox4x32_10(_ptr(c), _ptr(k), _ptr(out))
    return out


def seed_key(seed):
    """Philox key words of a 64-bit seed: (low word, high word)."""
    seed = int(seed) & 0xFFFFFFFFFFFFFFFF
    return (seed & 0xFFFFFFFF, seed >> 32)


def make_cfg(p):
    """Oracle configuration from a workload parameter dict (see workloads.py)."""
    c = OrcCfg()
    c.dims = p["dims"]
    c.nx, c.ny = p["n_cells"]
    c.molecule = p.get("molecule", HARD_SPHERE)
    c.vr = int(p.get("vr", 0))
    c.majorant = int(p.get("majorant", 0))
    c.n_inst = p["n_cells"][0] if p["dims"] == 0 else 0
    c.max_wall_hits = p.get("max_wall_hits", 64)
    c.Lx, c.Ly = p.get("length", (1.0, 1.0))
    c.dt, c.sigma, c.FN = p["dt"], p["sigma"], p["FN"]
    c.vr_T0 = p.get("vr_T0", 1.0)
    for k in range(4):
        c.wall_kind[k] = p.get("wall_kind", (0, 0, 0, 0))[k]
        c.wall_T[k] = p.get("wall_T", (1.0, 1.0, 1.0, 1.0))[k]
        for d in range(3):
            c.wall_u[3 * k + d] = p.get("wall_u", ((0, 0, 0),) * 4)[k][d]
    c.key[0], c.key[1] = seed_key(p.get("seed", 0))
    c.mlp_delta = p.get("mlp_delta", 0.0)
    c.omega = float(p.get("omega", 0.5))
    c.alpha = float(p.get("alpha", 1.0))
    c.vr_reconstruct = int(p.get("vr_reconstruct", 0))
    c.vr_kappa = float(p.get("vr_kappa", 1.0))
    c.mlp_min_n = int(p.get("mlp_min_n", 0))
    return c


class Oracle:
    """Holds the particle state of one oracle run (numpy arrays, in place)."""

    def __init__(self, params, particles, dtype=np.float64, layout=None):
        """layout (walled runs): the particle sequence the next step starts
        from, as indices into the given arrays; None takes the initial
        sequence (grouped by cell, ascending id inside a cell), "storage" the
        given storage order (a state read back in its own sequence)."""
        self.p = dict(params)
        self.dtype = np.dtype(dtype)
        self.sfx = _sfx(dtype)
        n = len(particles["cx"])
        self.n = n
        def arr(name, fill=0.0):
            v = particles.get(name)
            if v is None:
                return np.full(n, fill, dtype=self.dtype)
            return np.ascontiguousarray(v, dtype=self.dtype).copy()
        self.x = arr("x")
        self.y = arr("y")
        self.cx, self.cy, self.cz = arr("cx"), arr("cy"), arr("cz")
        self.w = arr("w", 1.0)
        self.id = np.ascontiguousarray(particles.get("id", np.arange(n)), dtype=np.uint32).copy()
        self.cfg = make_cfg(self.p)
        self.ncell = self.p["n_cells"][0] * (self.p["n_cells"][1] if self.p["dims"] == 2 else 1)
        self._keep = []
        if self.p["dims"] == 0:
            off = np.ascontiguousarray(params["inst_offset"], dtype=np.int64)
            self._keep.append(off)
            self.cfg.inst_offset = off.ctypes.data
        if params.get("cell_volume") is not None:
            vol = np.ascontiguousarray(params["cell_volume"], dtype=np.float64)
            self._keep.append(vol)
            self.cfg.cell_volume = vol.ctypes.data
        if params.get("cell_ids") is not None:
            ids = np.ascontiguousarray(params["cell_ids"], dtype=np.int64)
            self._keep.append(ids)
            self.cfg.cell_ids = ids.ctypes.data
        if params.get("mlp") is not None:
            w = np.ascontiguousarray(params["mlp"], dtype=np.float32)
            assert w.size == MLP_NPARAM
            self._keep.append(w)
            self.cfg.mlp = w.ctypes.data
        self.sums = np.zeros((self.ncell, NSUM), dtype=np.float64)
        self.counters = np.zeros((self.ncell, 2), dtype=np.uint64)
        self.diag = OrcDiag()
        self.step = 0
        self.layout = None
        if self.p["dims"] >= 1:
            if layout is None:
                self.layout = np.zeros(n, dtype=np.int64)
                getattr(lib(), "orc_initial_layout" + self.sfx)(
                    ctypes.byref(self.cfg), n, _ptr(self.x), _ptr(self.y), _ptr(self.id), _ptr(self.layout))
            elif isinstance(layout, str) and layout == "storage":
                self.layout = np.arange(n, dtype=np.int64)
            else:
                self.layout = np.ascontiguousarray(layout, dtype=np.int64).copy()
                assert len(self.layout) == n

    def run(self, nsteps, learned_log=False):
        f = getattr(lib(), "orc_run" + self.sfx)
        log = np.zeros((nsteps, self.ncell), dtype=np.int32) if learned_log else None
        rc = f(ctypes.byref(self.cfg), self.n, _ptr(self.x), _ptr(self.y), _ptr(self.cx),
               _ptr(self.cy), _ptr(self.cz), _ptr(self.w), _ptr(self.id), _ptr(self.layout), self.step, nsteps,
               _ptr(self.sums), _ptr(self.counters), ctypes.byref(self.diag), _ptr(log))
        self.step += nsteps
        if rc != 0:
            raise RuntimeError("oracle run failed with status %d" % rc)
        return log

    def run_sampled(self, cells):
        """One step in which every particle streams and is grouped but only the
        listed cells collide and are sampled (outputs the oracle can compute one
        by one at full size)."""
        only = np.ascontiguousarray(np.unique(np.asarray(cells, dtype=np.int64)))
        self.cfg.only_cells = only.ctypes.data
        self.cfg.n_only = len(only)
        try:
            self.run(1)
        finally:
            self.cfg.only_cells = None
            self.cfg.n_only = 0

    def reset_samples(self):
        self.sums[:] = 0.0
        self.counters[:] = 0

    def state(self):
        """Particle state sorted by id (positions, velocities, weights)."""
        o = np.argsort(self.id, kind="stable")
        return {k: getattr(self, k)[o].copy() for k in ("x", "y", "cx", "cy", "cz", "w", "id")}

    def sequence_state(self):
        """Particle state in the current particle sequence (walled runs): the
        order in which the next step groups the particles."""
        o = self.layout if self.layout is not None else np.arange(self.n)
        return {k: getattr(self, k)[o].copy() for k in ("x", "y", "cx", "cy", "cz", "w", "id")}


def exact_bound(cx, cy, cz, dtype=np.float64):
    cx, cy, cz = (np.ascontiguousarray(a, dtype=dtype) for a in (cx, cy, cz))
    return getattr(lib(), "orc_exact_bound" + _sfx(dtype))(_ptr(cx), _ptr(cy), _ptr(cz), None, len(cx))


def diameter(cx, cy, cz, dtype=np.float64):
    cx, cy, cz = (np.ascontiguousarray(a, dtype=dtype) for a in (cx, cy, cz))
    return getattr(lib(), "orc_diameter" + _sfx(dtype))(_ptr(cx), _ptr(cy), _ptr(cz), None, len(cx))


def direction(key, k, cell, step, dtype=np.float64):
    kk = np.asarray(key, dtype=np.uint32)
    out = np.zeros(3, dtype=dtype)
    getattr(lib(), "orc_direction" + _sfx(dtype))(_ptr(kk), k, cell, step, _ptr(out))
    return out


def wall_draw(key, hit, pid, step, Tw, dtype=np.float64):
    kk = np.asarray(key, dtype=np.uint32)
    out = np.zeros(3, dtype=dtype)
    getattr(lib(), "orc_wall_draw" + _sfx(dtype))(_ptr(kk), hit, pid, step, Tw, _ptr(out))
    return out


def wall_ratio(c, Tw, uw, T0, dtype=np.float64):
    cc = np.ascontiguousarray(c, dtype=dtype)
    u = np.ascontiguousarray(uw, dtype=np.float64)
    return getattr(lib(), "orc_wall_ratio" + _sfx(dtype))(_ptr(cc), Tw, _ptr(u), T0)


def vr_update(accepted, p, wi, wj, dtype=np.float64):
    a = np.array([wi], dtype=dtype)
    b = np.array([wj], dtype=dtype)
    getattr(lib(), "orc_vr_update" + _sfx(dtype))(int(accepted), p, _ptr(a), _ptr(b))
    return a[0], b[0]


def scatter(ci, cj, n, dtype=np.float64):
    a = np.array(ci, dtype=dtype)
    b = np.array(cj, dtype=dtype)
    nn = np.array(n, dtype=dtype)
    d = a - b
    g2 = (d[0] * d[0] + d[1] * d[1]) + d[2] * d[2]
    getattr(lib(), "orc_scatter" + _sfx(dtype))(_ptr(a), _ptr(b), g2, _ptr(nn))
    return a, b


def scatter_vss(ci, cj, n, alpha, dtype=np.float64):
    """Variable-soft-sphere collision of one pair: deflection from the
    isotropic unit vector n, exponent alpha (1 = isotropic)."""
    a = np.array(ci, dtype=dtype)
    b = np.array(cj, dtype=dtype)
    nn = np.array(n, dtype=dtype)
    getattr(lib(), "orc_scatter_vss" + _sfx(dtype))(_ptr(a), _ptr(b), _ptr(nn), 1.0 / alpha)
    return a, b


def pair(key, k, cell, step, n, dtype=np.float64):
    kk = np.asarray(key, dtype=np.uint32)
    i = ctypes.c_uint32()
    j = ctypes.c_uint32()
    U = np.zeros(1, dtype=dtype)
    getattr(lib(), "orc_pair" + _sfx(dtype))(_ptr(kk), k, cell, step, n, ctypes.byref(i),
                                             ctypes.byref(j), _ptr(U))
    return i.value, j.value, U[0]


def mlp_forward_f32(params, feats):
    w = np.ascontiguousarray(params, dtype=np.float32)
    f = np.ascontiguousarray(feats, dtype=np.float32)
    return lib().orc_mlp_forward_f32_f64(_ptr(w), _ptr(f))


def features(cx, cy, cz, FNum, V, dtype=np.float64):
    cx, cy, cz = (np.ascontiguousarray(a, dtype=dtype) for a in (cx, cy, cz))
    out = np.zeros(6, dtype=np.float32)
    getattr(lib(), "orc_features" + _sfx(dtype))(_ptr(cx), _ptr(cy), _ptr(cz), None, len(cx),
                                                 FNum, V, _ptr(out))
    return out


def vr_reconstruct(cx, cy, cz, w, T0, dtype=np.float64):
    """Re-estimated weights of one cell (returns (new weights, replaced?))."""
    cx, cy, cz = (np.ascontiguousarray(a, dtype=dtype) for a in (cx, cy, cz))
    ww = np.ascontiguousarray(w, dtype=dtype).copy()
    ok = getattr(lib(), "orc_vr_reconstruct" + _sfx(dtype))(_ptr(cx), _ptr(cy), _ptr(cz), _ptr(ww), None,
                                                            len(cx), float(T0))
    return ww, bool(ok)


def cell_of(params, x, y, dtype=np.float64):
    cfg = make_cfg(params)
    return getattr(lib(), "orc_cell_of" + _sfx(dtype))(ctypes.byref(cfg), x, y)


def estimators(sums, n_samples, FN, V, vr=False, vr_n0=None, vr_T0=None):
    """Cell estimates from time-summed raw sums (ratio estimators, FP64).

    n = S0 F_N / (V n_samp); u = S1 / S0; T = (tr S2 / S0 - |u|^2) / 3;
    P_de = n (S2_de / S0 - u_d u_e); q_d = 1/2 n (<c_d c^2> - 2 u_e <c_d c_e>
    - u_d <c^2> + 2 u_d |u|^2).  With variance reduction, each raw average
    <Q> is replaced by the reference-equilibrium value plus the (1 - W)
    weighted deviation: (F_N / V) sum (1 - W) Q / n_samp.
    """
    s = np.asarray(sums, dtype=np.float64)
    V = np.broadcast_to(np.asarray(V, dtype=np.float64), s.shape[:1])
    if not vr:
        dens_sum = s[:, 0:13] * (FN / (V[:, None] * n_samples))  # density-weighted moments
    else:
        # reference equilibrium (n0, 0, T0): <1> = n0, <c> = 0, <c_d c_e> = n0 T0 delta,
        # <c_d |c|^2> = 0
        eq = np.zeros(13)
        eq[0] = vr_n0
        eq[4:7] = vr_n0 * vr_T0
        dens_sum = eq[None, :] + s[:, 13:26] * (FN / (V[:, None] * n_samples))
    n = dens_sum[:, 0]
    with np.errstate(invalid="ignore", divide="ignore"):
        u = dens_sum[:, 1:4] / n[:, None]
        m2 = dens_sum[:, 4:10] / n[:, None]   # xx yy zz xy xz yz
        m3 = dens_sum[:, 10:13] / n[:, None]
        uu = (u ** 2).sum(1)
        T = ((m2[:, 0] + m2[:, 1] + m2[:, 2]) - uu) / 3.0
        full = np.empty((len(n), 3, 3))
        idx = [(0, 0), (1, 1), (2, 2), (0, 1), (0, 2), (1, 2)]
        for k, (a, b) in enumerate(idx):
            full[:, a, b] = m2[:, k]
            full[:, b, a] = m2[:, k]
        P = n[:, None, None] * (full - u[:, :, None] * u[:, None, :])
        c2m = m2[:, 0] + m2[:, 1] + m2[:, 2]
        q = 0.5 * n[:, None] * (m3 - 2.0 * np.einsum("ne,nde->nd", u, full)
                                - u * c2m[:, None] + 2.0 * u * uu[:, None])
    return {"n": n, "u": u, "T": T, "P": P, "q": q}


def vhs_pow(x, a):
    """x^a as the VHS acceptance computes it (fixed operation sequence)."""
    return lib().orc_vhs_pow(float(x), float(a))
