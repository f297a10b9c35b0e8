"""Thin Python binding of the C ABI in include/dsmc.h (argument marshalling only).

Every step of the hot path runs in the HIP library ``_lib/libdsmc_hip.so``;
this module only builds the C structs, lets PyTorch own device memory and
streams, and passes raw pointers.  If the library is missing the binding
raises: there is no CPU fallback.
"""
import ctypes
import os

import numpy as np

from . import build as _build

NSUM = 26
NEST = 14
MLP_NPARAM = 4673
MLP_NSTATS = 14
MLP_NOALLOC_MAX = 4096
CALIB_NDELTA, CALIB_NBINS, CALIB_FIELDS = 128, 8, 4
ABI_VERSION = 5

STATUS = {0: "DSMC_OK", -1: "DSMC_EINVAL", -2: "DSMC_ENOMEM", -3: "DSMC_EHIP",
          -4: "DSMC_ENONFINITE", -5: "DSMC_EWALLHITS", -6: "DSMC_ECAPACITY", -7: "DSMC_EABI"}


class DsmcError(RuntimeError):
    def __init__(self, code, where):
        self.code = code
        super().__init__("%s failed: %s (%d)" % (where, STATUS.get(code, "?"), code))


class Config(ctypes.Structure):
    _fields_ = [
        ("abi_version", ctypes.c_int32), ("dims", ctypes.c_int32), ("real_bytes", ctypes.c_int32),
        ("molecule", ctypes.c_int32), ("n_cells", ctypes.c_int32 * 2), ("majorant", ctypes.c_int32),
        ("vr", ctypes.c_int32), ("length", ctypes.c_double * 2), ("dt", ctypes.c_double),
        ("sigma", ctypes.c_double), ("FN", ctypes.c_double), ("vr_T0", ctypes.c_double),
        ("wall_kind", ctypes.c_int32 * 4), ("wall_T", ctypes.c_double * 4),
        ("wall_u", (ctypes.c_double * 3) * 4), ("seed", ctypes.c_uint64),
        ("n_particles", ctypes.c_int64), ("cell_volume", ctypes.c_void_p),
        ("inst_offset", ctypes.c_void_p), ("max_wall_hits", ctypes.c_int32),
        ("schedule", ctypes.c_int32), ("persistent_waves", ctypes.c_int32), ("vr_reconstruct", ctypes.c_int32),
        ("chunk_work", ctypes.c_int64), ("omega", ctypes.c_double), ("alpha", ctypes.c_double),
        ("vr_kappa", ctypes.c_double), ("wide_min", ctypes.c_int32), ("occupancy", ctypes.c_int32),
        ("cells_per_wave", ctypes.c_int32), ("waves_per_cell", ctypes.c_int32),
    ]


class CalibModel(ctypes.Structure):
    _fields_ = [(k, ctypes.c_double) for k in ("n_scale", "cand_scale", "eps", "cost_network", "cost_member",
                                                "cost_verify")]


def estimators(sums, n_samples, FN, volume=None, volume_uniform=1.0, vr=False, vr_n0=0.0, vr_T0=1.0):
    """Cell estimates from running sums (the library's dsmc_estimators):
    columns n, u_x, u_y, u_z, T, P_xx, P_yy, P_zz, P_xy, P_xz, P_yz, q_x, q_y, q_z."""
    L = load()
    s = np.ascontiguousarray(sums, dtype=np.float64)
    nc = s.shape[0]
    vol = None if volume is None else np.ascontiguousarray(np.broadcast_to(volume, (nc,)), dtype=np.float64)
    out = np.zeros((nc, NEST), dtype=np.float64)
    check(L.dsmc_estimators(s.ctypes.data, nc, int(n_samples), float(FN), vol.ctypes.data if vol is not None else None,
                            float(volume_uniform), int(bool(vr)), float(vr_n0), float(vr_T0), out.ctypes.data),
          "dsmc_estimators")
    return out


class Soa(ctypes.Structure):
    _fields_ = [(k, ctypes.c_void_p) for k in ("x", "y", "cx", "cy", "cz", "w", "id")]


class Diag(ctypes.Structure):
    _fields_ = [(k, ctypes.c_uint64) for k in (
        "steps", "candidates", "accepted", "overshoot", "wall_hits", "learned_used", "fallback",
        "learned_skip", "vr_nonfinite", "big_cells", "bounds_violations", "bounds_checked")]


_lib = None


def lib_path():
    """The in-tree library, or the build named by DSMC_HIP_LIB (for instance
    the bounds-checking variant, _lib/libdsmc_hip_bounds.so)."""
    return os.environ.get("DSMC_HIP_LIB") or _build.LIB


def load():
    """Load the HIP library (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    # torch ships its own HIP runtime; importing it first makes the library
    # bind to that same runtime instead of loading a second one
    import torch  # noqa: F401
    path = lib_path()
    if not os.path.exists(path):
        raise RuntimeError("HIP library %s is missing: run __graft_entry__.build() or "
                           "python -m paper_2301_05985_amd.build" % path)
    L = ctypes.CDLL(path)
    P, I32, I64, D = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double
    sig = {
        "dsmc_workspace_size": [P, P],
        "dsmc_init": [P, P, P, ctypes.c_size_t, P, P],
        "dsmc_step": [P, I32],
        "dsmc_sample": [P, P, P, P, I32],
        "dsmc_particles": [P, P],
        "dsmc_diagnostics": [P, P],
        "dsmc_set_step": [P, ctypes.c_uint64],
        "dsmc_set_majorant_model": [P, P, I64, D, I32],
        "dsmc_checkpoint": [P, P, P],
        "dsmc_restore": [P, P, ctypes.c_size_t],
        "dsmc_profile_step": [P, P, I32, P, P, I32],
        "dsmc_destroy": [P],
        "dsmc_collect_features": [P, P, P, P, P],
        "dsmc_estimators": [P, I64, ctypes.c_uint64, D, P, D, I32, D, D, P],
        "dsmc_mlp_standardize": [P, P, I64, P, P, P, P],
        "dsmc_mlp_fold_inputs": [P, P, P],
        "dsmc_mlp_to_bf16": [P, I64, P, P],
        "dsmc_mlp_calibrate": [P, P, P, P, P, I64, P, P, ctypes.c_size_t, P, P, P, P],
        "dsmc_mlp_forward": [P, P, I64, P, P],
        "dsmc_mlp_loss_grad": [P, P, P, I64, D, P, P, P, P],
        "dsmc_mlp_loss_grad_noalloc": [P, P, P, I64, D, P, P, P],
        "dsmc_mlp_adam": [P, P, P, P, I64, I64, D, D, D, D, P],
    }
    for name, args in sig.items():
        f = getattr(L, name)
        f.argtypes = args
        f.restype = ctypes.c_int
    L.dsmc_status_string.argtypes = [ctypes.c_int]
    L.dsmc_status_string.restype = ctypes.c_char_p
    L.dsmc_mlp_scratch_floats.argtypes = [I64]
    L.dsmc_mlp_scratch_floats.restype = I64
    L.dsmc_mlp_calib_work_bytes.argtypes = [I64]
    L.dsmc_mlp_calib_work_bytes.restype = ctypes.c_size_t
    _lib = L
    return L


def check(code, where):
    if code != 0:
        raise DsmcError(code, where)


def make_config(p, n_particles):
    """C config struct from a workload parameter dict (see workloads.py)."""
    c = Config()
    c.abi_version = ABI_VERSION
    c.dims = p["dims"]
    c.real_bytes = 8 if p.get("real", "f64") == "f64" else 4
    c.molecule = p.get("molecule", 0)
    c.n_cells[0], c.n_cells[1] = p["n_cells"]
    c.majorant = int(p.get("majorant", 0))
    c.vr = int(p.get("vr", 0))
    c.length[0], c.length[1] = p.get("length", (1.0, 1.0))
    c.dt, c.sigma, c.FN = p["dt"], p["sigma"], p["FN"]
    c.vr_T0 = p.get("vr_T0", 1.0)
    for k in range(4):
        c.wall_kind[k] = p.get("wall_kind", (0, 0, 0, 0))[k]
        c.wall_T[k] = p.get("wall_T", (1.0,) * 4)[k]
        for d in range(3):
            c.wall_u[k][d] = p.get("wall_u", ((0.0, 0.0, 0.0),) * 4)[k][d]
    c.seed = int(p.get("seed", 0)) & 0xFFFFFFFFFFFFFFFF
    c.n_particles = n_particles
    c.max_wall_hits = p.get("max_wall_hits", 64)
    c.schedule = int(p.get("schedule", 0))
    c.persistent_waves = int(p.get("persistent_waves", 0))
    c.chunk_work = int(p.get("chunk_work", 0))
    c.omega = float(p.get("omega", 0.5))
    c.alpha = float(p.get("alpha", 1.0))
    c.vr_reconstruct = int(p.get("vr_reconstruct", 0))
    c.vr_kappa = float(p.get("vr_kappa", 1.0))
    c.wide_min = int(p.get("wide_min", 0))
    c.occupancy = int(p.get("occupancy", 0))
    c.cells_per_wave = int(p.get("cells_per_wave", 0))
    c.waves_per_cell = int(p.get("waves_per_cell", 0))
    return c


class Simulation:
    """One DSMC run on the GPU: torch owns the particle arrays and workspace."""

    FIELDS = ("x", "y", "cx", "cy", "cz", "w")

    def __init__(self, params, particles, device="cuda:0", stream=None):
        import torch
        self.torch = torch
        self.L = load()
        self.p = dict(params)
        self.device = torch.device(device)
        self.rdtype = torch.float64 if self.p.get("real", "f64") == "f64" else torch.float32
        self.rb = 8 if self.rdtype == torch.float64 else 4
        n = len(particles["cx"])
        self.n = n
        self.cfg = make_config(self.p, n)
        self._host_keep = []
        if self.p["dims"] == 0:
            off = np.ascontiguousarray(self.p["inst_offset"], dtype=np.int64)
            self._host_keep.append(off)
            self.cfg.inst_offset = off.ctypes.data
        if self.p.get("cell_volume") is not None:
            vol = np.ascontiguousarray(self.p["cell_volume"], dtype=np.float64)
            self._host_keep.append(vol)
            self.cfg.cell_volume = vol.ctypes.data
        self.ncell = self.p["n_cells"][0] * (self.p["n_cells"][1] if self.p["dims"] == 2 else 1)
        # particle arrays (caller-owned device memory)
        np_dt = np.float64 if self.rb == 8 else np.float32
        self.t = {}
        for k in self.FIELDS:
            v = particles.get(k)
            if v is None:
                v = np.ones(n) if k == "w" else np.zeros(n)
            self.t[k] = torch.from_numpy(np.ascontiguousarray(v, dtype=np_dt)).to(self.device)
        ids = particles.get("id", np.arange(n, dtype=np.uint32))
        self.t["id"] = torch.from_numpy(np.ascontiguousarray(ids, dtype=np.uint32).view(np.int32)).to(self.device)
        # workspace, 256-byte aligned
        ws = ctypes.c_size_t()
        check(self.L.dsmc_workspace_size(ctypes.byref(self.cfg), ctypes.byref(ws)), "dsmc_workspace_size")
        self.ws_bytes = ws.value
        self.ws_raw = torch.zeros(self.ws_bytes + 256, dtype=torch.uint8, device=self.device)
        base = self.ws_raw.data_ptr()
        self.ws_off = (-base) % 256
        self.ws_ptr = base + self.ws_off
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        soa = Soa(*[self.t[k].data_ptr() for k in self.FIELDS], self.t["id"].data_ptr())
        ctx = ctypes.c_void_p()
        check(self.L.dsmc_init(ctypes.byref(self.cfg), ctypes.byref(soa), ctypes.c_void_p(self.ws_ptr),
                               self.ws_bytes, ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(ctx)),
              "dsmc_init")
        self.ctx = ctx

    def __del__(self):
        try:
            if getattr(self, "ctx", None):
                self.L.dsmc_destroy(self.ctx)
                self.ctx = None
        except Exception:
            pass

    def close(self):
        if self.ctx:
            check(self.L.dsmc_destroy(self.ctx), "dsmc_destroy")
            self.ctx = None

    def step(self, n=1):
        check(self.L.dsmc_step(self.ctx, int(n)), "dsmc_step")

    def sample(self, reset=False):
        sums = np.zeros((self.ncell, NSUM), dtype=np.float64)
        cnt = np.zeros((self.ncell, 2), dtype=np.uint64)
        ns = ctypes.c_uint64()
        check(self.L.dsmc_sample(self.ctx, sums.ctypes.data, cnt.ctypes.data, ctypes.byref(ns), int(reset)),
              "dsmc_sample")
        return sums, cnt, ns.value

    def diagnostics(self):
        d = Diag()
        rc = self.L.dsmc_diagnostics(self.ctx, ctypes.byref(d))
        out = {k: getattr(d, k) for k, _ in Diag._fields_}
        out["status"] = rc
        return out

    def _view(self, ptr, nbytes_per, dtype):
        """Torch view of a device pointer that lies in one of our allocations."""
        torch = self.torch
        for k in self.FIELDS + ("id",):
            if ptr == self.t[k].data_ptr():
                return self.t[k]
        off = ptr - self.ws_raw.data_ptr()
        if 0 <= off < self.ws_raw.numel():
            return self.ws_raw[off:off + self.n * nbytes_per].view(dtype)
        raise RuntimeError("pointer outside the run's buffers")

    def particles(self):
        """Current particle state as numpy arrays sorted by id."""
        torch = self.torch
        cur = Soa()
        check(self.L.dsmc_particles(self.ctx, ctypes.byref(cur)), "dsmc_particles")
        torch.cuda.synchronize(self.device)
        out = {}
        for k in self.FIELDS:
            ptr = getattr(cur, k)
            out[k] = self._view(ptr, self.rb, self.rdtype).cpu().numpy().copy() if ptr else None
        out["id"] = self._view(cur.id, 4, torch.int32).cpu().numpy().view(np.uint32).copy()
        o = np.argsort(out["id"], kind="stable")
        return {k: (v[o] if v is not None else None) for k, v in out.items()}

    def sequence(self):
        """Current particle state as numpy arrays in storage order, which for
        walled runs is the particle sequence (grouped by cell)."""
        t = self.raw_particles()
        self.torch.cuda.synchronize(self.device)
        out = {k: (v.cpu().numpy().copy() if v is not None else None) for k, v in t.items() if k != "id"}
        out["id"] = t["id"].cpu().numpy().view(np.uint32).copy()
        return out

    def raw_particles(self):
        """Current particle state in storage order (torch tensors on the device)."""
        torch = self.torch
        cur = Soa()
        check(self.L.dsmc_particles(self.ctx, ctypes.byref(cur)), "dsmc_particles")
        out = {k: (self._view(getattr(cur, k), self.rb, self.rdtype) if getattr(cur, k) else None)
               for k in self.FIELDS}
        out["id"] = self._view(cur.id, 4, torch.int32)
        return out

    def set_step(self, s):
        check(self.L.dsmc_set_step(self.ctx, int(s)), "dsmc_set_step")

    def checkpoint(self):
        nb = ctypes.c_size_t()
        check(self.L.dsmc_checkpoint(self.ctx, None, ctypes.byref(nb)), "dsmc_checkpoint")
        blob = np.zeros(nb.value, dtype=np.uint8)
        check(self.L.dsmc_checkpoint(self.ctx, blob.ctypes.data, ctypes.byref(nb)), "dsmc_checkpoint")
        return blob

    def restore(self, blob):
        check(self.L.dsmc_restore(self.ctx, blob.ctypes.data, blob.nbytes), "dsmc_restore")

    def profile_step(self):
        ms = np.zeros(16, dtype=np.float32)
        nk = ctypes.c_int32()
        names = ctypes.create_string_buffer(1024)
        check(self.L.dsmc_profile_step(self.ctx, ms.ctypes.data, 16, ctypes.byref(nk), names, 1024),
              "dsmc_profile_step")
        nm = names.value.decode().split("\n")[: nk.value]
        return list(zip(nm, ms[: nk.value].tolist()))

    def set_majorant_model(self, bf16_weights, delta, min_n=0):
        w = np.ascontiguousarray(bf16_weights, dtype=np.uint16)
        check(self.L.dsmc_set_majorant_model(self.ctx, w.ctypes.data, w.size, float(delta), int(min_n)),
              "dsmc_set_majorant_model")
