"""Learned collision majorant: training data, GPU training, export.

Pipeline (every arithmetic step runs in the HIP library through the C ABI;
PyTorch only holds device memory and the stream, and shuffles row indices):
  1. run batched homogeneous cells with the exact majorant and collect, every
     few steps, each cell's six moment features, the label log2 of its
     exact largest pairwise relative speed, and on held-out runs the exact
     bound and the verification's |S| <= 64 threshold (dsmc_collect_features);
  2. standardise the features (dsmc_mlp_standardize) and train the
     6-64-64-1 network on the GPU with the project's forward, backward and
     Adam kernels (dsmc_mlp_loss_grad, dsmc_mlp_adam), expectile loss with
     tau = 0.95;
  3. fold the standardisation into the first layer (dsmc_mlp_fold_inputs),
     round to bfloat16 (dsmc_mlp_to_bf16), and choose the lattice margin
     delta and the cell-size gate min_n on the held-out cells against the
     measured costs of the network and of the verification
     (dsmc_mlp_calibrate);
  4. load the model into a run with dsmc_set_majorant_model.
"""
import ctypes
import math
import os

import numpy as np

from . import binding
from . import workloads as W

NPARAM = binding.MLP_NPARAM


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr())


def collect(sim, with_bound=False):
    """Features [n_cells, 6], labels log2(largest pair speed) [n_cells] and,
    optionally, log2 of the exact bound and of the |S| <= 64 threshold
    [n_cells] (torch, on the device; -inf labels mark cells of fewer than
    two particles, which every later step skips)."""
    torch = sim.torch
    mk = lambda: torch.empty(sim.ncell, dtype=torch.float32, device=sim.device)
    f = torch.empty((sim.ncell, 6), dtype=torch.float32, device=sim.device)
    y = mk()
    b, sl = (mk(), mk()) if with_bound else (None, None)
    binding.check(sim.L.dsmc_collect_features(sim.ctx, _ptr(f), _ptr(y), _ptr(b) if b is not None else None,
                                              _ptr(sl) if sl is not None else None),
                  "dsmc_collect_features")
    return (f, y, b, sl) if with_bound else (f, y)


def generate(seeds=(1, 2, 3, 4), steps=256, every=4, n_inst=4096, nmin=50, nmax=2000, dt=0.05, with_bound=False):
    """Samples from batched runs with the exact majorant (concatenated on
    the device)."""
    import torch
    cols = []
    for sd in seeds:
        p, parts = W.batched(n_inst=n_inst, nmin=nmin, nmax=nmax, real="f32", dt=dt, seed=sd, init_seed=sd)
        sim = binding.Simulation(p, parts)
        for s in range(0, steps, every):
            cols.append(collect(sim, with_bound))
            sim.step(every)
        sim.close()
    return tuple(torch.cat([c[k] for c in cols]).contiguous() for k in range(len(cols[0])))


def init_params(seed=0, device="cuda"):
    """He initialisation (weights ~ N(0, 2 / fan_in)), zero biases, as a device tensor."""
    import torch
    rng = np.random.default_rng(seed)
    W1 = rng.standard_normal((64, 6)) * np.sqrt(2.0 / 6)
    W2 = rng.standard_normal((64, 64)) * np.sqrt(2.0 / 64)
    w3 = rng.standard_normal(64) * np.sqrt(2.0 / 64)
    p = np.concatenate([W1.ravel(), np.zeros(64), W2.ravel(), np.zeros(64), w3, [0.0]]).astype(np.float32)
    return torch.from_numpy(p).to(device)


class Trainer:
    """Adam training of the network on device tensors x [n, 6], y [n]."""

    def __init__(self, params, batch=4096, lr=1e-3, tau=0.95, betas=(0.9, 0.999), eps=1e-8):
        import torch
        self.torch = torch
        self.L = binding.load()
        self.p = params
        self.dev = params.device
        self.batch = batch
        self.lr, self.tau, self.betas, self.eps = lr, tau, betas, eps
        self.m = torch.zeros_like(params)
        self.v = torch.zeros_like(params)
        self.g = torch.zeros_like(params)
        self.loss = torch.zeros(1, dtype=torch.float32, device=self.dev)
        nsc = self.L.dsmc_mlp_scratch_floats(batch)
        self.scratch = torch.empty(nsc, dtype=torch.float32, device=self.dev)
        self.t = 0
        self.stream = ctypes.c_void_p(torch.cuda.current_stream(self.dev).cuda_stream)

    def loss_grad(self, xb, yb):
        binding.check(self.L.dsmc_mlp_loss_grad(_ptr(self.p), _ptr(xb), _ptr(yb), len(yb), self.tau,
                                                _ptr(self.g), _ptr(self.loss), _ptr(self.scratch), self.stream),
                      "dsmc_mlp_loss_grad")
        return self.g, self.loss

    def step(self, xb, yb):
        self.loss_grad(xb, yb)
        self.t += 1
        binding.check(self.L.dsmc_mlp_adam(_ptr(self.p), _ptr(self.g), _ptr(self.m), _ptr(self.v), NPARAM, self.t,
                                           self.lr, self.betas[0], self.betas[1], self.eps, self.stream),
                      "dsmc_mlp_adam")

    def epoch(self, x, y, seed):
        """One pass over shuffled mini-batches; returns the mean batch loss."""
        torch = self.torch
        n = len(y)
        g = torch.Generator(device="cpu").manual_seed(int(seed))
        perm = torch.randperm(n, generator=g).to(self.dev)
        losses = []
        for s in range(0, n - self.batch + 1, self.batch):
            idx = perm[s:s + self.batch]
            self.step(x[idx].contiguous(), y[idx].contiguous())
            losses.append(self.loss.cpu().numpy()[0])
        return float(np.mean(losses)) if losses else float("nan")


def _stream(device):
    import torch
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


def forward(params, x):
    import torch
    L = binding.load()
    y = torch.empty(len(x), dtype=torch.float32, device=x.device)
    binding.check(L.dsmc_mlp_forward(_ptr(params), _ptr(x), len(x), _ptr(y), _stream(x.device)),
                  "dsmc_mlp_forward")
    return y


def standardize(x, y):
    """Standardised features and the statistics (library call): returns
    (xs, stats_dev, stats_host) with stats = means[6], standard deviations[6],
    mean label, rows (rows with a non-finite label are left out)."""
    import torch
    L = binding.load()
    xs = torch.empty_like(x)
    stats_dev = torch.empty(binding.MLP_NSTATS, dtype=torch.float64, device=x.device)
    stats = np.zeros(binding.MLP_NSTATS, dtype=np.float64)
    binding.check(L.dsmc_mlp_standardize(_ptr(x), _ptr(y), len(y), _ptr(xs), _ptr(stats_dev), stats.ctypes.data,
                                         _stream(x.device)), "dsmc_mlp_standardize")
    return xs, stats_dev, stats


def export_bf16(params, stats_dev=None):
    """Fold the standardisation into the first layer (in place, if stats_dev
    is given) and round to bfloat16; returns (bits on the device, bits as
    numpy uint16)."""
    import torch
    L = binding.load()
    if stats_dev is not None:
        binding.check(L.dsmc_mlp_fold_inputs(_ptr(params), _ptr(stats_dev), _stream(params.device)),
                      "dsmc_mlp_fold_inputs")
    bits = torch.empty(NPARAM, dtype=torch.int16, device=params.device)
    binding.check(L.dsmc_mlp_to_bf16(_ptr(params), NPARAM, _ptr(bits), _stream(params.device)), "dsmc_mlp_to_bf16")
    return bits, bits.cpu().numpy().view(np.uint16).copy()


# Costs of the learned majorant in candidate-equivalents, from the kernels'
# measured time per step on the batched cells (4096 cells, mean 1025
# particles, 1.28e-4 us per NTC candidate of the exact method): features,
# network and lattice 8 us per step (15 per cell); the membership pass 5 us
# over three quarters of the cells (0.0125 per particle); collecting S, the
# pair check and the extra candidates of fallback cells 12 us (30 per cell).
COSTS = dict(cost_network=15.0, cost_member=0.0125, cost_verify=30.0)


def calibrate(bits_dev, xv, yv, bv, sv, sigma, dt, FN=1.0, V=1.0, eps=2.0 ** -20, costs=None):
    """Margin delta and size gate min_n (library call, see dsmc_mlp_calibrate);
    returns (delta, min_n, table [NDELTA][NBINS][FIELDS])."""
    import torch
    L = binding.load()
    c = dict(COSTS if costs is None else costs)
    model = binding.CalibModel(n_scale=V / FN, cand_scale=0.5 * FN * sigma * dt / V, eps=eps, **c)
    nb = L.dsmc_mlp_calib_work_bytes(len(yv))
    raw = torch.empty(nb + 256, dtype=torch.uint8, device=xv.device)
    off = (-raw.data_ptr()) % 256
    delta = ctypes.c_double()
    min_n = ctypes.c_int32()
    table = np.zeros((binding.CALIB_NDELTA, binding.CALIB_NBINS, binding.CALIB_FIELDS), dtype=np.float64)
    binding.check(L.dsmc_mlp_calibrate(_ptr(bits_dev), _ptr(xv), _ptr(yv), _ptr(bv), _ptr(sv), len(yv),
                                       ctypes.byref(model), ctypes.c_void_p(raw.data_ptr() + off), nb,
                                       ctypes.byref(delta), ctypes.byref(min_n), table.ctypes.data,
                                       _stream(xv.device)), "dsmc_mlp_calibrate")
    return delta.value, min_n.value, table


def train_model(n_epochs=8, seeds=(1, 2, 3, 4), val_seed=5, steps=256, every=4, seed=0,
                n_inst=4096, nmin=50, nmax=2000, dt=0.05, costs=None, log=None):
    """Full pipeline: data, training, bf16 export, margin and gate; returns a dict."""
    import torch
    x, y = generate(seeds=seeds, steps=steps, every=every, n_inst=n_inst, nmin=nmin, nmax=nmax, dt=dt)
    xv, yv, bv, sv = generate(seeds=(val_seed,), steps=max(steps // 4, every), every=every, n_inst=n_inst,
                              nmin=nmin, nmax=nmax, dt=dt, with_bound=True)
    # train on standardised inputs; the exported network takes the raw
    # features the collision kernel computes
    xs, stats_dev, stats = standardize(x, y)
    params = init_params(seed, x.device)
    # start the output bias at the mean label so training begins near the data
    params[-1] = float(stats[12])
    tr = Trainer(params)
    hist = []
    for e in range(n_epochs):
        hist.append(tr.epoch(xs, y, seed=1000 + e))
        if log:
            log("epoch %d mean loss %.6f" % (e, hist[-1]))
    bits_dev, bits = export_bf16(params, stats_dev)
    sigma = math.sqrt(math.pi) / (4.0 * 0.5 * (nmin + nmax))  # the batched workload's cross-section
    delta, min_n, table = calibrate(bits_dev, xv, yv, bv, sv, sigma, dt, costs=costs)
    torch.cuda.synchronize()
    return {"bits": bits, "delta": delta, "min_n": min_n, "calibration": table, "loss_history": hist,
            "n_train": int(stats[13]), "n_val": int(len(yv))}


def save(path, model):
    os.makedirs(os.path.dirname(path), exist_ok=True)
    np.savez(path, bits=model["bits"], delta=np.array([model["delta"]]), min_n=np.array([model.get("min_n", 0)]),
             loss_history=np.array(model["loss_history"]), n_train=np.array([model["n_train"]]))


def load_model(path):
    d = np.load(path)
    return {"bits": d["bits"].astype(np.uint16), "delta": float(d["delta"][0]), "min_n": int(d["min_n"][0])}


def simulation_with_model(params, particles, model):
    """A Simulation using the learned majorant (params must set majorant=1)."""
    if isinstance(model, str):
        model = load_model(model)
    sim = binding.Simulation(dict(params, majorant=1), particles)
    sim.set_majorant_model(model["bits"], model["delta"], model.get("min_n", 0))
    return sim
