"""Learned collision majorant: training data, GPU training, export.

Pipeline (every arithmetic step runs in the HIP library through the C ABI):
  1. run batched homogeneous cells with the exact majorant and collect, every
     few steps, each cell's six moment features and the label log2 of its
     exact largest pairwise relative speed (dsmc_collect_features);
  2. train the 6-64-64-1 network on the GPU with the project's forward,
     backward and Adam kernels (dsmc_mlp_loss_grad, dsmc_mlp_adam), expectile
     loss with tau = 0.95;
  3. round the weights to bfloat16 and choose the lattice margin delta on a
     held-out run to maximise the expected saving of NTC candidates (cells
     whose proposal fails verification fall back to the exact bound);
  4. load the model into a run with dsmc_set_majorant_model.
PyTorch only holds device memory and the stream.
"""
import ctypes
import os

import numpy as np

from . import binding
from . import workloads as W

NPARAM = binding.MLP_NPARAM


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr())


def collect(sim, with_bound=False):
    """Features [n_cells, 6], labels log2(largest pair speed) [n_cells] and,
    optionally, log2 of the exact bound [n_cells] (torch, on the device)."""
    torch = sim.torch
    f = torch.empty((sim.ncell, 6), dtype=torch.float32, device=sim.device)
    y = torch.empty(sim.ncell, dtype=torch.float32, device=sim.device)
    b = torch.empty(sim.ncell, dtype=torch.float32, device=sim.device) if with_bound else None
    binding.check(sim.L.dsmc_collect_features(sim.ctx, _ptr(f), _ptr(y), _ptr(b) if b is not None else None),
                  "dsmc_collect_features")
    return (f, y, b) if with_bound else (f, y)


def generate(seeds=(1, 2, 3, 4), steps=256, every=4, n_inst=4096, nmin=50, nmax=2000, dt=0.05, with_bound=False):
    """Training samples from batched runs with the exact majorant."""
    import torch
    xs, ys, bs = [], [], []
    for sd in seeds:
        p, parts = W.batched(n_inst=n_inst, nmin=nmin, nmax=nmax, real="f32", dt=dt, seed=sd, init_seed=sd)
        sim = binding.Simulation(p, parts)
        for s in range(0, steps, every):
            out = collect(sim, with_bound)
            xs.append(out[0])
            ys.append(out[1])
            if with_bound:
                bs.append(out[2])
            sim.step(every)
        sim.close()
    x = torch.cat(xs)
    y = torch.cat(ys)
    ok = torch.isfinite(y)
    if with_bound:
        return x[ok].contiguous(), y[ok].contiguous(), torch.cat(bs)[ok].contiguous()
    return x[ok].contiguous(), y[ok].contiguous()


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
        tot = torch.zeros(1, dtype=torch.float64, device=self.dev)
        nb = 0
        for s in range(0, n - self.batch + 1, self.batch):
            idx = perm[s:s + self.batch]
            self.step(x[idx].contiguous(), y[idx].contiguous())
            tot += self.loss.double()
            nb += 1
        return float(tot.item()) / max(nb, 1)


def forward(params, x):
    import torch
    L = binding.load()
    y = torch.empty(len(x), dtype=torch.float32, device=x.device)
    binding.check(L.dsmc_mlp_forward(_ptr(params), _ptr(x), len(x), _ptr(y),
                                     ctypes.c_void_p(torch.cuda.current_stream(x.device).cuda_stream)),
                  "dsmc_mlp_forward")
    return y


def to_bf16_bits(params):
    """Round to bfloat16 (nearest, ties to even); returns uint16 numpy bits."""
    import torch
    return params.detach().to(torch.bfloat16).view(torch.int16).cpu().numpy().view(np.uint16).copy()


def bf16_to_float(bits, device):
    import torch
    b = torch.from_numpy(np.asarray(bits, dtype=np.uint16).view(np.int16).copy()).to(device)
    return b.view(torch.bfloat16).float()


def calibrate_delta(bits, x, y, bound, grid=None):
    """Lattice margin delta (log2 units) that maximises the expected saving of
    NTC candidates on held-out cells, with the bfloat16 weights the collision
    kernel uses.  A cell's proposal 2^(ceil(64 (y_pred + delta)) / 64) is used
    when it lies between the cell's largest pair speed and its exact bound,
    and then saves candidates in proportion to N^2 (bound - proposal); below
    the largest pair speed it falls back (no saving), above the bound it is
    skipped.  N comes from the density feature (unit volume)."""
    import torch
    p = bf16_to_float(bits, x.device)
    pred = forward(p, x).double()
    yd, bd = y.double(), bound.double()
    n2 = torch.pow(2.0, x[:, 0].double()) ** 2
    if grid is None:
        grid = np.arange(-0.5, 0.5, 0.0025)
    best, best_gain = float(grid[-1]), -1.0
    gb = torch.pow(2.0, bd)
    for d in grid:
        k = torch.ceil(64.0 * (pred + float(d)))
        gp_log = k / 64.0
        used = (gp_log >= yd) & (gp_log < bd)
        gain = float((n2 * (gb - torch.pow(2.0, gp_log)) * used).sum().item())
        if gain > best_gain:
            best, best_gain = float(d), gain
    return best


def train_model(n_epochs=8, seeds=(1, 2, 3, 4), val_seed=5, steps=256, every=4, seed=0,
                n_inst=4096, nmin=50, nmax=2000, log=None):
    """Full pipeline: data, training, bf16 export, margin; returns a dict."""
    import torch
    x, y = generate(seeds=seeds, steps=steps, every=every, n_inst=n_inst, nmin=nmin, nmax=nmax)
    xv, yv, bv = generate(seeds=(val_seed,), steps=max(steps // 4, every), every=every, n_inst=n_inst,
                          nmin=nmin, nmax=nmax, with_bound=True)
    # train on standardised inputs, then fold the standardisation into the
    # first layer (W1 / s, b1 - W1 m / s) so the exported network takes the
    # raw features the collision kernel computes
    mu = x.mean(0)
    sd = x.std(0).clamp_min(1e-6)
    xs = ((x - mu) / sd).contiguous()
    params = init_params(seed, x.device)
    # start the output bias at the mean label so training begins near the data
    params[-1] = float(y.mean().item())
    tr = Trainer(params)
    hist = []
    for e in range(n_epochs):
        hist.append(tr.epoch(xs, y, seed=1000 + e))
        if log:
            log("epoch %d mean loss %.6f" % (e, hist[-1]))
    torch.cuda.synchronize()
    W1 = params[:64 * 6].view(64, 6)
    b1 = params[64 * 6:64 * 6 + 64]
    b1 -= (W1 * (mu / sd)[None, :]).sum(1)
    W1 /= sd[None, :]
    bits = to_bf16_bits(params)
    delta = calibrate_delta(bits, xv, yv, bv)
    return {"bits": bits, "delta": delta, "loss_history": hist, "n_train": int(len(y)), "n_val": int(len(yv))}


def save(path, model):
    os.makedirs(os.path.dirname(path), exist_ok=True)
    np.savez(path, bits=model["bits"], delta=np.array([model["delta"]]),
             loss_history=np.array(model["loss_history"]), n_train=np.array([model["n_train"]]))


def load_model(path):
    d = np.load(path)
    return {"bits": d["bits"].astype(np.uint16), "delta": float(d["delta"][0])}


def simulation_with_model(params, particles, model):
    """A Simulation using the learned majorant (params must set majorant=1)."""
    if isinstance(model, str):
        model = load_model(model)
    sim = binding.Simulation(dict(params, majorant=1), particles)
    sim.set_majorant_model(model["bits"], model["delta"])
    return sim
