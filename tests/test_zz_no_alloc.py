"""The allocation-free loss-gradient entry point (dsmc_mlp_loss_grad_noalloc)
against dsmc_mlp_loss_grad with caller-owned scratch, through the C ABI.

Both run the same kernels in the same order on the same inputs, so the
gradient and the loss must be bit-identical.  Two calls in a row, the second
with fewer samples, check that the library's scratch (which keeps the
previous call's contents) is fully rewritten by every call.  The size limit
and argument checks are host-side and launch nothing."""
import ctypes
import sys

import numpy as np
import pytest

from paper_2301_05985_amd import binding

pytestmark = pytest.mark.gpu


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr())


def _inputs(torch, n, seed):
    g = torch.Generator().manual_seed(seed)
    params = (torch.randn(binding.MLP_NPARAM, generator=g) * 0.2).float()
    x = torch.randn(n, 6, generator=g).float()
    y = (torch.randn(n, generator=g) + 2.0).float()
    y[::97] = float("nan")  # rows without a label are skipped
    return [t.to("cuda:0") for t in (params, x, y)]


def _reference(L, torch, params, x, y, n, tau, stream):
    grad = torch.empty(binding.MLP_NPARAM, device="cuda:0")
    loss = torch.empty(1, device="cuda:0")
    scratch = torch.empty(L.dsmc_mlp_scratch_floats(n) + 2, device="cuda:0")
    binding.check(L.dsmc_mlp_loss_grad(_ptr(params), _ptr(x), _ptr(y), n, tau, _ptr(grad), _ptr(loss),
                                       _ptr(scratch), ctypes.c_void_p(stream)), "dsmc_mlp_loss_grad")
    return grad, loss


def _noalloc(L, torch, params, x, y, n, tau, stream):
    grad = torch.full((binding.MLP_NPARAM,), float("nan"), device="cuda:0")
    loss = torch.full((1,), float("nan"), device="cuda:0")
    binding.check(L.dsmc_mlp_loss_grad_noalloc(_ptr(params), _ptr(x), _ptr(y), n, tau, _ptr(grad), _ptr(loss),
                                               ctypes.c_void_p(stream)), "dsmc_mlp_loss_grad_noalloc")
    return grad, loss


def test_noalloc_loss_grad_matches_scratch_version(gpu):
    import torch
    print("[gpu case] no-alloc loss/grad: 3000 then 700 samples", flush=True)
    sys.stdout.flush()
    L = binding.load()
    stream = torch.cuda.current_stream().cuda_stream
    for n, seed, tau in ((3000, 1, 0.95), (700, 2, 0.8)):
        params, x, y = _inputs(torch, n, seed)
        g_ref, l_ref = _reference(L, torch, params, x, y, n, tau, stream)
        g_new, l_new = _noalloc(L, torch, params, x, y, n, tau, stream)
        torch.cuda.synchronize()
        a, b = g_ref.cpu().numpy(), g_new.cpu().numpy()
        assert np.isfinite(a).all() and np.abs(a).max() > 0
        assert np.array_equal(a, b), np.flatnonzero(a != b)[:5]
        assert np.array_equal(l_ref.cpu().numpy(), l_new.cpu().numpy())


def test_noalloc_rejects_sizes_beyond_its_scratch(gpu):
    import torch
    L = binding.load()
    params, x, y = _inputs(torch, 8, 3)
    out = torch.empty(binding.MLP_NPARAM + 1, device="cuda:0")
    big = binding.MLP_NOALLOC_MAX + 1
    rc = L.dsmc_mlp_loss_grad_noalloc(_ptr(params), _ptr(x), _ptr(y), big, 0.95, _ptr(out), _ptr(out), None)
    assert rc == -1
    rc = L.dsmc_mlp_loss_grad_noalloc(_ptr(params), _ptr(x), _ptr(y), 0, 0.95, _ptr(out), _ptr(out), None)
    assert rc == -1
    rc = L.dsmc_mlp_loss_grad_noalloc(None, _ptr(x), _ptr(y), 8, 0.95, _ptr(out), _ptr(out), None)
    assert rc == -1
    # the largest admissible size runs
    params, x, y = _inputs(torch, binding.MLP_NOALLOC_MAX, 4)
    g_ref, l_ref = _reference(L, torch, params, x, y, binding.MLP_NOALLOC_MAX, 0.95,
                              torch.cuda.current_stream().cuda_stream)
    g_new, l_new = _noalloc(L, torch, params, x, y, binding.MLP_NOALLOC_MAX, 0.95,
                            torch.cuda.current_stream().cuda_stream)
    torch.cuda.synchronize()
    assert np.array_equal(g_ref.cpu().numpy(), g_new.cpu().numpy())
    assert np.array_equal(l_ref.cpu().numpy(), l_new.cpu().numpy())
