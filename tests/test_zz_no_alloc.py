"""The no-allocation adjoint step (lbm_adjoint_step_noalloc) against the
workspace entry point it stands for (lbm_adjoint_step), through the C ABI:
identical cotangents and gradients, bit for bit (the same kernels and
summation order), on two calls in a row, the second on a smaller lattice
whose blocks reuse a prefix of the library's scratch array."""
import ctypes

import numpy as np
import pytest
import torch

import inputs
from oracle import oracle as O

pytestmark = pytest.mark.gpu


def _p(t):
    return ctypes.c_void_p(t.data_ptr())


@pytest.mark.parametrize("order", ["large_then_small"])
def test_noalloc_adjoint_step_matches_workspace_step(order):
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1512_08042_amd import _lib

    L = _lib.lib()
    s = torch.cuda.current_stream()
    sp = ctypes.c_void_p(s.cuda_stream)
    for nx, ny, q, y_mode, tau, g in ((1024, 512, 37, 1, 38.9, 1e-4), (300, 200, 9, 0, 0.83, 2e-3)):
        lat = O.lattice(q)
        f = torch.as_tensor(inputs.populations(nx + q, lat["w"], nx * ny, 0.1), device="cuda").contiguous()
        lam = torch.as_tensor(inputs.populations(ny + q, lat["w"], nx * ny, 0.5), device="cuda").contiguous()
        cfg = _lib.LbmConfig(nx, ny, q, y_mode, tau, g, 0, 0)
        size = ctypes.c_size_t()
        assert L.lbm_adjoint_workspace(ctypes.byref(cfg), 0, ctypes.byref(size)) == 0
        work = torch.empty(size.value, dtype=torch.uint8, device="cuda")
        out_a, out_b = torch.empty_like(lam), torch.empty_like(lam)
        grad_a = torch.tensor([0.25, -0.5], dtype=torch.float64, device="cuda")
        grad_b = grad_a.clone()
        assert L.lbm_adjoint_step(ctypes.byref(cfg), _p(f), _p(lam), _p(out_a), _p(grad_a), _p(work), sp) == 0
        assert L.lbm_adjoint_step_noalloc(ctypes.byref(cfg), _p(f), _p(lam), _p(out_b), _p(grad_b), sp) == 0
        torch.cuda.synchronize()
        assert torch.equal(out_a, out_b), (nx, ny, q)
        assert torch.equal(grad_a, grad_b), (nx, ny, q, grad_a.tolist(), grad_b.tolist())
        assert grad_a[0].item() != 0.25  # the step added its contribution
        del work


def test_noalloc_adjoint_step_rejects_oversized_lattices():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1512_08042_amd import _lib

    L = _lib.lib()
    p = ctypes.c_void_p(256)  # never dereferenced: rejected before any GPU work
    big = _lib.LbmConfig(2049, 2048, 9, 0, 0.8, 0.0, 0, 0)  # 4,196,352 nodes > 4,194,304
    assert L.lbm_adjoint_step_noalloc(ctypes.byref(big), p, p, p, p, None) == _lib.ECAPACITY
    ok = _lib.LbmConfig(2048, 2048, 9, 0, 0.8, 0.0, 0, 0)  # exactly the limit: accepted (same pointer -> EINVAL)
    assert L.lbm_adjoint_step_noalloc(ctypes.byref(ok), p, p, p, p, None) == _lib.EINVAL
