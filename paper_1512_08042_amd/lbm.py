"""Differentiable lattice path: BGK roll-outs, Hermite coefficients and the
DSMC2LB projection as torch.autograd.Functions whose forward and backward
passes both run in the library's HIP kernels (include/dsmc.h).

The backward of a roll-out is the hand-written adjoint of the collide-and-
stream step (Section 3.1, relaxation time of Eq. (tau)), replayed from
checkpoints: the forward keeps the populations every `every` steps and the
backward recomputes one segment at a time.  Gradients reach the initial
populations, the body force g and the relaxation time tau; the Hermite and
projection adjoints (Eq. (discretefunctions), Eq. (nordercoefficients)) carry
a moment mismatch at coupling nodes back to the LB populations and to the
DSMC moment averages.  There is no CPU path: every call needs the GPU.
"""
from __future__ import annotations

import ctypes

import torch

from . import _lib
from ._lib import check, lib

NH = {0: 1, 1: 3, 2: 6, 3: 10}  # Hermite coefficients up to each order


def _stream() -> int:
    return torch.cuda.current_stream().cuda_stream


def _cfg(nx, ny, q, y_mode, tau, g):
    return _lib.LbmConfig(int(nx), int(ny), int(q), int(y_mode), float(tau), float(g), 0, 0)


def _f64(t: torch.Tensor, shape=None) -> torch.Tensor:
    if not t.is_cuda or t.dtype != torch.float64:
        raise TypeError("expected a CUDA float64 tensor")
    t = t.contiguous()
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError("expected shape %s, got %s" % (tuple(shape), tuple(t.shape)))
    return t


def _scalar(v) -> float:
    return float(v.detach().item()) if isinstance(v, torch.Tensor) else float(v)


def _like_param(value: torch.Tensor, p):
    if isinstance(p, torch.Tensor):
        return value.to(device=p.device, dtype=p.dtype).reshape(p.shape)
    return None


class LbmRollout(torch.autograd.Function):
    """f_N = nsteps lattice steps from f0 (device, float64 [Q][nx*ny])."""

    @staticmethod
    def forward(ctx, f0, g, tau, nx, ny, q, y_mode, nsteps, every):
        nn = nx * ny
        f0 = _f64(f0, (q, nn))
        cfg = _cfg(nx, ny, q, y_mode, _scalar(tau), _scalar(g))
        f = f0.detach().clone()
        tmp = torch.empty_like(f)
        nck = (nsteps + every - 1) // every
        ckpt = torch.empty((max(nck, 1), q, nn), dtype=torch.float64, device=f.device)
        check(lib().lbm_step_checkpointed(ctypes.byref(cfg), f.data_ptr(), tmp.data_ptr(), ckpt.data_ptr(),
                                          int(nsteps), int(every), _stream()), "lbm_step_checkpointed")
        ctx.ckpt = ckpt
        ctx.cfg = cfg
        ctx.meta = (nsteps, every)
        ctx.params = (g, tau)
        return f

    @staticmethod
    def backward(ctx, f_bar):
        nsteps, every = ctx.meta
        cfg = ctx.cfg
        lam = f_bar.detach().to(torch.float64).contiguous().clone()
        grad = torch.zeros(2, dtype=torch.float64, device=lam.device)
        size = ctypes.c_size_t()
        check(lib().lbm_adjoint_workspace(ctypes.byref(cfg), int(every), ctypes.byref(size)),
              "lbm_adjoint_workspace")
        work = torch.empty(int(size.value) + 256, dtype=torch.uint8, device=lam.device)
        wp = (work.data_ptr() + 255) & ~255
        check(lib().lbm_adjoint(ctypes.byref(cfg), ctx.ckpt.data_ptr(), int(nsteps), int(every), lam.data_ptr(),
                                grad.data_ptr(), wp, _stream()), "lbm_adjoint")
        g, tau = ctx.params
        ctx.ckpt = None
        return lam, _like_param(grad[0], g), _like_param(grad[1], tau), None, None, None, None, None, None


def rollout(f0, g, tau, nx, ny, q, y_mode=0, nsteps=1, every=20):
    """Differentiable roll-out; g and tau may be tensors that require grad."""
    if every < 1 or nsteps < 0:
        raise ValueError("need every >= 1 and nsteps >= 0")
    return LbmRollout.apply(f0, g, tau, int(nx), int(ny), int(q), int(y_mode), int(nsteps), int(every))


class HermiteMoments(torch.autograd.Function):
    """a[n][i] = sum_q f[q][nodes[i]] H(n)(xi_q) for n up to order."""

    @staticmethod
    def forward(ctx, f, nodes, q, order):
        f = _f64(f)
        nodes = nodes.to(torch.int32).contiguous()
        out = torch.empty((NH[order], nodes.numel()), dtype=torch.float64, device=f.device)
        check(lib().lbm_hermite_moments(int(q), int(order), f.data_ptr(), f.shape[1], nodes.data_ptr(),
                                        nodes.numel(), out.data_ptr(), _stream()), "lbm_hermite_moments")
        ctx.save_for_backward(nodes)
        ctx.meta = (q, order, f.shape)
        return out

    @staticmethod
    def backward(ctx, a_bar):
        (nodes,) = ctx.saved_tensors
        q, order, shape = ctx.meta
        f_bar = torch.zeros(shape, dtype=torch.float64, device=a_bar.device)
        a_bar = a_bar.detach().to(torch.float64).contiguous()
        check(lib().lbm_hermite_moments_adjoint(int(q), int(order), a_bar.data_ptr(), nodes.data_ptr(),
                                                nodes.numel(), f_bar.data_ptr(), shape[1], _stream()),
              "lbm_hermite_moments_adjoint")
        return f_bar, None, None, None


def hermite_moments(f, nodes, q, order):
    """Differentiable Hermite coefficients at distinct node ids."""
    return HermiteMoments.apply(f, nodes, int(q), int(order))


class ProjectMoments(torch.autograd.Function):
    """DSMC2LB projection of per-cell moment averages avg[11][ncells]."""

    @staticmethod
    def forward(ctx, avg, ppc, q, order, kT_over_m):
        avg = _f64(avg)
        ncells = avg.shape[1]
        out = torch.empty((q, ncells), dtype=torch.float64, device=avg.device)
        check(lib().dsmc_project_moments(avg.data_ptr(), ncells, int(ppc), float(kT_over_m), int(q), int(order),
                                         out.data_ptr(), _stream()), "dsmc_project_moments")
        ctx.save_for_backward(avg)
        ctx.meta = (ppc, q, order, kT_over_m)
        return out

    @staticmethod
    def backward(ctx, f_bar):
        (avg,) = ctx.saved_tensors
        ppc, q, order, kT = ctx.meta
        f_bar = f_bar.detach().to(torch.float64).contiguous()
        avg_bar = torch.empty_like(avg)
        check(lib().dsmc_project_moments_adjoint(f_bar.data_ptr(), avg.data_ptr(), avg.shape[1], int(ppc),
                                                 float(kT), int(q), int(order), avg_bar.data_ptr(), _stream()),
              "dsmc_project_moments_adjoint")
        return avg_bar, None, None, None, None


def project_moments(avg, ppc, q, order, kT_over_m=1.0):
    """Differentiable DSMC2LB projection."""
    return ProjectMoments.apply(avg, int(ppc), int(q), int(order), float(kT_over_m))


def coupling_mismatch(f_lb, nodes, f_dsmc, cells, q, order=3):
    """J = 1/2 sum_i sum_n (a(n)(f_lb at nodes[i]) - a(n)(f_dsmc at cells[i]))^2:
    the moment mismatch of the LB populations and the projected DSMC
    populations at the coupling nodes, differentiable in both."""
    a_lb = hermite_moments(f_lb, nodes, q, order)
    a_d = hermite_moments(f_dsmc, cells, q, order)
    return 0.5 * ((a_lb - a_d) ** 2).sum()
