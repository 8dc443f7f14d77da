"""torch.autograd interface over the library's device path.

`energy(A, ctx, terms)` is the energy per site as a differentiable function
of the site tensors A (a CUDA float64 tensor [Ly][Lx][d][D][D][D][D]): the
forward pass loads A into the library context, converges the CTMRG
environment (ctm_converge) and evaluates the energy and its gradient in one
call (ipeps_energy_grad_dev: the reverse pass through the unrolled CTMRG
iterations, Sec. III A, in the gradient mode and checkpointing that the
context's options select); the backward pass scales the stored gradient by
the incoming cotangent.  `precondition(ctx, g)` returns the preconditioned
direction x = (N_env + delta)^-1 g of Eq. (9) with the local metric of the
converged environment (precond_apply_dev).

Only argument marshalling happens here: every step of the computation runs
in the library's kernels, and A, g and x stay on the device.  The library
runs on the context's own HIP stream; the current torch stream is
synchronised before each call, and each call returns with its results
written.
"""
from __future__ import annotations

import torch

from . import binding


def _check(t: torch.Tensor, name: str, shape=None) -> torch.Tensor:
    if not isinstance(t, torch.Tensor) or not t.is_cuda or \
            t.dtype != torch.float64:
        raise TypeError(f"{name} must be a CUDA float64 tensor")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} has shape {tuple(t.shape)}, the context "
                         f"expects {tuple(shape)}")
    return t.contiguous()


class Energy(torch.autograd.Function):
    """e(A) with de/dA from the library (see the module docstring)."""

    @staticmethod
    def forward(ctx, A, lib_ctx, terms, tol, max_iter):
        A = _check(A, "A", lib_ctx.shape)
        g = torch.empty_like(A)
        torch.cuda.current_stream(A.device).synchronize()
        lib_ctx.set_state_dev(A.data_ptr())
        n_it, delta, ok = lib_ctx.converge(tol, max_iter)
        e = lib_ctx.energy_grad_dev(terms, g.data_ptr())
        ctx.save_for_backward(g)
        out = torch.tensor(e, dtype=torch.float64, device=A.device)
        lib_ctx.last_converge = (n_it, delta, ok)
        return out

    @staticmethod
    def backward(ctx, ge):
        (g,) = ctx.saved_tensors
        return ge * g, None, None, None, None


def energy(A: torch.Tensor, lib_ctx: binding.Context, terms,
           tol: float = 1e-10, max_iter: int = 200) -> torch.Tensor:
    """Energy per site (0-d tensor) whose backward gives de/dA.

    When no gradient can be asked for (A does not require one, or autograd
    is off) only the energy is evaluated: the reverse pass through the
    unrolled iterations, several times the cost of the energy itself, is
    skipped."""
    if torch.is_grad_enabled() and A.requires_grad:
        return Energy.apply(A, lib_ctx, terms, tol, max_iter)
    A = _check(A, "A", lib_ctx.shape)
    torch.cuda.current_stream(A.device).synchronize()
    lib_ctx.set_state_dev(A.data_ptr())
    lib_ctx.last_converge = lib_ctx.converge(tol, max_iter)
    e, _ = lib_ctx.energy_grad(terms, grad=False)
    return torch.tensor(e, dtype=torch.float64, device=A.device)


def precondition(lib_ctx: binding.Context, g: torch.Tensor,
                 delta: float = 1e-4, cg_tol: float = 0.0,
                 cg_maxiter: int = 20) -> torch.Tensor:
    """x = (N_env + delta)^-1 g on the context's converged environment."""
    g = _check(g, "g", lib_ctx.shape)
    x = torch.empty_like(g)
    torch.cuda.current_stream(g.device).synchronize()
    lib_ctx.precond_dev(g.data_ptr(), x.data_ptr(), delta, cg_tol,
                        cg_maxiter)
    return x
