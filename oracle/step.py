"""One preconditioned step of the hot path, composed from the oracle parts.

TEST INFRASTRUCTURE ONLY (see the package header).

converge the environment (CTMRG) -> energy and gradient (K-step unrolled
derivative from the converged environment, Sec. IV A) -> preconditioned
direction x = (N_local + delta I)^-1 g (Eqs. (4), (11), Sec. III B-C) with the
local metric taken from the converged environment.
"""
from __future__ import annotations

import time

from . import ctmrg, gradient, metric


def run_step(A, terms, chi: int, tol: float, max_iter: int, K: int,
             delta: float, cg_tol: float, cg_maxiter: int,
             eps: float = 1e-12, env=None) -> dict:
    t0 = time.perf_counter()
    env, n_iter, dl = ctmrg.converge(A, chi, tol, max_iter, eps, env)
    t1 = time.perf_counter()
    e, g = gradient.grad_K(A, terms, env, chi, K, eps)
    t2 = time.perf_counter()
    x, cg_it, res, brk = metric.precondition(env, A, g, delta, cg_tol,
                                             cg_maxiter)
    t3 = time.perf_counter()
    return dict(env=env, n_iter=n_iter, delta=dl, e=e, g=g.numpy(),
                x=x.numpy(), cg_iter=cg_it, cg_resid=res, breakdown=brk,
                spectra=ctmrg.corner_spectra(env).numpy(),
                seconds=dict(converge=t1 - t0, grad=t2 - t1,
                             precond=t3 - t2))
