"""Energy gradient dE/dA: the plain FP64 oracle.

TEST INFRASTRUCTURE ONLY (see the package header).

The paper differentiates the energy by backward-mode AD through the last
steps of the contraction (Sec. III A; Sec. IV A, the "(3+20)" configuration).
The oracle does the same with PyTorch's CPU autograd over its own einsums; the
only hand-written derivative is that of the truncated SVD of a cut matrix,
which uses the FULL spectrum (LAPACK) so that the discarded singular vectors
enter exactly:

  Mbar = U [ (F o (U^T Ubar - Ubar^T U)) S + S (F o (V^T Vbar - Vbar^T V))
             + diag(Sbar) ] V^T,   F_ij = 1/(s_j^2 - s_i^2)  (i != j),

with the cotangents of the discarded triplets equal to zero, F_ij = 0 when
both i and j are discarded, and the Lorentzian form x/(x^2 + eta^2),
eta = 1e-12 * s_1^2, in place of 1/x (it differs from 1/x only for
near-degenerate pairs).

Gradient modes (A is real and enters both ket and bra; the gradient is with
respect to every real entry of every unit-cell tensor):
  grad_full(N)  derivative of A -> e(A, env_N(A)), through the trace-boundary
                start and N iterations;
  grad_K        derivative of A -> e(A, F^K(A, env*)) with the converged env*
                held fixed: the unrolled "(3+20)" form with K = 20;
  grad_fp       grad_K with K doubled until the cotangent that reaches env* is
                below 1e-13 of the one leaving the last step: the fixed-point
                gradient.

Parity status: pinned by central finite differences of the same function
(tests/test_oracle_grad.py) and by exact invariances (<g, A> = 0).
"""
from __future__ import annotations

import torch

from .ctmrg import (F64, Env, Lattice, as_sites, ctm_step, cut_svd,
                    double_layer, init_env)
from .observables import energy


class _TruncatedSVD(torch.autograd.Function):
    @staticmethod
    def forward(ctx, M, k_fn):
        U, S, V = cut_svd(M)
        k = k_fn(S)
        ctx.save_for_backward(U, S, V)
        ctx.k = k
        return U[:, :k].clone(), S[:k].clone(), V[:, :k].clone()

    @staticmethod
    def backward(ctx, gU, gS, gV):
        U, S, V = ctx.saved_tensors
        k = ctx.k
        n = S.shape[0]
        Ub = torch.zeros(n, n, dtype=F64)
        Vb = torch.zeros(n, n, dtype=F64)
        Sb = torch.zeros(n, dtype=F64)
        Ub[:, :k] = gU
        Vb[:, :k] = gV
        Sb[:k] = gS
        s2 = S * S
        x = s2[None, :] - s2[:, None]            # x_ij = s_j^2 - s_i^2
        eta = 1e-12 * s2[0]
        F = x / (x * x + eta * eta)
        F.fill_diagonal_(0.0)
        kept = torch.arange(n) < k
        F = F * (kept[:, None] | kept[None, :]).to(F64)
        Au = U.transpose(0, 1) @ Ub
        Bv = V.transpose(0, 1) @ Vb
        G = (F * (Au - Au.transpose(0, 1))) * S[None, :] \
            + S[:, None] * (F * (Bv - Bv.transpose(0, 1))) + torch.diag(Sb)
        return U @ G @ V.transpose(0, 1), None


def differentiable_svd(M, k_fn):
    return _TruncatedSVD.apply(M, k_fn)


def _setup(A):
    A = torch.as_tensor(A, dtype=F64).detach().clone().requires_grad_(True)
    lat = Lattice(A.shape[1], A.shape[0])
    a_sites = [double_layer(t) for t in as_sites(A)]
    return A, lat, a_sites


def grad_full(A, terms, chi: int, n_iter: int, eps: float = 1e-12):
    """(e, g): derivative through the start and n_iter iterations."""
    A, lat, a_sites = _setup(A)
    env = init_env(a_sites, lat, chi)
    for _ in range(n_iter):
        env = ctm_step(a_sites, env, lat, chi, eps, svd_fn=differentiable_svd)
    e = energy(env, A, terms)
    (g,) = torch.autograd.grad(e, A)
    return float(e.detach()), g.detach()


def _unrolled(A, terms, env_star: Env, chi: int, K: int, eps: float,
              env_leaves: bool):
    A, lat, a_sites = _setup(A)
    env = env_star.detach()
    leaves = []
    if env_leaves:
        for row in env.C + env.T:
            for t in row:
                t.requires_grad_(True)
                leaves.append(t)
    for _ in range(K):
        env = ctm_step(a_sites, env, lat, chi, eps, svd_fn=differentiable_svd)
    last = [t for row in env.C + env.T for t in row]
    e = energy(env, A, terms)
    return A, e, leaves, last


def grad_K(A, terms, env_star: Env, chi: int, K: int, eps: float = 1e-12):
    """(e, g): derivative of A -> e(A, F^K(A, env*)), env* held fixed."""
    A, e, _, _ = _unrolled(A, terms, env_star, chi, K, eps, False)
    (g,) = torch.autograd.grad(e, A)
    return float(e.detach()), g.detach()


def grad_fp(A, terms, env_star: Env, chi: int, K0: int = 20,
            rel: float = 1e-13, K_max: int = 640, eps: float = 1e-12):
    """(e, g, K): grad_K with K doubled until the cotangent reaching env* is
    below ``rel`` times the cotangent of the final environment."""
    K = K0
    while True:
        A_, e, leaves, last = _unrolled(A, terms, env_star, chi, K, eps, True)
        grads = torch.autograd.grad(e, [A_] + leaves + last,
                                    allow_unused=True)
        g = grads[0]
        into = grads[1:1 + len(leaves)]
        out = grads[1 + len(leaves):]
        n_in = sum(float((t * t).sum()) for t in into if t is not None) ** 0.5
        n_out = sum(float((t * t).sum()) for t in out if t is not None) ** 0.5
        if n_in <= rel * max(n_out, 1e-300) or K >= K_max:
            return float(e.detach()), g.detach(), K
        K *= 2


def energy_of(A, terms, env_star: Env, chi: int, K: int,
              eps: float = 1e-12) -> float:
    """e(A, F^K(A, env*)) without gradient (finite-difference checks)."""
    A = torch.as_tensor(A, dtype=F64)
    lat = Lattice(A.shape[1], A.shape[0])
    a_sites = [double_layer(t) for t in as_sites(A)]
    env = env_star.detach()
    with torch.no_grad():
        for _ in range(K):
            env = ctm_step(a_sites, env, lat, chi, eps)
        return float(energy(env, A, terms))


def energy_full(A, terms, chi: int, n_iter: int, eps: float = 1e-12) -> float:
    """e(A, env_N(A)) from the trace-boundary start, without gradient."""
    A = torch.as_tensor(A, dtype=F64)
    lat = Lattice(A.shape[1], A.shape[0])
    a_sites = [double_layer(t) for t in as_sites(A)]
    with torch.no_grad():
        env = init_env(a_sites, lat, chi)
        for _ in range(n_iter):
            env = ctm_step(a_sites, env, lat, chi, eps)
        return float(energy(env, A, terms))
