"""Local-metric preconditioner and the preconditioned gradient: the oracle.

TEST INFRASTRUCTURE ONLY (see the package header).

* Local metric (Eq. (11)): the first term of the tangent-space metric
  N_ij = <d_i psi | d_j psi> (Eqs. (9)-(10)), i.e. the single-site
  environment of a site tensor.  For site s with ring E[(l u r d), (l' u' r'
  d')] (ket legs unprimed, bra legs primed; the eight environment tensors
  with the site removed) the operator acts on x[s_phys, l, u, r, d] as
      (N x)[t, l', u', r', d'] = sum_{lurd} E[(lurd), (l'u'r'd')] x[t, lurd] / Z
  with the physical index passed through and Z = <A, E A> the norm of the
  3x3 block.  It ignores the Hamiltonian, as the paper notes.
* Regularisation (Sec. III B): P = N + delta I.
* Preconditioned gradient (Eq. (4), Sec. III C): g' = P^-1 g, solved
  implicitly.  The paper uses one GMRES cycle of dimension 30; P is symmetric
  (the environment is invariant under exchanging ket and bra), so this oracle
  uses plain conjugate gradients (Hestenes-Stiefel, x0 = 0, FP64) and, for
  comparison, a direct dense solve.
* Large unit cells (Sec. IV B): one independent operator and one independent
  solve per unit-cell tensor.

Parity status: pinned by tests/test_oracle_metric.py (CG against the direct
solve and against the Krylov-space minimiser, delta -> infinity, the
quadratic-model identity of Eq. (5), the product-state closed form).
"""
from __future__ import annotations

import torch

from .ctmrg import F64, Env
from .observables import site_environment


def local_metric(env: Env, s: int, A_site) -> tuple:
    """(E, Z): E as a [ket (D^4), bra (D^4)] matrix and the norm Z."""
    A_site = torch.as_tensor(A_site, dtype=F64)
    D = A_site.shape[1]
    E4 = site_environment(env, s)                       # [l, u, r, d] fused
    E8 = E4.reshape(D, D, D, D, D, D, D, D)             # l l' u u' r r' d d'
    E = E8.permute(0, 2, 4, 6, 1, 3, 5, 7).reshape(D ** 4, D ** 4)
    a = A_site.reshape(A_site.shape[0], D ** 4)
    Z = torch.einsum("sk,kb,sb->", a, E, a)
    return E, Z


def metric_apply(E, Z, x_site):
    """(N x) for one site: x[t, ket] -> sum_ket E[ket, bra] x[t, ket] / Z."""
    x = torch.as_tensor(x_site, dtype=F64)
    d = x.shape[0]
    y = x.reshape(d, -1) @ E / Z
    return y.reshape(x.shape)


def cg(apply_fn, g, delta: float, tol: float, maxiter: int):
    """Conjugate gradients on (N + delta I) x = g from x0 = 0.

    Stops when ||r|| <= tol ||g|| or after ``maxiter`` iterations.  Returns
    (x, n_iter, rel_resid, breakdown); breakdown means p^T (N + delta) p <= 0
    was met and the current x is returned.
    """
    g = torch.as_tensor(g, dtype=F64)
    x = torch.zeros_like(g)
    r = g.clone()
    p = r.clone()
    gnorm = float(torch.linalg.norm(g))
    if gnorm == 0.0:
        return x, 0, 0.0, False
    rr = float((r * r).sum())
    it = 0
    while it < maxiter and rr ** 0.5 > tol * gnorm:
        Ap = apply_fn(p) + delta * p
        pAp = float((p * Ap).sum())
        if not pAp > 0.0:
            return x, it, rr ** 0.5 / gnorm, True
        alpha = rr / pAp
        x = x + alpha * p
        r = r - alpha * Ap
        rr_new = float((r * r).sum())
        p = r + (rr_new / rr) * p
        rr = rr_new
        it += 1
    return x, it, rr ** 0.5 / gnorm, False


def precondition(env: Env, A, g, delta: float, tol: float, maxiter: int):
    """x = (N_local + delta I)^-1 g, one CG per unit-cell site.

    Returns (x, max n_iter, max relative residual, any breakdown)."""
    A = torch.as_tensor(A, dtype=F64)
    g = torch.as_tensor(g, dtype=F64)
    Ly, Lx = A.shape[0], A.shape[1]
    x = torch.zeros_like(g)
    n_it, res, brk = 0, 0.0, False
    for y in range(Ly):
        for xx in range(Lx):
            s = y * Lx + xx
            E, Z = local_metric(env, s, A[y, xx])
            xs, it, rr, b = cg(lambda v: metric_apply(E, Z, v), g[y, xx],
                               delta, tol, maxiter)
            x[y, xx] = xs
            n_it, res, brk = max(n_it, it), max(res, rr), brk or b
    return x, n_it, res, brk


def solve_direct(env: Env, A, g, delta: float):
    """Dense LU solve of (N_local + delta I) x = g, per site."""
    A = torch.as_tensor(A, dtype=F64)
    g = torch.as_tensor(g, dtype=F64)
    Ly, Lx = A.shape[0], A.shape[1]
    x = torch.zeros_like(g)
    for y in range(Ly):
        for xx in range(Lx):
            s = y * Lx + xx
            E, Z = local_metric(env, s, A[y, xx])
            d = A.shape[2]
            Nop = E.transpose(0, 1) / Z + delta * torch.eye(E.shape[0],
                                                            dtype=F64)
            xs = torch.linalg.solve(Nop, g[y, xx].reshape(d, -1).T).T
            x[y, xx] = xs.reshape(g[y, xx].shape)
    return x
