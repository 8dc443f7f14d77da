"""Full tangent-space metric (Eq. (10)) applied matrix-free, and GMRES:
the plain FP64 oracle.

TEST INFRASTRUCTURE ONLY (see the package header).

Sec. III A defines the metric N_ij = <d_i psi | d_j psi> of the iPEPS
manifold, an infinite sum of terms with the ket vacancy and the bra vacancy
at all separations (Eq. (10)), and obtains its action on a tangent vector B
as the derivative with respect to the bra of the overlap with the tangent
vector, i.e. a mixed second derivative of the norm.  For the infinite,
normalised state the per-site quantity is used here:

  F(A_ket, A_bra) = log kappa,  kappa = n_site n_corner / (n_h n_v)

with the CTMRG environment of the double layer a = sum_s A_ket (x) A_bra
(fused leg (k, k') with k from the ket), run K iterations from the converged
environment env* of A (as the K-step gradient), and the four networks of a
1x1 cell: n_site the ring of eight environment tensors around a, n_corner
Tr(C1 C2 C3 C4), n_h the top and bottom rows C1 T1 C2 / C4 T3 C3 closed on
each other, n_v the left and right columns C1 C2 / T4 T2 / C4 C3 closed on
each other.  Its mixed Hessian is the connected metric (the log removes the
part along the state itself):

  N B = d/dA_bra [ D_ket F (A, A)[B] ],

evaluated here by a central difference in the ket direction of the bra
gradient (reverse mode, as the gradient):

  N B ~ (grad_bra F(A + h B, A) - grad_bra F(A - h B, A)) / (2 h),
  h = rel_step |A| / |B|  (rel_step = 1e-5 by default).

The networks are closed, so F does not change under gauge transformations
of the environment bonds, and F(A_ket, A_bra) = F(A_bra, A_ket); F(c A_ket,
A_bra) = F + log c.  Hence N is symmetric, N A = 0, <grad_bra F, A> = 1, and
the infinitesimal gauge transformations of the virtual bonds are (up to the
truncation of the environment) zero modes, which the local metric does not
have (Sec. III B).

The preconditioned direction solves (N + delta I) x = g by restarted GMRES
(Sec. III C: one cycle of 30 Krylov vectors), x0 = 0, Arnoldi with modified
Gram-Schmidt, the small least-squares problem by Givens rotations, stopping
early when the residual estimate is below tol |g| or when the new Krylov
vector is below 1e-12 of the product it came from (an invariant subspace).

Parity status: pinned by tests/test_oracle_full_metric.py: the product-state
closed form (the projected metric (I - phi phi^T / |phi|^2) / |phi|^2 on the
index-0 block, zero elsewhere) for D = 1 and D = 2, the symmetry of N, N A =
0, the gauge zero modes, the stationarity of log kappa in the environment at
the fixed point (the first derivative equals the single-site one), the
O(h^2) consistency of the difference, and GMRES against the minimal-residual
solution over an explicit Krylov basis and against direct solves.
"""
from __future__ import annotations

import numpy as np
import torch

from .ctmrg import F64, Lattice, ctm_step
from .gradient import differentiable_svd


def mixed_double_layer(Ak: torch.Tensor, Ab: torch.Tensor) -> torch.Tensor:
    """a[(l l'), ...] = sum_s Ak[s,l,u,r,d] Ab[s,l',u',r',d']."""
    D = Ak.shape[1]
    a = torch.einsum("slurd,sLURD->lLuUrRdD", Ak, Ab)
    return a.reshape(D * D, D * D, D * D, D * D)


def log_kappa_env(env, a) -> torch.Tensor:
    """log |kappa| of a 1x1 cell from its environment and double layer."""
    C, T = [env.C[c][0] for c in range(4)], [env.T[c][0] for c in range(4)]
    ring = torch.einsum("ij,jek,km,mbn,np,pzq,qw,wgi->gebz",
                        C[0], T[0], C[1], T[1], C[2], T[2], C[3], T[3])
    n_site = torch.einsum("gebz,gebz->", ring, a)
    n_corner = torch.einsum("ij,jk,kl,li->", C[0], C[1], C[2], C[3])
    n_h = torch.einsum("ij,jek,km,mn,neq,qi->", C[0], T[0], C[1], C[2],
                       T[2], C[3])
    n_v = torch.einsum("ij,jk,kel,lm,mn,nei->", C[0], C[1], T[1], C[2],
                       C[3], T[3])
    return (torch.log(torch.abs(n_site)) + torch.log(torch.abs(n_corner)) -
            torch.log(torch.abs(n_h)) - torch.log(torch.abs(n_v)))


def log_kappa(Ak, Ab, env_star, chi: int, K: int, eps: float = 1e-12):
    """F(A_ket, A_bra): K CTMRG iterations of the mixed double layer from
    env*, then log kappa (differentiable in both tensors)."""
    a = mixed_double_layer(Ak, Ab)
    lat = Lattice(1, 1)
    env = env_star.detach()
    for _ in range(K):
        env = ctm_step([a], env, lat, chi, eps, svd_fn=differentiable_svd)
    return log_kappa_env(env, a)


def grad_bra(Ak, Ab, env_star, chi: int, K: int) -> np.ndarray:
    """d F / d A_bra at (A_ket, A_bra), site tensors [d][D]^4."""
    Ak = torch.as_tensor(Ak, dtype=F64)
    Ab = torch.as_tensor(Ab, dtype=F64).clone().requires_grad_(True)
    F = log_kappa(Ak, Ab, env_star, chi, K)
    (g,) = torch.autograd.grad(F, Ab)
    return g.numpy()


def metric_apply(A, B, env_star, chi: int, K: int,
                 rel_step: float = 1e-5) -> np.ndarray:
    """N B by the central difference of the bra gradient along B in the
    ket (1x1 cell: A, B are [d][D]^4 site tensors)."""
    A = np.asarray(A, dtype=np.float64)
    B = np.asarray(B, dtype=np.float64)
    nb = np.linalg.norm(B)
    if nb == 0.0:
        return np.zeros_like(B)
    h = rel_step * np.linalg.norm(A) / nb
    gp = grad_bra(A + h * B, A, env_star, chi, K)
    gm = grad_bra(A - h * B, A, env_star, chi, K)
    return (gp - gm) / (2.0 * h)


def gmres(apply_fn, g: np.ndarray, m: int = 30, tol: float = 0.0):
    """One GMRES cycle of at most m Krylov vectors from x0 = 0 for
    apply_fn(x) = g (flat vectors).  Returns (x, vectors used, relative
    residual estimate |g - apply_fn(x)| / |g| from the rotated Hessenberg
    system)."""
    g = np.asarray(g, dtype=np.float64).ravel()
    beta = np.linalg.norm(g)
    if beta == 0.0:
        return np.zeros_like(g), 0, 0.0
    V = [g / beta]
    H = np.zeros((m + 1, m))
    cs, sn = np.zeros(m), np.zeros(m)
    e = np.zeros(m + 1)
    e[0] = beta
    k = 0
    for j in range(m):
        # Arnoldi step, modified Gram-Schmidt
        w = np.asarray(apply_fn(V[j]), dtype=np.float64).ravel()
        wn = np.linalg.norm(w)
        for i in range(j + 1):
            H[i, j] = w @ V[i]
            w = w - H[i, j] * V[i]
        hn = np.linalg.norm(w)
        H[j + 1, j] = hn
        # the earlier Givens rotations applied to the new column, then the
        # rotation that zeroes its subdiagonal entry
        for i in range(j):
            t = cs[i] * H[i, j] + sn[i] * H[i + 1, j]
            H[i + 1, j] = -sn[i] * H[i, j] + cs[i] * H[i + 1, j]
            H[i, j] = t
        r = np.hypot(H[j, j], H[j + 1, j])
        cs[j], sn[j] = H[j, j] / r, H[j + 1, j] / r
        H[j, j], H[j + 1, j] = r, 0.0
        e[j + 1] = -sn[j] * e[j]
        e[j] = cs[j] * e[j]
        k = j + 1
        # stop at the tolerance, or when the Krylov space is invariant up to
        # rounding (the new vector is below 1e-12 of the product it came
        # from): then x solves the system exactly
        if abs(e[j + 1]) <= tol * beta or hn <= 1e-12 * wn:
            break
        V.append(w / hn)
    # back substitution with the triangular k x k block
    y = np.zeros(k)
    for i in range(k - 1, -1, -1):
        y[i] = (e[i] - H[i, i + 1:k] @ y[i + 1:k]) / H[i, i]
    x = sum(y[i] * V[i] for i in range(k))
    return x, k, abs(e[k]) / beta


def precondition_full(A, g, env_star, chi: int, K: int, delta: float,
                      m: int = 30, tol: float = 0.0, rel_step: float = 1e-5):
    """x = (N + delta I)^-1 g by one GMRES cycle (1x1 cell)."""
    A = np.asarray(A, dtype=np.float64)
    site = A.reshape(A.shape[2:]) if A.ndim == 7 else A
    gs = np.asarray(g, dtype=np.float64).reshape(site.shape)

    def op(v):
        v = v.reshape(site.shape)
        return (metric_apply(site, v, env_star, chi, K, rel_step) +
                delta * v).ravel()

    x, k, res = gmres(op, gs.ravel(), m, tol)
    return x.reshape(np.asarray(g).shape), k, res


def precondition_local_gmres(env_star, A, g, delta: float, m: int = 30,
                             tol: float = 0.0):
    """x = (N_local + delta I)^-1 g per unit-cell site by one GMRES cycle
    (the Krylov solve of Sec. III C applied to the local metric, Eq. (11)).
    Returns (x, largest number of vectors used, largest residual)."""
    from .metric import local_metric, metric_apply as local_apply
    A = torch.as_tensor(A, dtype=F64)
    g = torch.as_tensor(g, dtype=F64)
    Ly, Lx = A.shape[0], A.shape[1]
    x = torch.zeros_like(g)
    k_max, r_max = 0, 0.0
    for y in range(Ly):
        for xx in range(Lx):
            E, Z = local_metric(env_star, y * Lx + xx, A[y, xx])
            shape = g[y, xx].shape

            def op(v):
                v = torch.as_tensor(v.reshape(shape))
                return (local_apply(E, Z, v) + delta * v).numpy().ravel()

            xs, k, res = gmres(op, g[y, xx].numpy().ravel(), m, tol)
            x[y, xx] = torch.as_tensor(xs.reshape(shape))
            k_max, r_max = max(k_max, k), max(r_max, res)
    return x, k_max, r_max
