"""C4v-symmetric real ansatz and QR-based CTMRG for it: the plain FP64 oracle.

TEST INFRASTRUCTURE ONLY (see the package header).

Sec. IV A uses a one-site C4v-symmetric real iPEPS (the sublattice spin
flip making the antiferromagnet a one-site problem) and obtains its
environment with a QR-based CTMRG; imposing the symmetry fixes the gauge.
The QR-CTMRG papers are cited but not reproduced, so this module fixes one
reading, written out step by step:

* ansatz: A_s = the average of A over the eight elements of the square's
  symmetry group acting on the virtual legs [l, u, r, d] (the four
  rotations, each with and without the left-right mirror), a linear
  projector; the energy is a function of A through A_s, so its gradient is
  the projection of the gradient at A_s;
* environment: one corner C (chi x chi, symmetric) and one edge T
  (chi x D^2 x chi, symmetric in its two chi legs) stand for all four
  corners and edges (ring order C T C T C T C T with the conventions of
  ctmrg.py); the double layer a of A_s is invariant under the rotations;
* start: the trace boundary (bond dimension D^2);
* one iteration: the enlarged corner M = T C T a as a (c D^2) x (c D^2)
  matrix (c the current bond dimension; M is symmetric); while c D^2 <=
  chi the bond grows without truncation (Q = identity); otherwise the kept
  space comes from one step of block subspace iteration with QR on b =
  chi + p columns (oversampling p = max(8, ceil(chi / 4)), b made
  even): Y = M V with V the previous iteration's b-column block
  (the first b unit vectors when there is none of that shape), the thin QR
  Y = Q0 R with diag R > 0 (a column whose R diagonal is below 1e-6 of the
  column scale |Y|_F / sqrt(b) is dropped: set to zero), then the
  Rayleigh-Ritz rotation B = Q0^T M Q0 = W Lambda W^T with the chi
  eigenvalues of largest |lambda| first (ties: the larger signed value)
  and the others after them, each group in descending signed order (a
  pair +-lambda is then never reordered from one iteration to the next),
  the rotated block Q0 W with every
  column's entry of largest |v_r| (1 + r / (2 n)) made positive, and Q its
  first chi columns; C' = Q^T M Q, T' = Q^T (T a) Q, each made exactly
  symmetric ((X + X^T) / 2 on its chi legs) and divided by its Frobenius
  norm; the rotated block is the next iteration's V.  No SVD of the
  (chi D^2)-dimensional corner is taken: the QR and a b x b
  eigendecomposition replace it, and the subspace converges together with
  the environment (the sign rule on the block keeps its basis the same from
  one iteration to the next at the fixed point, which makes the warm start
  consistent);
* convergence: the singular values of C (|eigenvalues|), sum-normalised,
  zero padded to chi; Delta = the 2-norm of their change.
* K-step gradient: A -> e(A_s, F^K(C*, T*, V*)) with the converged
  (C*, T*, V*) held fixed, reverse mode through all K iterations (the
  block V included), through the QR (PyTorch's thin-QR derivative) and the
  eigendecomposition (the symmetric-eigenvector derivative with the
  Lorentzian x / (x^2 + eta^2), eta = 1e-12 max|lambda|, in place of
  1 / (lambda_j - lambda_i)).

Parity status: pinned by tests/test_oracle_c4v.py: the projector property
and invariance of the ansatz, the energy and corner spectrum of the
converged environment against the general four-corner SVD CTMRG of
ctmrg.py on the same symmetric state, a product state in closed form, the
gradient against central finite differences of the same function, and the
gradient at a symmetric state equal to the projection of the general
gradient.
"""
from __future__ import annotations

import torch

from .ctmrg import F64, Env, double_layer, enlarged_corner


def symmetrize(A_site) -> torch.Tensor:
    """A_s: the group average of A[s, l, u, r, d] over the virtual legs."""
    A = torch.as_tensor(A_site, dtype=F64)
    out = torch.zeros_like(A)
    B = A
    for _ in range(4):
        out = out + B + B.permute(0, 3, 2, 1, 4)   # B and its mirror l <-> r
        B = B.permute(0, 4, 1, 2, 3)              # rotation: [d, l, u, r]
    return out / 8.0


def init_env(a: torch.Tensor):
    """Trace boundary: (C, T) of bond dimension D^2, normalised."""
    D2 = a.shape[0]
    D = int(round(D2 ** 0.5))
    t = torch.eye(D, dtype=F64).reshape(D2)
    C = torch.einsum("g,e,gebf->fb", t, t, a)
    T = torch.einsum("e,gebf->gfb", t, a)
    return C / torch.linalg.norm(C), T / torch.linalg.norm(T)


def block_size(chi: int) -> int:
    """b = chi + p, p = max(8, ceil(chi / 4)), even."""
    b = chi + max(8, -(-chi // 4))
    b += b % 2
    return b


def _qr_positive(Y):
    """Thin QR with diag R > 0; columns with a negligible R diagonal are
    set to zero."""
    Q, R = torch.linalg.qr(Y)
    d = torch.diagonal(R).detach()
    scale = torch.linalg.norm(Y.detach()) / Y.shape[1] ** 0.5
    s = torch.sign(d)
    s = torch.where(d.abs() <= 1e-6 * scale, torch.zeros_like(s), s)
    return Q * s[None, :]


def _sign_fix_columns(V):
    """Each column's entry of largest |v_r| (1 + r / (2 n)) made positive."""
    n = V.shape[0]
    wt = 1.0 + torch.arange(n, dtype=F64) / (2.0 * n)
    idx = torch.argmax(V.detach().abs() * wt[:, None], dim=0)
    s = torch.sign(V.detach()[idx, torch.arange(V.shape[1])])
    s = torch.where(s == 0, torch.ones_like(s), s)
    return V * s[None, :]


class _EighKept(torch.autograd.Function):
    """Eigenvectors of a symmetric matrix: the k of largest |lambda| (ties:
    the larger signed value) first, then the others, each group in
    descending signed order; with the broadened derivative."""

    @staticmethod
    def forward(ctx, B, k):
        lam, W = torch.linalg.eigh(B)
        lam, W = lam.flip(0), W.flip(1)          # descending signed order
        n = lam.shape[0]
        by_abs = sorted(range(n), key=lambda i: (-abs(float(lam[i])), i))
        kept = set(by_abs[:k])
        idx = [i for i in range(n) if i in kept] + \
              [i for i in range(n) if i not in kept]
        idx = torch.tensor(idx)
        lam, W = lam[idx], W[:, idx]
        ctx.save_for_backward(lam, W)
        return W

    @staticmethod
    def backward(ctx, Wb):
        lam, W = ctx.saved_tensors
        x = lam[None, :] - lam[:, None]          # x_ij = lambda_j - lambda_i
        eta = 1e-12 * lam.abs().max()
        F = x / (x * x + eta * eta)
        F.fill_diagonal_(0.0)
        Bb = W @ (F * (W.transpose(0, 1) @ Wb)) @ W.transpose(0, 1)
        return 0.5 * (Bb + Bb.transpose(0, 1)), None


def step(C, T, a, V, chi: int):
    """One iteration: (C', T', V') with V' the next warm-start block (None
    while the bond grows)."""
    D2 = a.shape[0]
    c = C.shape[0]
    M = enlarged_corner(C, T, T, a)
    n = M.shape[0]
    if n <= chi:
        Q = torch.eye(n, dtype=F64)
        Vn = None
    else:
        b = block_size(chi)
        if V is None or tuple(V.shape) != (n, b):
            V = torch.eye(n, dtype=F64)[:, :b]
        Q0 = _qr_positive(M @ V)
        B = Q0.transpose(0, 1) @ M @ Q0
        W = _EighKept.apply(0.5 * (B + B.transpose(0, 1)), chi)
        Vn = _sign_fix_columns(Q0 @ W)
        Q = Vn[:, :chi]
    k = Q.shape[1]
    Cn = Q.transpose(0, 1) @ M @ Q
    Cn = 0.5 * (Cn + Cn.transpose(0, 1))
    Tn = torch.einsum("jgx,jek,gebf,kby->xfy", Q.reshape(c, D2, k), T, a,
                      Q.reshape(c, D2, k))
    Tn = 0.5 * (Tn + Tn.permute(2, 1, 0))
    return Cn / torch.linalg.norm(Cn), Tn / torch.linalg.norm(Tn), Vn


def spectrum(C, chi: int) -> torch.Tensor:
    s = torch.linalg.svdvals(C.detach())
    s = s / s.sum()
    out = torch.zeros(chi, dtype=F64)
    out[:s.shape[0]] = s
    return out


def converge(A_site, chi: int, tol: float, max_iter: int, start=None):
    """QR-CTMRG of A_s from the trace boundary (or start = (C, T, V)) until
    Delta < tol or max_iter iterations: ((C, T, V), n_iter, Delta)."""
    a = double_layer(symmetrize(A_site))
    if start is None:
        C, T = init_env(a)
        V = None
    else:
        C, T, V = start
    s_old = spectrum(C, chi)
    dl = float("inf")
    it = 0
    with torch.no_grad():
        while it < max_iter:
            C, T, V = step(C, T, a, V, chi)
            it += 1
            s = spectrum(C, chi)
            dl = float(torch.linalg.norm(s - s_old))
            s_old = s
            if dl < tol:
                break
    return (C, T, V), it, dl


def as_env(C, T, chi: int) -> Env:
    """The four-corner environment of ctmrg.py (one site), zero padded."""
    c, D2 = C.shape[0], T.shape[1]
    Cp = torch.zeros(chi, chi, dtype=F64)
    Cp[:c, :c] = C
    Tp = torch.zeros(chi, D2, chi, dtype=F64)
    Tp[:c, :, :c] = T
    return Env([[Cp] for _ in range(4)], [[Tp] for _ in range(4)])


def _as_env_ad(C, T):
    return Env([[C] for _ in range(4)], [[T] for _ in range(4)])


def energy(A_site, terms, envc, chi: int) -> float:
    from .observables import energy as e_of
    C, T, _ = envc
    As = symmetrize(A_site)
    with torch.no_grad():
        return float(e_of(as_env(C, T, chi), As[None, None], terms))


def grad_K(A_site, terms, envc, chi: int, K: int):
    """(e, g): derivative of A -> e(A_s, F^K(C*, T*, V*)), the converged
    (C*, T*, V*) held fixed; g has the shape of A_site."""
    from .observables import energy as e_of
    A = torch.as_tensor(A_site, dtype=F64).detach().clone()
    A.requires_grad_(True)
    As = symmetrize(A)
    a = double_layer(As)
    C, T, V = (None if t is None else t.detach() for t in envc)
    for _ in range(K):
        C, T, V = step(C, T, a, V, chi)
    e = e_of(_as_env_ad(C, T), As[None, None], terms)
    (g,) = torch.autograd.grad(e, A)
    return float(e.detach()), g.detach()


def energy_K(A_site, terms, envc, chi: int, K: int) -> float:
    """e(A_s, F^K(C*, T*, V*)) without gradient (finite differences)."""
    from .observables import energy as e_of
    As = symmetrize(A_site)
    a = double_layer(As)
    C, T, V = envc
    with torch.no_grad():
        for _ in range(K):
            C, T, V = step(C, T, a, V, chi)
        return float(e_of(_as_env_ad(C, T), As[None, None], terms))
