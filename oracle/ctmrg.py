"""CTMRG environment of an iPEPS: the plain FP64 oracle.

TEST INFRASTRUCTURE ONLY (see the package header).

The paper obtains the environment tensors of the energy network (Sec. III A,
the "gray circles" of Eq. (7)) by a CTMRG contraction and leaves the scheme to
the contractor.  This oracle fixes one scheme, written out step by step:

* double-layer tensor a = sum_s A_s (x) A_s (A is real, so conj(A) = A), every
  virtual leg fused as (ket k, bra k') -> k*D + k';
* trace-boundary start: every environment tensor is a double layer whose
  outward legs are closed with delta_{k k'}, zero padded to chi;
* one iteration = the simultaneous four-corner move: for every 2x2 plaquette
  the four enlarged corners Q_c = T_{c-1} C_c T_c a, and for each of its four
  cuts the half-system matrix M = Q_a Q_b (the two corners that meet at the
  cut, contracted over it) with its truncated SVD M ~ U S V^T (LAPACK full
  SVD, keep k = min(chi, #{s_i > eps * s_1}), sign fixed as in cut_svd)
  and the projectors
  P = Q_b V S^-1/2 (into Q_a's columns) and Pt = S^-1/2 U^T Q_a (into Q_b's
  rows), so that Q_a P Pt Q_b is the best rank-k approximation of M;
* renormalised corner C_c' = Pt Q_c P, renormalised edge
  T_c' = Pt (T_c a) P, each divided by its Frobenius norm;
* convergence: the singular values of every corner, normalised to sum 1 and
  zero padded to chi; Delta = max over corners of the 2-norm of their change.

Leg conventions (all clockwise, ring order C1 T1 C2 T2 C3 T3 C4 T4):
  C_c[ccw, cw]          (C1 = upper-left, C2 = upper-right, ...)
  T_c[ccw, in, cw]      (T1 = top edge, T2 = right, T3 = bottom, T4 = left)
  a[l, u, r, d]         a_c = a with its legs cyclically shifted by c, so that
                        a_c[g, e, b, f] has g facing T_{c-1}, e facing T_c,
                        b on the clockwise cut and f on the counter-clockwise
                        cut of corner c.
With these conventions all four corners are the same contraction.

Parity status: pinned by tests/test_oracle_pins.py (product states in closed
form, brute-force contraction of 4x3 and 6x5 finite lattices, decoupled
chains against the exact 1D transfer matrix, invariances, fixed-point
residual).
"""
from __future__ import annotations

from dataclasses import dataclass
from typing import List

import torch

F64 = torch.float64

# position of corner c's site inside a 2x2 plaquette (UL, UR, LR, LL)
PLAQ_OFFSET = [(0, 0), (1, 0), (1, 1), (0, 1)]
# the renormalised corner built around site s becomes the corner of s + move
CORNER_MOVE = [(1, 1), (-1, 1), (-1, -1), (1, -1)]
# the renormalised edge T_c of site s becomes the edge of s + move
EDGE_MOVE = [(0, 1), (-1, 0), (0, -1), (1, 0)]
# trace-boundary start: site whose closed double layer is corner / edge c
INIT_CORNER_SITE = [(-1, -1), (1, -1), (1, 1), (-1, 1)]
INIT_EDGE_SITE = [(0, -1), (1, 0), (0, 1), (-1, 0)]


@dataclass(frozen=True)
class Lattice:
    Lx: int
    Ly: int

    @property
    def n(self) -> int:
        return self.Lx * self.Ly

    def idx(self, x: int, y: int) -> int:
        return (y % self.Ly) * self.Lx + (x % self.Lx)

    def xy(self, i: int):
        return i % self.Lx, i // self.Lx

    def shift(self, i: int, d) -> int:
        x, y = self.xy(i)
        return self.idx(x + d[0], y + d[1])


@dataclass
class Env:
    """C[c][site] (chi x chi) and T[c][site] (chi x D^2 x chi)."""
    C: List[List[torch.Tensor]]
    T: List[List[torch.Tensor]]

    def detach(self) -> "Env":
        return Env([[t.detach().clone() for t in row] for row in self.C],
                   [[t.detach().clone() for t in row] for row in self.T])


# --------------------------------------------------------------------------
def double_layer(A: torch.Tensor) -> torch.Tensor:
    """a[(l l'), (u u'), (r r'), (d d')] = sum_s A[s,l,u,r,d] A[s,l',u',r',d']."""
    D = A.shape[1]
    a = torch.einsum("slurd,sLURD->lLuUrRdD", A, A)
    return a.reshape(D * D, D * D, D * D, D * D)


def open_double_layer(A: torch.Tensor) -> torch.Tensor:
    """ao[s, s', (l l'), ...]: the double layer with the physical legs open
    (ket s, bra s')."""
    d, D = A.shape[0], A.shape[1]
    ao = torch.einsum("slurd,tLURD->stlLuUrRdD", A, A)
    return ao.reshape(d, d, D * D, D * D, D * D, D * D)


def rotate(a: torch.Tensor, c: int) -> torch.Tensor:
    """a_c: the last four legs of a cyclically shifted by c (clockwise)."""
    lead = list(range(a.dim() - 4))
    base = a.dim() - 4
    return a.permute(*lead, *[base + (c + i) % 4 for i in range(4)])


def _pad(t: torch.Tensor, shape) -> torch.Tensor:
    out = torch.zeros(shape, dtype=t.dtype)
    sl = tuple(slice(0, s) for s in t.shape)
    out[sl] = t
    return out


def _trace_vector(D: int) -> torch.Tensor:
    """vec(identity) on a fused (k, k') leg: closes a virtual bond of the
    ket with the same bond of the bra."""
    return torch.eye(D, dtype=F64).reshape(D * D)


def init_env(a_sites, lat: Lattice, chi: int) -> Env:
    """Trace-boundary environment, bond dimension D^2 zero padded to chi."""
    D2 = a_sites[0].shape[0]
    if chi < D2:
        raise ValueError("chi must be >= D^2")
    D = int(round(D2 ** 0.5))
    e = _trace_vector(D)
    C = [[None] * lat.n for _ in range(4)]
    T = [[None] * lat.n for _ in range(4)]
    for s in range(lat.n):
        for c in range(4):
            ac = rotate(a_sites[lat.shift(s, INIT_CORNER_SITE[c])], c)
            Cc = torch.einsum("g,e,gebf->fb", e, e, ac)
            C[c][s] = _pad(Cc, (chi, chi))
            ac = rotate(a_sites[lat.shift(s, INIT_EDGE_SITE[c])], c)
            Tc = torch.einsum("e,gebf->gfb", e, ac)
            T[c][s] = _pad(Tc, (chi, D2, chi))
    return Env(C, T)


# --------------------------------------------------------------------------
def enlarged_corner(C, Tprev, Tc, ac) -> torch.Tensor:
    """Q_c[(m f), (k b)] = sum T_{c-1}[m,g,i] C_c[i,j] T_c[j,e,k] a_c[g,e,b,f].

    Rows: the counter-clockwise cut (chi x D^2); columns: the clockwise cut.
    """
    chi, D2 = C.shape[0], Tc.shape[1]
    Q = torch.einsum("mgi,ij,jek,gebf->mfkb", Tprev, C, Tc, ac)
    return Q.reshape(chi * D2, chi * D2)


def cut_svd(M: torch.Tensor):
    """Full SVD by LAPACK with a deterministic sign: in every left singular
    vector u the entry r maximising |u_r| (1 + r/(2n)) is made positive (the
    right vector takes the same sign).  The weight breaks the exact ties
    between the (k,k') and (k',k) entries that the ket-bra exchange symmetry
    of the double layer creates.  Returns U, S, V (M = U diag(S) V^T)."""
    U, S, Vh = torch.linalg.svd(M)
    V = Vh.transpose(0, 1)
    n = U.shape[0]
    w = 1.0 + torch.arange(n, dtype=U.dtype) / (2.0 * n)
    piv = torch.argmax(U.abs() * w[:, None], dim=0)
    sgn = torch.sign(U[piv, torch.arange(U.shape[1])])
    sgn = torch.where(sgn == 0, torch.ones_like(sgn), sgn)
    return U * sgn, S, V * sgn


def kept_rank(S: torch.Tensor, chi: int, eps: float) -> int:
    """k = min(chi, #{s_i > eps * s_1})."""
    s1 = float(S[0])
    if not s1 > 0.0:
        raise ValueError("cut matrix is zero")
    return min(chi, int((S > eps * s1).sum()))


def cut_projectors(Qa, Qb, chi: int, eps: float, svd_fn=None):
    """Projectors of one cut from M = Qa Qb (Qa's columns meet Qb's rows).

    P = Qb V_k S_k^-1/2 (n x chi), Pt = S_k^-1/2 U_k^T Qa (chi x n), zero
    padded beyond k.  ``svd_fn`` maps (M, k_fn) to the kept (U, S, V); the
    gradient module passes its differentiable version.
    """
    M = Qa @ Qb
    if svd_fn is None:
        U, S, V = cut_svd(M)
        k = kept_rank(S, chi, eps)
        U, S, V = U[:, :k], S[:k], V[:, :k]
    else:
        U, S, V = svd_fn(M, lambda s: kept_rank(s, chi, eps))
    k = S.shape[0]
    rs = S.rsqrt()
    P = (Qb @ V) * rs
    Pt = rs[:, None] * (U.transpose(0, 1) @ Qa)
    n = Qa.shape[0]
    if k < chi:
        P = torch.cat([P, torch.zeros(n, chi - k, dtype=P.dtype)], dim=1)
        Pt = torch.cat([Pt, torch.zeros(chi - k, n, dtype=Pt.dtype)], dim=0)
    return P, Pt, S


def renormalised_edge(Pt, Tc, ac, P) -> torch.Tensor:
    """T_c'[x, f, y] = sum Pt[x,(j g)] T_c[j,e,k] a_c[g,e,b,f] P[(k b), y]."""
    chi, D2 = Tc.shape[0], Tc.shape[1]
    return torch.einsum("xjg,jek,gebf,kby->xfy",
                        Pt.reshape(chi, chi, D2), Tc, ac,
                        P.reshape(chi, D2, chi))


def ctm_step(a_sites, env: Env, lat: Lattice, chi: int, eps: float = 1e-12,
             svd_fn=None, return_spectra: bool = False):
    """One simultaneous four-corner CTMRG iteration on the whole unit cell."""
    n = lat.n
    Q = [[enlarged_corner(env.C[c][s], env.T[(c - 1) % 4][s], env.T[c][s],
                          rotate(a_sites[s], c)) for s in range(n)]
         for c in range(4)]
    P = [[None] * n for _ in range(4)]
    Pt = [[None] * n for _ in range(4)]
    spectra = [[None] * n for _ in range(4)]
    for p in range(n):                      # plaquette with upper-left site p
        for c in range(4):
            sa = lat.shift(p, PLAQ_OFFSET[c])
            sb = lat.shift(p, PLAQ_OFFSET[(c + 1) % 4])
            P[c][p], Pt[c][p], spectra[c][p] = cut_projectors(
                Q[c][sa], Q[(c + 1) % 4][sb], chi, eps, svd_fn)
    C = [[None] * n for _ in range(4)]
    T = [[None] * n for _ in range(4)]
    neg = lambda o: (-o[0], -o[1])          # noqa: E731
    for s in range(n):
        for c in range(4):
            p = lat.shift(s, neg(PLAQ_OFFSET[c]))          # s at corner c
            Cn = Pt[(c - 1) % 4][p] @ Q[c][s] @ P[c][p]
            C[c][lat.shift(s, CORNER_MOVE[c])] = Cn / torch.linalg.norm(Cn)
            p_ccw = lat.shift(s, neg(PLAQ_OFFSET[(c + 1) % 4]))
            Tn = renormalised_edge(Pt[c][p_ccw], env.T[c][s],
                                   rotate(a_sites[s], c), P[c][p])
            T[c][lat.shift(s, EDGE_MOVE[c])] = Tn / torch.linalg.norm(Tn)
    out = Env(C, T)
    if return_spectra:
        return out, spectra
    return out


def corner_spectra(env: Env) -> torch.Tensor:
    """[4, n_sites, chi]: singular values of every corner, sum-normalised."""
    rows = []
    for c in range(4):
        row = []
        for Cc in env.C[c]:
            s = torch.linalg.svdvals(Cc.detach())
            row.append(s / s.sum())
        rows.append(torch.stack(row))
    return torch.stack(rows)


def spectra_change(s_new: torch.Tensor, s_old: torch.Tensor) -> float:
    return float(torch.linalg.norm(s_new - s_old, dim=-1).max())


def as_sites(A) -> list:
    """A[Ly, Lx, d, D, D, D, D] (numpy or torch) -> list of site tensors."""
    A = torch.as_tensor(A, dtype=F64)
    Ly, Lx = A.shape[0], A.shape[1]
    return [A[y, x] for y in range(Ly) for x in range(Lx)]


def converge(A, chi: int, tol: float, max_iter: int, eps: float = 1e-12,
             env: Env = None):
    """Run CTMRG from the trace boundary (or ``env``) until Delta < tol or
    ``max_iter`` iterations.  Returns (env, n_iter, Delta)."""
    A = torch.as_tensor(A, dtype=F64)
    lat = Lattice(A.shape[1], A.shape[0])
    a_sites = [double_layer(t) for t in as_sites(A)]
    if env is None:
        env = init_env(a_sites, lat, chi)
    s_old = corner_spectra(env)
    delta = float("inf")
    it = 0
    with torch.no_grad():
        while it < max_iter:
            env = ctm_step(a_sites, env, lat, chi, eps)
            it += 1
            s_new = corner_spectra(env)
            delta = spectra_change(s_new, s_old)
            s_old = s_new
            if delta < tol:
                break
    return env, it, delta
