"""Reduced density matrices and the energy per site: the plain FP64 oracle.

TEST INFRASTRUCTURE ONLY (see the package header).

The energy functional E(A) = <psi|H|psi>/<psi|psi> (Eq. (6)) is evaluated
from the environment as in Eq. (7): for every Hamiltonian term the network of
environment tensors around the sites it acts on, with the physical legs of
those sites left open, gives a reduced density matrix rho; the term
contributes Tr(h rho)/Tr(rho).

* nearest neighbours (1,0) and (0,1): the 2x1 (1x2) block
      C1 T1 T1 C2 / T4 A A T2 / C4 T3 T3 C3
  built from the environments of the two sites;
* next-nearest neighbours (1,1) and (1,-1): the 2x2 plaquette of the four
  enlarged corners with the two diagonal sites open;
* on-site terms: the 3x3 block around one site.

rho is indexed rho[(s1 s2), (t1 t2)] with ket legs s and bra legs t; a term
matrix h[(s1 s2), (s1' s2')] contributes sum_{s,t} h[t, s] rho[s, t].
The energy per site is the sum over all terms divided by the number of
unit-cell sites.

Parity status: pinned by tests/test_oracle_pins.py (product-state closed
form, brute-force finite lattices, decoupled chains, invariances).
"""
from __future__ import annotations

import torch

from .ctmrg import (F64, Env, Lattice, double_layer, enlarged_corner,
                    open_double_layer, rotate, as_sites)


def _halves_h(env: Env, lat: Lattice, s1: int, s2: int, ao1, ao2):
    C, T = env.C, env.T
    HL = torch.einsum("ij,mgi,qm,jek,wzq,stgebz->kbwst",
                      C[0][s1], T[3][s1], C[3][s1], T[0][s1], T[2][s1], ao1)
    HR = torch.einsum("kej,ji,ibm,mq,qzw,stvebz->kvwst",
                      T[0][s2], C[1][s2], T[1][s2], C[2][s2], T[2][s2], ao2)
    return HL, HR


def rdm_h(env: Env, lat: Lattice, A_sites, x: int, y: int) -> torch.Tensor:
    """rho of the horizontal bond (x,y)-(x+1,y), [(s1 s2), (t1 t2)]."""
    s1, s2 = lat.idx(x, y), lat.idx(x + 1, y)
    ao1, ao2 = open_double_layer(A_sites[s1]), open_double_layer(A_sites[s2])
    HL, HR = _halves_h(env, lat, s1, s2, ao1, ao2)
    rho = torch.einsum("kbwst,kbwuv->sutv", HL, HR)
    d = rho.shape[0]
    return rho.reshape(d * d, d * d)


def rdm_v(env: Env, lat: Lattice, A_sites, x: int, y: int) -> torch.Tensor:
    """rho of the vertical bond (x,y)-(x,y+1), [(s1 s2), (t1 t2)]."""
    C, T = env.C, env.T
    s1, s2 = lat.idx(x, y), lat.idx(x, y + 1)
    ao1, ao2 = open_double_layer(A_sites[s1]), open_double_layer(A_sites[s2])
    HT = torch.einsum("ij,jek,kp,mgi,pbn,stgebz->mznst",
                      C[0][s1], T[0][s1], C[1][s1], T[3][s1], T[1][s1], ao1)
    HB = torch.einsum("qgm,wq,vyw,pv,nbp,stgzby->mznst",
                      T[3][s2], C[3][s2], T[2][s2], C[2][s2], T[1][s2], ao2)
    rho = torch.einsum("mznst,mznuv->sutv", HT, HB)
    d = rho.shape[0]
    return rho.reshape(d * d, d * d)


def _open_corner(env: Env, s: int, c: int, ao):
    """Enlarged corner with the physical legs of its site open:
    Q[(m f), (k b), s, t]."""
    C, T = env.C, env.T
    chi, D2 = C[c][s].shape[0], T[c][s].shape[1]
    d = ao.shape[0]
    Q = torch.einsum("mgi,ij,jek,stgebf->mfkbst",
                     T[(c - 1) % 4][s], C[c][s], T[c][s], rotate(ao, c))
    return Q.reshape(chi * D2, chi * D2, d, d)


def _plain_corner(env: Env, s: int, c: int, a):
    return enlarged_corner(env.C[c][s], env.T[(c - 1) % 4][s], env.T[c][s],
                           rotate(a, c))


def rdm_diag(env: Env, lat: Lattice, A_sites, x: int, y: int):
    """rho of the next-nearest pair (x,y)-(x+1,y+1) from the 2x2 plaquette
    with upper-left site (x,y)."""
    s00, s10 = lat.idx(x, y), lat.idx(x + 1, y)
    s11, s01 = lat.idx(x + 1, y + 1), lat.idx(x, y + 1)
    Q0 = _open_corner(env, s00, 0, open_double_layer(A_sites[s00]))
    Q1 = _plain_corner(env, s10, 1, double_layer(A_sites[s10]))
    Q2 = _open_corner(env, s11, 2, open_double_layer(A_sites[s11]))
    Q3 = _plain_corner(env, s01, 3, double_layer(A_sites[s01]))
    rho = torch.einsum("XYst,YZ,ZWuv,WX->sutv", Q0, Q1, Q2, Q3)
    d = rho.shape[0]
    return rho.reshape(d * d, d * d)


def rdm_anti(env: Env, lat: Lattice, A_sites, x: int, y: int):
    """rho of the next-nearest pair (x,y)-(x+1,y-1) from the 2x2 plaquette
    with upper-left site (x,y-1); site 1 is (x,y) (its lower-left corner)."""
    s00, s10 = lat.idx(x, y - 1), lat.idx(x + 1, y - 1)
    s11, s01 = lat.idx(x + 1, y), lat.idx(x, y)
    Q0 = _plain_corner(env, s00, 0, double_layer(A_sites[s00]))
    Q1 = _open_corner(env, s10, 1, open_double_layer(A_sites[s10]))
    Q2 = _plain_corner(env, s11, 2, double_layer(A_sites[s11]))
    Q3 = _open_corner(env, s01, 3, open_double_layer(A_sites[s01]))
    rho = torch.einsum("XY,YZuv,ZW,WXst->sutv", Q0, Q1, Q2, Q3)
    d = rho.shape[0]
    return rho.reshape(d * d, d * d)


def site_environment(env: Env, s: int) -> torch.Tensor:
    """E[l, u, r, d] (each a fused D^2 leg): the ring of the eight
    environment tensors of site s with the site itself removed."""
    C, T = env.C, env.T
    return torch.einsum("ij,jek,km,mbn,np,pzq,qw,wgi->gebz",
                        C[0][s], T[0][s], C[1][s], T[1][s], C[2][s],
                        T[2][s], C[3][s], T[3][s])


def rdm_site(env: Env, lat: Lattice, A_sites, x: int, y: int):
    """One-site rho[s, t] from the 3x3 block around (x,y)."""
    s = lat.idx(x, y)
    E = site_environment(env, s)
    return torch.einsum("gebz,stgebz->st", E, open_double_layer(A_sites[s]))


def term_value(rho: torch.Tensor, h) -> torch.Tensor:
    h = torch.as_tensor(h, dtype=F64)
    return torch.einsum("ts,st->", h, rho) / torch.trace(rho)


def energy(env: Env, A, terms, return_terms: bool = False):
    """Energy per unit-cell site: sum_terms coef * Tr(h rho)/Tr(rho) / n."""
    A = torch.as_tensor(A, dtype=F64)
    lat = Lattice(A.shape[1], A.shape[0])
    A_sites = as_sites(A)
    total = torch.zeros((), dtype=F64)
    parts = []
    for (kind, site, dx, dy, coef, mat) in terms:
        x, y = lat.xy(site)
        if kind == 0:
            rho = rdm_site(env, lat, A_sites, x, y)
        elif (dx, dy) == (1, 0):
            rho = rdm_h(env, lat, A_sites, x, y)
        elif (dx, dy) == (0, 1):
            rho = rdm_v(env, lat, A_sites, x, y)
        elif (dx, dy) == (1, 1):
            rho = rdm_diag(env, lat, A_sites, x, y)
        elif (dx, dy) == (1, -1):
            rho = rdm_anti(env, lat, A_sites, x, y)
        else:
            raise ValueError(f"unsupported displacement {(dx, dy)}")
        v = coef * term_value(rho, mat)
        parts.append(v)
        total = total + v
    e = total / lat.n
    if return_terms:
        return e, parts
    return e
