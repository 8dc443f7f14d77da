"""Belief-propagation (chi = 1) environment and its metric preconditioner:
the plain FP64 oracle.

TEST INFRASTRUCTURE ONLY (see the package header).

Sec. III A (after Eq. (11)) reduces the local metric further by giving the
environment tensors around a site bond dimension 1, an environment that
belief propagation provides (a mean-field environment, App. A).  Written out
here for the double-layer network of the unit cell:

* every bond of the double-layer lattice carries two messages, one per
  direction; the message that arrives at leg L of site s is a D x D matrix
  m_s^L[k, k'] on that leg's ket/bra pair (fused k*D + k', as in the double
  layer);
* one update replaces every message by the contraction of the neighbour's
  double layer a with the three messages arriving at the neighbour's other
  legs, open on the leg that faces s (all messages from the previous
  update: a parallel schedule), then normalises it to unit Frobenius norm
  with a positive trace;
* the start is the trace message delta_{k k'} (the trace-boundary start of
  the CTMRG environment);
* converged when the largest change of a message is below tol;
* the environment of site s is the product of its four incoming messages,
  E[(l l'), (u u'), (r r'), (d d')] = m^L[l, l'] m^U[u, u'] m^R[r, r']
  m^D[d, d'], and the metric acts like the local metric (Eq. (11)):
  N x = (E x) / Z with Z = <A, E A>, physical index passed through;
* the preconditioned direction solves (N + delta I) x = g per site by a
  dense solve of the d D^4 x d D^4 system.

Neighbours: the left leg of s meets the right leg of s - (1, 0), the up leg
meets the down leg of s - (0, 1) ("up" points to row y - 1).

Parity status: pinned by tests/test_oracle_bp.py: on decoupled horizontal
chains (a tree, where belief propagation is exact) the chain messages are
the dominant eigenvectors of the chain transfer matrix, computed by a
library eigensolver; on embedded product states the direction has the
closed form of the product-state preconditioner.
"""
from __future__ import annotations

import numpy as np
import torch

from .ctmrg import F64, Lattice, as_sites, double_layer

# leg order of the double layer a[l, u, r, d]; the leg facing each
# direction's neighbour and the neighbour's displacement
LEGS = ("l", "u", "r", "d")
OPP = {"l": "r", "r": "l", "u": "d", "d": "u"}
NEIGH = {"l": (-1, 0), "r": (1, 0), "u": (0, -1), "d": (0, 1)}


def _contract_out(a, msgs_in, out_leg):
    """Contract a[l, u, r, d] with the incoming messages (D^2 vectors) on
    every leg but out_leg; returns a D^2 vector on out_leg."""
    t = a
    # contract legs in the order l, u, r, d, skipping out_leg
    remaining = list(LEGS)
    for leg in LEGS:
        if leg == out_leg:
            continue
        pos = remaining.index(leg)
        t = torch.tensordot(t, msgs_in[leg], dims=([pos], [0]))
        remaining.pop(pos)
    return t


def _normalise(v, D):
    m = v.reshape(D, D)
    tr = torch.trace(m)
    v = v / torch.linalg.norm(v)
    if tr < 0:
        v = -v
    return v


def bp_messages(A, tol: float = 1e-12, max_iter: int = 500):
    """Messages m[s][leg] (D^2 vectors) arriving at every leg of every
    site, the number of updates, and the last change."""
    A = torch.as_tensor(A, dtype=F64)
    lat = Lattice(A.shape[1], A.shape[0])
    D = A.shape[3]
    a = [double_layer(t) for t in as_sites(A)]
    trace = torch.eye(D, dtype=F64).reshape(-1)
    trace = trace / torch.linalg.norm(trace)
    msgs = [{leg: trace.clone() for leg in LEGS} for _ in range(lat.n)]
    it, change = 0, float("inf")
    while it < max_iter:
        new = [dict() for _ in range(lat.n)]
        change = 0.0
        for s in range(lat.n):
            for leg in LEGS:
                nb = lat.shift(s, NEIGH[leg])
                v = _contract_out(a[nb], msgs[nb], OPP[leg])
                v = _normalise(v, D)
                new[s][leg] = v
                change = max(change, float(torch.linalg.norm(
                    v - msgs[s][leg])))
        msgs = new
        it += 1
        if change < tol:
            break
    return msgs, it, change


def bp_environment(msgs_s, D: int) -> torch.Tensor:
    """E[(l u r d), (l' u' r' d')] of one site from its four messages."""
    M = [msgs_s[leg].reshape(D, D) for leg in LEGS]
    E = torch.einsum("ab,ce,fg,hi->acfhbegi", *M)
    return E.reshape(D ** 4, D ** 4)


def precondition_bp(A, g, delta: float, tol: float = 1e-12,
                    max_iter: int = 500):
    """x = (N_BP + delta I)^-1 g per site by a dense solve; returns
    (x, BP updates, last message change)."""
    A = torch.as_tensor(A, dtype=F64)
    g = torch.as_tensor(np.asarray(g), dtype=F64)
    msgs, it, change = bp_messages(A, tol, max_iter)
    Ly, Lx, d, D = A.shape[0], A.shape[1], A.shape[2], A.shape[3]
    x = torch.zeros_like(g)
    for y in range(Ly):
        for xx in range(Lx):
            s = y * Lx + xx
            E = bp_environment(msgs[s], D)
            As = A[y, xx].reshape(d, D ** 4)
            Z = float(torch.einsum("ti,ij,tj->", As, E, As))
            N = torch.kron(torch.eye(d, dtype=F64), E) / Z
            P = N + delta * torch.eye(d * D ** 4, dtype=F64)
            x[y, xx] = torch.linalg.solve(P, g[y, xx].reshape(-1)).reshape(
                g[y, xx].shape)
    return x, it, change
