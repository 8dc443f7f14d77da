"""Pins of the spin-1/2 Kitaev brick-wall terms by their content (Eq. (13)).

The terms of the 2x2 Kitaev workload place two spins (a, b) on every square
site with local index s = 2 s_a + s_b.  These tests read the term matrices
themselves, not the bookkeeping that produced them:
  * every term is decomposed into Pauli strings on its spins (projection
    with the trace inner product, an independent generic routine): it must
    be exactly -K_g S^g S^g on one pair of spins, with K_x, K_y, K_z chosen
    distinct so that a swapped coupling or operator fails;
  * the bond graph read from those strings must be the honeycomb lattice:
    every spin has one x, one y and one z bond, the graph is bipartite
    (a spins only meet b spins), and on a 4x4 torus the plaquette operators
    W_p (the product, around each hexagon, of the Pauli operator of the bond
    leaving the hexagon at each site) are conserved: the Pauli string of
    W_p commutes with every term (two Pauli strings commute iff they differ
    on an even number of sites) - the defining property of the model;
  * on a 2x2 torus the Hamiltonian assembled from the terms equals, matrix
    element by matrix element, the one built directly from a honeycomb
    geometry (A and B sublattices, bond type from the bond direction) in
    the same spin order, and so do their spectra.
"""
import itertools

import numpy as np
import pytest

from paper_2511_09546_amd import inputs

PAULI = {
    "I": np.eye(2, dtype=complex),
    "x": np.array([[0, 1], [1, 0]], dtype=complex),
    "y": np.array([[0, -1j], [1j, 0]]),
    "z": np.array([[1, 0], [0, -1]], dtype=complex),
}
KX, KY, KZ = 1.3, 0.7, 0.4


def _pauli_decompose(h, n_spins):
    """{string: coefficient} with h = sum_P c_P P, c_P = Tr(P^dag h) / 2^n."""
    out = {}
    for labels in itertools.product("Ixyz", repeat=n_spins):
        P = np.array([[1.0 + 0j]])
        for l in labels:
            P = np.kron(P, PAULI[l])
        c = np.trace(P.conj().T @ h) / 2 ** n_spins
        if abs(c) > 1e-12:
            out["".join(labels)] = c
    return out


def _bonds(Lx, Ly):
    """Bonds read from the term matrices: (spin i, spin j, type, coef) with
    spin = (x, y, 'a' or 'b')."""
    terms = inputs.terms_kitaev_brickwall(Lx, Ly, KX, KY, KZ)
    bonds = []
    for kind, site, dx, dy, coef, mat in terms:
        x, y = site % Lx, site // Lx
        if kind == 0:
            spins = [(x, y, "a"), (x, y, "b")]
            dec = _pauli_decompose(np.asarray(mat) * coef, 2)
        else:
            x2, y2 = (x + dx) % Lx, (y + dy) % Ly
            spins = [(x, y, "a"), (x, y, "b"), (x2, y2, "a"), (x2, y2, "b")]
            dec = _pauli_decompose(np.asarray(mat) * coef, 4)
        assert len(dec) == 1, f"term is not a single Pauli string: {dec}"
        (string, c), = dec.items()
        act = [(sp, l) for sp, l in zip(spins, string) if l != "I"]
        assert len(act) == 2 and act[0][1] == act[1][1]
        g = act[0][1]
        bonds.append((act[0][0], act[1][0], g, c))
    return bonds


def test_terms_are_single_kitaev_couplings():
    """-K_g S^g S^g = -(K_g / 4) sigma^g sigma^g, with the right K per type
    and the bond on the spins the mapping names."""
    K = {"x": KX, "y": KY, "z": KZ}
    for i, j, g, c in _bonds(2, 2):
        assert abs(c.imag) < 1e-15
        assert c.real == pytest.approx(-K[g] / 4, abs=1e-15)
        if g == "z":
            assert i[:2] == j[:2] and {i[2], j[2]} == {"a", "b"}
        else:
            # x and y bonds leave spin b of a site for spin a of its
            # right / lower neighbour
            assert i[2] == "b" and j[2] == "a"
            d = ((j[0] - i[0]) % 2, (j[1] - i[1]) % 2)
            assert d == ((1, 0) if g == "x" else (0, 1))


def test_bond_graph_is_honeycomb_with_conserved_plaquettes():
    # 4 x 4: cycles that wind around the torus are longer than six bonds
    Lx = Ly = 4
    bonds = _bonds(Lx, Ly)
    spins = sorted({s for b in bonds for s in b[:2]})
    assert len(spins) == 2 * Lx * Ly
    nb = {s: {} for s in spins}
    for i, j, g, _ in bonds:
        assert g not in nb[i] and g not in nb[j]
        nb[i][g] = j
        nb[j][g] = i
        assert i[2] != j[2]                       # bipartite: a -- b
    for s in spins:
        assert sorted(nb[s]) == ["x", "y", "z"]
    # hexagons: simple 6-cycles through alternating bond types
    hexes = set()
    for s0 in spins:
        stack = [(s0, [s0], None)]
        while stack:
            s, path, last = stack.pop()
            for g, t in nb[s].items():
                if g == last:
                    continue
                if t == s0 and len(path) == 6:
                    hexes.add(frozenset(path))
                elif t not in path and len(path) < 6:
                    stack.append((t, path + [t], g))
    # one hexagon per unit cell of the honeycomb
    assert len(hexes) == Lx * Ly
    index = {s: k for k, s in enumerate(spins)}

    def string(ops):
        out = ["I"] * len(spins)
        for s, l in ops.items():
            out[index[s]] = l
        return out

    def commute(p, q):
        diff = sum(1 for a, b in zip(p, q) if a != "I" and b != "I" and a != b)
        return diff % 2 == 0

    terms = [string({i: g, j: g}) for i, j, g, _ in bonds]
    for hx in hexes:
        ops = {}
        for s in hx:
            inside = [g for g, t in nb[s].items() if t in hx]
            assert len(inside) == 2
            (out,) = set("xyz") - set(inside)
            ops[s] = out
        W = string(ops)
        assert all(commute(W, t) for t in terms)
        # a string with one site changed no longer commutes with every term
        s0 = next(iter(hx))
        ops2 = dict(ops)
        ops2[s0] = "z" if ops[s0] != "z" else "x"
        assert not all(commute(string(ops2), t) for t in terms)


def _embed(ops, n):
    """Kronecker product of one-spin operators {position: matrix}."""
    M = np.array([[1.0 + 0j]])
    for k in range(n):
        M = np.kron(M, ops.get(k, PAULI["I"]))
    return M


def test_two_by_two_torus_matches_honeycomb_built_directly():
    Lx = Ly = 2
    n = 2 * Lx * Ly
    # spin order of the square-lattice sites: (a, b) of site 0, 1, ...

    def pos(x, y, sp):
        return 2 * ((y % Ly) * Lx + (x % Lx)) + (0 if sp == "a" else 1)

    H_terms = np.zeros((2 ** n, 2 ** n))
    for kind, site, dx, dy, coef, mat in inputs.terms_kitaev_brickwall(
            Lx, Ly, KX, KY, KZ):
        x, y = site % Lx, site // Lx
        mat = coef * np.asarray(mat)
        if kind == 0:
            sites = [site]
        else:
            sites = [site, ((y + dy) % Ly) * Lx + (x + dx) % Lx]
        # act on the 4- or 16-dimensional space of the named sites: permute
        # the full space so that those sites come first
        rest = [s for s in range(Lx * Ly) if s not in sites]
        order = sites + rest
        dim_rest = 4 ** len(rest)
        big = np.kron(mat, np.eye(dim_rest))
        axes = [2 * s + k for s in order for k in (0, 1)]
        inv = np.argsort(axes)
        big = big.reshape([2] * (2 * n))
        big = big.transpose(list(inv) + [n + i for i in inv])
        H_terms += big.reshape(2 ** n, 2 ** n)

    # honeycomb geometry: A at R = i a1 + j a2, B at R + d_z; the three
    # bond vectors from A to B are d_x, d_y, d_z at 120 degrees, the bond
    # type is the direction; a1 = d_z - d_x, a2 = d_z - d_y
    dz = np.array([0.0, 1.0])
    dx_ = np.array([np.sqrt(3) / 2, -0.5])
    dy_ = np.array([-np.sqrt(3) / 2, -0.5])
    a1, a2 = dz - dx_, dz - dy_
    L1, L2 = Lx * a1, Ly * a2
    cellinv = np.linalg.inv(np.stack([L1, L2], axis=1))

    def wrap(r):
        f = cellinv @ r
        f -= np.floor(f + 1e-9)
        return np.stack([L1, L2], axis=1) @ f

    A_pos = {(i, j): wrap(i * a1 + j * a2) for i in range(Lx)
             for j in range(Ly)}
    B_pos = {(i, j): wrap(i * a1 + j * a2 + dz) for i in range(Lx)
             for j in range(Ly)}
    K = {"x": KX, "y": KY, "z": KZ}
    H_geo = np.zeros((2 ** n, 2 ** n), dtype=complex)
    for (i, j), ra in A_pos.items():
        for g, dv in (("x", dx_), ("y", dy_), ("z", dz)):
            target = wrap(ra + dv)
            (bij,) = [k for k, rb in B_pos.items()
                      if np.allclose(rb, target, atol=1e-9)]
            H_geo += -K[g] / 4 * _embed(
                {pos(i, j, "a"): PAULI[g], pos(*bij, "b"): PAULI[g]}, n)
    assert np.abs(H_geo.imag).max() < 1e-14
    assert np.allclose(H_terms, H_geo.real, atol=1e-14)
    ev_t = np.linalg.eigvalsh(H_terms)
    ev_g = np.linalg.eigvalsh(H_geo.real)
    assert np.allclose(ev_t, ev_g, atol=1e-12)
