"""Pins of the CPU oracle against what the paper and the mathematics fix.

Each test checks the oracle against something other than itself:
  * closed forms of product states (any chi);
  * exact contraction of small finite lattices by an independent row-by-row
    transfer (the untruncated CTMRG from the trace boundary equals a finite
    open lattice);
  * decoupled chains against the exact 1D transfer-matrix fixed point;
  * exact invariances (scale, orthogonal virtual gauge, physical rotation,
    lattice rotation) and fixed-point self-consistency.
"""
import numpy as np
import pytest
import torch

from oracle import ctmrg, observables
from paper_2511_09546_amd import inputs

F64 = torch.float64


def _energy(A, terms, chi, n_iter=None, tol=1e-13, max_iter=400):
    if n_iter is not None:
        A_t = torch.as_tensor(A)
        lat = ctmrg.Lattice(A_t.shape[1], A_t.shape[0])
        a = [ctmrg.double_layer(t) for t in ctmrg.as_sites(A_t)]
        env = ctmrg.init_env(a, lat, chi)
        for _ in range(n_iter):
            env = ctmrg.ctm_step(a, env, lat, chi)
    else:
        env, _, _ = ctmrg.converge(A, chi, tol, max_iter)
    return float(observables.energy(env, A, terms)), env


# ---------------------------------------------------------------- inputs
def test_hamiltonian_spectra():
    ss = np.linalg.eigvalsh(inputs.heisenberg_ss())
    rot = inputs.heisenberg_rotated()
    assert np.allclose(rot, rot.T)
    assert np.allclose(np.sort(np.linalg.eigvalsh(rot)), np.sort(ss))
    assert np.allclose(np.sort(ss), [-0.75, 0.25, 0.25, 0.25])
    # rotated bond written out: (-sx sx + sy sy - sz sz)/4
    want = 0.25 * np.array([[-1, 0, 0, -2], [0, 1, 0, 0],
                            [0, 0, 1, 0], [-2, 0, 0, -1]])
    assert np.allclose(rot, want)
    for g in "xyz":
        assert np.allclose(np.sort(np.linalg.eigvalsh(inputs.kitaev_bond(g))),
                           [-0.25, -0.25, 0.25, 0.25])


def test_rotation_symmetry_of_bonds():
    for th in (0.3, 1.1):
        R = np.array([[np.cos(th), -np.sin(th)], [np.sin(th), np.cos(th)]])
        RR = np.kron(R, R)
        for h in (inputs.heisenberg_ss(), inputs.heisenberg_rotated()):
            assert np.allclose(RR.T @ h @ RR, h)


def test_kitaev_brickwall_bond_count():
    """Every spin of the brick-wall mapping has one x, one y and one z bond."""
    terms = inputs.terms_kitaev_brickwall(2, 2)
    count = {}
    for kind, site, dx, dy, coef, mat in terms:
        x, y = site % 2, site // 2
        if kind == 0:
            for sp in "ab":
                count.setdefault((x, y, sp), []).append("z")
        elif (dx, dy) == (1, 0):
            count.setdefault((x, y, "b"), []).append("x")
            count.setdefault(((x + 1) % 2, y, "a"), []).append("x")
        else:
            count.setdefault((x, y, "b"), []).append("y")
            count.setdefault((x, (y + 1) % 2, "a"), []).append("y")
    assert len(count) == 8
    for v in count.values():
        assert sorted(v) == ["x", "y", "z"]


# ---------------------------------------------------------------- P1 / P2
def _product_energy(phi, terms, n_sites=1):
    """Closed form: sum_terms coef (phi phi)^T h (phi phi) / |phi|^4 / n."""
    phi = np.asarray(phi, float)
    q = np.kron(phi, phi)
    tot = 0.0
    for kind, site, dx, dy, coef, mat in terms:
        if kind == 0:
            tot += coef * phi @ mat @ phi / (phi @ phi)
        else:
            tot += coef * q @ mat @ q / (phi @ phi) ** 2
    return tot / n_sites


@pytest.mark.parametrize("chi", [1, 3])
def test_product_state_closed_form(chi):
    rng = np.random.default_rng(11)
    phi = rng.standard_normal(2)
    for J2, want in ((0.0, -0.5), (0.5, -0.25)):
        terms = inputs.terms_j1j2(1, 1, 1.0, J2)
        e, _ = _energy(inputs.product_state(phi), terms, chi, n_iter=3)
        assert abs(e - want) < 1e-13
    h = rng.standard_normal((4, 4))
    h = h + h.T
    terms = [(1, 0, 1, 0, 0.7, h), (1, 0, 0, 1, -0.4, h.T @ h),
             (1, 0, 1, 1, 0.3, h), (1, 0, 1, -1, 0.2, np.eye(4) + h)]
    e, _ = _energy(inputs.product_state(phi), terms, chi, n_iter=3)
    assert abs(e - _product_energy(phi, terms)) < 1e-13


@pytest.mark.parametrize("D,chi", [(2, 4), (3, 9), (3, 12)])
def test_embedded_product_state(D, chi):
    rng = np.random.default_rng(12)
    phi = rng.standard_normal(2)
    h = rng.standard_normal((4, 4))
    terms = [(1, 0, 1, 0, 1.0, h), (1, 0, 0, 1, 0.5, h @ h.T),
             (1, 0, 1, 1, 0.25, h.T)]
    e, _ = _energy(inputs.product_state(phi, D), terms, chi, n_iter=4)
    assert abs(e - _product_energy(phi, terms)) < 1e-13


# ---------------------------------------------------------------- P4
def _bruteforce_rdm(A, W, H, open_sites):
    """Exact contraction of a finite W x H open lattice of double layers
    whose outer virtual legs are closed with delta_{k k'}; the sites in
    ``open_sites`` ((col,row), listed in row-major order) keep their
    physical legs.  Written independently of the oracle: its own double
    layer and a row-by-row transfer with tensordot.  Returns rho normalised
    to unit trace, [(s1 s2), (t1 t2)] for two open sites, [s, t] for one."""
    d, D = A.shape[0], A.shape[1]
    D2 = D * D
    a = np.einsum("slurd,tLURD->stlLuUrRdD", A, A).reshape(d, d, D2, D2, D2,
                                                          D2)
    closed = np.einsum("sslurd->lurd", a)
    e = np.eye(D).reshape(D2)
    vec = np.ones(())
    for _ in range(W):
        vec = np.multiply.outer(vec, e)          # axes: in_0..in_{W-1}
    n_extra = 0
    for row in range(H):
        T = np.multiply.outer(e, vec)           # h, in_0.., extras
        for col in range(W):
            is_open = (col, row) in open_sites
            site = a if is_open else closed
            # T axes: [h, out_0..out_{col-1}, in_col..in_{W-1}, extras]
            l_ax, u_ax = (2, 3) if is_open else (0, 1)
            R = np.tensordot(T, site, axes=([0, 1 + col], [l_ax, u_ax]))
            # R axes: [out_0..out_{col-1}, in_{col+1}.., extras, (s,t), r, d]
            nd = R.ndim
            R = np.moveaxis(R, nd - 2, 0)       # r -> new h
            R = np.moveaxis(R, nd - 1, 1 + col)  # d -> out_col
            if is_open:
                first = 1 + W + n_extra          # s, t follow the old extras
                R = np.moveaxis(R, [first, first + 1], [nd - 2, nd - 1])
                n_extra += 2
            T = R
        vec = np.tensordot(e, T, axes=([0], [0]))
    for _ in range(W):
        vec = np.tensordot(e, vec, axes=([0], [0]))
    if len(open_sites) == 1:
        rho = vec.reshape(d, d)
    else:
        rho = vec.reshape(d, d, d, d).transpose(0, 2, 1, 3).reshape(d * d,
                                                                     d * d)
    return rho / np.trace(rho)


def _oracle_rdms(A, chi, n_iter):
    A_t = torch.as_tensor(A[None, None])
    lat = ctmrg.Lattice(1, 1)
    sites = ctmrg.as_sites(A_t)
    a = [ctmrg.double_layer(t) for t in sites]
    env = ctmrg.init_env(a, lat, chi)
    for _ in range(n_iter):
        env = ctmrg.ctm_step(a, env, lat, chi)
    n = lambda r: (r / torch.trace(r)).numpy()     # noqa: E731
    return (n(observables.rdm_h(env, lat, sites, 0, 0)),
            n(observables.rdm_v(env, lat, sites, 0, 0)),
            n(observables.rdm_diag(env, lat, sites, 0, 0)),
            n(observables.rdm_anti(env, lat, sites, 0, 0)),
            n(observables.rdm_site(env, lat, sites, 0, 0)), env)


def test_bruteforce_zero_iterations():
    A = np.random.default_rng(21).standard_normal((2, 2, 2, 2, 2))
    rh, rv, rd, ra, r1, _ = _oracle_rdms(A, 4, 0)
    assert np.abs(rh - _bruteforce_rdm(A, 4, 3, [(1, 1), (2, 1)])).max() < 1e-13
    assert np.abs(rv - _bruteforce_rdm(A, 3, 4, [(1, 1), (1, 2)])).max() < 1e-13
    assert np.abs(rd - _bruteforce_rdm(A, 4, 4, [(1, 1), (2, 2)])).max() < 1e-13
    # anti-diagonal: site 1 = lower-left (1,2), site 2 = upper-right (2,1);
    # the brute force orders open sites row-major, i.e. (2,1) first
    bf = _bruteforce_rdm(A, 4, 4, [(2, 1), (1, 2)])
    bf = bf.reshape(2, 2, 2, 2).transpose(1, 0, 3, 2).reshape(4, 4)
    assert np.abs(ra - bf).max() < 1e-13
    assert np.abs(r1 - _bruteforce_rdm(A, 3, 3, [(1, 1)])).max() < 1e-13


def test_bruteforce_one_iteration_untruncated():
    """chi = 16 = D^4 with D = 2: the first iteration truncates nothing, so
    the 2x1 network is the exact 6x5 finite lattice (and 5x6 vertically)."""
    A = np.random.default_rng(22).standard_normal((2, 2, 2, 2, 2))
    rh, rv, rd, ra, r1, env = _oracle_rdms(A, 16, 1)
    # the cut matrices must have full effective rank 16 for P Pt = 1
    A_t = torch.as_tensor(A[None, None])
    lat = ctmrg.Lattice(1, 1)
    a = [ctmrg.double_layer(t) for t in ctmrg.as_sites(A_t)]
    env0 = ctmrg.init_env(a, lat, 16)
    _, spectra = ctmrg.ctm_step(a, env0, lat, 16, return_spectra=True)
    for c in range(4):
        S = spectra[c][0]
        assert S.shape[0] == 16 and float(S[-1] / S[0]) > 1e-10
    assert np.abs(rh - _bruteforce_rdm(A, 6, 5, [(2, 2), (3, 2)])).max() < 1e-12
    assert np.abs(rv - _bruteforce_rdm(A, 5, 6, [(2, 2), (2, 3)])).max() < 1e-12


# ---------------------------------------------------------------- P3
def _chain_reference(B):
    """Exact 1D transfer-matrix RDMs of the chain B[s, l, r]."""
    d, D = B.shape[0], B.shape[1]
    E = np.einsum("slr,sLR->lLrR", B, B).reshape(D * D, D * D)
    w, vl = np.linalg.eig(E.T)
    L = np.real(vl[:, np.argmax(np.abs(w))])
    w, vr = np.linalg.eig(E)
    R = np.real(vr[:, np.argmax(np.abs(w))])
    Bs = np.einsum("slr,tLR->stlLrR", B, B).reshape(d, d, D * D, D * D)
    rho2 = np.einsum("a,stab,uvbc,c->sutv", L, Bs, Bs, R).reshape(d * d,
                                                                  d * d)
    rho1 = np.einsum("a,stab,b->st", L, Bs, R)
    return rho2 / np.trace(rho2), rho1 / np.trace(rho1)


@pytest.mark.parametrize("vertical", [False, True])
def test_decoupled_chains(vertical):
    D, d, chi = 2, 2, 4
    B = np.random.default_rng(31).standard_normal((d, D, D))
    A = np.zeros((d, D, D, D, D))
    if vertical:
        A[:, 0, :, 0, :] = B            # B[s, u, d]
    else:
        A[:, :, 0, :, 0] = B            # B[s, l, r]
    # the corners of decoupled chains are rank one, so their spectra never
    # change and cannot signal convergence: iterate a fixed number of times
    # (the edges converge like a power method, ratio ~0.79 here)
    lat = ctmrg.Lattice(1, 1)
    sites = ctmrg.as_sites(torch.as_tensor(A[None, None]))
    a = [ctmrg.double_layer(t) for t in sites]
    env = ctmrg.init_env(a, lat, chi)
    for _ in range(200):
        env = ctmrg.ctm_step(a, env, lat, chi)
    rh = observables.rdm_h(env, lat, sites, 0, 0)
    rv = observables.rdm_v(env, lat, sites, 0, 0)
    rh, rv = (rh / torch.trace(rh)).numpy(), (rv / torch.trace(rv)).numpy()
    along, r1 = _chain_reference(B)
    across = np.kron(r1, r1)
    if vertical:
        rh, rv = rv, rh
    assert np.abs(rh - along).max() < 1e-10
    assert np.abs(rv - across).max() < 1e-10


# ---------------------------------------------------------------- P5 / P6
@pytest.fixture(scope="module")
def random_d2():
    A = inputs.random_state(5, 1, 1, 2, 2)
    terms = inputs.terms_j1j2(1, 1, 1.0, 0.3)
    e, env = _energy(A, terms, 6)
    return A, terms, e, env


def test_scale_invariance(random_d2):
    A, terms, e, _ = random_d2
    e2, _ = _energy(3.7 * A, terms, 6)
    assert abs(e2 - e) < 1e-11


def test_orthogonal_gauge_invariance(random_d2):
    A, terms, e, _ = random_d2
    rng = np.random.default_rng(41)
    O1, _ = np.linalg.qr(rng.standard_normal((2, 2)))
    O2, _ = np.linalg.qr(rng.standard_normal((2, 2)))
    Ag = np.einsum("yxslurd,lL,uU,rR,dD->yxsLURD", A, O1, O2, O1, O2)
    e2, _ = _energy(Ag, terms, 6)
    assert abs(e2 - e) < 1e-11


def test_physical_rotation_invariance(random_d2):
    A, terms, e, _ = random_d2
    th = 0.77
    R = np.array([[np.cos(th), -np.sin(th)], [np.sin(th), np.cos(th)]])
    Ar = np.einsum("ts,yxslurd->yxtlurd", R, A)
    e2, _ = _energy(Ar, terms, 6)
    assert abs(e2 - e) < 1e-11


def test_lattice_rotation_and_mirror(random_d2):
    A, terms, e, _ = random_d2
    # rotate the picture by 90 degrees clockwise: new right = old up, ...
    Arot = np.einsum("yxslurd->yxsdlur", A)
    # mirror left <-> right
    Amir = A.transpose(0, 1, 2, 5, 4, 3, 6)
    for A2 in (Arot, Amir):
        e2, _ = _energy(A2, terms, 6)
        assert abs(e2 - e) < 1e-10


def test_fixed_point_self_consistency(random_d2):
    A, terms, e, env = random_d2
    A_t = torch.as_tensor(A)
    lat = ctmrg.Lattice(1, 1)
    sites = ctmrg.as_sites(A_t)
    a = [ctmrg.double_layer(t) for t in sites]
    env2 = ctmrg.ctm_step(a, env, lat, 6)
    assert ctmrg.spectra_change(ctmrg.corner_spectra(env2),
                                ctmrg.corner_spectra(env)) < 1e-12
    rh = observables.rdm_h(env, lat, sites, 0, 0)
    rv = observables.rdm_v(env, lat, sites, 0, 0)
    for r in (rh, rv):
        r = r / torch.trace(r)
        assert float((r - r.T).abs().max()) < 1e-10
        assert float(torch.linalg.eigvalsh(0.5 * (r + r.T)).min()) > -1e-8
    # one-site rho from either bond agrees up to the truncation error
    r1h = (rh / torch.trace(rh)).reshape(2, 2, 2, 2).diagonal(dim1=1,
                                                              dim2=3).sum(-1)
    r1v = (rv / torch.trace(rv)).reshape(2, 2, 2, 2).diagonal(dim1=1,
                                                              dim2=3).sum(-1)
    assert float((r1h - r1v).abs().max()) < 1e-3


def test_two_by_two_cell_reduces_to_one_by_one(random_d2):
    """The same tensor on all four sites of a 2x2 cell gives the 1x1 result
    (pins the multi-site bookkeeping of projectors and moves)."""
    A, terms, e, _ = random_d2
    A4 = np.tile(A, (2, 2, 1, 1, 1, 1, 1))
    terms4 = inputs.terms_j1j2(2, 2, 1.0, 0.3)
    e4, _ = _energy(A4, terms4, 6, n_iter=None)
    assert abs(e4 - e) < 1e-11
