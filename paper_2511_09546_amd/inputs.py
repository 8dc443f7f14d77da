"""Seeded synthetic inputs shared by the tests, the bench and the oracle checks.

This module holds only problem data: random site tensors, the Hamiltonian
term lists of the models the paper studies (and the J1-J2 and spin-1/2 Kitaev
variants used as workloads), and the workload definitions.  It contains none
of the method's arithmetic (no contraction, no environment, no solver), and it
imports nothing else from this package, so both the device path and the CPU
oracle can be fed from it.

Conventions
-----------
* Site tensor of one unit-cell site: real ``A[s, l, u, r, d]`` (physical leg,
  then the virtual legs left, up, right, down; "up" points to row y-1).
* Unit cell: ``A[y, x, s, l, u, r, d]`` with site index ``y*Lx + x``.
* A Hamiltonian term is ``(kind, site, dx, dy, coef, mat)``.  ``kind`` 0 is an
  on-site ``d x d`` matrix, ``kind`` 1 a two-site ``d^2 x d^2`` matrix, row
  major in ``[(s1 s2), (s1' s2')]`` where site 1 is ``site`` and site 2 is
  ``site + (dx, dy)`` (periodic in the unit cell).  Supported displacements are
  (1,0), (0,1), (1,1) and (1,-1).
"""
from __future__ import annotations

import numpy as np

# --------------------------------------------------------------------------
# spin-1/2 operators (Pauli matrices / 2); sigma^y (x) sigma^y is real, so all
# two-site terms below are real matrices.
_SX = np.array([[0.0, 1.0], [1.0, 0.0]])
_SZ = np.array([[1.0, 0.0], [0.0, -1.0]])
_ISY = np.array([[0.0, 1.0], [-1.0, 0.0]])      # i * sigma^y (real)
_I2 = np.eye(2)


def sigma_y_sigma_y() -> np.ndarray:
    """sigma^y (x) sigma^y = -(i sigma^y) (x) (i sigma^y), a real 4x4 matrix."""
    return -np.kron(_ISY, _ISY)


def heisenberg_ss() -> np.ndarray:
    """S_i . S_j for two spin-1/2 (Eq. (12)), basis |s1 s2>, s=0 is up."""
    return 0.25 * (np.kron(_SX, _SX) + sigma_y_sigma_y() + np.kron(_SZ, _SZ))


def heisenberg_rotated() -> np.ndarray:
    """S_i . S_j after a pi rotation about S^y of the second spin.

    The single-site ansatz of Sec. IV A flips the spin on every second site;
    the rotation exp(-i pi S^y) = i sigma^y is real, so the rotated bond
    matrix stays real: (-sx sx + sy sy - sz sz)/4.
    """
    u = np.kron(_I2, _ISY)
    return u.T @ heisenberg_ss() @ u


def kitaev_bond(gamma: str) -> np.ndarray:
    """S^gamma (x) S^gamma for two spin-1/2 (Eq. (13) with spin 1/2)."""
    if gamma == "x":
        return 0.25 * np.kron(_SX, _SX)
    if gamma == "y":
        return 0.25 * sigma_y_sigma_y()
    if gamma == "z":
        return 0.25 * np.kron(_SZ, _SZ)
    raise ValueError(gamma)


# --------------------------------------------------------------------------
# term lists
def terms_j1j2(Lx: int, Ly: int, J1: float = 1.0, J2: float = 0.0,
               rotated: bool = True):
    """Square-lattice J1-J2 Heisenberg model on an Lx x Ly unit cell.

    With ``rotated`` the nearest-neighbour bonds use the sublattice-rotated
    matrix (single-site ansatz of Sec. IV A); next-nearest neighbours sit on
    the same sublattice and keep S.S.
    """
    hnn = heisenberg_rotated() if rotated else heisenberg_ss()
    hnnn = heisenberg_ss()
    terms = []
    for y in range(Ly):
        for x in range(Lx):
            s = y * Lx + x
            terms.append((1, s, 1, 0, J1, hnn))
            terms.append((1, s, 0, 1, J1, hnn))
            if J2 != 0.0:
                terms.append((1, s, 1, 1, J2, hnnn))
                terms.append((1, s, 1, -1, J2, hnnn))
    return terms


def terms_kitaev_brickwall(Lx: int, Ly: int, Kx=1.0, Ky=1.0, Kz=1.0):
    """Spin-1/2 honeycomb Kitaev model, H = -sum K_g S^g S^g (Eq. (13) sign).

    Brick-wall mapping on the square lattice: every square site holds two
    spins (a, b) with local basis s = 2*s_a + s_b (d = 4).  The z bond is the
    on-site a-b pair, the x bond joins b(x,y) to a(x+1,y) and the y bond joins
    b(x,y) to a(x,y+1); every spin then has exactly one bond of each type.
    """
    ones = np.eye(2)
    onsite = -Kz * np.kron(_SZ, _SZ) * 0.25
    sxb = np.kron(ones, _SX) * 0.5      # S^x on spin b of site 1
    sxa = np.kron(_SX, ones) * 0.5      # S^x on spin a of site 2
    # S^y S^y is real as a two-spin product: (i sy)(x)(i sy) * (-1)
    iyb = np.kron(ones, _ISY) * 0.5
    iya = np.kron(_ISY, ones) * 0.5
    hx = -Kx * np.kron(sxb, sxa)
    hy = -Ky * (-np.kron(iyb, iya))
    terms = []
    for y in range(Ly):
        for x in range(Lx):
            s = y * Lx + x
            terms.append((0, s, 0, 0, 1.0, onsite))
            terms.append((1, s, 1, 0, 1.0, hx))
            terms.append((1, s, 0, 1, 1.0, hy))
    return terms


# --------------------------------------------------------------------------
# random site tensors
def random_state(seed: int, Lx: int, Ly: int, d: int, D: int) -> np.ndarray:
    """A[y,x,s,l,u,r,d] iid N(0,1) from numpy's default_rng(seed), C order,
    divided by max|A|."""
    rng = np.random.default_rng(seed)
    g = rng.standard_normal((Ly, Lx, d, D, D, D, D))
    return g / np.abs(g).max()


def afm_seeded_state(seed: int, D: int, weight: float = 0.1) -> np.ndarray:
    """1x1 state N(0,1) + weight * (product state phi at virtual index 0).

    In the sublattice-rotated frame the Neel state is uniform; phi = (1, 0)
    is taken (every real phi has the same product-state energy).  Divided
    by max|A| afterwards.
    """
    rng = np.random.default_rng(seed)
    g = rng.standard_normal((1, 1, 2, D, D, D, D))
    g[0, 0, 0, 0, 0, 0, 0] += weight
    return g / np.abs(g).max()


def product_state(phi, D: int = 1, Lx: int = 1, Ly: int = 1) -> np.ndarray:
    """Product state phi embedded at virtual index 0 of a bond-D tensor."""
    phi = np.asarray(phi, dtype=np.float64)
    A = np.zeros((Ly, Lx, phi.size, D, D, D, D))
    A[:, :, :, 0, 0, 0, 0] = phi
    return A


# --------------------------------------------------------------------------
# workloads (sizes and recipes; each one names its seed)
WORKLOADS = {
    # 1x1, d=2, D=2, chi=8, Heisenberg (rotated), 30 CTMRG iterations,
    # CG to relative residual 1e-10, delta 1e-4.
    "d2chi8": dict(Lx=1, Ly=1, d=2, D=2, chi=8, seed=1, J2=0.0,
                   n_iter=30, tol=0.0, cg_tol=1e-10, cg_maxiter=200,
                   delta=1e-4, grad_K=20),
    # 1x1, d=2, D=4, chi=32, AFM-seeded, converge to 1e-10, 20 CG iterations.
    "d4chi32": dict(Lx=1, Ly=1, d=2, D=4, chi=32, seed=2, J2=0.0,
                    n_iter=200, tol=1e-10, cg_tol=0.0, cg_maxiter=20,
                    delta=1e-4, grad_K=20, afm=True),
    # 1x1, d=2, D=6, chi=72, J1-J2 with J2 = 0.5.
    "d6chi72": dict(Lx=1, Ly=1, d=2, D=6, chi=72, seed=3, J2=0.5,
                    n_iter=200, tol=1e-10, cg_tol=0.0, cg_maxiter=20,
                    delta=1e-4, grad_K=20),
    # 2x2 cell, d=4 spin-1/2 Kitaev brick wall, D=5, chi=50.
    "kitaev2x2": dict(Lx=2, Ly=2, d=4, D=5, chi=50, seed=40, model="kitaev",
                      n_iter=200, tol=1e-10, cg_tol=0.0, cg_maxiter=20,
                      delta=1e-4, grad_K=20),
}


def workload_state(name: str) -> np.ndarray:
    w = WORKLOADS[name]
    if w.get("afm"):
        return afm_seeded_state(w["seed"], w["D"])
    if w.get("model") == "kitaev":
        # one seed per unit-cell tensor: seed, seed+1, ...
        Ls = []
        for i in range(w["Lx"] * w["Ly"]):
            Ls.append(random_state(w["seed"] + i, 1, 1, w["d"], w["D"])[0, 0])
        return np.stack(Ls).reshape(w["Ly"], w["Lx"], w["d"], *(w["D"],) * 4)
    return random_state(w["seed"], w["Lx"], w["Ly"], w["d"], w["D"])


def workload_terms(name: str):
    w = WORKLOADS[name]
    if w.get("model") == "kitaev":
        return terms_kitaev_brickwall(w["Lx"], w["Ly"])
    return terms_j1j2(w["Lx"], w["Ly"], 1.0, w.get("J2", 0.0))
