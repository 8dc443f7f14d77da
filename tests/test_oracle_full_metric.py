"""Pins of the full-metric oracle (Eq. (10), Sec. III A) and of its GMRES
solve (Sec. III C) against what the mathematics fixes: product states in
closed form, the symmetry and zero modes of the connected metric, the
stationarity of the per-site log-norm at the fixed point, and the
minimal-residual property of GMRES."""
import numpy as np
import pytest
import torch

from oracle import ctmrg, full_metric as fm, metric
from paper_2511_09546_amd import inputs

D, CHI, K = 2, 12, 6


@pytest.fixture(scope="module")
def state():
    A = inputs.random_state(3, 1, 1, 2, D)
    env, _, dl = ctmrg.converge(A, CHI, 1e-12, 300)
    assert dl < 1e-11
    return A[0, 0], env


def _projected(phi, b):
    p2 = phi @ phi
    return (b - phi * (phi @ b) / p2) / p2


def test_product_state_D1_closed_form():
    # D = 1: the state is the product of phi; per site the connected metric
    # is (I - phi phi^T / |phi|^2) / |phi|^2
    phi = np.array([0.8, -0.3, 0.5])
    A1 = phi.reshape(3, 1, 1, 1, 1)
    env, _, _ = ctmrg.converge(A1[None, None], 1, 1e-12, 10)
    B = np.random.default_rng(1).standard_normal(A1.shape)
    N = fm.metric_apply(A1, B, env, 1, 3).ravel()
    ex = _projected(phi, B.ravel())
    assert np.abs(N - ex).max() < 1e-9 * np.abs(ex).max()


def test_product_state_D2_zero_block():
    # the same product state carried on virtual index 0 of D = 2 bonds:
    # tangent directions with a nonzero virtual index give the zero state
    phi = np.array([0.8, -0.3, 0.5])
    A2 = np.zeros((3, 2, 2, 2, 2))
    A2[:, 0, 0, 0, 0] = phi
    env, _, _ = ctmrg.converge(A2[None, None], 4, 1e-12, 10)
    B = np.random.default_rng(2).standard_normal(A2.shape)
    N = fm.metric_apply(A2, B, env, 4, 3)
    ex = np.zeros_like(B)
    ex[:, 0, 0, 0, 0] = _projected(phi, B[:, 0, 0, 0, 0])
    assert np.abs(N - ex).max() < 1e-9 * np.abs(ex).max()


def test_symmetric_and_state_is_zero_mode(state):
    site, env = state
    rng = np.random.default_rng(0)
    B1, B2 = rng.standard_normal((2,) + site.shape)
    N1 = fm.metric_apply(site, B1, env, CHI, K)
    N2 = fm.metric_apply(site, B2, env, CHI, K)
    a, b = np.sum(B2 * N1), np.sum(B1 * N2)
    assert abs(a - b) < 1e-8 * abs(a)
    NA = fm.metric_apply(site, site, env, CHI, K)
    assert np.linalg.norm(NA) < 1e-8 * np.linalg.norm(N1) * \
        np.linalg.norm(site) / np.linalg.norm(B1)
    # positive semidefinite on random directions
    assert np.sum(B1 * N1) > 0 and np.sum(B2 * N2) > 0


def _gauge_dirs(site, rng):
    X, Y = rng.standard_normal((2, D, D))
    Bh = -np.einsum("lm,smurd->slurd", X, site) + \
        np.einsum("slumd,mr->slurd", site, X)
    Bv = -np.einsum("um,slmrd->slurd", Y, site) + \
        np.einsum("slurm,md->slurd", site, Y)
    return Bh, Bv


def test_gauge_directions_are_zero_modes_of_full_not_local(state):
    # infinitesimal gauge transformations of the bonds leave the state
    # unchanged: zero modes of the full metric; the local metric does not
    # have them
    site, env = state
    rng = np.random.default_rng(4)
    Br = rng.standard_normal(site.shape)
    r_rand = np.linalg.norm(fm.metric_apply(site, Br, env, CHI, K)) / \
        np.linalg.norm(Br)
    E, Z = metric.local_metric(env, 0, torch.as_tensor(site))
    for Bg in _gauge_dirs(site, rng):
        r = np.linalg.norm(fm.metric_apply(site, Bg, env, CHI, K)) / \
            np.linalg.norm(Bg)
        assert r < 1e-4 * r_rand
        loc = metric.metric_apply(E, Z, Bg).numpy()
        assert np.linalg.norm(loc) / np.linalg.norm(Bg) > 0.05 * r_rand


def test_log_norm_stationary_in_environment(state):
    # at the fixed point log kappa does not change to first order with the
    # environment, so its bra gradient through K iterations equals the
    # single-site one E A / Z; and F(A, c A) = F + log c gives <g, A> = 1
    site, env = state
    g = fm.grad_bra(site, site, env, CHI, K)
    E, Z = metric.local_metric(env, 0, torch.as_tensor(site))
    gl = metric.metric_apply(E, Z, site).numpy()
    assert np.linalg.norm(g - gl) < 1e-3 * np.linalg.norm(gl)
    assert abs(np.sum(g * site) - 1.0) < 1e-12


def test_stationarity_pin_catches_missing_normalisation(state, monkeypatch):
    # planted mistake: kappa without the 1/(n_h n_v) factor
    site, env = state
    orig = fm.log_kappa_env

    def wrong(env_, a):
        C, T = [env_.C[c][0] for c in range(4)], [env_.T[c][0]
                                                   for c in range(4)]
        n_h = torch.einsum("ij,jek,km,mn,neq,qi->", C[0], T[0], C[1], C[2],
                           T[2], C[3])
        n_v = torch.einsum("ij,jk,kel,lm,mn,nei->", C[0], C[1], T[1], C[2],
                           C[3], T[3])
        return orig(env_, a) + torch.log(torch.abs(n_h * n_v))

    monkeypatch.setattr(fm, "log_kappa_env", wrong)
    g = fm.grad_bra(site, site, env, CHI, K)
    E, Z = metric.local_metric(env, 0, torch.as_tensor(site))
    gl = metric.metric_apply(E, Z, site).numpy()
    assert np.linalg.norm(g - gl) > 1e-2 * np.linalg.norm(gl)


def test_difference_step_consistency(state):
    site, env = state
    B = np.random.default_rng(5).standard_normal(site.shape)
    a = fm.metric_apply(site, B, env, CHI, K, rel_step=1e-5)
    b = fm.metric_apply(site, B, env, CHI, K, rel_step=2e-5)
    c = fm.metric_apply(site, B, env, CHI, K, rel_step=1e-3)
    assert np.linalg.norm(a - b) < 1e-8 * np.linalg.norm(a)
    # O(h^2): at h = 1e-3 the difference is about 1e-6
    assert np.linalg.norm(a - c) < 1e-4 * np.linalg.norm(a)


# ------------------------------------------------------------------ GMRES
def _minres_over_krylov(M, b, k):
    # the GMRES iterate: argmin |b - M x| over span{b, M b, ..., M^(k-1) b},
    # from an orthonormal Krylov basis by QR and a least-squares solve
    Kb = np.empty((len(b), k))
    v = b.copy()
    for j in range(k):
        Kb[:, j] = v
        v = M @ v
    Q, _ = np.linalg.qr(Kb)
    y, *_ = np.linalg.lstsq(M @ Q, b, rcond=None)
    return Q @ y


@pytest.mark.parametrize("sym", [True, False])
def test_gmres_minimal_residual_and_exact(sym):
    rng = np.random.default_rng(7 + sym)
    n = 12
    M = rng.standard_normal((n, n))
    M = M @ M.T + n * np.eye(n) if sym else M + 3 * np.sqrt(n) * np.eye(n)
    b = rng.standard_normal(n)
    for k in (1, 3, 6):
        x, used, res = fm.gmres(lambda v: M @ v, b, m=k)
        assert used == k
        xr = _minres_over_krylov(M, b, k)
        assert np.linalg.norm(x - xr) < 1e-10 * np.linalg.norm(xr)
        true = np.linalg.norm(b - M @ x) / np.linalg.norm(b)
        assert abs(res - true) < 1e-12
    # with more vectors allowed than the dimension the cycle ends once the
    # Krylov space is invariant (one step later than n where single-pass
    # Gram-Schmidt has lost orthogonality at the 1e-8 level)
    x, used, res = fm.gmres(lambda v: M @ v, b, m=30)
    assert n <= used <= n + 1
    assert np.linalg.norm(x - np.linalg.solve(M, b)) < 1e-10 * \
        np.linalg.norm(x)
    # early stop at a relative tolerance
    x, used, res = fm.gmres(lambda v: M @ v, b, m=30, tol=1e-3)
    assert res <= 1e-3 and used < n


def test_local_gmres_matches_direct_solve(state):
    site, env = state
    A = site[None, None]
    g = np.random.default_rng(9).standard_normal(A.shape)
    x, used, res = fm.precondition_local_gmres(env, A, g, 1e-2, m=32)
    xd = metric.solve_direct(env, A, g, 1e-2)
    xd = xd.numpy() if hasattr(xd, "numpy") else np.asarray(xd)
    assert np.linalg.norm(x.numpy() - xd) < 1e-8 * np.linalg.norm(xd)


def test_full_gmres_product_state_inverse():
    # D = 1: (N + delta) has eigenvalues 1/|phi|^2 + delta (orthogonal to
    # phi) and delta (along phi); three Krylov vectors solve it exactly
    phi = np.array([0.8, -0.3, 0.5])
    A1 = phi.reshape(3, 1, 1, 1, 1)
    env, _, _ = ctmrg.converge(A1[None, None], 1, 1e-12, 10)
    g = np.random.default_rng(3).standard_normal(A1.shape)
    delta = 0.1
    x, used, res = fm.precondition_full(A1, g, env, 1, 3, delta)
    p2 = phi @ phi
    gv = g.ravel()
    par = phi * (phi @ gv) / p2
    ex = par / delta + (gv - par) / (1.0 / p2 + delta)
    assert np.abs(x.ravel() - ex).max() < 1e-8 * np.abs(ex).max()
    assert res < 1e-10
