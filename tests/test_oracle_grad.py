"""Pins of the oracle gradient: finite differences of the same function,
exact invariances, and the SVD adjoint on its own."""
import numpy as np
import pytest
import torch

from oracle import ctmrg, gradient
from paper_2511_09546_amd import inputs

F64 = torch.float64


def test_svd_adjoint_against_finite_differences():
    """The full-spectrum truncated-SVD adjoint, through the projector pair
    P = Qb V S^-1/2, Pt = S^-1/2 U^T Qa, on a gauge-invariant loss."""
    rng = np.random.default_rng(1)
    n, k = 10, 4
    Qa0 = torch.tensor(rng.standard_normal((n, n)))
    Qb0 = torch.tensor(rng.standard_normal((n, n)))
    W = torch.tensor(rng.standard_normal((n, n)))
    X = torch.tensor(rng.standard_normal((n, n)))
    Y = torch.tensor(rng.standard_normal((n, n)))

    def loss(Qa, Qb):
        P, Pt, _ = ctmrg.cut_projectors(Qa, Qb, k, 1e-12,
                                        svd_fn=gradient.differentiable_svd)
        return (W * (P @ Pt)).sum() + torch.trace(Pt @ X @ P @ Pt @ Y @ P)

    Qa = Qa0.clone().requires_grad_(True)
    Qb = Qb0.clone().requires_grad_(True)
    ga, gb = torch.autograd.grad(loss(Qa, Qb), [Qa, Qb])
    h = 1e-6
    for trial in range(3):
        Va = torch.tensor(rng.standard_normal((n, n)))
        Vb = torch.tensor(rng.standard_normal((n, n)))
        with torch.no_grad():
            fd = (loss(Qa0 + h * Va, Qb0 + h * Vb)
                  - loss(Qa0 - h * Va, Qb0 - h * Vb)) / (2 * h)
        an = float((ga * Va).sum() + (gb * Vb).sum())
        assert abs(an - float(fd)) < 1e-7 * max(1.0, abs(an))


@pytest.fixture(scope="module")
def small_case():
    A = inputs.random_state(7, 1, 1, 2, 2)
    terms = inputs.terms_j1j2(1, 1, 1.0, 0.4)
    chi = 6
    env, it, delta = ctmrg.converge(A, chi, 1e-14, 500)
    return A, terms, chi, env


def _fd(f, A, v, h):
    return (f(A + h * v) - f(A - h * v)) / (2 * h)


def test_grad_full_finite_differences(small_case):
    A, terms, chi, _ = small_case
    N = 6
    e, g = gradient.grad_full(A, terms, chi, N)
    rng = np.random.default_rng(2)
    for _ in range(3):
        v = rng.standard_normal(A.shape)
        v /= np.linalg.norm(v)
        fd = _fd(lambda X: gradient.energy_full(X, terms, chi, N), A, v, 1e-5)
        an = float((g.numpy() * v).sum())
        assert abs(an - fd) < 1e-8 * max(abs(an), 1e-3)


def test_grad_K_finite_differences(small_case):
    A, terms, chi, env = small_case
    K = 5
    e, g = gradient.grad_K(A, terms, env, chi, K)
    rng = np.random.default_rng(3)
    for _ in range(3):
        v = rng.standard_normal(A.shape)
        v /= np.linalg.norm(v)
        fd = _fd(lambda X: gradient.energy_of(X, terms, env, chi, K), A, v,
                 1e-5)
        an = float((g.numpy() * v).sum())
        assert abs(an - fd) < 1e-8 * max(abs(an), 1e-3)


def test_grad_orthogonal_to_A_and_rotation(small_case):
    """Scale invariance gives <g, A> = 0; invariance of the J1-J2 bonds under
    a common real rotation R(theta) of every physical leg gives
    <g, (J x 1) A> = 0 with J the rotation generator."""
    A, terms, chi, env = small_case
    e, g = gradient.grad_K(A, terms, env, chi, 4)
    g = g.numpy()
    assert abs((g * A).sum()) < 1e-12 * np.linalg.norm(g) * np.linalg.norm(A)
    J = np.array([[0.0, -1.0], [1.0, 0.0]])
    JA = np.einsum("ts,yxslurd->yxtlurd", J, A)
    assert abs((g * JA).sum()) < 1e-10 * np.linalg.norm(g) * np.linalg.norm(A)


def test_grad_fp_converges_and_matches_fd(small_case):
    """The fixed-point gradient is the derivative of the converged energy;
    checked against central differences of fully reconverged energies."""
    A, terms, chi, env = small_case
    e, g, K = gradient.grad_fp(A, terms, env, chi, K0=10, rel=1e-12)
    assert K <= 320
    e20, g20 = gradient.grad_K(A, terms, env, chi, 2 * K)
    assert np.abs(g.numpy() - g20.numpy()).max() < 1e-9

    def e_conv(X):
        env2, _, _ = ctmrg.converge(X, chi, 1e-15, 2000, env=env)
        from oracle import observables
        return float(observables.energy(env2, X, terms))

    rng = np.random.default_rng(4)
    v = rng.standard_normal(A.shape)
    v /= np.linalg.norm(v)
    fd = _fd(e_conv, A, v, 1e-5)
    an = float((g.numpy() * v).sum())
    assert abs(an - fd) < 1e-6 * max(abs(an), 1e-3)


def test_product_state_gradient_closed_form():
    """D = 1: e(A) = f(phi) exactly, with
    f = sum_b c_b (phi phi)^T h_b (phi phi) / |phi|^4; its gradient is
    written out by hand here."""
    rng = np.random.default_rng(5)
    phi = rng.standard_normal(2)
    h = rng.standard_normal((4, 4))
    terms = [(1, 0, 1, 0, 1.0, h), (1, 0, 0, 1, 0.6, h.T @ h)]
    A = inputs.product_state(phi)
    lat_env, _, _ = ctmrg.converge(A, 1, 1e-14, 10)
    e, g = gradient.grad_K(A, terms, lat_env, 1, 3)
    H = sum(c * m for (_, _, _, _, c, m) in terms)
    Hs = (H + H.T).reshape(2, 2, 2, 2)
    q = np.kron(phi, phi)
    n2 = phi @ phi
    W = np.einsum("ijkl,k,l->ij", Hs, phi, phi)
    dnum = W @ phi + W.T @ phi
    want = dnum / n2 ** 2 - 4 * (q @ H @ q) * phi / n2 ** 3
    got = g.numpy()[0, 0, :, 0, 0, 0, 0]
    assert np.abs(got - want).max() < 1e-12
    assert abs(e - q @ H @ q / n2 ** 2) < 1e-13
