"""Pins of the oracle's local metric and solver."""
import numpy as np
import pytest
import torch

from oracle import ctmrg, metric, observables
from paper_2511_09546_amd import inputs

F64 = torch.float64


@pytest.fixture(scope="module")
def case():
    A = inputs.random_state(9, 1, 1, 2, 2)
    chi = 8
    env, _, _ = ctmrg.converge(A, chi, 1e-13, 500)
    E, Z = metric.local_metric(env, 0, torch.as_tensor(A[0, 0]))
    return A, env, E, Z


def test_metric_symmetric_and_norm(case):
    A, env, E, Z = case
    assert float((E - E.T).abs().max() / E.abs().max()) < 1e-12
    # <y, N x> Z equals the 3x3 block with x in the ket and y in the bra,
    # contracted through the fused double-layer legs
    rng = np.random.default_rng(1)
    x = torch.tensor(rng.standard_normal(A[0, 0].shape))
    y = torch.tensor(rng.standard_normal(A[0, 0].shape))
    D = x.shape[1]
    axy = torch.einsum("slurd,sLURD->lLuUrRdD", x, y).reshape(D * D, D * D,
                                                             D * D, D * D)
    E4 = observables.site_environment(env, 0)
    want = float(torch.einsum("gebz,gebz->", E4, axy))
    got = float((y * metric.metric_apply(E, Z, x)).sum() * Z)
    assert abs(got - want) < 1e-12 * abs(want)
    # and Z is the norm network <A, E A>
    a = ctmrg.double_layer(torch.as_tensor(A[0, 0]))
    assert abs(float(Z) - float(torch.einsum("gebz,gebz->", E4, a))) \
        < 1e-12 * abs(float(Z))


def test_cg_matches_direct_solve(case):
    A, env, E, Z = case
    g = np.random.default_rng(2).standard_normal(A.shape)
    x_cg, it, res, brk = metric.precondition(env, A, g, 1e-2, 1e-13, 500)
    x_d = metric.solve_direct(env, A, g, 1e-2)
    assert not brk and res < 1e-13
    assert float((x_cg - x_d).norm() / x_d.norm()) < 1e-9


def test_cg_iterate_is_krylov_minimiser(case):
    """After m steps CG minimises the (N + delta)-energy norm of the error
    over the Krylov space K_m(N + delta, g); built here by Gram-Schmidt with
    full reorthogonalisation."""
    A, env, E, Z = case
    delta = 1e-2
    g = torch.tensor(np.random.default_rng(3).standard_normal(A[0, 0].shape))
    op = lambda v: metric.metric_apply(E, Z, v) + delta * v   # noqa: E731
    m = 6
    x_cg, it, _, _ = metric.cg(lambda v: metric.metric_apply(E, Z, v), g,
                               delta, 0.0, m)
    assert it == m
    basis = []
    v = g.clone()
    for _ in range(m):
        for _ in range(2):
            for b in basis:
                v = v - (b * v).sum() * b
        v = v / v.norm()
        basis.append(v)
        v = op(v)
    V = torch.stack([b.reshape(-1) for b in basis], 1)
    AV = torch.stack([op(b).reshape(-1) for b in basis], 1)
    y = torch.linalg.solve(V.T @ AV, V.T @ g.reshape(-1))
    x_k = (V @ y).reshape(g.shape)
    assert float((x_cg - x_k).norm() / x_k.norm()) < 1e-8


def test_large_delta_limit(case):
    A, env, E, Z = case
    g = np.random.default_rng(4).standard_normal(A.shape)
    delta = 1e9
    x, _, _, _ = metric.precondition(env, A, g, delta, 1e-14, 50)
    assert float((x * delta - torch.tensor(g)).norm() / np.linalg.norm(g)) \
        < 1e-8


def test_quadratic_model_one_step():
    """Eq. (5): with P equal to the Hessian of f = x^T A x / 2 - b^T x, the
    preconditioned gradient P^-1 (A x - b) is x - x*."""
    rng = np.random.default_rng(5)
    M = rng.standard_normal((12, 12))
    H = torch.tensor(M @ M.T + 12 * np.eye(12))
    b = torch.tensor(rng.standard_normal(12))
    x = torch.tensor(rng.standard_normal(12))
    x_star = torch.linalg.solve(H, b)
    gp, it, res, brk = metric.cg(lambda v: H @ v, H @ x - b, 0.0, 1e-14, 100)
    assert float((gp - (x - x_star)).norm()) < 1e-12 * float(x.norm())


def test_product_state_preconditioner_closed_form():
    """Embedded product state: only the all-zero virtual component of the
    ring survives, so N = 1_d (x) e0 e0^T / |phi|^2 and
    x = g / (1/|phi|^2 + delta) on that component, g / delta elsewhere."""
    rng = np.random.default_rng(6)
    phi = rng.standard_normal(2)
    A = inputs.product_state(phi, D=2)
    env, _, _ = ctmrg.converge(A, 4, 1e-14, 20)
    g = rng.standard_normal(A.shape)
    delta = 0.3
    x, _, res, _ = metric.precondition(env, A, g, delta, 1e-14, 200)
    want = g / delta
    want[..., 0, 0, 0, 0] = g[..., 0, 0, 0, 0] / (1.0 / (phi @ phi) + delta)
    assert np.abs(x.numpy() - want).max() < 1e-12
