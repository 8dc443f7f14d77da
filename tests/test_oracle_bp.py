"""Pins of the oracle's belief-propagation (chi = 1) preconditioner.

  * decoupled horizontal chains A[s,l,u,r,d] = B[s,l,r] delta_u0 delta_d0
    form a tree, on which belief propagation is exact: the messages along
    the chain are the dominant left and right eigenvectors of the chain
    transfer matrix t = sum_s B_s (x) B_s (computed by numpy's general
    eigensolver), the vertical ones the projector on index 0;
  * an embedded product state (only virtual index 0 nonzero): every message
    is the projector on index 0, N = I_d (x) P_0 / |phi|^2, and the
    preconditioned direction is g / (1/|phi|^2 + delta) on the index-0
    block and g / delta elsewhere (the closed form of the product-state
    preconditioner, Eq. (11) with environment bond dimension 1).
"""
import numpy as np
import pytest
import torch

from oracle import bp
from paper_2511_09546_amd import inputs


def _dominant(M):
    w, v = np.linalg.eig(M)
    k = np.argmax(np.abs(w))
    u = np.real(v[:, k])
    u = u / np.linalg.norm(u)
    D = int(round(np.sqrt(u.size)))
    return u if np.trace(u.reshape(D, D)) > 0 else -u


@pytest.mark.parametrize("D", [2, 3])
def test_chain_messages_are_transfer_eigenvectors(D):
    rng = np.random.default_rng(40 + D)
    B = rng.standard_normal((2, D, D))
    # positive-definite-ish chain: add a dominant identity part for a gap
    B[0] += 1.5 * np.eye(D)
    A = np.zeros((1, 1, 2, D, D, D, D))
    A[0, 0, :, :, 0, :, 0] = B
    msgs, it, change = bp.bp_messages(A, tol=1e-13, max_iter=2000)
    assert change < 1e-13
    t = np.einsum("sab,scd->acbd", B, B).reshape(D * D, D * D)
    left = _dominant(t.T)     # m_L' = t^T m_L
    right = _dominant(t)      # m_R' = t m_R
    m = msgs[0]
    assert np.allclose(m["l"].numpy(), left, atol=1e-10)
    assert np.allclose(m["r"].numpy(), right, atol=1e-10)
    e0 = np.zeros(D * D)
    e0[0] = 1.0
    assert np.allclose(m["u"].numpy(), e0, atol=1e-14)
    assert np.allclose(m["d"].numpy(), e0, atol=1e-14)


@pytest.mark.parametrize("D,delta", [(2, 1e-3), (3, 0.2)])
def test_product_state_closed_form(D, delta):
    phi = np.array([0.6, -1.3])
    A = inputs.product_state(phi, D)
    g = np.random.default_rng(7).standard_normal(A.shape)
    x, it, change = bp.precondition_bp(A, g, delta)
    want = g / delta
    want[0, 0, :, 0, 0, 0, 0] = g[0, 0, :, 0, 0, 0, 0] / (
        1.0 / (phi @ phi) + delta)
    assert np.allclose(x.numpy(), want, rtol=1e-12, atol=1e-12)


def test_two_by_two_cell_of_identical_tensors():
    """A 2x2 cell of four copies of one tensor has the messages of the 1x1
    cell on every site (the update is translation invariant)."""
    A1 = inputs.random_state(12, 1, 1, 2, 2)
    A4 = np.broadcast_to(A1, (2, 2) + A1.shape[2:]).copy()
    m1, _, _ = bp.bp_messages(A1, tol=1e-12)
    m4, _, _ = bp.bp_messages(A4, tol=1e-12)
    for s in range(4):
        for leg in bp.LEGS:
            assert torch.allclose(m4[s][leg], m1[0][leg], atol=1e-11)
