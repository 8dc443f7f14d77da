"""Pins of the C4v ansatz and QR-CTMRG oracle (Sec. IV A) against what the
mathematics fixes: the group projector, the general four-corner SVD CTMRG
on the same symmetric state (an independent contraction route), a product
state in closed form, and finite differences of the same function."""
import numpy as np
import pytest
import torch

from oracle import c4v, ctmrg, gradient, observables
from oracle.ctmrg import F64, double_layer
from paper_2511_09546_amd import inputs


def test_symmetrize_is_group_projector():
    A = torch.as_tensor(inputs.random_state(1, 1, 1, 2, 3)[0, 0])
    As = c4v.symmetrize(A)
    assert torch.allclose(c4v.symmetrize(As), As, atol=1e-15)
    rot = As.permute(0, 4, 1, 2, 3)
    mir = As.permute(0, 3, 2, 1, 4)
    assert torch.allclose(rot, As, atol=1e-15)
    assert torch.allclose(mir, As, atol=1e-15)
    # orthogonal projector: <B, P A> = <P B, A>
    B = torch.as_tensor(inputs.random_state(2, 1, 1, 2, 3)[0, 0])
    assert abs(float((B * As).sum() - (c4v.symmetrize(B) * A).sum())) < 1e-13
    # the double layer is invariant under the rotations and the diagonal
    # reflection, which makes the enlarged corner symmetric
    a = double_layer(As)
    assert torch.allclose(a, a.permute(1, 2, 3, 0), atol=1e-15)
    assert torch.allclose(a, a.permute(1, 0, 3, 2), atol=1e-15)


@pytest.mark.parametrize("D,chi,J2,seed", [(2, 16, 0.3, 11), (3, 18, 0.3, 11),
                                           (2, 32, 0.0, 4)])
def test_matches_general_ctmrg(D, chi, J2, seed):
    A = inputs.random_state(seed, 1, 1, 2, D)[0, 0]
    envc, it, dl = c4v.converge(A, chi, 1e-13, 500)
    assert dl < 1e-13
    terms = inputs.terms_j1j2(1, 1, 1.0, J2)
    e1 = c4v.energy(A, terms, envc, chi)
    As = c4v.symmetrize(A)[None, None].numpy()
    env, _, dlg = ctmrg.converge(As, chi, 1e-13, 500)
    assert dlg < 1e-13
    e2 = float(observables.energy(env, As, terms))
    assert abs(e1 - e2) < 1e-12 * abs(e2)
    s = c4v.spectrum(envc[0], chi)
    sg = ctmrg.corner_spectra(env)[0, 0]
    assert float((s - sg).abs().max()) < 1e-11


def test_product_state_energy():
    # virtual index 0 only: a product state of phi; every bond gives
    # tr(h rho (x) rho), rho = phi phi^T / |phi|^2
    phi = np.array([0.6, -0.8])
    A = np.zeros((2, 2, 2, 2, 2))
    A[:, 0, 0, 0, 0] = phi
    envc, it, dl = c4v.converge(A, 8, 1e-13, 50)
    terms = inputs.terms_j1j2(1, 1, 1.0, 0.4)
    rho = np.outer(phi, phi) / (phi @ phi)
    ex = sum(t[4] * np.trace(np.asarray(t[5]) @ np.kron(rho, rho))
             if t[0] == 1 else 0.0 for t in _terms_tuples(terms))
    e = c4v.energy(A, terms, envc, 8)
    assert abs(e - ex) < 1e-12


def _terms_tuples(terms):
    out = []
    for t in terms:
        if isinstance(t, dict):
            out.append((t["kind"], t["site"], t["dx"], t["dy"], t["coef"],
                        t["mat"]))
        else:
            out.append(tuple(t))
    return out


@pytest.fixture(scope="module")
def conv():
    A = inputs.random_state(11, 1, 1, 2, 2)[0, 0]
    envc, _, dl = c4v.converge(A, 16, 1e-13, 500)
    return A, envc


def test_grad_K_finite_differences(conv):
    A, envc = conv
    terms = inputs.terms_j1j2(1, 1, 1.0, 0.3)
    K = 5
    e, g = c4v.grad_K(A, terms, envc, 16, K)
    g = g.numpy()
    # the gradient lies in the symmetric subspace
    assert np.abs(c4v.symmetrize(g).numpy() - g).max() < 1e-14
    rng = np.random.default_rng(3)
    for _ in range(3):
        B = rng.standard_normal(A.shape)
        h = 1e-5
        fd = (c4v.energy_K(A + h * B, terms, envc, 16, K) -
              c4v.energy_K(A - h * B, terms, envc, 16, K)) / (2 * h)
        an = float(np.sum(g * B))
        assert abs(fd - an) < 1e-7 * max(abs(an), 1e-3)


def test_grad_matches_projected_general_gradient(conv):
    # the same physical derivative through the other contractor: the
    # four-corner SVD CTMRG gradient at A_s, projected on the symmetric
    # subspace (both K-step forms approximate the fixed-point derivative)
    A, envc = conv
    terms = inputs.terms_j1j2(1, 1, 1.0, 0.3)
    _, g = c4v.grad_K(A, terms, envc, 16, 20)
    As = c4v.symmetrize(A)[None, None].numpy()
    env, _, _ = ctmrg.converge(As, 16, 1e-13, 500)
    _, gg = gradient.grad_K(As, terms, env, 16, 20)
    gp = c4v.symmetrize(gg[0, 0]).numpy()
    err = np.linalg.norm(g.numpy() - gp) / np.linalg.norm(gp)
    assert err < 1e-6
