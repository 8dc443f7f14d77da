"""The torch.autograd interface: its forward and backward are the library's
energy and gradient (identical to the C-ABI host path on the same state),
the gradient agrees with central differences of the energy through the same
interface, and precondition() is precond_apply."""
import numpy as np
import pytest
import torch

from paper_2511_09546_amd import autograd, binding, inputs

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)


def test_energy_backward_is_library_gradient():
    _say("autograd energy/backward vs C-ABI, d4chi32")
    w = inputs.WORKLOADS["d4chi32"]
    A0 = inputs.workload_state("d4chi32")
    terms = inputs.workload_terms("d4chi32")
    with binding.Context(A0, w["chi"]) as ref:
        ref.converge(w["tol"], w["n_iter"])
        e_ref, g_ref = ref.energy_grad(terms, grad=True)
        x_ref, _, _, _ = ref.precond(g_ref, w["delta"], w["cg_tol"],
                                     w["cg_maxiter"])
    with binding.Context(A0, w["chi"]) as ctx:
        A = torch.tensor(A0, dtype=torch.float64, device="cuda:0",
                         requires_grad=True)
        e = autograd.energy(A, ctx, terms, w["tol"], w["n_iter"])
        e.backward()
        g = A.grad.detach()
        x = autograd.precondition(ctx, g, w["delta"], w["cg_tol"],
                                  w["cg_maxiter"])
    with binding.Context(A0, w["chi"]) as ctx:
        # no gradient asked for: the energy alone, from the same network
        with torch.no_grad():
            e_only = autograd.energy(A.detach(), ctx, terms, w["tol"],
                                     w["n_iter"])
    _say(f"  e {e.item()!r} vs {e_ref!r}, energy only {e_only.item()!r}")
    # the gradient path reports the energy after its K unrolled iterations
    # from the converged environment, the energy alone that of the
    # environment itself: equal to the convergence tolerance
    assert abs(e_only.item() - e_ref) <= 1e-10 * abs(e_ref)
    assert e.item() == e_ref
    assert np.array_equal(g.cpu().numpy(), g_ref)
    assert np.array_equal(x.cpu().numpy(), x_ref)


def test_autograd_gradient_vs_central_differences():
    """Fixed-point gradient mode at D=2, chi=6 on a state whose CTMRG
    converges to 1e-13 in about 50 iterations (the converged environment is
    then a function of A, so the derivative of the converged energy is the
    fixed-point gradient): central differences with h = 1e-5 along three
    seeded directions, through autograd.energy on both sides."""
    _say("autograd gradient vs central differences, D=2 chi=6")
    A0 = inputs.random_state(7, 1, 1, 2, 2)
    terms = inputs.terms_j1j2(1, 1, 1.0, 0.4)
    o = binding.default_opts()
    o.grad_mode = binding.GRAD_FP
    o.grad_K = 8
    rng = np.random.default_rng(4)
    with binding.Context(A0, 6, opts=o) as ctx:
        A = torch.tensor(A0, dtype=torch.float64, device="cuda:0",
                         requires_grad=True)
        e = autograd.energy(A, ctx, terms, 1e-13, 400)
        (g,) = torch.autograd.grad(e, A)
        g = g.cpu().numpy()
        h = 1e-5
        for k in range(3):
            v = rng.standard_normal(A0.shape)
            v /= np.linalg.norm(v)
            f = []
            for sgn in (1, -1):
                At = torch.tensor(A0 + sgn * h * v, dtype=torch.float64,
                                  device="cuda:0")
                f.append(autograd.energy(At, ctx, terms, 1e-13, 400).item())
            fd = (f[0] - f[1]) / (2 * h)
            ad = float(np.sum(g * v))
            _say(f"  direction {k}: autograd {ad:.10e} fd {fd:.10e}")
            assert abs(fd - ad) < 1e-6 * np.linalg.norm(g)


def test_wrong_tensor_is_rejected():
    A0 = inputs.random_state(3, 1, 1, 2, 2)
    with binding.Context(A0, 4) as ctx:
        with pytest.raises(TypeError):
            autograd.energy(torch.tensor(A0), ctx, [])
        with pytest.raises(ValueError):
            autograd.energy(torch.zeros((1, 1, 2, 2, 2, 2, 3),
                                        dtype=torch.float64, device="cuda:0"),
                            ctx, [])
