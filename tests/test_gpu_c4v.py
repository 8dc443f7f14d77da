"""The device C4v ansatz and QR-CTMRG (Sec. IV A) against the CPU oracle:
the same iteration from the trace boundary (iteration count, energy,
corner spectrum), and the K-step gradient from the very same converged
(C, T, V) (the oracle's, uploaded), element by element."""
import numpy as np
import pytest
import torch

from oracle import c4v
from paper_2511_09546_amd import binding, inputs

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)


CASES = [(2, 16, 0.3, 11), (3, 18, 0.3, 11), (2, 32, 0.0, 4),
         (3, 160, 0.3, 11)]  # the last: block 200, beyond 128


@pytest.mark.parametrize("D,chi,J2,seed", CASES)
def test_converge_matches_oracle(D, chi, J2, seed):
    _say(f"c4v converge D={D} chi={chi}")
    A = inputs.random_state(seed, 1, 1, 2, D)
    terms = inputs.terms_j1j2(1, 1, 1.0, J2)
    envc, it_or, dl_or = c4v.converge(A[0, 0], chi, 1e-12, 300)
    e_or = c4v.energy(A[0, 0], terms, envc, chi)
    s_or = c4v.spectrum(envc[0], chi).numpy()
    with binding.Context(A, chi) as ctx:
        it, dl, ok = ctx.c4v_converge(1e-12, 300)
        e, _ = ctx.c4v_energy_grad(terms, grad=False)
        # the replicated four-corner environment serves the general entry
        # points: the energy of the K iterations' environment equals the
        # energy at the converged one to the convergence level
        e_gen, _ = ctx.energy_grad(terms, grad=False)
        s = ctx.spectra()[0, 0]
        As = binding.get_state(ctx)
    _say(f"  iters {it} vs {it_or}, e {e!r} vs {e_or!r} (general {e_gen!r})")
    assert ok
    # at chi = 160 the change of the spectrum approaches 1e-12 at the
    # rounding level of the b = 200 QR and eigen steps: the two sides can
    # stop a few iterations apart (energy and spectrum bounds unchanged)
    assert abs(it - it_or) <= (1 if chi <= 32 else 3)
    assert abs(e - e_or) < 1e-11 * abs(e_or)
    assert abs(e_gen - e_or) < 1e-11 * abs(e_or)
    assert np.abs(s - s_or).max() < 1e-10
    assert np.abs(As[0, 0] - c4v.symmetrize(A[0, 0]).numpy()).max() < 1e-15


@pytest.mark.parametrize("D,chi,J2,seed,K", [c + (K,) for c in CASES[:2]
                                               for K in (5, 20)] +
                         [CASES[3] + (3,)])
def test_grad_same_env(D, chi, J2, seed, K):
    _say(f"c4v grad D={D} chi={chi} K={K}")
    A = inputs.random_state(seed, 1, 1, 2, D)
    terms = inputs.terms_j1j2(1, 1, 1.0, J2)
    envc, _, _ = c4v.converge(A[0, 0], chi, 1e-13, 300)
    e_or, g_or = c4v.grad_K(A[0, 0], terms, envc, chi, K)
    g_or = g_or.numpy()
    C, T, V = (t.numpy() for t in envc)
    o = binding.default_opts()
    o.grad_K = K
    with binding.Context(A, chi, opts=o) as ctx:
        ctx.c4v_set_env(C, T, V)
        e, g = ctx.c4v_energy_grad(terms)
        dg = torch.zeros(A.shape, dtype=torch.float64, device="cuda:0")
        torch.cuda.synchronize()
        e2 = ctx.c4v_energy_grad_dev(terms, dg.data_ptr())
        g2 = dg.cpu().numpy()
        C2, T2, V2, bond = ctx.c4v_get_env()
    err = np.abs(g[0, 0] - g_or).max() / np.abs(g_or).max()
    _say(f"  e {e!r} vs {e_or!r}; max elementwise {err:.2e}")
    assert abs(e - e_or) < 1e-12 * abs(e_or)
    assert err < 1e-10
    assert e2 == e and np.array_equal(g2, g)
    # the gradient call leaves the converged environment as it was
    assert bond == chi
    assert np.array_equal(C2, C) and np.array_equal(T2, T)
    assert np.array_equal(V2, V)


def test_errors():
    A = inputs.random_state(1, 1, 1, 2, 2)
    terms = inputs.terms_j1j2(1, 1, 1.0, 0.0)
    with binding.Context(A, 8) as ctx:
        with pytest.raises(binding.IpepsError) as ei:
            ctx.c4v_energy_grad(terms)
        assert ei.value.status == binding.ESTATE
    A2 = inputs.random_state(2, 2, 1, 2, 2)
    with binding.Context(A2, 8) as ctx:
        with pytest.raises(binding.IpepsError) as ei:
            ctx.c4v_converge(1e-8, 10)
        assert ei.value.status == binding.ENOTIMPL
    assert binding.c4v_block_size(72) == 90
    assert binding.c4v_block_size(16) == 24
    assert binding.c4v_block_size(129) == 162
    assert binding.c4v_block_size(409) == 512
    assert binding.c4v_block_size(410) == -1
    for chi in (72, 129, 200, 409):
        assert binding.c4v_block_size(chi) == c4v.block_size(chi)
