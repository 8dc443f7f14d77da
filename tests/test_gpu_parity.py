"""FP64 parity of the device path with the CPU oracle (1e-10 relative).

Small workloads run the oracle live on the same seeded inputs:
  * one CTMRG iteration from the oracle's own environment, element by
    element (same sign convention, so the tensors themselves agree);
  * energies and corner spectra after converging;
  * the preconditioned direction for a given g.
"""
import numpy as np
import pytest
import torch

from oracle import ctmrg, metric, observables
from paper_2511_09546_amd import binding, inputs

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)


def _oracle_env_arrays(env):
    C = np.stack([np.stack([t.numpy() for t in row]) for row in env.C])
    T = np.stack([np.stack([t.numpy() for t in row]) for row in env.T])
    return C, T


def _oracle_env(C, T):
    return ctmrg.Env([[torch.tensor(C[c, s]) for s in range(C.shape[1])]
                      for c in range(4)],
                     [[torch.tensor(T[c, s]) for s in range(T.shape[1])]
                      for c in range(4)])


@pytest.mark.parametrize("name,D,chi,iters", [("d2", 2, 8, 5),
                                              ("d3", 3, 12, 4)])
def test_one_step_elementwise(name, D, chi, iters):
    _say(f"one-step parity {name} D={D} chi={chi}")
    A = inputs.random_state(17, 1, 1, 2, D)
    lat = ctmrg.Lattice(1, 1)
    a = [ctmrg.double_layer(t) for t in ctmrg.as_sites(torch.tensor(A))]
    env = ctmrg.init_env(a, lat, chi)
    for _ in range(iters):
        env = ctmrg.ctm_step(a, env, lat, chi)
    env1 = ctmrg.ctm_step(a, env, lat, chi)
    C0, T0 = _oracle_env_arrays(env)
    C1, T1 = _oracle_env_arrays(env1)
    with binding.Context(A, chi) as ctx:
        ctx.set_env(C0, T0)
        ctx.converge(0.0, 1)
        Cg, Tg = ctx.get_env()
    assert np.abs(Cg - C1).max() < 1e-11
    assert np.abs(Tg - T1).max() < 1e-11


def test_energy_at_given_env():
    """Pure contraction parity: oracle environment in, energy out (all four
    bond directions of the J1-J2 model)."""
    _say("energy at oracle env")
    A = inputs.random_state(18, 1, 1, 2, 3)
    terms = inputs.terms_j1j2(1, 1, 1.0, 0.45)
    env, _, _ = ctmrg.converge(A, 10, 1e-9, 100)
    e_or = float(observables.energy(env, A, terms))
    C, T = _oracle_env_arrays(env)
    with binding.Context(A, 10) as ctx:
        ctx.set_env(C, T)
        e, _ = ctx.energy_grad(terms, grad=False)
    assert abs(e - e_or) < 1e-12 * abs(e_or)


@pytest.mark.parametrize("name", ["d2chi8", "d4chi32"])
def test_converged_energy_and_spectra(name):
    w = inputs.WORKLOADS[name]
    _say(f"converge parity {name}")
    A = inputs.workload_state(name)
    terms = inputs.workload_terms(name)
    tol = w["tol"] if w["tol"] > 0 else 0.0
    env, it_or, _ = ctmrg.converge(A, w["chi"], tol, w["n_iter"])
    e_or = float(observables.energy(env, A, terms))
    spec_or = ctmrg.corner_spectra(env).numpy()
    with binding.Context(A, w["chi"]) as ctx:
        it, dl, ok = ctx.converge(tol, w["n_iter"])
        e, _ = ctx.energy_grad(terms, grad=False)
        spec = ctx.spectra()
        g = np.random.default_rng(1).standard_normal(A.shape)
        x, cg_it, res, brk = ctx.precond(g, w["delta"], w["cg_tol"],
                                         w["cg_maxiter"])
    _say(f"  iters gpu {it} oracle {it_or}; e {e!r} vs {e_or!r}")
    assert it == it_or
    assert abs(e - e_or) < 1e-10 * abs(e_or)
    assert np.abs(spec - spec_or).max() < 1e-10
    x_or, it2, res2, _ = metric.precondition(env, A, g, w["delta"],
                                             w["cg_tol"], w["cg_maxiter"])
    x_or = x_or.numpy()
    ex = np.linalg.norm(x - x_or) / np.linalg.norm(x_or)
    ex_max = np.abs(x - x_or).max() / np.abs(x_or).max()
    _say(f"  x rel {ex:.2e}, max elementwise / max|x| {ex_max:.2e}")
    assert cg_it == it2
    assert ex < 1e-10 and ex_max < 1e-10


def test_errors_and_state():
    _say("status codes")
    A = inputs.random_state(1, 1, 1, 2, 2)
    terms = inputs.terms_j1j2(1, 1)
    with binding.Context(A, 4) as ctx:
        with pytest.raises(binding.IpepsError) as ei:
            ctx.energy_grad(terms, grad=False)
        assert ei.value.status == binding.ESTATE
        ctx.converge(1e-10, 50)
        with pytest.raises(binding.IpepsError) as ei:
            ctx.precond(np.zeros(A.shape), -1.0, 1e-8, 10)
        assert ei.value.status == binding.EINVAL
        bad = [(1, 0, 2, 0, 1.0, np.eye(4))]
        with pytest.raises(binding.IpepsError) as ei:
            ctx.energy_grad(bad, grad=False)
        assert ei.value.status == binding.EINVAL
