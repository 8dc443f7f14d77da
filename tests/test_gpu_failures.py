"""Error paths of the C ABI, forced from the host (every kernel still runs to
its normal end): the warnings of a CTMRG, projector SVD or complement solve
that stops at its iteration limit, an injected CG breakdown, an allocation
failure under a device-memory budget with a clean context afterwards."""
import numpy as np
import pytest

from paper_2511_09546_amd import binding, inputs

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)


def _state():
    w = inputs.WORKLOADS["d2chi8"]
    return w, inputs.workload_state("d2chi8"), inputs.workload_terms("d2chi8")


def test_ctm_not_converged_at_max_iter():
    _say("failure: CTMRG max_iter=1")
    w, A, terms = _state()
    with binding.Context(A, w["chi"]) as ctx:
        it, dl, ok = ctx.converge(1e-14, 1)
        assert it == 1 and not ok
        assert ctx.last_status == binding.NOT_CONVERGED
        # the environment of the last iteration is kept and usable
        e, g = ctx.energy_grad(terms, grad=True)
        assert np.isfinite(e) and np.all(np.isfinite(g))


def test_projector_svd_iteration_limit_is_reported():
    """svd_max_iter = 1 with a cold (random) start block cannot reach the
    1e-15 residual: ctm_converge and ipeps_energy_grad return their outputs
    with the NOT_CONVERGED warning, and the counter says so."""
    _say("failure: projector SVD svd_max_iter=1")
    w, A, terms = _state()
    o = binding.default_opts()
    o.svd_max_iter = 1
    o.svd_tol = 1e-15
    o.grad_K = 2
    with binding.Context(A, w["chi"], opts=o) as ctx:
        it, dl, ok = ctx.converge(0.0, 3)        # fixed count: no tol miss
        assert it == 3
        assert ctx.last_status == binding.NOT_CONVERGED
        n0 = ctx.stats()["svd_unconverged"]
        assert n0 >= 1
        e, g = ctx.energy_grad(terms, grad=True)
        assert ctx.last_status == binding.NOT_CONVERGED
        assert ctx.stats()["svd_unconverged"] > n0
        assert np.isfinite(e) and np.all(np.isfinite(g))
    # the same run with the default limit reports nothing
    o.svd_max_iter = 50
    o.svd_tol = 1e-13
    with binding.Context(A, w["chi"], opts=o) as ctx:
        ctx.converge(0.0, 3)
        assert ctx.last_status == binding.OK
        ctx.energy_grad(terms, grad=True)
        assert ctx.last_status == binding.OK
        assert ctx.stats()["svd_unconverged"] == 0


def test_complement_solve_iteration_limit_is_reported():
    """A complement-solve tolerance below the FP64 rounding floor makes the
    solves of the SVD adjoint stop at their iteration limit: the gradient is
    still returned, with the warning."""
    _say("failure: complement CG below its floor")
    # D = 4, chi = 32: the complement of the kept vectors (dimension 480)
    # is much larger than the deflation space (16 vectors), so CG has to
    # iterate (at D = 2, chi = 8 the deflation space covers it all)
    w = inputs.WORKLOADS["d4chi32"]
    A = inputs.workload_state("d4chi32")
    terms = inputs.workload_terms("d4chi32")
    o = binding.default_opts()
    o.adj_cg_tol = 1e-17
    o.grad_K = 1
    with binding.Context(A, w["chi"], opts=o) as ctx:
        ctx.converge(0.0, 10)
        e, g = ctx.energy_grad(terms, grad=True)
        assert ctx.last_status == binding.NOT_CONVERGED
        assert ctx.stats()["cg_unconverged"] > 0
        assert np.all(np.isfinite(g))


def test_injected_cg_breakdown_returns_last_iterate():
    _say("failure: CG breakdown before iteration 3")
    w, A, terms = _state()
    g = np.random.default_rng(3).standard_normal(A.shape)
    with binding.Context(A, w["chi"]) as ctx:
        ctx.converge(0.0, 10)
        x3, it3, _, brk3 = ctx.precond(g, 1e-4, 0.0, 3)
        assert it3 == 3 and not brk3
        ctx.set_fault(2, 3)
        xb, itb, _, brk = ctx.precond(g, 1e-4, 0.0, 50)
        assert brk and itb == 3
        assert np.array_equal(xb, x3)
        ctx.set_fault(0)
        x, it, _, brk = ctx.precond(g, 1e-4, 0.0, 5)
        assert not brk and it == 5


def test_allocation_failure_is_enomem_and_context_recovers():
    """Under a device-memory budget far below the gradient's working set the
    call fails with ENOMEM, writes nothing, and the context gives the same
    results as a fresh one once the budget is lifted."""
    _say("failure: memory budget 1 MB")
    w, A, terms = _state()
    with binding.Context(A, w["chi"]) as ref:
        ref.converge(0.0, 10)
        e_ref, g_ref = ref.energy_grad(terms, grad=True)
    with binding.Context(A, w["chi"]) as ctx:
        ctx.converge(0.0, 10)
        ctx.set_fault(1, 1 << 20)
        with pytest.raises(binding.IpepsError) as ei:
            ctx.energy_grad(terms, grad=True)
        assert ei.value.status == binding.ENOMEM
        ctx.set_fault(0)
        e, g = ctx.energy_grad(terms, grad=True)
    assert e == e_ref
    assert np.array_equal(g, g_ref)
