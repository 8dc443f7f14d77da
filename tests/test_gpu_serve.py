"""The request loop on the GPU: requests that run concurrently (worker
processes, own contexts and streams) give exactly the results of the same
requests run alone, and a warm start from a cached environment reaches the
same fixed point in fewer iterations."""
import numpy as np
import pytest

from paper_2511_09546_amd import binding, inputs, serve

pytestmark = pytest.mark.gpu


def _solo(req):
    o = binding.default_opts()
    o.prec = req.prec
    o.grad_K = req.grad_K
    o.grad_checkpoint = req.grad_checkpoint or 0
    with binding.Context(req.A, req.chi, opts=o) as ctx:
        it, dl, ok = ctx.converge(req.tol, req.max_iter)
        e, g = ctx.energy_grad(req.terms, grad=True)
        x, cg, res, brk = ctx.precond(g, req.delta, req.cg_tol,
                                      req.cg_maxiter)
    return e, g, x, it


@pytest.mark.parametrize("prec,ckpt", [(binding.FP64, None),
                                       (binding.FP32, None),
                                       (binding.FP64, 1)])
def test_concurrent_equals_solo(prec, ckpt):
    print(f"serve concurrent vs solo prec={prec} checkpoint={ckpt}",
          flush=True)
    specs = [(2, 8, 0.0), (3, 12, 0.3), (2, 6, 0.5), (3, 10, 0.1),
             (2, 8, 0.2), (3, 9, 0.4)]
    reqs = [serve.Request(A=inputs.random_state(700 + i, 1, 1, 2, D), chi=chi,
                          terms=inputs.terms_j1j2(1, 1, 1.0, J2), prec=prec,
                          max_iter=60, grad_K=6, grad_checkpoint=ckpt)
            for i, (D, chi, J2) in enumerate(specs)]
    srv = serve.Server(50e9, workers=4)
    futs = [srv.submit(r) for r in reqs]
    res = [f.result(timeout=120) for f in futs]
    srv.close()
    assert srv.max_running >= 2
    # the windows that hold the device work of the requests (host clock
    # around their calls) overlap for at least two of them
    assert serve.max_overlap([r.window for r in res]) >= 2
    for r, out in zip(reqs, res):
        e, g, x, it = _solo(r)
        assert out.ctm_iters == it
        assert out.e == e
        assert np.array_equal(out.g, g) and np.array_equal(out.x, x)


def test_warm_start_sweep():
    print("serve warm-start sweep", flush=True)
    A = inputs.random_state(811, 1, 1, 2, 3)
    srv = serve.Server(50e9, workers=1)
    res = []
    for J2 in (0.0, 0.25, 0.5):
        req = serve.Request(A=A, chi=12, terms=inputs.terms_j1j2(1, 1, 1.0, J2),
                            prec=binding.FP64, grad_K=6, state_key="s811")
        res.append(srv.submit(req).result(timeout=120))
    srv.close()
    assert not res[0].warm and res[1].warm and res[2].warm
    # a converged FP64 environment converges again in one iteration
    assert res[1].ctm_iters == 1 and res[2].ctm_iters == 1 < res[0].ctm_iters
    for J2, r in zip((0.0, 0.25, 0.5), res):
        req = serve.Request(A=A, chi=12, terms=inputs.terms_j1j2(1, 1, 1.0, J2),
                            prec=binding.FP64, grad_K=6)
        e, g, x, it = _solo(req)
        assert abs(r.e - e) < 1e-9 * abs(e)


def test_sweep_requests_wait_for_their_state_fp32():
    """Two states, three couplings each, all submitted at once to two
    workers: a request whose state is still running waits for it and then
    starts from the environment it left (FP32 contractions: a few CTMRG
    iterations instead of a cold convergence)."""
    print("serve sweep, FP32, concurrent submission", flush=True)
    states = [(inputs.random_state(6001, 1, 1, 2, 4), 40),
              (inputs.random_state(6001, 1, 1, 2, 5), 60)]
    srv = serve.Server(100e9, workers=2)
    futs = []
    for J2 in (0.0, 0.3, 0.6):
        for i, (A, chi) in enumerate(states):
            futs.append(srv.submit(serve.Request(
                A=A, chi=chi, terms=inputs.terms_j1j2(1, 1, 1.0, J2),
                prec=binding.FP32, grad_K=6, state_key=f"sweep-{i}")))
    res = [f.result(timeout=300) for f in futs]
    srv.close()
    cold = [r.ctm_iters for r in res if not r.warm]
    warm = [r.ctm_iters for r in res if r.warm]
    print(f"  cold {cold}, warm {warm}", flush=True)
    assert len(cold) == 2 and len(warm) == 4
    assert max(warm) <= 6 < min(cold)
