"""precond_apply_dev_noalloc against precond_apply_dev through the C ABI.

Two calls in a row on different states, the second smaller, each compared
element by element with the allocating entry point on the same context
(FP64: within 1e-12 relative; the lean metric application splits the batched
product per physical index, so the rounding order of a split-K reduction
may differ), with equal CG iteration counts, and no growth of the context's
memory pool across the allocation-free call.
"""
import numpy as np
import pytest
import torch

from paper_2511_09546_amd import binding, inputs

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)


def _compare(D, chi, seed, Lx=1, Ly=1, d=2):
    _say(f"noalloc vs precond_apply_dev: {Lx}x{Ly} d={d} D={D} chi={chi}")
    A = np.stack([inputs.random_state(seed + i, 1, 1, d, D)[0, 0]
                  for i in range(Lx * Ly)]).reshape(Ly, Lx, d, *(D,) * 4)
    assert binding.noalloc_bytes(Lx, Ly, d, D, chi) <= \
        binding.NOALLOC_SCRATCH_BYTES
    g = np.random.default_rng(seed + 100).standard_normal(A.shape)
    with binding.Context(A, chi) as ctx:
        ctx.converge(1e-9, 60)
        dg = torch.tensor(g, dtype=torch.float64, device="cuda:0")
        dx1 = torch.zeros_like(dg)
        dx2 = torch.full_like(dg, 7.0)   # stale contents must not leak in
        torch.cuda.synchronize()
        it1, r1, b1 = ctx.precond_dev(dg.data_ptr(), dx1.data_ptr(), 1e-4,
                                      0.0, 20)
        before = ctx.stats()["pool_bytes"]
        it2, r2, b2 = ctx.precond_dev_noalloc(dg.data_ptr(), dx2.data_ptr(),
                                              1e-4, 0.0, 20)
        after = ctx.stats()["pool_bytes"]
        x1, x2 = dx1.cpu().numpy(), dx2.cpu().numpy()
    err = np.abs(x2 - x1).max() / np.abs(x1).max()
    _say(f"  iters {it1} / {it2}, resid {r1:.3e} / {r2:.3e}, "
         f"max rel diff {err:.2e}, pool {before} -> {after}")
    assert it1 == it2 and b1 == b2
    assert abs(r1 - r2) <= 1e-10 * max(r1, 1e-300) + 1e-15
    assert err < 1e-12
    assert after == before


def test_noalloc_matches_precond_two_calls():
    # first call on the larger state, then a smaller one: the second call
    # reuses the scratch area that the first one left filled
    _compare(D=4, chi=32, seed=21)
    _compare(D=2, chi=8, seed=22)


def test_noalloc_two_by_two_cell():
    _compare(D=3, chi=12, seed=30, Lx=2, Ly=2, d=4)


def test_noalloc_refuses_oversized_state():
    """A state whose working set exceeds the scratch array is refused before
    any work (IPEPS_ESCRATCH)."""
    D, chi = 6, 100
    need = binding.noalloc_bytes(1, 1, 2, D, chi)
    _say(f"noalloc oversized: needs {need} bytes")
    assert need > binding.NOALLOC_SCRATCH_BYTES
    A = inputs.random_state(5, 1, 1, 2, D)
    with binding.Context(A, chi) as ctx:
        C, T = ctx.get_env()
        ctx.set_env(C, T)      # an environment to precondition with
        dg = torch.zeros(A.shape, dtype=torch.float64, device="cuda:0")
        dx = torch.zeros_like(dg)
        with pytest.raises(binding.IpepsError) as ei:
            ctx.precond_dev_noalloc(dg.data_ptr(), dx.data_ptr(), 1e-4, 0.0,
                                    5)
        assert ei.value.status == binding.ESCRATCH
