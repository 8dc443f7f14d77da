"""Memory hygiene of the device path: with the memory check mode
(IPEPS_MEMCHECK=2: guard bands around every device tensor, every new tensor
filled with NaN, released blocks held back from reuse until verified) one
step of every entry point leaves every guard band intact (no kernel writes
outside its tensor) and gives bitwise the results of the same step without
the check (no kernel reads memory that nothing wrote)."""
import os

import numpy as np
import pytest

from paper_2511_09546_amd import binding, inputs

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)


def _step(A, chi, terms, prec, ckpt, mode, extra):
    """(results, guard damage per phase) of one step with IPEPS_MEMCHECK =
    mode for the contexts created here."""
    old = os.environ.get("IPEPS_MEMCHECK")
    os.environ["IPEPS_MEMCHECK"] = str(mode)
    try:
        o = binding.default_opts()
        o.prec = prec
        o.grad_K = 6
        o.grad_checkpoint = ckpt
        out, dmg = [], []
        with binding.Context(A, chi, opts=o) as ctx:
            it, dl, ok = ctx.converge(1e-10, 80)
            dmg.append(ctx.memcheck())
            e, g = ctx.energy_grad(terms, grad=True)
            dmg.append(ctx.memcheck())
            x, cg, res, brk = ctx.precond(g, 1e-4, 0.0, 20)
            dmg.append(ctx.memcheck())
            out += [it, e, g, x]
            if extra:
                out.append(ctx.precond_gmres(g, 1e-4, m=8)[0])
                dmg.append(ctx.memcheck())
                ctx.bp_converge()
                out.append(ctx.precond_bp(g, 1e-4))
                dmg.append(ctx.memcheck())
                out.append(ctx.metric_full(g))
                dmg.append(ctx.memcheck())
        if extra:
            # the C4v path (QR-CTMRG, its gradient)
            with binding.Context(A, chi, opts=o) as ctx:
                out.append(ctx.c4v_converge(1e-10, 100))
                dmg.append(ctx.memcheck())
                out += list(ctx.c4v_energy_grad(terms))
                dmg.append(ctx.memcheck())
        return out, dmg
    finally:
        if old is None:
            os.environ.pop("IPEPS_MEMCHECK", None)
        else:
            os.environ["IPEPS_MEMCHECK"] = old


def _same(a, b):
    if isinstance(a, tuple):
        return all(_same(x, y) for x, y in zip(a, b))
    if isinstance(a, np.ndarray):
        return np.array_equal(a, b)
    return a == b


@pytest.mark.parametrize("D,chi,prec,ckpt,extra", [
    (2, 8, binding.FP64, 0, True),
    (3, 18, binding.FP32, 0, False),
    (3, 20, binding.FP32, 1, False),
    (3, 18, binding.BF16, 0, False),
    (4, 34, binding.FP32, 0, False),
])
def test_step_stays_inside_its_tensors(D, chi, prec, ckpt, extra):
    _say(f"memcheck D={D} chi={chi} prec={prec} checkpoint={ckpt}")
    A = inputs.random_state(900 + D, 1, 1, 2, D)
    terms = inputs.terms_j1j2(1, 1, 1.0, 0.3)
    plain, none = _step(A, chi, terms, prec, ckpt, 0, extra)
    checked, dmg = _step(A, chi, terms, prec, ckpt, 2, extra)
    _say(f"  damaged guard bands per phase {dmg}")
    assert all(n == -1 for n in none)
    assert dmg == [0] * len(dmg)
    assert all(_same(p, c) for p, c in zip(plain, checked))
