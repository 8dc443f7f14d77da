"""Mixed contraction arithmetic (ipeps_prec IPEPS_FP32 and IPEPS_BF16): the
FP32 GEMM against the rounding-error bound of an FP32 dot product, the
BF16x3 GEMM against its split-rounding bound, and the whole step in both
arithmetics against the FP64 oracle's stored values.

Bounds used:
  * GEMM: |fl(A B) - A B| <= gamma_{K+2} |A| |B| elementwise, gamma_m =
    m u / (1 - m u), u = 2^-24 (operands rounded to FP32, then K products
    accumulated in FP32 in any order).
  * energy per site: within 1e-5 of the FP64 value (absolute), the accuracy
    the mixed-precision mode is built for; measured about 1e-8.
  * gradient and preconditioned direction: the environment of the FP32 run
    is converged to its spectrum-change floor 1e-7, the projector SVD to
    residual 1e-5 and the complement solves of the unrolled adjoint to
    relative residual 1e-5, all on FP32 products; the gradient then carries
    relative errors of order 1e-5 (measured 4e-6 at D=2, 1.3e-5 at D=6) and
    x = (N + 1e-4)^-1 g about the same.  The tests allow 1e-4 on both.
"""
import json
import os

import numpy as np
import pytest

from paper_2511_09546_amd import binding, inputs

pytestmark = pytest.mark.gpu
# BF16x3 (three BF16 products of a two-term split, about 16 significant
# bits): environment converged to its spectrum floor 3e-6, projector
# residual 1e-3, complement solves 1e-3; measured relative errors of g and x
# up to 5e-4 (D=2 chi=8), energies within 3.4e-7
BF16_REL = 2e-3
GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _say(msg):
    print(msg, flush=True)


@pytest.mark.parametrize("tA,tB,M,N,K", [(0, 0, 200, 130, 300),
                                         (1, 0, 129, 72, 2592),
                                         (0, 1, 300, 48, 1296),
                                         (0, 0, 2592, 72, 2592),
                                         # 128 x 128 tiles, every
                                         # transpose, ragged M, N, K
                                         (1, 0, 530, 600, 1000),
                                         (0, 1, 530, 600, 1000),
                                         (1, 1, 530, 600, 1000),
                                         (0, 0, 517, 613, 131),
                                         # direct LDS loads (even extents,
                                         # K >= 256), split K, ragged tiles
                                         (0, 0, 1296, 1296, 512),
                                         (0, 0, 260, 258, 4000),
                                         (1, 1, 130, 386, 2050),
                                         # the same with 128 x 144 tiles
                                         (0, 0, 300, 288, 512),
                                         (1, 0, 260, 432, 600),
                                         (0, 1, 260, 432, 600),
                                         (1, 1, 260, 432, 600),
                                         # narrow direct-load tiles
                                         (0, 0, 300, 72, 2592),
                                         (1, 0, 300, 96, 1000),
                                         (0, 1, 260, 40, 600),
                                         # 96-row tiles, split K
                                         (1, 0, 72, 72, 2592),
                                         (1, 0, 96, 72, 5184),
                                         (0, 0, 72, 2592, 2592),
                                         (1, 1, 90, 200, 700)])
def test_fp32_gemm_error_bound(tA, tB, M, N, K):
    _say(f"fp32 gemm {tA}{tB} {M}x{N}x{K}")
    rng = np.random.default_rng(M + N + K)
    A = rng.standard_normal((M, K))
    B = rng.standard_normal((K, N))
    C0 = rng.standard_normal((M, N))
    Aop = A.T.copy() if tA else A
    Bop = B.T.copy() if tB else B
    C = binding.debug_gemm_prec(binding.FP32, Aop, Bop, C0, tA=bool(tA),
                                tB=bool(tB), alpha=1.0, beta=0.0)
    ref = A @ B
    u = 2.0 ** -24
    m = K + 2
    gamma = m * u / (1 - m * u)
    bound = gamma * (np.abs(A) @ np.abs(B))
    err = np.abs(C - ref)
    _say(f"  max err/bound {np.max(err / bound):.3f}")
    assert np.all(err <= bound)
    # and it is not silently the FP64 path
    assert np.max(err) > 0.0


@pytest.mark.parametrize("name", ["d2chi8", "d4chi32", "d6chi72",
                                  "kitaev2x2"])
def test_fp32_step_against_golden(name):
    _step_against_golden(name, binding.FP32, 1e-4)


@pytest.mark.parametrize("name", ["d2chi8", "d4chi32", "d6chi72",
                                  "kitaev2x2"])
def test_bf16x3_step_against_golden(name):
    _step_against_golden(name, binding.BF16, BF16_REL)


@pytest.mark.parametrize("name,prec", [("d2chi8", binding.BF16X1),
                                       ("d4chi32", binding.BF16X1),
                                       ("d4chi32", binding.BF16)])
def test_ladder_steps_up_to_fp32(name, prec):
    """BF16 -> FP32 ladder (ipeps_opts.ladder): the converge phase ends in
    FP32 (the arithmetic the context reports for its next calls), and the
    step then meets the FP32 bounds against the FP64 oracle."""
    _step_against_golden(name, prec, 1e-4, ladder=1)


def _step_against_golden(name, prec, rel, ladder=0):
    _say(f"prec {prec} ladder {ladder} step vs golden {name}")
    gold = json.load(open(os.path.join(GOLDEN, f"{name}.json")))
    w = inputs.WORKLOADS[name]
    A = inputs.workload_state(name)
    terms = inputs.workload_terms(name)
    g_or = np.array(gold["g"]).reshape(A.shape)
    x_or = np.array(gold["x"]).reshape(A.shape)
    o = binding.default_opts()
    o.prec = prec
    o.ladder = ladder
    with binding.Context(A, w["chi"], opts=o) as ctx:
        it, dl, ok = ctx.converge(w["tol"], w["n_iter"])
        if ladder:
            assert ctx.stats()["work_prec"] == binding.FP32
        e, g = ctx.energy_grad(terms, grad=True)
        x, cg_it, res, brk = ctx.precond(g, w["delta"], w["cg_tol"],
                                         w["cg_maxiter"])
    eg = np.linalg.norm(g - g_or) / np.linalg.norm(g_or)
    ex = np.linalg.norm(x - x_or) / np.linalg.norm(x_or)
    _say(f"  iters {it} (delta {dl:.1e}) vs {gold['n_iter']}, e {e!r} vs "
         f"{gold['e']!r} (diff {e - gold['e']:.1e}), grad rel {eg:.2e}, "
         f"x rel {ex:.2e}")
    assert abs(e - gold["e"]) < 1e-5
    assert eg < rel
    assert ex < rel


@pytest.mark.parametrize("tA,tB,M,N,K", [(0, 0, 200, 130, 300),
                                         (1, 0, 129, 72, 2592),
                                         (0, 1, 300, 48, 1296),
                                         (0, 0, 640, 1296, 1296),
                                         # operands split once into planes
                                         # (both read by >= 4 tiles), all
                                         # transposes, ragged M, N, K
                                         (1, 0, 530, 400, 1000),
                                         (0, 1, 530, 400, 1000),
                                         (1, 1, 530, 400, 1000),
                                         (0, 0, 517, 389, 131),
                                         # 96-row tiles, split K
                                         (1, 0, 72, 72, 2592),
                                         (0, 0, 80, 300, 1000)])
def test_bf16x3_gemm_error_bound(tA, tB, M, N, K):
    """x = hi + lo + r with hi = bf16(fl32(x)), lo = bf16(fl32(x) - hi) and
    BF16 unit roundoff 2^-8: |fl32(x) - hi| <= 2^-8 |x|, so
    |r| <= (2^-24 + 2^-16) |x| (FP32 rounding, then the rounding of the
    second term); the dropped lo*lo term is at most 2^-16 |a||b| and the three
    exact BF16 products accumulate in FP32.  Bound per element:
    (2 (2^-24 + 2^-16) + 2^-16 + gamma_{3K}) (|A||B|)."""
    _say(f"bf16x3 gemm {tA}{tB} {M}x{N}x{K}")
    rng = np.random.default_rng(M * N + K)
    A = rng.standard_normal((M, K))
    B = rng.standard_normal((K, N))
    Aop = A.T.copy() if tA else A
    Bop = B.T.copy() if tB else B
    C = binding.debug_gemm_prec(binding.BF16, Aop, Bop, np.zeros((M, N)),
                                tA=bool(tA), tB=bool(tB))
    ref = A @ B
    u = 2.0 ** -24
    g = 3 * K * u / (1 - 3 * K * u)
    bound = (2 * (u + 2.0 ** -16) + 2.0 ** -16 + g) * (np.abs(A) @ np.abs(B))
    err = np.abs(C - ref)
    _say(f"  max err/bound {np.max(err / bound):.3f}")
    assert np.all(err <= bound)
    assert np.max(err) > 0.0


@pytest.mark.parametrize("tA,tB,M,N,K", [(0, 0, 200, 130, 300),
                                         (1, 0, 129, 72, 2592),
                                         (0, 0, 640, 1296, 1296),
                                         (1, 1, 530, 400, 1000),
                                         (0, 1, 517, 389, 131),
                                         (1, 0, 72, 72, 2592)])
def test_bf16x1_gemm_error_bound(tA, tB, M, N, K):
    """Single BF16 products: a -> bf16(fl32(a)) with
    |a - bf16(fl32(a))| <= eps |a|, eps = 2^-24 + 2^-8 (1 + 2^-24), so one
    product is off by at most (2 eps + eps^2) |a||b|, and K of them
    accumulate in FP32: bound (2 eps + eps^2 + gamma_K) (|A||B|)."""
    _say(f"bf16x1 gemm {tA}{tB} {M}x{N}x{K}")
    rng = np.random.default_rng(M * N + K + 1)
    A = rng.standard_normal((M, K))
    B = rng.standard_normal((K, N))
    Aop = A.T.copy() if tA else A
    Bop = B.T.copy() if tB else B
    C = binding.debug_gemm_prec(binding.BF16X1, Aop, Bop, np.zeros((M, N)),
                                tA=bool(tA), tB=bool(tB))
    ref = A @ B
    u = 2.0 ** -24
    eps = u + 2.0 ** -8 * (1 + u)
    g = K * u / (1 - K * u)
    bound = (2 * eps + eps * eps + g) * (np.abs(A) @ np.abs(B))
    err = np.abs(C - ref)
    _say(f"  max err/bound {np.max(err / bound):.3f}")
    assert np.all(err <= bound)
    # coarser than the three-product split: not silently BF16x3
    C3 = binding.debug_gemm_prec(binding.BF16, Aop, Bop, np.zeros((M, N)),
                                 tA=bool(tA), tB=bool(tB))
    assert np.max(err) > 10 * np.max(np.abs(C3 - ref))


def test_profile_network_family_is_a_subset():
    """Family 5 (GEMMs of the network contractions) counts a proper subset of
    the FP32 GEMM launches: the projector-SVD and complement-solve products
    are FP32 GEMMs outside it."""
    _say("profile families d2chi8 FP32")
    w = inputs.WORKLOADS["d2chi8"]
    A = inputs.workload_state("d2chi8")
    terms = inputs.workload_terms("d2chi8")
    o = binding.default_opts()
    o.prec = binding.FP32
    with binding.Context(A, w["chi"], opts=o) as ctx:
        ctx.profile(True)
        ctx.converge(w["tol"], w["n_iter"])
        ctx.energy_grad(terms, grad=True)
        n32, t32, f32, _ = ctx.profile_read(binding.PROF_GEMM32)
        nn, tn, fn, _ = ctx.profile_read(binding.PROF_NET)
        n64, _, _, _ = ctx.profile_read(binding.PROF_GEMM)
        ctx.profile(False)
    _say(f"  fp32 {n32} launches, network {nn}, fp64 {n64}")
    assert 0 < nn < n32
    assert 0 < fn < f32 and 0 < tn < t32
    assert n64 > 0  # the SVD's own products stay FP64
