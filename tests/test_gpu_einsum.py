"""The contraction planner against numpy.einsum, with the permuted output
written by the GEMM epilogue (scattered layout) and, for comparison, by a
separate permute pass: both agree with numpy to rounding, and with each
other bitwise (alpha = 1, beta 0 or 1: the epilogue stores the value the
permute pass would), in FP64 and FP32 products, for the contractions of the
CTMRG and energy networks at small ragged sizes, batched items, batch
labels and outputs too scattered for the epilogue."""
import numpy as np
import pytest

from paper_2511_09546_amd import binding

pytestmark = pytest.mark.gpu

CHI, DD, DS = 5, 4, 2   # chi, D^2 (fused double-layer leg), d

CASES = [
    # (spec, shape of A, shape of B)
    ("mgek,gebf->mfkb", (CHI, DD, DD, CHI), (DD, DD, DD, DD)),
    ("mgj,jek->mkge", (CHI, DD, CHI), (CHI, DD, CHI)),
    ("mkge,gebf->mfkb", (CHI, CHI, DD, DD), (DD, DD, DD, DD)),
    ("jgx,jek->xkge", (CHI, DD, CHI), (CHI, DD, CHI)),
    ("xkbf,kby->xfy", (CHI, CHI, DD, DD), (CHI, DD, CHI)),
    ("mgek,stgebf->mfkbst", (CHI, DD, DD, CHI), (DS, DS, DD, DD, DD, DD)),
    ("XYst,YZ->XZst", (12, 12, DS, DS), (12, 12)),
    ("sij,sjk->isk", (3, 7, 6), (3, 6, 9)),       # batch label, not leading
    ("abcde,eg->gdbca", (2, 3, 2, 3, 5), (5, 4)),  # too scattered: fallback
    ("ij,jk->ki", (33, 17), (17, 29)),
]


def _rand(shape, seed):
    return np.random.default_rng(seed).standard_normal(shape)


@pytest.mark.parametrize("prec", [binding.FP64, binding.FP32])
@pytest.mark.parametrize("beta", [0.0, 1.0])
@pytest.mark.parametrize("case", range(len(CASES)))
def test_scattered_output_matches_permute_and_numpy(case, beta, prec):
    spec, sa, sb = CASES[case]
    count = 3
    A = _rand((count,) + sa, 10 + case)
    B = _rand((count,) + sb, 20 + case)
    ref = np.stack([np.einsum(spec, A[i], B[i]) for i in range(count)])
    C0 = _rand(ref.shape, 30 + case)
    ref = ref + beta * C0
    out0, n0 = binding.debug_einsum(spec, A, B, C0, prec=prec, mode=0,
                                    beta=beta)
    out1, n1 = binding.debug_einsum(spec, A, B, C0, prec=prec, mode=1,
                                    beta=beta)
    print(f"{spec} beta={beta} prec={prec}: scattered launches {n0}",
          flush=True)
    assert n1 == 0
    assert np.array_equal(out0, out1)
    scale = np.abs(ref).max()
    tol = 1e-13 if prec == binding.FP64 else 1e-5
    assert np.abs(out0 - ref).max() <= tol * scale * np.sqrt(A.size)


def test_network_contractions_take_the_scattered_epilogue():
    """The enlarged-corner and edge contractions do not fall back to a
    permute pass (their innermost output label is a column label)."""
    for spec, sa, sb in [CASES[i] for i in (0, 1, 2, 3, 5)]:
        A = _rand((2,) + sa, 1)
        B = _rand((2,) + sb, 2)
        out = np.zeros((2,) + np.einsum(spec, A[0], B[0]).shape)
        _, n = binding.debug_einsum(spec, A, B, out)
        print(f"{spec}: scattered launches {n}", flush=True)
        assert n >= 1


def test_alpha_and_general_beta():
    spec, sa, sb = CASES[0]
    A = _rand((2,) + sa, 3)
    B = _rand((2,) + sb, 4)
    C0 = _rand((2, CHI, DD, CHI, DD), 5)
    ref = np.stack([-0.75 * np.einsum(spec, A[i], B[i]) for i in range(2)])
    ref += 0.5 * C0
    out, n = binding.debug_einsum(spec, A, B, C0, alpha=-0.75, beta=0.5)
    assert n >= 1
    assert np.abs(out - ref).max() <= 1e-13 * np.abs(ref).max() * 100
