"""Unit checks of single device kernels against plain numpy FP64."""
import numpy as np
import pytest

from paper_2511_09546_amd import binding

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)


@pytest.mark.parametrize("M,N,K,tA,tB", [
    (16, 16, 4, False, False), (64, 64, 16, False, False),
    (70, 33, 19, False, False), (70, 33, 19, True, False),
    (70, 33, 19, False, True), (70, 33, 19, True, True),
    (129, 200, 300, False, False), (5, 300, 1, False, False),
    (300, 200, 700, False, False), (300, 200, 700, True, False),
    (300, 200, 700, False, True), (300, 200, 700, True, True),
    (2592, 96, 2592, False, False), (2592, 72, 2592, True, False),
    (257, 65, 33, True, True), (36, 36, 20000, False, False),
    (100, 1000, 16, False, True),
    # 65 to 96 rows: 96-row tiles, split K
    (72, 72, 2592, True, False), (96, 130, 5000, True, False),
    (80, 24, 3000, False, True),
    # at most 4 x 4 outputs with a long K: vector-unit kernel, chunked K
    (4, 4, 20000, False, False), (3, 4, 9001, True, False),
    (4, 2, 70000, False, True), (1, 1, 4096, True, True),
    (2, 3, 1100000, False, False)])
def test_gemm(M, N, K, tA, tB):
    _say(f"gemm {M}x{N}x{K} tA={tA} tB={tB}")
    rng = np.random.default_rng(M * N + K)
    A = rng.standard_normal((K, M) if tA else (M, K))
    B = rng.standard_normal((N, K) if tB else (K, N))
    C0 = rng.standard_normal((M, N))
    C = binding.debug_gemm(A, B, C0, tA, tB, alpha=0.7, beta=-0.3)
    ref = 0.7 * ((A.T if tA else A) @ (B.T if tB else B)) - 0.3 * C0
    assert np.abs(C - ref).max() < 1e-12 * max(1.0, np.abs(ref).max()) * K


@pytest.mark.parametrize("prec", [binding.FP32, binding.BF16])
def test_small_output_gemm_is_fp64(prec):
    """Products with at most 4 x 4 outputs and K >= 4096 run as FP64 FMAs
    whatever the contraction arithmetic: FP64 accuracy, not FP32's."""
    _say(f"small-output gemm 4x3x50000, prec {prec}")
    rng = np.random.default_rng(11)
    A = rng.standard_normal((4, 50000))
    B = rng.standard_normal((50000, 3))
    C0 = rng.standard_normal((4, 3))
    C = binding.debug_gemm_prec(prec, A, B, C0, alpha=1.5, beta=0.5)
    ref = 1.5 * (A @ B) + 0.5 * C0
    assert np.abs(C - ref).max() < 1e-10


def test_gemm_split_k():
    _say("gemm split-K 36x36x5000")
    rng = np.random.default_rng(3)
    A = rng.standard_normal((36, 5000))
    B = rng.standard_normal((5000, 36))
    C = binding.debug_gemm(A, B, np.zeros((36, 36)))
    assert np.abs(C - A @ B).max() < 1e-10


@pytest.mark.parametrize("shape,perm,beta", [
    ((7, 5, 3), (2, 0, 1), 0.0),             # generic path
    ((40, 3, 70), (2, 1, 0), 0.0),           # tiled, ragged tiles
    ((33, 36, 34), (0, 2, 1), -0.5),         # tiled, accumulate
    ((2, 3, 4, 5, 6, 7), (5, 3, 1, 0, 2, 4), 0.0),
    ((300, 4, 300, 4), (0, 3, 2, 1), 0.0),  # tiled, 90000 outer tiles
    ((5, 4, 3, 6), (0, 3, 2, 1), -0.5),      # tile of 4 x 256
    ((130, 6, 70), (2, 1, 0), 0.0),          # q longer than one tile
    ((40, 300), (1, 0), 0.0),                # short output row: one tile
    ((5, 36, 2600), (0, 2, 1), -0.5),        # the same, D^2 = 36, accumulate
    ((4, 1000), (1, 0), 0.0),                # row of 4: TQ capped at 256
    ((3, 4), (0, 1), 0.5)])                  # identity: plain copy
def test_permute(shape, perm, beta):
    _say(f"permute {shape} {perm} beta={beta}")
    rng = np.random.default_rng(len(shape) + shape[0])
    X = rng.standard_normal(shape)
    out0 = rng.standard_normal(tuple(shape[p] for p in perm))
    out = binding.debug_permute(X, perm, alpha=0.7, beta=beta, out=out0)
    ref = 0.7 * np.transpose(X, perm) + beta * out0
    assert np.array_equal(out, ref) if beta == 0.0 else \
        np.abs(out - ref).max() < 1e-15


@pytest.mark.parametrize("b,batch", [(2, 1), (8, 3), (32, 2), (96, 1),
                                     (128, 1)])
def test_sym_eig(b, batch):
    _say(f"sym_eig b={b} batch={batch}")
    rng = np.random.default_rng(b)
    X = rng.standard_normal((batch, b, b))
    G = X + X.transpose(0, 2, 1)
    lam, V = binding.debug_sym_eig(G)
    for i in range(batch):
        ref = np.sort(np.linalg.eigvalsh(G[i]))[::-1]
        assert np.abs(lam[i] - ref).max() < 1e-12 * np.abs(ref).max() * b
        assert np.abs(V[i].T @ V[i] - np.eye(b)).max() < 1e-13 * b
        assert np.abs(V[i] @ np.diag(lam[i]) @ V[i].T - G[i]).max() \
            < 1e-12 * np.abs(G[i]).max() * b


@pytest.mark.parametrize("b,batch", [(130, 2), (192, 1), (256, 3)])
def test_sym_eig_large_block(b, batch):
    """Blocks beyond 128 (the global-memory Jacobi kernel): the same bounds
    as the LDS kernel, on random and on nearly diagonal graded matrices."""
    _say(f"sym_eig large b={b} batch={batch}")
    rng = np.random.default_rng(b)
    X = rng.standard_normal((batch, b, b))
    G = X + X.transpose(0, 2, 1)
    # the last entry: graded diagonal plus a small symmetric perturbation
    d = np.logspace(0, -8, b)
    E = 1e-6 * rng.standard_normal((b, b))
    G[-1] = np.diag(d) + (E + E.T) * np.sqrt(np.outer(d, d))
    lam, V = binding.debug_sym_eig(G)
    for i in range(batch):
        ref = np.sort(np.linalg.eigvalsh(G[i]))[::-1]
        assert np.abs(lam[i] - ref).max() < 1e-12 * np.abs(ref).max() * b
        assert np.abs(V[i].T @ V[i] - np.eye(b)).max() < 1e-13 * b
        assert np.abs(V[i] @ np.diag(lam[i]) @ V[i].T - G[i]).max() \
            < 1e-12 * np.abs(G[i]).max() * b


def test_svd_ts_graded_large_block():
    """The graded tall-skinny SVD at b = 192 (global-memory Jacobi)."""
    _say("svd_ts graded, b = 192")
    rng = np.random.default_rng(6)
    n, b = 700, 192
    Q1, _ = np.linalg.qr(rng.standard_normal((n, b)))
    Q2, _ = np.linalg.qr(rng.standard_normal((b, b)))
    s_true = np.logspace(0, -10, b)
    W = (Q1 * s_true) @ Q2.T
    U, s, J = binding.debug_svd_ts(W[None])
    # rounding of the Gram products and of b - 1 rotations per sweep: the
    # b = 24 bounds scaled by b / 24
    assert np.abs(s[0] - s_true).max() < 1e-14 * b / 24
    big = s_true >= 1e-5
    assert np.abs(s[0][big] / s_true[big] - 1).max() < 1e-10
    assert np.abs(U[0].T @ U[0] - np.eye(b)).max() < 1e-12 * b / 24
    assert np.abs(W @ J[0] - U[0] * s[0]).max() < 1e-13 * b / 24
    assert np.abs(J[0].T @ J[0] - np.eye(b)).max() < 1e-13 * b / 24


def test_svd_ts_graded():
    """Singular values spanning 10 orders of magnitude: absolute accuracy
    1e-14 s_1 for all of them, relative accuracy 1e-10 down to 1e-5 s_1 (the
    second Gram/Jacobi pass restores what squaring lost in the first)."""
    _say("svd_ts graded")
    rng = np.random.default_rng(5)
    n, b = 300, 24
    Q1, _ = np.linalg.qr(rng.standard_normal((n, b)))
    Q2, _ = np.linalg.qr(rng.standard_normal((b, b)))
    s_true = np.logspace(0, -10, b)
    W = (Q1 * s_true) @ Q2.T
    U, s, J = binding.debug_svd_ts(W[None])
    assert np.abs(s[0] - s_true).max() < 1e-14
    big = s_true >= 1e-5
    assert np.abs(s[0][big] / s_true[big] - 1).max() < 1e-10
    assert np.abs(U[0].T @ U[0] - np.eye(b)).max() < 1e-12
    assert np.abs(W @ J[0] - U[0] * s[0]).max() < 1e-13
    assert np.abs(J[0].T @ J[0] - np.eye(b)).max() < 1e-13
