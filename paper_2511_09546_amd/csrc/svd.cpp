// Truncated SVD of the half-system cut matrices M = Qa Qb (never formed).
//
// Block subspace iteration with Rayleigh-Ritz on M^T M, warm-started from the
// right singular block of the previous CTMRG iteration (the products with
// Qa, Qb in the contraction precision, everything else in FP64):
//   W = M X = Qa (Qb X)                       (two GEMMs)
//   W J = U diag(s)   (tall-skinny SVD, below), V = X J
//   Z = M^T U = Qb^T (Qa^T U)                 (two GEMMs)
//   stop when max_{i<chi} ||Z_i - s_i V_i|| <= tol * s_1, else X = orth(Z)
//   (Cholesky QR of the column-normalised Z).
// When the block covers the whole space (b >= n) X is the identity and one
// pass gives the exact SVD.
//
// Tall-skinny SVD of W (n x b): two passes of "Gram matrix W^T W, Jacobi
// eigendecomposition W^T W = J diag(l) J^T, W <- W J".  The first pass makes
// the columns nearly orthogonal; the second works on a graded, nearly
// diagonal Gram matrix, where Jacobi is relatively accurate, and restores the
// relative accuracy of the small singular values.  s = column norms; values
// below 1e-13 of the largest are set to zero with a zero column (rank
// deficient blocks, e.g. zero-padded environments, stay orthonormal where
// they are nonzero).
#include <algorithm>
#include <cmath>

#include "ipeps_impl.hpp"

namespace ipeps {

void svd_ts(Device& dev, const Tensor& W, int batch, int64_t n, int b,
            Tensor& U, Tensor& S, Tensor& J, double tol2) {
  PrecScope f64(dev, PREC_FP64);
  const int64_t sW = n * b, sG = (int64_t)b * b;
  Tensor G = dev.empty({batch, b, b});
  Tensor J1 = dev.empty({batch, b, b});
  Tensor J2 = dev.empty({batch, b, b});
  Tensor lam = dev.empty({batch, b});
  Tensor B1 = dev.empty({batch, n, b});
  // pass 1
  gemm(dev, true, false, b, b, n, 1.0, W.ptr, b, sW, W.ptr, b, sW, 0.0, G.ptr,
       b, sG, batch);
  // pass 1 only has to make the columns nearly orthogonal (cosines below
  // 1e-8); pass 2 then converges in a sweep or two to full accuracy
  sym_eig_jacobi(dev, G.ptr, J1.ptr, lam.ptr, b, batch, 1e-8);
  gemm(dev, false, false, n, b, b, 1.0, W.ptr, b, sW, J1.ptr, b, sG, 0.0,
       B1.ptr, b, sW, batch);
  // pass 2
  gemm(dev, true, false, b, b, n, 1.0, B1.ptr, b, sW, B1.ptr, b, sW, 0.0,
       G.ptr, b, sG, batch);
  sym_eig_jacobi(dev, G.ptr, J2.ptr, lam.ptr, b, batch, tol2);
  if (U.numel() != batch * n * b) U = dev.empty({batch, n, b});
  if (S.numel() != batch * b) S = dev.empty({batch, b});
  if (J.numel() != batch * sG) J = dev.empty({batch, b, b});
  gemm(dev, false, false, n, b, b, 1.0, B1.ptr, b, sW, J2.ptr, b, sG, 0.0,
       U.ptr, b, sW, batch);
  gemm(dev, false, false, b, b, b, 1.0, J1.ptr, b, sG, J2.ptr, b, sG, 0.0,
       J.ptr, b, sG, batch);
  col_norms(dev, U.ptr, n, b, S.ptr, batch, sW, b);
  // columns at rounding level (<= 1e-13 of the largest) are exact zeros:
  // normalising them would inject non-orthogonal noise into the subspace
  null_threshold(dev, S.ptr, b, 1e-13, batch, b);
  col_scale(dev, U.ptr, n, b, S.ptr, 0, nullptr, batch, sW, b);
}

void orth_block(Device& dev, const Tensor& Z, int batch, int64_t n, int b,
                Tensor& X) {
  PrecScope f64(dev, PREC_FP64);
  const int64_t sZ = n * b, sG = (int64_t)b * b;
  Tensor cn = dev.empty({batch, b});
  col_norms(dev, Z.ptr, n, b, cn.ptr, batch, sZ, b);
  null_threshold(dev, cn.ptr, b, 1e-13, batch, b);
  Tensor Zs = dev.empty({batch, n, b});
  axpby(dev, batch * sZ, 1.0, Z.ptr, 0.0, Zs.ptr);
  // null columns of Z (directions M does not reach while the environment
  // is rank deficient, e.g. a small bond still growing towards chi) are
  // refilled with fresh pseudo-random directions before the orthogonal
  // basis is formed: dropped, they would never come back, and the block
  // would stay short of chi directions once the rank has grown
  fill_null_cols(dev, Zs.ptr, n, b, cn.ptr, batch, 0x0b10c5eedull);
  col_norms(dev, Zs.ptr, n, b, cn.ptr, batch, sZ, b);
  col_scale(dev, Zs.ptr, n, b, cn.ptr, 0, nullptr, batch, sZ, b);
  Tensor G = dev.empty({batch, b, b}), R = dev.empty({batch, b, b});
  gemm(dev, true, false, b, b, n, 1.0, Zs.ptr, b, sZ, Zs.ptr, b, sZ, 0.0,
       G.ptr, b, sG, batch);
  chol_orth_factor(dev, G.ptr, R.ptr, b, batch);
  X = dev.empty({batch, n, b});
  gemm(dev, false, false, n, b, b, 1.0, Zs.ptr, b, sZ, R.ptr, b, sG, 0.0,
       X.ptr, b, sZ, batch);
}

void qmul(Device& dev, int prec, bool tA, int64_t M, int64_t N, int64_t K,
          const std::vector<const double*>& Q,
          const std::vector<const float*>& Q32, int64_t ldq,
          const std::vector<const double*>& B, int64_t ldb,
          const std::vector<double*>& C, int64_t ldc) {
  PrecScope ps(dev, prec);
  if (!Q32.empty())
    gemm_ptrs_a32(dev, tA, false, M, N, K, 1.0, Q32, ldq, B, ldb, 0.0, C,
                  ldc);
  else
    gemm_ptrs(dev, tA, false, M, N, K, 1.0, Q, ldq, B, ldb, 0.0, C, ldc);
}

int subspace_block(int n, int chi, int oversample) {
  int p = oversample > 0 ? oversample : std::max(16, chi / 3);
  int b = chi + p;
  if (b % 2) ++b;
  if (b >= n) {
    b = n + (n % 2);
  }
  if (b > MAX_BLOCK) b = MAX_BLOCK;
  if (b < n && b <= chi) throw ArgError("chi too large for the projector SVD");
  return b;
}

void projector_svd(Device& dev, const CutBatch& cb, Tensor& X, bool warm,
                   Tensor& U, Tensor& S, Tensor& V, Tensor& keep,
                   const SvdParams& prm, SvdStats* stats) {
  const int nc = cb.ncut, b = cb.b;
  const int64_t n = cb.n;
  const bool direct = b >= n;
  const int64_t sX = n * b;
  if (X.numel() != nc * sX) {
    X = dev.empty({nc, n, b});
    warm = false;
  }
  if (direct) {
    eye(dev, X.ptr, n, b, nc, sX);
  } else if (!warm) {
    random_block(dev, X.ptr, nc * sX, 0x5eed1234ull);
    Tensor Uo, So, Jo;
    svd_ts(dev, X, nc, n, b, Uo, So, Jo);
    X = Uo;
  }
  // per-cut block addresses of [nc][n][b] tensors
  auto ptrs = [&](const Tensor& t) {
    std::vector<double*> v(nc);
    for (int c = 0; c < nc; ++c) v[c] = t.ptr + c * sX;
    return v;
  };
  auto cptrs = [&](const Tensor& t) {
    std::vector<const double*> v(nc);
    for (int c = 0; c < nc; ++c) v[c] = t.ptr + c * sX;
    return v;
  };
  Tensor T1 = dev.empty({nc, n, b});
  Tensor W = dev.empty({nc, n, b});
  Tensor Z = dev.empty({nc, n, b});
  Tensor J;
  Tensor res = dev.empty({nc});
  std::vector<double> hres(nc);
  V = dev.empty({nc, n, b});
  int it = 0;
  double worst = 0.0;
  // with FP32 products the residual levels off at a few 1e-6 s_1 (BF16x3:
  // a few 1e-4, single BF16 products about 1e-2): the tolerance is raised
  // to that arithmetic's floor and the iteration also ends when an
  // iteration no longer halves the residual
  const bool lowp = dev.cprec != PREC_FP64;
  const double tol = std::max(prm.tol, prec_floors(dev.cprec).svd_res);
  bool stalled = false;
  double prev = INFINITY;
  for (;;) {
    ++it;
    qmul(dev, dev.cprec, false, n, b, n, cb.Qb, cb.Qb32, n, cptrs(X), b,
         ptrs(T1), b);
    qmul(dev, dev.cprec, false, n, b, n, cb.Qa, cb.Qa32, n, cptrs(T1), b,
         ptrs(W), b);
    svd_ts(dev, W, nc, n, b, U, S, J, lowp ? 1e-12 : 1e-15);
    {
      PrecScope f64(dev, PREC_FP64);
      gemm(dev, false, false, n, b, b, 1.0, X.ptr, b, sX, J.ptr, b,
           (int64_t)b * b, 0.0, V.ptr, b, sX, nc);
    }
    if (direct) break;
    qmul(dev, dev.cprec, true, n, b, n, cb.Qa, cb.Qa32, n, cptrs(U), b,
         ptrs(T1), b);
    qmul(dev, dev.cprec, true, n, b, n, cb.Qb, cb.Qb32, n, cptrs(T1), b,
         ptrs(Z), b);
    svd_residual(dev, Z.ptr, V.ptr, S.ptr, n, b, std::min(cb.chi, b), res.ptr,
                 nc, sX, b);
    dev.download(res, hres.data());
    worst = *std::max_element(hres.begin(), hres.end());
    if (worst <= tol || it >= prm.max_iter) break;
    if (lowp && it >= 3 && worst > 0.5 * prev) {
      stalled = true;
      break;
    }
    prev = worst;
    // next block: an orthonormal basis of span(Z) (Cholesky QR of the
    // column-normalised Z, whose columns are nearly orthogonal since
    // Z ~ V S); the Rayleigh-Ritz step of the next pass makes the result
    // independent of the basis chosen.  Fresh buffer: X may alias the
    // previous call's V, which the backward tape keeps
    Tensor Xn;
    orth_block(dev, Z, nc, n, b, Xn);
    X = Xn;
  }
  sign_fix(dev, U.ptr, V.ptr, n, b, nc, sX, sX);
  if (keep.numel() < nc) keep = dev.empty({nc});
  kept_rank(dev, S.ptr, b, cb.chi, prm.cutoff, (int*)keep.ptr, nc, b);
  X = V;  // warm start of the next call
  if (stats) {
    stats->iters += it;
    stats->calls += 1;
    stats->worst_residual = std::max(stats->worst_residual, worst);
    // ended by the iteration limit above the tolerance in effect (not at
    // the rounding floor of a low-precision arithmetic): the projectors are
    // less accurate than asked, which the entry points report as a warning
    if (!direct && !stalled && worst > tol) ++stats->svd_unconverged;
  }
}

}  // namespace ipeps
