// Restarted GMRES, one cycle (Sec. III C: the preconditioned gradient is
// obtained from P g' = g by matrix-vector products only, one outer GMRES
// iteration with a Krylov space of 30 vectors).
//
// The Krylov basis V (m+1 vectors of length n) stays on the device; each
// Arnoldi step orthogonalises the new product against the basis with two
// passes of classical Gram-Schmidt, each one product with V^T and one with
// V (GEMMs in FP64), so a step costs one operator application, four thin
// GEMMs, two norms and one download of its m+2 coefficients.  The small
// Hessenberg least-squares problem (Givens rotations, back substitution)
// is host arithmetic on at most 31 x 30 numbers.
#include <cmath>
#include <vector>

#include "ipeps_impl.hpp"

namespace ipeps {

int gmres(Device& dev, int64_t n, const double* b, double* x, int m,
          double tol, const std::function<void(const double*, double*)>& op,
          double* rel_resid) {
  const int caller = dev.cprec;
  Tensor V = dev.empty({(int64_t)m + 1, n});
  // h: coefficients of the two passes ([m+1] each), then |w| before and
  // after the orthogonalisation
  Tensor h = dev.empty({2 * ((int64_t)m + 1) + 2});
  double* h1 = h.ptr;
  double* h2 = h.ptr + (m + 1);
  double* nw = h.ptr + 2 * (m + 1);
  nrm2(dev, b, n, nw);
  double beta = 0.0;
  Tensor nw_t = h.view({(int64_t)h.numel()});
  nw_t.ptr = nw;
  nw_t.shape = {1};
  dev.download(nw_t, &beta);
  if (!(beta > 0.0)) {
    fill(dev, x, n, 0.0);
    if (rel_resid) *rel_resid = 0.0;
    return 0;
  }
  axpby(dev, n, 1.0 / beta, b, 0.0, V.ptr);
  std::vector<double> H((size_t)(m + 1) * m, 0.0), cs(m), sn(m),
      e(m + 1, 0.0), hv(2 * (m + 1) + 2);
  auto Hr = [&](int i, int j) -> double& { return H[(size_t)i * m + j]; };
  e[0] = beta;
  int k = 0;
  for (int j = 0; j < m; ++j) {
    double* w = V.ptr + (int64_t)(j + 1) * n;
    {
      PrecScope ps(dev, caller);
      op(V.ptr + (int64_t)j * n, w);
    }
    PrecScope ps(dev, PREC_FP64);
    nrm2(dev, w, n, nw);
    // two passes: c = V_j w, w -= V_j^T c over the first j+1 vectors
    gemm(dev, false, false, j + 1, 1, n, 1.0, V.ptr, n, 0, w, 1, 0, 0.0, h1,
         1, 0);
    gemm(dev, true, false, n, 1, j + 1, -1.0, V.ptr, n, 0, h1, 1, 0, 1.0, w,
         1, 0);
    gemm(dev, false, false, j + 1, 1, n, 1.0, V.ptr, n, 0, w, 1, 0, 0.0, h2,
         1, 0);
    gemm(dev, true, false, n, 1, j + 1, -1.0, V.ptr, n, 0, h2, 1, 0, 1.0, w,
         1, 0);
    nrm2(dev, w, n, nw + 1);
    dev.download(h, hv.data());
    for (int i = 0; i <= j; ++i) Hr(i, j) = hv[i] + hv[m + 1 + i];
    const double wn = hv[2 * (m + 1)];
    const double hn = hv[2 * (m + 1) + 1];
    Hr(j + 1, j) = hn;
    // the earlier rotations on the new column, then the one that zeroes
    // its subdiagonal entry
    for (int i = 0; i < j; ++i) {
      const double t = cs[i] * Hr(i, j) + sn[i] * Hr(i + 1, j);
      Hr(i + 1, j) = -sn[i] * Hr(i, j) + cs[i] * Hr(i + 1, j);
      Hr(i, j) = t;
    }
    const double r = std::hypot(Hr(j, j), Hr(j + 1, j));
    cs[j] = Hr(j, j) / r;
    sn[j] = Hr(j + 1, j) / r;
    Hr(j, j) = r;
    Hr(j + 1, j) = 0.0;
    e[j + 1] = -sn[j] * e[j];
    e[j] = cs[j] * e[j];
    k = j + 1;
    if (std::fabs(e[j + 1]) <= tol * beta || hn <= 1e-12 * wn) break;
    axpby(dev, n, 1.0 / hn, w, 0.0, w);
  }
  std::vector<double> y(k, 0.0);
  for (int i = k - 1; i >= 0; --i) {
    double t = e[i];
    for (int l = i + 1; l < k; ++l) t -= Hr(i, l) * y[l];
    y[i] = t / Hr(i, i);
  }
  PrecScope ps(dev, PREC_FP64);
  Tensor y_t = h.view({(int64_t)h.numel()});
  y_t.shape = {(int64_t)k};
  dev.upload(y_t, y.data());
  gemm(dev, true, false, n, 1, k, 1.0, V.ptr, n, 0, h1, 1, 0, 0.0, x, 1, 0);
  if (rel_resid) *rel_resid = std::fabs(e[k]) / beta;
  return k;
}

}  // namespace ipeps
