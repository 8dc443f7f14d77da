// Test hooks declared in include/ipeps_debug.h.
#include "../../include/ipeps.h"
#include "../../include/ipeps_debug.h"
#include "ipeps_impl.hpp"

#include <vector>

using namespace ipeps;

namespace {
template <class F>
int run(F&& f) {
  try {
    prime_attributes();
    Device dev;
    dev.stream = nullptr;
    f(dev);
    dev.sync();
    return IPEPS_OK;
  } catch (const ArgError&) {
    return IPEPS_EINVAL;
  } catch (const OomError&) {
    return IPEPS_ENOMEM;
  } catch (...) {
    return IPEPS_EHIP;
  }
}
}  // namespace

extern "C" {

int ipeps_debug_gemm(int tA, int tB, int M, int N, int K, double alpha,
                     const double* A, const double* B, double beta,
                     double* C) {
  if (!A || !B || !C || M < 1 || N < 1 || K < 1) return IPEPS_EINVAL;
  return run([&](Device& dev) {
    Tensor a = dev.empty({(int64_t)M * K}), b = dev.empty({(int64_t)K * N}),
           c = dev.empty({(int64_t)M * N});
    dev.upload(a, A);
    dev.upload(b, B);
    dev.upload(c, C);
    gemm(dev, tA != 0, tB != 0, M, N, K, alpha, a.ptr, tA ? M : K, 0, b.ptr,
         tB ? K : N, 0, beta, c.ptr, N, 0, 1);
    dev.download(c, C);
  });
}

int ipeps_debug_gemm_prec(int prec, int tA, int tB, int M, int N, int K,
                          double alpha, const double* A, const double* B,
                          double beta, double* C) {
  if (!A || !B || !C || M < 1 || N < 1 || K < 1 ||
      (prec < IPEPS_FP64 || prec > IPEPS_BF16X1))
    return IPEPS_EINVAL;
  return run([&](Device& dev) {
    Tensor a = dev.empty({(int64_t)M * K}), b = dev.empty({(int64_t)K * N}),
           c = dev.empty({(int64_t)M * N});
    dev.upload(a, A);
    dev.upload(b, B);
    dev.upload(c, C);
    PrecScope ps(dev, prec);
    gemm(dev, tA != 0, tB != 0, M, N, K, alpha, a.ptr, tA ? M : K, 0, b.ptr,
         tB ? K : N, 0, beta, c.ptr, N, 0, 1);
    dev.download(c, C);
  });
}

int ipeps_debug_gemm_time(int prec, int tA, int tB, int M, int N, int K,
                          int batch, int reps, double* us_per_call) {
  if (!us_per_call || M < 1 || N < 1 || K < 1 || batch < 1 || reps < 1 ||
      (prec < IPEPS_FP64 || prec > IPEPS_BF16X1))
    return IPEPS_EINVAL;
  return run([&](Device& dev) {
    const int64_t sA = (int64_t)M * K, sB = (int64_t)K * N,
                  sC = (int64_t)M * N;
    Tensor a = dev.empty({batch * sA}), b = dev.empty({batch * sB}),
           c = dev.empty({batch * sC});
    random_block(dev, a.ptr, batch * sA, 1);
    random_block(dev, b.ptr, batch * sB, 2);
    PrecScope ps(dev, prec);
    auto call = [&]() {
      gemm(dev, tA != 0, tB != 0, M, N, K, 1.0, a.ptr, tA ? M : K, sA,
           b.ptr, tB ? K : N, sB, 0.0, c.ptr, N, sC, batch);
    };
    call();
    hipEvent_t e0, e1;
    IPEPS_HIP(hipEventCreate(&e0));
    IPEPS_HIP(hipEventCreate(&e1));
    IPEPS_HIP(hipEventRecord(e0, dev.stream));
    for (int r = 0; r < reps; ++r) call();
    IPEPS_HIP(hipEventRecord(e1, dev.stream));
    IPEPS_HIP(hipEventSynchronize(e1));
    float ms = 0.0f;
    IPEPS_HIP(hipEventElapsedTime(&ms, e0, e1));
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    *us_per_call = 1e3 * ms / reps;
  });
}

int ipeps_debug_permute(int rank, const long* shape, const int* perm,
                        double alpha, const double* in, double beta,
                        double* out) {
  if (!shape || !perm || !in || !out || rank < 1 || rank > 12)
    return IPEPS_EINVAL;
  std::vector<int64_t> sh(rank), osh(rank);
  std::vector<int> pm(rank), seen(rank, 0);
  int64_t n = 1;
  for (int d = 0; d < rank; ++d) {
    if (shape[d] < 1 || perm[d] < 0 || perm[d] >= rank || seen[perm[d]])
      return IPEPS_EINVAL;
    seen[perm[d]] = 1;
    sh[d] = shape[d];
    pm[d] = perm[d];
    n *= shape[d];
    if (n >= (1LL << 31)) return IPEPS_EINVAL;
  }
  for (int d = 0; d < rank; ++d) osh[d] = sh[pm[d]];
  return run([&](Device& dev) {
    Tensor a = dev.empty(sh), b = dev.empty(osh);
    dev.upload(a, in);
    dev.upload(b, out);
    permute(dev, a, pm, b, alpha, beta);
    dev.download(b, out);
  });
}

int ipeps_debug_einsum(const char* spec, int prec, int mode, int count,
                       int rankA, const long* shapeA, const double* A,
                       int rankB, const long* shapeB, const double* B,
                       double alpha, double beta, double* out,
                       int* scattered) {
  if (!spec || !A || !B || !out || !scattered || count < 1 || count > 64 ||
      rankA < 1 || rankA > 12 || rankB < 1 || rankB > 12 || mode < 0 ||
      mode > 1 || (prec < IPEPS_FP64 || prec > IPEPS_BF16X1))
    return IPEPS_EINVAL;
  const std::string sp(spec);
  const size_t c = sp.find(','), ar = sp.find("->");
  if (c == std::string::npos || ar == std::string::npos || ar < c ||
      (int)c != rankA || (int)(ar - c - 1) != rankB)
    return IPEPS_EINVAL;
  const std::string la = sp.substr(0, c), lb = sp.substr(c + 1, ar - c - 1),
                    lo = sp.substr(ar + 2);
  std::vector<int64_t> sa(shapeA, shapeA + rankA), sb(shapeB, shapeB + rankB),
      so;
  for (char ch : lo) {
    const size_t i = la.find(ch), j = lb.find(ch);
    if (i == std::string::npos && j == std::string::npos) return IPEPS_EINVAL;
    so.push_back(i != std::string::npos ? sa[i] : sb[j]);
  }
  int64_t na = 1, nb = 1, no = 1;
  for (auto x : sa) na *= x;
  for (auto x : sb) nb *= x;
  for (auto x : so) no *= x;
  if (na < 1 || nb < 1 || no < 1 || count * std::max(na, std::max(nb, no)) >=
                                         (1LL << 31))
    return IPEPS_EINVAL;
  return run([&](Device& dev) {
    std::vector<Tensor> ta, tb, to;
    for (int i = 0; i < count; ++i) {
      Tensor a = dev.empty(sa), b = dev.empty(sb), o = dev.empty(so);
      dev.upload(a, A + i * na);
      dev.upload(b, B + i * nb);
      dev.upload(o, out + i * no);
      ta.push_back(a);
      tb.push_back(b);
      to.push_back(o);
    }
    dev.allow_scatter = mode == 0;
    PrecScope ps(dev, prec);
    einsum_into_n(dev, sp, ta, tb, to, alpha, beta);
    for (int i = 0; i < count; ++i) dev.download(to[i], out + i * no);
    *scattered = (int)dev.scatter_count;
  });
}

int ipeps_debug_sym_eig(int b, int batch, const double* G, double* V,
                        double* lam) {
  if (!G || !V || !lam || b < 2 || b > 512 || b % 2 || batch < 1)
    return IPEPS_EINVAL;
  return run([&](Device& dev) {
    Tensor g = dev.empty({batch, b, b}), v = dev.empty({batch, b, b}),
           l = dev.empty({batch, b});
    dev.upload(g, G);
    sym_eig_jacobi(dev, g.ptr, v.ptr, l.ptr, b, batch);
    dev.download(v, V);
    dev.download(l, lam);
  });
}

int ipeps_debug_svd_ts(int n, int b, int batch, const double* W, double* U,
                       double* s, double* J) {
  if (!W || !U || !s || !J || n < 1 || b < 2 || b > 512 || b % 2 ||
      batch < 1)
    return IPEPS_EINVAL;
  return run([&](Device& dev) {
    Tensor w = dev.empty({batch, n, b});
    dev.upload(w, W);
    Tensor u, sv, j;
    svd_ts(dev, w, batch, n, b, u, sv, j);
    dev.download(u, U);
    dev.download(sv, s);
    dev.download(j, J);
  });
}

}  // extern "C"
