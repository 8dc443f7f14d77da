// Belief-propagation (environment bond dimension 1) environment and the
// preconditioner built on it (Sec. III A after Eq. (11); App. A).
//
// Every leg L of every unit-cell site s receives a message m_s^L, a D x D
// matrix on the leg's ket/bra pair (fused k*D + k' like the double layer).
// One update (parallel schedule: every new message from the previous ones)
// replaces m_s^L by the double layer a of the neighbour across L contracted
// with the three messages arriving at the neighbour's other legs, open on
// the leg that faces s, normalised to unit Frobenius norm with a positive
// trace.  The start is the trace message delta_{k k'}.  The update stops
// when the largest change of a message is below tol.
//
// The site environment is E = m^L (x) m^U (x) m^R (x) m^D and the metric
// acts as N x = (E x) / Z, Z = <A, E A> (Eq. (11) with chi = 1).  Its
// regularised inverse is applied in closed form: with the (symmetrised)
// messages diagonalised, m^k = V_k diag(lambda_k) V_k^T, x is rotated into
// the product eigenbasis by four mode products, divided elementwise by
// lambda_l lambda_u lambda_r lambda_d / Z + delta, and rotated back.  The
// D x D eigendecompositions run in the batched Jacobi kernel (odd D padded
// by one decoupled row with a large negative diagonal, which sorts last).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>

#include "ipeps_impl.hpp"

namespace ipeps {

namespace {

// Normalise every message of a batch (one workgroup per message): unit
// Frobenius norm with a positive trace; change[i] = |m_new - m_old|.
__global__ __launch_bounds__(256) void bp_finish_kernel(
    double* __restrict__ v, const double* __restrict__ old, int n, int D,
    double* __restrict__ change) {
  __shared__ double red[2][256];
  const int t = threadIdx.x;
  double* m = v + (long)blockIdx.x * n;
  const double* o = old + (long)blockIdx.x * n;
  double ss = 0.0, tr = 0.0;
  for (int i = t; i < n; i += 256) {
    const double x = m[i];
    ss += x * x;
    if (i % (D + 1) == 0) tr += x;
  }
  red[0][t] = ss;
  red[1][t] = tr;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (t < w) {
      red[0][t] += red[0][t + w];
      red[1][t] += red[1][t + w];
    }
    __syncthreads();
  }
  const double nrm = sqrt(red[0][0]);
  const double s = nrm > 0.0 ? (red[1][0] < 0.0 ? -1.0 : 1.0) / nrm : 0.0;
  __syncthreads();
  double dd = 0.0;
  for (int i = t; i < n; i += 256) {
    const double x = m[i] * s;
    m[i] = x;
    const double e = x - o[i];
    dd += e * e;
  }
  red[0][t] = dd;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (t < w) red[0][t] += red[0][t + w];
    __syncthreads();
  }
  if (t == 0) change[blockIdx.x] = sqrt(red[0][0]);
}

// G[k] (b x b) = the symmetrised message k as a D x D matrix, padded (for
// b = D + 1) by a decoupled row and column with a large negative diagonal.
__global__ void bp_pad_kernel(const double* __restrict__ msg, int D, int b,
                              double* __restrict__ G, int count) {
  const long total = (long)count * b * b;
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < total;
       e += (long)gridDim.x * blockDim.x) {
    const int k = (int)(e / (b * b)), r = (int)(e / b % b), c = (int)(e % b);
    double v = 0.0;
    if (r < D && c < D) {
      const double* m = msg + (long)k * D * D;
      v = 0.5 * (m[r * D + c] + m[c * D + r]);
    } else if (r == c) {
      v = -1e30;
    }
    G[e] = v;
  }
}

// Copy the leading D x D block of each b x b eigenvector matrix and the
// first D eigenvalues.
__global__ void bp_crop_kernel(const double* __restrict__ Vb,
                               const double* __restrict__ lb, int D, int b,
                               double* __restrict__ V, double* __restrict__ l,
                               int count) {
  const long total = (long)count * D * D;
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < total;
       e += (long)gridDim.x * blockDim.x) {
    const int k = (int)(e / (D * D)), r = (int)(e / D % D), c = (int)(e % D);
    V[e] = Vb[(long)k * b * b + (long)r * b + c];
    if (r == 0) l[(long)k * D + c] = lb[(long)k * b + c];
  }
}

// out[t][i][j][k][l] = x[...] * w, w = lam0[i] lam1[j] lam2[k] lam3[l]
// (mode 0), or x[...] / (w * zs[0] + delta) (mode 1; zs[0] = 1 / Z).
__global__ void bp_kron_scale_kernel(const double* __restrict__ x,
                                     double* __restrict__ out, int d, int D,
                                     const double* __restrict__ lam,
                                     const double* __restrict__ zs,
                                     double delta, int mode) {
  const long D4 = (long)D * D * D * D, total = (long)d * D4;
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < total;
       e += (long)gridDim.x * blockDim.x) {
    const long r = e % D4;
    const int i = (int)(r / ((long)D * D * D)), j = (int)(r / (D * D) % D),
              k = (int)(r / D % D), l = (int)(r % D);
    const double w = lam[i] * lam[D + j] * lam[2 * D + k] * lam[3 * D + l];
    out[e] = mode == 0 ? x[e] * w : x[e] / (w * zs[0] + delta);
  }
}

int grid1(long n) { return (int)std::max<long>(1, std::min<long>((n + 255) / 256, 4096)); }

constexpr int LEG_DX[4] = {-1, 0, 1, 0};  // neighbour across l, u, r, d
constexpr int LEG_DY[4] = {0, -1, 0, 1};

// x_out = (V_0^(T) (x) V_1^(T) (x) V_2^(T) (x) V_3^(T)) x on the four
// virtual legs of x[t][l][u][r][d] (transposed factors when `fwd`, i.e. the
// rotation into the eigenbasis); V: [4][D][D] row major.
void mode_products(Device& dev, int d, int D, const double* V,
                   const double* x, double* tmp, double* out, bool fwd) {
  PrecScope f64(dev, PREC_FP64);
  const int64_t D2 = (int64_t)D * D, D3 = D2 * D;
  const double* V0 = V;
  const double* V1 = V + D2;
  const double* V2 = V + 2 * D2;
  const double* V3 = V + 3 * D2;
  // leg l: x as [t][l][(u r d)]: y[t] = op(V0) x[t]
  gemm(dev, fwd, false, D, D3, D, 1.0, V0, D, 0, x, D3, D * D3, 0.0, tmp, D3,
       D * D3, d);
  // leg u: [(t l)][u][(r d)]
  gemm(dev, fwd, false, D, D2, D, 1.0, V1, D, 0, tmp, D2, D3, 0.0, out, D2,
       D3, (int64_t)d * D);
  // leg r: [(t l u)][r][d]
  gemm(dev, fwd, false, D, D, D, 1.0, V2, D, 0, out, D, D2, 0.0, tmp, D, D2,
       (int64_t)d * D2);
  // leg d: [(t l u r)][d] times V3 (rotation in: x V3; back: x V3^T)
  gemm(dev, false, !fwd, (int64_t)d * D3, D, D, 1.0, tmp, D, 0, V3, D, 0,
       0.0, out, D, 0, 1);
}

}  // namespace

int bp_converge(Context& cx, double tol, int max_iter, int* n_iter,
                double* change) {
  Device& dev = cx.dev;
  PrecScope f64(dev, PREC_FP64);
  const int ns = cx.nsite(), D = cx.D, D2 = cx.D2;
  const int nm = 4 * ns;
  if (cx.bp_msg.numel() != (int64_t)nm * D2) {
    cx.bp_msg = dev.empty({nm, D2});
    std::vector<double> h((size_t)nm * D2, 0.0);
    const double v = 1.0 / std::sqrt((double)D);
    for (int m = 0; m < nm; ++m)
      for (int k = 0; k < D; ++k) h[(size_t)m * D2 + k * D + k] = v;
    dev.upload(cx.bp_msg, h.data());
  }
  Tensor nw = dev.empty({nm, D2});
  Tensor ch = dev.empty({nm});
  std::vector<double> hch(nm);
  int it = 0;
  double worst = INFINITY;
  // a_0[l][u][r][d] of a site: the unrotated double layer
  const int64_t a4 = (int64_t)D2 * D2 * D2 * D2;
  Tensor t3 = dev.empty({(int64_t)D2 * D2 * D2});
  Tensor t2 = dev.empty({(int64_t)D2 * D2});
  while (it < max_iter) {
    for (int s = 0; s < ns; ++s)
      for (int L = 0; L < 4; ++L) {
        // message into leg L of s: the neighbour's double layer with the
        // messages into its legs other than the opposite one
        const int nb = cx.lat.shift(s, LEG_DX[L], LEG_DY[L]);
        const int out = (L + 2) % 4;
        const double* a = cx.a_rot.ptr + (int64_t)nb * 4 * a4;  // a_0
        auto msg = [&](int leg) {
          return cx.bp_msg.ptr + ((int64_t)nb * 4 + leg) * D2;
        };
        // contract the legs in the order l, u, r, d (skipping `out`) one
        // GEMV at a time: a viewed as [leg][rest] or [rest][leg]
        int rank = 4;
        const double* cur = a;
        double* bufs[2] = {t3.ptr, t2.ptr};
        int bi = 0;
        // position of each remaining leg in cur
        std::vector<int> legs = {0, 1, 2, 3};
        for (int leg = 0; leg < 4; ++leg) {
          if (leg == out) continue;
          const int pos = (int)(std::find(legs.begin(), legs.end(), leg) -
                                legs.begin());
          int64_t before = 1, after = 1;
          for (int q = 0; q < pos; ++q) before *= D2;
          for (int q = pos + 1; q < rank; ++q) after *= D2;
          double* dst = (rank == 2) ? nw.ptr + ((int64_t)s * 4 + L) * D2
                                    : bufs[bi];
          // dst[b][a] = sum_k cur[b][k][a] m[k]
          gemm(dev, true, false, after, 1, D2, 1.0, cur, after, D2 * after,
               msg(leg), 1, 0, 0.0, dst, 1, after, before);
          cur = dst;
          bi ^= 1;
          legs.erase(legs.begin() + pos);
          --rank;
        }
      }
    hipLaunchKernelGGL(bp_finish_kernel, dim3(nm), dim3(256), 0, dev.stream,
                       nw.ptr, cx.bp_msg.ptr, D2, D, ch.ptr);
    IPEPS_HIP(hipGetLastError());
    std::swap(cx.bp_msg, nw);
    dev.download(ch, hch.data());
    worst = *std::max_element(hch.begin(), hch.end());
    ++it;
    if (worst < tol) break;
  }
  cx.bp_valid = true;
  if (n_iter) *n_iter = it;
  if (change) *change = worst;
  return worst < tol ? 0 : 1;
}

int precondition_bp(Context& cx, const double* g_in, double delta,
                    double* x_out, bool on_device) {
  Device& dev = cx.dev;
  PrecScope f64(dev, PREC_FP64);
  const int ns = cx.nsite(), d = cx.d, D = cx.D, D2 = cx.D2;
  const int b = D + (D % 2);
  const int64_t m = (int64_t)d * D2 * D2;
  Tensor g = dev.empty({ns, m}), x = dev.empty({ns, m});
  if (on_device)
    axpby(dev, ns * m, 1.0, g_in, 0.0, g.ptr);
  else
    dev.upload(g, g_in);
  Tensor G = dev.empty({4, b, b}), Vb = dev.empty({4, b, b}),
         lb = dev.empty({4, b});
  Tensor V = dev.empty({4, D, D}), lam = dev.empty({4, D});
  Tensor u = dev.empty({m}), w = dev.empty({m}), tmp = dev.empty({m});
  Tensor zs = dev.empty({2});
  for (int s = 0; s < ns; ++s) {
    const double* msg = cx.bp_msg.ptr + (int64_t)s * 4 * D2;
    hipLaunchKernelGGL(bp_pad_kernel, dim3(grid1(4L * b * b)), dim3(256), 0,
                       dev.stream, msg, D, b, G.ptr, 4);
    IPEPS_HIP(hipGetLastError());
    sym_eig_jacobi(dev, G.ptr, Vb.ptr, lb.ptr, b, 4);
    hipLaunchKernelGGL(bp_crop_kernel, dim3(grid1(4L * D * D)), dim3(256), 0,
                       dev.stream, Vb.ptr, lb.ptr, D, b, V.ptr, lam.ptr, 4);
    IPEPS_HIP(hipGetLastError());
    // Z = <A~, Lambda A~> with A~ the site tensor in the eigenbasis
    const double* As = cx.A.ptr + (int64_t)s * m;
    mode_products(dev, d, D, V.ptr, As, tmp.ptr, u.ptr, true);
    hipLaunchKernelGGL(bp_kron_scale_kernel, dim3(grid1(m)), dim3(256), 0,
                       dev.stream, u.ptr, w.ptr, d, D, lam.ptr, zs.ptr, 0.0,
                       0);
    IPEPS_HIP(hipGetLastError());
    dot(dev, u.ptr, w.ptr, m, zs.ptr + 1);
    double hz[2];
    dev.download(zs, hz);
    const double zh[2] = {1.0 / hz[1], hz[1]};
    dev.upload(zs, zh);
    // x = V (Lambda / Z + delta)^-1 V^T g
    mode_products(dev, d, D, V.ptr, g.ptr + s * m, tmp.ptr, u.ptr, true);
    hipLaunchKernelGGL(bp_kron_scale_kernel, dim3(grid1(m)), dim3(256), 0,
                       dev.stream, u.ptr, w.ptr, d, D, lam.ptr, zs.ptr, delta,
                       1);
    IPEPS_HIP(hipGetLastError());
    mode_products(dev, d, D, V.ptr, w.ptr, tmp.ptr, x.ptr + s * m, false);
  }
  if (on_device) {
    axpby(dev, ns * m, 1.0, x.ptr, 0.0, x_out);
    dev.sync();
  } else {
    dev.download(x, x_out);
  }
  return 0;
}

}  // namespace ipeps
