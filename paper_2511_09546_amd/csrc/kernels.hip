// Hand-written gfx950 kernels of the iPEPS library (FP64 path).
//
//  (the FP64 matrix-core GEMM is in gemm.hip)
//  * permute: generic rank <= 8 transpose, coalesced writes.
//  * deterministic two-stage FP64 reductions (dot, 2-norm).
//  * sym_eig_jacobi: batched parallel cyclic Jacobi eigensolver, one
//    workgroup per matrix, the matrix resident in LDS.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <map>
#include <mutex>

#include "engine.hpp"

namespace ipeps {

typedef double f64x4 __attribute__((ext_vector_type(4)));

// --------------------------------------------------------------- permute
// Division by the output extents through a multiply-high (Granlund and
// Montgomery's round-up method): for an extent e >= 2, l = ceil(log2 e),
// mul = ceil(2^(31+l) / e) < 2^32 and q = floor(x mul / 2^(31+l)) equals
// floor(x / e) for every 0 <= x < 2^31 (the rounding of mul adds less than
// x / 2^(31+l) < 1/e, which cannot carry past the next integer).
struct PermArgs {
  int rank;
  int out_shape[12];
  int in_stride[12];      // input stride along output dimension i
  unsigned mul[12];       // division by out_shape[i]: see above
  int shr[12];            // l - 1
};

__global__ void permute_kernel(const double* __restrict__ in,
                               double* __restrict__ out, int n, PermArgs p,
                               double alpha, double beta) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += gridDim.x * blockDim.x) {
    int rem = i, off = 0;
    for (int d = p.rank - 1; d >= 0; --d) {
      const int e = p.out_shape[d];
      const int q =
          e == 1 ? rem : (int)(__umulhi((unsigned)rem, p.mul[d]) >> p.shr[d]);
      off += (rem - q * e) * p.in_stride[d];
      rem = q;
    }
    double v = alpha * in[off];
    if (beta != 0.0) v += beta * out[i];
    out[i] = v;
  }
}

static int grid_for(int64_t n, int block) {
  int64_t g = (n + block - 1) / block;
  return (int)std::max<int64_t>(1, std::min<int64_t>(g, 8192));
}

// Tiled permute for the case where the output's innermost dimension is not
// the input's: a TQ x TL tile over (q = the output dimension that is
// innermost in the input, l = the innermost output dimension) goes through
// LDS, so that reads run along q and writes along l, both coalesced.  TQ is
// the extent of q itself when that is at most 96 (the bond dimensions D^2
// and chi here: no lanes wasted on a partial tile), else 64, and
// TL = min(2048 / TQ, 256), except that an output row of at most 48 (with
// q longer than 96) is one tile wide, TL = l and TQ = min(2048 / TL, 256);
// the 256 threads cover 256 / TQ rows of the tile per pass when reading
// and 256 / TL when writing.  The remaining output
// dimensions enumerate tiles in blockIdx.y (grid-stride, div/mod once per
// tile).
constexpr int PERM_TILE = 2048;  // elements of one tile
struct TileArgs {
  int rank;            // remaining dimensions
  int shape[12];
  long in_stride[12];
  long out_stride[12];
  int nq, nl;          // extents of q and l
  long sq_out;         // output stride of q (input stride of q is 1)
  long sl_in;          // input stride of l (output stride of l is 1)
  int bq, bl;          // tile extents TQ, TL
  int tq, tl;          // tiles along q and l
};

__global__ __launch_bounds__(256) void permute_tiled_kernel(
    const double* __restrict__ in, double* __restrict__ out, TileArgs a,
    int nrest, double alpha, double beta) {
  __shared__ double tile[PERM_TILE + 256];  // [TL][TQ + 1]
  const int TQ = a.bq, TL = a.bl, SQ = TQ + 1;
  const int q0 = (blockIdx.x / a.tl) * TQ, l0 = (blockIdx.x % a.tl) * TL;
  const int tid = threadIdx.x;
  // reading: this thread's q and first l row; writing: its l and first q
  const int rq = tid % TQ, rl0 = tid / TQ, rstep = 256 / TQ;
  const int wl = tid % TL, wq0 = tid / TL, wstep = 256 / TL;
  const bool rin = rl0 < rstep && q0 + rq < a.nq;
  const bool win = wq0 < wstep && l0 + wl < a.nl;
  for (int r0 = blockIdx.y; r0 < nrest; r0 += gridDim.y) {
    int rest = r0;  // below 2^31: the tensor has fewer elements
    long oin = 0, oout = 0;
    for (int d = a.rank - 1; d >= 0; --d) {
      const int q = rest / a.shape[d];
      const int i = rest - q * a.shape[d];
      oin += i * a.in_stride[d];
      oout += i * a.out_stride[d];
      rest = q;
    }
    if (rin) {
      const double* src = in + oin + q0 + rq;
      for (int ll = rl0; ll < TL && l0 + ll < a.nl; ll += rstep)
        tile[ll * SQ + rq] = src[(long)(l0 + ll) * a.sl_in];
    }
    __syncthreads();
    if (win) {
      double* dst = out + oout + l0 + wl;
      for (int qq = wq0; qq < TQ && q0 + qq < a.nq; qq += wstep) {
        double* o = dst + (long)(q0 + qq) * a.sq_out;
        double v = alpha * tile[wl * SQ + qq];
        if (beta != 0.0) v += beta * *o;
        *o = v;
      }
    }
    __syncthreads();
  }
}

void permute(Device& dev, const Tensor& in, const std::vector<int>& perm,
             Tensor& out, double alpha, double beta) {
  const int r = in.rank();
  if ((int)perm.size() != r || out.rank() != r)
    throw ArgError("permute: rank mismatch");
  // fold: drop size-1 dims and merge output dims that are contiguous in the
  // input
  std::vector<int64_t> istride(r);
  int64_t s = 1;
  for (int d = r - 1; d >= 0; --d) {
    istride[d] = s;
    s *= in.shape[d];
  }
  std::vector<int64_t> oshape, ostr;
  for (int i = 0; i < r; ++i) {
    if (out.shape[i] != in.shape[perm[i]])
      throw ArgError("permute: shape mismatch");
    if (in.shape[perm[i]] == 1) continue;
    const int64_t st = istride[perm[i]];
    if (!oshape.empty() && ostr.back() == st * in.shape[perm[i]]) {
      oshape.back() *= in.shape[perm[i]];
      ostr.back() = st;
    } else {
      oshape.push_back(in.shape[perm[i]]);
      ostr.push_back(st);
    }
  }
  const int64_t n = in.numel();
  if (n == 0) return;
  if (n >= (1LL << 31)) throw ArgError("permute: tensor too large");
  if (oshape.size() == 1 && ostr[0] == 1) {
    // contiguous: plain copy/axpby
    axpby(dev, n, alpha, in.ptr, beta, out.ptr);
    return;
  }
  if (oshape.empty()) {
    axpby(dev, n, alpha, in.ptr, beta, out.ptr);
    return;
  }
  if (oshape.size() > 12) throw ArgError("permute: rank > 12");
  // output dimension that is innermost in the input
  int qd = -1;
  for (int i = 0; i < (int)oshape.size(); ++i)
    if (ostr[i] == 1) qd = i;
  const int ld = (int)oshape.size() - 1;
  if (qd >= 0 && qd != ld && oshape[qd] >= 4 && oshape[ld] >= 4) {
    TileArgs a{};
    std::vector<int64_t> ostride(oshape.size());
    int64_t st = 1;
    for (int i = ld; i >= 0; --i) {
      ostride[i] = st;
      st *= oshape[i];
    }
    a.nq = (int)oshape[qd];
    a.nl = (int)oshape[ld];
    a.sq_out = ostride[qd];
    a.sl_in = ostr[ld];
    if (a.nq > 96 && a.nl <= 48) {
      // a short output row (D^2 = 36): one tile spans it, TQ = 2048 / TL
      a.bl = a.nl;
      a.bq = std::min(PERM_TILE / a.nl, 256);
    } else {
      a.bq = a.nq <= 96 ? a.nq : 64;
      a.bl = std::min(PERM_TILE / a.bq, 256);
    }
    a.tq = (a.nq + a.bq - 1) / a.bq;
    a.tl = (a.nl + a.bl - 1) / a.bl;
    int64_t nrest = 1;
    for (int i = 0; i < ld; ++i) {
      if (i == qd) continue;
      a.shape[a.rank] = (int)oshape[i];
      a.in_stride[a.rank] = ostr[i];
      a.out_stride[a.rank] = ostride[i];
      ++a.rank;
      nrest *= oshape[i];
    }
    if (dev.prof.on)
      dev.prof.begin(dev.stream, PROF_PERMUTE, 0.0,
                     8.0 * n * (beta != 0.0 ? 3 : 2));
    hipLaunchKernelGGL(permute_tiled_kernel,
                       dim3(a.tq * a.tl, (int)std::min<int64_t>(nrest, 65535)),
                       dim3(256), 0, dev.stream, in.ptr, out.ptr, a,
                       (int)nrest, alpha, beta);
    if (dev.prof.on) dev.prof.end(dev.stream);
    IPEPS_HIP(hipGetLastError());
    return;
  }
  PermArgs p{};
  p.rank = (int)oshape.size();
  for (int i = 0; i < p.rank; ++i) {
    p.out_shape[i] = (int)oshape[i];
    p.in_stride[i] = (int)ostr[i];
    const uint64_t e = (uint64_t)oshape[i];
    int l = 0;
    while ((1ull << l) < e) ++l;  // ceil(log2 e)
    if (e >= 2) {
      p.mul[i] = (unsigned)(((1ull << (31 + l)) + e - 1) / e);
      p.shr[i] = l - 1;
    }
  }
  if (dev.prof.on)
    dev.prof.begin(dev.stream, PROF_PERMUTE, 0.0,
                   8.0 * n * (beta != 0.0 ? 3 : 2));
  hipLaunchKernelGGL(permute_kernel, dim3(grid_for(n, 256)), dim3(256), 0,
                     dev.stream, in.ptr, out.ptr, (int)n, p, alpha, beta);
  if (dev.prof.on) dev.prof.end(dev.stream);
  IPEPS_HIP(hipGetLastError());
}

Tensor permuted(Device& dev, const Tensor& in, const std::vector<int>& perm) {
  std::vector<int64_t> sh(perm.size());
  for (size_t i = 0; i < perm.size(); ++i) sh[i] = in.shape[perm[i]];
  Tensor out = dev.empty(sh);
  permute(dev, in, perm, out);
  return out;
}

// ------------------------------------------------------------ elementwise
__global__ void fill_kernel(double* x, int64_t n, double v) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    x[i] = v;
}

void fill(Device& dev, double* x, int64_t n, double v) {
  if (n <= 0) return;
  hipLaunchKernelGGL(fill_kernel, dim3(grid_for(n, 256)), dim3(256), 0,
                     dev.stream, x, n, v);
  IPEPS_HIP(hipGetLastError());
}

__global__ void axpby_kernel(int64_t n, double a, const double* x, double b,
                             double* y) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    double v = a * x[i];
    if (b != 0.0) v += b * y[i];
    y[i] = v;
  }
}

void axpby(Device& dev, int64_t n, double a, const double* x, double b,
           double* y) {
  if (n <= 0) return;
  hipLaunchKernelGGL(axpby_kernel, dim3(grid_for(n, 256)), dim3(256), 0,
                     dev.stream, n, a, x, b, y);
  IPEPS_HIP(hipGetLastError());
}

__global__ void to_f32_kernel(const double* x, float* y, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    y[i] = (float)x[i];
}

void to_f32(Device& dev, const double* x, float* y, int64_t n) {
  if (n <= 0) return;
  hipLaunchKernelGGL(to_f32_kernel, dim3(grid_for(n, 256)), dim3(256), 0,
                     dev.stream, x, y, n);
  IPEPS_HIP(hipGetLastError());
}

__global__ void to_f64_kernel(const float* x, double* y, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    y[i] = (double)x[i];
}

void to_f64(Device& dev, const float* x, double* y, int64_t n) {
  if (n <= 0) return;
  hipLaunchKernelGGL(to_f64_kernel, dim3(grid_for(n, 256)), dim3(256), 0,
                     dev.stream, x, y, n);
  IPEPS_HIP(hipGetLastError());
}

// dst (cols x rows) = src^T (rows x cols), row major, 32 x 32 tiles staged
// through LDS (row stride 33) so that reads and writes are both coalesced.
template <typename T>
__global__ __launch_bounds__(256) void transpose_kernel(
    const T* __restrict__ src, T* __restrict__ dst, int64_t rows,
    int64_t cols) {
  __shared__ T tile[32][33];
  const int64_t r0 = (int64_t)blockIdx.y * 32, c0 = (int64_t)blockIdx.x * 32;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;  // ty < 8
  for (int i = ty; i < 32; i += 8) {
    const int64_t r = r0 + i, c = c0 + tx;
    if (r < rows && c < cols) tile[i][tx] = src[r * cols + c];
  }
  __syncthreads();
  for (int i = ty; i < 32; i += 8) {
    const int64_t c = c0 + i, r = r0 + tx;
    if (c < cols && r < rows) dst[c * rows + r] = tile[tx][i];
  }
}

template <typename T>
static void transpose_t(Device& dev, const T* src, T* dst, int64_t rows,
                        int64_t cols) {
  if (rows <= 0 || cols <= 0) return;
  if ((rows + 31) / 32 > 65535) throw ArgError("transpose: too many rows");
  hipLaunchKernelGGL(transpose_kernel<T>,
                     dim3((unsigned)((cols + 31) / 32),
                          (unsigned)((rows + 31) / 32)),
                     dim3(256), 0, dev.stream, src, dst, rows, cols);
  IPEPS_HIP(hipGetLastError());
}

void transpose(Device& dev, const double* src, double* dst, int64_t rows,
               int64_t cols) {
  transpose_t(dev, src, dst, rows, cols);
}

void transpose(Device& dev, const float* src, float* dst, int64_t rows,
               int64_t cols) {
  transpose_t(dev, src, dst, rows, cols);
}

__global__ void scale_dev_kernel(double* x, int64_t n, const double* s,
                                 int inverse) {
  const double f = inverse ? 1.0 / s[0] : s[0];
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    x[i] *= f;
}

void scale_dev(Device& dev, double* x, int64_t n, const double* s,
               bool inverse) {
  if (n <= 0) return;
  hipLaunchKernelGGL(scale_dev_kernel, dim3(grid_for(n, 256)), dim3(256), 0,
                     dev.stream, x, n, s, (int)inverse);
  IPEPS_HIP(hipGetLastError());
}

// ------------------------------------------------------------- reductions
// Stage 1: each of G blocks reduces a strided range; stage 2 adds the G
// partials in a fixed order.  Bitwise deterministic for a fixed n.
constexpr int RED_BLOCK = 256;
constexpr int RED_GRID = 256;

__device__ inline double block_sum(double v, double* sh) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  if (lane == 0) sh[w] = v;
  __syncthreads();
  double t = 0.0;
  if (threadIdx.x == 0)
    for (int i = 0; i < (int)(blockDim.x >> 6); ++i) t += sh[i];
  __syncthreads();
  return t;
}

__global__ __launch_bounds__(RED_BLOCK) void dot_partial_kernel(
    const double* __restrict__ x, const double* __restrict__ y, int64_t n,
    double* __restrict__ part) {
  __shared__ double sh[RED_BLOCK / 64];
  double v = 0.0;
  for (int64_t i = blockIdx.x * (int64_t)RED_BLOCK + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * RED_BLOCK)
    v += x[i] * y[i];
  v = block_sum(v, sh);
  if (threadIdx.x == 0) part[blockIdx.x] = v;
}

__global__ __launch_bounds__(RED_BLOCK) void final_sum_kernel(
    const double* __restrict__ part, int np, double* out, int take_sqrt) {
  __shared__ double sh[RED_BLOCK / 64];
  double v = 0.0;
  for (int i = threadIdx.x; i < np; i += RED_BLOCK) v += part[i];
  v = block_sum(v, sh);
  if (threadIdx.x == 0) out[0] = take_sqrt ? sqrt(v) : v;
}

static void reduce_dot(Device& dev, const double* x, const double* y,
                       int64_t n, double* out, int take_sqrt) {
  Tensor part = dev.empty({RED_GRID});
  const int g = (int)std::max<int64_t>(
      1, std::min<int64_t>(RED_GRID, (n + RED_BLOCK - 1) / RED_BLOCK));
  hipLaunchKernelGGL(dot_partial_kernel, dim3(g), dim3(RED_BLOCK), 0,
                     dev.stream, x, y, n, part.ptr);
  hipLaunchKernelGGL(final_sum_kernel, dim3(1), dim3(RED_BLOCK), 0,
                     dev.stream, part.ptr, g, out, take_sqrt);
  IPEPS_HIP(hipGetLastError());
}

void dot(Device& dev, const double* x, const double* y, int64_t n,
         double* out) {
  reduce_dot(dev, x, y, n, out, 0);
}

void nrm2(Device& dev, const double* x, int64_t n, double* out) {
  reduce_dot(dev, x, x, n, out, 1);
}

// ------------------------------------------------------- column utilities
__global__ void col_norms_kernel(const double* __restrict__ X, int64_t n,
                                 int b, double* __restrict__ out, long sX,
                                 long sOut) {
  // one wave per column; rows strided over 64 lanes
  const int bt = blockIdx.y;
  const int j = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (j >= b) return;
  const double* x = X + bt * sX;
  double v = 0.0;
  for (int64_t i = lane; i < n; i += 64) {
    const double t = x[i * b + j];
    v += t * t;
  }
  for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
  if (lane == 0) out[bt * sOut + j] = sqrt(v);
}

void col_norms(Device& dev, const double* X, int64_t n, int b, double* out,
               int batch, int64_t sX, int64_t sOut) {
  dim3 grid((b + 3) / 4, batch);
  hipLaunchKernelGGL(col_norms_kernel, grid, dim3(256), 0, dev.stream, X, n,
                     b, out, (long)sX, (long)sOut);
  IPEPS_HIP(hipGetLastError());
}

__global__ void col_scale_kernel(double* __restrict__ X, int64_t n, int b,
                                 const double* __restrict__ s, int mode,
                                 const int* __restrict__ keep, long sX,
                                 long sS) {
  const int bt = blockIdx.y;
  double* x = X + bt * sX;
  const double* ss = s + bt * sS;
  const int64_t total = n * b;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < total;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int j = (int)(i % b);
    const double v = ss[j];
    double f;
    if (mode == 0) {
      f = v != 0.0 ? 1.0 / v : 0.0;
    } else if (mode == 1) {
      const int k = keep ? keep[bt] : b;
      f = (j < k && v > 0.0) ? 1.0 / sqrt(v) : 0.0;
    } else {
      f = v;
    }
    x[i] *= f;
  }
}

void col_scale(Device& dev, double* X, int64_t n, int b, const double* s,
               int mode, const int* keep, int batch, int64_t sX,
               int64_t sS) {
  dim3 grid(grid_for(n * b, 256), batch);
  hipLaunchKernelGGL(col_scale_kernel, grid, dim3(256), 0, dev.stream, X, n,
                     b, s, mode, keep, (long)sX, (long)sS);
  IPEPS_HIP(hipGetLastError());
}

// Raises a kernel's dynamic LDS limit to at least `bytes` (once per kernel
// and size; the largest sizes are raised by prime_kernel_attributes before
// the first context exists, so that no attribute changes while other host
// threads launch kernels; contexts on several host threads may get here
// together).
static void allow_lds(const void* fn, size_t bytes) {
  static std::mutex mu;
  static std::map<const void*, size_t> done;
  std::lock_guard<std::mutex> lock(mu);
  size_t& have = done[fn];
  if (bytes <= have) return;
  IPEPS_HIP(hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize,
                                (int)bytes));
  have = bytes;
}

// ------------------------------------------------------- Jacobi eigensolver
// Parallel cyclic Jacobi (round-robin pairing, b-1 rounds of b/2 disjoint
// rotations per sweep).  The rotation of pair (p,q) annihilates G[p][q]
// (Golub & Van Loan, symmetric Schur 2x2): G_pq is set to zero and the two
// diagonal entries take their closed forms G_pp - t G_pq, G_qq + t G_pq, so
// no rounding noise re-creates the annihilated entry; a pair is skipped when
// |G_pq| <= tol sqrt|G_pp G_qq| (relative criterion, so small eigenvalues of
// graded matrices keep their relative accuracy).  Stops when no pair meets
// the criterion, which is tested before every sweep (or after 40 sweeps).
//
// One round is a single pass over the 2x2 blocks of G: with R_i the row
// combination of pair i, block (a, c) becomes R_a G_ac R_c^T, and the
// diagonal blocks take the closed forms above; blocks are disjoint, so a
// round needs one barrier after the rotation parameters and one after the
// update (each element of G and V is read and written once per round).
//
// Layout: G is symmetric and only its upper triangle is stored and updated
// (row stride b + 1), so a round touches the b/2 (b/2 + 1)/2 blocks with
// a <= c, half of the full matrix.  The eigenvector matrix is kept
// transposed, Vt[p][k] = V[k][p]: the rotation of pair (p, q) combines rows
// p and q of Vt, which consecutive lanes read at consecutive k (no LDS bank
// conflicts).  Vt lives in LDS when it fits next to G (b <= 96), else in the
// output buffer in global memory.  Every thread's blocks and (pair, k)
// items are fixed for the whole solve and are computed once, into
// registers.
constexpr int JAC_THREADS = 1024;
constexpr int JAC_MAXB = 128;
// most blocks and (pair, k) items of one thread at b = JAC_MAXB
constexpr int JAC_GBLK = (64 * 65 / 2 + JAC_THREADS - 1) / JAC_THREADS;  // 3
constexpr int JAC_VITEM = (64 * 128 + JAC_THREADS - 1) / JAC_THREADS;    // 8

size_t jacobi_lds_bytes(int b, bool vlds) {
  const size_t h = b / 2;
  size_t n = (size_t)b * (b + 1) * sizeof(double)  // G, upper triangle
             + h * 5 * sizeof(double)  // c, s, G_pp, G_qq, t G_pq
             + h * 2 * sizeof(int);    // p, q
  if (vlds) n += (size_t)b * b * sizeof(double);
  return n;
}

template <bool VLDS>
__global__ __launch_bounds__(JAC_THREADS) void sym_eig_jacobi_kernel(
    double* __restrict__ Gall, double* __restrict__ Vall,
    double* __restrict__ lamall, int b, double tol) {
  extern __shared__ double lds[];
  const int S = b + 1, h = b / 2;
  double* G = lds;        // b x S, entries p <= q
  double* cs = G + b * S;  // h: rotation cosines
  double* sn = cs + h;     // h: sines
  double* dp = sn + h;     // h: G_pp before the rotation
  double* dq = dp + h;     // h: G_qq
  double* tq = dq + h;     // h: t G_pq
  int* pp = (int*)(tq + h);  // h: pair (p, q), p < q
  int* qq = pp + h;
  __shared__ int rotated;
  const int bt = blockIdx.x;
  double* Gg = Gall + (long)bt * b * b;
  double* Vout = Vall + (long)bt * b * b;
  double* Vt = VLDS ? (double*)(qq + h) : Vout;  // 2h ints: 8-aligned
  double* lam = lamall + (long)bt * b;
  const int tid = threadIdx.x;
  for (int e = tid; e < b * b; e += JAC_THREADS) {
    const int p = e / b, q = e - p * b;
    if (p <= q) G[p * S + q] = Gg[e];
    Vt[e] = p == q ? 1.0 : 0.0;
  }
  // this thread's blocks (a, c), a <= c, enumerated row by row, and its
  // (pair, k) items of the Vt update, packed as a | c << 16
  const int nblk = h * (h + 1) / 2, nitem = h * b;
  int blk[JAC_GBLK], item[JAC_VITEM];
#pragma unroll
  for (int j = 0; j < JAC_GBLK; ++j) {
    const int t = tid + j * JAC_THREADS;
    int a = 0;
    if (t < nblk)
      while (t >= (a + 1) * h - (a + 1) * a / 2) ++a;
    const int c = a + t - (a * h - a * (a - 1) / 2);
    blk[j] = a | c << 16;
  }
  const float invb = 1.0f / (float)b;
#pragma unroll
  for (int j = 0; j < JAC_VITEM; ++j) {
    const int t = tid + j * JAC_THREADS;
    // t / b exactly: (t + 1/2)/b is at least 1/(2b) away from an integer
    const int i = (int)(((float)t + 0.5f) * invb);
    item[j] = i | (t - i * b) << 16;
  }
  auto gi = [S](int x, int y) { return x < y ? x * S + y : y * S + x; };
  __syncthreads();
  for (int sweep = 0; sweep < 40; ++sweep) {
    // a sweep rotates some pair iff some pair exceeds the criterion now (if
    // none does, the first round changes nothing and neither do the
    // others): test all pairs first instead of running a sweep to find out
    if (tid == 0) rotated = 0;
    __syncthreads();
    bool any = false;
    for (int e = tid; e < b * b; e += JAC_THREADS) {
      const int p = e / b, q = e - p * b;
      if (p < q) {
        const double apq = G[p * S + q];
        any |= apq != 0.0 &&
               fabs(apq) > tol * sqrt(fabs(G[p * S + p] * G[q * S + q]));
      }
    }
    if (any) rotated = 1;
    __syncthreads();
    if (!rotated) break;
    for (int r = 0; r < b - 1; ++r) {
      // pairs of this round, rotation parameters from the current G
      if (tid < h) {
        const int i = tid, j = b - 1 - i;
        int p = i == 0 ? 0 : 1 + (i - 1 + r) % (b - 1);
        int q = 1 + (j - 1 + r) % (b - 1);
        if (p > q) {
          const int t = p;
          p = q;
          q = t;
        }
        const double apq = G[p * S + q];
        const double app = G[p * S + p], aqq = G[q * S + q];
        double c = 1.0, s = 0.0, tg = 0.0;
        if (apq != 0.0 && fabs(apq) > tol * sqrt(fabs(app * aqq))) {
          const double tau = (aqq - app) / (2.0 * apq);
          const double t = (tau >= 0.0 ? 1.0 : -1.0) /
                           (fabs(tau) + sqrt(1.0 + tau * tau));
          c = 1.0 / sqrt(1.0 + t * t);
          s = t * c;
          tg = t * apq;
        }
        cs[i] = c;
        sn[i] = s;
        dp[i] = app;
        dq[i] = aqq;
        tq[i] = tg;
        pp[i] = p;
        qq[i] = q;
      }
      __syncthreads();
      // G <- R G R^T on the upper triangle, block by block
#pragma unroll
      for (int j = 0; j < JAC_GBLK; ++j) {
        if (tid + j * JAC_THREADS >= nblk) break;
        const int a = blk[j] & 0xffff, c = blk[j] >> 16;
        const double sa = sn[a];
        const int pa = pp[a], qa = qq[a];
        if (a == c) {
          if (sa != 0.0) {
            G[pa * S + qa] = 0.0;
            G[pa * S + pa] = dp[a] - tq[a];
            G[qa * S + qa] = dq[a] + tq[a];
          }
          continue;
        }
        const double sc = sn[c];
        if (sa == 0.0 && sc == 0.0) continue;
        const double ca = cs[a], cc = cs[c];
        const int pc = pp[c], qc = qq[c];
        const int i00 = gi(pa, pc), i01 = gi(pa, qc);
        const int i10 = gi(qa, pc), i11 = gi(qa, qc);
        const double g00 = G[i00], g01 = G[i01], g10 = G[i10], g11 = G[i11];
        // rows: (R_a G)
        const double h00 = ca * g00 - sa * g10, h01 = ca * g01 - sa * g11;
        const double h10 = sa * g00 + ca * g10, h11 = sa * g01 + ca * g11;
        // columns: (R_a G) R_c^T
        G[i00] = cc * h00 - sc * h01;
        G[i01] = sc * h00 + cc * h01;
        G[i10] = cc * h10 - sc * h11;
        G[i11] = sc * h10 + cc * h11;
      }
      // V <- V R^T: rows p, q of Vt
#pragma unroll
      for (int j = 0; j < JAC_VITEM; ++j) {
        if (tid + j * JAC_THREADS >= nitem) break;
        const int i = item[j] & 0xffff, k = item[j] >> 16;
        const double s = sn[i];
        if (s == 0.0) continue;
        const double c = cs[i];
        const int p = pp[i], q = qq[i];
        const double vp = Vt[p * b + k], vq = Vt[q * b + k];
        Vt[p * b + k] = c * vp - s * vq;
        Vt[q * b + k] = s * vp + c * vq;
      }
      __syncthreads();
    }
  }
  // sort by descending eigenvalue (stable rank of every diagonal entry);
  // pp/qq and cs/sn are contiguous, giving b ints and b doubles of LDS
  int* rk = pp;
  double* ev = cs;
  for (int i = tid; i < b; i += JAC_THREADS) {
    const double g = G[i * S + i];
    int rank = 0;
    for (int j = 0; j < b; ++j) {
      const double gj = G[j * S + j];
      rank += (gj > g) || (gj == g && j < i);
    }
    rk[i] = rank;
  }
  __syncthreads();
  for (int i = tid; i < b; i += JAC_THREADS) ev[rk[i]] = G[i * S + i];
  __syncthreads();
  // G is no longer needed: V[k][rk[i]] = Vt[i][k] staged through it
  for (int e = tid; e < b * b; e += JAC_THREADS) {
    const int i = e / b, k = e - i * b;
    G[k * b + rk[i]] = Vt[e];
  }
  __syncthreads();
  for (int e = tid; e < b * b; e += JAC_THREADS) {
    Vout[e] = G[e];
    Gg[e] = (e / b == e % b) ? ev[e / b] : 0.0;
  }
  for (int i = tid; i < b; i += JAC_THREADS) lam[i] = ev[i];
}

// The same parallel cyclic Jacobi for larger matrices (JAC_MAXB < b <=
// JAC_BIGB): G (upper triangle, row stride b + 1) and the transposed
// eigenvector matrix live in global memory (one workgroup per matrix, so
// both stay in its compute unit's cache and the barriers order every
// access); only the rotations of a round and the (a, c) block list are in
// LDS.  Same rotations, criterion, stopping rule and sort as
// sym_eig_jacobi_kernel.
constexpr int JACB_THREADS = 1024;
constexpr int JAC_BIGB = 512;

__global__ __launch_bounds__(JACB_THREADS) void sym_eig_jacobi_big_kernel(
    double* __restrict__ Gall, double* __restrict__ Vall,
    double* __restrict__ lamall, double* __restrict__ Wall, int b,
    double tol) {
  extern __shared__ double lds[];
  const int S = b + 1, h = b / 2;
  double* cs = lds;
  double* sn = cs + h;
  double* dp = sn + h;
  double* dq = dp + h;
  double* tq = dq + h;
  int* pp = (int*)(tq + h);
  int* qq = pp + h;
  int* blk = qq + h;  // h (h + 1) / 2 packed blocks a | c << 16
  __shared__ int rotated;
  const int bt = blockIdx.x;
  double* Gg = Gall + (long)bt * b * b;
  double* Vt = Vall + (long)bt * b * b;
  double* G = Wall + (long)bt * b * S;
  double* lam = lamall + (long)bt * b;
  const int tid = threadIdx.x;
  const int nblk = h * (h + 1) / 2, nitem = h * b;
  for (int e = tid; e < b * b; e += JACB_THREADS) {
    const int p = e / b, q = e - p * b;
    if (p <= q) G[p * S + q] = Gg[e];
    Vt[e] = p == q ? 1.0 : 0.0;
  }
  for (int a = tid; a < h; a += JACB_THREADS) {
    const int base = a * h - a * (a - 1) / 2;  // blocks of rows < a
    for (int c = a; c < h; ++c) blk[base + c - a] = a | c << 16;
  }
  auto gi = [S](int x, int y) { return x < y ? x * S + y : y * S + x; };
  __syncthreads();
  for (int sweep = 0; sweep < 40; ++sweep) {
    if (tid == 0) rotated = 0;
    __syncthreads();
    bool any = false;
    for (int e = tid; e < b * b; e += JACB_THREADS) {
      const int p = e / b, q = e - p * b;
      if (p < q) {
        const double apq = G[p * S + q];
        any |= apq != 0.0 &&
               fabs(apq) > tol * sqrt(fabs(G[p * S + p] * G[q * S + q]));
      }
    }
    if (any) rotated = 1;
    __syncthreads();
    if (!rotated) break;
    for (int r = 0; r < b - 1; ++r) {
      for (int i = tid; i < h; i += JACB_THREADS) {
        const int j = b - 1 - i;
        int p = i == 0 ? 0 : 1 + (i - 1 + r) % (b - 1);
        int q = 1 + (j - 1 + r) % (b - 1);
        if (p > q) {
          const int t = p;
          p = q;
          q = t;
        }
        const double apq = G[p * S + q];
        const double app = G[p * S + p], aqq = G[q * S + q];
        double c = 1.0, s = 0.0, tg = 0.0;
        if (apq != 0.0 && fabs(apq) > tol * sqrt(fabs(app * aqq))) {
          const double tau = (aqq - app) / (2.0 * apq);
          const double t = (tau >= 0.0 ? 1.0 : -1.0) /
                           (fabs(tau) + sqrt(1.0 + tau * tau));
          c = 1.0 / sqrt(1.0 + t * t);
          s = t * c;
          tg = t * apq;
        }
        cs[i] = c;
        sn[i] = s;
        dp[i] = app;
        dq[i] = aqq;
        tq[i] = tg;
        pp[i] = p;
        qq[i] = q;
      }
      __syncthreads();
      for (int t = tid; t < nblk; t += JACB_THREADS) {
        const int a = blk[t] & 0xffff, c = blk[t] >> 16;
        const double sa = sn[a];
        const int pa = pp[a], qa = qq[a];
        if (a == c) {
          if (sa != 0.0) {
            G[pa * S + qa] = 0.0;
            G[pa * S + pa] = dp[a] - tq[a];
            G[qa * S + qa] = dq[a] + tq[a];
          }
          continue;
        }
        const double sc = sn[c];
        if (sa == 0.0 && sc == 0.0) continue;
        const double ca = cs[a], cc = cs[c];
        const int pc = pp[c], qc = qq[c];
        const int i00 = gi(pa, pc), i01 = gi(pa, qc);
        const int i10 = gi(qa, pc), i11 = gi(qa, qc);
        const double g00 = G[i00], g01 = G[i01], g10 = G[i10], g11 = G[i11];
        const double h00 = ca * g00 - sa * g10, h01 = ca * g01 - sa * g11;
        const double h10 = sa * g00 + ca * g10, h11 = sa * g01 + ca * g11;
        G[i00] = cc * h00 - sc * h01;
        G[i01] = sc * h00 + cc * h01;
        G[i10] = cc * h10 - sc * h11;
        G[i11] = sc * h10 + cc * h11;
      }
      for (int t = tid; t < nitem; t += JACB_THREADS) {
        const int i = t / b, k = t - i * b;
        const double s = sn[i];
        if (s == 0.0) continue;
        const double c = cs[i];
        const int p = pp[i], q = qq[i];
        const double vp = Vt[p * b + k], vq = Vt[q * b + k];
        Vt[p * b + k] = c * vp - s * vq;
        Vt[q * b + k] = s * vp + c * vq;
      }
      __syncthreads();
    }
  }
  // sort by descending eigenvalue (stable rank of every diagonal entry)
  int* rk = pp;  // pp, qq: b ints
  double* ev = cs;  // cs, sn: b doubles
  for (int i = tid; i < b; i += JACB_THREADS) {
    const double g = G[i * S + i];
    int rank = 0;
    for (int j = 0; j < b; ++j) {
      const double gj = G[j * S + j];
      rank += (gj > g) || (gj == g && j < i);
    }
    rk[i] = rank;
  }
  __syncthreads();
  for (int i = tid; i < b; i += JACB_THREADS) ev[rk[i]] = G[i * S + i];
  __syncthreads();
  // G is no longer needed: V[k][rk[i]] = Vt[i][k] staged through it
  for (int e = tid; e < b * b; e += JACB_THREADS) {
    const int i = e / b, k = e - i * b;
    G[k * b + rk[i]] = Vt[e];
  }
  __syncthreads();
  for (int e = tid; e < b * b; e += JACB_THREADS) {
    Vt[e] = G[e];
    Gg[e] = (e / b == e % b) ? ev[e / b] : 0.0;
  }
  for (int i = tid; i < b; i += JACB_THREADS) lam[i] = ev[i];
}

void sym_eig_jacobi(Device& dev, double* G, double* V, double* lam, int b,
                    int batch, double tol) {
  if (b % 2 != 0 || b < 2 || b > JAC_BIGB)
    throw ArgError("sym_eig_jacobi: b must be even and <= 512");
  if (b > JAC_MAXB) {
    const int h = b / 2;
    const size_t lds = (size_t)h * 5 * sizeof(double) +
                       (size_t)h * 2 * sizeof(int) +
                       (size_t)h * (h + 1) / 2 * sizeof(int);
    allow_lds((const void*)sym_eig_jacobi_big_kernel, lds);
    Tensor w = dev.empty({batch, b, b + 1});
    if (dev.prof.on) dev.prof.begin(dev.stream, PROF_JACOBI, 0.0, 0.0);
    hipLaunchKernelGGL(sym_eig_jacobi_big_kernel, dim3(batch),
                       dim3(JACB_THREADS), lds, dev.stream, G, V, lam, w.ptr,
                       b, tol);
    if (dev.prof.on) dev.prof.end(dev.stream);
    IPEPS_HIP(hipGetLastError());
    return;
  }
  const bool vlds = b <= 96;
  const size_t lds = jacobi_lds_bytes(b, vlds);
  const void* fn = vlds ? (const void*)sym_eig_jacobi_kernel<true>
                        : (const void*)sym_eig_jacobi_kernel<false>;
  if (lds > 65536) allow_lds(fn, lds);
  if (dev.prof.on) dev.prof.begin(dev.stream, PROF_JACOBI, 0.0, 0.0);
  if (vlds)
    hipLaunchKernelGGL(sym_eig_jacobi_kernel<true>, dim3(batch),
                       dim3(JAC_THREADS), lds, dev.stream, G, V, lam, b, tol);
  else
    hipLaunchKernelGGL(sym_eig_jacobi_kernel<false>, dim3(batch),
                       dim3(JAC_THREADS), lds, dev.stream, G, V, lam, b, tol);
  if (dev.prof.on) dev.prof.end(dev.stream);
  IPEPS_HIP(hipGetLastError());
}

}  // namespace ipeps

namespace ipeps {

// Orthonormalising factor of a block with unit columns: from its Gram
// matrix G = Z^T Z (b x b, diagonal 1 or 0), the Cholesky factor G = L L^T
// and R = L^-T, so that Z R has orthonormal columns.  One workgroup per
// matrix, G in LDS.  A pivot below 1e-12 (a column that is zero or lies in
// the span of the earlier ones) drops that direction: its row and column of
// R are zero and Z R has a zero column there.  The inverse is formed by
// column-wise forward substitution into the free upper triangle of G.
// With glob (b > 128) the b x b work matrix is a global scratch block per
// matrix instead of LDS (one workgroup each, so the barriers order it).
__global__ __launch_bounds__(256) void chol_orth_kernel(
    const double* __restrict__ Gall, double* __restrict__ Rall, int b,
    double* __restrict__ glob) {
  extern __shared__ double lds[];
  // row stride b + 1 in LDS: a column (fixed k, consecutive rows), which
  // the trailing update and the triangular inverse read across the lanes,
  // then spreads over the banks instead of hitting one bank (stride b = 96
  // doubles is a multiple of the bank count)
  const int S = glob ? b : b + 1;
  double* G = glob ? glob + (long)blockIdx.x * b * b : lds;  // b*S
  double* dg = glob ? lds : G + b * S;  // b: pivots
  const int bt = blockIdx.x, tid = threadIdx.x, nt = blockDim.x;
  const double* Gg = Gall + (long)bt * b * b;
  double* R = Rall + (long)bt * b * b;
  for (int e = tid; e < b * b; e += nt) G[(e / b) * S + e % b] = Gg[e];
  __syncthreads();
  for (int k = 0; k < b; ++k) {
    if (tid == 0) {
      const double d = G[k * S + k];
      dg[k] = d > 1e-12 ? sqrt(d) : 0.0;
    }
    __syncthreads();
    const double p = dg[k];
    for (int i = k + 1 + tid; i < b; i += nt)
      G[i * S + k] = p > 0.0 ? G[i * S + k] / p : 0.0;
    __syncthreads();
    // trailing lower triangle: G[i][j] -= L[i][k] L[j][k], k < j <= i
    const int m = b - k - 1;
    for (int e = tid; e < m * m; e += nt) {
      const int i = k + 1 + e / m, j = k + 1 + e % m;
      if (j <= i) G[i * S + j] -= G[i * S + k] * G[j * S + k];
    }
    __syncthreads();
  }
  // Y = L^-1 by columns: thread j owns column j, stored transposed in the
  // upper triangle (Y[i][j] at G[j][i], i >= j; the diagonal slot is free
  // because the pivots live in dg)
  for (int j = tid; j < b; j += nt) {
    for (int i = j; i < b; ++i) {
      double acc = (i == j) ? 1.0 : 0.0;
      for (int k = j; k < i; ++k) acc -= G[i * S + k] * G[j * S + k];
      const double y = dg[i] > 0.0 ? acc / dg[i] : 0.0;
      G[j * S + i] = y;
    }
  }
  __syncthreads();
  // R = L^-T: R[j][i] = Y[i][j] for i >= j, else 0
  for (int e = tid; e < b * b; e += nt) {
    const int j = e / b, i = e % b;
    R[e] = i >= j ? G[j * S + i] : 0.0;
  }
}

void chol_orth_factor(Device& dev, const double* G, double* R, int b,
                      int batch) {
  if (b < 1 || b > 512) throw ArgError("chol_orth_factor: b must be <= 512");
  Tensor w;
  size_t lds = ((size_t)b * (b + 1) + b) * sizeof(double);
  if (b > 128) {
    w = dev.empty({batch, b, b});
    lds = (size_t)b * sizeof(double);
  }
  if (lds > 65536) allow_lds((const void*)chol_orth_kernel, lds);
  hipLaunchKernelGGL(chol_orth_kernel, dim3(batch), dim3(256), lds,
                     dev.stream, G, R, b, b > 128 ? w.ptr : nullptr);
  IPEPS_HIP(hipGetLastError());
}

// ------------------------------------------------------- SVD helper kernels
// Deterministic pseudo-random start block: splitmix64 of (seed, index)
// mapped to (-1, 1).
__global__ void random_block_kernel(double* X, int64_t n, uint64_t seed) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    uint64_t z = seed + 0x9E3779B97F4A7C15ull * (uint64_t)(i + 1);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    z ^= z >> 31;
    X[i] = (double)(z >> 11) * (2.0 / 9007199254740992.0) - 1.0;
  }
}

void random_block(Device& dev, double* X, int64_t n, uint64_t seed) {
  hipLaunchKernelGGL(random_block_kernel, dim3(grid_for(n, 256)), dim3(256),
                     0, dev.stream, X, n, seed);
  IPEPS_HIP(hipGetLastError());
}

// X (n x b, batched) = identity in the leading min(n, b) block.
__global__ void eye_kernel(double* X, int64_t n, int b, long sX) {
  double* x = X + blockIdx.y * sX;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
       i < n * b; i += (int64_t)gridDim.x * blockDim.x)
    x[i] = (i / b == i % b) ? 1.0 : 0.0;
}

void eye(Device& dev, double* X, int64_t n, int b, int batch, int64_t sX) {
  hipLaunchKernelGGL(eye_kernel, dim3(grid_for(n * b, 256), batch), dim3(256),
                     0, dev.stream, X, n, b, (long)sX);
  IPEPS_HIP(hipGetLastError());
}

// Sign convention: in every column u of U the entry r maximising
// |u_r| (1 + r/(2n)) (first one on ties) is made positive; the same column of
// V takes the same sign.  The weight separates the entries (k,k') and (k',k)
// that the ket-bra exchange symmetry of the double layer makes equal in
// magnitude.
__global__ void sign_fix_kernel(double* U, double* V, int64_t n, int b,
                                long sU, long sV) {
  const int bt = blockIdx.y;
  const int j = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (j >= b) return;
  double* u = U + bt * sU;
  double* v = V + bt * sV;
  double best = -1.0;
  int64_t bi = 0;
  for (int64_t i = lane; i < n; i += 64) {
    const double a = fabs(u[i * b + j]) * (1.0 + (double)i / (2.0 * (double)n));
    if (a > best) {
      best = a;
      bi = i;
    }
  }
  for (int o = 32; o > 0; o >>= 1) {
    const double ob = __shfl_down(best, o, 64);
    const int64_t oi = __shfl_down(bi, o, 64);
    if (ob > best || (ob == best && oi < bi)) {
      best = ob;
      bi = oi;
    }
  }
  bi = __shfl(bi, 0, 64);
  const double sg = u[bi * b + j] < 0.0 ? -1.0 : 1.0;
  if (sg < 0.0) {
    for (int64_t i = lane; i < n; i += 64) {
      u[i * b + j] = -u[i * b + j];
      v[i * b + j] = -v[i * b + j];
    }
  }
}

void sign_fix(Device& dev, double* U, double* V, int64_t n, int b, int batch,
              int64_t sU, int64_t sV) {
  dim3 grid((b + 3) / 4, batch);
  hipLaunchKernelGGL(sign_fix_kernel, grid, dim3(256), 0, dev.stream, U, V, n,
                     b, (long)sU, (long)sV);
  IPEPS_HIP(hipGetLastError());
}

// keep[bt] = min(chi, #{s_i > cut * s_0})
__global__ void kept_rank_kernel(const double* S, int b, int chi, double cut,
                                 int* keep, long sS) {
  const int bt = blockIdx.x;
  if (threadIdx.x != 0) return;
  const double* s = S + bt * sS;
  const double thr = cut * s[0];
  int k = 0;
  for (int i = 0; i < b; ++i) k += (s[i] > thr) ? 1 : 0;
  keep[bt] = k < chi ? k : chi;
}

void kept_rank(Device& dev, const double* S, int b, int chi, double cut,
               int* keep, int batch, int64_t sS) {
  hipLaunchKernelGGL(kept_rank_kernel, dim3(batch), dim3(64), 0, dev.stream,
                     S, b, chi, cut, keep, (long)sS);
  IPEPS_HIP(hipGetLastError());
}

// Residual of the top-k triplets: r[bt] = max_{i<k} ||Z_i - s_i V_i|| / s_0
// (Z = M^T U).  Stage 1 sweeps rows with coalesced reads (64 columns per
// workgroup, 32 row groups), stage 2 adds the partials per column in a fixed
// order and takes the maximum.
__global__ __launch_bounds__(256) void svd_residual_partial_kernel(
    const double* __restrict__ Z, const double* __restrict__ V,
    const double* __restrict__ S, int64_t n, int b, double* __restrict__ part,
    long sZ, long sS) {
  __shared__ double red[4][64];
  const int bt = blockIdx.z;
  const int c = blockIdx.x * 64 + (threadIdx.x & 63);
  const int r0 = threadIdx.x >> 6;
  const double* z = Z + bt * sZ;
  const double* v = V + bt * sZ;
  double acc = 0.0;
  if (c < b) {
    const double sc = S[bt * sS + c];
    for (int64_t i = blockIdx.y * 4 + r0; i < n; i += 4 * 32) {
      const double t = z[i * b + c] - sc * v[i * b + c];
      acc += t * t;
    }
  }
  red[r0][threadIdx.x & 63] = acc;
  __syncthreads();
  if (threadIdx.x < 64 && c < b)
    part[((long)bt * 32 + blockIdx.y) * b + c] =
        red[0][threadIdx.x] + red[1][threadIdx.x] + red[2][threadIdx.x] +
        red[3][threadIdx.x];
}

__global__ void svd_residual_final_kernel(const double* __restrict__ part,
                                          const double* __restrict__ S, int b,
                                          int k, double* r, long sS) {
  const int bt = blockIdx.x;
  __shared__ double red[128];
  double worst = 0.0;
  for (int c = threadIdx.x; c < k; c += blockDim.x) {
    double v = 0.0;
    for (int g = 0; g < 32; ++g) v += part[((long)bt * 32 + g) * b + c];
    worst = fmax(worst, sqrt(v));
  }
  red[threadIdx.x] = worst;
  __syncthreads();
  if (threadIdx.x == 0) {
    double w = 0.0;
    for (int i = 0; i < (int)blockDim.x; ++i) w = fmax(w, red[i]);
    const double s0 = S[bt * sS];
    r[bt] = s0 > 0.0 ? w / s0 : 0.0;
  }
}

void svd_residual(Device& dev, const double* Z, const double* V,
                  const double* S, int64_t n, int b, int k, double* r,
                  int batch, int64_t sZ, int64_t sS) {
  Tensor part = dev.empty({batch, 32, b});
  hipLaunchKernelGGL(svd_residual_partial_kernel,
                     dim3((b + 63) / 64, 32, batch), dim3(256), 0,
                     dev.stream, Z, V, S, n, b, part.ptr, (long)sZ,
                     (long)sS);
  hipLaunchKernelGGL(svd_residual_final_kernel, dim3(batch), dim3(128), 0,
                     dev.stream, part.ptr, S, b, k, r, (long)sS);
  IPEPS_HIP(hipGetLastError());
}

// Zero-padded 3-D copy: out[A][B][C] (pre-zeroed) <- in[a][b][c] in its
// leading corner.
__global__ void pad3_kernel(const double* in, double* out, int a, int b, int c,
                            int B, int C) {
  const int64_t n = (int64_t)a * b * c;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int k = (int)(i % c);
    const int j = (int)((i / c) % b);
    const int l = (int)(i / ((int64_t)b * c));
    out[((int64_t)l * B + j) * C + k] = in[i];
  }
}

void pad3(Device& dev, const double* in, double* out, int a, int b, int c,
          int B, int C) {
  const int64_t n = (int64_t)a * b * c;
  hipLaunchKernelGGL(pad3_kernel, dim3(grid_for(n, 256)), dim3(256), 0,
                     dev.stream, in, out, a, b, c, B, C);
  IPEPS_HIP(hipGetLastError());
}

__global__ void crop3_add_kernel(const double* gout, double* gin, int a,
                                 int b, int c, int B, int C) {
  const int64_t n = (int64_t)a * b * c;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int k = (int)(i % c);
    const int j = (int)((i / c) % b);
    const int l = (int)(i / ((int64_t)b * c));
    gin[i] += gout[((int64_t)l * B + j) * C + k];
  }
}

void crop3_add(Device& dev, const double* gout, double* gin, int a, int b,
               int c, int B, int C) {
  const int64_t n = (int64_t)a * b * c;
  if (n <= 0) return;
  hipLaunchKernelGGL(crop3_add_kernel, dim3(grid_for(n, 256)), dim3(256), 0,
                     dev.stream, gout, gin, a, b, c, B, C);
  IPEPS_HIP(hipGetLastError());
}

// Corner-spectrum change: spec[bt] (b values, sorted) normalised to sum 1
// into out (chi values, zero padded); delta[0] = max_bt ||out - old||_2 and
// old <- out.  One workgroup.
__global__ void spectra_update_kernel(const double* S, int b, int chi,
                                      int batch, long sS, double* cur,
                                      double* old, double* delta) {
  __shared__ double red[64];
  double worst = 0.0;
  for (int bt = 0; bt < batch; ++bt) {
    const double* s = S + bt * sS;
    double tot = 0.0;
    for (int i = threadIdx.x; i < b; i += blockDim.x) tot += s[i];
    for (int o = 32; o > 0; o >>= 1) tot += __shfl_down(tot, o, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = tot;
    __syncthreads();
    double sum = 0.0;
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) sum += red[w];
    __syncthreads();
    double acc = 0.0;
    for (int i = threadIdx.x; i < chi; i += blockDim.x) {
      const double v = (i < b && sum > 0.0) ? s[i] / sum : 0.0;
      const double dlt = v - old[bt * chi + i];
      acc += dlt * dlt;
      cur[bt * chi + i] = v;
      old[bt * chi + i] = v;
    }
    for (int o = 32; o > 0; o >>= 1) acc += __shfl_down(acc, o, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
    __syncthreads();
    double t = 0.0;
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) t += red[w];
    worst = fmax(worst, sqrt(t));
    __syncthreads();
  }
  if (threadIdx.x == 0) delta[0] = worst;
}

void spectra_update(Device& dev, const double* S, int b, int chi, int batch,
                    int64_t sS, double* cur, double* old, double* delta) {
  hipLaunchKernelGGL(spectra_update_kernel, dim3(1), dim3(256), 0, dev.stream,
                     S, b, chi, batch, (long)sS, cur, old, delta);
  IPEPS_HIP(hipGetLastError());
}

}  // namespace ipeps

namespace ipeps {

// ------------------------------------------------------------ term energy
// value = sum_{s,t} h[t][s] rho[s][t], tr = sum_s rho[s][s];
// acc[0] += coef * value / tr;
// rho_bar[s][t] = coef * (h[t][s] - (value/tr) delta_st) / tr  (cotangent of
// rho for the backward pass), if rho_bar != nullptr.  One workgroup.
__global__ void term_energy_kernel(const double* rho, const double* h, int m,
                                   double coef, double* acc,
                                   double* rho_bar) {
  __shared__ double red[2][64];
  double v = 0.0, tr = 0.0;
  for (int i = threadIdx.x; i < m * m; i += blockDim.x) {
    const int s = i / m, t = i % m;
    v += h[t * m + s] * rho[i];
    if (s == t) tr += rho[i];
  }
  for (int o = 32; o > 0; o >>= 1) {
    v += __shfl_down(v, o, 64);
    tr += __shfl_down(tr, o, 64);
  }
  if ((threadIdx.x & 63) == 0) {
    red[0][threadIdx.x >> 6] = v;
    red[1][threadIdx.x >> 6] = tr;
  }
  __syncthreads();
  double V = 0.0, TR = 0.0;
  for (int w = 0; w < (int)(blockDim.x >> 6); ++w) {
    V += red[0][w];
    TR += red[1][w];
  }
  const double e = V / TR;
  if (threadIdx.x == 0) acc[0] += coef * e;
  if (rho_bar)
    for (int i = threadIdx.x; i < m * m; i += blockDim.x) {
      const int s = i / m, t = i % m;
      rho_bar[i] = coef * (h[t * m + s] - (s == t ? e : 0.0)) / TR;
    }
}

void term_energy(Device& dev, const double* rho, const double* h, int m,
                 double coef, double* acc, double* rho_bar) {
  hipLaunchKernelGGL(term_energy_kernel, dim3(1), dim3(256), 0, dev.stream,
                     rho, h, m, coef, acc, rho_bar);
  IPEPS_HIP(hipGetLastError());
}

// Split-K partial tiles: C = alpha * sum_s part[s] + beta * C.
__global__ void splitk_reduce_kernel(const double* part, int S, int64_t M,
                                     int64_t N, double alpha, double beta,
                                     double* C, int64_t ldc) {
  const int64_t mn = M * N;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < mn;
       i += (int64_t)gridDim.x * blockDim.x) {
    double v = 0.0;
    for (int s = 0; s < S; ++s) v += part[s * mn + i];
    const int64_t r = i / N, c = i % N;
    double o = alpha * v;
    if (beta != 0.0) o += beta * C[r * ldc + c];
    C[r * ldc + c] = o;
  }
}

void splitk_reduce(Device& dev, const double* part, int S, int64_t M,
                   int64_t N, double alpha, double beta, double* C,
                   int64_t ldc) {
  hipLaunchKernelGGL(splitk_reduce_kernel, dim3(grid_for(M * N, 256)),
                     dim3(256), 0, dev.stream, part, S, M, N, alpha, beta, C,
                     ldc);
  IPEPS_HIP(hipGetLastError());
}

}  // namespace ipeps

namespace ipeps {

// ------------------------------------------------------------- CG updates
// All scalars live on the device; a step is skipped when p^T A p <= 0 so
// that the host sees the breakdown with x still holding the last iterate.
__global__ void cg_update_xr_kernel(int64_t n, const double* rr,
                                    const double* pAp, const double* p,
                                    const double* Ap, double* x, double* r) {
  if (!(pAp[0] > 0.0)) return;
  const double alpha = rr[0] / pAp[0];
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    x[i] += alpha * p[i];
    r[i] -= alpha * Ap[i];
  }
}

void cg_update_xr(Device& dev, int64_t n, const double* rr, const double* pAp,
                  const double* p, const double* Ap, double* x, double* r) {
  hipLaunchKernelGGL(cg_update_xr_kernel, dim3(grid_for(n, 256)), dim3(256),
                     0, dev.stream, n, rr, pAp, p, Ap, x, r);
  IPEPS_HIP(hipGetLastError());
}

__global__ void cg_update_p_kernel(int64_t n, const double* rr_new,
                                   const double* rr, const double* pAp,
                                   const double* r, double* p) {
  if (!(pAp[0] > 0.0)) return;
  const double beta = rr_new[0] / rr[0];
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    p[i] = r[i] + beta * p[i];
}

void cg_update_p(Device& dev, int64_t n, const double* rr_new,
                 const double* rr, const double* pAp, const double* r,
                 double* p) {
  hipLaunchKernelGGL(cg_update_p_kernel, dim3(grid_for(n, 256)), dim3(256),
                     0, dev.stream, n, rr_new, rr, pAp, r, p);
  IPEPS_HIP(hipGetLastError());
}

// y = y / s[0] + delta * x
__global__ void scale_add_dev_kernel(int64_t n, const double* s,
                                     const double* x, double delta,
                                     double* y) {
  const double f = 1.0 / s[0];
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    y[i] = y[i] * f + delta * x[i];
}

void scale_add_dev(Device& dev, int64_t n, const double* s, const double* x,
                   double delta, double* y) {
  hipLaunchKernelGGL(scale_add_dev_kernel, dim3(grid_for(n, 256)), dim3(256),
                     0, dev.stream, n, s, x, delta, y);
  IPEPS_HIP(hipGetLastError());
}

}  // namespace ipeps

namespace ipeps {

// s[bt][j] <- 0 where s[bt][j] <= rel * max_j s[bt][j] (numerical null
// columns of a tall-skinny SVD are set to exactly zero instead of being
// normalised into noise).  One workgroup per batch entry.
__global__ void null_threshold_kernel(double* S, int b, double rel, long sS) {
  double* s = S + blockIdx.x * sS;
  __shared__ double red[64];
  double m = 0.0;
  for (int j = threadIdx.x; j < b; j += blockDim.x) m = fmax(m, s[j]);
  for (int o = 32; o > 0; o >>= 1) m = fmax(m, __shfl_down(m, o, 64));
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = m;
  __syncthreads();
  double mx = 0.0;
  for (int w = 0; w < (int)(blockDim.x >> 6); ++w) mx = fmax(mx, red[w]);
  for (int j = threadIdx.x; j < b; j += blockDim.x)
    if (s[j] <= rel * mx) s[j] = 0.0;
}

void null_threshold(Device& dev, double* S, int b, double rel, int batch,
                    int64_t sS) {
  hipLaunchKernelGGL(null_threshold_kernel, dim3(batch), dim3(128), 0,
                     dev.stream, S, b, rel, (long)sS);
  IPEPS_HIP(hipGetLastError());
}

// Columns c of X (batch x n x b, row major) with cn[bt][c] == 0 are
// overwritten by deterministic pseudo-random values in (-1, 1) (splitmix64
// of the seed and the element's index, as random_block); the others are
// left alone.
__global__ void fill_null_cols_kernel(double* X, int64_t n, int b,
                                      const double* cn, uint64_t seed) {
  const int bt = blockIdx.y;
  const int64_t nb = n * b;
  double* x = X + bt * nb;
  const double* c = cn + (int64_t)bt * b;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < nb;
       i += (int64_t)gridDim.x * blockDim.x) {
    if (c[i % b] != 0.0) continue;
    uint64_t z = seed + 0x9E3779B97F4A7C15ull * (uint64_t)(bt * nb + i + 1);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    z ^= z >> 31;
    x[i] = (double)(z >> 11) * (2.0 / 9007199254740992.0) - 1.0;
  }
}

void fill_null_cols(Device& dev, double* X, int64_t n, int b,
                    const double* cn, int batch, uint64_t seed) {
  hipLaunchKernelGGL(fill_null_cols_kernel,
                     dim3(grid_for(n * b, 256), batch), dim3(256), 0,
                     dev.stream, X, n, b, cn, seed);
  IPEPS_HIP(hipGetLastError());
}

}  // namespace ipeps

#include "ad.hpp"

namespace ipeps {

__global__ void normalize_backward_kernel(int64_t n, const double* y,
                                          const double* ybar,
                                          const double* nrm, const double* d,
                                          double* xbar) {
  const double inv = 1.0 / nrm[0], dd = d[0];
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    xbar[i] += (ybar[i] - y[i] * dd) * inv;
}

// Batched normalisation of up to NB_MAX vectors of any lengths: one
// partial-sum launch over (chunk, item), then one launch that reduces the
// item's partials in a fixed order and applies the elementwise step
//   forward   y_i = x_i / |x_i|,  nrm_i = |x_i|;
//   backward  xbar_i += (ybar_i - y_i <y_i, ybar_i>) / nrm_i.
constexpr int NB_CHUNKS = 64;

__global__ __launch_bounds__(256) void batch_dot_partial_kernel(
    NormBatch p, double* __restrict__ part) {
  __shared__ double sh[4];
  const int i = blockIdx.y, c = blockIdx.x;
  const long n = p.n[i];
  const double* a = p.a[i];
  const double* b = p.b[i];
  double v = 0.0;
  for (long e = (long)c * 256 + threadIdx.x; e < n;
       e += (long)NB_CHUNKS * 256)
    v += a[e] * b[e];
  v = block_sum(v, sh);
  if (threadIdx.x == 0) part[i * NB_CHUNKS + c] = v;
}

__global__ __launch_bounds__(256) void batch_normalize_kernel(
    NormBatch p, const double* __restrict__ part, double* __restrict__ nrm) {
  __shared__ double s;
  const int i = blockIdx.y;
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int c = 0; c < NB_CHUNKS; ++c) t += part[i * NB_CHUNKS + c];
    s = sqrt(t);
    if (blockIdx.x == 0) nrm[i] = s;
  }
  __syncthreads();
  const double f = 1.0 / s;
  const long n = p.n[i];
  const double* x = p.a[i];
  double* y = p.out[i];
  for (long e = blockIdx.x * 256L + threadIdx.x; e < n;
       e += (long)gridDim.x * 256)
    y[e] = x[e] * f;
}

__global__ __launch_bounds__(256) void batch_normalize_backward_kernel(
    NormBatch p, const double* __restrict__ part) {
  __shared__ double d;
  const int i = blockIdx.y;
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int c = 0; c < NB_CHUNKS; ++c) t += part[i * NB_CHUNKS + c];
    d = t;
  }
  __syncthreads();
  const double inv = 1.0 / p.nrm[i][0], dd = d;
  const long n = p.n[i];
  const double* y = p.a[i];
  const double* ybar = p.b[i];
  double* xbar = p.out[i];
  for (long e = blockIdx.x * 256L + threadIdx.x; e < n;
       e += (long)gridDim.x * 256)
    xbar[e] += (ybar[e] - y[e] * dd) * inv;
}

static int batch_blocks(const NormBatch& p, int count) {
  long m = 1;
  for (int i = 0; i < count; ++i) m = std::max(m, (p.n[i] + 255) / 256);
  return (int)std::min<long>(m, 1024);
}

void normalize_batch(Device& dev, const NormBatch& p, int count,
                     double* nrm) {
  if (count <= 0) return;
  if (count > NB_MAX) throw ArgError("normalize_batch: too many items");
  Tensor part = dev.empty({(int64_t)count * NB_CHUNKS});
  NormBatch q = p;
  for (int i = 0; i < count; ++i) q.b[i] = q.a[i];
  hipLaunchKernelGGL(batch_dot_partial_kernel, dim3(NB_CHUNKS, count),
                     dim3(256), 0, dev.stream, q, part.ptr);
  hipLaunchKernelGGL(batch_normalize_kernel,
                     dim3(batch_blocks(p, count), count), dim3(256), 0,
                     dev.stream, q, part.ptr, nrm);
  IPEPS_HIP(hipGetLastError());
}

void normalize_backward_batch(Device& dev, const NormBatch& p, int count) {
  if (count <= 0) return;
  if (count > NB_MAX)
    throw ArgError("normalize_backward_batch: too many items");
  Tensor part = dev.empty({(int64_t)count * NB_CHUNKS});
  hipLaunchKernelGGL(batch_dot_partial_kernel, dim3(NB_CHUNKS, count),
                     dim3(256), 0, dev.stream, p, part.ptr);
  hipLaunchKernelGGL(batch_normalize_backward_kernel,
                     dim3(batch_blocks(p, count), count), dim3(256), 0,
                     dev.stream, p, part.ptr);
  IPEPS_HIP(hipGetLastError());
}

void normalize_backward(Device& dev, int64_t len, const double* y,
                        const double* ybar, const double* nrm, double* xbar) {
  Tensor d = dev.empty({1});
  dot(dev, y, ybar, len, d.ptr);
  hipLaunchKernelGGL(normalize_backward_kernel, dim3(grid_for(len, 256)),
                     dim3(256), 0, dev.stream, len, y, ybar, nrm, d.ptr, xbar);
  IPEPS_HIP(hipGetLastError());
}

}  // namespace ipeps

namespace ipeps {

// ---------------------------------------------- projector backward helpers
// out[j] = sum_i X[i*m + j] * Y[i*m + j].  Stage 1: workgroup (cx, ry)
// covers the CB = ceil(m / ceil(m / 64)) columns of chunk cx (36 of 72 for
// chi = 72: no lanes idle on a partial chunk of 64) with G = 256 / CB row
// groups, sweeps rows ry G + g, ry G + g + G CD_R, ... with coalesced row
// reads, and writes one partial per column; stage 2 adds the CD_R partials
// in a fixed order.  The same layout serves the fused CG updates below.
constexpr int CD_R = 64;

struct ColMap {
  int cb, groups, c, g;  // chunk width, row groups, this column, its group
  __device__ ColMap(int m) {
    const int chunks = (m + 63) / 64;
    cb = (m + chunks - 1) / chunks;
    groups = 256 / cb;
    c = blockIdx.x * cb + (int)threadIdx.x % cb;
    g = (int)threadIdx.x / cb;
  }
  __device__ bool active(int m) const { return g < groups && c < m; }
};

__global__ __launch_bounds__(256) void coldot_partial_kernel(
    const double* __restrict__ X, const double* __restrict__ Y, int64_t n,
    int m, double* __restrict__ part, long sXY) {
  __shared__ double red[256];
  const ColMap cm(m);
  X += blockIdx.z * sXY;
  Y += blockIdx.z * sXY;
  double v = 0.0;
  if (cm.active(m))
    for (int64_t i = blockIdx.y * cm.groups + cm.g; i < n;
         i += (int64_t)cm.groups * CD_R)
      v += X[i * m + cm.c] * Y[i * m + cm.c];
  red[threadIdx.x] = v;
  __syncthreads();
  if ((int)threadIdx.x < cm.cb && cm.c < m) {
    double t = 0.0;
    for (int q = 0; q < cm.groups; ++q) t += red[q * cm.cb + threadIdx.x];
    part[((long)blockIdx.z * CD_R + blockIdx.y) * m + cm.c] = t;
  }
}

__global__ void coldot_final_kernel(const double* __restrict__ part, int m,
                                    double* __restrict__ out) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= m) return;
  const double* p = part + (long)blockIdx.y * CD_R * m;
  double v = 0.0;
  for (int r = 0; r < CD_R; ++r) v += p[r * m + c];
  out[(long)blockIdx.y * m + c] = v;
}

// workgroup columns of the chunked layout
static int col_chunks(int m) { return (m + 63) / 64; }

void coldot(Device& dev, const double* X, const double* Y, int64_t n, int m,
            double* out, int batch, int64_t sXY) {
  Tensor part = dev.empty({batch, CD_R, m});
  hipLaunchKernelGGL(coldot_partial_kernel, dim3(col_chunks(m), CD_R, batch),
                     dim3(256), 0, dev.stream, X, Y, n, m, part.ptr,
                     (long)sXY);
  hipLaunchKernelGGL(coldot_final_kernel, dim3((m + 127) / 128, batch),
                     dim3(128), 0, dev.stream, part.ptr, m, out);
  IPEPS_HIP(hipGetLastError());
}

// w[j] = s_j^-1/2 for j < keep (and s_j > 0), else 0; j < chi.
__global__ void proj_weights_kernel(const double* S, const int* keep, int chi,
                                    double* w, int sS) {
  const int j = threadIdx.x + blockIdx.x * blockDim.x, bt = blockIdx.y;
  if (j >= chi) return;
  const double s = S[bt * sS + j];
  w[bt * chi + j] = (j < keep[bt] && s > 0.0) ? 1.0 / sqrt(s) : 0.0;
}

void proj_weights(Device& dev, const double* S, const int* keep, int chi,
                  double* w, int batch, int sS) {
  hipLaunchKernelGGL(proj_weights_kernel, dim3((chi + 127) / 128, batch),
                     dim3(128), 0, dev.stream, S, keep, chi, w, sS);
  IPEPS_HIP(hipGetLastError());
}

// sbar[j] = -1/2 s_j^-3/2 (wbar1[j] + wbar2[j]) for j < keep, else 0
__global__ void proj_sbar_kernel(const double* S, const int* keep, int chi,
                                 const double* wb1, const double* wb2,
                                 double* sbar, int sS) {
  const int j = threadIdx.x + blockIdx.x * blockDim.x, bt = blockIdx.y;
  if (j >= chi) return;
  const double s = S[bt * sS + j];
  const int o = bt * chi + j;
  sbar[o] = (j < keep[bt] && s > 0.0)
                ? -0.5 * (wb1[o] + wb2[o]) / (s * sqrt(s))
                : 0.0;
}

void proj_sbar(Device& dev, const double* S, const int* keep, int chi,
               const double* wb1, const double* wb2, double* sbar, int batch,
               int sS) {
  hipLaunchKernelGGL(proj_sbar_kernel, dim3((chi + 127) / 128, batch),
                     dim3(128), 0, dev.stream, S, keep, chi, wb1, wb2, sbar,
                     sS);
  IPEPS_HIP(hipGetLastError());
}

// Kept block of the SVD adjoint (chi x chi, zero outside i, j < keep):
// G_ij = F_ij (Au_ij - Au_ji) s_j + s_i F_ij (Av_ij - Av_ji) + d_ij sbar_i,
// F_ij = x/(x^2 + eta^2), x = s_j^2 - s_i^2, eta = 1e-12 s_0^2, F_ii = 0.
__global__ void svd_gkk_kernel(const double* Au, const double* Av,
                               const double* S, const double* sbar,
                               const int* keep, int chi, double* G, int sS) {
  const int bt = blockIdx.y;
  const long off = (long)bt * chi * chi;
  Au += off;
  Av += off;
  G += off;
  S += (long)bt * sS;
  sbar += (long)bt * chi;
  const int k = keep[bt];
  const double eta = 1e-12 * S[0] * S[0];
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < chi * chi;
       e += gridDim.x * blockDim.x) {
    const int i = e / chi, j = e % chi;
    double g = 0.0;
    if (i < k && j < k) {
      if (i == j) {
        g = sbar[i];
      } else {
        const double si = S[i], sj = S[j];
        const double x = sj * sj - si * si;
        const double F = x / (x * x + eta * eta);
        g = F * (Au[i * chi + j] - Au[j * chi + i]) * sj +
            si * F * (Av[i * chi + j] - Av[j * chi + i]);
      }
    }
    G[e] = g;
  }
}

void svd_gkk(Device& dev, const double* Au, const double* Av, const double* S,
             const double* sbar, const int* keep, int chi, double* G,
             int batch, int sS) {
  hipLaunchKernelGGL(svd_gkk_kernel,
                     dim3(grid_for((int64_t)chi * chi, 256), batch),
                     dim3(256), 0, dev.stream, Au, Av, S, sbar, keep, chi, G,
                     sS);
  IPEPS_HIP(hipGetLastError());
}

// X (n x m) columns j >= keep set to zero
__global__ void mask_cols_kernel(double* X, int64_t n, int m,
                                 const int* keep) {
  const int k = keep[blockIdx.y];
  X += (long)blockIdx.y * n * m;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n * m;
       e += (int64_t)gridDim.x * blockDim.x)
    if ((int)(e % m) >= k) X[e] = 0.0;
}

void mask_cols(Device& dev, double* X, int64_t n, int m, const int* keep,
               int batch) {
  hipLaunchKernelGGL(mask_cols_kernel, dim3(grid_for(n * m, 256), batch),
                     dim3(256), 0, dev.stream, X, n, m, keep);
  IPEPS_HIP(hipGetLastError());
}

// Column-wise CG on blocks of `rows` x m (per-column scalars):
//   mode 0: alpha_j = rr_j / pAp_j (0 when pAp_j <= 0 or rr_j == 0);
//           x += alpha p; r -= alpha Ap
//   mode 1: p = r + (rrn_j / rr_j) p  (beta 0 when rr_j == 0)
__global__ void colcg_kernel(int mode, int64_t rows, int m, const double* rr,
                             const double* den, double* x, double* r,
                             double* p, const double* Ap, int64_t rpb) {
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
       e < rows * m; e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t j = (e / (rpb * m)) * m + e % m;
    if (mode == 0) {
      const double a = (den[j] > 0.0 && rr[j] > 0.0) ? rr[j] / den[j] : 0.0;
      x[e] += a * p[e];
      r[e] -= a * Ap[e];
    } else {
      const double bta = rr[j] > 0.0 ? den[j] / rr[j] : 0.0;
      p[e] = r[e] + bta * p[e];
    }
  }
}

// One CG step of column-wise systems, fused with the reductions around it.
// Workgroups (column chunks) x (CD_R row groups) x batch in coldot's
// layout, so the sums keep coldot's order.
//   step: a_j = num_j / den_j (0 unless both > 0), x += a p, r -= a A p,
//         partial sums of r_j^2 into part[batch][CD_R][m];
//   dir:  rr_new_j = sum of the partials, p = r + (rr_new_j / rr_old_j) p
//         (0 unless rr_old_j > 0).
__global__ __launch_bounds__(256) void colcg_step_kernel(
    int64_t n, int m, const double* __restrict__ num,
    const double* __restrict__ den, double* __restrict__ x,
    double* __restrict__ r, const double* __restrict__ p,
    const double* __restrict__ Ap, double* __restrict__ part) {
  __shared__ double red[256];
  const ColMap cm(m);
  const int c = cm.c, bt = blockIdx.z;
  const long off = (long)bt * n * m;
  double v = 0.0;
  if (cm.active(m)) {
    const double nu = num[(long)bt * m + c], de = den[(long)bt * m + c];
    const double a = (de > 0.0 && nu > 0.0) ? nu / de : 0.0;
    for (int64_t i = blockIdx.y * cm.groups + cm.g; i < n;
         i += (int64_t)cm.groups * CD_R) {
      const long e = off + i * m + c;
      x[e] += a * p[e];
      const double rv = r[e] - a * Ap[e];
      r[e] = rv;
      v += rv * rv;
    }
  }
  red[threadIdx.x] = v;
  __syncthreads();
  if ((int)threadIdx.x < cm.cb && c < m) {
    double t = 0.0;
    for (int q = 0; q < cm.groups; ++q) t += red[q * cm.cb + threadIdx.x];
    part[((long)bt * CD_R + blockIdx.y) * m + c] = t;
  }
}

__global__ __launch_bounds__(256) void colcg_dir_kernel(
    int64_t n, int m, const double* __restrict__ part,
    const double* __restrict__ rr_old, double* __restrict__ rr_new,
    const double* __restrict__ r, double* __restrict__ p) {
  __shared__ double beta[256];
  const ColMap cm(m);
  const int c = cm.c, bt = blockIdx.z;
  if ((int)threadIdx.x < cm.cb) {
    double b = 0.0;
    if (c < m) {
      const double* pp = part + (long)bt * CD_R * m + c;
      double sum = 0.0;
      for (int q = 0; q < CD_R; ++q) sum += pp[(long)q * m];
      const double ro = rr_old[(long)bt * m + c];
      b = ro > 0.0 ? sum / ro : 0.0;
      if (blockIdx.y == 0) rr_new[(long)bt * m + c] = sum;
    }
    beta[threadIdx.x] = b;
  }
  __syncthreads();
  if (!cm.active(m)) return;
  const double bb = beta[(int)threadIdx.x % cm.cb];
  const long off = (long)bt * n * m;
  for (int64_t i = blockIdx.y * cm.groups + cm.g; i < n;
       i += (int64_t)cm.groups * CD_R) {
    const long e = off + i * m + c;
    p[e] = r[e] + bb * p[e];
  }
}

void colcg_step(Device& dev, int64_t n, int m, int batch, const double* num,
                const double* den, double* x, double* r, const double* p,
                const double* Ap, double* part) {
  hipLaunchKernelGGL(colcg_step_kernel, dim3(col_chunks(m), CD_R, batch),
                     dim3(256), 0, dev.stream, n, m, num, den, x, r, p, Ap,
                     part);
  IPEPS_HIP(hipGetLastError());
}

void colcg_dir(Device& dev, int64_t n, int m, int batch, const double* part,
               const double* rr_old, double* rr_new, const double* r,
               double* p) {
  hipLaunchKernelGGL(colcg_dir_kernel, dim3(col_chunks(m), CD_R, batch),
                     dim3(256), 0, dev.stream, n, m, part, rr_old, rr_new, r,
                     p);
  IPEPS_HIP(hipGetLastError());
}

int colcg_parts() { return CD_R; }

void colcg(Device& dev, int mode, int64_t rows, int m, const double* rr,
           const double* den, double* x, double* r, double* p,
           const double* Ap, int64_t rows_per_batch) {
  hipLaunchKernelGGL(colcg_kernel, dim3(grid_for(rows * m, 256)), dim3(256),
                     0, dev.stream, mode, rows, m, rr, den, x, r, p, Ap,
                     rows_per_batch > 0 ? rows_per_batch : rows);
  IPEPS_HIP(hipGetLastError());
}

// Deflation of the complement solves (projector backward).  W is an
// orthonormal basis of pairs [w_u; 0], [0; w_v] in the complement of the kept
// singular vectors, H = [[0, P_D M], [P'_D M^T, 0]] and, for kept column j,
// A_j = s_j I - H.  With K = W^T H W = Phi diag(lambda) Phi^T the Galerkin
// matrix is W^T A_j W = Phi diag(s_j - lambda) Phi^T, so one eigenbasis
// serves every column.
//
// K from B1 = W_u^T P_D M W_v and B2 = W_v^T P'_D M^T W_u (equal to B1^T up
// to rounding; the mean is used): K = [[0, B], [B^T, 0]], [batch][2m][2m].
__global__ void defl_build_k_kernel(const double* B1, const double* B2, int m,
                                    double* K) {
  const int bt = blockIdx.y, m2 = 2 * m;
  B1 += (long)bt * m * m;
  B2 += (long)bt * m * m;
  K += (long)bt * m2 * m2;
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < m2 * m2;
       e += gridDim.x * blockDim.x) {
    const int i = e / m2, j = e % m2;
    double v = 0.0;
    if (i < m && j >= m)
      v = 0.5 * (B1[i * m + (j - m)] + B2[(j - m) * m + i]);
    else if (i >= m && j < m)
      v = 0.5 * (B1[j * m + (i - m)] + B2[(i - m) * m + j]);
    K[e] = v;
  }
}

void defl_build_k(Device& dev, const double* B1, const double* B2, int m,
                  double* K, int batch) {
  hipLaunchKernelGGL(defl_build_k_kernel,
                     dim3(grid_for((int64_t)4 * m * m, 256), batch), dim3(256),
                     0, dev.stream, B1, B2, m, K);
  IPEPS_HIP(hipGetLastError());
}

// x <- 1/sqrt(x) where x > thr, else 0
__global__ void inv_sqrt_clip_kernel(double* x, int64_t n, double thr) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    x[i] = x[i] > thr ? 1.0 / sqrt(x[i]) : 0.0;
}

void inv_sqrt_clip(Device& dev, double* x, int64_t n, double thr) {
  if (n <= 0) return;
  hipLaunchKernelGGL(inv_sqrt_clip_kernel, dim3(grid_for(n, 256)), dim3(256),
                     0, dev.stream, x, n, thr);
  IPEPS_HIP(hipGetLastError());
}

// Coefficients in the eigenbasis of K, [batch][2m][chi], from
// H = [(W Phi)^T r; (H W Phi)^T r] ([batch][4m][chi]):
//   mode 0: c = h1 / (s_j - lambda)                (x0 = W Phi c)
//   mode 1: c = (s_j h1 - h2) / (s_j - lambda)      (p -= W Phi c)
//   mode 2: c = y (s_j + lambda) h1 / (y^2 + eta^2), y = s_j^2 - lambda^2,
//           eta = 1e-12 s_1^2                        (broadened x0)
// Zero for masked columns (j >= keep) and, in modes 0 and 1, where
// s_j - lambda <= 1e-12 s_1 (that direction is left out of the deflation
// space of column j).
__global__ void defl_coef_kernel(int mode, const double* S, const int* keep,
                                 const double* lam, int chi, int m2, int sS,
                                 const double* H, double* out) {
  const int bt = blockIdx.y;
  const double* s = S + (long)bt * sS;
  const double* l = lam + (long)bt * m2;
  H += (long)bt * 2 * m2 * chi;
  out += (long)bt * m2 * chi;
  const int k = keep[bt];
  const double guard = 1e-12 * s[0];
  const double eta = 1e-12 * s[0] * s[0];
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < m2 * chi;
       e += gridDim.x * blockDim.x) {
    const int i = e / chi, j = e % chi;
    const double sj = s[j], dd = sj - l[i];
    double v = 0.0;
    if (mode == 2) {
      // broadened Galerkin coefficient y (s_j + lambda) / (y^2 + eta^2),
      // y = s_j^2 - lambda^2: 1 / (s_j - lambda) away from s_j, bounded
      // through it
      if (j < k) {
        const double y = (sj - l[i]) * (sj + l[i]);
        v = y / (y * y + eta * eta) * (sj + l[i]) * H[e];
      }
    } else if (j < k && dd > guard) {
      const double h1 = H[e];
      v = mode == 0 ? h1 / dd : (sj * h1 - H[m2 * chi + e]) / dd;
    }
    out[e] = v;
  }
}

void defl_coef(Device& dev, int mode, const double* S, const int* keep,
               const double* lam, int chi, int m2, int sS, const double* H,
               double* out, int batch) {
  hipLaunchKernelGGL(defl_coef_kernel,
                     dim3(grid_for((int64_t)m2 * chi, 256), batch), dim3(256),
                     0, dev.stream, mode, S, keep, lam, chi, m2, sS, H, out);
  IPEPS_HIP(hipGetLastError());
}

// y[r] = sum_s x[r][s][s] (x: rows x d x d)
__global__ void trace_dd_kernel(const double* __restrict__ x, int64_t rows,
                                int d, double* __restrict__ y) {
  const int64_t dd = (int64_t)d * d;
  for (int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; r < rows;
       r += (int64_t)gridDim.x * blockDim.x) {
    double v = 0.0;
    for (int s = 0; s < d; ++s) v += x[r * dd + s * (d + 1)];
    y[r] = v;
  }
}

void trace_dd(Device& dev, const double* x, int64_t rows, int d, double* y) {
  if (rows <= 0) return;
  hipLaunchKernelGGL(trace_dd_kernel, dim3(grid_for(rows, 256)), dim3(256), 0,
                     dev.stream, x, rows, d, y);
  IPEPS_HIP(hipGetLastError());
}

// gx[r][s][t] = beta gx[r][s][t] + (s == t) g[r]
__global__ void trace_dd_backward_kernel(const double* __restrict__ g,
                                         int64_t rows, int d,
                                         double* __restrict__ gx,
                                         double beta) {
  const int64_t dd = (int64_t)d * d, n = rows * dd;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t r = e / dd;
    const int q = (int)(e - r * dd);
    double v = (q % (d + 1) == 0) ? g[r] : 0.0;
    if (beta != 0.0) v += beta * gx[e];
    gx[e] = v;
  }
}

void trace_dd_backward(Device& dev, const double* g, int64_t rows, int d,
                       double* gx, double beta) {
  const int64_t n = rows * d * d;
  if (n <= 0) return;
  hipLaunchKernelGGL(trace_dd_backward_kernel, dim3(grid_for(n, 256)),
                     dim3(256), 0, dev.stream, g, rows, d, gx, beta);
  IPEPS_HIP(hipGetLastError());
}

// y[i][j] = a * s_j * x[i][j] + b * y[i][j]   (column-scaled axpby)
__global__ void col_axpby_kernel(int64_t n, int m, double a, const double* s,
                                 const double* x, double b, double* y,
                                 int64_t rpb, int64_t sS) {
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n * m;
       e += (int64_t)gridDim.x * blockDim.x) {
    const double sj = s ? s[(e / (rpb * m)) * sS + e % m] : 1.0;
    double v = a * sj * x[e];
    if (b != 0.0) v += b * y[e];
    y[e] = v;
  }
}

void col_axpby(Device& dev, int64_t n, int m, double a, const double* s,
               const double* x, double b, double* y, int64_t rows_per_batch,
               int64_t sS) {
  hipLaunchKernelGGL(col_axpby_kernel, dim3(grid_for(n * m, 256)), dim3(256),
                     0, dev.stream, n, m, a, s, x, b, y,
                     rows_per_batch > 0 ? rows_per_batch : n, sS);
  IPEPS_HIP(hipGetLastError());
}

}  // namespace ipeps

namespace ipeps {

// dst[r*ldd + c] = src[r*lds + c], rows x cols
__global__ void copy2d_kernel(const double* src, int64_t lds, double* dst,
                              int64_t ldd, int64_t rows, int64_t cols,
                              int64_t sSrc, int64_t sDst) {
  src += blockIdx.y * sSrc;
  dst += blockIdx.y * sDst;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
       e < rows * cols; e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t r = e / cols, c = e % cols;
    dst[r * ldd + c] = src[r * lds + c];
  }
}

void copy2d(Device& dev, const double* src, int64_t lds, double* dst,
            int64_t ldd, int64_t rows, int64_t cols, int batch, int64_t sSrc,
            int64_t sDst) {
  hipLaunchKernelGGL(copy2d_kernel, dim3(grid_for(rows * cols, 256), batch),
                     dim3(256), 0, dev.stream, src, lds, dst, ldd, rows, cols,
                     sSrc, sDst);
  IPEPS_HIP(hipGetLastError());
}

}  // namespace ipeps

namespace ipeps {

// ------------------------------------------------ C4v QR-CTMRG helpers
// out[i][j] = M[max(i,j)][min(i,j)] (the lower triangle mirrored), b x b
__global__ void copyltu_kernel(const double* M, double* out, int b) {
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < b * b;
       e += gridDim.x * blockDim.x) {
    const int i = e / b, j = e % b;
    out[e] = i >= j ? M[i * b + j] : M[j * b + i];
  }
}

void copyltu(Device& dev, const double* M, double* out, int b) {
  hipLaunchKernelGGL(copyltu_kernel, dim3(grid_for((int64_t)b * b, 256)),
                     dim3(256), 0, dev.stream, M, out, b);
  IPEPS_HIP(hipGetLastError());
}

// out[i][j] = F_ij X[i][j], F_ij = x / (x^2 + eta^2), x = lam_j - lam_i,
// F_ii = 0; eta = rel * max|lam|
__global__ void eig_fmul_kernel(const double* lam, const double* X,
                                double* out, int b, double rel) {
  double mx = 0.0;
  for (int i = 0; i < b; ++i) mx = fmax(mx, fabs(lam[i]));
  const double eta = rel * mx;
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < b * b;
       e += gridDim.x * blockDim.x) {
    const int i = e / b, j = e % b;
    const double x = lam[j] - lam[i];
    out[e] = i == j ? 0.0 : X[e] * x / (x * x + eta * eta);
  }
}

void eig_fmul(Device& dev, const double* lam, const double* X, double* out,
              int b, double rel) {
  hipLaunchKernelGGL(eig_fmul_kernel, dim3(grid_for((int64_t)b * b, 256)),
                     dim3(256), 0, dev.stream, lam, X, out, b, rel);
  IPEPS_HIP(hipGetLastError());
}

// Reorders eigenpairs given in descending signed order: the k of largest
// |lambda| (ties: the larger signed value, i.e. the lower index) first,
// then the others, each group keeping its descending signed order.  One
// workgroup; b <= 512.
__global__ void eig_order_kept_kernel(const double* lam, const double* W,
                                      double* lam_out, double* W_out, int b,
                                      int k) {
  __shared__ int src[512];
  if (threadIdx.x == 0) {
    int nk = 0, nd = k;
    for (int i = 0; i < b; ++i) {
      // rank of i by (|lambda| descending, index ascending)
      int r = 0;
      const double ai = fabs(lam[i]);
      for (int j = 0; j < b; ++j) {
        const double aj = fabs(lam[j]);
        r += (aj > ai || (aj == ai && j < i)) ? 1 : 0;
      }
      if (r < k)
        src[nk++] = i;
      else
        src[nd++] = i;
    }
  }
  __syncthreads();
  for (int e = threadIdx.x; e < b * b; e += blockDim.x) {
    const int r = e / b, c = e % b;
    W_out[e] = W[r * b + src[c]];
  }
  for (int c = threadIdx.x; c < b; c += blockDim.x) lam_out[c] = lam[src[c]];
}

void eig_order_kept(Device& dev, const double* lam, const double* W,
                    double* lam_out, double* W_out, int b, int k) {
  if (b < 1 || b > 512 || k < 0 || k > b)
    throw ArgError("eig_order_kept: needs 0 <= k <= b <= 512");
  hipLaunchKernelGGL(eig_order_kept_kernel, dim3(1), dim3(256), 0,
                     dev.stream, lam, W, lam_out, W_out, b, k);
  IPEPS_HIP(hipGetLastError());
}

// s[j] = sign of the entry of column j of X (n x b, row major) maximising
// |x_rj| (1 + r / (2n)) (first on ties), +1 for a zero column.  One wave
// per column.
__global__ void col_sign_kernel(const double* X, int64_t n, int b,
                                double* s) {
  const int j = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (j >= b) return;
  double best = -1.0;
  int64_t bi = 0;
  for (int64_t i = lane; i < n; i += 64) {
    const double a = fabs(X[i * b + j]) * (1.0 + (double)i / (2.0 * (double)n));
    if (a > best) {
      best = a;
      bi = i;
    }
  }
  for (int o = 32; o > 0; o >>= 1) {
    const double ob = __shfl_down(best, o, 64);
    const int64_t oi = __shfl_down(bi, o, 64);
    if (ob > best || (ob == best && oi < bi)) {
      best = ob;
      bi = oi;
    }
  }
  if (lane == 0) s[j] = X[bi * b + j] < 0.0 ? -1.0 : 1.0;
}

void col_sign(Device& dev, const double* X, int64_t n, int b, double* s) {
  hipLaunchKernelGGL(col_sign_kernel, dim3((b + 3) / 4), dim3(256), 0,
                     dev.stream, X, n, b, s);
  IPEPS_HIP(hipGetLastError());
}

// the largest dynamic LDS each kernel here can ask for (see allow_lds)
void prime_kernel_attributes() {
  allow_lds((const void*)sym_eig_jacobi_kernel<true>,
            jacobi_lds_bytes(96, true));
  allow_lds((const void*)sym_eig_jacobi_kernel<false>,
            jacobi_lds_bytes(JAC_MAXB, false));
  {
    const size_t h = JAC_BIGB / 2;
    allow_lds((const void*)sym_eig_jacobi_big_kernel,
              h * 5 * sizeof(double) + h * 2 * sizeof(int) +
                  h * (h + 1) / 2 * sizeof(int));
  }
  allow_lds((const void*)chol_orth_kernel,
            ((size_t)128 * 129 + 128) * sizeof(double));
}

}  // namespace ipeps
