// FP64 GEMM on the gfx950 matrix cores (v_mfma_f64_16x16x4_f64).
//
// C[b] = alpha op(A[b]) op(B[b]) + beta C[b], row major.
//
// Workgroup: 256 threads = 4 waves of 64 lanes arranged WM x WN; the block
// tile BM x BN is staged through LDS in BK = 16 deep slices, double
// buffered: while the waves run the MFMAs of slice k out of one LDS buffer,
// every thread already holds slice k+1 in registers (global loads issued
// before the MFMAs) and writes it to the other buffer afterwards, so there
// is one barrier per slice and the global latency hides behind the MFMAs.
// Transposes are template parameters so that every global load is
// coalesced along the contiguous dimension of its operand.
//
// Skinny products (the n x n x chi products of the projector SVD and of the
// backward complement solves, or K >> M N) split K across workgroups into a
// partial buffer reduced in a fixed order afterwards, so that the grid
// covers all 256 CUs and the result is deterministic.
//
// MFMA f64 16x16x4 lane layout (checked on gfx950): lane l supplies
// A[l%16][l/16] and B[l/16][l%16]; the 16x16 result holds D[l/16 + 4r][l%16]
// in register r of lane l.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>

#include "engine.hpp"

namespace ipeps {

typedef double f64x4 __attribute__((ext_vector_type(4)));

namespace {

constexpr int BK = 16;
constexpr int PAD = 2;

template <int BM, int BN, int WM, int WN, bool TA, bool TB>
__global__ __launch_bounds__(256, 2) void gemm64_kernel(
    int M, int N, int K, double alpha, const double* __restrict__ A,
    long lda, long sA, const double* __restrict__ B, long ldb, long sB,
    double beta, double* __restrict__ C, long ldc, long sC, int tiles_n,
    int splits, int kchunk, double* __restrict__ part,
    const double* const* __restrict__ Ap, const double* const* __restrict__ Bp,
    double* const* __restrict__ Cp) {
  static_assert(WM * WN == 4, "4 waves");
  constexpr int WTM = BM / WM, WTN = BN / WN;
  constexpr int TM = WTM / 16, TN = WTN / 16;
  constexpr int AE = BM * BK / 256, BE = BK * BN / 256;
  __shared__ double As[2][BK][BM + PAD];
  __shared__ double Bs[2][BK][BN + PAD];

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave / WN, wn = wave % WN;
  const int bz = blockIdx.y / splits, sp = blockIdx.y % splits;
  A = Ap ? Ap[bz] : A + (long)bz * sA;
  B = Bp ? Bp[bz] : B + (long)bz * sB;
  const int m0 = (blockIdx.x / tiles_n) * BM;
  const int n0 = (blockIdx.x % tiles_n) * BN;
  const int kbeg = sp * kchunk;
  const int kend = min(K, kbeg + kchunk);

  double ra[AE], rb[BE];
  auto load = [&](int kb) {
#pragma unroll
    for (int i = 0; i < AE; ++i) {
      const int e = tid + i * 256;
      int mm, kk;
      if (!TA) {
        mm = e / BK;
        kk = e % BK;
      } else {
        kk = e / BM;
        mm = e % BM;
      }
      const int gm = m0 + mm, gk = kb + kk;
      double v = 0.0;
      if (gm < M && gk < kend)
        v = TA ? A[(long)gk * lda + gm] : A[(long)gm * lda + gk];
      ra[i] = v;
    }
#pragma unroll
    for (int i = 0; i < BE; ++i) {
      const int e = tid + i * 256;
      int kk, nn;
      if (!TB) {
        kk = e / BN;
        nn = e % BN;
      } else {
        nn = e / BK;
        kk = e % BK;
      }
      const int gk = kb + kk, gn = n0 + nn;
      double v = 0.0;
      if (gk < kend && gn < N)
        v = TB ? B[(long)gn * ldb + gk] : B[(long)gk * ldb + gn];
      rb[i] = v;
    }
  };
  auto store = [&](int buf) {
#pragma unroll
    for (int i = 0; i < AE; ++i) {
      const int e = tid + i * 256;
      if (!TA)
        As[buf][e % BK][e / BK] = ra[i];
      else
        As[buf][e / BM][e % BM] = ra[i];
    }
#pragma unroll
    for (int i = 0; i < BE; ++i) {
      const int e = tid + i * 256;
      if (!TB)
        Bs[buf][e / BN][e % BN] = rb[i];
      else
        Bs[buf][e % BK][e / BK] = rb[i];
    }
  };

  f64x4 acc[TM][TN];
#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int j = 0; j < TN; ++j) acc[i][j] = f64x4{0.0, 0.0, 0.0, 0.0};

  if (kbeg < kend) {
    load(kbeg);
    store(0);
  }
  __syncthreads();
  int buf = 0;
  for (int kb = kbeg; kb < kend; kb += BK) {
    const bool more = kb + BK < kend;
    if (more) load(kb + BK);
#pragma unroll
    for (int k4 = 0; k4 < BK; k4 += 4) {
      double a[TM], b[TN];
#pragma unroll
      for (int i = 0; i < TM; ++i)
        a[i] = As[buf][k4 + (lane >> 4)][wm * WTM + i * 16 + (lane & 15)];
#pragma unroll
      for (int j = 0; j < TN; ++j)
        b[j] = Bs[buf][k4 + (lane >> 4)][wn * WTN + j * 16 + (lane & 15)];
#pragma unroll
      for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 0; j < TN; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[i], b[j],
                                                           acc[i][j], 0, 0,
                                                           0);
    }
    if (more) store(buf ^ 1);
    __syncthreads();
    buf ^= 1;
  }

  // epilogue: direct (splits == 1) or partial tile (split K)
  double* out;
  long ldo;
  if (splits == 1) {
    out = Cp ? Cp[bz] : C + (long)bz * sC;
    ldo = ldc;
  } else {
    out = part + ((long)sp * gridDim.y / splits + bz) * (long)M * N;
    ldo = N;
  }
#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int j = 0; j < TN; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = m0 + wm * WTM + i * 16 + (lane >> 4) + 4 * r;
        const int col = n0 + wn * WTN + j * 16 + (lane & 15);
        if (row < M && col < N) {
          if (splits == 1) {
            double v = alpha * acc[i][j][r];
            if (beta != 0.0) v += beta * out[(long)row * ldo + col];
            out[(long)row * ldo + col] = v;
          } else {
            out[(long)row * ldo + col] = acc[i][j][r];
          }
        }
      }
}

// part layout [S][batch][M][N]; C[b] = alpha sum_s part[s][b] + beta C[b]
__global__ void splitk_sum_kernel(const double* __restrict__ part, int S,
                                  int batch, long M, long N, double alpha,
                                  double beta, double* __restrict__ C,
                                  long ldc, long sC,
                                  double* const* __restrict__ Cp) {
  const long mn = M * N, tot = mn * batch;
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < tot;
       e += (long)gridDim.x * blockDim.x) {
    const long b = e / mn, i = e % mn;
    double v = 0.0;
    for (int s = 0; s < S; ++s) v += part[((long)s * batch + b) * mn + i];
    const long r = i / N, c = i % N;
    double* cp = (Cp ? Cp[b] : C + b * sC) + r * ldc + c;
    double o = alpha * v;
    if (beta != 0.0) o += beta * *cp;
    *cp = o;
  }
}

template <int BM, int BN, int WM, int WN>
void launch_cfg(Device& dev, bool tA, bool tB, int M, int N, int K,
                double alpha, const double* A, long lda, long sA,
                const double* B, long ldb, long sB, double beta, double* C,
                long ldc, long sC, int batch, const double* const* Ap,
                const double* const* Bp, double* const* Cp) {
  const long tm = (M + BM - 1) / BM, tn = (N + BN - 1) / BN;
  const long tiles = tm * tn;
  // split K until the grid covers the chip (>= 320 workgroups), keeping at
  // least 256 of K per split
  int S = 1;
  const long want = 320;
  if (tiles * batch < want && K >= 512) {
    S = (int)std::min<long>((want + tiles * batch - 1) / (tiles * batch),
                            K / 256);
    S = std::max(1, std::min(S, 64));
  }
  int kchunk = (K + S - 1) / S;
  kchunk = (kchunk + BK - 1) / BK * BK;
  S = (K + kchunk - 1) / kchunk;
  Tensor part;
  if (S > 1) part = dev.empty({(int64_t)S * batch * M * N});
  if (tiles * batch * S >= (1L << 31) || (long)batch * S > 65535)
    throw ArgError("gemm: grid too large");
  dim3 grid((unsigned)tiles, (unsigned)(batch * S));
  // the profiler brackets the matrix-core kernel alone (split-K partial
  // sums are a kernel of their own), with the algorithmic 2 M N K flops
  if (dev.prof.on)
    dev.prof.begin(dev.stream, PROF_GEMM, 2.0 * M * N * K * batch,
                   8.0 * batch * ((double)M * K + (double)K * N +
                                  (beta != 0.0 ? 2.0 : 1.0) * M * N));
  auto go = [&](auto kern) {
    hipLaunchKernelGGL(kern, grid, dim3(256), 0, dev.stream, M, N, K, alpha,
                       A, lda, sA, B, ldb, sB, beta, C, ldc, sC, (int)tn, S,
                       kchunk, part.ptr, Ap, Bp, Cp);
  };
  if (!tA && !tB) go(gemm64_kernel<BM, BN, WM, WN, false, false>);
  if (tA && !tB) go(gemm64_kernel<BM, BN, WM, WN, true, false>);
  if (!tA && tB) go(gemm64_kernel<BM, BN, WM, WN, false, true>);
  if (tA && tB) go(gemm64_kernel<BM, BN, WM, WN, true, true>);
  if (dev.prof.on) dev.prof.end(dev.stream);
  IPEPS_HIP(hipGetLastError());
  if (S > 1) {
    const long tot = (long)batch * M * N;
    const int g = (int)std::max<long>(1, std::min<long>((tot + 255) / 256,
                                                        8192));
    hipLaunchKernelGGL(splitk_sum_kernel, dim3(g), dim3(256), 0, dev.stream,
                       part.ptr, S, batch, (long)M, (long)N, alpha, beta, C,
                       ldc, sC, Cp);
    IPEPS_HIP(hipGetLastError());
  }
}

}  // namespace

static void dispatch(Device& dev, bool tA, bool tB, int64_t M, int64_t N,
                     int64_t K, double alpha, const double* A, int64_t lda,
                     int64_t sA, const double* B, int64_t ldb, int64_t sB,
                     double beta, double* C, int64_t ldc, int64_t sC,
                     int64_t batch, const double* const* Ap,
                     const double* const* Bp, double* const* Cp) {
  if (M >= (1LL << 31) || N >= (1LL << 31) || K >= (1LL << 31) ||
      batch > 65535)
    throw ArgError("gemm: size out of range");
  const int m = (int)M, n = (int)N, k = (int)K, bt = (int)batch;
#define IPEPS_CFG(BM_, BN_, WM_, WN_)                                        \
  launch_cfg<BM_, BN_, WM_, WN_>(dev, tA, tB, m, n, k, alpha, A, lda, sA, B, \
                                 ldb, sB, beta, C, ldc, sC, bt, Ap, Bp, Cp)
  if (M >= 128) {
    // narrow N (chi-wide blocks of the projector SVD and the complement
    // solves): 4 waves stacked along M, tile width rounded up to 16
    if (N <= 48)
      IPEPS_CFG(128, 48, 4, 1);
    else if (N <= 64)
      IPEPS_CFG(128, 64, 4, 1);
    else if (N <= 80)
      IPEPS_CFG(128, 80, 4, 1);
    else if (N <= 96)
      IPEPS_CFG(128, 96, 4, 1);
    else
      IPEPS_CFG(128, 128, 2, 2);
  } else if (N >= 128) {
    IPEPS_CFG(64, 128, 2, 2);
  } else {
    IPEPS_CFG(64, 64, 2, 2);
  }
#undef IPEPS_CFG
}

void gemm(Device& dev, bool tA, bool tB, int64_t M, int64_t N, int64_t K,
          double alpha, const double* A, int64_t lda, int64_t sA,
          const double* B, int64_t ldb, int64_t sB, double beta, double* C,
          int64_t ldc, int64_t sC, int64_t batch) {
  if (M <= 0 || N <= 0 || batch <= 0) return;
  if (K == 0) {
    for (int64_t b = 0; b < batch; ++b)
      for (int64_t m = 0; m < M; ++m)
        axpby(dev, N, 0.0, C + b * sC + m * ldc, beta, C + b * sC + m * ldc);
    return;
  }
  dispatch(dev, tA, tB, M, N, K, alpha, A, lda, sA, B, ldb, sB, beta, C, ldc,
           sC, batch, nullptr, nullptr, nullptr);
}

void gemm_ptrs(Device& dev, bool tA, bool tB, int64_t M, int64_t N,
               int64_t K, double alpha, const std::vector<const double*>& A,
               int64_t lda, const std::vector<const double*>& B, int64_t ldb,
               double beta, const std::vector<double*>& C, int64_t ldc) {
  const int64_t batch = (int64_t)A.size();
  if (M <= 0 || N <= 0 || batch <= 0 || K <= 0) return;
  if ((int64_t)B.size() != batch || (int64_t)C.size() != batch)
    throw ArgError("gemm_ptrs: pointer counts differ");
  // one upload of the three pointer arrays (stream ordered, pageable copy)
  std::vector<double> h(3 * batch);
  std::memcpy(h.data(), A.data(), 8 * batch);
  std::memcpy(h.data() + batch, B.data(), 8 * batch);
  std::memcpy(h.data() + 2 * batch, C.data(), 8 * batch);
  Tensor d = dev.empty({3 * batch});
  dev.upload(d, h.data());
  const double* const* Ap = (const double* const*)d.ptr;
  const double* const* Bp = (const double* const*)(d.ptr + batch);
  double* const* Cp = (double* const*)(d.ptr + 2 * batch);
  dispatch(dev, tA, tB, M, N, K, alpha, A[0], lda, 0, B[0], ldb, 0, beta,
           C[0], ldc, 0, batch, Ap, Bp, Cp);
}

}  // namespace ipeps
