// Dense GEMM on the gfx950 matrix cores, FP64 in memory.
//
// C[b] = alpha op(A[b]) op(B[b]) + beta C[b], row major, with the products
// computed in one of three arithmetics (Device::cprec):
//   FP64  v_mfma_f64_16x16x4_f64, operands and accumulation in FP64;
//   FP32  v_mfma_f32_16x16x4_f32, operands rounded to FP32 when they are
//         staged into LDS, FP32 accumulation, result written in FP64;
//   BF16x3 v_mfma_f32_16x16x32_bf16 on a two-term BF16 split of each
//         operand (three products, FP32 accumulation), gemm_bf16x3_kernel.
//
// Workgroup: 256 threads = 4 waves of 64 lanes arranged WM x WN; the block
// tile BM x BN is staged through LDS in BK = 16 deep slices, double
// buffered: while the waves run the MFMAs of slice k out of one LDS buffer,
// every thread already holds slice k+1 in registers (global loads issued
// before the MFMAs) and writes it to the other buffer afterwards, so there
// is one barrier per slice and the global latency hides behind the MFMAs.
// Every global load is coalesced along the contiguous dimension of its
// operand, and the LDS layout follows it: an operand read along K is kept
// row-major with an odd row stride (BK + 1), one read along M or N is kept
// K-major; either way the 16 lanes of an MFMA operand fetch hit distinct
// banks.
//
// Skinny products (the n x n x chi products of the projector SVD and of the
// backward complement solves, or K >> M N) split K across workgroups into a
// partial buffer reduced in a fixed order afterwards, so that the grid
// covers all 256 CUs and the result is deterministic.
//
// Batches address their operands either by strides or by up to 16 pointer
// triples passed by value in the kernel arguments.
//
// MFMA 16x16x4 lane layouts (checked on gfx950): lane l supplies
// A[l%16][l/16] and B[l/16][l%16]; the 16x16 result holds, in register r of
// lane l, D[l/16 + 4r][l%16] for FP64 and D[4(l/16) + r][l%16] for FP32.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <map>
#include <mutex>
#include <cstring>
#include <type_traits>

#include "engine.hpp"

namespace ipeps {

typedef double f64x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

namespace {

// LDS row padding.  FP64 tiles: row stride BK + 1 for operands read along
// K, X + 2 for operands read along M/N (X = BM or BN).  FP32 tiles (4-byte
// banks): BK + 2 puts the 16 rows x 2 K values that half a wave reads for
// one MFMA operand on 32 distinct banks, and a K-major stride of 16 mod 32
// puts K rows k and k+1 of 16 consecutive columns on distinct banks.
template <bool F32>
struct Pad {
  static constexpr int K = F32 ? 2 : 1;
  static constexpr int M(int x) { return F32 ? ((16 - x) % 32 + 32) % 32 : 2; }
};
constexpr int MAXP = 16;  // pointer triples per launch

struct PtrArgs {
  const void* a[MAXP];  // double, or float for FP32-stored A
  const double* b[MAXP];
  double* c[MAXP];
};

// offset of index x in a mixed-radix layout of n digits (CMap)
__device__ __forceinline__ long cmap_off(int n, const int* e, const int64_t* s,
                                         int x) {
  long o = 0;
#pragma unroll
  for (int i = 0; i < CMAP_DIGITS; ++i) {
    if (i >= n) break;
    if (i == n - 1) {
      o += (long)x * s[i];
      break;
    }
    const int q = x / e[i];
    o += (long)(x - q * e[i]) * s[i];
    x = q;
  }
  return o;
}
__device__ __forceinline__ long cmap_row(const CMap& cm, int row, long ldc) {
  return cm.nr == 0 ? (long)row * ldc : cmap_off(cm.nr, cm.re, cm.rs, row);
}
__device__ __forceinline__ long cmap_col(const CMap& cm, int col) {
  return cm.nr == 0 ? (long)col : cmap_off(cm.nc, cm.ce, cm.cs, col);
}
// C[bz] of a strided batch (element strides count floats for FP32 C)
__device__ __forceinline__ double* cbase(double* C, long bz, long sC,
                                         int c32) {
  return c32 ? (double*)((float*)C + bz * sC) : C + bz * sC;
}
// element idx of C, FP64 or FP32 storage
__device__ __forceinline__ double cload(const double* C, long idx, int c32) {
  return c32 ? (double)((const float*)C)[idx] : C[idx];
}
__device__ __forceinline__ void cstore(double* C, long idx, double v,
                                       int c32) {
  if (c32)
    ((float*)C)[idx] = (float)v;
  else
    C[idx] = v;
}

// Epilogue of a tile of 16 x 16 MFMA blocks: out = alpha acc + beta out
// (one split) or the partial sums (split K).  Register r of block (i, j)
// holds row 4 (l / 16) + r (FP32 and BF16 layouts, L32) or l / 16 + 4 r
// (FP64) and column l % 16.  With beta != 0 the C values of a block row are
// all loaded before any of them is stored: the compiler cannot tell that a
// store does not alias a later load, and would wait one memory round trip
// per element.
template <bool L32, int TM, int TN, typename V, typename PT>
__device__ __forceinline__ void store_tile(const V (&acc)[TM][TN], int lane,
                                           int r0, int c0, int M, int N,
                                           double alpha, double beta,
                                           double* out, long ldc, PT* pout,
                                           int splits, const CMap& cm) {
  // offsets of this lane's TN columns in C (the layout cm describes)
  long coff[TN];
  if (splits == 1) {
#pragma unroll
    for (int j = 0; j < TN; ++j)
      coff[j] = cmap_col(cm, c0 + j * 16 + (lane & 15));
  }
#pragma unroll
  for (int i = 0; i < TM; ++i) {
    long roff[4];
    if (splits == 1) {
#pragma unroll
      for (int r = 0; r < 4; ++r)
        roff[r] = cmap_row(
            cm, r0 + i * 16 + (L32 ? 4 * (lane >> 4) + r : (lane >> 4) + 4 * r),
            ldc);
    }
    double cv[TN][4];
    if (splits == 1 && beta != 0.0) {
#pragma unroll
      for (int j = 0; j < TN; ++j)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int row =
              r0 + i * 16 + (L32 ? 4 * (lane >> 4) + r : (lane >> 4) + 4 * r);
          const int col = c0 + j * 16 + (lane & 15);
          cv[j][r] =
              row < M && col < N ? cload(out, roff[r] + coff[j], cm.c32) : 0.0;
        }
    }
#pragma unroll
    for (int j = 0; j < TN; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row =
            r0 + i * 16 + (L32 ? 4 * (lane >> 4) + r : (lane >> 4) + 4 * r);
        const int col = c0 + j * 16 + (lane & 15);
        if (row < M && col < N) {
          if (splits == 1) {
            double v = alpha * (double)acc[i][j][r];
            if (beta != 0.0) v += beta * cv[j][r];
            cstore(out, roff[r] + coff[j], v, cm.c32);
          } else {
            pout[(long)row * N + col] = acc[i][j][r];
          }
        }
      }
  }
}

template <typename TI, int BM, int BN, int WM, int WN, bool TA, bool TB,
          bool F32, bool KM, int BK>
__global__ __launch_bounds__(256, 2) void gemm_kernel(
    int M, int N, int K, double alpha, const void* __restrict__ Av,
    long lda, long sA, const double* __restrict__ B, long ldb, long sB,
    double beta, double* __restrict__ C, long ldc, long sC, int tiles_n,
    int splits, int kchunk, void* __restrict__ part, int use_ptrs,
    PtrArgs ptrs, CMap cm) {
  static_assert(WM * WN == 4, "4 waves");
  using T = typename std::conditional<F32, float, double>::type;
  using V4 = typename std::conditional<F32, f32x4, f64x4>::type;
  constexpr int WTM = BM / WM, WTN = BN / WN;
  constexpr int TM = WTM / 16, TN = WTN / 16;
  constexpr int AE = BM * BK / 256, BE = BK * BN / 256;
  // A: k-major [BK][BM + MPAD] when TA (or KM), else m-major [BM][BK + KPAD]
  constexpr bool AK = TA || KM, BKM = !TB || KM;
  constexpr int KPAD = Pad<F32>::K;
  constexpr int A_ROWS = AK ? BK : BM;
  constexpr int A_COLS = AK ? BM + Pad<F32>::M(BM) : BK + KPAD;
  constexpr int B_ROWS = BKM ? BK : BN;
  constexpr int B_COLS = BKM ? BN + Pad<F32>::M(BN) : BK + KPAD;
  __shared__ T As[2][A_ROWS][A_COLS];
  __shared__ T Bs[2][B_ROWS][B_COLS];

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave / WN, wn = wave % WN;
  // Workgroups are dealt round-robin to the 8 XCDs, each with its own L2.
  // Renumber them so that XCD x works on the x-th contiguous range of
  // (tile, split, batch) indices: its concurrent workgroups share operand
  // rows and columns in its L2 instead of every XCD fetching all of them.
  const int gx = gridDim.x;
  const int total = gx * gridDim.y;
  const int lin = blockIdx.x + gx * blockIdx.y;
  const int q8 = total / 8, r8 = total % 8, xcd = lin % 8;
  const int vid = xcd * q8 + min(xcd, r8) + lin / 8;
  const int bx = vid % gx, by = vid / gx;
  const int bz = by / splits, sp = by % splits;
  const TI* A = use_ptrs ? (const TI*)ptrs.a[bz] : (const TI*)Av + (long)bz * sA;
  B = use_ptrs ? ptrs.b[bz] : B + (long)bz * sB;
  const int m0 = (bx / tiles_n) * BM;
  const int n0 = (bx % tiles_n) * BN;
  const int kbeg = sp * kchunk;
  const int kend = min(K, kbeg + kchunk);

  // raw FP64 values stay in registers until the LDS store, so the global
  // loads remain in flight across the MFMAs of the current slice
  TI ra[AE];
  double rb[BE];
  auto load = [&](int kb) {
#pragma unroll
    for (int i = 0; i < AE; ++i) {
      const int e = tid + i * 256;
      const int mm = TA ? e % BM : e / BK, kk = TA ? e / BM : e % BK;
      const int gm = m0 + mm, gk = kb + kk;
      TI v = 0;
      if (gm < M && gk < kend)
        v = TA ? A[(long)gk * lda + gm] : A[(long)gm * lda + gk];
      ra[i] = v;
    }
#pragma unroll
    for (int i = 0; i < BE; ++i) {
      const int e = tid + i * 256;
      const int nn = TB ? e / BK : e % BN, kk = TB ? e % BK : e / BN;
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
      const int mm = TA ? e % BM : e / BK, kk = TA ? e / BM : e % BK;
      if (AK)
        As[buf][kk][mm] = (T)ra[i];
      else
        As[buf][mm][kk] = (T)ra[i];
    }
#pragma unroll
    for (int i = 0; i < BE; ++i) {
      const int e = tid + i * 256;
      const int nn = TB ? e / BK : e % BN, kk = TB ? e % BK : e / BN;
      if (BKM)
        Bs[buf][kk][nn] = (T)rb[i];
      else
        Bs[buf][nn][kk] = (T)rb[i];
    }
  };

  V4 acc[TM][TN];
#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int j = 0; j < TN; ++j) acc[i][j] = V4{0, 0, 0, 0};

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
      const int kq = k4 + (lane >> 4);
      T a[TM], b[TN];
#pragma unroll
      for (int i = 0; i < TM; ++i) {
        const int r = wm * WTM + i * 16 + (lane & 15);
        a[i] = AK ? As[buf][kq][r] : As[buf][r][kq];
      }
#pragma unroll
      for (int j = 0; j < TN; ++j) {
        const int c = wn * WTN + j * 16 + (lane & 15);
        b[j] = BKM ? Bs[buf][kq][c] : Bs[buf][c][kq];
      }
#pragma unroll
      for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 0; j < TN; ++j) {
          if constexpr (F32)
            acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(
                a[i], b[j], acc[i][j], 0, 0, 0);
          else
            acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(
                a[i], b[j], acc[i][j], 0, 0, 0);
        }
    }
    if (more) store(buf ^ 1);
    __syncthreads();
    buf ^= 1;
  }

  // epilogue: direct (splits == 1) or partial tile (split K), the partial
  // sums kept in the accumulator's type (exact)
  double* out = use_ptrs ? ptrs.c[bz] : cbase(C, bz, sC, cm.c32);
  T* pout = (T*)part + ((long)sp * (gridDim.y / splits) + bz) * (long)M * N;
  store_tile<F32>(acc, lane, m0 + wm * WTM, n0 + wn * WTN, M, N, alpha, beta,
                  out, ldc, pout, splits, cm);
}

// BF16x3 arithmetic: every FP64 operand x is split into x_hi = bf16(x) and
// x_lo = bf16(x - x_hi) when staged into LDS, and each product is
// a_hi b_hi + a_hi b_lo + a_lo b_hi on v_mfma_f32_16x16x32_bf16 with FP32
// accumulation (about 16 significant bits per product, the a_lo b_lo term
// being below that).  K slices of 32; the tiles are kept row-major along K
// in LDS (A as [BM][K], B as [BN][K]) so that each lane fetches its 8
// consecutive K values with one 16-byte read.  One LDS buffer: the next
// slice is loaded into registers while the MFMAs of the current one run.
// Lane layout of the 16x16x32 BF16 MFMA (checked on gfx950): lane l supplies
// A[l%16][8(l/16) + t] and B[8(l/16) + t][l%16], t = 0..7; the result holds
// D[4(l/16) + r][l%16] in register r.
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

template <typename TI, int BM, int BN, int WM, int WN, bool TA, bool TB,
          int NP>
__global__ __launch_bounds__(256, 2) void gemm_bf16x3_kernel(
    int M, int N, int K, double alpha, const void* __restrict__ Av,
    long lda, long sA, const double* __restrict__ B, long ldb, long sB,
    double beta, double* __restrict__ C, long ldc, long sC, int tiles_n,
    int splits, int kchunk, void* __restrict__ part, int use_ptrs,
    PtrArgs ptrs, CMap cm) {
  static_assert(WM * WN == 4, "4 waves");
  constexpr int BK = 32, KP = BK + 8;  // 80-byte rows, 16-byte aligned reads
  constexpr int WTM = BM / WM, WTN = BN / WN;
  constexpr int TM = WTM / 16, TN = WTN / 16;
  constexpr int AE = BM * BK / 256, BE = BK * BN / 256;
  __shared__ __attribute__((aligned(16))) __bf16 Ah[BM][KP];
  __shared__ __attribute__((aligned(16))) __bf16 Al[BM][KP];
  __shared__ __attribute__((aligned(16))) __bf16 Bh[BN][KP];
  __shared__ __attribute__((aligned(16))) __bf16 Bl[BN][KP];

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave / WN, wn = wave % WN;
  const int gx = gridDim.x;
  const int total = gx * gridDim.y;
  const int lin = blockIdx.x + gx * blockIdx.y;
  const int q8 = total / 8, r8 = total % 8, xcd = lin % 8;
  const int vid = xcd * q8 + min(xcd, r8) + lin / 8;
  const int bx = vid % gx, by = vid / gx;
  const int bz = by / splits, sp = by % splits;
  const TI* A = use_ptrs ? (const TI*)ptrs.a[bz] : (const TI*)Av + (long)bz * sA;
  B = use_ptrs ? ptrs.b[bz] : B + (long)bz * sB;
  const int m0 = (bx / tiles_n) * BM;
  const int n0 = (bx % tiles_n) * BN;
  const int kbeg = sp * kchunk;
  const int kend = min(K, kbeg + kchunk);

  TI ra[AE];
  double rb[BE];
  auto load = [&](int kb) {
#pragma unroll
    for (int i = 0; i < AE; ++i) {
      const int e = tid + i * 256;
      const int mm = TA ? e % BM : e / BK, kk = TA ? e / BM : e % BK;
      const int gm = m0 + mm, gk = kb + kk;
      TI v = 0;
      if (gm < M && gk < kend)
        v = TA ? A[(long)gk * lda + gm] : A[(long)gm * lda + gk];
      ra[i] = v;
    }
#pragma unroll
    for (int i = 0; i < BE; ++i) {
      const int e = tid + i * 256;
      const int nn = TB ? e / BK : e % BN, kk = TB ? e % BK : e / BN;
      const int gk = kb + kk, gn = n0 + nn;
      double v = 0.0;
      if (gk < kend && gn < N)
        v = TB ? B[(long)gn * ldb + gk] : B[(long)gk * ldb + gn];
      rb[i] = v;
    }
  };
  auto split = [](auto v, __bf16& h, __bf16& l) {
    const float f = (float)v;
    h = (__bf16)f;
    if constexpr (NP == 3) l = (__bf16)(f - (float)h);
  };
  auto store = [&]() {
#pragma unroll
    for (int i = 0; i < AE; ++i) {
      const int e = tid + i * 256;
      const int mm = TA ? e % BM : e / BK, kk = TA ? e / BM : e % BK;
      split(ra[i], Ah[mm][kk], Al[mm][kk]);
    }
#pragma unroll
    for (int i = 0; i < BE; ++i) {
      const int e = tid + i * 256;
      const int nn = TB ? e / BK : e % BN, kk = TB ? e % BK : e / BN;
      split(rb[i], Bh[nn][kk], Bl[nn][kk]);
    }
  };

  f32x4 acc[TM][TN];
#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int j = 0; j < TN; ++j) acc[i][j] = f32x4{0, 0, 0, 0};

  if (kbeg < kend) {
    load(kbeg);
    store();
  }
  __syncthreads();
  const int kq = 8 * (lane >> 4);
  for (int kb = kbeg; kb < kend; kb += BK) {
    const bool more = kb + BK < kend;
    if (more) load(kb + BK);
    bf16x8 ah[TM], al[TM];
#pragma unroll
    for (int i = 0; i < TM; ++i) {
      const int r = wm * WTM + i * 16 + (lane & 15);
      ah[i] = *(const bf16x8*)&Ah[r][kq];
      if constexpr (NP == 3) al[i] = *(const bf16x8*)&Al[r][kq];
    }
#pragma unroll
    for (int j = 0; j < TN; ++j) {
      const int c = wn * WTN + j * 16 + (lane & 15);
      const bf16x8 bh = *(const bf16x8*)&Bh[c][kq];
#pragma unroll
      for (int i = 0; i < TM; ++i)
        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[i], bh,
                                                            acc[i][j], 0, 0, 0);
      if constexpr (NP == 3) {
        const bf16x8 bl = *(const bf16x8*)&Bl[c][kq];
#pragma unroll
        for (int i = 0; i < TM; ++i) {
          acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(
              ah[i], bl, acc[i][j], 0, 0, 0);
          acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(
              al[i], bh, acc[i][j], 0, 0, 0);
        }
      }
    }
    __syncthreads();
    if (more) store();
    __syncthreads();
  }

  // split K: FP32 partial sums (exact copies of the accumulators)
  double* out = use_ptrs ? ptrs.c[bz] : cbase(C, bz, sC, cm.c32);
  float* pout =
      (float*)part + ((long)sp * (gridDim.y / splits) + bz) * (long)M * N;
  store_tile<true>(acc, lane, m0 + wm * WTM, n0 + wn * WTN, M, N, alpha,
                   beta, out, ldc, pout, splits, cm);
}

// FP32 products with direct global-to-LDS loads (`global_load_lds_dwordx4`:
// lane l of a wave writes its 16 bytes at LDS base + 16 l, checked on
// gfx950), for FP64 operands whose contiguous extent and leading dimension
// are even and whose addresses are 16-byte aligned (`lds_ok`).  The tiles
// stay FP64 in LDS and are rounded to FP32 when read into the MFMA
// operands, so the loads need no registers and no LDS stores: the loads of
// slice t + 1 are in flight while the MFMAs of slice t run, without the
// register staging of gemm_kernel.  128 x 128 tiles, 2 x 2 waves, BK = 16,
// two LDS stages of 2 x 16 KB.  The products, their order and the FP32
// rounding are those of gemm_kernel's 128 x 128 FP32 instantiation.
typedef __attribute__((address_space(3))) void lds_void;

// LDS bytes of the two stages of a 128 x BN tile with A stored in TI
template <typename TI>
constexpr size_t lds_stage_bytes(int BN) {
  return 2 * 16 * (128 * sizeof(TI) + 8 * BN);
}

template <typename TI, int BN, int WM, int WN, bool TA, bool TB>
__global__ __launch_bounds__(256, 2) void gemm_f32_lds_kernel(
    int M, int N, int K, double alpha, const void* __restrict__ Av,
    long lda, long sA, const double* __restrict__ B0, long ldb, long sB,
    double beta, double* __restrict__ C, long ldc, long sC, int tiles_n,
    int splits, int kchunk, void* __restrict__ part, int use_ptrs,
    PtrArgs ptrs, CMap cm) {
  static_assert(WM * WN == 4, "4 waves");
  constexpr int BM = 128, BK = 16, NS = 2;
  constexpr int WTM = BM / WM, WTN = BN / WN, TM = WTM / 16, TN = WTN / 16;
  constexpr int TEA = BM * BK, TEB = BK * BN;  // elements per operand tile
  constexpr int EA = 16 / sizeof(TI);          // A elements per 16 bytes
  constexpr int CA = BK / EA;                  // chunks per K row of A
  constexpr int NIA = TEA / (64 * EA);         // 1 KB loads of an A tile
  constexpr int NAW = NIA / 4;                 // per wave
  constexpr int NIB = TEB / 128;               // 1 KB loads of a B tile
  constexpr int NBW = (NIB + 3) / 4;           // per wave (some idle)
  static_assert(NIA % 4 == 0, "A loads per wave");
  extern __shared__ __attribute__((aligned(16))) double lds_tiles[];
  TI* const As0 = (TI*)lds_tiles;
  double* const Bs0 = (double*)(As0 + TEA);
  TI* const As1 = (TI*)(Bs0 + TEB);
  double* const Bs1 = (double*)(As1 + TEA);
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave / WN, wn = wave % WN;
  const int gx = gridDim.x;
  const int total = gx * gridDim.y;
  const int lin = blockIdx.x + gx * blockIdx.y;
  const int q8 = total / 8, r8 = total % 8, xcd = lin % 8;
  const int vid = xcd * q8 + min(xcd, r8) + lin / 8;
  const int bx = vid % gx, by = vid / gx;
  const int bz = by / splits, sp = by % splits;
  const TI* A = use_ptrs ? (const TI*)ptrs.a[bz] : (const TI*)Av + (long)bz * sA;
  const double* B = use_ptrs ? ptrs.b[bz] : B0 + (long)bz * sB;
  const int m0 = (bx / tiles_n) * BM;
  const int n0 = (bx % tiles_n) * BN;
  const int kbeg = sp * kchunk;
  const int kend = min(K, kbeg + kchunk);
  // Loads of 64 x 16 bytes: wave w issues A loads q = w + 4 j (NIA of
  // them) and B loads q = w + 4 j (NIB), lane l taking chunk L = 64 q + l
  // of the tile.  K-contiguous tiles (A not transposed, B transposed) hold
  // row r's K values in C chunks (C = 16 / elements per chunk) at chunks
  // C r + (c ^ (r mod C)) (the XOR spreads one K column of consecutive rows
  // over the banks); MN-contiguous tiles hold K row k at chunks X k / E + cc
  // (X = BM or BN, E elements per chunk).  Rows and K beyond the operand
  // are clamped into it (finite values that only reach discarded outputs,
  // or are zeroed on A's side in fetch).
  long aoff[NAW], boff[NBW];
  int ak[NAW], bk[NBW];  // K offset of the chunk within the slice
#pragma unroll
  for (int j = 0; j < NAW; ++j) {
    const int L = 64 * (wave + 4 * j) + lane;
    if (!TA) {
      const int r = L / CA, c = (L % CA) ^ (r % CA);
      aoff[j] = (long)min(m0 + r, M - 1) * lda;
      ak[j] = EA * c;
    } else {
      const int k = L / (BM / EA), cc = L % (BM / EA);
      aoff[j] = min(m0 + EA * cc, M - EA);
      ak[j] = k;
    }
  }
#pragma unroll
  for (int j = 0; j < NBW; ++j) {
    const int L = 64 * min(wave + 4 * j, NIB - 1) + lane;
    if (TB) {
      const int r = L >> 3, c = (L & 7) ^ (r & 7);
      boff[j] = (long)min(n0 + r, N - 1) * ldb;
      bk[j] = 2 * c;
    } else {
      const int k = L / (BN / 2), cc = L % (BN / 2);
      boff[j] = min(n0 + 2 * cc, N - 2);
      bk[j] = k;
    }
  }
  auto issue = [&](TI* as, double* bs, int kb) {
#pragma unroll
    for (int j = 0; j < NAW; ++j) {
      const TI* ga;
      if (!TA)
        ga = A + aoff[j] + min(kb + ak[j], K - EA);
      else
        ga = A + (long)min(kb + ak[j], K - 1) * lda + aoff[j];
      __builtin_amdgcn_global_load_lds(
          (const void*)ga, (lds_void*)(as + 64 * EA * (wave + 4 * j)), 16, 0,
          0);
    }
#pragma unroll
    for (int j = 0; j < NBW; ++j) {
      if (wave + 4 * j < NIB) {  // wave-uniform
        const double* gb;
        if (TB)
          gb = B + boff[j] + min(kb + bk[j], K - 2);
        else
          gb = B + (long)min(kb + bk[j], K - 1) * ldb + boff[j];
        __builtin_amdgcn_global_load_lds(
            (const void*)gb, (lds_void*)(bs + 128 * (wave + 4 * j)), 16, 0,
            0);
      }
    }
  };
  f32x4 acc[TM][TN];
#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int j = 0; j < TN; ++j) acc[i][j] = f32x4{0, 0, 0, 0};
  // all MFMA operands of one slice, read from LDS and rounded to FP32
  float fa[BK / 4][TM], fb[BK / 4][TN];
  auto fetch = [&](const TI* as, const double* bs, int kb) {
    const int klim = kend - kb;
#pragma unroll
    for (int s4 = 0; s4 < BK / 4; ++s4) {
      const int kq = 4 * s4 + (lane >> 4);
#pragma unroll
      for (int i = 0; i < TM; ++i) {
        const int r = wm * WTM + i * 16 + (lane & 15);
        const TI v = !TA ? as[(r * CA + ((kq / EA) ^ (r % CA))) * EA + kq % EA]
                         : as[kq * BM + r];
        fa[s4][i] = kq < klim ? (float)v : 0.0f;
      }
#pragma unroll
      for (int j = 0; j < TN; ++j) {
        const int n = wn * WTN + j * 16 + (lane & 15);
        const double v = TB ? bs[(n * 8 + ((kq >> 1) ^ (n & 7))) * 2 + (kq & 1)]
                            : bs[kq * BN + n];
        fb[s4][j] = (float)v;
      }
    }
  };
  auto mma = [&]() {
    // raised issue priority while the MFMAs run, so that a wave of another
    // workgroup in its load and conversion phase fills the gaps instead
    // of delaying the MFMA chain
    __builtin_amdgcn_s_setprio(1);
#pragma unroll
    for (int s4 = 0; s4 < BK / 4; ++s4)
#pragma unroll
      for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 0; j < TN; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(
              fa[s4][i], fb[s4][j], acc[i][j], 0, 0, 0);
    __builtin_amdgcn_s_setprio(0);
  };
  // Two stages.  Slice t: wait for its loads (each wave its own, then a
  // barrier), read all its operands into registers, start the loads of
  // slice t + 1 into the other stage (every wave has finished reading that
  // stage: it passed this barrier after its reads of slice t - 1), then the
  // MFMAs of slice t run while those loads are in flight.
  static_assert(NS == 2, "two stages");
  auto bar = []() {
    asm volatile("" ::: "memory");
    __builtin_amdgcn_s_barrier();
    asm volatile("" ::: "memory");
  };
  constexpr int W_VM0 = 0xf70, W_LGKM0 = 0xc07f;
  const int T = kbeg < kend ? (kend - kbeg + BK - 1) / BK : 0;
  if (T > 0) issue(As0, Bs0, kbeg);
  for (int t = 0; t < T; t += 2) {
    __builtin_amdgcn_s_waitcnt(W_VM0);
    bar();
    fetch(As0, Bs0, kbeg + t * BK);
    __builtin_amdgcn_s_waitcnt(W_LGKM0);
    if (t + 1 < T) issue(As1, Bs1, kbeg + (t + 1) * BK);
    mma();
    if (t + 1 >= T) break;
    __builtin_amdgcn_s_waitcnt(W_VM0);
    bar();
    fetch(As1, Bs1, kbeg + (t + 1) * BK);
    __builtin_amdgcn_s_waitcnt(W_LGKM0);
    if (t + 2 < T) issue(As0, Bs0, kbeg + (t + 2) * BK);
    mma();
  }
  double* out = use_ptrs ? ptrs.c[bz] : cbase(C, bz, sC, cm.c32);
  float* pout = (float*)part + ((long)sp * (gridDim.y / splits) + bz) * (long)M * N;
  store_tile<true>(acc, lane, m0 + wm * WTM, n0 + wn * WTN, M, N, alpha,
                   beta, out, ldc, pout, splits, cm);
}

// part layout [S][batch][M][N] (FP64, or FP32 for FP32 accumulators);
// C[b] = alpha sum_s part[s][b] + beta C[b], summed in FP64 in the order of
// s.  Grid (element groups, batch entry): each thread sums V consecutive
// elements of one row (V = 4 when N is a multiple of 4, then every split's
// four partial sums are one 16-byte load, or two), so the batch entry, row
// and column are found once per thread, not per element.
template <typename PT, int V>
__global__ __launch_bounds__(256) void splitk_sum_kernel(
    const PT* __restrict__ part, int S, int M, int N, double alpha,
    double beta, double* __restrict__ C, long ldc, long sC, int use_ptrs,
    PtrArgs ptrs, CMap cm) {
  const int b = blockIdx.y;
  const long mn = (long)M * N;
  const long i0 = ((long)blockIdx.x * blockDim.x + threadIdx.x) * V;
  if (i0 >= mn) return;
  const long sstride = (long)gridDim.y * mn;
  const PT* p = part + (long)b * mn + i0;
  double v[V];
#pragma unroll
  for (int q = 0; q < V; ++q) v[q] = 0.0;
#pragma unroll 4
  for (int s = 0; s < S; ++s) {
    const PT* ps = p + (long)s * sstride;
    if constexpr (V == 4 && sizeof(PT) == 4) {
      const float4 t = *reinterpret_cast<const float4*>(ps);
      v[0] += (double)t.x;
      v[1] += (double)t.y;
      v[2] += (double)t.z;
      v[3] += (double)t.w;
    } else if constexpr (V == 4) {
      const double2 t0 = *reinterpret_cast<const double2*>(ps);
      const double2 t1 = *reinterpret_cast<const double2*>(ps + 2);
      v[0] += t0.x;
      v[1] += t0.y;
      v[2] += t1.x;
      v[3] += t1.y;
    } else {
      v[0] += (double)ps[0];
    }
  }
  const int r = (int)(i0 / N), c0 = (int)(i0 - (long)r * N);
  double* base = use_ptrs ? ptrs.c[b] : cbase(C, b, sC, cm.c32);
  const long roff = cmap_row(cm, r, ldc);
#pragma unroll
  for (int q = 0; q < V; ++q) {
    const long off = roff + cmap_col(cm, c0 + q);
    double o = alpha * v[q];
    if (beta != 0.0) o += beta * cload(base, off, cm.c32);
    cstore(base, off, o, cm.c32);
  }
}

// BF16x3 operands split once per launch.  A large product reads every
// element of A in N / BN column tiles and every element of B in M / BM row
// tiles; converting at every read makes gemm_bf16x3_kernel VALU-bound
// (about 16 VALU instructions per MFMA).  For those products each operand
// is split once into hi and lo planes, rows zero-padded to the tile size
// and K to a multiple of 32, stored as 16 x 32 blocks of 1 KB
// ([batch][Rp/16][Kp/32][16][32], so that one wave's 64 16-byte loads of a
// K slice read one contiguous block), and the product kernel copies the
// planes into LDS with 16-byte moves.  The split
// values (x -> fl32(x) -> hi = bf16, lo = bf16(fl32(x) - hi)) and the MFMA
// sequence are those of gemm_bf16x3_kernel.
struct SplitArgs {
  const void* src[MAXP];  // per batch entry
  long ld;                // source leading dimension
  int R, K, Rp, Kp;       // operand rows x K, padded extents
  __bf16* hi;
  __bf16* lo;
};

// element (r, k) of the operand: src[k * ld + r] when TRANS, else
// src[r * ld + k]; 32 x 32 tiles through LDS so that reads are coalesced
// along the source's contiguous index and writes along K
template <typename TI, bool TRANS>
__global__ __launch_bounds__(256) void split_bf16_kernel(SplitArgs a) {
  __shared__ float tile[32][33];
  const int bz = blockIdx.z;
  const TI* src = (const TI*)a.src[bz];
  const int k0 = blockIdx.x * 32, r0 = blockIdx.y * 32;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const int u = ty + 8 * j;
    const int rr = TRANS ? tx : u, kk = TRANS ? u : tx;
    const int r = r0 + rr, k = k0 + kk;
    float v = 0.0f;
    if (r < a.R && k < a.K)
      v = (float)(TRANS ? src[(long)k * a.ld + r] : src[(long)r * a.ld + k]);
    tile[rr][kk] = v;
  }
  __syncthreads();
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const int rr = ty + 8 * j, r = r0 + rr, k = k0 + tx;
    if (r < a.Rp && k < a.Kp) {
      const float f = tile[rr][tx];
      const __bf16 h = (__bf16)f;
      const long o = (long)bz * a.Rp * a.Kp +
                     ((long)(r >> 4) * (a.Kp >> 5) + (k >> 5)) * 512 +
                     (r & 15) * 32 + (k & 31);
      a.hi[o] = h;
      if (a.lo) a.lo[o] = (__bf16)(f - (float)h);
    }
  }
}

// C[b] = alpha A B + beta C from split planes A (Mp x Kp), B (Np x Kp)
// (block layout above); tiles BM x BN, K slices of 32, LDS in the layout
// of gemm_bf16x3_kernel; split K and XCD numbering as there.
template <int BM, int BN, int WM, int WN, int NP>
__global__ __launch_bounds__(256, 2) void gemm_bf16x3_ps_kernel(
    int M, int N, int Kp, double alpha, const __bf16* __restrict__ Ah,
    const __bf16* __restrict__ Al, long sA, const __bf16* __restrict__ Bh,
    const __bf16* __restrict__ Bl, long sB, double beta,
    double* __restrict__ C, long ldc, long sC, int tiles_n, int splits,
    int kchunk, void* __restrict__ part, int use_ptrs, PtrArgs ptrs, CMap cm) {
  static_assert(WM * WN == 4, "4 waves");
  constexpr int BK = 32, KP = BK + 8;
  constexpr int WTM = BM / WM, WTN = BN / WN;
  constexpr int TM = WTM / 16, TN = WTN / 16;
  // 16-byte chunks (8 bf16) of one slice: rows x 4 per plane
  constexpr int AC = (BM * 4 + 255) / 256, BC = (BN * 4 + 255) / 256;
  // one LDS buffer (36 KB at 128 x 96): four workgroups fit a CU, which
  // hides more latency than double buffering at two
  __shared__ __attribute__((aligned(16))) __bf16 Ahs[1][BM][KP];
  __shared__ __attribute__((aligned(16))) __bf16 Als[1][BM][KP];
  __shared__ __attribute__((aligned(16))) __bf16 Bhs[1][BN][KP];
  __shared__ __attribute__((aligned(16))) __bf16 Bls[1][BN][KP];

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave / WN, wn = wave % WN;
  const int gx = gridDim.x;
  const int total = gx * gridDim.y;
  const int lin = blockIdx.x + gx * blockIdx.y;
  const int q8 = total / 8, r8 = total % 8, xcd = lin % 8;
  const int vid = xcd * q8 + min(xcd, r8) + lin / 8;
  const int bx = vid % gx, by = vid / gx;
  const int bz = by / splits, sp = by % splits;
  const int m0 = (bx / tiles_n) * BM;
  const int n0 = (bx % tiles_n) * BN;
  const int kbeg = sp * kchunk;
  const int kend = min(Kp, kbeg + kchunk);
  // planes in 16 x 32 blocks: row block rb, K block kb of a plane start at
  // (rb * Kp/32 + kb) * 512
  Ah += (long)bz * sA + (long)(m0 >> 4) * (Kp >> 5) * 512;
  Al += (long)bz * sA + (long)(m0 >> 4) * (Kp >> 5) * 512;
  Bh += (long)bz * sB + (long)(n0 >> 4) * (Kp >> 5) * 512;
  Bl += (long)bz * sB + (long)(n0 >> 4) * (Kp >> 5) * 512;
  const long rbs = (long)(Kp >> 5) * 512;  // row-block stride

  // 16-byte chunk c of a slice: K quarter q = c % 4 of row ps_row(c); the
  // 16 lanes of one LDS store take rows r, r+4, r+8, r+12 (80-byte rows:
  // 20 r mod 64 covers the 64 banks in four disjoint runs of 16)
  auto ps_row = [](int c) {
    return (c >> 6) * 16 + ((c >> 2) & 3) * 4 + ((c >> 4) & 3);
  };
  // staging registers, one array per plane (plain loops, so that they
  // stay in registers)
  u32x4 rah[AC], ral[AC], rbh[BC], rbl[BC];
#define PS_LOAD(kb)                                                        \
  {                                                                        \
    _Pragma("unroll") for (int i = 0; i < AC; ++i) {                       \
      const int c = tid + i * 256, row = ps_row(c), q = c & 3;                \
      if (c < BM * 4) {                                                    \
        const long o = (row >> 4) * rbs + ((kb) >> 5) * 512 +              \
                       (row & 15) * 32 + 8 * q;                            \
        rah[i] = *(const u32x4*)(Ah + o);                                  \
        if constexpr (NP == 3) ral[i] = *(const u32x4*)(Al + o);           \
      }                                                                    \
    }                                                                      \
    _Pragma("unroll") for (int i = 0; i < BC; ++i) {                       \
      const int c = tid + i * 256, row = ps_row(c), q = c & 3;                \
      if (c < BN * 4) {                                                    \
        const long o = (row >> 4) * rbs + ((kb) >> 5) * 512 +              \
                       (row & 15) * 32 + 8 * q;                            \
        rbh[i] = *(const u32x4*)(Bh + o);                                  \
        if constexpr (NP == 3) rbl[i] = *(const u32x4*)(Bl + o);           \
      }                                                                    \
    }                                                                      \
  }
#define PS_STORE()                                                         \
  {                                                                        \
    _Pragma("unroll") for (int i = 0; i < AC; ++i) {                       \
      const int c = tid + i * 256, row = ps_row(c), q = c & 3;                \
      if (c < BM * 4) {                                                    \
        *(u32x4*)&Ahs[0][row][8 * q] = rah[i];                             \
        if constexpr (NP == 3) *(u32x4*)&Als[0][row][8 * q] = ral[i];      \
      }                                                                    \
    }                                                                      \
    _Pragma("unroll") for (int i = 0; i < BC; ++i) {                       \
      const int c = tid + i * 256, row = ps_row(c), q = c & 3;                \
      if (c < BN * 4) {                                                    \
        *(u32x4*)&Bhs[0][row][8 * q] = rbh[i];                             \
        if constexpr (NP == 3) *(u32x4*)&Bls[0][row][8 * q] = rbl[i];      \
      }                                                                    \
    }                                                                      \
  }

  f32x4 acc[TM][TN];
#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int j = 0; j < TN; ++j) acc[i][j] = f32x4{0, 0, 0, 0};

  if (kbeg < kend) {
    PS_LOAD(kbeg);
    PS_STORE();
  }
  __syncthreads();
  const int kq = 8 * (lane >> 4);
  constexpr int buf = 0;
  for (int kb = kbeg; kb < kend; kb += BK) {
    const bool more = kb + BK < kend;
    if (more) PS_LOAD(kb + BK);
    bf16x8 ah[TM], al[TM];
#pragma unroll
    for (int i = 0; i < TM; ++i) {
      const int r = wm * WTM + i * 16 + (lane & 15);
      ah[i] = *(const bf16x8*)&Ahs[buf][r][kq];
      if constexpr (NP == 3) al[i] = *(const bf16x8*)&Als[buf][r][kq];
    }
#pragma unroll
    for (int j = 0; j < TN; ++j) {
      const int c = wn * WTN + j * 16 + (lane & 15);
      const bf16x8 bh = *(const bf16x8*)&Bhs[buf][c][kq];
#pragma unroll
      for (int i = 0; i < TM; ++i)
        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[i], bh,
                                                            acc[i][j], 0, 0, 0);
      if constexpr (NP == 3) {
        const bf16x8 bl = *(const bf16x8*)&Bls[buf][c][kq];
#pragma unroll
        for (int i = 0; i < TM; ++i) {
          acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(
              ah[i], bl, acc[i][j], 0, 0, 0);
          acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(
              al[i], bh, acc[i][j], 0, 0, 0);
        }
      }
    }
    __syncthreads();
    if (more) PS_STORE();
    __syncthreads();
  }
#undef PS_LOAD
#undef PS_STORE

  // split K: FP32 partial sums (exact copies of the accumulators)
  double* out = use_ptrs ? ptrs.c[bz] : cbase(C, bz, sC, cm.c32);
  float* pout =
      (float*)part + ((long)sp * (gridDim.y / splits) + bz) * (long)M * N;
  store_tile<true>(acc, lane, m0 + wm * WTM, n0 + wn * WTN, M, N, alpha,
                   beta, out, ldc, pout, splits, cm);
}

struct Call {
  bool tA, tB;
  int M, N, K, batch;
  double alpha, beta;
  const void* A;  // double, or float when a32
  long lda, sA;
  const double* B;
  long ldb, sB;
  double* C;
  long ldc, sC;
  const PtrArgs* ptrs;  // null: strided batch
  bool a32 = false;     // A stored in FP32
  CMap cm{};            // layout of C (nr == 0: row major, ldc)
};

// The split-K reduction of a product (partial sums in part, S splits).
template <typename PT>
void launch_splitk_sum(Device& dev, const void* part, int S, const Call& c) {
  PtrArgs pa{};
  if (c.ptrs) pa = *c.ptrs;
  const long mn = (long)c.M * c.N;
  const bool v4 = c.N % 4 == 0;
  const long groups = v4 ? mn / 4 : mn;
  const long gx = (groups + 255) / 256;
  if (gx >= (1L << 31) || c.batch > 65535)
    throw ArgError("gemm: reduction grid too large");
  const dim3 grid((unsigned)gx, (unsigned)c.batch);
  if (v4)
    hipLaunchKernelGGL((splitk_sum_kernel<PT, 4>), grid, dim3(256), 0,
                       dev.stream, (const PT*)part, S, c.M, c.N, c.alpha,
                       c.beta, c.C, c.ldc, c.sC, c.ptrs ? 1 : 0, pa, c.cm);
  else
    hipLaunchKernelGGL((splitk_sum_kernel<PT, 1>), grid, dim3(256), 0,
                       dev.stream, (const PT*)part, S, c.M, c.N, c.alpha,
                       c.beta, c.C, c.ldc, c.sC, c.ptrs ? 1 : 0, pa, c.cm);
  IPEPS_HIP(hipGetLastError());
}

// BF16x3 product through split planes (see split_bf16_kernel): chosen when
// both operands are read by at least four tiles and the batch fits one
// pointer set
template <int BM, int BN>
bool presplit_pays(const Call& c) {
  return c.M >= 4 * BM && c.N >= 4 * BN && c.K >= 128 && c.batch <= MAXP;
}

template <int BM, int BN, int WM, int WN, int NP>
void launch_presplit(Device& dev, const Call& c) {
  auto up = [](long x, long m) { return (x + m - 1) / m * m; };
  const int Mp = (int)up(c.M, BM), Np = (int)up(c.N, BN);
  const int Kp = (int)up(c.K, 32);
  const long sA = (long)Mp * Kp, sB = (long)Np * Kp;
  // hi (and, for three products, lo) planes of A and B (bf16) in one
  // buffer
  const long np = NP == 3 ? 2 : 1;
  const long nbf = np * c.batch * (sA + sB);
  Tensor planes = dev.empty({(nbf + 3) / 4});
  __bf16* Ah = (__bf16*)planes.ptr;
  __bf16* Al = NP == 3 ? Ah + c.batch * sA : nullptr;
  __bf16* Bh = Ah + np * c.batch * sA;
  __bf16* Bl = NP == 3 ? Bh + c.batch * sB : nullptr;
  const long tm = Mp / BM, tn = Np / BN, tiles = tm * tn;
  int S = 1;
  if (tiles * c.batch < 512 && c.K >= 512) {
    S = (int)std::min<long>((512 + tiles * c.batch - 1) / (tiles * c.batch),
                            c.K / 256);
    S = std::max(1, std::min(S, 64));
  }
  int kchunk = (Kp + S - 1) / S;
  kchunk = (kchunk + 31) / 32 * 32;
  S = (Kp + kchunk - 1) / kchunk;
  Tensor part;  // FP32 partial sums
  if (S > 1) part = dev.empty({((int64_t)S * c.batch * c.M * c.N + 1) / 2});
  if (tiles >= (1L << 31) || (long)c.batch * S > 65535 ||
      Mp / 32 > 65535 || Np / 32 > 65535)
    throw ArgError("gemm: grid too large");
  if (dev.prof.on)
    dev.prof.begin(dev.stream, PROF_GEMM16, 2.0 * c.M * c.N * c.K * c.batch,
                   c.batch * ((c.a32 ? 4.0 : 8.0) * c.M * c.K +
                              8.0 * ((double)c.K * c.N +
                                     (c.beta != 0.0 ? 2.0 : 1.0) * c.M * c.N)));
  SplitArgs a{}, b{};
  const size_t ea = c.a32 ? 4 : 8;
  for (int i = 0; i < c.batch; ++i) {
    a.src[i] = c.ptrs ? c.ptrs->a[i]
                      : (const void*)((const char*)c.A + (size_t)i * c.sA * ea);
    b.src[i] = c.ptrs ? (const void*)c.ptrs->b[i]
                      : (const void*)(c.B + (size_t)i * c.sB);
  }
  a.ld = c.lda;
  a.R = c.M;
  a.K = c.K;
  a.Rp = Mp;
  a.Kp = Kp;
  a.hi = Ah;
  a.lo = Al;
  b.ld = c.ldb;
  b.R = c.N;
  b.K = c.K;
  b.Rp = Np;
  b.Kp = Kp;
  b.hi = Bh;
  b.lo = Bl;
  const dim3 ga(Kp / 32, Mp / 32, c.batch), gb(Kp / 32, Np / 32, c.batch);
  // A element (m, k): A[k lda + m] when transposed, else A[m lda + k];
  // B element (n, k): B[n ldb + k] when transposed, else B[k ldb + n]
  if (c.a32) {
    if (c.tA)
      hipLaunchKernelGGL((split_bf16_kernel<float, true>), ga, dim3(256), 0,
                         dev.stream, a);
    else
      hipLaunchKernelGGL((split_bf16_kernel<float, false>), ga, dim3(256), 0,
                         dev.stream, a);
  } else {
    if (c.tA)
      hipLaunchKernelGGL((split_bf16_kernel<double, true>), ga, dim3(256), 0,
                         dev.stream, a);
    else
      hipLaunchKernelGGL((split_bf16_kernel<double, false>), ga, dim3(256),
                         0, dev.stream, a);
  }
  if (c.tB)
    hipLaunchKernelGGL((split_bf16_kernel<double, false>), gb, dim3(256), 0,
                       dev.stream, b);
  else
    hipLaunchKernelGGL((split_bf16_kernel<double, true>), gb, dim3(256), 0,
                       dev.stream, b);
  PtrArgs pa{};
  if (c.ptrs) pa = *c.ptrs;
  hipLaunchKernelGGL((gemm_bf16x3_ps_kernel<BM, BN, WM, WN, NP>),
                     dim3((unsigned)tiles, (unsigned)(c.batch * S)),
                     dim3(256), 0, dev.stream, c.M, c.N, Kp, c.alpha, Ah, Al,
                     sA, Bh, Bl, sB, c.beta, c.C, c.ldc, c.sC, (int)tn, S,
                     kchunk, part.ptr, c.ptrs ? 1 : 0, pa, c.cm);
  if (dev.prof.on) dev.prof.end(dev.stream);
  IPEPS_HIP(hipGetLastError());
  if (S > 1) launch_splitk_sum<float>(dev, part.ptr, S, c);
}

// Split of K for a grid of tb tiles (BM x BN each; mn_batch outputs in
// all).  The workgroups (wg = tb S) are dealt over the 256 CUs, whose
// matrix cores the resident workgroups share, so the products take about
// ceil(wg / 256) times the time of one workgroup (2 BM BN kchunk flops at
// half the per-CU peak `flops_cu`), stretched by 1 + 128 / wg when few
// workgroups per CU are left to hide latency; a split also writes and
// re-reads S partial sums of `pbytes` bytes each (at 2 TB/s, about what the
// separate reduction kernel reaches).  The split minimises the sum (the
// larger split on ties), with at least 64 of K per split, at most 256
// splits and 2048 workgroups.  Against measured sweeps of the split: on the
// 8 x (2592 x 72 x 2592) products 3 splits are the fastest (101 us, 6: 105,
// 8: 110), and it picks 3; on the small 8 x (72 x 72 x 2592)
// products, which wait on memory latency slice by slice, 8 splits of 64-row
// tiles took 27 us and 27 splits of one 96-row tile take 16 us (it picks
// 27, hence the floor of 64 of K per split).
int split_k(long tb, int K, int BK, int BM, int BN, long mn_batch,
            int pbytes, double flops_cu, int& kchunk) {
  auto up = [](long x, long m) { return (x + m - 1) / m * m; };
  int best = 1;
  double best_t = -1.0;
  kchunk = (int)up(K, BK);
  if (K >= 512 && tb < 2048) {
    const long smax = std::min<long>(
        {256L, (long)K / 64, std::max<long>(1, 2048 / tb)});
    for (long s = 1; s <= smax; ++s) {
      const long kc = up((K + s - 1) / s, BK);
      const long se = (K + kc - 1) / kc;
      const long wg = tb * se;
      double t = (double)((wg + 255) / 256) * 2.0 * BM * BN * kc /
                 (0.5 * flops_cu) * (1.0 + 128.0 / wg);
      if (se > 1) t += (double)se * mn_batch * 2.0 * pbytes / 2e12;
      if (best_t < 0.0 || t <= best_t) {
        best_t = t;
        best = (int)se;
        kchunk = (int)kc;
      }
    }
  }
  return best;
}

// per-CU matrix-core peaks (flop/s): FP64, FP32, BF16x3 (three BF16
// products per product) and single BF16 products
constexpr double CU_PEAK[4] = {78.6e12 / 256, 157.3e12 / 256,
                               2.5e15 / 3 / 256, 2.5e15 / 256};

// Products with at most 4 x 4 outputs per batch entry and a long K (overlaps
// and norms of whole tensors, K up to 4 D^8): a matrix-core tile would be
// almost all padding and the split-K grid too small to stream the operands,
// so these run as FP64 FMAs on the vector units.  The K range is cut into
// S fixed chunks, one workgroup each, reduced in a fixed order (lanes by a
// butterfly, then the waves, then the chunks in small_sum_kernel), so the
// result is deterministic.
constexpr int SMALL_T = 256;
constexpr int SMALL_MAXS = 256;

template <typename TI, bool TA, bool TB>
__global__ __launch_bounds__(SMALL_T) void gemm_small_kernel(
    int M, int N, int K, const TI* __restrict__ A0, long lda, long sA,
    const double* __restrict__ B0, long ldb, long sB, int kchunk,
    double* __restrict__ part, int use_ptrs, PtrArgs ptrs) {
  const int sp = blockIdx.x, bz = blockIdx.y;
  const TI* A = use_ptrs ? (const TI*)ptrs.a[bz] : A0 + (long)bz * sA;
  const double* B = use_ptrs ? ptrs.b[bz] : B0 + (long)bz * sB;
  const int k0 = sp * kchunk, k1 = min(K, k0 + kchunk);
  double acc[4][4];
#pragma unroll
  for (int m = 0; m < 4; ++m)
#pragma unroll
    for (int n = 0; n < 4; ++n) acc[m][n] = 0.0;
  for (int k = k0 + (int)threadIdx.x; k < k1; k += SMALL_T) {
    double a[4], b[4];
#pragma unroll
    for (int m = 0; m < 4; ++m)
      a[m] = m < M ? (double)(TA ? A[(long)k * lda + m] : A[(long)m * lda + k])
                   : 0.0;
#pragma unroll
    for (int n = 0; n < 4; ++n)
      b[n] = n < N ? (TB ? B[(long)n * ldb + k] : B[(long)k * ldb + n]) : 0.0;
#pragma unroll
    for (int m = 0; m < 4; ++m)
#pragma unroll
      for (int n = 0; n < 4; ++n) acc[m][n] = fma(a[m], b[n], acc[m][n]);
  }
  __shared__ double red[SMALL_T / 64][16];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
  for (int m = 0; m < 4; ++m)
#pragma unroll
    for (int n = 0; n < 4; ++n) {
      double v = acc[m][n];
#pragma unroll
      for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
      if (lane == 0) red[w][m * 4 + n] = v;
    }
  __syncthreads();
  const int mn = M * N;
  if ((int)threadIdx.x < mn) {
    const int m = threadIdx.x / N, n = threadIdx.x % N;
    double v = 0.0;
#pragma unroll
    for (int ww = 0; ww < SMALL_T / 64; ++ww) v += red[ww][m * 4 + n];
    part[((long)sp * gridDim.y + bz) * mn + threadIdx.x] = v;
  }
}

// C[b] = alpha sum_s part[s][b] + beta C[b] for at most 16 outputs per
// batch entry, one workgroup per entry: thread t sums the chunks s = t,
// t + 256, ... and the workgroup adds the thread sums in a fixed tree
__global__ __launch_bounds__(SMALL_T) void small_sum_kernel(
    const double* __restrict__ part, int S, int M, int N, double alpha,
    double beta, double* __restrict__ C, long ldc, long sC, int use_ptrs,
    PtrArgs ptrs, CMap cm) {
  const int bz = blockIdx.x, batch = gridDim.x, mn = M * N;
  __shared__ double red[SMALL_T];
  double* Cb = use_ptrs ? ptrs.c[bz] : cbase(C, bz, sC, cm.c32);
  for (int o = 0; o < mn; ++o) {
    double v = 0.0;
    for (int sp = threadIdx.x; sp < S; sp += SMALL_T)
      v += part[((long)sp * batch + bz) * mn + o];
    red[threadIdx.x] = v;
    __syncthreads();
    for (int h = SMALL_T / 2; h > 0; h >>= 1) {
      if ((int)threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
      __syncthreads();
    }
    if (threadIdx.x == 0) {
      const long off = cmap_row(cm, o / N, ldc) + cmap_col(cm, o % N);
      double r = alpha * red[0];
      if (beta != 0.0) r += beta * cload(Cb, off, cm.c32);
      cstore(Cb, off, r, cm.c32);
    }
    __syncthreads();
  }
}

bool small_pays(const Call& c) {
  return c.M <= 4 && c.N <= 4 && c.K >= 4096;
}

void launch_small(Device& dev, const Call& c) {
  // about 16 K values per thread and chunk, at most SMALL_MAXS chunks
  int S = (int)std::min<long>(SMALL_MAXS, ((long)c.K + 16 * SMALL_T - 1) /
                                              (16 * SMALL_T));
  S = std::max(S, 1);
  const int kchunk = (c.K + S - 1) / S;
  S = (c.K + kchunk - 1) / kchunk;
  if (c.batch > 65535) throw ArgError("gemm: grid too large");
  Tensor part = dev.empty({(int64_t)S * c.batch * c.M * c.N});
  PtrArgs pa{};
  if (c.ptrs) pa = *c.ptrs;
  const int up = c.ptrs ? 1 : 0;
  const dim3 grid((unsigned)S, (unsigned)c.batch);
  auto go = [&](auto ti) {
    using TI = decltype(ti);
    const TI* A = (const TI*)c.A;
    if (!c.tA && !c.tB)
      hipLaunchKernelGGL((gemm_small_kernel<TI, false, false>), grid,
                         dim3(SMALL_T), 0, dev.stream, c.M, c.N, c.K, A, c.lda,
                         c.sA, c.B, c.ldb, c.sB, kchunk, part.ptr, up, pa);
    if (c.tA && !c.tB)
      hipLaunchKernelGGL((gemm_small_kernel<TI, true, false>), grid,
                         dim3(SMALL_T), 0, dev.stream, c.M, c.N, c.K, A, c.lda,
                         c.sA, c.B, c.ldb, c.sB, kchunk, part.ptr, up, pa);
    if (!c.tA && c.tB)
      hipLaunchKernelGGL((gemm_small_kernel<TI, false, true>), grid,
                         dim3(SMALL_T), 0, dev.stream, c.M, c.N, c.K, A, c.lda,
                         c.sA, c.B, c.ldb, c.sB, kchunk, part.ptr, up, pa);
    if (c.tA && c.tB)
      hipLaunchKernelGGL((gemm_small_kernel<TI, true, true>), grid,
                         dim3(SMALL_T), 0, dev.stream, c.M, c.N, c.K, A, c.lda,
                         c.sA, c.B, c.ldb, c.sB, kchunk, part.ptr, up, pa);
  };
  if (c.a32)
    go(float());
  else
    go(double());
  IPEPS_HIP(hipGetLastError());
  hipLaunchKernelGGL(small_sum_kernel, dim3(c.batch), dim3(SMALL_T), 0,
                     dev.stream, part.ptr, S, c.M, c.N, c.alpha, c.beta, c.C,
                     c.ldc, c.sC, up, pa, c.cm);
  IPEPS_HIP(hipGetLastError());
}

// Raises a kernel's dynamic LDS limit to `bytes` once.  Every limit the
// direct-load kernels need is raised by prime_gemm_attributes before the
// first context exists, so that no attribute changes while other host
// threads launch kernels (contexts of a serving loop); this is the fallback
// for anything not primed.
std::mutex g_lds_mu;
std::map<const void*, size_t> g_lds_done;
void allow_dyn_lds(const void* fn, size_t bytes) {
  std::lock_guard<std::mutex> lock(g_lds_mu);
  size_t& have = g_lds_done[fn];
  if (bytes <= have) return;
  IPEPS_HIP(hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize,
                                (int)bytes));
  have = bytes;
}

template <typename TI, int BN, int WM, int WN>
void prime_lds_kernels() {
  constexpr size_t lb = lds_stage_bytes<TI>(BN);
  allow_dyn_lds((const void*)gemm_f32_lds_kernel<TI, BN, WM, WN, false, false>,
                lb);
  allow_dyn_lds((const void*)gemm_f32_lds_kernel<TI, BN, WM, WN, true, false>,
                lb);
  allow_dyn_lds((const void*)gemm_f32_lds_kernel<TI, BN, WM, WN, false, true>,
                lb);
  allow_dyn_lds((const void*)gemm_f32_lds_kernel<TI, BN, WM, WN, true, true>,
                lb);
}

template <typename TI>
void prime_lds_all() {
  prime_lds_kernels<TI, 48, 4, 1>();
  prime_lds_kernels<TI, 64, 4, 1>();
  prime_lds_kernels<TI, 80, 4, 1>();
  prime_lds_kernels<TI, 96, 4, 1>();
  prime_lds_kernels<TI, 128, 2, 2>();
  prime_lds_kernels<TI, 144, 4, 1>();
}

// direct-load conditions: 16-byte aligned operands whose contiguous extent
// and leading dimension are even
bool lds_ok(const Call& c) {
  auto al = [](const void* p) { return ((uintptr_t)p & 15) == 0; };
  const int ea = c.a32 ? 4 : 2;  // A elements per 16 bytes
  const int xa = c.tA ? c.M : c.K, xb = c.tB ? c.K : c.N;
  if (xa % ea || xb % 2 || c.lda % ea || c.ldb % 2) return false;
  if (c.K < 4 || c.M < 4 || c.N < 2) return false;
  if (c.ptrs) {
    for (int i = 0; i < c.batch; ++i)
      if (!al(c.ptrs->a[i]) || !al(c.ptrs->b[i])) return false;
  } else {
    if (!al(c.A) || !al(c.B) || c.sA % ea || c.sB % 2) return false;
  }
  return true;
}

// P: 0 = FP64, 1 = FP32, 2 = BF16x3, 3 = single BF16 arithmetic
template <int BM, int BN, int WM, int WN, int P, bool LDSK = false>
void launch_cfg(Device& dev, const Call& c) {
  constexpr int NP = P == 3 ? 1 : 3;  // BF16 products per product
  if constexpr (P >= 2) {
    if (presplit_pays<BM, BN>(c)) {
      launch_presplit<BM, BN, WM, WN, NP>(dev, c);
      return;
    }
  }
  constexpr bool F32 = P == 1;
  constexpr int BK = P >= 2 ? 32 : 16;
  const long tm = (c.M + BM - 1) / BM, tn = (c.N + BN - 1) / BN;
  const long tiles = tm * tn;
  int kchunk;
  int S = split_k(tiles * c.batch, c.K, BK, BM, BN, (long)c.M * c.N * c.batch,
                  P == 0 ? 8 : 4, CU_PEAK[P], kchunk);
  // partial sums in the accumulators' type: FP64, or FP32 (FP32 and BF16x3)
  const int64_t npart = (int64_t)S * c.batch * c.M * c.N;
  Tensor part;
  if (S > 1) part = dev.empty({P == 0 ? npart : (npart + 1) / 2});
  if (tiles >= (1L << 31) || (long)c.batch * S > 65535)
    throw ArgError("gemm: grid too large");
  dim3 grid((unsigned)tiles, (unsigned)(c.batch * S));
  PtrArgs pa{};
  if (c.ptrs) pa = *c.ptrs;
  const int up = c.ptrs ? 1 : 0;
  // the profiler brackets the matrix-core kernel alone (split-K partial
  // sums are a kernel of their own), with the algorithmic 2 M N K flops
  if (dev.prof.on)
    dev.prof.begin(dev.stream,
                   P == 0 ? PROF_GEMM : (P == 1 ? PROF_GEMM32 : PROF_GEMM16),
                   2.0 * c.M * c.N * c.K * c.batch,
                   c.batch * ((c.a32 ? 4.0 : 8.0) * c.M * c.K +
                              8.0 * ((double)c.K * c.N +
                                     (c.beta != 0.0 ? 2.0 : 1.0) * c.M * c.N)),
                   P == 1 && BN == 144);
  auto go = [&](auto kern) {
    hipLaunchKernelGGL(kern, grid, dim3(256), 0, dev.stream, c.M, c.N, c.K,
                       c.alpha, c.A, c.lda, c.sA, c.B, c.ldb, c.sB, c.beta,
                       c.C, c.ldc, c.sC, (int)tn, S, kchunk, part.ptr, up, pa,
                       c.cm);
  };
  if constexpr (LDSK) {
    static_assert(P == 1 && BM == 128, "LDS kernel: FP32, 128 rows");
    auto gol = [&](auto kern, size_t lb) {
      allow_dyn_lds((const void*)kern, lb);
      hipLaunchKernelGGL(kern, grid, dim3(256), lb, dev.stream, c.M, c.N,
                         c.K, c.alpha, c.A, c.lda, c.sA, c.B, c.ldb, c.sB,
                         c.beta, c.C, c.ldc, c.sC, (int)tn, S, kchunk,
                         part.ptr, up, pa, c.cm);
    };
    auto pickl = [&](auto ti) {
      using TI = decltype(ti);
      constexpr size_t lb = lds_stage_bytes<TI>(BN);
      if (!c.tA && !c.tB)
        gol(gemm_f32_lds_kernel<TI, BN, WM, WN, false, false>, lb);
      if (c.tA && !c.tB)
        gol(gemm_f32_lds_kernel<TI, BN, WM, WN, true, false>, lb);
      if (!c.tA && c.tB)
        gol(gemm_f32_lds_kernel<TI, BN, WM, WN, false, true>, lb);
      if (c.tA && c.tB)
        gol(gemm_f32_lds_kernel<TI, BN, WM, WN, true, true>, lb);
    };
    if (c.a32)
      pickl(float());
    else
      pickl(double());
  }
  auto pick = [&](auto ti) {
    using TI = decltype(ti);
    if constexpr (P >= 2) {
      if (!c.tA && !c.tB)
        go(gemm_bf16x3_kernel<TI, BM, BN, WM, WN, false, false, NP>);
      if (c.tA && !c.tB)
        go(gemm_bf16x3_kernel<TI, BM, BN, WM, WN, true, false, NP>);
      if (!c.tA && c.tB)
        go(gemm_bf16x3_kernel<TI, BM, BN, WM, WN, false, true, NP>);
      if (c.tA && c.tB)
        go(gemm_bf16x3_kernel<TI, BM, BN, WM, WN, true, true, NP>);
    } else {
      if (!c.tA && !c.tB)
        go(gemm_kernel<TI, BM, BN, WM, WN, false, false, F32, false, BK>);
      if (c.tA && !c.tB)
        go(gemm_kernel<TI, BM, BN, WM, WN, true, false, F32, false, BK>);
      if (!c.tA && c.tB)
        go(gemm_kernel<TI, BM, BN, WM, WN, false, true, F32, false, BK>);
      if (c.tA && c.tB)
        go(gemm_kernel<TI, BM, BN, WM, WN, true, true, F32, false, BK>);
    }
  };
  if constexpr (LDSK) {
  } else if constexpr (P == 0) {
    pick(double());
  } else {
    if (c.a32)
      pick(float());
    else
      pick(double());
  }
  if (dev.prof.on) dev.prof.end(dev.stream);
  IPEPS_HIP(hipGetLastError());
  if (S > 1) {
    if constexpr (P == 0)
      launch_splitk_sum<double>(dev, part.ptr, S, c);
    else
      launch_splitk_sum<float>(dev, part.ptr, S, c);
  }
}

// Time model of a tile choice: the workgroups (tiles times the split of
// launch_cfg) are dealt over the 256 CUs, whose matrix cores the resident
// workgroups share, so a launch takes about ceil(workgroups / 256) times
// the multiply-adds of one workgroup (BM BN kchunk, padding included).
// The 128 x 144 FP32 tile runs at two waves per SIMD instead of three,
// hence the 5 % handicap where it is compared.
double tile_cost(const Call& c, int BM, int BN, int BK) {
  const long tiles = (long)((c.M + BM - 1) / BM) * ((c.N + BN - 1) / BN);
  int kchunk;
  const long S = split_k(tiles * c.batch, c.K, BK, BM, BN,
                         (long)c.M * c.N * c.batch, 4, CU_PEAK[1], kchunk);
  const long wg = tiles * c.batch * S;
  return (double)((wg + 255) / 256) * BM * BN * kchunk;
}

template <int P>
void dispatch_prec(Device& dev, const Call& c) {
  if (c.M >= 128) {
    // narrow N (chi-wide blocks of the projector SVD and the complement
    // solves): 4 waves stacked along M, tile width rounded up to 16
    // (FP32: direct LDS loads where the operands allow)
    const bool direct = P == 1 && c.K >= 256 && lds_ok(c);
    if (c.N <= 48)
      direct ? launch_cfg<128, 48, 4, 1, P, P == 1>(dev, c)
             : launch_cfg<128, 48, 4, 1, P>(dev, c);
    else if (c.N <= 64)
      direct ? launch_cfg<128, 64, 4, 1, P, P == 1>(dev, c)
             : launch_cfg<128, 64, 4, 1, P>(dev, c);
    else if (c.N <= 80)
      direct ? launch_cfg<128, 80, 4, 1, P, P == 1>(dev, c)
             : launch_cfg<128, 80, 4, 1, P>(dev, c);
    else if (c.N <= 96)
      direct ? launch_cfg<128, 96, 4, 1, P, P == 1>(dev, c)
             : launch_cfg<128, 96, 4, 1, P>(dev, c);
    else if constexpr (P >= 2)  // BF16x3: 128 x 128 would spill registers
      launch_cfg<128, 96, 4, 1, P>(dev, c);
    else if constexpr (P == 1) {
      // FP32: 128 x 144 tiles (4 waves of 32 x 144; D^4 = 1296 and its
      // multiples by D^2 are multiples of 144) or 128 x 128 tiles, the
      // latter with direct LDS loads where the operands allow; by the time
      // model, with the measured handicaps of the 144-wide tile (two waves
      // per SIMD, x 1.05) and the advantage of the direct loads (x 0.82)
      const double c128 = tile_cost(c, 128, 128, 16);
      const double c144 = tile_cost(c, 128, 144, 16);
      const bool direct = c.K >= 256 && lds_ok(c);
      // inner size below 256 and a large output (the n x n cut-matrix
      // gradients accumulated from n x 2 chi factors, outer products of
      // chi-wide blocks): the time goes into writing (and with beta,
      // reading) C, and 64 x 64 tiles keep more workgroups storing at once
      // than 128 x 128 ones (3 ms less per FP32 step at D = 6, chi = 72;
      // the same products in the same order)
      if (c.K < 256 && c.M >= 1024 && c.N >= 1024)
        launch_cfg<64, 64, 2, 2, P>(dev, c);
      else if (direct && c144 < c128)
        launch_cfg<128, 144, 4, 1, P, true>(dev, c);
      else if (direct)
        launch_cfg<128, 128, 2, 2, P, true>(dev, c);
      else if (c144 * 1.05 < c128)
        launch_cfg<128, 144, 4, 1, P>(dev, c);
      else
        launch_cfg<128, 128, 2, 2, P>(dev, c);
    } else
      launch_cfg<128, 128, 2, 2, P>(dev, c);
  } else if (c.M > 64 && c.M <= 96) {
    // 65..96 rows (chi = 72 and D^2 + 60 wide blocks of the complement
    // solves and the projector SVD): one 96-row tile instead of a 64-row
    // tile and a mostly empty second one
    if (c.N > 96)
      launch_cfg<96, 128, 2, 2, P>(dev, c);
    else
      launch_cfg<96, 96, 2, 2, P>(dev, c);
  } else if (c.N >= 128) {
    launch_cfg<64, 128, 2, 2, P>(dev, c);
  } else {
    launch_cfg<64, 64, 2, 2, P>(dev, c);
  }
}

void dispatch(Device& dev, const Call& c) {
  if (small_pays(c)) {
    launch_small(dev, c);
    return;
  }
  if (dev.cprec == PREC_FP32)
    dispatch_prec<1>(dev, c);
  else if (dev.cprec == PREC_FP64)
    dispatch_prec<0>(dev, c);
  else if (dev.cprec == PREC_BF16)
    dispatch_prec<2>(dev, c);
  else
    dispatch_prec<3>(dev, c);
}

void check_sizes(int64_t M, int64_t N, int64_t K, int64_t batch) {
  if (M >= (1LL << 31) || N >= (1LL << 31) || K >= (1LL << 31) ||
      batch > 65535)
    throw ArgError("gemm: size out of range");
}

}  // namespace

void gemm(Device& dev, bool tA, bool tB, int64_t M, int64_t N, int64_t K,
          double alpha, const double* A, int64_t lda, int64_t sA,
          const double* B, int64_t ldb, int64_t sB, double beta, double* C,
          int64_t ldc, int64_t sC, int64_t batch, const CMap* cm) {
  if (M <= 0 || N <= 0 || batch <= 0) return;
  if (K == 0) {
    if (cm && (cm->nr || cm->c32))
      throw ArgError("gemm: scattered or FP32 C with K = 0");
    for (int64_t b = 0; b < batch; ++b)
      for (int64_t m = 0; m < M; ++m)
        axpby(dev, N, 0.0, C + b * sC + m * ldc, beta, C + b * sC + m * ldc);
    return;
  }
  check_sizes(M, N, K, batch);
  Call c{tA, tB, (int)M, (int)N, (int)K, (int)batch, alpha, beta, A, lda, sA,
         B, ldb, sB, C, ldc, sC, nullptr};
  if (cm) c.cm = *cm;
  dispatch(dev, c);
}

namespace {
template <class TA>
void gemm_ptrs_impl(Device& dev, bool tA, bool tB, int64_t M, int64_t N,
                    int64_t K, double alpha, const std::vector<const TA*>& A,
                    int64_t lda, const std::vector<const double*>& B,
                    int64_t ldb, double beta, const std::vector<double*>& C,
                    int64_t ldc, const CMap* cm = nullptr) {
  const int64_t batch = (int64_t)A.size();
  if (M <= 0 || N <= 0 || batch <= 0 || K <= 0) return;
  if ((int64_t)B.size() != batch || (int64_t)C.size() != batch)
    throw ArgError("gemm_ptrs: pointer counts differ");
  check_sizes(M, N, K, batch);
  // operand addresses travel in the kernel arguments, MAXP per launch
  for (int64_t b0 = 0; b0 < batch; b0 += MAXP) {
    const int nb = (int)std::min<int64_t>(MAXP, batch - b0);
    PtrArgs pa{};
    for (int i = 0; i < nb; ++i) {
      pa.a[i] = A[b0 + i];
      pa.b[i] = B[b0 + i];
      pa.c[i] = C[b0 + i];
    }
    Call c{tA, tB, (int)M, (int)N, (int)K, nb, alpha, beta, pa.a[0], lda, 0,
           pa.b[0], ldb, 0, pa.c[0], ldc, 0, &pa, sizeof(TA) == 4};
    if (cm) c.cm = *cm;
    dispatch(dev, c);
  }
}
}  // namespace

void gemm_ptrs(Device& dev, bool tA, bool tB, int64_t M, int64_t N,
               int64_t K, double alpha, const std::vector<const double*>& A,
               int64_t lda, const std::vector<const double*>& B, int64_t ldb,
               double beta, const std::vector<double*>& C, int64_t ldc,
               const CMap* cm) {
  gemm_ptrs_impl(dev, tA, tB, M, N, K, alpha, A, lda, B, ldb, beta, C, ldc,
                 cm);
}

void gemm_ptrs_a32(Device& dev, bool tA, bool tB, int64_t M, int64_t N,
                   int64_t K, double alpha,
                   const std::vector<const float*>& A, int64_t lda,
                   const std::vector<const double*>& B, int64_t ldb,
                   double beta, const std::vector<double*>& C, int64_t ldc,
                   const CMap* cm) {
  if (dev.cprec == PREC_FP64)
    throw ArgError("gemm_ptrs_a32: FP32 operands need FP32 or BF16x3 products");
  gemm_ptrs_impl(dev, tA, tB, M, N, K, alpha, A, lda, B, ldb, beta, C, ldc,
                 cm);
}

// the LDS limits of every direct-load GEMM instantiation the dispatcher
// can pick (see allow_dyn_lds)
void prime_gemm_attributes() {
  prime_lds_all<double>();
  prime_lds_all<float>();
}

}  // namespace ipeps
