// Internal engine of the iPEPS library: device memory, dense FP64 tensors on
// one HIP stream, and the launch wrappers of the hand-written gfx950 kernels.
// Errors inside the engine are C++ exceptions; the C ABI (api.cpp) turns them
// into status codes.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <map>
#include <memory>
#include <stdexcept>
#include <string>
#include <vector>

namespace ipeps {

struct HipError : std::runtime_error {
  explicit HipError(const std::string& s) : std::runtime_error(s) {}
};
struct OomError : std::runtime_error {
  explicit OomError(const std::string& s) : std::runtime_error(s) {}
};
struct ArgError : std::runtime_error {
  explicit ArgError(const std::string& s) : std::runtime_error(s) {}
};
struct NotImplError : std::runtime_error {
  explicit NotImplError(const std::string& s) : std::runtime_error(s) {}
};

#define IPEPS_HIP(call)                                                   \
  do {                                                                    \
    hipError_t e__ = (call);                                              \
    if (e__ != hipSuccess)                                                \
      throw ::ipeps::HipError(std::string(#call) + ": " +                \
                              hipGetErrorString(e__));                    \
  } while (0)

// Caching device allocator owned by one context: freed blocks are kept and
// handed out again (best fit, at most 1/8 larger than the request), so the
// reservation stays close to the peak of live bytes.  At destruction (after
// the context's stream has drained) the blocks go to a process-wide idle
// list that later contexts draw from before calling hipMalloc; the idle list
// is returned to HIP when an allocation runs out of memory.
class Pool {
 public:
  Pool() = default;
  Pool(const Pool&) = delete;
  Pool& operator=(const Pool&) = delete;
  ~Pool();
  // returns a block of *got >= bytes bytes
  void* alloc(size_t bytes, size_t* got);
  void release(void* p, size_t block_bytes);
  size_t reserved() const { return reserved_; }
  size_t peak_live() const { return peak_live_; }
  // bytes in use at once beyond which alloc fails with OomError (a budget
  // the caller sets; no limit by default)
  void set_limit(size_t bytes) { limit_ = bytes; }
  // Arena mode: between begin_arena and end_arena every block is carved
  // from the fixed region [base, base + bytes) (a bump pointer; blocks
  // released meanwhile are handed out again, best fit within 1/8), and
  // nothing is taken from HIP, the idle list or this pool's cached blocks;
  // a request that does not fit throws OomError.  Blocks of the region that
  // are released after end_arena are dropped.
  void begin_arena(void* base, size_t bytes);
  void end_arena();
  size_t arena_peak() const { return arena_peak_; }
  bool in_arena() const { return arena_ != nullptr; }
  // Memory check mode (Device::memcheck): released blocks are held back
  // instead of handed out again until take_held() passes them to the
  // checker, which returns them with reissue()
  void hold_released(bool on) { hold_ = on; }
  size_t held_bytes() const { return held_bytes_; }
  std::vector<std::pair<void*, size_t>> take_held();
  void reissue(void* p, size_t block_bytes) { free_.emplace(block_bytes, p); }

 private:
  std::multimap<size_t, void*> free_;
  std::vector<std::pair<void*, size_t>> all_;
  size_t reserved_ = 0, live_ = 0, peak_live_ = 0;
  size_t limit_ = SIZE_MAX;
  char* arena_ = nullptr;            // active region (null: none)
  size_t arena_size_ = 0, arena_top_ = 0, arena_peak_ = 0;
  const char* arena_lo_ = nullptr;   // last region, for late releases
  const char* arena_hi_ = nullptr;
  std::multimap<size_t, void*> arena_free_;
  bool hold_ = false;
  size_t held_bytes_ = 0;
  std::vector<std::pair<void*, size_t>> held_;
};

// Returns blocks of the idle list (those of destroyed contexts) to HIP,
// largest first, until at most keep_bytes remain; returns the bytes left.
size_t trim_idle_to(size_t keep_bytes);

struct Buffer {
  void* p = nullptr;
  size_t bytes = 0;  // block size
  Pool* pool = nullptr;
  ~Buffer() {
    if (p) pool->release(p, bytes);
  }
};

// Dense row-major tensor in device memory (shared ownership of the buffer;
// views share it).  FP64, or FP32 when f32 is set: then ptr holds numel()
// floats.  FP32 storage is used for contraction intermediates whose every
// reader rounds them to FP32 anyway (operands of FP32 and BF16x3 products).
struct Tensor {
  std::shared_ptr<Buffer> buf;
  double* ptr = nullptr;
  std::vector<int64_t> shape;
  bool f32 = false;

  int64_t numel() const {
    int64_t n = 1;
    for (auto s : shape) n *= s;
    return n;
  }
  int rank() const { return (int)shape.size(); }
  Tensor view(std::vector<int64_t> s) const;   // same data, new shape
  Tensor slice0(int64_t i) const;              // sub-tensor along dim 0
};

// Optional timing of the library's own launches: HIP events on the launch
// stream around every launch of a kernel family, with the algorithmic FLOP
// and byte counts of each launch.
enum ProfFamily {
  PROF_GEMM = 0,     // FP64 matrix-core GEMM
  PROF_JACOBI = 1,
  PROF_PERMUTE = 2,
  PROF_GEMM32 = 3,   // FP32 matrix-core GEMM
  PROF_GEMM16 = 4,   // BF16x3 matrix-core GEMM
  PROF_NET = 5,      // GEMMs of the network contractions (einsum), any
                     // arithmetic: a subset of the three GEMM families
  PROF_WIDE = 6,     // the 128 x 144-tile FP32 GEMM (the chi^2 D^8-class
                     // network products): a subset of PROF_GEMM32
  PROF_N = 7
};

// Arithmetic of the GEMMs issued on a device (the contraction precision;
// the values match ipeps_prec of the C ABI).
enum Prec { PREC_FP64 = 0, PREC_FP32 = 1, PREC_BF16 = 2, PREC_BF16X1 = 3 };

// Rounding floors of a contraction arithmetic: the smallest corner-spectrum
// change CTMRG can resolve with it, and the relative residuals at which the
// projector SVD and the complement solves of its adjoint level off (FP64:
// none; the configured tolerances apply).
struct PrecFloors {
  double spectra, svd_res, cg_res;
};
inline PrecFloors prec_floors(int p) {
  switch (p) {
    case PREC_FP32: return {1e-7, 1e-5, 1e-5};
    case PREC_BF16: return {3e-6, 1e-3, 1e-3};
    case PREC_BF16X1: return {1e-3, 3e-2, 3e-2};
    default: return {0.0, 0.0, 0.0};
  }
}

struct Profiler {
  bool on = false;
  struct Rec {
    int fam;
    hipEvent_t a, b;
    double flop, bytes;
    bool net;   // issued by a network contraction
    bool wide;  // the 128 x 144-tile FP32 GEMM
  };
  bool net = false;  // launches now belong to a network contraction
  std::vector<Rec> recs;
  std::vector<hipEvent_t> pool;
  hipEvent_t get();
  void begin(hipStream_t s, int fam, double flop, double bytes,
             bool wide = false);
  void end(hipStream_t s);
  // launches, seconds, flop, bytes of one family (synchronises)
  void read(int fam, long* n, double* sec, double* flop, double* bytes);
  void clear();
  // create events ahead so that recording adds no hipEventCreate calls
  void reserve(size_t n);
  ~Profiler();
};

// Execution context: one stream and one pool.
// Memory check mode of the devices created while IPEPS_MEMCHECK is set in
// the environment (0 or unset: off): 1 = every block carries guard bands
// of MEMCHECK_GUARD bytes on both sides of the tensor, filled with a byte
// pattern when the tensor is created, and released blocks are held back
// from reuse until the next memcheck(), which verifies the bands of every
// live and held block after the stream has drained (a kernel writing past
// either end of its tensor changes them); 2 = also every new tensor is
// filled with NaN, so that results that read memory no kernel wrote differ
// from those of an unchecked run.
int memcheck_mode();
constexpr size_t MEMCHECK_GUARD = 16384;
constexpr size_t MEMCHECK_HOLD = (size_t)8 << 30;

struct Device {
  hipStream_t stream = nullptr;
  bool own_stream = false;
  Pool pool;
  Profiler prof;
  int memcheck = memcheck_mode();
  // check mode: raw block -> (tensor bytes, block bytes) of every block
  // handed out since its last verification
  std::map<void*, std::pair<size_t, size_t>> guarded;
  // verifies the guard bands (check mode; synchronises the stream),
  // reports each damaged band on stderr, returns their number and lets
  // the held blocks be reused.  It also runs by itself when the held
  // blocks reach MEMCHECK_HOLD bytes; damage found then is counted in
  // memcheck_pending.
  long memcheck_verify();
  long memcheck_pending = 0;
  int cprec = PREC_FP64;  // arithmetic of the GEMMs issued now
  // contractions may write a permuted output from the GEMM epilogue
  // (false: GEMM in its own order, then a permute pass); the count of the
  // contractions that did
  bool allow_scatter = true;
  long scatter_count = 0;

  Tensor empty(std::vector<int64_t> shape);
  Tensor empty_f32(std::vector<int64_t> shape);  // FP32 storage
  Tensor zeros(std::vector<int64_t> shape);
  Tensor scalar_buffer(int n);            // n doubles
  void upload(Tensor& t, const double* host);
  void download(const Tensor& t, double* host);
  void sync();
};

// Marks the launches of a scope as those of a network contraction (for the
// PROF_NET profile family) and restores the previous mark.
struct NetScope {
  Profiler& p;
  bool old;
  explicit NetScope(Profiler& pr) : p(pr), old(pr.net) { p.net = true; }
  ~NetScope() { p.net = old; }
  NetScope(const NetScope&) = delete;
  NetScope& operator=(const NetScope&) = delete;
};

// Sets the GEMM arithmetic for a scope and restores the previous one.
struct PrecScope {
  Device& d;
  int old;
  PrecScope(Device& dv, int p) : d(dv), old(dv.cprec) { d.cprec = p; }
  ~PrecScope() { d.cprec = old; }
  PrecScope(const PrecScope&) = delete;
  PrecScope& operator=(const PrecScope&) = delete;
};

// ---------------------------------------------------------------- kernels
// Scattered layout of a GEMM result: element (row, col) of C[b] lives at
// C[b] + roff(row) + coff(col), where roff splits row into nr mixed-radix
// digits (extents re[], least significant first) and sums digit * rs[],
// and coff does the same for col with ce[], cs[].  nr == 0 is the plain
// row-major layout with leading dimension ldc.  A permutation of the
// output labels of a contraction is such a layout, so the GEMM epilogue
// writes the permuted tensor directly.
constexpr int CMAP_DIGITS = 4;
struct CMap {
  int nr = 0, nc = 0;
  int c32 = 0;  // C stored in FP32 (offsets and strides count floats)
  int re[CMAP_DIGITS] = {0, 0, 0, 0}, ce[CMAP_DIGITS] = {0, 0, 0, 0};
  int64_t rs[CMAP_DIGITS] = {0, 0, 0, 0}, cs[CMAP_DIGITS] = {0, 0, 0, 0};
};

// C[b] = alpha op(A[b]) op(B[b]) + beta C[b], row major; op(A) is M x K
// (A[m*lda+k], or A[k*lda+m] when tA), op(B) is K x N (B[k*ldb+n], or
// B[n*ldb+k] when tB), batch strides sA, sB, sC in elements.  With cm, C[b]
// is in the scattered layout cm describes (ldc unused).
void gemm(Device& dev, bool tA, bool tB, int64_t M, int64_t N, int64_t K,
          double alpha, const double* A, int64_t lda, int64_t sA,
          const double* B, int64_t ldb, int64_t sB, double beta, double* C,
          int64_t ldc, int64_t sC, int64_t batch = 1,
          const CMap* cm = nullptr);

// Batched GEMM over arbitrary operand addresses (one launch): C[i] = alpha
// op(A[i]) op(B[i]) + beta C[i], same shapes and leading dimensions.
void gemm_ptrs(Device& dev, bool tA, bool tB, int64_t M, int64_t N,
               int64_t K, double alpha, const std::vector<const double*>& A,
               int64_t lda, const std::vector<const double*>& B, int64_t ldb,
               double beta, const std::vector<double*>& C, int64_t ldc,
               const CMap* cm = nullptr);

// gemm_ptrs with the A operands stored in FP32 (the products in the FP32
// or BF16x3 arithmetic of the device; FP64 is refused).
void gemm_ptrs_a32(Device& dev, bool tA, bool tB, int64_t M, int64_t N,
                   int64_t K, double alpha,
                   const std::vector<const float*>& A, int64_t lda,
                   const std::vector<const double*>& B, int64_t ldb,
                   double beta, const std::vector<double*>& C, int64_t ldc,
                   const CMap* cm = nullptr);
// Raises, once per process, the dynamic LDS limit of every kernel that
// needs more than the default, before any context launches work (safe to
// call from several threads; the first call does the work).
void prime_attributes();
// y[i] = (float) x[i]
void to_f32(Device& dev, const double* x, float* y, int64_t n);
// y[i] = (double) x[i]
void to_f64(Device& dev, const float* x, double* y, int64_t n);
// Up to NB_MAX vectors of any lengths, normalised in one pass (see
// normalize_batch): a[i] the input (forward) or y (backward), b[i] ybar
// (backward), out[i] y (forward) or xbar (backward, accumulated), nrm[i]
// |x_i| (backward input).
constexpr int NB_MAX = 16;
struct NormBatch {
  const double* a[NB_MAX];
  const double* b[NB_MAX];
  double* out[NB_MAX];
  const double* nrm[NB_MAX];
  long n[NB_MAX];
};
// out_i = a_i / |a_i|, nrm[i] = |a_i| (device array of count doubles)
void normalize_batch(Device& dev, const NormBatch& p, int count, double* nrm);
// out_i += (b_i - a_i <a_i, b_i>) / nrm_i[0]
void normalize_backward_batch(Device& dev, const NormBatch& p, int count);
// dst (cols x rows) = src^T (rows x cols), row major
void transpose(Device& dev, const double* src, double* dst, int64_t rows,
               int64_t cols);
void transpose(Device& dev, const float* src, float* dst, int64_t rows,
               int64_t cols);

// out = alpha * permute(in, perm) + beta * out (rank <= 12 after merging
// contiguous dims); out.shape[i] =
// in.shape[perm[i]].
void permute(Device& dev, const Tensor& in, const std::vector<int>& perm,
             Tensor& out, double alpha = 1.0, double beta = 0.0);
Tensor permuted(Device& dev, const Tensor& in, const std::vector<int>& perm);

void fill(Device& dev, double* x, int64_t n, double v);
// y = a * x + b * y
void axpby(Device& dev, int64_t n, double a, const double* x, double b,
           double* y);
// x[i] *= s[0] (device scalar), or x[i] /= s[0] when inverse
void scale_dev(Device& dev, double* x, int64_t n, const double* s,
               bool inverse);
// out[0] = sum x*y (deterministic two-stage reduction), FP64
void dot(Device& dev, const double* x, const double* y, int64_t n,
         double* out);
// out[0] = sqrt(sum x*x)
void nrm2(Device& dev, const double* x, int64_t n, double* out);

// Batched symmetric eigendecomposition by parallel cyclic Jacobi, one
// workgroup per matrix: G[bt] (b x b row major, b even, b <= 128) is
// overwritten by its diagonalised form, V[bt] (b x b row major) receives
// the eigenvectors as columns, lam[bt] the eigenvalues; both sorted by
// descending eigenvalue.  Pairs with |G_pq| <= tol sqrt|G_pp G_qq| are not
// rotated.
void sym_eig_jacobi(Device& dev, double* G, double* V, double* lam, int b,
                    int batch = 1, double tol = 1e-15);

// Column 2-norms of an n x b row-major matrix: out[j] = ||X[:, j]||.
void col_norms(Device& dev, const double* X, int64_t n, int b, double* out,
               int batch = 1, int64_t sX = 0, int64_t sOut = 0);
// X[:, j] *= f(s[j]) with f = 1/s (0 if s == 0) (mode 0), s^-1/2 masked by
// keep (mode 1), plain s (mode 2).
void col_scale(Device& dev, double* X, int64_t n, int b, const double* s,
               int mode, const int* keep = nullptr, int batch = 1,
               int64_t sX = 0, int64_t sS = 0);

// ------------------------------------------------------------ contractions
// Pairwise tensor contraction with single-character labels, e.g.
// "mgi,ij->mgj".  Labels in both inputs and the output are batch labels,
// in both inputs only are contracted, in one input and the output are free.
// Implemented as (at most) permutes + one batched GEMM; the plan avoids
// permutes where the GEMM transposes allow.
Tensor einsum(Device& dev, const std::string& spec, const Tensor& A,
              const Tensor& B);
// out = alpha * einsum(...) + beta * out (out has the output shape)
void einsum_into(Device& dev, const std::string& spec, const Tensor& A,
                 const Tensor& B, Tensor& out, double alpha = 1.0,
                 double beta = 0.0);
// The same contraction for several items of one shape (one plan, the
// products of all items in one pointer-batched GEMM launch).  The outputs
// must be distinct tensors.
void einsum_into_n(Device& dev, const std::string& spec,
                   const std::vector<Tensor>& A, const std::vector<Tensor>& B,
                   const std::vector<Tensor>& out, double alpha = 1.0,
                   double beta = 0.0);
// f32: the outputs stored in FP32 (only where the device's product
// arithmetic is not FP64; otherwise FP64).
std::vector<Tensor> einsum_n(Device& dev, const std::string& spec,
                             const std::vector<Tensor>& A,
                             const std::vector<Tensor>& B, bool f32 = false);

}  // namespace ipeps

namespace ipeps {
void random_block(Device& dev, double* X, int64_t n, uint64_t seed);
void eye(Device& dev, double* X, int64_t n, int b, int batch, int64_t sX);
void sign_fix(Device& dev, double* U, double* V, int64_t n, int b, int batch,
              int64_t sU, int64_t sV);
void kept_rank(Device& dev, const double* S, int b, int chi, double cut,
               int* keep, int batch, int64_t sS);
void svd_residual(Device& dev, const double* Z, const double* V,
                  const double* S, int64_t n, int b, int k, double* r,
                  int batch, int64_t sZ, int64_t sS);
void pad3(Device& dev, const double* in, double* out, int a, int b, int c,
          int B, int C);
// adjoint of pad3: gin[l][j][k] += gout[(l B + j) C + k]
void crop3_add(Device& dev, const double* gout, double* gin, int a, int b,
               int c, int B, int C);
void spectra_update(Device& dev, const double* S, int b, int chi, int batch,
                    int64_t sS, double* cur, double* old, double* delta);
}  // namespace ipeps

namespace ipeps {
void term_energy(Device& dev, const double* rho, const double* h, int m,
                 double coef, double* acc, double* rho_bar);
void splitk_reduce(Device& dev, const double* part, int S, int64_t M,
                   int64_t N, double alpha, double beta, double* C,
                   int64_t ldc);
}  // namespace ipeps

namespace ipeps {
// columns with a zero entry in cn replaced by pseudo-random ones
void fill_null_cols(Device& dev, double* X, int64_t n, int b,
                    const double* cn, int batch, uint64_t seed);
void null_threshold(Device& dev, double* S, int b, double rel, int batch,
                    int64_t sS);
// R = L^-T from the Cholesky factor of G = L L^T (b x b, batched); dropped
// (dependent) directions give zero rows and columns.
void chol_orth_factor(Device& dev, const double* G, double* R, int b,
                      int batch);
// out[i][j] = M[max(i,j)][min(i,j)] (lower triangle mirrored), b x b
void copyltu(Device& dev, const double* M, double* out, int b);
// out = F o X, F_ij = x / (x^2 + eta^2), x = lam_j - lam_i, F_ii = 0,
// eta = rel max|lam| (the broadened eigenvector derivative), b x b
void eig_fmul(Device& dev, const double* lam, const double* X, double* out,
              int b, double rel);
// Eigenpairs in descending signed order (lam, columns of W, b x b)
// reordered: the k of largest |lambda| first (ties: the larger signed
// value), then the others, each group in descending signed order
void eig_order_kept(Device& dev, const double* lam, const double* W,
                    double* lam_out, double* W_out, int b, int k);
// s[j] = sign of the entry of column j of X (n x b) maximising
// |x_rj| (1 + r / (2n)) (first on ties), +1 for a zero column
void col_sign(Device& dev, const double* X, int64_t n, int b, double* s);
}  // namespace ipeps

namespace ipeps {
// Column dots of `batch` n x m row-major blocks (stride sXY):
// out[bt][j] = sum_i X[bt][i][j] Y[bt][i][j]
void coldot(Device& dev, const double* X, const double* Y, int64_t n, int m,
            double* out, int batch = 1, int64_t sXY = 0);
void proj_weights(Device& dev, const double* S, const int* keep, int chi,
                  double* w, int batch = 1, int sS = 0);
void proj_sbar(Device& dev, const double* S, const int* keep, int chi,
               const double* wb1, const double* wb2, double* sbar,
               int batch = 1, int sS = 0);
void svd_gkk(Device& dev, const double* Au, const double* Av, const double* S,
             const double* sbar, const int* keep, int chi, double* G,
             int batch = 1, int sS = 0);
void mask_cols(Device& dev, double* X, int64_t n, int m, const int* keep,
               int batch = 1);
// rows = total rows of all batches; per-(batch, column) scalars use
// rows_per_batch (0 = one batch)
void colcg(Device& dev, int mode, int64_t rows, int m, const double* rr,
           const double* den, double* x, double* r, double* p,
           const double* Ap, int64_t rows_per_batch = 0);
// Fused column-wise CG (batch blocks of n x m, row major): colcg_step
// does x += a p, r -= a A p with a = num / den per column and leaves the
// per-column partial sums of r^2 in part ([batch][colcg_parts()][m]);
// colcg_dir reduces them to rr_new and sets p = r + (rr_new / rr_old) p.
void colcg_step(Device& dev, int64_t n, int m, int batch, const double* num,
                const double* den, double* x, double* r, const double* p,
                const double* Ap, double* part);
void colcg_dir(Device& dev, int64_t n, int m, int batch, const double* part,
               const double* rr_old, double* rr_new, const double* r,
               double* p);
int colcg_parts();
void col_axpby(Device& dev, int64_t n, int m, double a, const double* s,
               const double* x, double b, double* y,
               int64_t rows_per_batch = 0, int64_t sS = 0);
void defl_build_k(Device& dev, const double* B1, const double* B2, int m,
                  double* K, int batch);
void inv_sqrt_clip(Device& dev, double* x, int64_t n, double thr);
void defl_coef(Device& dev, int mode, const double* S, const int* keep,
               const double* lam, int chi, int m2, int sS, const double* H,
               double* out, int batch);
// y[r] = sum_s x[r][s][s], x: rows x d x d
void trace_dd(Device& dev, const double* x, int64_t rows, int d, double* y);
// gx[r][s][t] = beta gx[r][s][t] + (s == t) g[r]
void trace_dd_backward(Device& dev, const double* g, int64_t rows, int d,
                       double* gx, double beta);
void copy2d(Device& dev, const double* src, int64_t lds, double* dst,
            int64_t ldd, int64_t rows, int64_t cols, int batch = 1,
            int64_t sSrc = 0, int64_t sDst = 0);
}  // namespace ipeps
