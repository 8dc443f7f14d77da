/*
 * ipeps_debug.h -- test hooks of the iPEPS library.  They run single kernels
 * of the library on host data (device memory is allocated and released
 * inside the call, on the null stream) so that tests can check them in
 * isolation.  Not part of the hot path.
 */
#ifndef IPEPS_DEBUG_H
#define IPEPS_DEBUG_H

#ifdef __cplusplus
extern "C" {
#endif

/* C = alpha op(A) op(B) + beta C with the library's FP64 matrix-core GEMM;
 * row-major host arrays: op(A) M x K (A is M x K, or K x M when tA),
 * op(B) K x N (B is K x N, or N x K when tB), C M x N.  Returns a status. */
int ipeps_debug_gemm(int tA, int tB, int M, int N, int K, double alpha,
                     const double* A, const double* B, double beta,
                     double* C);

/* ipeps_debug_gemm with the products in the arithmetic `prec` (ipeps_prec:
 * IPEPS_FP64, IPEPS_FP32 or IPEPS_BF16, the last as three BF16 products of a
 * two-term split; operands and result stay FP64 in memory). */
int ipeps_debug_gemm_prec(int prec, int tA, int tB, int M, int N, int K,
                          double alpha, const double* A, const double* B,
                          double beta, double* C);

/* Average device time in microseconds of one strided-batched GEMM call
 * (C = op(A) op(B) on `batch` pseudo-random M x K, K x N operands, split-K
 * reduction included), over `reps` calls after one warm-up call. */
int ipeps_debug_gemm_time(int prec, int tA, int tB, int M, int N, int K,
                          int batch, int reps, double* us_per_call);

/* Symmetric eigendecomposition of `batch` b x b row-major matrices G (b even,
 * b <= 512) by the library's Jacobi kernel: V (columns = eigenvectors) and
 * lam, sorted by descending eigenvalue. */
int ipeps_debug_sym_eig(int b, int batch, const double* G, double* V,
                        double* lam);

/* Tall-skinny SVD W J = U diag(s) of `batch` n x b row-major matrices by
 * the library's two-pass Gram/Jacobi routine (b even, b <= 512). */
int ipeps_debug_svd_ts(int n, int b, int batch, const double* W, double* U,
                       double* s, double* J);

/* out = alpha permute(in) + beta out by the library's permute kernels:
 * in is a row-major host tensor of rank `rank` (1..12) and shape `shape`,
 * out has shape shape[perm[0]], ..., shape[perm[rank - 1]] (perm is a
 * permutation of 0..rank-1); out[i_0..i_{r-1}] = in[j] with j[perm[d]] =
 * i_d.  Fewer than 2^31 elements.  Returns a status. */
int ipeps_debug_permute(int rank, const long* shape, const int* perm,
                        double alpha, const double* in, double beta,
                        double* out);

/* out = alpha einsum(spec, A, B) + beta out by the library's contraction
 * planner, on host data: spec like "mgek,gebf->mfkb" (single-letter
 * labels; every label of an operand is either shared with the other one or
 * kept in the output); `count` independent items of the same shapes, item i
 * at A + i |A|, B + i |B|, out + i |out| (contracted in one batched launch,
 * as the network's contractions are); products in the arithmetic `prec`
 * (ipeps_prec).  mode 0: the planner's choice, which may write a permuted
 * output straight from the GEMM epilogue; mode 1: never (GEMM in its own
 * order, then a permute pass).  *scattered receives the number of launches
 * that wrote a scattered output.  Returns a status. */
int ipeps_debug_einsum(const char* spec, int prec, int mode, int count,
                       int rankA, const long* shapeA, const double* A,
                       int rankB, const long* shapeB, const double* B,
                       double alpha, double beta, double* out,
                       int* scattered);

/* Iteration counters of a context since its creation: out[0] subspace
 * iterations, out[1] projector-SVD calls, out[2] largest final subspace
 * residual (relative to s_1), out[3] complement-CG iterations of the
 * backward pass, out[4] complement solves, out[5] device memory held by the
 * context's pool in bytes, out[6] peak of the bytes in use, out[7] the
 * number of unrolled iterations of the last gradient, out[8] projector SVDs
 * and out[9] complement solves that stopped at their iteration limit above
 * their tolerance, out[10] the arithmetic (ipeps_prec) the context's next
 * contractions use, out[11] the largest true relative residual of a
 * complement solve (recorded with test hook 4; out has 12 entries). */
struct ipeps_ctx;
int ipeps_debug_stats(struct ipeps_ctx* ctx, double* out);

/* Memory check of a context created while IPEPS_MEMCHECK was set in the
 * environment (1: guard bands of 16 KiB around every device tensor, released
 * blocks held back from reuse until the next check; 2: also every new
 * tensor filled with NaN).  Synchronises the context's stream, verifies the
 * bands of every live and held block, writes one line per damaged band to
 * stderr (tensor size and address, side, distance of the nearest changed
 * byte) and sets *damaged to their number, or to -1 when the context was
 * created without the check; the held blocks are reusable afterwards.
 * ctm_free runs the same verification.  For finding kernels that write
 * outside their tensors, or read memory no kernel wrote: never enabled in
 * production runs. */
int ipeps_debug_memcheck(struct ipeps_ctx* ctx, long* damaged);

/* Failure injection for the error-path tests (forced from the host; every
 * kernel still runs to its normal end):
 *   kind 0  clear all injected faults;
 *   kind 1  device-memory budget of the context: allocations that would
 *           take the bytes in use above `value` fail (ENOMEM from the call);
 *   kind 2  precond_apply stops before CG iteration `value` as if it had
 *           met p^T (N + delta) p <= 0 (ECG_BREAKDOWN, x = last iterate);
 *   kind 3  deflation vectors per half of the complement solves of the
 *           projector backward: at most `value` (32; 0 = no deflation);
 *   kind 4  value != 0: after every complement solve, recompute its true
 *           residual (ipeps_debug_stats out[11]).
 * Returns a status (EINVAL for an unknown kind or a negative value). */
int ipeps_debug_set_fault(struct ipeps_ctx* ctx, int kind, double value);

#ifdef __cplusplus
}
#endif
#endif /* IPEPS_DEBUG_H */
