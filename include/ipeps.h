/*
 * ipeps.h -- C ABI of the MI355X (gfx950) library for one preconditioned
 * gradient step of an iPEPS (arXiv:2511.09546):
 *
 *   ctm_init          double-layer tensor and trace-boundary environment
 *   ctm_converge      CTMRG to a fixed point (the environment of Sec. III A,
 *                     "gray circles" of Eq. (7))
 *   ipeps_energy_grad energy per site E(A) (Eqs. (6)-(7)) and its gradient
 *                     dE/dA (Sec. III A; K-step unrolled backward pass,
 *                     Sec. IV A)
 *   precond_apply     preconditioned gradient x = (N_local + delta I)^-1 g
 *                     (Eq. (4); local metric Eq. (11); regularisation
 *                     Sec. III B; implicit solve Sec. III C) by conjugate
 *                     gradients
 *
 * Every call returns an int status (ipeps_status) and never aborts or throws.
 * Negative values are errors (outputs untouched), positive values warnings
 * (outputs valid).  Plain C types only; host arrays are row-major C order.
 *
 * Ownership: the caller owns every host array; inputs are copied during the
 * call and never retained or modified.  The context owns all device memory
 * it allocates until ctm_free.  One host thread may use a context at a time;
 * distinct contexts may be used concurrently on distinct streams.
 *
 * Tensor layouts:
 *   site tensors   A[Ly][Lx][d][D][D][D][D], legs (physical, left, up,
 *                  right, down); "up" points to row y-1; site index y*Lx+x;
 *                  real FP64.
 *   gradient, directions: same layout as A.
 *   Hamiltonian terms: ipeps_term below.
 */
#ifndef IPEPS_H
#define IPEPS_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ipeps_ctx ipeps_ctx;

typedef enum {
  IPEPS_OK = 0,
  IPEPS_NOT_CONVERGED = 1,  /* warning: Delta >= tol after max_iter; the
                               environment of the last iteration is kept */
  IPEPS_STATIONARY = 2,     /* warning (ipeps_lbfgs_step): no descent
                               direction left; nothing was changed */
  IPEPS_EINVAL = -1,        /* bad argument (null pointer, sizes, non-finite
                               values, chi < D^2, delta <= 0, ...) */
  IPEPS_ENOMEM = -2,        /* device allocation failed */
  IPEPS_EHIP = -3,          /* a HIP runtime call failed */
  IPEPS_ECG_BREAKDOWN = -4, /* CG met p^T (N + delta) p <= 0; x holds the
                               last iterate (written in this case) */
  IPEPS_ESTATE = -5,        /* call out of order (e.g. energy before any
                               ctm_converge) */
  IPEPS_ENOTIMPL = -6,      /* option not implemented */
  IPEPS_ESCRATCH = -7       /* the state is too large for the fixed scratch
                               area of precond_apply_dev_noalloc */
} ipeps_status;

/* Arithmetic of the dense contractions (every product of the CTMRG and
 * energy networks, of the metric, and the products with the cut matrices
 * inside the projector SVD and its adjoint).  Projector SVD (Gram matrices,
 * Jacobi, subspace rotations), SVD-adjoint algebra, normalisation,
 * convergence measure, energy traces and CG inner products are FP64 in every
 * mode.  Inputs, outputs and the environment are FP64 in every mode; in the
 * FP32 and BF16 modes the intermediates that only products read are kept
 * in FP32.
 *   IPEPS_FP64  FP64 matrix cores;
 *   IPEPS_FP32  operands rounded to FP32, FP32 accumulation; ctm_converge
 *               raises tolerances below 1e-7 to 1e-7;
 *   IPEPS_BF16  each operand split into two BF16 terms, three BF16 products
 *               (about 16 significant bits), FP32 accumulation;
 *               ctm_converge raises tolerances below 3e-6 to 3e-6;
 *   IPEPS_BF16X1 one BF16 product per operand pair (operands rounded to
 *               BF16, 8 significant bits), FP32 accumulation;
 *               ctm_converge raises tolerances below 1e-3 to 1e-3. */
typedef enum {
  IPEPS_FP64 = 0,
  IPEPS_FP32 = 1,
  IPEPS_BF16 = 2,
  IPEPS_BF16X1 = 3
} ipeps_prec;

/* One Hamiltonian term (Eq. (12), Eq. (13)).
 *   kind 0: on-site d x d matrix acting on unit-cell site `site`;
 *   kind 1: two-site d^2 x d^2 matrix on (site, site + (dx, dy)), periodic in
 *           the unit cell, (dx, dy) in {(1,0), (0,1), (1,1), (1,-1)}.
 * mat is row-major [(s1 s2)][(s1' s2')] (site 1 first); it is read during the
 * call only.  The term contributes coef * Tr(h rho) / Tr(rho), where rho is
 * the reduced density matrix of its sites; the energy per site is the sum
 * over terms divided by Lx*Ly. */
typedef struct {
  int kind;
  int site;
  int dx, dy;
  double coef;
  const double* mat;
} ipeps_term;

typedef struct {
  int prec;           /* ipeps_prec of the contractions */
  double svd_cutoff;  /* keep singular values > svd_cutoff * s_1 (1e-12) */
  int grad_K;         /* unrolled CTMRG iterations in the gradient (20) */
  int svd_oversample; /* extra subspace columns beyond chi (0 = automatic) */
  int svd_max_iter;   /* max subspace iterations per projector (50) */
  double svd_tol;     /* subspace residual tolerance, relative to s_1
                         (1e-13) */
  int grad_mode;      /* ipeps_grad_mode of ipeps_energy_grad (K-step) */
  double adj_tol;     /* fixed-point mode: stop when the cotangent reaching
                         the converged environment is below adj_tol times
                         the one leaving the last iteration (1e-13) */
  int grad_checkpoint; /* 0 (default): ipeps_energy_grad keeps the
                          intermediates of all unrolled iterations resident;
                          1: it keeps only each iteration's input environment
                          and recomputes the iteration in the backward pass
                          (one iteration resident, about one more forward
                          pass of work; same gradient up to rounding) */
  double adj_cg_tol;  /* relative residual at which the complement solves of
                         the truncated-SVD adjoint stop when their products
                         are FP64 (1e-12); FP32 and BF16 products stop at
                         their own rounding floor */
  int ladder;         /* precision ladder (with prec IPEPS_BF16 or
                         IPEPS_BF16X1): 1 = ctm_converge runs its iterations
                         in the BF16 arithmetic until the spectrum change
                         reaches that arithmetic's floor or stops falling,
                         then in FP32 down to the FP32 floor;
                         ipeps_energy_grad and precond_apply then run in
                         FP32.  0 (default) = one arithmetic throughout */
} ipeps_opts;

/* What ipeps_energy_grad differentiates (Sec. III A, Sec. IV A):
 *   IPEPS_GRAD_FULL  A -> e(A, F^K(A, env0(A))): K iterations from the
 *                    trace-boundary start, all of them differentiated;
 *   IPEPS_GRAD_K     A -> e(A, F^K(A, env*)), env* the environment of the
 *                    last ctm_converge held fixed (the unrolled "(3+20)"
 *                    configuration with K = 20);
 *   IPEPS_GRAD_FP    IPEPS_GRAD_K with K doubled (from grad_K, at most 32
 *                    grad_K) until the cotangent reaching env* is below
 *                    adj_tol times the one leaving the last iteration: the
 *                    derivative at the fixed point. */
typedef enum {
  IPEPS_GRAD_FULL = 0,
  IPEPS_GRAD_K = 1,
  IPEPS_GRAD_FP = 2
} ipeps_grad_mode;

/* Fill *opts with the defaults listed above. */
void ipeps_default_opts(ipeps_opts* opts);

/* Create a context, upload A, build the double layer and the trace-boundary
 * environment (bond dimension D^2, zero padded to chi).
 *   ctx       out: new context (on success)
 *   Lx, Ly    unit cell (>= 1), d physical dimension, D bond dimension,
 *   chi       environment dimension, chi >= D^2
 *   A         host, A[Ly][Lx][d][D][D][D][D]
 *   opts      NULL for the defaults
 *   hip_stream a hipStream_t to run on, or NULL for a context-owned stream
 * Errors: EINVAL, ENOMEM, EHIP. */
int ctm_init(ipeps_ctx** ctx, int Lx, int Ly, int d, int D, int chi,
             const double* A, const ipeps_opts* opts, void* hip_stream);

/* Replace the site tensors of an existing context (same shapes), keeping its
 * environment as a warm start. Errors: EINVAL, EHIP. */
int ctm_set_state(ipeps_ctx* ctx, const double* A);

/* CTMRG iterations (one iteration = the simultaneous move of all four
 * corners of every unit-cell plaquette with SVD-truncated half-system
 * projectors) until Delta < tol or max_iter iterations.  Delta is the largest
 * 2-norm change of the sum-normalised singular values of any corner.
 * tol <= 0 runs exactly max_iter iterations.  In the reduced-precision
 * modes (see ipeps_prec) the iteration also stops, NOT_CONVERGED, once Delta
 * is within 100 times the mode's floor and has not fallen below 0.9 of its
 * smallest value for 8 iterations (a state whose kept spectrum reaches the
 * rounding of the products).  After ipeps_set_env / ipeps_set_env_dev the
 * environment is taken as near its fixed point: the first iteration runs
 * with FP64 products and an SVD as accurate as the tolerance asks.
 *   n_iter, delta  out (may be NULL)
 * Returns OK, NOT_CONVERGED (warning), or an error. */
int ctm_converge(ipeps_ctx* ctx, double tol, int max_iter, int* n_iter,
                 double* delta);

/* Energy per site and (if grad != NULL) its gradient with respect to every
 * real entry of A: the derivative of A -> e(A, F^K(A, env*)) where env* is
 * the environment of the last ctm_converge (held fixed) and F one CTMRG
 * iteration, K = opts.grad_K.  e_per_site: host scalar out; grad: host,
 * layout of A.  Errors: EINVAL, ESTATE, EHIP, ENOMEM. */
int ipeps_energy_grad(ipeps_ctx* ctx, int n_terms, const ipeps_term* terms,
                      double* e_per_site, double* grad);

/* Preconditioned direction x = (N_local + delta I)^-1 g, one independent CG
 * solve per unit-cell site, from x0 = 0, on the environment of the last
 * ctm_converge.  N_local acts on site tensor x as
 * (N x)[t,l',u',r',d'] = sum E[(lurd),(l'u'r'd')] x[t,lurd] / Z with E the
 * ring of the eight environment tensors of the site and Z = <A, E A>.
 * CG stops when ||r|| <= cg_tol ||g|| or after cg_maxiter iterations.
 *   g        host, layout of A;  delta > 0
 *   x        host out, layout of A
 *   n_iter   out: largest iteration count over sites (may be NULL)
 *   rel_resid out: largest ||r||/||g|| over sites (may be NULL)
 * Errors: EINVAL, ESTATE, EHIP, ENOMEM, ECG_BREAKDOWN (x written). */
int precond_apply(ipeps_ctx* ctx, const double* g, double delta,
                  double cg_tol, int cg_maxiter, double* x, int* n_iter,
                  double* rel_resid);

/* Device-pointer twins of ctm_set_state, ipeps_energy_grad and
 * precond_apply: identical semantics, but A, grad, g and x are device
 * pointers (FP64, same layouts) that the caller keeps resident; no host
 * copies of the site tensors.  The caller makes its device inputs ready
 * before the call (e.g. synchronises the stream that wrote them); each call
 * returns after its results are written (the context stream is
 * synchronised).  Scalars (energy, iteration counts, residuals) still go to
 * host pointers.  Non-finite device inputs are not detected. */
int ctm_set_state_dev(ipeps_ctx* ctx, const double* d_A);
int ipeps_energy_grad_dev(ipeps_ctx* ctx, int n_terms, const ipeps_term* terms,
                          double* e_per_site, double* d_grad);
int precond_apply_dev(ipeps_ctx* ctx, const double* d_g, double delta,
                      double cg_tol, int cg_maxiter, double* d_x, int* n_iter,
                      double* rel_resid);

/* Allocation-free precond_apply_dev, for callers that cannot allocate
 * device memory during the call (code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc).  Same arguments,
 * semantics and results as precond_apply_dev (d_g, d_x device pointers in
 * the layout of A); the metric is applied one physical index at a time.
 * Every temporary of the call lives in one fixed scratch array of
 * IPEPS_NOALLOC_SCRATCH_BYTES per GPU, held from the library's load until
 * the process ends; the call makes no hipMalloc, hipFree or other
 * allocating call.  All calls on one GPU share that array: calls that
 * overlap in time on one GPU (from any context or thread) race and must be
 * serialised by the caller.  A state whose working set
 * (precond_noalloc_bytes) exceeds the array is refused with
 * IPEPS_ESCRATCH before any work.  Errors: EINVAL, ESTATE, ESCRATCH, EHIP,
 * ECG_BREAKDOWN (x written). */
#define IPEPS_NOALLOC_SCRATCH_BYTES ((size_t)192 << 20)
int precond_apply_dev_noalloc(ipeps_ctx* ctx, const double* d_g,
                              double delta, double cg_tol, int cg_maxiter,
                              double* d_x, int* n_iter, double* rel_resid);

/* Scratch bytes precond_apply_dev_noalloc needs for a state of these sizes
 * (an upper estimate; host only).  Returns 0 for invalid sizes. */
size_t precond_noalloc_bytes(int Lx, int Ly, int d, int D, int chi);

/* ------------------------------------------------------------------------
 * C4v-symmetric real ansatz with a QR-based CTMRG (Sec. IV A: a one-site
 * C4v-symmetric real iPEPS, the symmetry fixing the gauge, its environment
 * from a QR-CTMRG, the gradient by reverse mode through the last K
 * iterations).  1x1 unit cells, D >= 2, chi <= 408 (block <= 512).
 *
 * The state is used through its projection A_s, the average of A over the
 * eight elements of the square's symmetry group acting on the virtual legs
 * [l, u, r, d]; c4v_converge and c4v_set_env replace the context's A by
 * A_s.  The environment is one corner C [chi][chi] and one edge T
 * [chi][D^2][chi] (both symmetric in their chi legs) standing for all four
 * corners and edges, plus the warm-start block V [chi D^2][b] of the
 * subspace iteration, b = c4v_block_size(chi) = chi + max(8, ceil(chi/4))
 * made even (-1 when above 512).  One iteration: enlarged corner M = T C T a;
 * while the bond c has c D^2 <= chi it grows untruncated; otherwise one
 * step of block subspace iteration, Q0 = qr(M V) (Cholesky QR in two
 * passes, diag R > 0), Rayleigh-Ritz W of Q0^T M Q0 (the chi eigenvalues of
 * largest |lambda| first, each group in descending signed order),
 * V' = Q0 W with each column's entry of largest |v_r| (1 + r/(2n)) made
 * positive, Q = the first chi columns of V'; C' = Q^T M Q, T' = Q^T (T a) Q,
 * symmetrised and normalised.  The four-corner environment with every
 * corner C and every edge T is written too, so ipeps_energy_grad,
 * precond_apply and the other metric entry points work on it.
 *
 * c4v_converge: from the trace boundary (first call) or the previous C4v
 * environment, until the corner-spectrum change is below tol (raised to
 * the arithmetic's floor) or max_iter iterations.  Returns OK,
 * NOT_CONVERGED (warning), or an error.
 * c4v_energy_grad(_dev): energy per site and the gradient of
 * A -> e(A_s, F^K(C*, T*, V*)) with the converged (C*, T*, V*) held fixed
 * (K = grad_K), which lies in the symmetric subspace; grad NULL for the
 * energy alone (the energy of the last K iterations' environment).
 * c4v_get_env / c4v_set_env: C, T, V host buffers of the sizes above (V
 * may be NULL; on set, NULL means no warm-start block); *bond receives the
 * bond dimension reached (0: none yet).  Setting takes the bond as chi.
 * Errors: EINVAL, ESTATE (no C4v environment), ENOTIMPL (cell larger than
 * 1x1, D < 2 or chi > 408), ENOMEM, EHIP. */
int c4v_block_size(int chi);
int c4v_converge(ipeps_ctx* ctx, double tol, int max_iter, int* n_iter,
                 double* delta);
int c4v_energy_grad(ipeps_ctx* ctx, int n_terms, const ipeps_term* terms,
                    double* e_per_site, double* grad);
int c4v_energy_grad_dev(ipeps_ctx* ctx, int n_terms, const ipeps_term* terms,
                        double* e_per_site, double* d_grad);
int c4v_get_env(ipeps_ctx* ctx, double* C, double* T, double* V, int* bond);
int c4v_set_env(ipeps_ctx* ctx, const double* C, const double* T,
                const double* V);

/* ------------------------------------------------------------------------
 * GMRES solve of the local-metric system (Sec. III C: P g' = g by
 * matrix-vector products only, one outer GMRES iteration of 30 Krylov
 * vectors): the operator of precond_apply, (N_local + delta I), solved per
 * site by one GMRES cycle from x0 = 0 with at most m vectors, stopping
 * early when the residual estimate is <= tol |g| or the Krylov space is
 * invariant (the new vector below 1e-12 of the product it came from).
 *   g, x      layout of A; host (precond_apply_gmres) or device pointers
 *             (precond_apply_gmres_dev)
 *   m         1..256 (30 in the paper)
 *   n_used    out: largest number of Krylov vectors over sites (or NULL)
 *   rel_resid out: largest residual estimate / |g| over sites (or NULL)
 * Errors: EINVAL, ESTATE (no ctm_converge for this state), ENOMEM, EHIP. */
int precond_apply_gmres(ipeps_ctx* ctx, const double* g, double delta, int m,
                        double tol, double* x, int* n_used,
                        double* rel_resid);
int precond_apply_gmres_dev(ipeps_ctx* ctx, const double* d_g, double delta,
                            int m, double tol, double* d_x, int* n_used,
                            double* rel_resid);

/* ------------------------------------------------------------------------
 * Full tangent-space metric (Eq. (10), Sec. III A) of a 1x1 unit cell,
 * applied matrix-free.  N is the mixed ket/bra second derivative of the
 * per-site log-norm F(A_ket, A_bra) = log |kappa|, kappa = n_site n_corner /
 * (n_h n_v): the closed networks of the cell (the ring around the mixed
 * double layer a = sum_p A_ket (x) A_bra; the four corners; the ring with
 * one column removed; with one row removed) on the environment that
 * grad_K CTMRG iterations of a produce from the converged environment of
 * A (ctm_converge first).  The log removes the overlap along the state:
 * N is the connected sum over vacancy separations, symmetric, N A = 0, and
 * infinitesimal gauge transformations of the bonds are zero modes (up to
 * the truncation of the environment).
 *
 * log_norm_grad: F at (A_ket, A) and dF/dA_bra.  A_ket host, layout of A,
 * or NULL for A itself; F host out; g host out (layout of A) or NULL for F
 * only.  With A_ket = A, <g, A> = 1.
 *
 * metric_full_apply: NB = N B by the central difference
 *   (dF/dA_bra(A + h B, A) - dF/dA_bra(A - h B, A)) / (2 h),
 *   h = rel_step |A| / |B|;
 * rel_step 0 selects 1e-5 in FP64 arithmetic and 3e-3 otherwise (the
 * context's late arithmetic: the difference amplifies the rounding of the
 * gradients by |A| / (h |B|)).  Two gradient evaluations per call.
 *
 * precond_apply_full: x = (N + delta I)^-1 g by one GMRES cycle of at most
 * m vectors (stopping rules of precond_apply_gmres); m + 1 metric
 * applications at most.
 *
 * _dev variants take device pointers (same layouts).  Errors: EINVAL,
 * ESTATE (no ctm_converge), ENOTIMPL (unit cell larger than 1x1: there the
 * full metric couples the tensors of the cell), ENOMEM, EHIP. */
int log_norm_grad(ipeps_ctx* ctx, const double* A_ket, double* F,
                  double* g);
int metric_full_apply(ipeps_ctx* ctx, const double* B, double rel_step,
                      double* NB);
int metric_full_apply_dev(ipeps_ctx* ctx, const double* d_B, double rel_step,
                          double* d_NB);
int precond_apply_full(ipeps_ctx* ctx, const double* g, double delta, int m,
                       double tol, double rel_step, double* x, int* n_used,
                       double* rel_resid);
int precond_apply_full_dev(ipeps_ctx* ctx, const double* d_g, double delta,
                           int m, double tol, double rel_step, double* d_x,
                           int* n_used, double* rel_resid);

/* Sum-normalised singular values of every corner, out[4][Lx*Ly][chi] (host),
 * zero padded. Errors: EINVAL, EHIP. */
int ipeps_corner_spectra(ipeps_ctx* ctx, double* out);

/* Copy the environment to / from the host: C[4][Lx*Ly][chi][chi] then
 * T[4][Lx*Ly][chi][D*D][chi].  Index c = 0..3 runs over the upper-left,
 * upper-right, lower-right and lower-left corners and over the top, right,
 * bottom and left edges of a site.  Legs are in clockwise order around the
 * site: C_c[counter-clockwise leg][clockwise leg], T_c[counter-clockwise
 * leg][leg into the site (ket k, bra k' fused as k*D+k')][clockwise leg].
 * Size in doubles: 4*n*chi*chi + 4*n*chi*D*D*chi (ipeps_env_size). */
int ipeps_get_env(ipeps_ctx* ctx, double* out);
int ipeps_set_env(ipeps_ctx* ctx, const double* in);

/* Device-pointer twins of ipeps_get_env / ipeps_set_env: the same layout
 * and size, in device memory the caller keeps (e.g. environments kept
 * resident as warm starts by a request loop); non-finite values are not
 * detected.  Return after the copy is complete.  Errors: EINVAL, EHIP. */
int ipeps_get_env_dev(ipeps_ctx* ctx, double* d_out);
int ipeps_set_env_dev(ipeps_ctx* ctx, const double* d_in);

/* Size in doubles of the environment buffer of ipeps_get_env. */
size_t ipeps_env_size(int Lx, int Ly, int D, int chi);

/* Device bytes a context needs at its peak (the ipeps_energy_grad call,
 * which keeps every intermediate of the K = opts->grad_K unrolled CTMRG
 * iterations, or of one with opts->grad_checkpoint, next to the energy
 * network's tape): an upper estimate for admission decisions, 8 bytes times
 * n_sites * chi^2 D^4 * (46 K + 220) (K = 1 with checkpointing) plus the
 * double-layer tensors
 * (n_sites * 4 (d^2 + 1) D^8) and the environment.  opts NULL = defaults.
 * Returns 0 for invalid sizes.  Host-only; no device call. */
size_t ipeps_footprint_bytes(int Lx, int Ly, int d, int D, int chi,
                             const ipeps_opts* opts);

/* Device memory that destroyed contexts left cached for later contexts of
 * the process (ctm_free keeps a context's blocks in a process-wide list,
 * from which later contexts allocate first) is returned to HIP, largest
 * blocks first, until at most keep_bytes remain cached; *remaining (may be
 * NULL) receives the bytes still cached.  For long-lived processes that
 * share the device with others, e.g. the worker processes of a request
 * loop: without it the cache holds the largest working set any context of
 * the process has had.  Thread-safe (the list is locked; its blocks are
 * idle).  Errors: EHIP. */
int ipeps_release_cache(size_t keep_bytes, size_t* remaining);

/* Kernel timing of the context's own launches, for roofline reports: with
 * on = 1 the context records HIP events on its stream around every launch
 * of the timed kernel families (clearing earlier records); on = 0 stops.
 * Families: 0 = GEMM (FP64 matrix-core GEMM, all shapes), 1 = Jacobi
 * eigensolver, 2 = permute, 3 = FP32 GEMM, 4 = BF16x3 GEMM, 5 = the GEMM
 * launches of the tensor-network contractions (double layer, CTMRG moves,
 * energy network and their reverse passes; any arithmetic, a subset of
 * 0, 3 and 4: the products of the projector SVD and of the complement
 * solves are not in it), 6 = the FP32 GEMM with 128 x 144 tiles (the
 * chi^2 D^8-class products of those contractions: enlarged corners,
 * renormalised edges, open corners; a subset of 3).
 * ipeps_profile_read returns, for one family,
 * the number of launches, their summed device time in seconds and their
 * algorithmic FLOP and byte counts (2 M N K flop; the operand and result
 * bytes of each launch).  Errors: EINVAL, EHIP. */
int ipeps_profile_enable(ipeps_ctx* ctx, int on);
int ipeps_profile_read(ipeps_ctx* ctx, int family, long* launches,
                       double* seconds, double* flop, double* bytes);

/* ------------------------------------------------------------------------
 * Belief-propagation preconditioner (Sec. III A after Eq. (11); App. A):
 * the local metric with environment bond dimension 1, the environment of a
 * site being the product of four D x D messages that belief propagation on
 * the double-layer network provides (a mean-field environment).
 *
 * bp_converge: parallel message updates from the trace message (or from the
 * context's previous messages: a warm start) until the largest change of a
 * normalised message (unit Frobenius norm, positive trace) is below tol or
 * max_iter updates.  Returns OK, NOT_CONVERGED (warning, messages kept), or
 * an error.  The messages belong to the site tensors at the call; a new
 * state (ctm_set_state*) needs a new bp_converge. */
int bp_converge(ipeps_ctx* ctx, double tol, int max_iter, int* n_iter,
                double* change);

/* Messages of the last bp_converge, host out[Ly*Lx][4][D*D]: the message
 * arriving at the left, up, right and down leg of each site, as row-major
 * D x D matrices on the leg's (ket, bra) pair.  Errors: EINVAL, ESTATE. */
int ipeps_bp_messages(ipeps_ctx* ctx, double* out);

/* x = (N_BP + delta I)^-1 g per site, N_BP x = (E x) / Z with
 * E = m_l (x) m_u (x) m_r (x) m_d and Z = <A, E A>, applied in closed form
 * in the eigenbasis of the (symmetrised) messages.  g, x: layout of A, host
 * (precond_apply_bp) or device pointers (precond_apply_bp_dev).  Errors:
 * EINVAL, ESTATE (no bp_converge for the current state), EHIP. */
int precond_apply_bp(ipeps_ctx* ctx, const double* g, double delta,
                     double* x);
int precond_apply_bp_dev(ipeps_ctx* ctx, const double* d_g, double delta,
                         double* d_x);

/* ------------------------------------------------------------------------
 * Preconditioned L-BFGS on the state of a context (Sec. II, Eqs. (1)-(4):
 * the preconditioned gradient P^-1 g enters the quasi-Newton update; the
 * regularised local metric P = N_local + delta I of Sec. III B with an
 * adaptive delta; L-BFGS with history m = 200 and the Hager-Zhang line
 * search of Sec. IV A).  The two-loop recursion starts from H_0 = P^-1
 * (one precond_apply solve at the current point per iteration) or, with
 * precondition = 0, from H_0 = gamma I (gamma = s^T y / y^T y of the newest
 * pair).  Every line-search evaluation writes x + a d into the context,
 * converges its environment from the previous one (ctm_tol, ctm_max_iter)
 * and takes the energy and the gradient in the context's gradient mode and
 * arithmetic.  A step is accepted at the first evaluation meeting the Wolfe
 * or the approximate Wolfe condition of Hager and Zhang (parameters hz_*);
 * after max_evals evaluations the step with the lowest energy is taken.
 * A pair (s, y) enters the history when s^T y > 1e-12 |s| |y|.  The first
 * trial step is 1 (psi0 max|x| / max|g| for the first iteration without
 * the preconditioner).  delta_mode: 0 fixed delta0, 1 |E_{k+1} - E_k|,
 * 2 |g_{k+1}|^2, clamped to [delta_min, delta_max]. */
typedef struct {
  int m;               /* history pairs (200) */
  int precondition;    /* 1 (default): H_0 = P^-1 with the local metric
                          (CG, precond_apply);
                          2: with the belief-propagation metric
                          (bp_converge to ctm_tol within ctm_max_iter
                          updates at every point, precond_apply_bp);
                          3: the local metric by GMRES
                          (precond_apply_gmres, gmres_m vectors);
                          4: the full metric by GMRES (precond_apply_full,
                          gmres_m vectors, 1x1 cells; ENOTIMPL otherwise);
                          0: H_0 = gamma I */
  int delta_mode;      /* 0 fixed, 1 energy change (default), 2 |g|^2 */
  double delta0;       /* delta of the first iteration (1e-2) */
  double delta_min, delta_max;  /* clamp of the adaptive delta (1e-12, 1) */
  double ctm_tol;      /* CTMRG tolerance of every evaluation (1e-10) */
  int ctm_max_iter;    /* (200) */
  double cg_tol;       /* preconditioner CG: relative residual (0) */
  int cg_maxiter;      /* and iteration count (20) */
  int max_evals;       /* line-search evaluations per iteration (20) */
  double psi0;         /* first trial step without preconditioner (0.01) */
  double hz_delta, hz_sigma, hz_eps, hz_theta, hz_gamma, hz_rho;
                       /* 0.1, 0.9, 1e-6, 0.5, 0.66, 5 */
  int gmres_m;         /* Krylov vectors of the GMRES solves (30); the
                          GMRES solves stop early at cg_tol */
  double fd_step;      /* full metric: rel_step of metric_full_apply (0:
                          by arithmetic) */
} ipeps_lbfgs_params;

typedef struct {
  double e;            /* energy per site at the new point */
  double alpha;        /* accepted step along the direction */
  int n_evals;         /* energy+gradient evaluations of the iteration */
  int ls_ok;           /* 1: the step met the line-search conditions */
  double gnorm;        /* |g| at the new point */
  double delta;        /* delta for the next iteration */
  int ctm_iters;       /* CTMRG iterations of the iteration's evaluations */
} ipeps_lbfgs_info;

typedef struct ipeps_lbfgs ipeps_lbfgs;

void ipeps_lbfgs_default_params(ipeps_lbfgs_params* p);

/* Create an optimiser for the context's current state and Hamiltonian
 * (terms copied) and evaluate there (e0: energy per site, may be NULL).
 * The optimiser keeps device buffers in the context (2 m + 7 state-sized
 * vectors) and must be freed before the context.  params NULL = defaults.
 * Errors: EINVAL, ENOMEM, EHIP; warning NOT_CONVERGED. */
int ipeps_lbfgs_create(ipeps_ctx* ctx, int n_terms, const ipeps_term* terms,
                       const ipeps_lbfgs_params* params, ipeps_lbfgs** opt,
                       double* e0);

/* One iteration: direction, line search, history update; the context
 * holds the new state and its environment afterwards (read A with
 * ipeps_get_state).  info may be NULL.  Returns OK; NOT_CONVERGED when the
 * line search ended without meeting its conditions or an evaluation
 * returned a warning (the step is still taken); STATIONARY when no descent
 * direction exists (nothing changed); or an error. */
int ipeps_lbfgs_step(ipeps_lbfgs* opt, ipeps_lbfgs_info* info);

void ipeps_lbfgs_free(ipeps_lbfgs* opt);

/* Copy the context's site tensors to the host, layout of A. */
int ipeps_get_state(ipeps_ctx* ctx, double* A);

/* Release the context and all its device memory (NULL is a no-op). */
void ctm_free(ipeps_ctx* ctx);

/* Static description of a status code. */
const char* ipeps_strerror(int status);

/* Library version string. */
const char* ipeps_version(void);

#ifdef __cplusplus
}
#endif
#endif /* IPEPS_H */
