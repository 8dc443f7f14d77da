// State of one iPEPS context and the declarations of the hot-path stages.
#pragma once

#include <array>
#include <functional>
#include <new>
#include <utility>
#include <vector>

#include "../../include/ipeps.h"
#include "ad.hpp"
#include "engine.hpp"

namespace ipeps {

// Runs f (returning a status) and maps the engine's exceptions to status
// codes: the C ABI never throws.
template <class F>
int guarded_call(F&& f) {
  try {
    return f();
  } catch (const ArgError&) {
    return IPEPS_EINVAL;
  } catch (const NotImplError&) {
    return IPEPS_ENOTIMPL;
  } catch (const OomError&) {
    return IPEPS_ENOMEM;
  } catch (const std::bad_alloc&) {
    return IPEPS_ENOMEM;
  } catch (const HipError&) {
    return IPEPS_EHIP;
  } catch (...) {
    return IPEPS_EHIP;
  }
}

// ---------------------------------------------------------------- SVD
struct CutBatch {
  int ncut = 0;
  int64_t n = 0;   // cut matrix side chi * D^2
  int b = 0;       // subspace block (even)
  int chi = 0;
  std::vector<const double*> Qa, Qb;  // n x n row major, per cut
  // FP32 copies of the same matrices (empty in FP64 arithmetic)
  std::vector<const float*> Qa32, Qb32;
};

// C[i] = op(Q[i]) B[i] for the cut matrices Q (n x n, leading dimension
// ldq), in arithmetic `prec`, from the FP32 copies when there are any.
void qmul(Device& dev, int prec, bool tA, int64_t M, int64_t N, int64_t K,
          const std::vector<const double*>& Q,
          const std::vector<const float*>& Q32, int64_t ldq,
          const std::vector<const double*>& B, int64_t ldb,
          const std::vector<double*>& C, int64_t ldc);

struct SvdParams {
  double tol = 1e-13;
  int max_iter = 50;
  double cutoff = 1e-12;
};

struct SvdStats {
  long iters = 0;
  long calls = 0;
  double worst_residual = 0.0;
  long cg_iters = 0;    // complement solves of the backward pass
  long cg_solves = 0;
  // calls that ended at their iteration limit above the tolerance in effect
  long svd_unconverged = 0;   // projector SVDs (svd_max_iter)
  long cg_unconverged = 0;    // complement solves of the backward pass
  // largest |rhs - A x| / |rhs| of a complement solve, recomputed after the
  // solve (only with Context::check_true_residual)
  double cg_true_residual = 0.0;
};

// tol2: Jacobi criterion of the second pass (1e-15 gives the full FP64
// accuracy; with FP32 or BF16x3 products upstream 1e-12 is below their
// rounding and saves a sweep)
void svd_ts(Device& dev, const Tensor& W, int batch, int64_t n, int b,
            Tensor& U, Tensor& S, Tensor& J, double tol2 = 1e-15);
int subspace_block(int n, int chi, int oversample);
void projector_svd(Device& dev, const CutBatch& cb, Tensor& X, bool warm,
                   Tensor& U, Tensor& S, Tensor& V, Tensor& keep,
                   const SvdParams& prm, SvdStats* stats);

// ------------------------------------------------------------- lattice
// Clockwise conventions (c = 0..3: upper-left, upper-right, lower-right,
// lower-left corner; top, right, bottom, left edge):
//   C_c[ccw, cw], T_c[ccw, in, cw], a_c = a with legs cyclically shifted by c
//   so that a_c[g, e, b, f] has g facing T_{c-1}, e facing T_c, b on the
//   clockwise and f on the counter-clockwise cut of corner c.
struct Lattice {
  int Lx = 1, Ly = 1;
  int n() const { return Lx * Ly; }
  int idx(int x, int y) const {
    x %= Lx;
    if (x < 0) x += Lx;
    y %= Ly;
    if (y < 0) y += Ly;
    return y * Lx + x;
  }
  int shift(int s, int dx, int dy) const {
    return idx(s % Lx + dx, s / Lx + dy);
  }
};

// largest subspace block (b x b Gram, eigen and Cholesky problems of the
// projector SVD and the C4v QR-CTMRG)
constexpr int MAX_BLOCK = 512;
constexpr int PLAQ_OFFSET[4][2] = {{0, 0}, {1, 0}, {1, 1}, {0, 1}};
constexpr int CORNER_MOVE[4][2] = {{1, 1}, {-1, 1}, {-1, -1}, {1, -1}};
constexpr int EDGE_MOVE[4][2] = {{0, 1}, {-1, 0}, {0, -1}, {1, 0}};
constexpr int INIT_CORNER_SITE[4][2] = {{-1, -1}, {1, -1}, {1, 1}, {-1, 1}};
constexpr int INIT_EDGE_SITE[4][2] = {{0, -1}, {1, 0}, {0, 1}, {-1, 0}};

// Environment: C[c][s] (chi x chi) and T[c][s] (chi x D2 x chi) stored in
// two contiguous tensors [4][nsite][...].
struct Env {
  Tensor C, T;
};

// Environment on the differentiation tape: one Var per tensor, index
// c * nsite + s.
struct VEnv {
  std::vector<Var> C, T;
};


struct Context {
  Device dev;
  Lattice lat;
  int d = 0, D = 0, D2 = 0, chi = 0;
  int64_t n = 0;        // chi * D2
  int b = 0;            // subspace block
  int prec = 0;
  double cutoff = 1e-12;
  int grad_K = 20;
  int grad_mode = 1;     // ipeps_grad_mode
  double adj_tol = 1e-13;
  int grad_ckpt = 0;     // recompute the unrolled iterations in the backward
  int grad_K_used = 0;   // K of the last gradient (fixed-point mode)
  double adj_cg_tol = 1e-12;  // complement solves, FP64 products
  int ladder = 0;        // BF16 -> FP32 precision ladder
  // arithmetic of the contractions of the next call: prec, or FP32 once the
  // ladder has stepped up
  int work_prec = 0;
  // test hooks: precondition() stops as at a breakdown before this CG
  // iteration (-1: never)
  int fault_cg_breakdown_at = -1;
  // complement solves of the projector backward: at most this many
  // deflation vectors per half (32); diagnostics of their true residual
  int defl_max = 32;
  bool check_true_residual = false;
  // belief-propagation messages [nsite][4 legs l, u, r, d][D^2] and whether
  // they were converged for the current site tensors
  Tensor bp_msg;
  bool bp_valid = false;
  SvdParams svd;
  SvdStats stats;

  Tensor A;             // [nsite][d][D][D][D][D]
  Tensor a_rot;         // [nsite][4][D2][D2][D2][D2]
  Tensor ao_rot;        // [nsite][4][d][d][D2]^4 (built on demand)
  Env env;
  bool have_env = false;
  bool converged_once = false;
  // the environment was set from outside (ipeps_set_env*) for the current
  // site tensors and is taken to be near its fixed point
  bool env_injected = false;
  Tensor Xwarm;         // [ncut][n][b] right singular blocks (warm start)
  bool have_warm = false;
  // solution of the last complement solve of the projector backward
  // ([ncut][2][n][chi]), the start of the next one within one gradient
  Tensor cg_warm;
  bool have_cg_warm = false;
  // eigenbasis of the deflation Galerkin matrix of that solve, and the
  // squared right-hand-side norms of the gradient's first solve over K^2
  // (the residual scale of the later solves); used, like cg_warm, only
  // within one gradient
  Tensor defl_phi;
  std::vector<double> cg_ref;
  Tensor spec_cur, spec_old;  // [4*nsite][chi]
  // right singular vectors of the corners at the last spectrum (the warm
  // start of the next one) and the calls since the last cold start
  Tensor spec_J;
  int spec_J_age = 0;

  int device = 0;        // HIP device of the context (current at ctm_init)

  // C4v QR-CTMRG state (1x1 cell): corner [chi][chi], edge [chi][D2][chi],
  // warm-start block [chi D2][c4v_b]; c4v_c the bond dimension reached (0:
  // no C4v environment yet)
  Tensor c4v_C, c4v_T, c4v_V;
  int c4v_c = 0;
  int c4v_b = 0;
  bool c4v_sym = false;  // A holds its own symmetric projection

  int nsite() const { return lat.n(); }
  int ncut() const { return 4 * lat.n(); }
  Tensor Cv(const Env& e, int c, int s) const;
  Tensor Tv(const Env& e, int c, int s) const;
  Tensor av(int s, int c) const;
};

// ctmrg.cpp
void build_double_layer(Context& cx);
void init_env(Context& cx);
std::vector<Var> arot_leaves(Tape& tp, Context& cx);
std::vector<Var> arot_from_sites(Tape& tp, Context& cx,
                                 const std::vector<Var>& As);
// double layers of ket Ks[s] and bra Bs[s] (different tensors), rotated
std::vector<Var> arot_from_pairs(Tape& tp, Context& cx,
                                 const std::vector<Var>& Ks,
                                 const std::vector<Var>& Bs);
std::vector<Var> site_leaves(Tape& tp, Context& cx, bool req);
VEnv venv_leaves(Tape& tp, Context& cx, const Env& e, bool req = false);
// The trace-boundary environment as a function of the double layers on the
// tape (the start of the full-N gradient).
VEnv init_env_ad(Tape& tp, Context& cx, const std::vector<Var>& arot);
Env env_pack(Context& cx, const VEnv& v);
// The double layers with their last two legs exchanged, a[g e f b]: the
// layout in which the corner and edge products read them.
std::vector<Var> arot_fb(Tape& tp, const std::vector<Var>& arot);
// One simultaneous CTMRG iteration on the tape (arotf: arot_fb(arot), made
// here when not given).
VEnv ctm_step_ad(Tape& tp, Context& cx, const VEnv& in,
                 const std::vector<Var>& arot,
                 const std::vector<Var>* arotf = nullptr);
// Plain forward iteration (nothing recorded).
void ctm_step(Context& cx, const Env& in, Env& out);
// CTMRG iterations on the context's environment until the corner-spectrum
// change is below tol (raised to the floor of the arithmetic; tol <= 0: a
// fixed count) or max_iter; runs the precision ladder.  Returns 1 when tol
// was not reached or a projector SVD stopped above its tolerance, else 0.
int converge_env(Context& cx, double tol, int max_iter, int* n_iter,
                 double* delta);
// Arithmetic of the gradient and the preconditioner: the context's, or FP32
// behind the precision ladder.
inline int late_prec(const Context& cx) {
  return cx.ladder ? (int)PREC_FP32 : cx.prec;
}
double corner_spectra_change(Context& cx, const Env& e);
void corner_spectra(Context& cx, const Env& e, Tensor& out);

// projector.cpp: differentiable projectors of a batch of cuts
std::pair<std::vector<Var>, std::vector<Var>> projector_op(
    Tape& tp, Context& cx, const std::vector<Var>& Qa,
    const std::vector<Var>& Qb);

// observables.cpp
struct TermSpec {
  int kind, site, dx, dy;
  double coef;
  std::vector<double> mat;
};
// Energy per site on the tape; with recording on, the cotangent of every
// reduced density matrix is seeded (d e / d rho), ready for backward().
double energy_ad(Tape& tp, Context& cx, const VEnv& e,
                 const std::vector<Var>& As, const std::vector<Var>& arot,
                 const std::vector<TermSpec>& terms);
double energy(Context& cx, const Env& e, const std::vector<TermSpec>& terms);
// Checks and copies the Hamiltonian terms of the C ABI (status code).
int parse_terms(const Context& cx, int n_terms, const ipeps_term* H,
                std::vector<TermSpec>& out);

// metric.cpp
// g and x are host pointers, or device pointers when on_device; lean applies
// the metric one physical index at a time (smallest working set)
int precondition(Context& cx, const double* g, double delta, double cg_tol,
                 int cg_maxiter, double* x, int* n_iter, double* rel_resid,
                 bool on_device = false, bool lean = false);
// bp.hip: belief-propagation (chi = 1) environment; returns 1 when tol was
// not reached within max_iter updates
int bp_converge(Context& cx, double tol, int max_iter, int* n_iter,
                double* change);
// x = (N_BP + delta I)^-1 g per site in closed form (g, x host pointers, or
// device pointers when on_device)
int precondition_bp(Context& cx, const double* g, double delta, double* x,
                    bool on_device);
// Device bytes precondition(..., lean = true) works in at most (an upper
// estimate of its temporaries, split-K partial sums included).
size_t precondition_lean_bytes(int nsite, int d, int D, int chi);
// x = (N_local + delta I)^-1 g per site by one GMRES cycle of at most m
// Krylov vectors (g, x host pointers, or device pointers when on_device);
// n_used: largest vector count over sites, rel_resid: largest residual
// estimate
void precondition_gmres(Context& cx, const double* g, double delta, int m,
                        double tol, double* x, int* n_used, double* rel_resid,
                        bool on_device);

// gmres.cpp
// One GMRES cycle from x0 = 0 for op(x) = b, op(in, out) on device vectors
// of length n; Arnoldi by classical Gram-Schmidt with one
// re-orthogonalisation, the Hessenberg least-squares problem by Givens
// rotations on the host.  Stops after m vectors, when the residual
// estimate is <= tol |b|, or when the new Krylov vector is below 1e-12 of
// the product it came from.  x: device out.  Returns the vectors used;
// *rel_resid the residual estimate / |b|.
int gmres(Device& dev, int64_t n, const double* b, double* x, int m,
          double tol, const std::function<void(const double*, double*)>& op,
          double* rel_resid);

// full_metric.cpp (1x1 unit cell)
// F = log kappa of the mixed double layer (ket Ak, bra the context's A),
// K = grad_K CTMRG iterations from the converged environment; gbra
// (device, may be null) receives dF/dA_bra.  Ak: device, layout of A.
double log_kappa_grad(Context& cx, const double* Ak, double* gbra);
// NB = N B, the full metric by the central difference of the bra gradient
// along B in the ket with step rel_step |A| / |B| (device vectors)
void full_metric_apply(Context& cx, const double* B, double* NB,
                       double rel_step);
// x = (N + delta I)^-1 g by one GMRES cycle (host or device pointers)
void precondition_full(Context& cx, const double* g, double delta, int m,
                       double tol, double rel_step, double* x, int* n_used,
                       double* rel_resid, bool on_device);

// c4v.cpp (1x1 cell)
// block size of the subspace iteration: chi + max(8, ceil(chi/4)), even,
// at most 128
int c4v_block(int chi);
// out = the average of in [d][D]^4 over the square's symmetry group acting
// on the virtual legs (in and out device, distinct)
void c4v_symmetrize(Device& dev, const double* in, double* out, int d, int D);
// A <- A_s and the double layer rebuilt
void c4v_project_state(Context& cx);
// QR-CTMRG of the projected state until the corner-spectrum change is
// below tol (raised to the arithmetic's floor) or max_iter iterations;
// writes the replicated four-corner environment; returns 1 when tol was
// not reached
int c4v_converge(Context& cx, double tol, int max_iter, int* n_iter,
                 double* delta);
// (C, T, V) given (host or device; V null: no warm-start block), bond chi;
// the state is projected first
void c4v_set_env(Context& cx, const double* C, const double* T,
                 const double* V, bool on_device);
// energy per site and (grad non-null) the projected K-step gradient, the
// converged (C, T, V) held fixed
double c4v_energy_grad(Context& cx, const std::vector<TermSpec>& terms,
                       double* grad, bool on_device);

// adjoint.cpp
// grad is a host pointer, or a device pointer when on_device
double energy_grad(Context& cx, const std::vector<TermSpec>& terms,
                   double* grad, bool on_device = false);

}  // namespace ipeps

// The opaque context of the C ABI.
struct ipeps_ctx {
  ipeps::Context cx;
};
inline ipeps::Context& ipeps_context(ipeps_ctx* c) { return c->cx; }
