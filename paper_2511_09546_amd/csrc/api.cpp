// C ABI of the library (include/ipeps.h): argument checks, status codes,
// host <-> device copies.  Every entry point catches all exceptions.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>

#include "../../include/ipeps.h"
#include "../../include/ipeps_debug.h"
#include "ipeps_impl.hpp"

using namespace ipeps;

namespace {

template <class F>
int guarded(F&& f) {
  return guarded_call(std::forward<F>(f));
}

bool all_finite(const double* p, size_t n) {
  for (size_t i = 0; i < n; ++i)
    if (!std::isfinite(p[i])) return false;
  return true;
}

size_t state_size(const Context& cx) {
  return (size_t)cx.nsite() * cx.d * cx.D2 * cx.D2;
}

}  // namespace

extern "C" {

void ipeps_default_opts(ipeps_opts* o) {
  if (!o) return;
  o->prec = IPEPS_FP64;
  o->svd_cutoff = 1e-12;
  o->grad_K = 20;
  o->svd_oversample = 0;
  o->svd_max_iter = 50;
  o->svd_tol = 1e-13;
  o->grad_mode = IPEPS_GRAD_K;
  o->adj_tol = 1e-13;
  o->grad_checkpoint = 0;
  o->adj_cg_tol = 1e-12;
  o->ladder = 0;
}

const char* ipeps_version(void) { return "ipeps-mi355x 0.1"; }

const char* ipeps_strerror(int s) {
  switch (s) {
    case IPEPS_OK: return "ok";
    case IPEPS_NOT_CONVERGED: return "not converged (warning)";
    case IPEPS_STATIONARY: return "stationary point: no descent direction";
    case IPEPS_EINVAL: return "invalid argument";
    case IPEPS_ENOMEM: return "device out of memory";
    case IPEPS_EHIP: return "HIP runtime error";
    case IPEPS_ECG_BREAKDOWN: return "CG breakdown (p^T P p <= 0)";
    case IPEPS_ESTATE: return "call out of order";
    case IPEPS_ENOTIMPL: return "not implemented";
    case IPEPS_ESCRATCH:
      return "state too large for the fixed scratch area of "
             "precond_apply_dev_noalloc";
    default: return "unknown status";
  }
}

size_t ipeps_env_size(int Lx, int Ly, int D, int chi) {
  if (Lx < 1 || Ly < 1 || D < 1 || chi < 1) return 0;
  const size_t n = (size_t)Lx * Ly;
  return 4 * n * chi * chi + 4 * n * chi * (size_t)D * D * chi;
}

int ipeps_release_cache(size_t keep_bytes, size_t* remaining) {
  return guarded([&]() {
    const size_t left = trim_idle_to(keep_bytes);
    if (remaining) *remaining = left;
    return IPEPS_OK;
  });
}

size_t ipeps_footprint_bytes(int Lx, int Ly, int d, int D, int chi,
                             const ipeps_opts* opts) {
  if (Lx < 1 || Ly < 1 || d < 1 || D < 1 || chi < 1) return 0;
  ipeps_opts o;
  ipeps_default_opts(&o);
  if (opts) o = *opts;
  const double ns = (double)Lx * Ly, D2 = (double)D * D, D4 = D2 * D2;
  const double q = (double)chi * chi * D4;  // one enlarged corner
  // gradient intermediates of K unrolled iterations, or of one with
  // checkpointing (the stored input environments are small)
  const double K = o.grad_checkpoint ? 1.0 : (o.grad_K > 0 ? o.grad_K : 0);
  const double dbl = ns * 4.0 * ((double)d * d + 1.0) * D4 * D4;
  // 46 enlarged-corner sizes per resident unrolled iteration and 220 for
  // the energy network's tape and the rest (peaks measured per site: 957
  // and 163 at K = 20 without and with checkpointing, D = 6, chi = 72;
  // 1045 and 234 for the 2x2 Kitaev cell, D = 5, chi = 50)
  const double words = ns * q * (46.0 * K + 220.0) + dbl +
                       (double)ipeps_env_size(Lx, Ly, D, chi);
  return (size_t)(8.0 * words);
}

int ctm_init(ipeps_ctx** out, int Lx, int Ly, int d, int D, int chi,
             const double* A, const ipeps_opts* opts, void* hip_stream) {
  if (!out || !A || Lx < 1 || Ly < 1 || d < 1 || D < 1 || chi < D * D ||
      Lx * Ly > 64 || d > 16 || D > 16)
    return IPEPS_EINVAL;
  ipeps_opts o;
  ipeps_default_opts(&o);
  if (opts) o = *opts;
  if (o.prec != IPEPS_FP64 && o.prec != IPEPS_FP32 && o.prec != IPEPS_BF16 &&
      o.prec != IPEPS_BF16X1)
    return IPEPS_EINVAL;
  if (!(o.adj_cg_tol > 0.0) || (o.ladder != 0 && o.ladder != 1) ||
      (o.ladder == 1 && o.prec != IPEPS_BF16 && o.prec != IPEPS_BF16X1))
    return IPEPS_EINVAL;
  if (!(o.svd_cutoff >= 0.0) || o.grad_K < 0 || o.svd_max_iter < 1 ||
      !(o.svd_tol >= 0.0) || o.svd_oversample < 0 ||
      (o.grad_mode != IPEPS_GRAD_FULL && o.grad_mode != IPEPS_GRAD_K &&
       o.grad_mode != IPEPS_GRAD_FP) ||
      !(o.adj_tol > 0.0) || (o.grad_mode == IPEPS_GRAD_FP && o.grad_K < 1) ||
      (o.grad_checkpoint != 0 && o.grad_checkpoint != 1))
    return IPEPS_EINVAL;
  const size_t nA = (size_t)Lx * Ly * d * D * D * D * D;
  if (!all_finite(A, nA)) return IPEPS_EINVAL;
  ipeps_ctx* c = nullptr;
  int st = guarded([&]() {
    prime_attributes();
    c = new ipeps_ctx();
    Context& cx = c->cx;
    if (hip_stream) {
      cx.dev.stream = (hipStream_t)hip_stream;
    } else {
      IPEPS_HIP(hipStreamCreate(&cx.dev.stream));
      cx.dev.own_stream = true;
    }
    IPEPS_HIP(hipGetDevice(&cx.device));
    cx.lat.Lx = Lx;
    cx.lat.Ly = Ly;
    cx.d = d;
    cx.D = D;
    cx.D2 = D * D;
    cx.chi = chi;
    cx.n = (int64_t)chi * D * D;
    cx.prec = o.prec;
    cx.grad_K = o.grad_K;
    cx.grad_mode = o.grad_mode;
    cx.adj_tol = o.adj_tol;
    cx.grad_ckpt = o.grad_checkpoint;
    cx.adj_cg_tol = o.adj_cg_tol;
    cx.ladder = o.ladder;
    cx.work_prec = o.prec;
    cx.svd.cutoff = o.svd_cutoff;
    cx.svd.tol = o.svd_tol;
    cx.svd.max_iter = o.svd_max_iter;
    cx.b = subspace_block((int)cx.n, chi, o.svd_oversample);
    cx.A = cx.dev.empty({Lx * Ly, d, D, D, D, D});
    cx.dev.upload(cx.A, A);
    build_double_layer(cx);
    init_env(cx);
    (void)corner_spectra_change(cx, cx.env);  // reference spectra
    cx.dev.sync();
    return IPEPS_OK;
  });
  if (st != IPEPS_OK) {
    if (c) {
      hipStream_t s = c->cx.dev.stream;
      const bool own = c->cx.dev.own_stream;
      if (s) (void)hipStreamSynchronize(s);  // blocks are idle before reuse
      delete c;
      if (own && s) (void)hipStreamDestroy(s);
    }
    return st;
  }
  *out = c;
  return IPEPS_OK;
}

int ctm_set_state(ipeps_ctx* c, const double* A) {
  if (!c || !A) return IPEPS_EINVAL;
  Context& cx = c->cx;
  if (!all_finite(A, state_size(cx))) return IPEPS_EINVAL;
  return guarded([&]() {
    cx.dev.upload(cx.A, A);
    build_double_layer(cx);
    cx.dev.sync();
    return IPEPS_OK;
  });
}

int ctm_converge(ipeps_ctx* c, double tol, int max_iter, int* n_iter,
                 double* delta) {
  if (!c || max_iter < 0 || std::isnan(tol)) return IPEPS_EINVAL;
  Context& cx = c->cx;
  int it = 0, warn = 0;
  double dl = INFINITY;
  int st = guarded([&]() {
    warn = converge_env(cx, tol, max_iter, &it, &dl);
    return IPEPS_OK;
  });
  if (st != IPEPS_OK) return st;
  if (n_iter) *n_iter = it;
  if (delta) *delta = dl;
  return warn ? IPEPS_NOT_CONVERGED : IPEPS_OK;
}

// NOT_CONVERGED when a projector SVD or a complement solve of the call
// stopped at its iteration limit above its tolerance (outputs valid).
static int solver_warning(const Context& cx, long svd0, long cg0) {
  return (cx.stats.svd_unconverged != svd0 || cx.stats.cg_unconverged != cg0)
             ? IPEPS_NOT_CONVERGED
             : IPEPS_OK;
}

}  // extern "C"

int ipeps::parse_terms(const Context& cx, int n_terms, const ipeps_term* H,
                       std::vector<TermSpec>& out) {
  if (n_terms < 0 || (n_terms > 0 && !H)) return IPEPS_EINVAL;
  for (int i = 0; i < n_terms; ++i) {
    const ipeps_term& t = H[i];
    if (!t.mat || t.site < 0 || t.site >= cx.nsite() || !std::isfinite(t.coef))
      return IPEPS_EINVAL;
    TermSpec s;
    s.kind = t.kind;
    s.site = t.site;
    s.dx = t.dx;
    s.dy = t.dy;
    s.coef = t.coef;
    size_t m;
    if (t.kind == 0) {
      m = (size_t)cx.d;
    } else if (t.kind == 1) {
      const bool ok = (t.dx == 1 && t.dy == 0) || (t.dx == 0 && t.dy == 1) ||
                      (t.dx == 1 && t.dy == 1) || (t.dx == 1 && t.dy == -1);
      if (!ok) return IPEPS_EINVAL;
      m = (size_t)cx.d * cx.d;
    } else {
      return IPEPS_EINVAL;
    }
    if (!all_finite(t.mat, m * m)) return IPEPS_EINVAL;
    s.mat.assign(t.mat, t.mat + m * m);
    out.push_back(std::move(s));
  }
  return IPEPS_OK;
}

extern "C" {

int ipeps_energy_grad(ipeps_ctx* c, int n_terms, const ipeps_term* H,
                      double* e_per_site, double* grad) {
  if (!c || !e_per_site) return IPEPS_EINVAL;
  Context& cx = c->cx;
  std::vector<TermSpec> terms;
  int st = parse_terms(cx, n_terms, H, terms);
  if (st != IPEPS_OK) return st;
  if (!cx.converged_once) return IPEPS_ESTATE;
  double e = 0.0;
  const long svd0 = cx.stats.svd_unconverged, cg0 = cx.stats.cg_unconverged;
  st = guarded([&]() {
    PrecScope ps(cx.dev, late_prec(cx));
    if (grad) {
      e = energy_grad(cx, terms, grad);
    } else {
      e = energy(cx, cx.env, terms);
    }
    return IPEPS_OK;
  });
  if (st != IPEPS_OK) return st;
  *e_per_site = e;
  return solver_warning(cx, svd0, cg0);
}

int precond_apply(ipeps_ctx* c, const double* g, double delta, double cg_tol,
                  int cg_maxiter, double* x, int* n_iter, double* rel_resid) {
  if (!c || !g || !x || !(delta > 0.0) || !std::isfinite(delta) ||
      !(cg_tol >= 0.0) || cg_maxiter < 0)
    return IPEPS_EINVAL;
  Context& cx = c->cx;
  if (!all_finite(g, state_size(cx))) return IPEPS_EINVAL;
  if (!cx.converged_once) return IPEPS_ESTATE;
  int res = 0;
  int st = guarded([&]() {
    PrecScope ps(cx.dev, late_prec(cx));
    res = precondition(cx, g, delta, cg_tol, cg_maxiter, x, n_iter,
                       rel_resid);
    return IPEPS_OK;
  });
  if (st != IPEPS_OK) return st;
  return res;
}

int ctm_set_state_dev(ipeps_ctx* c, const double* dA) {
  if (!c || !dA) return IPEPS_EINVAL;
  Context& cx = c->cx;
  return guarded([&]() {
    axpby(cx.dev, cx.A.numel(), 1.0, dA, 0.0, cx.A.ptr);
    build_double_layer(cx);
    cx.dev.sync();
    return IPEPS_OK;
  });
}

int ipeps_energy_grad_dev(ipeps_ctx* c, int n_terms, const ipeps_term* H,
                          double* e_per_site, double* d_grad) {
  if (!c || !e_per_site || !d_grad) return IPEPS_EINVAL;
  Context& cx = c->cx;
  std::vector<TermSpec> terms;
  int st = parse_terms(cx, n_terms, H, terms);
  if (st != IPEPS_OK) return st;
  if (!cx.converged_once) return IPEPS_ESTATE;
  double e = 0.0;
  const long svd0 = cx.stats.svd_unconverged, cg0 = cx.stats.cg_unconverged;
  st = guarded([&]() {
    PrecScope ps(cx.dev, late_prec(cx));
    e = energy_grad(cx, terms, d_grad, true);
    return IPEPS_OK;
  });
  if (st != IPEPS_OK) return st;
  *e_per_site = e;
  return solver_warning(cx, svd0, cg0);
}

int precond_apply_dev(ipeps_ctx* c, const double* d_g, double delta,
                      double cg_tol, int cg_maxiter, double* d_x, int* n_iter,
                      double* rel_resid) {
  if (!c || !d_g || !d_x || !(delta > 0.0) || !std::isfinite(delta) ||
      !(cg_tol >= 0.0) || cg_maxiter < 0)
    return IPEPS_EINVAL;
  Context& cx = c->cx;
  if (!cx.converged_once) return IPEPS_ESTATE;
  int res = 0;
  int st = guarded([&]() {
    PrecScope ps(cx.dev, late_prec(cx));
    res = precondition(cx, d_g, delta, cg_tol, cg_maxiter, d_x, n_iter,
                       rel_resid, true);
    return IPEPS_OK;
  });
  if (st != IPEPS_OK) return st;
  return res;
}

int c4v_block_size(int chi) {
  return chi >= 1 && c4v_block(chi) <= MAX_BLOCK ? c4v_block(chi) : -1;
}

static int c4v_ok(const Context& cx) {
  if (cx.nsite() != 1 || cx.D < 2 || c4v_block(cx.chi) > MAX_BLOCK)
    return IPEPS_ENOTIMPL;
  return IPEPS_OK;
}

int c4v_converge(ipeps_ctx* c, double tol, int max_iter, int* n_iter,
                 double* delta) {
  if (!c || max_iter < 0 || std::isnan(tol)) return IPEPS_EINVAL;
  Context& cx = c->cx;
  int st = c4v_ok(cx);
  if (st != IPEPS_OK) return st;
  int it = 0, warn = 0;
  double dl = INFINITY;
  st = guarded([&]() {
    warn = ipeps::c4v_converge(cx, tol, max_iter, &it, &dl);
    return IPEPS_OK;
  });
  if (st != IPEPS_OK) return st;
  if (n_iter) *n_iter = it;
  if (delta) *delta = dl;
  return warn ? IPEPS_NOT_CONVERGED : IPEPS_OK;
}

static int c4v_eg_impl(ipeps_ctx* c, int n_terms, const ipeps_term* H,
                       double* e_per_site, double* grad, bool dev) {
  if (!c || !e_per_site) return IPEPS_EINVAL;
  Context& cx = c->cx;
  int st = c4v_ok(cx);
  if (st != IPEPS_OK) return st;
  std::vector<TermSpec> terms;
  st = parse_terms(cx, n_terms, H, terms);
  if (st != IPEPS_OK) return st;
  if (cx.c4v_c == 0) return IPEPS_ESTATE;
  double e = 0.0;
  st = guarded([&]() {
    PrecScope ps(cx.dev, late_prec(cx));
    e = ipeps::c4v_energy_grad(cx, terms, grad, dev);
    return IPEPS_OK;
  });
  if (st != IPEPS_OK) return st;
  *e_per_site = e;
  return IPEPS_OK;
}

int c4v_energy_grad(ipeps_ctx* c, int n_terms, const ipeps_term* H,
                    double* e_per_site, double* grad) {
  return c4v_eg_impl(c, n_terms, H, e_per_site, grad, false);
}

int c4v_energy_grad_dev(ipeps_ctx* c, int n_terms, const ipeps_term* H,
                        double* e_per_site, double* d_grad) {
  if (!d_grad) return IPEPS_EINVAL;
  return c4v_eg_impl(c, n_terms, H, e_per_site, d_grad, true);
}

int c4v_get_env(ipeps_ctx* c, double* C, double* T, double* V, int* bond) {
  if (!c || !C || !T) return IPEPS_EINVAL;
  Context& cx = c->cx;
  int st = c4v_ok(cx);
  if (st != IPEPS_OK) return st;
  if (cx.c4v_c == 0) return IPEPS_ESTATE;
  return guarded([&]() {
    cx.dev.download(cx.c4v_C, C);
    cx.dev.download(cx.c4v_T, T);
    if (V) {
      if (cx.c4v_V.ptr)
        cx.dev.download(cx.c4v_V, V);
      else
        std::fill(V, V + (size_t)cx.chi * cx.D2 * c4v_block(cx.chi), 0.0);
    }
    if (bond) *bond = cx.c4v_c;
    return IPEPS_OK;
  });
}

int c4v_set_env(ipeps_ctx* c, const double* C, const double* T,
                const double* V) {
  if (!c || !C || !T) return IPEPS_EINVAL;
  Context& cx = c->cx;
  int st = c4v_ok(cx);
  if (st != IPEPS_OK) return st;
  const size_t nc = (size_t)cx.chi * cx.chi, nt = nc * cx.D2;
  if (!all_finite(C, nc) || !all_finite(T, nt) ||
      (V && !all_finite(V, (size_t)cx.chi * cx.D2 * c4v_block(cx.chi))))
    return IPEPS_EINVAL;
  return guarded([&]() {
    ipeps::c4v_set_env(cx, C, T, V, false);
    return IPEPS_OK;
  });
}

static int gmres_args_ok(double delta, int m, double tol) {
  return delta > 0.0 && std::isfinite(delta) && m >= 1 && m <= 256 &&
         tol >= 0.0 && std::isfinite(tol);
}

static int precond_gmres_impl(ipeps_ctx* c, const double* g, double delta,
                              int m, double tol, double* x, int* n_used,
                              double* rel_resid, bool dev) {
  if (!c || !g || !x || !gmres_args_ok(delta, m, tol)) return IPEPS_EINVAL;
  Context& cx = c->cx;
  if (!dev && !all_finite(g, state_size(cx))) return IPEPS_EINVAL;
  if (!cx.converged_once) return IPEPS_ESTATE;
  return guarded([&]() {
    PrecScope ps(cx.dev, late_prec(cx));
    precondition_gmres(cx, g, delta, m, tol, x, n_used, rel_resid, dev);
    return IPEPS_OK;
  });
}

int precond_apply_gmres(ipeps_ctx* c, const double* g, double delta, int m,
                        double tol, double* x, int* n_used,
                        double* rel_resid) {
  return precond_gmres_impl(c, g, delta, m, tol, x, n_used, rel_resid, false);
}

int precond_apply_gmres_dev(ipeps_ctx* c, const double* d_g, double delta,
                            int m, double tol, double* d_x, int* n_used,
                            double* rel_resid) {
  return precond_gmres_impl(c, d_g, delta, m, tol, d_x, n_used, rel_resid,
                            true);
}

// the central-difference step of the full metric: 1e-5 |A| / |B| in FP64,
// 3e-3 |A| / |B| in the FP32-class arithmetics
static double full_step(const Context& cx, double rel_step) {
  if (rel_step > 0.0) return rel_step;
  return late_prec(cx) == PREC_FP64 ? 1e-5 : 3e-3;
}

static int full_ok(const Context& cx) {
  if (!cx.converged_once) return IPEPS_ESTATE;
  if (cx.nsite() != 1) return IPEPS_ENOTIMPL;
  return IPEPS_OK;
}

int log_norm_grad(ipeps_ctx* c, const double* A_ket, double* F, double* g) {
  if (!c || !F) return IPEPS_EINVAL;
  Context& cx = c->cx;
  if (A_ket && !all_finite(A_ket, state_size(cx))) return IPEPS_EINVAL;
  int st = full_ok(cx);
  if (st != IPEPS_OK) return st;
  return guarded([&]() {
    PrecScope ps(cx.dev, late_prec(cx));
    Tensor Ak = cx.A;
    if (A_ket) {
      Ak = cx.dev.empty(cx.A.shape);
      cx.dev.upload(Ak, A_ket);
    }
    Tensor gd;
    if (g) gd = cx.dev.empty(cx.A.shape);
    *F = log_kappa_grad(cx, Ak.ptr, g ? gd.ptr : nullptr);
    if (g) cx.dev.download(gd, g);
    return IPEPS_OK;
  });
}

static int metric_full_impl(ipeps_ctx* c, const double* B, double rel_step,
                            double* NB, bool dev) {
  if (!c || !B || !NB || !(rel_step >= 0.0) || !(rel_step < 1.0))
    return IPEPS_EINVAL;
  Context& cx = c->cx;
  if (!dev && !all_finite(B, state_size(cx))) return IPEPS_EINVAL;
  int st = full_ok(cx);
  if (st != IPEPS_OK) return st;
  return guarded([&]() {
    PrecScope ps(cx.dev, late_prec(cx));
    const double h = full_step(cx, rel_step);
    if (dev) {
      full_metric_apply(cx, B, NB, h);
      cx.dev.sync();
    } else {
      Tensor b = cx.dev.empty(cx.A.shape), y = cx.dev.empty(cx.A.shape);
      cx.dev.upload(b, B);
      full_metric_apply(cx, b.ptr, y.ptr, h);
      cx.dev.download(y, NB);
    }
    return IPEPS_OK;
  });
}

int metric_full_apply(ipeps_ctx* c, const double* B, double rel_step,
                      double* NB) {
  return metric_full_impl(c, B, rel_step, NB, false);
}

int metric_full_apply_dev(ipeps_ctx* c, const double* d_B, double rel_step,
                          double* d_NB) {
  return metric_full_impl(c, d_B, rel_step, d_NB, true);
}

static int precond_full_impl(ipeps_ctx* c, const double* g, double delta,
                             int m, double tol, double rel_step, double* x,
                             int* n_used, double* rel_resid, bool dev) {
  if (!c || !g || !x || !gmres_args_ok(delta, m, tol) ||
      !(rel_step >= 0.0) || !(rel_step < 1.0))
    return IPEPS_EINVAL;
  Context& cx = c->cx;
  if (!dev && !all_finite(g, state_size(cx))) return IPEPS_EINVAL;
  int st = full_ok(cx);
  if (st != IPEPS_OK) return st;
  return guarded([&]() {
    PrecScope ps(cx.dev, late_prec(cx));
    precondition_full(cx, g, delta, m, tol, full_step(cx, rel_step), x,
                      n_used, rel_resid, dev);
    return IPEPS_OK;
  });
}

int precond_apply_full(ipeps_ctx* c, const double* g, double delta, int m,
                       double tol, double rel_step, double* x, int* n_used,
                       double* rel_resid) {
  return precond_full_impl(c, g, delta, m, tol, rel_step, x, n_used,
                           rel_resid, false);
}

int precond_apply_full_dev(ipeps_ctx* c, const double* d_g, double delta,
                           int m, double tol, double rel_step, double* d_x,
                           int* n_used, double* rel_resid) {
  return precond_full_impl(c, d_g, delta, m, tol, rel_step, d_x, n_used,
                           rel_resid, true);
}

int bp_converge(ipeps_ctx* c, double tol, int max_iter, int* n_iter,
                double* change) {
  if (!c || max_iter < 1 || !(tol >= 0.0)) return IPEPS_EINVAL;
  Context& cx = c->cx;
  int warn = 0, it = 0;
  double ch = 0.0;
  int st = guarded([&]() {
    warn = ipeps::bp_converge(cx, tol, max_iter, &it, &ch);
    return IPEPS_OK;
  });
  if (st != IPEPS_OK) return st;
  if (n_iter) *n_iter = it;
  if (change) *change = ch;
  return warn ? IPEPS_NOT_CONVERGED : IPEPS_OK;
}

int ipeps_bp_messages(ipeps_ctx* c, double* out) {
  if (!c || !out) return IPEPS_EINVAL;
  Context& cx = c->cx;
  if (!cx.bp_valid) return IPEPS_ESTATE;
  return guarded([&]() {
    cx.dev.download(cx.bp_msg, out);
    return IPEPS_OK;
  });
}

int precond_apply_bp(ipeps_ctx* c, const double* g, double delta,
                     double* x) {
  if (!c || !g || !x || !(delta > 0.0) || !std::isfinite(delta))
    return IPEPS_EINVAL;
  Context& cx = c->cx;
  if (!all_finite(g, state_size(cx))) return IPEPS_EINVAL;
  if (!cx.bp_valid) return IPEPS_ESTATE;
  return guarded([&]() {
    precondition_bp(cx, g, delta, x, false);
    return IPEPS_OK;
  });
}

int precond_apply_bp_dev(ipeps_ctx* c, const double* d_g, double delta,
                         double* d_x) {
  if (!c || !d_g || !d_x || !(delta > 0.0) || !std::isfinite(delta))
    return IPEPS_EINVAL;
  Context& cx = c->cx;
  if (!cx.bp_valid) return IPEPS_ESTATE;
  return guarded([&]() {
    precondition_bp(cx, d_g, delta, d_x, true);
    return IPEPS_OK;
  });
}

int ipeps_get_state(ipeps_ctx* c, double* A) {
  if (!c || !A) return IPEPS_EINVAL;
  Context& cx = c->cx;
  return guarded([&]() {
    cx.dev.download(cx.A, A);
    return IPEPS_OK;
  });
}

int ipeps_corner_spectra(ipeps_ctx* c, double* out) {
  if (!c || !out) return IPEPS_EINVAL;
  Context& cx = c->cx;
  return guarded([&]() {
    (void)corner_spectra_change(cx, cx.env);
    cx.dev.download(cx.spec_cur, out);
    return IPEPS_OK;
  });
}

int ipeps_get_env(ipeps_ctx* c, double* out) {
  if (!c || !out) return IPEPS_EINVAL;
  Context& cx = c->cx;
  return guarded([&]() {
    cx.dev.download(cx.env.C, out);
    cx.dev.download(cx.env.T, out + cx.env.C.numel());
    return IPEPS_OK;
  });
}

int ipeps_set_env(ipeps_ctx* c, const double* in) {
  if (!c || !in) return IPEPS_EINVAL;
  Context& cx = c->cx;
  const size_t n = ipeps_env_size(cx.lat.Lx, cx.lat.Ly, cx.D, cx.chi);
  if (!all_finite(in, n)) return IPEPS_EINVAL;
  return guarded([&]() {
    Env e;
    e.C = cx.dev.empty({4, cx.nsite(), cx.chi, cx.chi});
    e.T = cx.dev.empty({4, cx.nsite(), cx.chi, cx.D2, cx.chi});
    cx.dev.upload(e.C, in);
    cx.dev.upload(e.T, in + e.C.numel());
    cx.env = e;
    cx.have_warm = false;
    cx.converged_once = true;
    cx.env_injected = true;
    cx.work_prec = cx.prec;  // a new environment climbs the ladder again
    (void)corner_spectra_change(cx, cx.env);
    cx.dev.sync();
    return IPEPS_OK;
  });
}

int ipeps_get_env_dev(ipeps_ctx* c, double* d_out) {
  if (!c || !d_out) return IPEPS_EINVAL;
  Context& cx = c->cx;
  return guarded([&]() {
    const int64_t nc = cx.env.C.numel();
    axpby(cx.dev, nc, 1.0, cx.env.C.ptr, 0.0, d_out);
    axpby(cx.dev, cx.env.T.numel(), 1.0, cx.env.T.ptr, 0.0, d_out + nc);
    cx.dev.sync();
    return IPEPS_OK;
  });
}

int ipeps_set_env_dev(ipeps_ctx* c, const double* d_in) {
  if (!c || !d_in) return IPEPS_EINVAL;
  Context& cx = c->cx;
  return guarded([&]() {
    Env e;
    e.C = cx.dev.empty({4, cx.nsite(), cx.chi, cx.chi});
    e.T = cx.dev.empty({4, cx.nsite(), cx.chi, cx.D2, cx.chi});
    axpby(cx.dev, e.C.numel(), 1.0, d_in, 0.0, e.C.ptr);
    axpby(cx.dev, e.T.numel(), 1.0, d_in + e.C.numel(), 0.0, e.T.ptr);
    cx.env = e;
    cx.have_warm = false;
    cx.converged_once = true;
    cx.env_injected = true;
    cx.work_prec = cx.prec;
    (void)corner_spectra_change(cx, cx.env);
    cx.dev.sync();
    return IPEPS_OK;
  });
}

int ipeps_profile_enable(ipeps_ctx* c, int on) {
  if (!c) return IPEPS_EINVAL;
  Context& cx = c->cx;
  return guarded([&]() {
    cx.dev.sync();
    cx.dev.prof.clear();
    cx.dev.prof.on = on != 0;
    if (on) cx.dev.prof.reserve(1 << 17);
    return IPEPS_OK;
  });
}

int ipeps_profile_read(ipeps_ctx* c, int family, long* launches,
                       double* seconds, double* flop, double* bytes) {
  if (!c || family < 0 || family >= PROF_N || !launches || !seconds ||
      !flop || !bytes)
    return IPEPS_EINVAL;
  Context& cx = c->cx;
  return guarded([&]() {
    cx.dev.prof.read(family, launches, seconds, flop, bytes);
    return IPEPS_OK;
  });
}

int ipeps_debug_stats(ipeps_ctx* c, double* out) {
  if (!c || !out) return IPEPS_EINVAL;
  const SvdStats& st = c->cx.stats;
  out[0] = (double)st.iters;
  out[1] = (double)st.calls;
  out[2] = st.worst_residual;
  out[3] = (double)st.cg_iters;
  out[4] = (double)st.cg_solves;
  out[5] = (double)c->cx.dev.pool.reserved();
  out[6] = (double)c->cx.dev.pool.peak_live();
  out[7] = (double)c->cx.grad_K_used;
  out[8] = (double)st.svd_unconverged;
  out[9] = (double)st.cg_unconverged;
  out[10] = (double)c->cx.work_prec;
  out[11] = st.cg_true_residual;
  return IPEPS_OK;
}

int ipeps_debug_memcheck(ipeps_ctx* c, long* damaged) {
  if (!c || !damaged) return IPEPS_EINVAL;
  Context& cx = c->cx;
  if (cx.dev.memcheck <= 0) {
    *damaged = -1;
    return IPEPS_OK;
  }
  return guarded([&]() {
    *damaged = cx.dev.memcheck_pending + cx.dev.memcheck_verify();
    cx.dev.memcheck_pending = 0;
    return IPEPS_OK;
  });
}

int ipeps_debug_set_fault(ipeps_ctx* c, int kind, double value) {
  if (!c || !(value >= 0.0)) return IPEPS_EINVAL;
  Context& cx = c->cx;
  switch (kind) {
    case 0:
      cx.dev.pool.set_limit(SIZE_MAX);
      cx.fault_cg_breakdown_at = -1;
      cx.defl_max = 32;
      cx.check_true_residual = false;
      return IPEPS_OK;
    case 1:
      cx.dev.pool.set_limit(value >= 1.8e19 ? SIZE_MAX : (size_t)value);
      return IPEPS_OK;
    case 2:
      cx.fault_cg_breakdown_at = value > 2e9 ? -1 : (int)value;
      return IPEPS_OK;
    case 3:
      cx.defl_max = value > 128 ? 128 : (int)value;
      return IPEPS_OK;
    case 4:
      cx.check_true_residual = value != 0.0;
      return IPEPS_OK;
    default:
      return IPEPS_EINVAL;
  }
}

void ctm_free(ipeps_ctx* c) {
  if (!c) return;
  hipStream_t s = c->cx.dev.stream;
  bool own = c->cx.dev.own_stream;
  if (s) (void)hipStreamSynchronize(s);
  if (c->cx.dev.memcheck > 0) {
    try {
      const long bad =
          c->cx.dev.memcheck_pending + c->cx.dev.memcheck_verify();
      if (bad) std::fprintf(stderr, "memcheck: %ld damaged guards\n", bad);
    } catch (...) {
    }
  }
  delete c;
  if (own && s) (void)hipStreamDestroy(s);
}

}  // extern "C"
