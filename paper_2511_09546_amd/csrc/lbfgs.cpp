// Preconditioned L-BFGS with the Hager-Zhang line search on the device state
// of a context (include/ipeps.h, ipeps_lbfgs_*).
//
// The paper minimises E(A) with L-BFGS (history m = 200, Hager-Zhang line
// search, Sec. IV A) and enters the preconditioned gradient P^-1 g of
// Sec. II (Eqs. (1)-(4)) with the regularised local metric P = N + delta I
// (Sec. III B) and an adaptive delta.  Here:
//   * two-loop recursion (Nocedal & Wright) over pairs (s_i, y_i) kept in
//     device ring buffers, with H_0 = P^-1 applied by the local-metric CG of
//     precondition() at the current point (no further scaling), or
//     H_0 = gamma I, gamma = s^T y / y^T y of the newest pair, without it;
//   * the line search of Hager and Zhang (SIAM J. Optim. 16 (2005) 170):
//     bracket by expansion (factor rho), then secant^2 steps with the update
//     rule and bisection when an interval shrinks by less than gamma; a step
//     is accepted at the first evaluation that meets the Wolfe condition or
//     the approximate Wolfe condition (slack eps |f(x_k)|); after max_evals
//     evaluations the evaluated step with the lowest energy is taken and
//     evaluated again, so that the context holds its environment;
//   * every evaluation of phi(a) = E(x + a d) writes x + a d into the
//     context, converges its environment from the previous evaluation's,
//     and takes the energy and the gradient (the context's gradient mode),
//     phi'(a) = g . d;
//   * a pair enters the history when s^T y > 1e-12 |s| |y| (oldest of m
//     dropped); the first trial step is 1 with the preconditioner and
//     psi0 max|x| / max|g| for the first iteration without it, 1 after;
//   * delta of the next iteration: |E_{k+1} - E_k| (mode 1), |g_{k+1}|^2
//     (mode 2) or delta0 (mode 0), clamped to [delta_min, delta_max].
// The vector work (dots, axpys, the metric solve, the evaluations) runs in
// the library's kernels; the scalar control of the line search runs on the
// host.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <functional>
#include <map>
#include <new>
#include <utility>

#include "../../include/ipeps.h"
#include "ipeps_impl.hpp"

namespace ipeps {

namespace {

struct Params {
  int m, precondition, delta_mode, ctm_max_iter, cg_maxiter, max_evals;
  double delta0, delta_min, delta_max, ctm_tol, cg_tol, psi0;
  double hz_delta, hz_sigma, hz_eps, hz_theta, hz_gamma, hz_rho;
  int gmres_m;
  double fd_step;
};

// Hager-Zhang line search on phi with phi(0) = phi0, phi'(0) = dphi0 < 0.
class HagerZhang {
 public:
  template <class F>
  HagerZhang(F&& phi, double phi0, double dphi0, double fscale,
             const Params& p)
      : phi_(std::forward<F>(phi)), phi0_(phi0), dphi0_(dphi0),
        thresh_(phi0 + p.hz_eps * fscale), p_(p) {}

  // runs from the trial step c; returns true when a step met the
  // conditions (a, f, df of that step), false when the budget ran out (the
  // evaluated step with the lowest phi)
  bool run(double c, double* a, double* f, double* df, int* evals) {
    double lo = 0.0, hi = 0.0;
    if (bracket(c, &lo, &hi)) {
      for (;;) {
        double A, B;
        if (!secant2(lo, hi, &A, &B)) break;
        if (B - A > p_.hz_gamma * (hi - lo))
          if (!update(A, B, 0.5 * (A + B), &A, &B)) break;
        if (A == lo && B == hi) {
          state_ = EXHAUSTED;  // no progress possible in floating point
          break;
        }
        lo = A;
        hi = B;
      }
    }
    *evals = (int)order_.size();
    if (state_ == FOUND) {
      *a = found_;
      *f = seen_[found_].first;
      *df = seen_[found_].second;
      return true;
    }
    if (order_.empty()) {
      *a = 0.0;
      *f = phi0_;
      *df = dphi0_;
      return false;
    }
    double best = order_[0];
    for (double t : order_)
      if (seen_[t].first < seen_[best].first) best = t;
    *a = best;
    *f = seen_[best].first;
    *df = seen_[best].second;
    return false;
  }

  double last() const { return order_.empty() ? 0.0 : order_.back(); }

 private:
  enum State { RUN, FOUND, EXHAUSTED };
  std::function<std::pair<double, double>(double)> phi_;
  double phi0_, dphi0_, thresh_;
  const Params& p_;
  std::map<double, std::pair<double, double>> seen_;
  std::vector<double> order_;
  State state_ = RUN;
  double found_ = 0.0;

  // phi(a); false when the search stops (a step met the conditions, or the
  // evaluation budget is spent)
  bool ev(double a, double* f, double* df) {
    auto it = seen_.find(a);
    if (it != seen_.end()) {
      *f = it->second.first;
      *df = it->second.second;
      return true;
    }
    if ((int)order_.size() >= p_.max_evals) {
      state_ = EXHAUSTED;
      return false;
    }
    const std::pair<double, double> v = phi_(a);
    seen_[a] = v;
    order_.push_back(a);
    *f = v.first;
    *df = v.second;
    const bool wolfe = p_.hz_delta * dphi0_ * a >= *f - phi0_ &&
                       *df >= p_.hz_sigma * dphi0_;
    const bool approx = (2.0 * p_.hz_delta - 1.0) * dphi0_ >= *df &&
                        *df >= p_.hz_sigma * dphi0_ && *f <= thresh_;
    if (wolfe || approx) {
      state_ = FOUND;
      found_ = a;
      return false;
    }
    return true;
  }

  double dphi_at(double a) {
    auto it = seen_.find(a);
    return it != seen_.end() ? it->second.second : dphi0_;
  }

  // phi'(b) < 0 and phi(b) above the threshold: move into [a, b] by theta
  bool bisect_update(double a, double b, double* ra, double* rb) {
    for (;;) {
      const double d = (1.0 - p_.hz_theta) * a + p_.hz_theta * b;
      double f, df;
      if (!ev(d, &f, &df)) return false;
      if (df >= 0.0) {
        *ra = a;
        *rb = d;
        return true;
      }
      if (f <= thresh_)
        a = d;
      else
        b = d;
    }
  }

  bool update(double a, double b, double c, double* ra, double* rb) {
    if (!(a < c && c < b)) {
      *ra = a;
      *rb = b;
      return true;
    }
    double f, df;
    if (!ev(c, &f, &df)) return false;
    if (df >= 0.0) {
      *ra = a;
      *rb = c;
      return true;
    }
    if (f <= thresh_) {
      *ra = c;
      *rb = b;
      return true;
    }
    return bisect_update(a, c, ra, rb);
  }

  double secant(double a, double b) {
    const double da = dphi_at(a), db = seen_[b].second;
    if (db == da) return 0.5 * (a + b);
    return (a * db - b * da) / (db - da);
  }

  bool secant2(double a, double b, double* ra, double* rb) {
    const double c = secant(a, b);
    double A, B;
    if (!update(a, b, c, &A, &B)) return false;
    if (c == B) return update(A, B, secant(b, B), ra, rb);
    if (c == A) return update(A, B, secant(a, A), ra, rb);
    *ra = A;
    *rb = B;
    return true;
  }

  // expand from c until phi' >= 0 or phi exceeds the threshold
  bool bracket(double c, double* ra, double* rb) {
    std::vector<std::pair<double, double>> cs;
    for (;;) {
      double f, df;
      if (!ev(c, &f, &df)) return false;
      if (df >= 0.0) {
        double a = 0.0;
        for (const auto& t : cs)
          if (t.second <= thresh_) a = t.first;
        *ra = a;
        *rb = c;
        return true;
      }
      cs.emplace_back(c, f);
      if (f > thresh_) return bisect_update(0.0, c, ra, rb);
      c = p_.hz_rho * c;
    }
  }
};

}  // namespace

struct Lbfgs {
  Context* cx = nullptr;
  std::vector<TermSpec> terms;
  Params p{};
  int64_t n = 0;
  Tensor x, g, d, q, r, xt, gt, sc;
  Tensor S, Y;              // [m][n] ring buffers of the pairs
  std::vector<double> rho;  // 1 / (y_i^T s_i) per slot
  int count = 0, head = 0;  // pairs stored; slot of the oldest
  double f = 0.0, delta = 0.0;
  int iter = 0;
  int warn = 0;             // an evaluation or solve returned a warning

  double dotd(const double* a, const double* b) {
    Device& dev = cx->dev;
    dot(dev, a, b, n, sc.ptr);
    double h = 0.0;
    dev.download(sc, &h);
    return h;
  }

  // evaluates at the point pt: context state, environment, energy and
  // gradient (into grad); returns E
  double evaluate(const double* pt, double* grad, int* ctm_iters) {
    Context& c = *cx;
    axpby(c.dev, n, 1.0, pt, 0.0, c.A.ptr);
    build_double_layer(c);
    int it = 0;
    double dl = 0.0;
    warn |= converge_env(c, p.ctm_tol, p.ctm_max_iter, &it, &dl);
    if (ctm_iters) *ctm_iters += it;
    const long svd0 = c.stats.svd_unconverged, cg0 = c.stats.cg_unconverged;
    double e;
    {
      PrecScope ps(c.dev, late_prec(c));
      e = energy_grad(c, terms, grad, true);
    }
    if (c.stats.svd_unconverged != svd0 || c.stats.cg_unconverged != cg0)
      warn = 1;
    return e;
  }

  int slot(int i) const { return (head + i) % p.m; }  // i-th oldest
  double* Sp(int i) { return S.ptr + (int64_t)slot(i) * n; }
  double* Yp(int i) { return Y.ptr + (int64_t)slot(i) * n; }

  // r = H_0 q
  void apply_h0(const double* qv, double* rv) {
    Context& c = *cx;
    if (p.precondition == 2) {
      // belief-propagation metric at the current point, from the trace
      // message (belief propagation can have several fixed points: a start
      // that does not depend on the path keeps the direction a function of
      // the point alone)
      int it = 0;
      double ch = 0.0;
      c.bp_msg = Tensor();
      warn |= bp_converge(c, p.ctm_tol, p.ctm_max_iter, &it, &ch);
      (void)precondition_bp(c, qv, delta, rv, true);
    } else if (p.precondition == 3) {
      // local metric, one GMRES cycle
      PrecScope ps(c.dev, late_prec(c));
      int k = 0;
      double res = 0.0;
      precondition_gmres(c, qv, delta, p.gmres_m, p.cg_tol, rv, &k, &res,
                         true);
    } else if (p.precondition == 4) {
      // full metric, one GMRES cycle
      PrecScope ps(c.dev, late_prec(c));
      int k = 0;
      double res = 0.0;
      const double h =
          p.fd_step > 0.0 ? p.fd_step
                          : (late_prec(c) == PREC_FP64 ? 1e-5 : 3e-3);
      precondition_full(c, qv, delta, p.gmres_m, p.cg_tol, h, rv, &k, &res,
                        true);
    } else if (p.precondition) {
      PrecScope ps(c.dev, late_prec(c));
      int it = 0;
      double res = 0.0;
      (void)precondition(c, qv, delta, p.cg_tol, p.cg_maxiter, rv, &it, &res,
                         true);
    } else {
      double gam = 1.0;
      if (count > 0) {
        double* s = Sp(count - 1);
        double* y = Yp(count - 1);
        gam = dotd(s, y) / dotd(y, y);
      }
      axpby(c.dev, n, gam, qv, 0.0, rv);
    }
  }

  // d = -H g by the two-loop recursion
  void direction() {
    Device& dev = cx->dev;
    axpby(dev, n, 1.0, g.ptr, 0.0, q.ptr);
    std::vector<double> alpha(count);
    for (int i = count - 1; i >= 0; --i) {
      alpha[i] = rho[slot(i)] * dotd(Sp(i), q.ptr);
      axpby(dev, n, -alpha[i], Yp(i), 1.0, q.ptr);
    }
    apply_h0(q.ptr, r.ptr);
    for (int i = 0; i < count; ++i) {
      const double beta = rho[slot(i)] * dotd(Yp(i), r.ptr);
      axpby(dev, n, alpha[i] - beta, Sp(i), 1.0, r.ptr);
    }
    axpby(dev, n, -1.0, r.ptr, 0.0, d.ptr);
  }

  double amax_host(const Tensor& t) {
    std::vector<double> h(n);
    cx->dev.download(t, h.data());
    double m = 0.0;
    for (double v : h) m = std::max(m, std::fabs(v));
    return m;
  }

  // one iteration; info out.  Returns 0, or 1 when the line search ended
  // without meeting its conditions or a warning came up; 2 at a stationary
  // point (no descent direction; nothing changed)
  int step(ipeps_lbfgs_info* info) {
    Device& dev = cx->dev;
    warn = 0;
    int ctm_iters = 0;
    direction();
    double dphi0 = dotd(g.ptr, d.ptr);
    if (!(dphi0 < 0.0)) {
      // lost descent (inconsistent curvature pairs): restart from H_0
      count = head = 0;
      direction();
      dphi0 = dotd(g.ptr, d.ptr);
      if (!(dphi0 < 0.0)) return 2;
    }
    const double c0 =
        (iter == 0 && !p.precondition) ? p.psi0 * amax_host(x) / amax_host(g)
                                       : 1.0;
    double last_eval = -1.0;
    // IPEPS_LBFGS_TRACE=1 prints every line-search evaluation to stderr
    static const bool trace = [] {
      const char* t = std::getenv("IPEPS_LBFGS_TRACE");
      return t && t[0] == '1';
    }();
    if (trace)
      std::fprintf(stderr, "lbfgs it %d: c %.17g phi0 %.17g dphi0 %.17g\n",
                   iter + 1, c0, f, dphi0);
    auto phi = [&](double a) -> std::pair<double, double> {
      axpby(dev, n, 1.0, x.ptr, 0.0, xt.ptr);
      axpby(dev, n, a, d.ptr, 1.0, xt.ptr);
      const int it0 = ctm_iters;
      const long cg0 = cx->stats.cg_unconverged;
      double fa = evaluate(xt.ptr, gt.ptr, &ctm_iters);
      last_eval = a;
      double dfa = dotd(gt.ptr, d.ptr);
      // a point whose gradient could not be computed (a complement solve
      // of the SVD adjoint stopped at its limit, or non-finite values) is
      // treated as infinitely high: the line search moves back from it
      if (cx->stats.cg_unconverged != cg0 || !std::isfinite(fa) ||
          !std::isfinite(dfa)) {
        fa = INFINITY;
        dfa = INFINITY;
      }
      if (trace)
        std::fprintf(stderr, "  eval a %.17g f %.17g df %.9e ctm %d\n", a,
                     fa, dfa, ctm_iters - it0);
      return {fa, dfa};
    };
    HagerZhang hz(phi, f, dphi0, std::fabs(f), p);
    double a = 0.0, fa = 0.0, dfa = 0.0;
    int nev = 0;
    const bool ok = hz.run(c0, &a, &fa, &dfa, &nev);
    // no usable point at all: stay at x (evaluated again below, so that
    // the context holds x's environment)
    if (!std::isfinite(fa)) a = 0.0;
    if (!ok || last_eval != a) {
      // make the accepted point the evaluated one (context state, gt)
      axpby(dev, n, 1.0, x.ptr, 0.0, xt.ptr);
      axpby(dev, n, a, d.ptr, 1.0, xt.ptr);
      fa = evaluate(xt.ptr, gt.ptr, &ctm_iters);
      ++nev;
    }
    // pair s = a d, y = g_new - g (in q and r, free after direction());
    // kept in the next slot when the curvature condition holds
    double* s = q.ptr;
    double* y = r.ptr;
    axpby(dev, n, a, d.ptr, 0.0, s);
    axpby(dev, n, 1.0, gt.ptr, 0.0, y);
    axpby(dev, n, -1.0, g.ptr, 1.0, y);
    const double sy = dotd(s, y);
    const double ss = dotd(s, s), yy = dotd(y, y);
    if (sy > 1e-12 * std::sqrt(ss) * std::sqrt(yy)) {
      const int nslot = count < p.m ? slot(count) : head;
      axpby(dev, n, 1.0, s, 0.0, S.ptr + (int64_t)nslot * n);
      axpby(dev, n, 1.0, y, 0.0, Y.ptr + (int64_t)nslot * n);
      if ((int)rho.size() < p.m) rho.resize(p.m);
      rho[nslot] = 1.0 / sy;
      if (count < p.m)
        ++count;
      else
        head = (head + 1) % p.m;
    }
    const double ggn = dotd(gt.ptr, gt.ptr);
    if (p.delta_mode == 1)
      delta = std::fabs(fa - f);
    else if (p.delta_mode == 2)
      delta = ggn;
    else
      delta = p.delta0;
    delta = std::min(std::max(delta, p.delta_min), p.delta_max);
    axpby(dev, n, 1.0, xt.ptr, 0.0, x.ptr);
    axpby(dev, n, 1.0, gt.ptr, 0.0, g.ptr);
    f = fa;
    ++iter;
    if (info) {
      info->e = f;
      info->alpha = a;
      info->n_evals = nev;
      info->ls_ok = ok ? 1 : 0;
      info->gnorm = std::sqrt(ggn);
      info->delta = delta;
      info->ctm_iters = ctm_iters;
    }
    dev.sync();
    return (!ok || warn) ? 1 : 0;
  }
};

}  // namespace ipeps

struct ipeps_lbfgs {
  ipeps::Lbfgs opt;
};

using namespace ipeps;

extern "C" {

void ipeps_lbfgs_default_params(ipeps_lbfgs_params* p) {
  if (!p) return;
  p->m = 200;
  p->precondition = 1;
  p->delta_mode = 1;
  p->delta0 = 1e-2;
  p->delta_min = 1e-12;
  p->delta_max = 1.0;
  p->ctm_tol = 1e-10;
  p->ctm_max_iter = 200;
  p->cg_tol = 0.0;
  p->cg_maxiter = 20;
  p->max_evals = 20;
  p->psi0 = 0.01;
  p->hz_delta = 0.1;
  p->hz_sigma = 0.9;
  p->hz_eps = 1e-6;
  p->hz_theta = 0.5;
  p->hz_gamma = 0.66;
  p->hz_rho = 5.0;
  p->gmres_m = 30;
  p->fd_step = 0.0;
}

int ipeps_lbfgs_create(ipeps_ctx* c, int n_terms, const ipeps_term* H,
                       const ipeps_lbfgs_params* prm, ipeps_lbfgs** out,
                       double* e0) {
  if (!c || !out) return IPEPS_EINVAL;
  ipeps_lbfgs_params q;
  ipeps_lbfgs_default_params(&q);
  if (prm) q = *prm;
  if (q.m < 1 || q.precondition < 0 || q.precondition > 4 ||
      q.gmres_m < 1 || q.gmres_m > 256 || !(q.fd_step >= 0.0) ||
      !(q.fd_step < 1.0) ||
      q.delta_mode < 0 || q.delta_mode > 2 || !(q.delta0 > 0.0) ||
      !(q.delta_min > 0.0) || !(q.delta_max >= q.delta_min) ||
      q.ctm_max_iter < 1 || q.cg_maxiter < 0 || !(q.cg_tol >= 0.0) ||
      q.max_evals < 1 || !(q.psi0 > 0.0) || !(q.hz_delta > 0.0) ||
      !(q.hz_sigma >= q.hz_delta && q.hz_sigma < 1.0) ||
      !(q.hz_eps >= 0.0) || !(q.hz_theta > 0.0 && q.hz_theta < 1.0) ||
      !(q.hz_gamma > 0.0 && q.hz_gamma < 1.0) || !(q.hz_rho > 1.0) ||
      std::isnan(q.ctm_tol))
    return IPEPS_EINVAL;
  Context& cx = ipeps_context(c);
  if (q.precondition == 4 && cx.nsite() != 1) return IPEPS_ENOTIMPL;
  std::vector<TermSpec> terms;
  int st = parse_terms(cx, n_terms, H, terms);
  if (st != IPEPS_OK) return st;
  ipeps_lbfgs* o = new (std::nothrow) ipeps_lbfgs();
  if (!o) return IPEPS_ENOMEM;
  Lbfgs& L = o->opt;
  L.cx = &cx;
  L.terms = std::move(terms);
  L.p = Params{q.m, q.precondition, q.delta_mode, q.ctm_max_iter,
               q.cg_maxiter, q.max_evals, q.delta0, q.delta_min,
               q.delta_max, q.ctm_tol, q.cg_tol, q.psi0, q.hz_delta,
               q.hz_sigma, q.hz_eps, q.hz_theta, q.hz_gamma, q.hz_rho,
               q.gmres_m, q.fd_step};
  L.delta = q.delta0;
  int warn = 0;
  st = guarded_call([&]() {
    Device& dev = cx.dev;
    L.n = cx.A.numel();
    const int64_t n = L.n;
    L.x = dev.empty({n});
    L.g = dev.empty({n});
    L.d = dev.empty({n});
    L.q = dev.empty({n});
    L.r = dev.empty({n});
    L.xt = dev.empty({n});
    L.gt = dev.empty({n});
    L.sc = dev.empty({1});
    L.S = dev.empty({(int64_t)q.m, n});
    L.Y = dev.empty({(int64_t)q.m, n});
    axpby(dev, n, 1.0, cx.A.ptr, 0.0, L.x.ptr);
    L.f = L.evaluate(L.x.ptr, L.g.ptr, nullptr);
    warn = L.warn;
    dev.sync();
    return IPEPS_OK;
  });
  if (st != IPEPS_OK) {
    delete o;
    return st;
  }
  if (e0) *e0 = L.f;
  *out = o;
  return warn ? IPEPS_NOT_CONVERGED : IPEPS_OK;
}

int ipeps_lbfgs_step(ipeps_lbfgs* o, ipeps_lbfgs_info* info) {
  if (!o) return IPEPS_EINVAL;
  int r = 0;
  int st = guarded_call([&]() {
    r = o->opt.step(info);
    return IPEPS_OK;
  });
  if (st != IPEPS_OK) return st;
  if (r == 2) return IPEPS_STATIONARY;
  return r ? IPEPS_NOT_CONVERGED : IPEPS_OK;
}

void ipeps_lbfgs_free(ipeps_lbfgs* o) {
  if (!o) return;
  if (o->opt.cx) (void)hipStreamSynchronize(o->opt.cx->dev.stream);
  delete o;
}

}  // extern "C"
