// Energy gradient by the reverse pass through unrolled CTMRG iterations
// (Sec. III A, "backward mode AD"; Sec. IV A, the "(3+20)" configuration).
// A enters every double layer (ket and bra) of every iteration and of the
// energy network; the tape records all of them and the backward pass
// accumulates dE/dA.  Three functions of A are differentiated
// (ipeps_grad_mode):
//   K-step     e(A, F^K(A, env*)), env* the converged environment, fixed;
//   full       e(A, F^K(A, env0(A))), env0 the trace-boundary start, so the
//              start and every iteration are differentiated;
//   fixed pt.  the K-step form with K doubled until the cotangent reaching
//              env* is below adj_tol times the one leaving the last
//              iteration (the derivative at the fixed point).
// All intermediates of the K iterations are kept resident (no
// recomputation): at D=6, chi=72 that is about 3 GB per iteration, small
// next to the 288 GB of one MI355X.
#include <algorithm>
#include <cmath>

#include "ad.hpp"
#include "ipeps_impl.hpp"

namespace ipeps {

namespace {

// sqrt(sum over the tensors of the squared norm of their gradients)
double grad_norm(Tape& tp, Device& dev, const std::vector<Var>& vs) {
  Tensor s = dev.empty({(int64_t)vs.size() + 1});
  std::vector<double> h(vs.size() + 1, 0.0);
  int k = 0;
  for (const Var& v : vs)
    if (tp.has_grad(v)) nrm2(dev, v->g.ptr, v->g.numel(), s.ptr + k++);
  if (k == 0) return 0.0;
  dev.download(s, h.data());
  double t = 0.0;
  for (int i = 0; i < k; ++i) t += h[i] * h[i];
  return std::sqrt(t);
}

std::vector<Var> all_of(const VEnv& e) {
  std::vector<Var> v = e.C;
  v.insert(v.end(), e.T.begin(), e.T.end());
  return v;
}

// one taped evaluation: value, gradient (into grad_host), and for the
// fixed-point test the cotangent norms into env* and out of the last
// iteration
double run(Context& cx, const std::vector<TermSpec>& terms, int K, bool full,
           bool env_req, double* grad_host, bool on_device, double* n_in,
           double* n_out) {
  Device& dev = cx.dev;
  Tape tp(dev, true);
  Var A = tp.leaf(cx.A, true);
  std::vector<Var> As(cx.nsite());
  for (int s = 0; s < cx.nsite(); ++s) As[s] = tp.slice0(A, s);
  std::vector<Var> arot = arot_from_sites(tp, cx, As);
  VEnv env0 = full ? init_env_ad(tp, cx, arot)
                   : venv_leaves(tp, cx, cx.env, env_req);
  VEnv env = env0;
  for (int k = 0; k < K; ++k) env = ctm_step_ad(tp, cx, env, arot);
  const double e = energy_ad(tp, cx, env, As, arot, terms);
  tp.backward();
  if (env_req) {
    *n_in = grad_norm(tp, dev, all_of(env0));
    *n_out = grad_norm(tp, dev, all_of(env));
  }
  const int64_t len = A->v.numel();
  if (on_device) {
    if (tp.has_grad(A))
      axpby(dev, len, 1.0, A->g.ptr, 0.0, grad_host);
    else
      fill(dev, grad_host, len, 0.0);
    dev.sync();
  } else if (tp.has_grad(A)) {
    dev.download(A->g, grad_host);
  } else {
    std::fill(grad_host, grad_host + len, 0.0);
  }
  return e;
}

}  // namespace

double energy_grad(Context& cx, const std::vector<TermSpec>& terms,
                   double* grad_host, bool on_device) {
  // the unrolled iterations must not move the projector-SVD warm start that
  // ctm_converge left behind: repeated calls on the same state then give
  // bitwise identical gradients
  const Tensor warm = cx.Xwarm;
  const bool have_warm = cx.have_warm;
  struct Restore {
    Context& c;
    Tensor w;
    bool h;
    ~Restore() {
      c.Xwarm = w;
      c.have_warm = h;
    }
  } restore{cx, warm, have_warm};
  const int K = cx.grad_K;
  double n_in = 0.0, n_out = 0.0;
  // the complement solves of one gradient start from each other's
  // solutions, never from an earlier gradient's
  cx.have_cg_warm = false;
  struct DropCg {
    Context& c;
    ~DropCg() {
      c.have_cg_warm = false;
      c.cg_warm = Tensor();
    }
  } drop_cg{cx};
  if (cx.grad_mode == 0) {
    // the full function starts, like a cold ctm_converge, without a warm
    // start for the first projector SVD
    cx.have_warm = false;
    cx.grad_K_used = K;
    return run(cx, terms, K, true, false, grad_host, on_device, &n_in,
               &n_out);
  }
  if (cx.grad_mode == 1) {
    cx.grad_K_used = K;
    return run(cx, terms, K, false, false, grad_host, on_device, &n_in,
               &n_out);
  }
  for (int k = K;; k *= 2) {
    cx.Xwarm = warm;
    cx.have_warm = have_warm;
    cx.have_cg_warm = false;
    const double e = run(cx, terms, k, false, true, grad_host, on_device,
                         &n_in, &n_out);
    cx.grad_K_used = k;
    if (n_in <= cx.adj_tol * std::max(n_out, 1e-300) || k >= 32 * K)
      return e;
  }
}

}  // namespace ipeps
