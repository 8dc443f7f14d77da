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
  const std::vector<Var> arotf = arot_fb(tp, arot);
  for (int k = 0; k < K; ++k) env = ctm_step_ad(tp, cx, env, arot, &arotf);
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

// Cotangents of a tape environment packed like an Env (zero where none
// arrived).
Env cot_pack(Tape& tp, Context& cx, const VEnv& v) {
  const int ns = cx.nsite(), chi = cx.chi, D2 = cx.D2;
  Env e;
  e.C = cx.dev.zeros({4, ns, chi, chi});
  e.T = cx.dev.zeros({4, ns, chi, D2, chi});
  const int64_t cs = (int64_t)chi * chi, ts = cs * D2;
  for (int i = 0; i < 4 * ns; ++i) {
    if (tp.has_grad(v.C[i]))
      axpby(cx.dev, cs, 1.0, v.C[i]->g.ptr, 0.0, e.C.ptr + i * cs);
    if (tp.has_grad(v.T[i]))
      axpby(cx.dev, ts, 1.0, v.T[i]->g.ptr, 0.0, e.T.ptr + i * ts);
  }
  return e;
}

// sqrt(|C|^2 + |T|^2) of a packed cotangent
double env_norm(Device& dev, const Env& e) {
  Tensor s = dev.empty({2});
  nrm2(dev, e.C.ptr, e.C.numel(), s.ptr);
  nrm2(dev, e.T.ptr, e.T.numel(), s.ptr + 1);
  double h[2];
  dev.download(s, h);
  return std::sqrt(h[0] * h[0] + h[1] * h[1]);
}

// The same evaluation with checkpointed recomputation: the K iterations run
// first without a tape, keeping only each iteration's input environment and
// projector-SVD warm start; the energy is differentiated on its own tape,
// then every iteration, last to first, is recomputed from its stored input
// on a tape of its own and differentiated with the cotangent of its output.
// One iteration's intermediates are resident at a time instead of K; the
// recomputation repeats the forward kernels on the same inputs, so the
// projectors and the values are the ones the forward pass produced.
double run_ckpt(Context& cx, const std::vector<TermSpec>& terms, int K,
                bool full, bool env_req, double* grad_host, bool on_device,
                double* n_in, double* n_out) {
  Device& dev = cx.dev;
  const int64_t len = cx.A.numel();
  Tensor gA = dev.zeros(cx.A.shape);
  // forward, values only
  Env e0;
  if (full) {
    Tape t(dev, false);
    e0 = env_pack(cx, init_env_ad(t, cx, arot_leaves(t, cx)));
  } else {
    e0 = cx.env;
  }
  std::vector<Env> in(K);
  std::vector<Tensor> warm(K);
  std::vector<char> have(K);
  Env e = e0;
  for (int k = 0; k < K; ++k) {
    in[k] = e;
    warm[k] = cx.Xwarm;
    have[k] = cx.have_warm;
    Env nxt;
    ctm_step(cx, e, nxt);
    e = nxt;
  }
  // energy at the last environment
  double energy = 0.0;
  Env cot;
  {
    Tape tp(dev, true);
    Var A = tp.leaf(cx.A, true);
    std::vector<Var> As(cx.nsite());
    for (int s = 0; s < cx.nsite(); ++s) As[s] = tp.slice0(A, s);
    std::vector<Var> arot = arot_from_sites(tp, cx, As);
    VEnv ve = venv_leaves(tp, cx, e, true);
    energy = energy_ad(tp, cx, ve, As, arot, terms);
    tp.backward();
    if (tp.has_grad(A)) axpby(dev, len, 1.0, A->g.ptr, 1.0, gA.ptr);
    cot = cot_pack(tp, cx, ve);
  }
  if (env_req) *n_out = env_norm(dev, cot);
  // iterations, last to first
  for (int k = K - 1; k >= 0; --k) {
    Tape tp(dev, true);
    Var A = tp.leaf(cx.A, true);
    std::vector<Var> As(cx.nsite());
    for (int s = 0; s < cx.nsite(); ++s) As[s] = tp.slice0(A, s);
    std::vector<Var> arot = arot_from_sites(tp, cx, As);
    const bool need_in = k > 0 || env_req || full;
    VEnv vin = venv_leaves(tp, cx, in[k], need_in);
    cx.Xwarm = warm[k];
    cx.have_warm = have[k];
    VEnv vout = ctm_step_ad(tp, cx, vin, arot);
    const int ns = cx.nsite();
    for (int c = 0; c < 4; ++c)
      for (int s = 0; s < ns; ++s) {
        vout.C[c * ns + s]->g = cx.Cv(cot, c, s);
        vout.T[c * ns + s]->g = cx.Tv(cot, c, s);
      }
    tp.backward();
    if (tp.has_grad(A)) axpby(dev, len, 1.0, A->g.ptr, 1.0, gA.ptr);
    if (need_in) cot = cot_pack(tp, cx, vin);
    in[k] = Env();
  }
  if (env_req) *n_in = env_norm(dev, cot);
  if (full) {
    // the trace-boundary start depends on A
    Tape tp(dev, true);
    Var A = tp.leaf(cx.A, true);
    std::vector<Var> As(cx.nsite());
    for (int s = 0; s < cx.nsite(); ++s) As[s] = tp.slice0(A, s);
    VEnv v0 = init_env_ad(tp, cx, arot_from_sites(tp, cx, As));
    const int ns = cx.nsite();
    for (int c = 0; c < 4; ++c)
      for (int s = 0; s < ns; ++s) {
        v0.C[c * ns + s]->g = cx.Cv(cot, c, s);
        v0.T[c * ns + s]->g = cx.Tv(cot, c, s);
      }
    tp.backward();
    if (tp.has_grad(A)) axpby(dev, len, 1.0, A->g.ptr, 1.0, gA.ptr);
  }
  if (on_device) {
    axpby(dev, len, 1.0, gA.ptr, 0.0, grad_host);
    dev.sync();
  } else {
    dev.download(gA, grad_host);
  }
  return energy;
}

double run_any(Context& cx, const std::vector<TermSpec>& terms, int K,
               bool full, bool env_req, double* grad_host, bool on_device,
               double* n_in, double* n_out) {
  return cx.grad_ckpt ? run_ckpt(cx, terms, K, full, env_req, grad_host,
                                 on_device, n_in, n_out)
                      : run(cx, terms, K, full, env_req, grad_host,
                            on_device, n_in, n_out);
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
      c.defl_phi = Tensor();
    }
  } drop_cg{cx};
  if (cx.grad_mode == 0) {
    // the full function starts, like a cold ctm_converge, without a warm
    // start for the first projector SVD
    cx.have_warm = false;
    cx.grad_K_used = K;
    return run_any(cx, terms, K, true, false, grad_host, on_device, &n_in,
               &n_out);
  }
  if (cx.grad_mode == 1) {
    cx.grad_K_used = K;
    return run_any(cx, terms, K, false, false, grad_host, on_device, &n_in,
               &n_out);
  }
  for (int k = K;; k *= 2) {
    cx.Xwarm = warm;
    cx.have_warm = have_warm;
    cx.have_cg_warm = false;
    const double e = run_any(cx, terms, k, false, true, grad_host, on_device,
                         &n_in, &n_out);
    cx.grad_K_used = k;
    if (n_in <= cx.adj_tol * std::max(n_out, 1e-300) || k >= 32 * K)
      return e;
  }
}

}  // namespace ipeps
