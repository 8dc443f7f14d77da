// Energy gradient: reverse pass through K unrolled CTMRG iterations from the
// converged environment env* (held fixed), the derivative of
// A -> e(A, F^K(A, env*)) (Sec. III A; the "(3+20)" configuration of
// Sec. IV A with K = 20).  A enters every double layer (ket and bra) of every
// iteration and of the energy network; the tape records all of them and the
// backward pass accumulates dE/dA.  All intermediates of the K iterations are
// kept resident (no recomputation): at D=6, chi=72 that is about 1 GB per
// iteration, small next to the 288 GB of one MI355X.
#include "ad.hpp"
#include "ipeps_impl.hpp"

namespace ipeps {

double energy_grad(Context& cx, const std::vector<TermSpec>& terms,
                   double* grad_host, bool on_device) {
  Device& dev = cx.dev;
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
  Tape tp(dev, true);
  Var A = tp.leaf(cx.A, true);
  std::vector<Var> As(cx.nsite());
  for (int s = 0; s < cx.nsite(); ++s) As[s] = tp.slice0(A, s);
  std::vector<Var> arot = arot_from_sites(tp, cx, As);
  VEnv env = venv_leaves(tp, cx, cx.env);
  for (int k = 0; k < cx.grad_K; ++k) env = ctm_step_ad(tp, cx, env, arot);
  const double e = energy_ad(tp, cx, env, As, arot, terms);
  tp.backward();
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

}  // namespace ipeps
