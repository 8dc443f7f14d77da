// Full tangent-space metric (Eq. (10), Sec. III A) applied matrix-free, and
// its regularised solve by GMRES (Sec. III C), for a 1x1 unit cell.
//
// The metric is the mixed ket/bra second derivative of the per-site
// log-norm F(A_ket, A_bra) = log kappa: the environment of the mixed double
// layer a = sum_p A_ket (x) A_bra is taken K = grad_K CTMRG iterations from
// the converged environment of A (as the K-step gradient), and kappa =
// n_site n_corner / (n_h n_v) with the four closed networks of the cell:
//   n_site    the ring of the eight environment tensors around a,
//   n_corner  Tr(C1 C2 C3 C4),
//   n_h       C1 T1 C2 over C4 T3 C3 (the ring with one column removed),
//   n_v       C1 C2 beside C4 C3 with T4, T2 (one row removed).
// The log subtracts the part of the overlap along the state itself, so the
// second derivative is the connected sum over the vacancy separations of
// Eq. (10), to the range the K iterations reach.  The bra derivative is one
// reverse pass over the taped iterations (the same tape as the energy
// gradient, with the ket and the bra as separate leaves, only the bra
// differentiated); the ket derivative along B is the central difference
//   N B = (dF/dA_bra(A + h B, A) - dF/dA_bra(A - h B, A)) / (2 h),
//   h = rel_step |A| / |B|,
// so one application costs two gradient evaluations.  Both evaluations
// start the projector SVDs from the same warm start, so the difference
// sees only the perturbation.
#include <cmath>
#include <vector>

#include "ad.hpp"
#include "ipeps_impl.hpp"

namespace ipeps {

namespace {

// sum of all entries of x * y as a [1] tensor (a batch of one product)
Var dot_all(Tape& tp, const Var& x, const Var& y) {
  const int64_t n = x->v.numel();
  return tp.einsum("xq,xq->x", tp.view(x, {1, n}), tp.view(y, {1, n}));
}

struct Nets {
  Var site, corner, h, v;
};

Nets kappa_networks(Tape& tp, const VEnv& e, const Var& a) {
  const Var &C1 = e.C[0], &C2 = e.C[1], &C3 = e.C[2], &C4 = e.C[3];
  const Var &T1 = e.T[0], &T2 = e.T[1], &T3 = e.T[2], &T4 = e.T[3];
  Nets n;
  // top row C1 T1 C2 [i, e, m] and bottom row C3 T3 C4 [n, z, w]
  Var top = tp.einsum("iek,km->iem", tp.einsum("ij,jek->iek", C1, T1), C2);
  Var bot = tp.einsum("nzq,qw->nzw", tp.einsum("np,pzq->nzq", C3, T3), C4);
  // ring E[l, u, r, d] = (T4 top)[w, l, u, m] (T2 bot)[m, r, d, w]
  Var lt = tp.einsum("wgi,iem->wgem", T4, top);
  Var rb = tp.einsum("mbn,nzw->mbzw", T2, bot);
  Var ring = tp.einsum("wgem,mbzw->gebz", lt, rb);
  n.site = dot_all(tp, ring, a);
  // corners only
  Var c12 = tp.einsum("ij,jk->ik", C1, C2);
  Var c34 = tp.einsum("kl,li->ik", C3, C4);
  n.corner = dot_all(tp, c12, c34);
  // top row closed on the bottom row: (top C3)[i, e, n] . (T3 C4)[i, e, n]
  Var tc = tp.einsum("iem,mn->ien", top, C3);
  Var t3c4 = tp.einsum("neq,qi->ien", T3, C4);
  n.h = dot_all(tp, tc, t3c4);
  // left column closed on the right column:
  // (C1 C2 T2 C3)[i, e, m] . (C4 T4)[i, e, m]
  Var col = tp.einsum("iel,lm->iem", tp.einsum("ik,kel->iel", c12, T2), C3);
  Var c4t4 = tp.einsum("mn,nei->iem", C4, T4);
  n.v = dot_all(tp, col, c4t4);
  return n;
}

}  // namespace

double log_kappa_grad(Context& cx, const double* Ak, double* gbra) {
  if (cx.nsite() != 1)
    throw NotImplError("full metric: 1x1 unit cell only");
  Device& dev = cx.dev;
  const int D = cx.D, D2 = cx.D2;
  // the iterations must not move the projector-SVD warm start that
  // ctm_converge left behind (every evaluation starts from the same one),
  // and the complement solves start cold in every evaluation
  struct Restore {
    Context& c;
    Tensor w;
    bool h;
    ~Restore() {
      c.Xwarm = w;
      c.have_warm = h;
      c.have_cg_warm = false;
      c.cg_warm = Tensor();
      c.defl_phi = Tensor();
    }
  } restore{cx, cx.Xwarm, cx.have_warm};
  cx.have_cg_warm = false;

  Tape tp(dev, gbra != nullptr);
  Tensor tk = cx.A.view({cx.d, D, D, D, D});
  tk.ptr = const_cast<double*>(Ak);
  Var ket = tp.leaf(tk, false);
  Var bra = tp.leaf(cx.A.view({cx.d, D, D, D, D}), true);
  std::vector<Var> arot = arot_from_pairs(tp, cx, {ket}, {bra});
  VEnv env = venv_leaves(tp, cx, cx.env, false);
  const std::vector<Var> arotf = arot_fb(tp, arot);
  for (int k = 0; k < cx.grad_K; ++k)
    env = ctm_step_ad(tp, cx, env, arot, &arotf);
  Nets n = kappa_networks(tp, env, tp.view(arot[0], {D2, D2, D2, D2}));
  // the four values in one download
  Tensor vals = dev.empty({4});
  const Var* nv[4] = {&n.site, &n.corner, &n.h, &n.v};
  for (int i = 0; i < 4; ++i)
    axpby(dev, 1, 1.0, (*nv[i])->v.ptr, 0.0, vals.ptr + i);
  double hv[4];
  dev.download(vals, hv);
  for (double v : hv)
    if (!(std::fabs(v) > 0.0) || !std::isfinite(v))
      throw ArgError("full metric: a norm network vanished or overflowed");
  const double F = std::log(std::fabs(hv[0])) + std::log(std::fabs(hv[1])) -
                   std::log(std::fabs(hv[2])) - std::log(std::fabs(hv[3]));
  if (!gbra) return F;
  // d log|n| / dn = 1 / n, with the signs of kappa's factors
  const double seed[4] = {1.0 / hv[0], 1.0 / hv[1], -1.0 / hv[2],
                          -1.0 / hv[3]};
  for (int i = 0; i < 4; ++i)
    if ((*nv[i])->req) dev.upload(tp.grad(*nv[i]), &seed[i]);
  tp.backward();
  const int64_t len = cx.A.numel();
  if (tp.has_grad(bra))
    axpby(dev, len, 1.0, bra->g.ptr, 0.0, gbra);
  else
    fill(dev, gbra, len, 0.0);
  return F;
}

void full_metric_apply(Context& cx, const double* B, double* NB,
                       double rel_step) {
  Device& dev = cx.dev;
  const int64_t len = cx.A.numel();
  Tensor s = dev.empty({2});
  {
    PrecScope ps(dev, PREC_FP64);
    nrm2(dev, cx.A.ptr, len, s.ptr);
    nrm2(dev, B, len, s.ptr + 1);
  }
  double nrm[2];
  dev.download(s, nrm);
  if (!(nrm[1] > 0.0)) {
    fill(dev, NB, len, 0.0);
    return;
  }
  const double h = rel_step * nrm[0] / nrm[1];
  Tensor Ak = dev.empty(cx.A.shape), gm = dev.empty(cx.A.shape);
  axpby(dev, len, 1.0, cx.A.ptr, 0.0, Ak.ptr);
  axpby(dev, len, h, B, 1.0, Ak.ptr);
  log_kappa_grad(cx, Ak.ptr, NB);
  axpby(dev, len, 1.0, cx.A.ptr, 0.0, Ak.ptr);
  axpby(dev, len, -h, B, 1.0, Ak.ptr);
  log_kappa_grad(cx, Ak.ptr, gm.ptr);
  axpby(dev, len, -0.5 / h, gm.ptr, 0.5 / h, NB);
}

void precondition_full(Context& cx, const double* g, double delta, int m,
                       double tol, double rel_step, double* x, int* n_used,
                       double* rel_resid, bool on_device) {
  Device& dev = cx.dev;
  const int64_t len = cx.A.numel();
  Tensor gd = dev.empty({len}), xd = dev.empty({len});
  if (on_device)
    axpby(dev, len, 1.0, g, 0.0, gd.ptr);
  else
    dev.upload(gd, g);
  auto op = [&](const double* v, double* y) {
    full_metric_apply(cx, v, y, rel_step);
    axpby(dev, len, delta, v, 1.0, y);
  };
  double res = 0.0;
  const int k = gmres(dev, len, gd.ptr, xd.ptr, m, tol, op, &res);
  if (on_device) {
    axpby(dev, len, 1.0, xd.ptr, 0.0, x);
    dev.sync();
  } else {
    dev.download(xd, x);
  }
  if (n_used) *n_used = k;
  if (rel_resid) *rel_resid = res;
}

}  // namespace ipeps
