// C4v-symmetric real ansatz and QR-based CTMRG (Sec. IV A: a one-site
// C4v-symmetric real iPEPS whose environment a QR-CTMRG provides, the
// symmetry fixing the gauge), and its K-step gradient.
//
// Ansatz: the site tensor is projected on the symmetric subspace, A_s = the
// average of A over the eight elements of the square's symmetry group on
// the virtual legs; the energy is a function of A through A_s and its
// gradient is the projection of the gradient at A_s.
//
// Environment: one corner C [chi][chi] (symmetric) and one edge T
// [chi][D^2][chi] (symmetric in its chi legs) stand for all four corners
// and edges.  One iteration on the enlarged corner M = T C T a
// ((chi D^2) x (chi D^2), symmetric):
//   growth     while the bond c satisfies c D^2 <= chi, no truncation: the
//              first chi unit vectors as Q (the zero padding beyond c D^2
//              carries zeros);
//   truncation one step of block subspace iteration on b = chi + p columns
//              (p = max(8, ceil(chi/4)), b even, <= 512): Y = M V with the
//              previous block V (the first b unit vectors at the first
//              truncation), Q0 = qr(Y) (Cholesky QR, two passes), the
//              Rayleigh-Ritz eigenvectors W of B = Q0^T M Q0 (Jacobi; the
//              chi of largest |lambda| first, each group in descending
//              signed order), V' = Q0 W with every column's entry of largest
//              |v_r| (1 + r/(2n)) made positive, Q = its first chi columns;
//   update     C' = Q^T M Q, T' = Q^T (T a) Q, each symmetrised on its chi
//              legs and normalised; V' is the next warm start.
// No SVD of the (chi D^2)-dimensional corner: one enlarged corner instead
// of four, one QR of an n x b block and one b x b eigendecomposition per
// iteration.  The iteration is written once on the differentiation tape,
// as the general CTMRG step is; the K-step gradient unrolls it from the
// converged (C, T, V).
#include <cmath>
#include <vector>

#include "ad.hpp"
#include "ipeps_impl.hpp"

namespace ipeps {

// ------------------------------------------------------------ tape ops
Var Tape::qr_q(const Var& Y) {
  PrecScope ps(dev, PREC_FP64);
  const int64_t n = Y->v.shape[0];
  const int b = (int)Y->v.shape[1];
  if (Y->v.rank() != 2 || b < 1 || b > MAX_BLOCK || n < b)
    throw ArgError("qr_q: needs an n x b matrix, b <= 512, n >= b");
  auto out = std::make_shared<Node>();
  Tensor nr = dev.empty({1});
  nrm2(dev, Y->v.ptr, n * b, nr.ptr);
  double ny = 0.0;
  dev.download(nr, &ny);
  Tensor Rinv = dev.zeros({b, b});
  out->v = dev.zeros({n, b});
  if (ny > 0.0 && std::isfinite(ny)) {
    // scaled so that the mean squared column norm is 1: the pivot
    // threshold of the Cholesky factor (1e-12 on G_kk) then drops columns
    // below 1e-6 of |Y|_F / sqrt(b)
    const double alpha = std::sqrt((double)b) / ny;
    Tensor Ys = dev.empty({n, b}), G = dev.empty({b, b});
    Tensor W1 = dev.empty({b, b}), W2 = dev.empty({b, b});
    Tensor Q1 = dev.empty({n, b});
    axpby(dev, n * b, alpha, Y->v.ptr, 0.0, Ys.ptr);
    gemm(dev, true, false, b, b, n, 1.0, Ys.ptr, b, 0, Ys.ptr, b, 0, 0.0,
         G.ptr, b, 0);
    chol_orth_factor(dev, G.ptr, W1.ptr, b, 1);
    gemm(dev, false, false, n, b, b, 1.0, Ys.ptr, b, 0, W1.ptr, b, 0, 0.0,
         Q1.ptr, b, 0);
    gemm(dev, true, false, b, b, n, 1.0, Q1.ptr, b, 0, Q1.ptr, b, 0, 0.0,
         G.ptr, b, 0);
    chol_orth_factor(dev, G.ptr, W2.ptr, b, 1);
    gemm(dev, false, false, n, b, b, 1.0, Q1.ptr, b, 0, W2.ptr, b, 0, 0.0,
         out->v.ptr, b, 0);
    // Q = Y R^-1 with R^-1 = alpha W1 W2
    gemm(dev, false, false, b, b, b, alpha, W1.ptr, b, 0, W2.ptr, b, 0, 0.0,
         Rinv.ptr, b, 0);
  }
  out->req = rec && Y->req;
  if (out->req)
    push([this, Y, out, Rinv, n, b]() {
      if (!has_grad(out)) return;
      PrecScope ps2(dev, PREC_FP64);
      // Ybar = (Qbar + Q copyltu(-Qbar^T Q)) R^-T
      const double* Q = out->v.ptr;
      const double* Qb = out->g.ptr;
      Tensor M = dev.empty({b, b}), L = dev.empty({b, b});
      gemm(dev, true, false, b, b, n, -1.0, Qb, b, 0, Q, b, 0, 0.0, M.ptr, b,
           0);
      copyltu(dev, M.ptr, L.ptr, b);
      Tensor X = dev.empty({n, b});
      axpby(dev, n * b, 1.0, Qb, 0.0, X.ptr);
      gemm(dev, false, false, n, b, b, 1.0, Q, b, 0, L.ptr, b, 0, 1.0, X.ptr,
           b, 0);
      gemm(dev, false, true, n, b, b, 1.0, X.ptr, b, 0, Rinv.ptr, b, 0, 1.0,
           grad(Y).ptr, b, 0);
    });
  return out;
}

Var Tape::eig_kept(const Var& B, int k) {
  PrecScope ps(dev, PREC_FP64);
  const int b = (int)B->v.shape[0];
  if (B->v.rank() != 2 || B->v.shape[1] != b || b % 2 || b > MAX_BLOCK)
    throw ArgError("eig_kept: needs a b x b matrix, b even, b <= 512");
  Tensor G = dev.empty({b, b}), V = dev.empty({b, b}), lam = dev.empty({b});
  axpby(dev, (int64_t)b * b, 1.0, B->v.ptr, 0.0, G.ptr);
  sym_eig_jacobi(dev, G.ptr, V.ptr, lam.ptr, b, 1);
  auto out = std::make_shared<Node>();
  out->v = dev.empty({b, b});
  Tensor lk = dev.empty({b});
  eig_order_kept(dev, lam.ptr, V.ptr, lk.ptr, out->v.ptr, b, k);
  out->req = rec && B->req;
  if (out->req)
    push([this, B, out, lk, b]() {
      if (!has_grad(out)) return;
      PrecScope ps2(dev, PREC_FP64);
      // Bbar = sym(W (F o (W^T Wbar)) W^T)
      const double* W = out->v.ptr;
      Tensor X = dev.empty({b, b}), Y = dev.empty({b, b});
      gemm(dev, true, false, b, b, b, 1.0, W, b, 0, out->g.ptr, b, 0, 0.0,
           X.ptr, b, 0);
      eig_fmul(dev, lk.ptr, X.ptr, Y.ptr, b, 1e-12);
      gemm(dev, false, false, b, b, b, 1.0, W, b, 0, Y.ptr, b, 0, 0.0, X.ptr,
           b, 0);
      gemm(dev, false, true, b, b, b, 1.0, X.ptr, b, 0, W, b, 0, 0.0, Y.ptr,
           b, 0);
      Tensor& gB = grad(B);
      axpby(dev, (int64_t)b * b, 0.5, Y.ptr, 1.0, gB.ptr);
      ipeps::permute(dev, Y.view({b, b}), {1, 0}, gB, 0.5, 1.0);
    });
  return out;
}

Var Tape::colscale(const Var& X, const Tensor& s) {
  const int64_t n = X->v.shape[0];
  const int b = (int)X->v.shape[1];
  auto out = std::make_shared<Node>();
  out->v = dev.empty(X->v.shape);
  axpby(dev, n * b, 1.0, X->v.ptr, 0.0, out->v.ptr);
  col_scale(dev, out->v.ptr, n, b, s.ptr, 2);
  out->req = rec && X->req;
  if (out->req)
    push([this, X, out, s, n, b]() {
      if (!has_grad(out)) return;
      Tensor t = dev.empty({n, b});
      axpby(dev, n * b, 1.0, out->g.ptr, 0.0, t.ptr);
      col_scale(dev, t.ptr, n, b, s.ptr, 2);
      axpby(dev, n * b, 1.0, t.ptr, 1.0, grad(X).ptr);
    });
  return out;
}

Var Tape::sym_pair(const Var& x, const std::vector<int>& perm) {
  for (size_t i = 0; i < perm.size(); ++i)
    if (perm[perm[i]] != (int)i)
      throw ArgError("sym_pair: the permutation must be its own inverse");
  auto out = std::make_shared<Node>();
  out->v = dev.empty(x->v.shape);
  const int64_t len = x->v.numel();
  ipeps::permute(dev, x->v, perm, out->v, 0.5, 0.0);
  axpby(dev, len, 0.5, x->v.ptr, 1.0, out->v.ptr);
  out->req = rec && x->req;
  if (out->req)
    push([this, x, out, perm, len]() {
      if (!has_grad(out)) return;
      Tensor& gx = grad(x);
      axpby(dev, len, 0.5, out->g.ptr, 1.0, gx.ptr);
      ipeps::permute(dev, out->g, perm, gx, 0.5, 1.0);
    });
  return out;
}

// ------------------------------------------------------------ the step
namespace {
void replicate_env(Context& cx);
}  // namespace

int c4v_block(int chi) {
  int b = chi + std::max(8, (chi + 3) / 4);
  b += b % 2;
  return b;
}

void c4v_set_env(Context& cx, const double* C, const double* T,
                 const double* V, bool on_device) {
  const int chi = cx.chi, D2 = cx.D2;
  cx.c4v_b = c4v_block(chi);
  c4v_project_state(cx);
  cx.c4v_C = cx.dev.empty({chi, chi});
  cx.c4v_T = cx.dev.empty({chi, D2, chi});
  cx.c4v_V = Tensor();
  if (V) cx.c4v_V = cx.dev.empty({(int64_t)chi * D2, cx.c4v_b});
  auto put = [&](Tensor& t, const double* src) {
    if (on_device)
      axpby(cx.dev, t.numel(), 1.0, src, 0.0, t.ptr);
    else
      cx.dev.upload(t, src);
  };
  put(cx.c4v_C, C);
  put(cx.c4v_T, T);
  if (V) put(cx.c4v_V, V);
  cx.c4v_c = chi;
  replicate_env(cx);
  (void)corner_spectra_change(cx, cx.env);
  cx.converged_once = true;
  cx.have_warm = false;
}

namespace {

// the first k columns of the n x n identity, as an n x k matrix
Tensor selector(Device& dev, int64_t n, int k) {
  Tensor E = dev.empty({n, k});
  eye(dev, E.ptr, n, k, 1, 0);
  return E;
}

struct C4vVars {
  Var C, T, V;  // V null while the bond grows
};

C4vVars c4v_step_ad(Tape& tp, Context& cx, const C4vVars& in, const Var& a,
                    bool grow) {
  Device& dev = tp.dev;
  const int chi = cx.chi, D2 = cx.D2, b = cx.c4v_b;
  const int64_t n = (int64_t)chi * D2;
  Var X1 = tp.einsum("mgi,ij->mgj", in.T, in.C);
  Var X2 = tp.einsum("mgj,jek->mgek", X1, in.T);
  Var M = tp.view(tp.einsum("mgek,gebf->mfkb", X2, a), {n, n});
  C4vVars out;
  Var Q;
  if (grow) {
    Q = tp.leaf(selector(dev, n, chi), false);
  } else {
    Var V = in.V ? in.V : tp.leaf(selector(dev, n, b), false);
    Var Q0 = tp.qr_q(tp.einsum("pq,qk->pk", M, V));
    Var B = tp.einsum("pk,pl->kl", Q0, tp.einsum("pq,qk->pk", M, Q0));
    Var W = tp.eig_kept(tp.sym_pair(B, {1, 0}), chi);
    Var Vr = tp.einsum("pk,kl->pl", Q0, W);
    Tensor sg = dev.empty({b});
    col_sign(dev, Vr->v.ptr, n, b, sg.ptr);
    out.V = tp.colscale(Vr, sg);
    Q = tp.einsum("pl,lm->pm", out.V,
                  tp.leaf(selector(dev, b, chi), false));
  }
  Var Cr = tp.einsum("pk,pm->km", Q, tp.einsum("pq,qm->pm", M, Q));
  Var Q3 = tp.view(Q, {chi, D2, chi});
  Var Y1 = tp.einsum("jgx,jek->xgek", Q3, in.T);
  Var Y2 = tp.einsum("xgek,gebf->xkbf", Y1, a);
  Var Tr = tp.einsum("xkbf,kby->xfy", Y2, Q3);
  std::vector<Var> nrm = tp.normalize_n(
      {tp.sym_pair(Cr, {1, 0}), tp.sym_pair(Tr, {2, 1, 0})});
  out.C = nrm[0];
  out.T = nrm[1];
  return out;
}

// the four-corner environment with every corner C and every edge T
void replicate_env(Context& cx) {
  const int chi = cx.chi, D2 = cx.D2;
  const int64_t cs = (int64_t)chi * chi, ts = cs * D2;
  if (cx.env.C.numel() != 4 * cs) cx.env.C = cx.dev.empty({4, 1, chi, chi});
  if (cx.env.T.numel() != 4 * ts)
    cx.env.T = cx.dev.empty({4, 1, chi, D2, chi});
  for (int c = 0; c < 4; ++c) {
    axpby(cx.dev, cs, 1.0, cx.c4v_C.ptr, 0.0, cx.env.C.ptr + c * cs);
    axpby(cx.dev, ts, 1.0, cx.c4v_T.ptr, 0.0, cx.env.T.ptr + c * ts);
  }
  cx.have_env = true;
}

// trace boundary: bond D^2, zero padded to chi
void c4v_init(Context& cx) {
  Device& dev = cx.dev;
  const int chi = cx.chi, D2 = cx.D2;
  std::vector<double> h((size_t)D2, 0.0);
  for (int k = 0; k < cx.D; ++k) h[(size_t)k * cx.D + k] = 1.0;
  Tensor tv = dev.empty({D2});
  dev.upload(tv, h.data());
  Tensor a = cx.av(0, 0);
  Tensor t1 = einsum(dev, "gebf,g->ebf", a, tv);
  Tensor cc = einsum(dev, "ebf,e->fb", t1, tv);
  Tensor tt = einsum(dev, "gebf,e->gfb", a, tv);
  cx.c4v_C = dev.zeros({chi, chi});
  cx.c4v_T = dev.zeros({chi, D2, chi});
  pad3(dev, cc.ptr, cx.c4v_C.ptr, 1, D2, D2, chi, chi);
  pad3(dev, tt.ptr, cx.c4v_T.ptr, D2, D2, D2, D2, chi);
  Tensor s = dev.empty({2});
  nrm2(dev, cx.c4v_C.ptr, cx.c4v_C.numel(), s.ptr);
  nrm2(dev, cx.c4v_T.ptr, cx.c4v_T.numel(), s.ptr + 1);
  scale_dev(dev, cx.c4v_C.ptr, cx.c4v_C.numel(), s.ptr, true);
  scale_dev(dev, cx.c4v_T.ptr, cx.c4v_T.numel(), s.ptr + 1, true);
  cx.c4v_c = D2;
  cx.c4v_V = Tensor();
}

}  // namespace

void c4v_symmetrize(Device& dev, const double* in, double* out, int d,
                    int D) {
  // out = (1/8) sum over the rotations R^k and their mirrors of in, legs
  // [p, l, u, r, d]: the rotation maps [l, u, r, d] to [d, l, u, r]
  Tensor x;
  x.ptr = const_cast<double*>(in);
  x.shape = {d, D, D, D, D};
  Tensor y;
  y.ptr = out;
  y.shape = {d, D, D, D, D};
  std::vector<int> rot = {0, 1, 2, 3, 4};
  bool first = true;
  for (int k = 0; k < 4; ++k) {
    ipeps::permute(dev, x, rot, y, 0.125, first ? 0.0 : 1.0);
    first = false;
    // the mirror l <-> r of the rotated tensor
    std::vector<int> mir = {rot[0], rot[3], rot[2], rot[1], rot[4]};
    ipeps::permute(dev, x, mir, y, 0.125, 1.0);
    // next rotation: new[l, u, r, d] = cur[d, l, u, r]
    rot = {rot[0], rot[4], rot[1], rot[2], rot[3]};
  }
}

void c4v_project_state(Context& cx) {
  const int64_t len = cx.A.numel();
  Tensor t = cx.dev.empty({len});
  c4v_symmetrize(cx.dev, cx.A.ptr, t.ptr, cx.d, cx.D);
  axpby(cx.dev, len, 1.0, t.ptr, 0.0, cx.A.ptr);
  build_double_layer(cx);
  cx.c4v_sym = true;
}

int c4v_converge(Context& cx, double tol, int max_iter, int* n_iter,
                 double* delta) {
  Device& dev = cx.dev;
  cx.c4v_b = c4v_block(cx.chi);
  c4v_project_state(cx);
  if (cx.c4v_c == 0 || cx.c4v_C.numel() != (int64_t)cx.chi * cx.chi)
    c4v_init(cx);
  replicate_env(cx);
  (void)corner_spectra_change(cx, cx.env);  // reference spectra
  double dl = INFINITY;
  int it = 0;
  const double tol_eff =
      tol > 0.0 ? std::max(tol, prec_floors(cx.work_prec).spectra) : tol;
  while (it < max_iter) {
    PrecScope ps(dev, cx.work_prec);
    Tape tp(dev, false);
    C4vVars in{tp.leaf(cx.c4v_C, false), tp.leaf(cx.c4v_T, false),
               cx.c4v_V.ptr ? tp.leaf(cx.c4v_V, false) : Var()};
    const bool grow = (int64_t)cx.c4v_c * cx.D2 <= cx.chi;
    C4vVars out = c4v_step_ad(tp, cx, in, tp.leaf(cx.av(0, 0), false), grow);
    cx.c4v_C = out.C->v;
    cx.c4v_T = out.T->v;
    if (out.V) cx.c4v_V = out.V->v;
    cx.c4v_c = grow ? cx.c4v_c * cx.D2 : cx.chi;
    ++it;
    replicate_env(cx);
    dl = corner_spectra_change(cx, cx.env);
    if (tol_eff > 0.0 && dl < tol_eff) break;
  }
  cx.converged_once = true;
  cx.have_warm = false;  // the general iteration starts its SVDs cold
  if (n_iter) *n_iter = it;
  if (delta) *delta = dl;
  return (tol > 0.0 && !(dl < tol_eff)) ? 1 : 0;
}

double c4v_energy_grad(Context& cx, const std::vector<TermSpec>& terms,
                       double* grad, bool on_device) {
  Device& dev = cx.dev;
  const int64_t len = cx.A.numel();
  if (!cx.c4v_sym) c4v_project_state(cx);
  Tape tp(dev, grad != nullptr);
  Var A = tp.leaf(cx.A, true);
  std::vector<Var> As{tp.slice0(A, 0)};
  std::vector<Var> arot = arot_from_sites(tp, cx, As);
  C4vVars st{tp.leaf(cx.c4v_C, false), tp.leaf(cx.c4v_T, false),
             cx.c4v_V.ptr ? tp.leaf(cx.c4v_V, false) : Var()};
  int c = cx.c4v_c;
  for (int k = 0; k < cx.grad_K; ++k) {
    const bool grow = (int64_t)c * cx.D2 <= cx.chi;
    C4vVars nx = c4v_step_ad(tp, cx, st, arot[0], grow);
    if (!nx.V) nx.V = st.V;
    st = nx;
    c = grow ? c * cx.D2 : cx.chi;
  }
  VEnv ve;
  ve.C.assign(4, st.C);
  ve.T.assign(4, st.T);
  const double e = energy_ad(tp, cx, ve, As, arot, terms);
  if (!grad) return e;
  tp.backward();
  Tensor g = dev.empty({len});
  if (tp.has_grad(A))
    c4v_symmetrize(dev, A->g.ptr, g.ptr, cx.d, cx.D);
  else
    fill(dev, g.ptr, len, 0.0);
  if (on_device) {
    axpby(dev, len, 1.0, g.ptr, 0.0, grad);
    dev.sync();
  } else {
    dev.download(g, grad);
  }
  return e;
}

}  // namespace ipeps
