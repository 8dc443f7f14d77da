// Differentiable SVD-truncated projectors of the half-system cuts.
//
// Forward (per cut, M = Qa Qb, top singular triplets from projector_svd):
//   P = Qb V_k S_k^-1/2,   Pt^T = Qa^T U_k S_k^-1/2  (zero beyond k).
// Backward: with w = S^-1/2 and cotangents Pb, Tb of P and Pt^T,
//   Qb_bar += Pb w V^T,  Qa_bar += U (Tb w)^T,
//   V_bar = Qb^T Pb w,   U_bar = Qa Tb w,   s_bar = -1/2 s^-3/2 w_bar,
// then the truncated-SVD adjoint M_bar = U_k B^T + C V_k^T with
//   B = V_k G_kk^T + b,  G_kk the kept-block matrix (Lorentzian 1/x),
//   [c_j; b_j] solving [[s_j, -M], [-M^T, s_j]] [c_j; b_j] =
//   [P_D u_bar_j; P'_D v_bar_j] on the complement of the kept singular
//   vectors (P_D = 1 - U_k U_k^T, P'_D = 1 - V_k V_k^T), which is
//   symmetric positive definite there (eigenvalues s_j +- s_i, i discarded)
//   and solved by column-wise CG with M applied as Qa (Qb x).  This equals
//   the full-spectrum formula sum over discarded i of
//   1/(s_j^2 - s_i^2) terms without forming the discarded vectors.
// Finally Qa_bar += M_bar Qb^T, Qb_bar += Qa^T M_bar in low-rank form.
#include <algorithm>
#include <cmath>

#include "ad.hpp"
#include "ipeps_impl.hpp"

namespace ipeps {

void copy2d(Device& dev, const double* src, int64_t lds, double* dst,
            int64_t ldd, int64_t rows, int64_t cols);

namespace {

// y <- y - Q (Q^T y), Q and y n x m
void project_out(Device& dev, const double* Q, double* y, int64_t n, int m) {
  Tensor t = dev.empty({m, m});
  gemm(dev, true, false, m, m, n, 1.0, Q, m, 0, y, m, 0, 0.0, t.ptr, m, 0);
  gemm(dev, false, false, n, m, m, -1.0, Q, m, 0, t.ptr, m, 0, 1.0, y, m, 0);
}

struct CutData {
  const double *Qa, *Qb;
  const double *U, *V, *S;  // U, V: n x b (ld b); S: b
  const int* keep;
  const double* w;          // chi
  const double *QbV, *QaU;  // n x chi unscaled
};

// Solve the complement system for all kept columns; returns [2][n][chi].
Tensor complement_solve(Device& dev, const CutData& cd, int64_t n, int chi,
                        int b, const Tensor& Ukm, const Tensor& Vkm,
                        const Tensor& rhs, SvdStats* st) {
  const int64_t rows = 2 * n;
  Tensor X = dev.zeros({2, n, chi});
  Tensor R = dev.empty({2, n, chi});
  Tensor Pp = dev.empty({2, n, chi});
  Tensor AP = dev.empty({2, n, chi});
  Tensor t1 = dev.empty({n, chi});
  Tensor sc = dev.empty({4, chi});  // rr, pAp, rr_new, rr0
  Tensor Sk = dev.empty({chi});
  // singular values as a column scale (first chi of the b values)
  axpby(dev, chi, 1.0, cd.S, 0.0, Sk.ptr);
  axpby(dev, rows * chi, 1.0, rhs.ptr, 0.0, R.ptr);
  axpby(dev, rows * chi, 1.0, rhs.ptr, 0.0, Pp.ptr);
  coldot(dev, R.ptr, R.ptr, rows, chi, sc.ptr);
  axpby(dev, chi, 1.0, sc.ptr, 0.0, sc.ptr + 3 * chi);
  std::vector<double> h(4 * chi);
  const double tol2 = 1e-24;
  int it = 0;
  const int max_it = 600;
  for (; it < max_it; ++it) {
    double* pc = Pp.ptr;
    double* pb = Pp.ptr + n * chi;
    double* ac = AP.ptr;
    double* ab = AP.ptr + n * chi;
    // ac = s p_c - P_D M p_b
    gemm(dev, false, false, n, chi, n, 1.0, cd.Qb, n, 0, pb, chi, 0, 0.0,
         t1.ptr, chi, 0);
    gemm(dev, false, false, n, chi, n, 1.0, cd.Qa, n, 0, t1.ptr, chi, 0, 0.0,
         ac, chi, 0);
    project_out(dev, Ukm.ptr, ac, n, chi);
    col_axpby(dev, n, chi, 1.0, Sk.ptr, pc, -1.0, ac);
    // ab = s p_b - P'_D M^T p_c
    gemm(dev, true, false, n, chi, n, 1.0, cd.Qa, n, 0, pc, chi, 0, 0.0,
         t1.ptr, chi, 0);
    gemm(dev, true, false, n, chi, n, 1.0, cd.Qb, n, 0, t1.ptr, chi, 0, 0.0,
         ab, chi, 0);
    project_out(dev, Vkm.ptr, ab, n, chi);
    col_axpby(dev, n, chi, 1.0, Sk.ptr, pb, -1.0, ab);
    coldot(dev, Pp.ptr, AP.ptr, rows, chi, sc.ptr + chi);
    colcg(dev, 0, rows, chi, sc.ptr, sc.ptr + chi, X.ptr, R.ptr, Pp.ptr,
          AP.ptr);
    coldot(dev, R.ptr, R.ptr, rows, chi, sc.ptr + 2 * chi);
    colcg(dev, 1, rows, chi, sc.ptr, sc.ptr + 2 * chi, X.ptr, R.ptr, Pp.ptr,
          AP.ptr);
    axpby(dev, chi, 1.0, sc.ptr + 2 * chi, 0.0, sc.ptr);
    if ((it + 1) % 4 == 0) {
      dev.download(sc, h.data());
      bool done = true;
      for (int j = 0; j < chi; ++j)
        if (h[3 * chi + j] > 0.0 && h[j] > tol2 * h[3 * chi + j]) done = false;
      if (done) {
        ++it;
        break;
      }
    }
  }
  if (st) {
    st->cg_iters += it;
    st->cg_solves += 1;
  }
  return X;
}

}  // namespace

std::pair<std::vector<Var>, std::vector<Var>> projector_op(
    Tape& tp, Context& cx, const std::vector<Var>& Qa,
    const std::vector<Var>& Qb) {
  Device& dev = tp.dev;
  const int nc = (int)Qa.size(), chi = cx.chi, b = cx.b;
  const int64_t n = cx.n, sUV = n * b;
  CutBatch cb;
  cb.ncut = nc;
  cb.n = n;
  cb.b = b;
  cb.chi = chi;
  for (int i = 0; i < nc; ++i) {
    cb.Qa.push_back(Qa[i]->v.ptr);
    cb.Qb.push_back(Qb[i]->v.ptr);
  }
  Tensor U, S, V, keep;
  projector_svd(dev, cb, cx.Xwarm, cx.have_warm, U, S, V, keep, cx.svd,
                &cx.stats);
  cx.have_warm = true;
  Tensor w = dev.empty({nc, chi});
  Tensor QbV = dev.empty({nc, n, chi}), QaU = dev.empty({nc, n, chi});
  std::vector<Var> P(nc), PtT(nc);
  const int* kp = (const int*)keep.ptr;
  for (int i = 0; i < nc; ++i) {
    proj_weights(dev, S.ptr + i * b, kp + i, chi, w.ptr + i * chi);
    gemm(dev, false, false, n, chi, n, 1.0, cb.Qb[i], n, 0, V.ptr + i * sUV,
         b, 0, 0.0, QbV.ptr + i * n * chi, chi, 0);
    gemm(dev, true, false, n, chi, n, 1.0, cb.Qa[i], n, 0, U.ptr + i * sUV, b,
         0, 0.0, QaU.ptr + i * n * chi, chi, 0);
    Tensor Pi = dev.empty({n, chi}), Ti = dev.empty({n, chi});
    col_axpby(dev, n, chi, 1.0, w.ptr + i * chi, QbV.ptr + i * n * chi, 0.0,
              Pi.ptr);
    col_axpby(dev, n, chi, 1.0, w.ptr + i * chi, QaU.ptr + i * n * chi, 0.0,
              Ti.ptr);
    P[i] = tp.leaf(Pi, false);
    PtT[i] = tp.leaf(Ti, false);
    P[i]->req = PtT[i]->req = tp.rec && (Qa[i]->req || Qb[i]->req);
  }
  bool any = false;
  for (int i = 0; i < nc; ++i) any = any || P[i]->req;
  if (!any) return {P, PtT};
  SvdStats* st = &cx.stats;
  tp.push([&tp, Qa, Qb, P, PtT, U, S, V, keep, w, QbV, QaU, n, chi, b, nc,
           st]() {
    Device& dev = tp.dev;
    const int64_t sUV = n * b;
    const int* kp = (const int*)keep.ptr;
    for (int i = 0; i < nc; ++i) {
      const bool hp = tp.has_grad(P[i]), ht = tp.has_grad(PtT[i]);
      if (!hp && !ht) continue;
      CutData cd;
      cd.Qa = Qa[i]->v.ptr;
      cd.Qb = Qb[i]->v.ptr;
      cd.U = U.ptr + i * sUV;
      cd.V = V.ptr + i * sUV;
      cd.S = S.ptr + i * b;
      cd.keep = kp + i;
      cd.w = w.ptr + i * chi;
      cd.QbV = QbV.ptr + i * n * chi;
      cd.QaU = QaU.ptr + i * n * chi;
      Tensor Pb = hp ? P[i]->g : dev.zeros({n, chi});
      Tensor Tb = ht ? PtT[i]->g : dev.zeros({n, chi});
      Tensor Pbw = dev.empty({n, chi}), Tbw = dev.empty({n, chi});
      col_axpby(dev, n, chi, 1.0, cd.w, Pb.ptr, 0.0, Pbw.ptr);
      col_axpby(dev, n, chi, 1.0, cd.w, Tb.ptr, 0.0, Tbw.ptr);
      double* gQa = Qa[i]->req ? tp.grad(Qa[i]).ptr : nullptr;
      double* gQb = Qb[i]->req ? tp.grad(Qb[i]).ptr : nullptr;
      // direct terms of P = Qb V w and Pt^T = Qa^T U w
      if (gQb)
        gemm(dev, false, true, n, n, chi, 1.0, Pbw.ptr, chi, 0, cd.V, b, 0,
             1.0, gQb, n, 0);
      if (gQa)
        gemm(dev, false, true, n, n, chi, 1.0, cd.U, b, 0, Tbw.ptr, chi, 0,
             1.0, gQa, n, 0);
      // s_bar through w = s^-1/2
      Tensor wb = dev.empty({3, chi});
      coldot(dev, cd.QbV, Pb.ptr, n, chi, wb.ptr);
      coldot(dev, cd.QaU, Tb.ptr, n, chi, wb.ptr + chi);
      proj_sbar(dev, cd.S, cd.keep, chi, wb.ptr, wb.ptr + chi,
                wb.ptr + 2 * chi);
      // U_bar, V_bar (columns >= k vanish with w)
      Tensor Vb = dev.empty({n, chi}), Ub = dev.empty({n, chi});
      gemm(dev, true, false, n, chi, n, 1.0, cd.Qb, n, 0, Pbw.ptr, chi, 0,
           0.0, Vb.ptr, chi, 0);
      gemm(dev, false, false, n, chi, n, 1.0, cd.Qa, n, 0, Tbw.ptr, chi, 0,
           0.0, Ub.ptr, chi, 0);
      // kept block
      Tensor Au = dev.empty({chi, chi}), Av = dev.empty({chi, chi}),
             Gkk = dev.empty({chi, chi});
      gemm(dev, true, false, chi, chi, n, 1.0, cd.U, b, 0, Ub.ptr, chi, 0,
           0.0, Au.ptr, chi, 0);
      gemm(dev, true, false, chi, chi, n, 1.0, cd.V, b, 0, Vb.ptr, chi, 0,
           0.0, Av.ptr, chi, 0);
      svd_gkk(dev, Au.ptr, Av.ptr, cd.S, wb.ptr + 2 * chi, cd.keep, chi,
              Gkk.ptr);
      // complement right-hand side [P_D U_bar; P'_D V_bar]
      Tensor Ukm = dev.empty({n, chi}), Vkm = dev.empty({n, chi});
      copy2d(dev, cd.U, b, Ukm.ptr, chi, n, chi);
      copy2d(dev, cd.V, b, Vkm.ptr, chi, n, chi);
      mask_cols(dev, Ukm.ptr, n, chi, cd.keep);
      mask_cols(dev, Vkm.ptr, n, chi, cd.keep);
      Tensor rhs = dev.empty({2, n, chi});
      axpby(dev, n * chi, 1.0, Ub.ptr, 0.0, rhs.ptr);
      axpby(dev, n * chi, 1.0, Vb.ptr, 0.0, rhs.ptr + n * chi);
      project_out(dev, Ukm.ptr, rhs.ptr, n, chi);
      project_out(dev, Vkm.ptr, rhs.ptr + n * chi, n, chi);
      Tensor cbv = complement_solve(dev, cd, n, chi, b, Ukm, Vkm, rhs, st);
      // B = V Gkk^T + b_part, C = c_part
      Tensor Bm = dev.empty({n, chi});
      axpby(dev, n * chi, 1.0, cbv.ptr + n * chi, 0.0, Bm.ptr);
      gemm(dev, false, true, n, chi, chi, 1.0, cd.V, b, 0, Gkk.ptr, chi, 0,
           1.0, Bm.ptr, chi, 0);
      const double* Cm = cbv.ptr;
      Tensor t1 = dev.empty({n, chi});
      if (gQa) {
        // Qa_bar += U (Qb B)^T + C (Qb V)^T
        gemm(dev, false, false, n, chi, n, 1.0, cd.Qb, n, 0, Bm.ptr, chi, 0,
             0.0, t1.ptr, chi, 0);
        gemm(dev, false, true, n, n, chi, 1.0, cd.U, b, 0, t1.ptr, chi, 0,
             1.0, gQa, n, 0);
        gemm(dev, false, true, n, n, chi, 1.0, Cm, chi, 0, cd.QbV, chi, 0,
             1.0, gQa, n, 0);
      }
      if (gQb) {
        // Qb_bar += (Qa^T U) B^T + (Qa^T C) V^T
        gemm(dev, false, true, n, n, chi, 1.0, cd.QaU, chi, 0, Bm.ptr, chi,
             0, 1.0, gQb, n, 0);
        gemm(dev, true, false, n, chi, n, 1.0, cd.Qa, n, 0, Cm, chi, 0, 0.0,
             t1.ptr, chi, 0);
        gemm(dev, false, true, n, n, chi, 1.0, t1.ptr, chi, 0, cd.V, b, 0,
             1.0, gQb, n, 0);
      }
    }
  });
  return {P, PtT};
}

}  // namespace ipeps
