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
//   and solved by column-wise CG with M applied as Qa (Qb x), deflated by the
//   subspace triplets beyond chi that the forward SVD already holds.  This equals
//   the full-spectrum formula (sum over discarded i of 1/(s_j^2 - s_i^2)
//   terms) without forming the discarded vectors.
// Finally Qa_bar += M_bar Qb^T, Qb_bar += Qa^T M_bar in low-rank form.
//
// All cuts of one CTMRG iteration are processed together: every product of
// a cut matrix is one batched launch over the cuts (pointer arrays), every
// chi-wide block operation one strided batched launch.
#include <algorithm>
#include <cmath>
#include <map>
#include <utility>

#include "ad.hpp"
#include "ipeps_impl.hpp"

namespace ipeps {

namespace {

// y[i] <- y[i] - Q[i] (Q[i]^T y[i]); Q, y: batch x n x m, strides sQ, sY
void project_out(Device& dev, const double* Q, int64_t sQ, double* y,
                 int64_t sY, int64_t n, int m, int batch) {
  Tensor t = dev.empty({batch, m, m});
  gemm(dev, true, false, m, m, n, 1.0, Q, m, sQ, y, m, sY, 0.0, t.ptr, m,
       (int64_t)m * m, batch);
  gemm(dev, false, false, n, m, m, -1.0, Q, m, sQ, t.ptr, m, (int64_t)m * m,
       1.0, y, m, sY, batch);
}

// gemm_ptrs in a given arithmetic (the products with the cut matrices are
// contractions and follow the contraction precision)
template <class... Args>
void gemm_ptrs_p(Device& dev, int prec, Args&&... args) {
  PrecScope s(dev, prec);
  gemm_ptrs(dev, std::forward<Args>(args)...);
}

template <class T>
std::vector<T> offsets(T base, int64_t stride, int count) {
  std::vector<T> v(count);
  for (int i = 0; i < count; ++i) v[i] = base + i * stride;
  return v;
}

}  // namespace

std::pair<std::vector<Var>, std::vector<Var>> projector_op(
    Tape& tp, Context& cx, const std::vector<Var>& Qa,
    const std::vector<Var>& Qb) {
  Device& dev = tp.dev;
  const int nc = (int)Qa.size(), chi = cx.chi, b = cx.b;
  const int64_t n = cx.n, sUV = n * b, sP = n * chi;
  CutBatch cb;
  cb.ncut = nc;
  cb.n = n;
  cb.b = b;
  cb.chi = chi;
  for (int i = 0; i < nc; ++i) {
    cb.Qa.push_back(Qa[i]->v.ptr);
    cb.Qb.push_back(Qb[i]->v.ptr);
  }
  // FP32 copies of the distinct cut matrices, read by every product with
  // them (subspace iteration, projectors, backward) when the contraction
  // arithmetic is FP32 or BF16x3: half the bytes of these memory-bound
  // products
  std::vector<Tensor> q32;
  if (dev.cprec != PREC_FP64) {
    std::map<const double*, const float*> made;
    auto conv = [&](const double* q) {
      auto it = made.find(q);
      if (it != made.end()) return it->second;
      Tensor t = dev.empty({(n * n + 1) / 2});
      to_f32(dev, q, (float*)t.ptr, n * n);
      q32.push_back(t);
      return made[q] = (const float*)t.ptr;
    };
    for (int i = 0; i < nc; ++i) {
      cb.Qa32.push_back(conv(cb.Qa[i]));
      cb.Qb32.push_back(conv(cb.Qb[i]));
    }
  }
  Tensor U, S, V, keep;
  projector_svd(dev, cb, cx.Xwarm, cx.have_warm, U, S, V, keep, cx.svd,
                &cx.stats);
  cx.have_warm = true;
  const int* kp = (const int*)keep.ptr;
  Tensor w = dev.empty({nc, chi});
  proj_weights(dev, S.ptr, kp, chi, w.ptr, nc, b);
  Tensor QbV = dev.empty({nc, n, chi}), QaU = dev.empty({nc, n, chi});
  qmul(dev, dev.cprec, false, n, chi, n, cb.Qb, cb.Qb32, n,
       offsets<const double*>(V.ptr, sUV, nc), b,
       offsets<double*>(QbV.ptr, sP, nc), chi);
  qmul(dev, dev.cprec, true, n, chi, n, cb.Qa, cb.Qa32, n,
       offsets<const double*>(U.ptr, sUV, nc), b,
       offsets<double*>(QaU.ptr, sP, nc), chi);
  Tensor Pall = dev.empty({nc, n, chi}), Tall = dev.empty({nc, n, chi});
  col_axpby(dev, nc * n, chi, 1.0, w.ptr, QbV.ptr, 0.0, Pall.ptr, n, chi);
  col_axpby(dev, nc * n, chi, 1.0, w.ptr, QaU.ptr, 0.0, Tall.ptr, n, chi);
  std::vector<Var> P(nc), PtT(nc);
  bool any = false;
  for (int i = 0; i < nc; ++i) {
    P[i] = tp.leaf(Pall.slice0(i), false);
    PtT[i] = tp.leaf(Tall.slice0(i), false);
    P[i]->req = PtT[i]->req = tp.rec && (Qa[i]->req || Qb[i]->req);
    any = any || P[i]->req;
  }
  if (!any) return {P, PtT};
  SvdStats* st = &cx.stats;
  Context* cxp = &cx;
  const std::vector<const float*> qa32 = cb.Qa32, qb32 = cb.Qb32;
  tp.push([&tp, Qa, Qb, P, PtT, U, S, V, keep, w, QbV, QaU, n, chi, b, nc,
           st, cxp, q32, qa32, qb32]() {
    Device& dev = tp.dev;
    // the products with the cut matrices keep the contraction precision of
    // the calling scope; the SVD-adjoint algebra around them is FP64
    const int cp = dev.cprec;
    PrecScope f64(dev, PREC_FP64);
    const int64_t sUV = n * b, sP = n * chi, s2 = 2 * n * chi;
    const int64_t sG = (int64_t)chi * chi;
    const int* kp = (const int*)keep.ptr;
    bool anyg = false;
    for (int i = 0; i < nc; ++i)
      anyg = anyg || tp.has_grad(P[i]) || tp.has_grad(PtT[i]);
    if (!anyg) return;
    std::vector<const double*> qa(nc), qb(nc), ui(nc), vi(nc);
    std::vector<double*> gqa, gqb;
    std::vector<int> ia, ib;
    for (int i = 0; i < nc; ++i) {
      qa[i] = Qa[i]->v.ptr;
      qb[i] = Qb[i]->v.ptr;
      ui[i] = U.ptr + i * sUV;
      vi[i] = V.ptr + i * sUV;
      if (Qa[i]->req) {
        gqa.push_back(tp.grad(Qa[i]).ptr);
        ia.push_back(i);
      }
      if (Qb[i]->req) {
        gqb.push_back(tp.grad(Qb[i]).ptr);
        ib.push_back(i);
      }
    }
    auto pick = [](const std::vector<const double*>& v,
                   const std::vector<int>& idx) {
      std::vector<const double*> r;
      for (int i : idx) r.push_back(v[i]);
      return r;
    };
    // gather the cotangents (zeros where none arrived)
    Tensor Pb = dev.zeros({nc, n, chi}), Tb = dev.zeros({nc, n, chi});
    for (int i = 0; i < nc; ++i) {
      if (tp.has_grad(P[i]))
        axpby(dev, sP, 1.0, P[i]->g.ptr, 0.0, Pb.ptr + i * sP);
      if (tp.has_grad(PtT[i]))
        axpby(dev, sP, 1.0, PtT[i]->g.ptr, 0.0, Tb.ptr + i * sP);
    }
    Tensor Pbw = dev.empty({nc, n, chi}), Tbw = dev.empty({nc, n, chi});
    col_axpby(dev, nc * n, chi, 1.0, w.ptr, Pb.ptr, 0.0, Pbw.ptr, n, chi);
    col_axpby(dev, nc * n, chi, 1.0, w.ptr, Tb.ptr, 0.0, Tbw.ptr, n, chi);
    const auto pbw = offsets<const double*>(Pbw.ptr, sP, nc);
    const auto tbw = offsets<const double*>(Tbw.ptr, sP, nc);
    // (the direct terms of P = Qb V w and Pt^T = Qa^T U w join the
    // complement terms at the end)
    // s_bar through w = s^-1/2
    Tensor wb = dev.empty({3, nc, chi});
    coldot(dev, QbV.ptr, Pb.ptr, n, chi, wb.ptr, nc, sP);
    coldot(dev, QaU.ptr, Tb.ptr, n, chi, wb.ptr + nc * chi, nc, sP);
    double* sbar = wb.ptr + 2 * nc * chi;
    proj_sbar(dev, S.ptr, kp, chi, wb.ptr, wb.ptr + nc * chi, sbar, nc, b);
    // U_bar, V_bar (columns >= k vanish with w)
    Tensor Vb = dev.empty({nc, n, chi}), Ub = dev.empty({nc, n, chi});
    qmul(dev, cp, true, n, chi, n, qb, qb32, n,
         pbw, chi, offsets<double*>(Vb.ptr, sP, nc), chi);
    qmul(dev, cp, false, n, chi, n, qa, qa32, n,
         tbw, chi, offsets<double*>(Ub.ptr, sP, nc), chi);
    // kept block
    Tensor Au = dev.empty({nc, chi, chi}), Av = dev.empty({nc, chi, chi}),
           Gkk = dev.empty({nc, chi, chi});
    gemm(dev, true, false, chi, chi, n, 1.0, U.ptr, b, sUV, Ub.ptr, chi, sP,
         0.0, Au.ptr, chi, sG, nc);
    gemm(dev, true, false, chi, chi, n, 1.0, V.ptr, b, sUV, Vb.ptr, chi, sP,
         0.0, Av.ptr, chi, sG, nc);
    svd_gkk(dev, Au.ptr, Av.ptr, S.ptr, sbar, kp, chi, Gkk.ptr, nc, b);
    // kept vectors as contiguous chi-wide blocks, columns >= k zeroed
    Tensor Ukm = dev.empty({nc, n, chi}), Vkm = dev.empty({nc, n, chi});
    copy2d(dev, U.ptr, b, Ukm.ptr, chi, n, chi, nc, sUV, sP);
    copy2d(dev, V.ptr, b, Vkm.ptr, chi, n, chi, nc, sUV, sP);
    mask_cols(dev, Ukm.ptr, n, chi, kp, nc);
    mask_cols(dev, Vkm.ptr, n, chi, kp, nc);
    // complement right-hand side [P_D U_bar; P'_D V_bar], [nc][2][n][chi]
    Tensor rhs = dev.empty({nc, 2, n, chi});
    copy2d(dev, Ub.ptr, chi, rhs.ptr, chi, n, chi, nc, sP, s2);
    copy2d(dev, Vb.ptr, chi, rhs.ptr + sP, chi, n, chi, nc, sP, s2);
    project_out(dev, Ukm.ptr, sP, rhs.ptr, s2, n, chi, nc);
    project_out(dev, Vkm.ptr, sP, rhs.ptr + sP, s2, n, chi, nc);

    // ---- column-wise deflated CG on A_j = [[s_j, -M], [-M^T, s_j]] (on the
    // complement), all columns of all cuts at once.
    // Deflation space: W = [[W_u, 0], [0, W_v]] with W_u, W_v orthonormal
    // bases of the subspace singular vectors chi..chi+m-1 projected on the
    // complement (the next triplets below the truncation, which set the
    // smallest eigenvalues s_j - s_i of A_j).  With H W = [[0, Y], [Zt, 0]],
    // Y = P_D M W_v, Zt = P'_D M^T W_u (formed once) and the eigenbasis Phi
    // of K = W^T H W, the Galerkin matrix of every column is
    // Phi diag(s_j - lambda) Phi^T.  Start x0 = W (W^T A_j W)^-1 W^T rhs, then
    // every search direction is made A_j-orthogonal to W, so CG runs on the
    // complement of W.  The Galerkin quantities are exact for any W, so the
    // solution does not depend on how well the triplets beyond chi have
    // converged; only the iteration count does.
    int m = std::min(b - chi, cxp->defl_max);
    if (m % 2) --m;
    if (m < 2) m = 0;
    const int m2 = 2 * m, m4 = 4 * m;
    const int64_t sXi = 2 * n * m4, sNm = n * m;
    Tensor X = dev.zeros({nc, 2, n, chi});
    // R, P, A P as consecutive slices: <r, p> and <p, A p> are then one
    // strided column-dot launch over 2 nc blocks
    Tensor RPA = dev.empty({3, nc, 2, n, chi});
    Tensor R = RPA.slice0(0), Pp = RPA.slice0(1), AP = RPA.slice0(2);
    Tensor t2 = dev.empty({nc, 2, n, chi});
    Tensor sc = dev.empty({5, nc, chi});  // <r, p>, pAp, rr, rr_new, rr0
    double *rp = sc.ptr, *pap = rp + nc * chi, *rr = pap + nc * chi,
           *rrn = rr + nc * chi, *rr0 = rrn + nc * chi;
    const int64_t tot = nc * s2;
    // transposed copies of the distinct cut matrices (in the storage the
    // products read: FP32 copies with FP32/BF16x3 products), so that every
    // product of A is an untransposed product and the two halves of A go
    // out in one launch each
    std::vector<Tensor> qt_keep;
    std::map<const void*, const void*> qt_made;
    auto qt = [&](const void* q, bool f32) {
      auto it = qt_made.find(q);
      if (it != qt_made.end()) return it->second;
      Tensor t = dev.empty({f32 ? (n * n + 1) / 2 : n * n});
      if (f32)
        transpose(dev, (const float*)q, (float*)t.ptr, n, n);
      else
        transpose(dev, (const double*)q, t.ptr, n, n);
      qt_keep.push_back(t);
      return qt_made[q] = (const void*)t.ptr;
    };
    const bool f32q = !qa32.empty();
    std::vector<const double*> s1q(2 * nc), s2q(2 * nc);
    std::vector<const float*> s1q32, s2q32;
    for (int c = 0; c < nc; ++c) {
      s1q[2 * c] = qb[c];
      s2q[2 * c] = qa[c];
      if (f32q) {
        s1q32.push_back(qb32[c]);
        s1q32.push_back((const float*)qt(qa32[c], true));
        s2q32.push_back(qa32[c]);
        s2q32.push_back((const float*)qt(qb32[c], true));
      } else {
        s1q[2 * c + 1] = (const double*)qt(qa[c], false);
        s2q[2 * c + 1] = (const double*)qt(qb[c], false);
      }
    }
    // kept vectors of both halves, interleaved per cut like out: [nc][2][n][chi]
    Tensor UVk = dev.empty({nc, 2, n, chi});
    copy2d(dev, Ukm.ptr, chi, UVk.ptr, chi, n, chi, nc, sP, s2);
    copy2d(dev, Vkm.ptr, chi, UVk.ptr + sP, chi, n, chi, nc, sP, s2);
    const auto t2w = offsets<double*>(t2.ptr, sP, 2 * nc);
    const auto t2r = offsets<const double*>(t2.ptr, sP, 2 * nc);
    const auto t1w = offsets<double*>(t2.ptr, sP, nc);  // n x chi per cut
    // out = A in = [s in_c - P_D Qa Qb in_b; s in_b - P'_D Qb^T Qa^T in_c]:
    // t = [Qb in_b; Qa^T in_c], then [Qa t_1; Qb^T t_2], both halves
    // projected off the kept vectors in one batched pair of products
    auto apply = [&](const Tensor& in, Tensor& out) {
      std::vector<const double*> bi(2 * nc);
      std::vector<double*> co(2 * nc);
      for (int c = 0; c < nc; ++c) {
        bi[2 * c] = in.ptr + c * s2 + sP;
        bi[2 * c + 1] = in.ptr + c * s2;
        co[2 * c] = out.ptr + c * s2;
        co[2 * c + 1] = out.ptr + c * s2 + sP;
      }
      qmul(dev, cp, false, n, chi, n, s1q, s1q32, n, bi, chi, t2w, chi);
      qmul(dev, cp, false, n, chi, n, s2q, s2q32, n, t2r, chi, co, chi);
      {
        // the projection is part of the operator: contraction precision,
        // like the products with the cut matrices (inner products and
        // residuals of the solve stay FP64)
        PrecScope ps(dev, cp);
        project_out(dev, UVk.ptr, sP, out.ptr, sP, n, chi, 2 * nc);
      }
      col_axpby(dev, nc * 2 * n, chi, 1.0, S.ptr, in.ptr, -1.0, out.ptr,
                2 * n, b);
    };
    // y (n x m blocks) <- y - Qk (Qk^T y), Qk the masked kept vectors
    auto off_kept = [&](const Tensor& Qk, double* y) {
      Tensor tk = dev.empty({nc, chi, m});
      gemm(dev, true, false, chi, m, n, 1.0, Qk.ptr, chi, sP, y, m, sNm, 0.0,
           tk.ptr, m, (int64_t)chi * m, nc);
      gemm(dev, false, false, n, m, chi, -1.0, Qk.ptr, chi, sP, tk.ptr, m,
           (int64_t)chi * m, 1.0, y, m, sNm, nc);
    };
    // Xi = [[W_u Phi_u, Y Phi_v], [W_v Phi_v, Zt Phi_u]]: [nc][2n][4m]; its
    // first 2m columns are W Phi, the last 2m are H W Phi
    Tensor Xi, lamK, Hd, Cf;
    if (m > 0) {
      // W: the subspace singular vectors chi..chi+m-1 of both sides.  They
      // are orthonormal and orthogonal to the kept ones already (columns of
      // the orthonormal U and V of the forward SVD; zero columns, from null
      // directions, stay zero and drop out of the Galerkin system)
      Tensor Wn = dev.empty({2, nc, n, m});
      copy2d(dev, U.ptr + chi, b, Wn.ptr, m, n, m, nc, sUV, sNm);
      copy2d(dev, V.ptr + chi, b, Wn.ptr + nc * sNm, m, n, m, nc, sUV, sNm);
      const double* Wu = Wn.ptr;
      const double* Wv = Wn.ptr + nc * sNm;
      // Y = P_D Qa Qb W_v, Zt = P'_D Qb^T Qa^T W_u
      Tensor T2 = dev.empty({nc, n, m}), YZ = dev.empty({2, nc, n, m});
      double* Y = YZ.ptr;
      double* Zt = YZ.ptr + nc * sNm;
      const auto t2w = offsets<double*>(T2.ptr, sNm, nc);
      const auto t2r = offsets<const double*>(T2.ptr, sNm, nc);
      qmul(dev, cp, false, n, m, n, qb, qb32, n,
           offsets<const double*>(Wv, sNm, nc), m, t2w, m);
      qmul(dev, cp, false, n, m, n, qa, qa32, n,
           t2r, m, offsets<double*>(Y, sNm, nc), m);
      qmul(dev, cp, true, n, m, n, qa, qa32, n,
           offsets<const double*>(Wu, sNm, nc), m, t2w, m);
      qmul(dev, cp, true, n, m, n, qb, qb32, n,
           t2r, m, offsets<double*>(Zt, sNm, nc), m);
      off_kept(Ukm, Y);
      off_kept(Vkm, Zt);
      // K = W^T H W and its eigenbasis
      Tensor Bk = dev.empty({2, nc, m, m});
      gemm(dev, true, false, m, m, n, 1.0, Wu, m, sNm, Y, m, sNm, 0.0,
           Bk.ptr, m, (int64_t)m * m, nc);
      gemm(dev, true, false, m, m, n, 1.0, Wv, m, sNm, Zt, m, sNm, 0.0,
           Bk.ptr + nc * m * m, m, (int64_t)m * m, nc);
      Tensor K = dev.empty({nc, m2, m2}), Phi = dev.empty({nc, m2, m2});
      lamK = dev.empty({nc, m2});
      defl_build_k(dev, Bk.ptr, Bk.ptr + nc * m * m, m, K.ptr, nc);
      const int64_t sPhi = (int64_t)m2 * m2;
      if (cxp->have_cg_warm && cxp->defl_phi.numel() == nc * sPhi) {
        // within one gradient the solves of consecutive unrolled
        // iterations see nearly the same K: in the eigenbasis Phi0 of the
        // previous solve's K, Phi0^T K Phi0 is nearly diagonal, and the
        // Jacobi solve finishes it in a sweep or two instead of the eight
        // or nine that the zero diagonal blocks of K itself take; Phi =
        // Phi0 Phi' is an eigenbasis of K to the same accuracy
        const double* P0 = cxp->defl_phi.ptr;
        Tensor KP = dev.empty({nc, m2, m2}), Kr = dev.empty({nc, m2, m2});
        Tensor Pr = dev.empty({nc, m2, m2});
        gemm(dev, false, false, m2, m2, m2, 1.0, K.ptr, m2, sPhi, P0, m2,
             sPhi, 0.0, KP.ptr, m2, sPhi, nc);
        gemm(dev, true, false, m2, m2, m2, 1.0, P0, m2, sPhi, KP.ptr, m2,
             sPhi, 0.0, Kr.ptr, m2, sPhi, nc);
        sym_eig_jacobi(dev, Kr.ptr, Pr.ptr, lamK.ptr, m2, nc);
        gemm(dev, false, false, m2, m2, m2, 1.0, P0, m2, sPhi, Pr.ptr, m2,
             sPhi, 0.0, Phi.ptr, m2, sPhi, nc);
      } else {
        sym_eig_jacobi(dev, K.ptr, Phi.ptr, lamK.ptr, m2, nc);
      }
      cxp->defl_phi = Phi;
      Xi = dev.empty({nc, 2 * n, m4});
      const double* Phu = Phi.ptr;
      const double* Phv = Phi.ptr + (int64_t)m * m2;
      gemm(dev, false, false, n, m2, m, 1.0, Wu, m, sNm, Phu, m2, sPhi, 0.0,
           Xi.ptr, m4, sXi, nc);
      gemm(dev, false, false, n, m2, m, 1.0, Y, m, sNm, Phv, m2, sPhi, 0.0,
           Xi.ptr + m2, m4, sXi, nc);
      gemm(dev, false, false, n, m2, m, 1.0, Wv, m, sNm, Phv, m2, sPhi, 0.0,
           Xi.ptr + n * m4, m4, sXi, nc);
      gemm(dev, false, false, n, m2, m, 1.0, Zt, m, sNm, Phu, m2, sPhi, 0.0,
           Xi.ptr + n * m4 + m2, m4, sXi, nc);
      Hd = dev.empty({nc, m4, chi});
      Cf = dev.empty({nc, m2, chi});
    }
    const int64_t sH = (int64_t)m4 * chi, sC = (int64_t)m2 * chi;
    // p -= W Phi diag(s_j - lambda)^-1 ((W Phi)^T A_j r)
    // (the two products of a CG iteration in the contraction precision, as
    // the operator's; the Galerkin coefficients in FP64)
    auto deflate = [&](const double* r, double* p) {
      PrecScope ps(dev, cp);
      gemm(dev, true, false, m4, chi, 2 * n, 1.0, Xi.ptr, m4, sXi, r, chi, s2,
           0.0, Hd.ptr, chi, sH, nc);
      defl_coef(dev, 1, S.ptr, kp, lamK.ptr, chi, m2, b, Hd.ptr, Cf.ptr, nc);
      gemm(dev, false, false, 2 * n, chi, m2, -1.0, Xi.ptr, m4, sXi, Cf.ptr,
           chi, sC, 1.0, p, chi, s2, nc);
    };
    coldot(dev, rhs.ptr, rhs.ptr, 2 * n, chi, rr0, nc, s2);
    axpby(dev, tot, 1.0, rhs.ptr, 0.0, R.ptr);
    // Start from the previous solve of this gradient when there is one (the
    // unrolled iterations near the fixed point solve nearly the same systems
    // with nearly parallel right-hand sides): x_g = alpha_j x_prev_j with
    // alpha_j = <rhs_j, A_j x_prev_j> / |A_j x_prev_j|^2, the multiple of the
    // previous solution with the smallest residual, r = rhs - alpha_j A_j
    // x_prev_j.  The Galerkin correction below then makes r orthogonal to W.
    // CG converges to the same solution from any start; only the iteration
    // count changes.
    const bool warm = cxp->have_cg_warm && cxp->cg_warm.numel() == tot;
    if (warm) {
      apply(cxp->cg_warm, AP);
      coldot(dev, AP.ptr, rhs.ptr, 2 * n, chi, rp, nc, s2);
      coldot(dev, AP.ptr, AP.ptr, 2 * n, chi, pap, nc, s2);
      colcg(dev, 0, nc * 2 * n, chi, rp, pap, X.ptr, R.ptr,
            cxp->cg_warm.ptr, AP.ptr, 2 * n);
    }
    if (m > 0) {
      // x += W Phi c and r -= A_j W Phi c = s_j W Phi c - (H W Phi) c for the
      // coefficients c in Cf
      Tensor Dx = dev.empty({nc, 2, n, chi});
      auto galerkin_add = [&]() {
        gemm(dev, false, false, 2 * n, chi, m2, 1.0, Xi.ptr, m4, sXi, Cf.ptr,
             chi, sC, 0.0, Dx.ptr, chi, s2, nc);
        axpby(dev, tot, 1.0, Dx.ptr, 1.0, X.ptr);
        col_axpby(dev, nc * 2 * n, chi, -1.0, S.ptr, Dx.ptr, 1.0, R.ptr,
                  2 * n, b);
        gemm(dev, false, false, 2 * n, chi, m2, 1.0, Xi.ptr + m2, m4, sXi,
             Cf.ptr, chi, sC, 1.0, R.ptr, chi, s2, nc);
      };
      if (warm) {
        // the warm start keeps no component in span(W): c = -(W Phi)^T x_g
        gemm(dev, true, false, m2, chi, 2 * n, -1.0, Xi.ptr, m4, sXi, X.ptr,
             chi, s2, 0.0, Cf.ptr, chi, sC, nc);
        galerkin_add();
      }
      // span(W) holds the discarded triplets next to the truncation, the
      // only ones that can come close to a kept one: there the solution is
      // the Galerkin one with the Lorentzian-broadened inverse,
      // c = rho / (s_j - lambda) (W Phi)^T r, rho = y^2 / (y^2 + eta^2),
      // y = s_j^2 - lambda^2, eta = 1e-12 s_1^2 (the broadening of the
      // kept block), i.e. x_j = y / (y^2 + eta^2) (s_j + lambda) in place
      // of 1 / (s_j - lambda)
      gemm(dev, true, false, m4, chi, 2 * n, 1.0, Xi.ptr, m4, sXi, R.ptr,
           chi, s2, 0.0, Hd.ptr, chi, sH, nc);
      defl_coef(dev, 2, S.ptr, kp, lamK.ptr, chi, m2, b, Hd.ptr, Cf.ptr, nc);
      galerkin_add();
      // the part of r in span(W) that the broadening leaves is not to be
      // solved: CG runs on the complement of W only
      gemm(dev, true, false, m2, chi, 2 * n, 1.0, Xi.ptr, m4, sXi, R.ptr,
           chi, s2, 0.0, Cf.ptr, chi, sC, nc);
      gemm(dev, false, false, 2 * n, chi, m2, -1.0, Xi.ptr, m4, sXi, Cf.ptr,
           chi, sC, 1.0, R.ptr, chi, s2, nc);
    }
    axpby(dev, tot, 1.0, R.ptr, 0.0, Pp.ptr);
    if (m > 0) deflate(R.ptr, Pp.ptr);
    coldot(dev, R.ptr, R.ptr, 2 * n, chi, rr, nc, s2);
    std::vector<double> h(5 * nc * chi);
    // relative residual 1e-12 with FP64 products; with FP32 products 1e-5
    // (BF16x3: 1e-3), and the solve also ends when two iterations no longer
    // reduce the worst relative residual by a factor 1/sqrt(2) (rounding
    // floor of the products).  Tested before the first iteration of a warm
    // start and after every second iteration.
    const bool lowp = cp != PREC_FP64;
    const double rtol = cp == PREC_FP64 ? cxp->adj_cg_tol
                                        : prec_floors(cp).cg_res;
    const double tol2 = rtol * rtol;
    double prev_worst = INFINITY;
    // <r, r> alternates between the rr and rr_new slices of sc (the fused
    // direction update writes the new value next to the old one)
    double* rrb[2] = {rr, rrn};
    int cur = 0;
    Tensor part = dev.empty({nc, colcg_parts(), chi});
    // Residual scale.  The first solve of a gradient belongs to the
    // unrolled iteration next to the energy, whose cotangent is the
    // largest; the cotangents reaching earlier iterations shrink by the
    // contraction factor of the CTMRG map per iteration, and so do the
    // right-hand sides of their solves.  Each later solve of the same
    // gradient stops at tol times the larger of its own right-hand side and
    // 1/K of the first one's (per cut and column): the error it leaves in
    // the gradient is then at most tol |rhs_first| / K, and the K solves
    // together at most about what the first one leaves, while the solves
    // of the iterations far from the energy end after few iterations or
    // none.
    const size_t ncol = (size_t)nc * chi;
    const bool use_ref = cxp->have_cg_warm && cxp->cg_ref.size() == ncol;
    bool set_ref = !cxp->have_cg_warm;
    auto converged = [&](bool stagnation) {
      dev.download(sc, h.data());
      bool done = true;
      double worst = 0.0;
      const double* hr = h.data() + (rrb[cur] - sc.ptr);  // rr
      const double* h0 = h.data() + 4 * nc * chi;  // rr0
      if (set_ref) {
        const double kk = (double)std::max(1, cxp->grad_K);
        const double k2 = kk * kk;
        cxp->cg_ref.assign(h0, h0 + ncol);
        for (double& v : cxp->cg_ref) v /= k2;
        set_ref = false;
      }
      for (size_t j = 0; j < ncol; ++j) {
        const double den = use_ref ? std::max(h0[j], cxp->cg_ref[j]) : h0[j];
        if (den > 0.0) {
          worst = std::max(worst, hr[j] / den);
          if (hr[j] > tol2 * den) done = false;
        }
      }
      if (stagnation && lowp && worst > 0.5 * prev_worst) done = true;
      prev_worst = worst;
      return done;
    };
    const int max_it = 600;
    int it = 0;
    const bool done0 = warm && converged(false);
    bool done = done0;
    for (; !done0 && it < max_it; ++it) {
      apply(Pp, AP);
      // x += alpha p, r -= alpha A p with alpha = <r, p> / <p, A p> (equal
      // to <r, r> / <p, A p> when p is exactly A-orthogonal to W)
      if (m > 0)  // <r, p> and <p, A p> (consecutive slices of RPA)
        coldot(dev, R.ptr, Pp.ptr, 2 * n, chi, rp, 2 * nc, s2);
      else
        coldot(dev, Pp.ptr, AP.ptr, 2 * n, chi, pap, nc, s2);
      colcg_step(dev, 2 * n, chi, nc, m > 0 ? rp : rrb[cur], pap, X.ptr,
                 R.ptr, Pp.ptr, AP.ptr, part.ptr);
      colcg_dir(dev, 2 * n, chi, nc, part.ptr, rrb[cur], rrb[cur ^ 1], R.ptr,
                Pp.ptr);
      cur ^= 1;
      if (m > 0) deflate(R.ptr, Pp.ptr);
      if ((it + 1) % 2 == 0 && converged(true)) {
        ++it;
        done = true;
        break;
      }
    }
    if (!done) ++st->cg_unconverged;
    if (cxp->check_true_residual) {
      // diagnostics: |rhs - A_j x_j| / |rhs_j| from a fresh application
      apply(X, AP);
      axpby(dev, tot, 1.0, rhs.ptr, -1.0, AP.ptr);
      coldot(dev, AP.ptr, AP.ptr, 2 * n, chi, rp, nc, s2);
      dev.download(sc, h.data());
      for (int j = 0; j < nc * chi; ++j)
        if (h[4 * nc * chi + j] > 0.0)
          st->cg_true_residual = std::max(
              st->cg_true_residual,
              std::sqrt(h[j] / h[4 * nc * chi + j]));
    }
    st->cg_iters += it;
    st->cg_solves += nc;
    cxp->cg_warm = X;
    cxp->have_cg_warm = true;
    // B = V Gkk^T + b_part, C = c_part
    Tensor Bm = dev.empty({nc, n, chi});
    copy2d(dev, X.ptr + sP, chi, Bm.ptr, chi, n, chi, nc, s2, sP);
    gemm(dev, false, true, n, chi, chi, 1.0, V.ptr, b, sUV, Gkk.ptr, chi, sG,
         1.0, Bm.ptr, chi, sP, nc);
    const auto bm = offsets<const double*>(Bm.ptr, sP, nc);
    const auto cm = offsets<const double*>(X.ptr, s2, nc);
    // Gradients of the cut matrices, each as one product of inner size
    // 2 chi (every n x n gradient is read and written once):
    //   Qa_bar += U (Qb B + T_w)^T + C (Qb V)^T
    //   Qb_bar += (Qa^T C + P_w) V^T + (Qa^T U) B^T
    // with the direct terms U T_w^T and P_w V^T of P = Qb V w and
    // Pt^T = Qa^T U w; the factors are packed side by side, n x 2 chi.
    const int64_t s2c = n * 2 * chi;
    Tensor Lp = dev.empty({nc, n, 2 * chi}), Rp = dev.empty({nc, n, 2 * chi});
    const auto lpr = offsets<const double*>(Lp.ptr, s2c, nc);
    const auto rpr = offsets<const double*>(Rp.ptr, s2c, nc);
    if (!gqa.empty()) {
      qmul(dev, cp, false, n, chi, n, qb, qb32, n, bm, chi, t1w, chi);
      axpby(dev, nc * sP, 1.0, Tbw.ptr, 1.0, t2.ptr);
      copy2d(dev, U.ptr, b, Lp.ptr, 2 * chi, n, chi, nc, sUV, s2c);
      copy2d(dev, X.ptr, chi, Lp.ptr + chi, 2 * chi, n, chi, nc, s2, s2c);
      copy2d(dev, t2.ptr, chi, Rp.ptr, 2 * chi, n, chi, nc, sP, s2c);
      copy2d(dev, QbV.ptr, chi, Rp.ptr + chi, 2 * chi, n, chi, nc, sP, s2c);
      gemm_ptrs_p(dev, cp, false, true, n, n, 2 * chi, 1.0, pick(lpr, ia),
                  2 * chi, pick(rpr, ia), 2 * chi, 1.0, gqa, n);
    }
    if (!gqb.empty()) {
      qmul(dev, cp, true, n, chi, n, qa, qa32, n, cm, chi, t1w, chi);
      axpby(dev, nc * sP, 1.0, Pbw.ptr, 1.0, t2.ptr);
      copy2d(dev, t2.ptr, chi, Lp.ptr, 2 * chi, n, chi, nc, sP, s2c);
      copy2d(dev, QaU.ptr, chi, Lp.ptr + chi, 2 * chi, n, chi, nc, sP, s2c);
      copy2d(dev, V.ptr, b, Rp.ptr, 2 * chi, n, chi, nc, sUV, s2c);
      copy2d(dev, Bm.ptr, chi, Rp.ptr + chi, 2 * chi, n, chi, nc, sP, s2c);
      gemm_ptrs_p(dev, cp, false, true, n, n, 2 * chi, 1.0, pick(lpr, ib),
                  2 * chi, pick(rpr, ib), 2 * chi, 1.0, gqb, n);
    }
  });
  return {P, PtT};
}

}  // namespace ipeps
