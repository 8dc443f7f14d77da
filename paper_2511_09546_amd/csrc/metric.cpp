// Local-metric preconditioner (Eq. (11)) with regularisation N + delta I
// (Sec. III B), solved by conjugate gradients (Sec. III C), one independent
// solve per unit-cell site (Sec. IV B).
//
// N is applied matrix-free from the converged environment: with the
// half-rings LT = T4 (C1 T1 C2) (left + top) and RB = T2 (C3 T3 C4) (right +
// bottom), the single-site ring is E[(l l'),(u u'),(r r'),(d d')] =
// sum_{w,m} LT[w,(l l'),(u u'),m] RB[m,(r r'),(d d'),w], and
//   (N x)[t, l'u'r'd'] = sum_{lurd} E x[t, lurd] / Z,  Z = <A, E A>.
// Two GEMMs per application (K = D^2, then K = chi^2 D^2) with LT and RB
// permuted once so that neither GEMM needs a permute.  CG scalars, dots and
// residuals are FP64; alpha and beta stay on the device.  The same operator
// is also solved by one GMRES cycle (precondition_gmres), the Krylov solve
// the paper names.
#include <cmath>

#include "ipeps_impl.hpp"

namespace ipeps {

namespace {

struct SiteMetric {
  Tensor LTq;  // [(l u), (l' u' w m)]   : [D^2][D^2 chi^2]
  Tensor RBq;  // [(w m r d), (r' d')]   : [chi^2 D^2][D^2]
  Tensor Zinv; // device scalar 1/Z
};

SiteMetric build_metric(Context& cx, const Env& e, int s) {
  Device& dev = cx.dev;
  const int D = cx.D, chi = cx.chi;
  SiteMetric sm;
  // each half ring is permuted and its unpermuted form released before the
  // other is built: at most three chi^2 D^4 buffers are live at once
  {
    Tensor Tp1 = einsum(dev, "ij,jek->iek", cx.Cv(e, 0, s), cx.Tv(e, 0, s));
    Tensor Tp = einsum(dev, "iek,km->iem", Tp1, cx.Cv(e, 1, s));
    Tensor LT = einsum(dev, "wgi,iem->wgem", cx.Tv(e, 3, s), Tp);
    // LT[w, l, l', u, u', m] -> [l, u, l', u', w, m]
    Tensor LT6 = LT.view({chi, D, D, D, D, chi});
    sm.LTq = permuted(dev, LT6, {1, 3, 2, 4, 0, 5});
  }
  {
    Tensor Bt1 = einsum(dev, "np,pzq->nzq", cx.Cv(e, 2, s), cx.Tv(e, 2, s));
    Tensor Bt = einsum(dev, "nzq,qw->nzw", Bt1, cx.Cv(e, 3, s));
    Tensor RB = einsum(dev, "mbn,nzw->mbzw", cx.Tv(e, 1, s), Bt);
    // RB[m, r, r', d, d', w] -> [w, m, r, d, r', d']
    Tensor RB6 = RB.view({chi, D, D, D, D, chi});
    sm.RBq = permuted(dev, RB6, {5, 0, 1, 3, 2, 4});
  }
  sm.Zinv = dev.empty({1});
  return sm;
}

// y = E x (unnormalised), x and y [d][D^4]; `lean` runs the physical
// index t one at a time through a W1 of one chi^2 D^4 block (the
// allocation-free entry point), else all of them in one batched product
void apply_ring(Context& cx, const SiteMetric& sm, const double* x,
                double* y, Tensor& W1, bool lean = false) {
  Device& dev = cx.dev;
  const int64_t D2 = cx.D2, chi = cx.chi;
  const int64_t Mq = D2 * chi * chi;  // (l' u' w m)
  const int64_t nb = lean ? 1 : cx.d;
  if (W1.numel() != nb * Mq * D2) W1 = dev.empty({nb, Mq, D2});
  for (int64_t t0 = 0; t0 < cx.d; t0 += nb) {
    const double* xt = x + t0 * D2 * D2;
    double* yt = y + t0 * D2 * D2;
    // W1[t][(l' u' w m)][(r d)] =
    //   sum_{(l u)} LTq[(l u)][(l' u' w m)] x[t][(l u)][(r d)]
    gemm(dev, true, false, Mq, D2, D2, 1.0, sm.LTq.ptr, Mq, 0, xt, D2,
         D2 * D2, 0.0, W1.ptr, D2, Mq * D2, nb);
    // y[t][(l' u')][(r' d')] = sum_{(w m r d)} W1[t][(l' u')][(w m r d)] RBq
    gemm(dev, false, false, D2, D2, chi * chi * D2, 1.0, W1.ptr,
         chi * chi * D2, Mq * D2, sm.RBq.ptr, D2, 0, 0.0, yt, D2, D2 * D2,
         nb);
  }
}

}  // namespace

size_t precondition_lean_bytes(int nsite, int d, int D, int chi) {
  // blocks as the pool rounds them (256 bytes; 64 KiB above 1 MiB)
  auto blk = [](double words) {
    double b = 8.0 * words;
    b = std::ceil(b / 256.0) * 256.0;
    if (b > 1048576.0) b = std::ceil(b / 65536.0) * 65536.0;
    return b;
  };
  const double D2 = (double)D * D, c = chi;
  const double q = c * c * D2 * D2;     // a half ring, or W1 of one index
  const double m = d * D2 * D2;         // one site tensor
  // LTq, RBq and one more half-ring block (the unpermuted ring, then W1);
  // two chi^2 D^2 products per half ring; g, x, r, p, Ap; the CG scalars,
  // the reduction partials of dot and 256 split-K partial sums of the
  // D^2 x D^2 product with K = chi^2 D^2; 1 MiB of slack
  const double bytes = 3.0 * blk(q) + 2.0 * blk(c * c * D2) +
                       2.0 * blk(nsite * m) + 3.0 * blk(m) + blk(8) +
                       4.0 * blk(4096) + blk(256.0 * D2 * D2) + 1048576.0;
  return (size_t)bytes;
}

// CG kernels live in kernels.hip
void cg_update_xr(Device& dev, int64_t n, const double* rr, const double* pAp,
                  const double* p, const double* Ap, double* x, double* r);
void cg_update_p(Device& dev, int64_t n, const double* rr_new,
                 const double* rr, const double* pAp, const double* r,
                 double* p);
void scale_add_dev(Device& dev, int64_t n, const double* s, const double* x,
                   double delta, double* y);

int precondition(Context& cx, const double* g_host, double delta,
                 double cg_tol, int cg_maxiter, double* x_host, int* n_iter,
                 double* rel_resid, bool on_device, bool lean) {
  Device& dev = cx.dev;
  const int ns = cx.nsite();
  const int64_t m = (int64_t)cx.d * cx.D2 * cx.D2;  // per-site length
  Tensor g = dev.empty({ns, m});
  if (on_device)
    axpby(dev, ns * m, 1.0, g_host, 0.0, g.ptr);
  else
    dev.upload(g, g_host);
  Tensor x = dev.zeros({ns, m});
  Tensor r = dev.empty({m}), p = dev.empty({m}), Ap = dev.empty({m});
  Tensor sc = dev.zeros({8});  // 0 rr, 1 pAp, 2 rr_new, 3 gnorm^2, 4 Z
  Tensor W1;
  int worst_it = 0;
  double worst_res = 0.0;
  bool breakdown = false;
  for (int s = 0; s < ns; ++s) {
    SiteMetric sm = build_metric(cx, cx.env, s);
    // Z = <A, E A>
    apply_ring(cx, sm, cx.A.ptr + s * m, Ap.ptr, W1, lean);
    dot(dev, cx.A.ptr + s * m, Ap.ptr, m, sc.ptr + 4);
    const double* gs = g.ptr + s * m;
    double* xs = x.ptr + s * m;
    axpby(dev, m, 1.0, gs, 0.0, r.ptr);
    axpby(dev, m, 1.0, gs, 0.0, p.ptr);
    dot(dev, r.ptr, r.ptr, m, sc.ptr + 0);
    double hs[8];
    dev.download(sc, hs);
    const double gnorm = std::sqrt(hs[0]);
    double rr = hs[0];
    int it = 0;
    if (gnorm > 0.0) {
      while (it < cg_maxiter && std::sqrt(rr) > cg_tol * gnorm) {
        if (it == cx.fault_cg_breakdown_at) {
          // test hook: handled like a detected breakdown at this iteration
          breakdown = true;
          break;
        }
        apply_ring(cx, sm, p.ptr, Ap.ptr, W1, lean);
        // Ap = Ap / Z + delta p
        scale_add_dev(dev, m, sc.ptr + 4, p.ptr, delta, Ap.ptr);
        dot(dev, p.ptr, Ap.ptr, m, sc.ptr + 1);
        cg_update_xr(dev, m, sc.ptr + 0, sc.ptr + 1, p.ptr, Ap.ptr, xs,
                     r.ptr);
        dot(dev, r.ptr, r.ptr, m, sc.ptr + 2);
        cg_update_p(dev, m, sc.ptr + 2, sc.ptr + 0, sc.ptr + 1, r.ptr,
                    p.ptr);
        dev.download(sc, hs);
        if (!(hs[1] > 0.0)) {
          // breakdown: the update kernels skipped this step, x holds the
          // last iterate
          breakdown = true;
          break;
        }
        rr = hs[2];
        // rr <- rr_new (device)
        axpby(dev, 1, 1.0, sc.ptr + 2, 0.0, sc.ptr + 0);
        ++it;
      }
    }
    worst_it = std::max(worst_it, it);
    worst_res = std::max(worst_res, gnorm > 0.0 ? std::sqrt(rr) / gnorm : 0.0);
    if (breakdown) break;
  }
  if (on_device) {
    axpby(dev, ns * m, 1.0, x.ptr, 0.0, x_host);
    dev.sync();
  } else {
    dev.download(x, x_host);
  }
  if (n_iter) *n_iter = worst_it;
  if (rel_resid) *rel_resid = worst_res;
  return breakdown ? -4 : 0;
}

void precondition_gmres(Context& cx, const double* g_in, double delta,
                        int m_kry, double tol, double* x_out, int* n_used,
                        double* rel_resid, bool on_device) {
  Device& dev = cx.dev;
  const int ns = cx.nsite();
  const int64_t m = (int64_t)cx.d * cx.D2 * cx.D2;  // per-site length
  Tensor g = dev.empty({ns, m});
  if (on_device)
    axpby(dev, ns * m, 1.0, g_in, 0.0, g.ptr);
  else
    dev.upload(g, g_in);
  Tensor x = dev.empty({ns, m});
  Tensor Ap = dev.empty({m});
  Tensor Z = dev.empty({1});
  Tensor W1;
  int worst_k = 0;
  double worst_res = 0.0;
  for (int s = 0; s < ns; ++s) {
    SiteMetric sm = build_metric(cx, cx.env, s);
    apply_ring(cx, sm, cx.A.ptr + s * m, Ap.ptr, W1);
    dot(dev, cx.A.ptr + s * m, Ap.ptr, m, Z.ptr);
    auto op = [&](const double* v, double* y) {
      apply_ring(cx, sm, v, y, W1);
      scale_add_dev(dev, m, Z.ptr, v, delta, y);
    };
    double res = 0.0;
    const int k = gmres(dev, m, g.ptr + s * m, x.ptr + s * m, m_kry, tol, op,
                        &res);
    worst_k = std::max(worst_k, k);
    worst_res = std::max(worst_res, res);
  }
  if (on_device) {
    axpby(dev, ns * m, 1.0, x.ptr, 0.0, x_out);
    dev.sync();
  } else {
    dev.download(x, x_out);
  }
  if (n_used) *n_used = worst_k;
  if (rel_resid) *rel_resid = worst_res;
}

}  // namespace ipeps
