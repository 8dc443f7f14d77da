// Reduced density matrices and the energy per site on the device
// (Eqs. (6)-(7)): every Hamiltonian term contributes coef Tr(h rho)/Tr(rho)
// with rho the network of environment tensors around its sites, physical
// legs of those sites open.
//   (1,0), (0,1): 2x1 / 1x2 block  C1 T1 T1 C2 / T4 A A T2 / C4 T3 T3 C3
//   (1,1), (1,-1): 2x2 plaquette of enlarged corners, diagonal sites open
//   on-site: the 3x3 block around the site.
#include <cmath>

#include "ipeps_impl.hpp"
#include "observables.hpp"

namespace ipeps {

Tensor site_view(const Context& cx, const Tensor& A, int s) {
  Tensor t = A;
  const int64_t sz = (int64_t)cx.d * cx.D * cx.D * cx.D * cx.D;
  t.ptr = A.ptr + s * sz;
  t.shape = {cx.d, cx.D, cx.D, cx.D, cx.D};
  return t;
}

// ao[s, t, (l l'), (u u'), (r r'), (d d')]
Tensor open_double_layer(Context& cx, int s) {
  const int D2 = cx.D2, d = cx.d;
  Tensor As = site_view(cx, cx.A, s);
  Tensor a10 = einsum(cx.dev, "sabce,tfghi->stafbgchei", As, As);
  return a10.view({d, d, D2, D2, D2, D2});
}

Tensor rotate_open(Context& cx, const Tensor& ao, int c) {
  if (c == 0) return ao;
  return permuted(cx.dev, ao,
                  {0, 1, 2 + c % 4, 2 + (c + 1) % 4, 2 + (c + 2) % 4,
                   2 + (c + 3) % 4});
}

Tensor rdm_h(Context& cx, const Env& e, int s1, int s2, const Tensor& ao1,
             const Tensor& ao2) {
  Device& dev = cx.dev;
  Tensor L1 = einsum(dev, "ij,mgi->jmg", cx.Cv(e, 0, s1), cx.Tv(e, 3, s1));
  Tensor L2 = einsum(dev, "jmg,qm->jgq", L1, cx.Cv(e, 3, s1));
  Tensor L3 = einsum(dev, "jgq,jek->gqek", L2, cx.Tv(e, 0, s1));
  Tensor L4 = einsum(dev, "gqek,wzq->gekwz", L3, cx.Tv(e, 2, s1));
  Tensor HL = einsum(dev, "gekwz,stgebz->kwstb", L4, ao1);
  Tensor R1 = einsum(dev, "ji,ibm->jbm", cx.Cv(e, 1, s2), cx.Tv(e, 1, s2));
  Tensor R2 = einsum(dev, "jbm,mq->jbq", R1, cx.Cv(e, 2, s2));
  Tensor R3 = einsum(dev, "kej,jbq->kebq", cx.Tv(e, 0, s2), R2);
  Tensor R4 = einsum(dev, "kebq,qzw->kebzw", R3, cx.Tv(e, 2, s2));
  Tensor HR = einsum(dev, "kebzw,stvebz->kwstv", R4, ao2);
  return einsum(dev, "kwstb,kwuvb->sutv", HL, HR);
}

Tensor rdm_v(Context& cx, const Env& e, int s1, int s2, const Tensor& ao1,
             const Tensor& ao2) {
  Device& dev = cx.dev;
  Tensor V1 = einsum(dev, "ij,jek->iek", cx.Cv(e, 0, s1), cx.Tv(e, 0, s1));
  Tensor V2 = einsum(dev, "iek,kp->iep", V1, cx.Cv(e, 1, s1));
  Tensor V3 = einsum(dev, "iep,mgi->epmg", V2, cx.Tv(e, 3, s1));
  Tensor V4 = einsum(dev, "epmg,pbn->emgbn", V3, cx.Tv(e, 1, s1));
  Tensor HT = einsum(dev, "emgbn,stgebz->mnstz", V4, ao1);
  Tensor W1 = einsum(dev, "qgm,wq->gmw", cx.Tv(e, 3, s2), cx.Cv(e, 3, s2));
  Tensor W2 = einsum(dev, "gmw,vyw->gmvy", W1, cx.Tv(e, 2, s2));
  Tensor W3 = einsum(dev, "gmvy,pv->gmyp", W2, cx.Cv(e, 2, s2));
  Tensor W4 = einsum(dev, "gmyp,nbp->gmynb", W3, cx.Tv(e, 1, s2));
  Tensor HB = einsum(dev, "gmynb,stgzby->mnstz", W4, ao2);
  return einsum(dev, "mnstz,mnuvz->sutv", HT, HB);
}

// enlarged corner of site s, corner c, with a (plain, [D2]^4 rotated) or an
// open rotated double layer ([d][d][D2]^4): returns [n][n] or [n][n][d][d]
Tensor corner_of(Context& cx, const Env& e, int c, int s, const Tensor& ac) {
  Device& dev = cx.dev;
  Tensor X1 = einsum(dev, "mgi,ij->mgj", cx.Tv(e, (c + 3) % 4, s),
                     cx.Cv(e, c, s));
  Tensor X2 = einsum(dev, "mgj,jek->mgek", X1, cx.Tv(e, c, s));
  if (ac.rank() == 4) {
    Tensor Q = einsum(dev, "mgek,gebf->mfkb", X2, ac);
    return Q.view({cx.n, cx.n});
  }
  Tensor Q = einsum(dev, "mgek,stgebf->mfkbst", X2, ac);
  return Q.view({cx.n, cx.n, cx.d, cx.d});
}

Tensor rdm_diag(Context& cx, const Env& e, int s00, int s10, int s11,
                int s01, bool anti) {
  Device& dev = cx.dev;
  if (!anti) {
    Tensor Q0 = corner_of(cx, e, 0, s00,
                          rotate_open(cx, open_double_layer(cx, s00), 0));
    Tensor Q1 = corner_of(cx, e, 1, s10, cx.av(s10, 1));
    Tensor Q2 = corner_of(cx, e, 2, s11,
                          rotate_open(cx, open_double_layer(cx, s11), 2));
    Tensor Q3 = corner_of(cx, e, 3, s01, cx.av(s01, 3));
    Tensor P1 = einsum(dev, "XYst,YZ->XZst", Q0, Q1);
    Tensor P2 = einsum(dev, "ZWuv,WX->ZXuv", Q2, Q3);
    return einsum(dev, "XZst,ZXuv->sutv", P1, P2);
  }
  Tensor Q0 = corner_of(cx, e, 0, s00, cx.av(s00, 0));
  Tensor Q1 = corner_of(cx, e, 1, s10,
                        rotate_open(cx, open_double_layer(cx, s10), 1));
  Tensor Q2 = corner_of(cx, e, 2, s11, cx.av(s11, 2));
  Tensor Q3 = corner_of(cx, e, 3, s01,
                        rotate_open(cx, open_double_layer(cx, s01), 3));
  Tensor P1 = einsum(dev, "XY,YZuv->XZuv", Q0, Q1);
  Tensor P2 = einsum(dev, "ZW,WXst->ZXst", Q2, Q3);
  return einsum(dev, "XZuv,ZXst->sutv", P1, P2);
}

// ring of the eight environment tensors of site s: E[l, u, r, d] (fused)
Tensor site_env(Context& cx, const Env& e, int s) {
  Device& dev = cx.dev;
  Tensor Tp1 = einsum(dev, "ij,jek->iek", cx.Cv(e, 0, s), cx.Tv(e, 0, s));
  Tensor Tp = einsum(dev, "iek,km->iem", Tp1, cx.Cv(e, 1, s));
  Tensor Bt1 = einsum(dev, "np,pzq->nzq", cx.Cv(e, 2, s), cx.Tv(e, 2, s));
  Tensor Bt = einsum(dev, "nzq,qw->nzw", Bt1, cx.Cv(e, 3, s));
  Tensor X = einsum(dev, "iem,mbn->iebn", Tp, cx.Tv(e, 1, s));
  Tensor Y = einsum(dev, "iebn,nzw->iebzw", X, Bt);
  return einsum(dev, "iebzw,wgi->gebz", Y, cx.Tv(e, 3, s));
}

Tensor rdm_site(Context& cx, const Env& e, int s) {
  Tensor E = site_env(cx, e, s);
  return einsum(cx.dev, "gebz,stgebz->st", E, open_double_layer(cx, s));
}

Tensor term_rdm(Context& cx, const Env& e, const TermSpec& t) {
  const Lattice& L = cx.lat;
  const int x = t.site % L.Lx, y = t.site / L.Lx;
  if (t.kind == 0) return rdm_site(cx, e, t.site);
  if (t.dx == 1 && t.dy == 0) {
    const int s2 = L.idx(x + 1, y);
    return rdm_h(cx, e, t.site, s2, open_double_layer(cx, t.site),
                 open_double_layer(cx, s2));
  }
  if (t.dx == 0 && t.dy == 1) {
    const int s2 = L.idx(x, y + 1);
    return rdm_v(cx, e, t.site, s2, open_double_layer(cx, t.site),
                 open_double_layer(cx, s2));
  }
  if (t.dx == 1 && t.dy == 1)
    return rdm_diag(cx, e, L.idx(x, y), L.idx(x + 1, y), L.idx(x + 1, y + 1),
                    L.idx(x, y + 1), false);
  if (t.dx == 1 && t.dy == -1)
    return rdm_diag(cx, e, L.idx(x, y - 1), L.idx(x + 1, y - 1),
                    L.idx(x + 1, y), L.idx(x, y), true);
  throw ArgError("unsupported term displacement");
}

double energy(Context& cx, const Env& e, const std::vector<TermSpec>& terms,
              Tensor* gA, Env* gEnv) {
  (void)gA;
  (void)gEnv;
  Device& dev = cx.dev;
  Tensor acc = dev.zeros({1});
  for (const auto& t : terms) {
    Tensor rho = term_rdm(cx, e, t);
    const int m = t.kind == 0 ? cx.d : cx.d * cx.d;
    Tensor h = dev.empty({m, m});
    dev.upload(h, t.mat.data());
    term_energy(dev, rho.ptr, h.ptr, m, t.coef / cx.nsite(), acc.ptr,
                nullptr);
  }
  double v = 0.0;
  dev.download(acc, &v);
  return v;
}

}  // namespace ipeps
