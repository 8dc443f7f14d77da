// Reduced density matrices and the energy per site on the device
// (Eqs. (6)-(7)): every Hamiltonian term contributes coef Tr(h rho)/Tr(rho)
// with rho the network of environment tensors around its sites, physical
// legs of those sites open.
//   (1,0), (0,1): 2x1 / 1x2 block  C1 T1 T1 C2 / T4 A A T2 / C4 T3 T3 C3
//   (1,1), (1,-1): 2x2 plaquette of enlarged corners, diagonal sites open
//   on-site: the 3x3 block around the site.
// Written on the differentiation tape so that the same contractions serve
// the energy and its backward pass.
#include <cmath>

#include "ad.hpp"
#include "ipeps_impl.hpp"

namespace ipeps {

namespace {

struct Net {
  Tape& tp;
  Context& cx;
  const VEnv& e;
  const std::vector<Var>& As;
  const std::vector<Var>& arot;
  int ns() const { return cx.nsite(); }
  Var C(int c, int s) const { return e.C[c * ns() + s]; }
  Var T(int c, int s) const { return e.T[c * ns() + s]; }
  Var a(int s, int c) const { return arot[s * 4 + c]; }
  Var E(const char* spec, const Var& x, const Var& y) {
    return tp.einsum(spec, x, y);
  }
  // ao[s, t, (l l'), (u u'), (r r'), (d d')]
  Var ao(int s, int c = 0) {
    const int D2 = cx.D2, d = cx.d;
    Var o = tp.view(E("sabce,tfghi->stafbgchei", As[s], As[s]),
                    {d, d, D2, D2, D2, D2});
    if (c == 0) return o;
    return tp.permute(o, {0, 1, 2 + c % 4, 2 + (c + 1) % 4, 2 + (c + 2) % 4,
                          2 + (c + 3) % 4});
  }
  Var rdm_h(int s1, int s2) {
    Var L1 = E("ij,mgi->jmg", C(0, s1), T(3, s1));
    Var L2 = E("jmg,qm->jgq", L1, C(3, s1));
    Var L3 = E("jgq,jek->gqek", L2, T(0, s1));
    Var L4 = E("gqek,wzq->gekwz", L3, T(2, s1));
    Var HL = E("gekwz,stgebz->kwstb", L4, ao(s1));
    Var R1 = E("ji,ibm->jbm", C(1, s2), T(1, s2));
    Var R2 = E("jbm,mq->jbq", R1, C(2, s2));
    Var R3 = E("kej,jbq->kebq", T(0, s2), R2);
    Var R4 = E("kebq,qzw->kebzw", R3, T(2, s2));
    Var HR = E("kebzw,stvebz->kwstv", R4, ao(s2));
    return E("kwstb,kwuvb->sutv", HL, HR);
  }
  Var rdm_v(int s1, int s2) {
    Var V1 = E("ij,jek->iek", C(0, s1), T(0, s1));
    Var V2 = E("iek,kp->iep", V1, C(1, s1));
    Var V3 = E("iep,mgi->epmg", V2, T(3, s1));
    Var V4 = E("epmg,pbn->emgbn", V3, T(1, s1));
    Var HT = E("emgbn,stgebz->mnstz", V4, ao(s1));
    Var W1 = E("qgm,wq->gmw", T(3, s2), C(3, s2));
    Var W2 = E("gmw,vyw->gmvy", W1, T(2, s2));
    Var W3 = E("gmvy,pv->gmyp", W2, C(2, s2));
    Var W4 = E("gmyp,nbp->gmynb", W3, T(1, s2));
    Var HB = E("gmynb,stgzby->mnstz", W4, ao(s2));
    return E("mnstz,mnuvz->sutv", HT, HB);
  }
  // enlarged corner c of site s, plain ([n][n]) or open ([n][n][d][d])
  Var corner(int c, int s, bool open) {
    const int64_t n = cx.n;
    Var X1 = E("mgi,ij->mgj", T((c + 3) % 4, s), C(c, s));
    Var X2 = E("mgj,jek->mgek", X1, T(c, s));
    if (!open) return tp.view(E("mgek,gebf->mfkb", X2, a(s, c)), {n, n});
    return tp.view(E("mgek,stgebf->mfkbst", X2, ao(s, c)),
                   {n, n, cx.d, cx.d});
  }
  Var rdm_diag(int s00, int s10, int s11, int s01, bool anti) {
    if (!anti) {
      Var Q0 = corner(0, s00, true), Q1 = corner(1, s10, false);
      Var Q2 = corner(2, s11, true), Q3 = corner(3, s01, false);
      Var P1 = E("XYst,YZ->XZst", Q0, Q1);
      Var P2 = E("ZWuv,WX->ZXuv", Q2, Q3);
      return E("XZst,ZXuv->sutv", P1, P2);
    }
    Var Q0 = corner(0, s00, false), Q1 = corner(1, s10, true);
    Var Q2 = corner(2, s11, false), Q3 = corner(3, s01, true);
    Var P1 = E("XY,YZuv->XZuv", Q0, Q1);
    Var P2 = E("ZW,WXst->ZXst", Q2, Q3);
    return E("XZuv,ZXst->sutv", P1, P2);
  }
  Var rdm_site(int s) {
    Var Tp1 = E("ij,jek->iek", C(0, s), T(0, s));
    Var Tp = E("iek,km->iem", Tp1, C(1, s));
    Var Bt1 = E("np,pzq->nzq", C(2, s), T(2, s));
    Var Bt = E("nzq,qw->nzw", Bt1, C(3, s));
    Var X = E("iem,mbn->iebn", Tp, T(1, s));
    Var Y = E("iebn,nzw->iebzw", X, Bt);
    Var Env = E("iebzw,wgi->gebz", Y, T(3, s));
    return E("gebz,stgebz->st", Env, ao(s));
  }
  Var term_rdm(const TermSpec& t) {
    const Lattice& L = cx.lat;
    const int x = t.site % L.Lx, y = t.site / L.Lx;
    if (t.kind == 0) return rdm_site(t.site);
    if (t.dx == 1 && t.dy == 0) return rdm_h(t.site, L.idx(x + 1, y));
    if (t.dx == 0 && t.dy == 1) return rdm_v(t.site, L.idx(x, y + 1));
    if (t.dx == 1 && t.dy == 1)
      return rdm_diag(L.idx(x, y), L.idx(x + 1, y), L.idx(x + 1, y + 1),
                      L.idx(x, y + 1), false);
    if (t.dx == 1 && t.dy == -1)
      return rdm_diag(L.idx(x, y - 1), L.idx(x + 1, y - 1), L.idx(x + 1, y),
                      L.idx(x, y), true);
    throw ArgError("unsupported term displacement");
  }
};

}  // namespace

double energy_ad(Tape& tp, Context& cx, const VEnv& e,
                 const std::vector<Var>& As, const std::vector<Var>& arot,
                 const std::vector<TermSpec>& terms) {
  Device& dev = cx.dev;
  Net net{tp, cx, e, As, arot};
  Tensor acc = dev.zeros({1});
  for (const auto& t : terms) {
    Var rho = net.term_rdm(t);
    const int m = t.kind == 0 ? cx.d : cx.d * cx.d;
    Tensor h = dev.empty({m, m});
    dev.upload(h, t.mat.data());
    double* rb = rho->req ? tp.grad(rho).ptr : nullptr;
    term_energy(dev, rho->v.ptr, h.ptr, m, t.coef / cx.nsite(), acc.ptr, rb);
  }
  double v = 0.0;
  dev.download(acc, &v);
  return v;
}

double energy(Context& cx, const Env& e, const std::vector<TermSpec>& terms) {
  Tape tp(cx.dev, false);
  VEnv v = venv_leaves(tp, cx, e);
  std::vector<Var> As = site_leaves(tp, cx, false);
  return energy_ad(tp, cx, v, As, arot_leaves(tp, cx), terms);
}

}  // namespace ipeps
