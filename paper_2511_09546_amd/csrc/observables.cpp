// Reduced density matrices and the energy per site on the device
// (Eqs. (6)-(7)): every Hamiltonian term contributes coef Tr(h rho)/Tr(rho)
// with rho the network of environment tensors around its sites, physical
// legs of those sites open.
//   (1,0), (0,1): 2x1 / 1x2 block  C1 T1 T1 C2 / T4 A A T2 / C4 T3 T3 C3
//   (1,1), (1,-1): 2x2 plaquette of enlarged corners, diagonal sites open
//   on-site: the 3x3 block around the site.
// Written on the differentiation tape so that the same contractions serve
// the energy and its backward pass.
#include <array>
#include <cmath>
#include <map>
#include <set>
#include <utility>

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
  // the same for an intermediate that only products read: FP32 storage
  // with FP32 or BF16 products (which round it to FP32 anyway)
  Var E32(const char* spec, const Var& x, const Var& y) {
    return tp.einsum_n(spec, {x}, {y}, true)[0];
  }
  // tensors shared by several terms of one evaluation, keyed by
  // (corner, site): the open double layers, the corner-edge products X2
  // and the enlarged corners (plain and with open physical legs)
  using Key = std::pair<int, int>;
  std::map<Key, Var> ao_c, x2_c, qo_c, qp_c;
  std::set<Key> open_and_plain;  // corners wanted both ways
  // ao[s, t, (l l'), (u u'), (r r'), (d d')]
  Var ao(int s, int c = 0) {
    auto it = ao_c.find({c, s});
    if (it != ao_c.end()) return it->second;
    const int D2 = cx.D2, d = cx.d;
    Var o;
    if (c == 0)
      o = tp.view(E("sabce,tfghi->stafbgchei", As[s], As[s]),
                  {d, d, D2, D2, D2, D2});
    else
      o = tp.permute(ao(s, 0), {0, 1, 2 + c % 4, 2 + (c + 1) % 4,
                                2 + (c + 2) % 4, 2 + (c + 3) % 4});
    return ao_c[{c, s}] = o;
  }
  // T_{c-1} C_c T_c of corner c at site s, grouped [m k | g e] for the
  // product with the double layer
  Var x2(int c, int s) {
    auto it = x2_c.find({c, s});
    if (it != x2_c.end()) return it->second;
    Var X1 = E("mgi,ij->mgj", T((c + 3) % 4, s), C(c, s));
    return x2_c[{c, s}] = E32("mgj,jek->mkge", X1, T(c, s));
  }
  // Each half of the 2x1 (1x2) block contracts the open double layer into
  // the corner-edge-corner-edge product over the two legs they share first
  // (chi^2 d^2 D^4 intermediate, like an open enlarged corner), then closes
  // the third edge; intermediates are written grouped for their next
  // product.
  Var rdm_h(int s1, int s2) {
    Var L1 = E("ij,mgi->jmg", C(0, s1), T(3, s1));
    Var L2 = E("jmg,qm->jgq", L1, C(3, s1));
    Var L3 = E32("jgq,jek->qkge", L2, T(0, s1));
    Var L5 = E32("qkge,stgebz->kstbqz", L3, ao(s1));
    Var HL = E("kstbqz,wzq->kwstb", L5, T(2, s1));
    Var R1 = E("ji,ibm->jbm", C(1, s2), T(1, s2));
    Var R2 = E("jbm,mq->jbq", R1, C(2, s2));
    Var R3 = E32("kej,jbq->kqeb", T(0, s2), R2);
    Var R5 = E32("kqeb,stvebz->kstvqz", R3, ao(s2));
    Var HR = E("kstvqz,qzw->kwstv", R5, T(2, s2));
    return E("kwstb,kwuvb->sutv", HL, HR);
  }
  Var rdm_v(int s1, int s2) {
    Var V1 = E("ij,jek->iek", C(0, s1), T(0, s1));
    Var V2 = E("iek,kp->iep", V1, C(1, s1));
    Var V3 = E32("iep,mgi->pmge", V2, T(3, s1));
    Var V5 = E32("pmge,stgebz->mstzpb", V3, ao(s1));
    Var HT = E("mstzpb,pbn->mnstz", V5, T(1, s1));
    Var W1 = E("qgm,wq->gmw", T(3, s2), C(3, s2));
    Var W2 = E("gmw,vyw->gmvy", W1, T(2, s2));
    Var W3 = E32("gmvy,pv->mpgy", W2, C(2, s2));
    Var W5 = E32("mpgy,stgzby->mstzpb", W3, ao(s2));
    Var HB = E("mstzpb,nbp->mnstz", W5, T(1, s2));
    return E("mnstz,mnuvz->sutv", HT, HB);
  }
  // enlarged corner c of site s, plain ([n][n]) or open ([n][n][d][d]);
  // a corner wanted both ways is built open once and traced over its
  // physical legs for the plain one
  Var corner(int c, int s, bool open) {
    const int64_t n = cx.n;
    const Key k{c, s};
    std::map<Key, Var>& cache = open ? qo_c : qp_c;
    auto it = cache.find(k);
    if (it != cache.end()) return it->second;
    Var q;
    if (open)
      q = tp.view(E("mkge,stgebf->mfkbst", x2(c, s), ao(s, c)),
                  {n, n, cx.d, cx.d});
    else if (open_and_plain.count(k))
      q = tp.trace_dd(corner(c, s, true));
    else
      q = tp.view(E("mkge,gebf->mfkb", x2(c, s), a(s, c)), {n, n});
    return cache[k] = q;
  }
  // the corners of the diagonal terms, [c] = (site, open)
  std::array<std::pair<int, bool>, 4> diag_corners(const TermSpec& t) const {
    const Lattice& L = cx.lat;
    const int x = t.site % L.Lx, y = t.site / L.Lx;
    if (t.dy == 1)
      return {{{L.idx(x, y), true}, {L.idx(x + 1, y), false},
               {L.idx(x + 1, y + 1), true}, {L.idx(x, y + 1), false}}};
    return {{{L.idx(x, y - 1), false}, {L.idx(x + 1, y - 1), true},
             {L.idx(x + 1, y), false}, {L.idx(x, y), true}}};
  }
  // marks the corners that the diagonal terms want both open and plain
  void plan(const std::vector<TermSpec>& terms) {
    std::set<Key> op, pl;
    for (const auto& t : terms) {
      if (t.kind == 0 || t.dx != 1 || (t.dy != 1 && t.dy != -1)) continue;
      const auto cs = diag_corners(t);
      for (int c = 0; c < 4; ++c)
        (cs[c].second ? op : pl).insert({c, cs[c].first});
    }
    for (const Key& k : op)
      if (pl.count(k)) open_and_plain.insert(k);
  }
  Var rdm_diag(int s00, int s10, int s11, int s01, bool anti) {
    // the corner choices of diag_corners
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
  net.plan(terms);
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
