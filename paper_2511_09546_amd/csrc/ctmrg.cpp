// CTMRG on the device: double layer, trace-boundary start, one simultaneous
// four-corner iteration with half-system SVD projectors, normalisation and
// the corner-spectrum convergence measure (Sec. III A: the environment of the
// energy network, Eq. (7)).  The iteration is written once, on the
// differentiation tape: with recording off it is the plain forward move,
// with recording on it is the step that the backward pass unrolls.
#include <algorithm>
#include <cmath>

#include "ad.hpp"
#include "ipeps_impl.hpp"

namespace ipeps {

Tensor Context::Cv(const Env& e, int c, int s) const {
  Tensor t = e.C;
  t.ptr = e.C.ptr + ((int64_t)c * nsite() + s) * chi * chi;
  t.shape = {chi, chi};
  return t;
}

Tensor Context::Tv(const Env& e, int c, int s) const {
  Tensor t = e.T;
  t.ptr = e.T.ptr + ((int64_t)c * nsite() + s) * chi * D2 * chi;
  t.shape = {chi, D2, chi};
  return t;
}

Tensor Context::av(int s, int c) const {
  Tensor t = a_rot;
  const int64_t a4 = (int64_t)D2 * D2 * D2 * D2;
  t.ptr = a_rot.ptr + ((int64_t)s * 4 + c) * a4;
  t.shape = {D2, D2, D2, D2};
  return t;
}

static std::vector<int> rot_perm(int c) {
  return {c % 4, (c + 1) % 4, (c + 2) % 4, (c + 3) % 4};
}

// a = sum_p A[p,l,u,r,d] A[p,l',u',r',d'], legs fused (k k') -> k*D + k',
// stored in the four clockwise rotations a_c.
void build_double_layer(Context& cx) {
  const int ns = cx.nsite(), D2 = cx.D2, D = cx.D;
  cx.bp_valid = false;  // the belief-propagation messages belong to old A
  cx.c4v_sym = false;   // A is no longer known to be projected
  cx.env_injected = false;  // an environment set before was for old A
  const int64_t a4 = (int64_t)D2 * D2 * D2 * D2;
  if (cx.a_rot.numel() != ns * 4 * a4)
    cx.a_rot = cx.dev.empty({ns, 4, D2, D2, D2, D2});
  for (int s = 0; s < ns; ++s) {
    Tensor As = cx.A;
    As.ptr = cx.A.ptr + (int64_t)s * cx.d * D * D * D * D;
    As.shape = {cx.d, D, D, D, D};
    Tensor a = einsum(cx.dev, "pabce,pfghi->afbgchei", As, As)
                   .view({D2, D2, D2, D2});
    for (int c = 0; c < 4; ++c) {
      Tensor dst = cx.av(s, c);
      permute(cx.dev, a, rot_perm(c), dst);
    }
  }
}

std::vector<Var> arot_leaves(Tape& tp, Context& cx) {
  std::vector<Var> r(4 * cx.nsite());
  for (int s = 0; s < cx.nsite(); ++s)
    for (int c = 0; c < 4; ++c) r[s * 4 + c] = tp.leaf(cx.av(s, c), false);
  return r;
}

std::vector<Var> arot_from_sites(Tape& tp, Context& cx,
                                 const std::vector<Var>& As) {
  return arot_from_pairs(tp, cx, As, As);
}

// a = sum_p K[p,l,u,r,d] B[p,l',u',r',d'] per site, fused (k k') with k
// from the ket K: the mixed double layer of two different site tensors
std::vector<Var> arot_from_pairs(Tape& tp, Context& cx,
                                 const std::vector<Var>& Ks,
                                 const std::vector<Var>& Bs) {
  const int D2 = cx.D2;
  std::vector<Var> r(4 * cx.nsite());
  for (int s = 0; s < cx.nsite(); ++s) {
    Var a = tp.view(tp.einsum("pabce,pfghi->afbgchei", Ks[s], Bs[s]),
                    {D2, D2, D2, D2});
    r[s * 4] = a;
    for (int c = 1; c < 4; ++c) r[s * 4 + c] = tp.permute(a, rot_perm(c));
  }
  return r;
}

std::vector<Var> site_leaves(Tape& tp, Context& cx, bool req) {
  Var A = tp.leaf(cx.A, req);
  std::vector<Var> r(cx.nsite());
  for (int s = 0; s < cx.nsite(); ++s) r[s] = tp.slice0(A, s);
  return r;
}

VEnv venv_leaves(Tape& tp, Context& cx, const Env& e, bool req) {
  VEnv v;
  const int ns = cx.nsite();
  v.C.resize(4 * ns);
  v.T.resize(4 * ns);
  for (int c = 0; c < 4; ++c)
    for (int s = 0; s < ns; ++s) {
      v.C[c * ns + s] = tp.leaf(cx.Cv(e, c, s), req);
      v.T[c * ns + s] = tp.leaf(cx.Tv(e, c, s), req);
    }
  return v;
}

VEnv init_env_ad(Tape& tp, Context& cx, const std::vector<Var>& arot) {
  const int ns = cx.nsite(), chi = cx.chi, D2 = cx.D2;
  std::vector<double> h((size_t)D2, 0.0);
  for (int k = 0; k < cx.D; ++k) h[(size_t)k * cx.D + k] = 1.0;
  Tensor tv = cx.dev.empty({D2});
  cx.dev.upload(tv, h.data());
  Var t = tp.leaf(tv, false);
  VEnv v;
  v.C.resize(4 * ns);
  v.T.resize(4 * ns);
  for (int s = 0; s < ns; ++s)
    for (int c = 0; c < 4; ++c) {
      const int sc = cx.lat.shift(s, INIT_CORNER_SITE[c][0],
                                  INIT_CORNER_SITE[c][1]);
      Var t1 = tp.einsum("gebf,g->ebf", arot[sc * 4 + c], t);
      Var cc = tp.einsum("ebf,e->fb", t1, t);
      v.C[c * ns + s] = tp.pad3(cc, 1, D2, D2, {chi, chi});
      const int se = cx.lat.shift(s, INIT_EDGE_SITE[c][0],
                                  INIT_EDGE_SITE[c][1]);
      Var tt = tp.einsum("gebf,e->gfb", arot[se * 4 + c], t);
      v.T[c * ns + s] = tp.pad3(tt, D2, D2, D2, {chi, D2, chi});
    }
  return v;
}

Env env_pack(Context& cx, const VEnv& v) {
  const int ns = cx.nsite(), chi = cx.chi, D2 = cx.D2;
  Env e;
  e.C = cx.dev.empty({4, ns, chi, chi});
  e.T = cx.dev.empty({4, ns, chi, D2, chi});
  const int64_t cs = (int64_t)chi * chi, ts = cs * D2;
  for (int i = 0; i < 4 * ns; ++i) {
    axpby(cx.dev, cs, 1.0, v.C[i]->v.ptr, 0.0, e.C.ptr + i * cs);
    axpby(cx.dev, ts, 1.0, v.T[i]->v.ptr, 0.0, e.T.ptr + i * ts);
  }
  return e;
}

// Trace-boundary start: corners and edges are double layers whose outward
// legs are closed with delta_{k k'}; bond dimension D^2 zero padded to chi.
void init_env(Context& cx) {
  const int ns = cx.nsite(), chi = cx.chi, D2 = cx.D2;
  Env e;
  e.C = cx.dev.zeros({4, ns, chi, chi});
  e.T = cx.dev.zeros({4, ns, chi, D2, chi});
  std::vector<double> h((size_t)D2, 0.0);
  for (int k = 0; k < cx.D; ++k) h[(size_t)k * cx.D + k] = 1.0;
  Tensor tv = cx.dev.empty({D2});
  cx.dev.upload(tv, h.data());
  for (int s = 0; s < ns; ++s)
    for (int c = 0; c < 4; ++c) {
      Tensor ac = cx.av(cx.lat.shift(s, INIT_CORNER_SITE[c][0],
                                     INIT_CORNER_SITE[c][1]), c);
      Tensor t1 = einsum(cx.dev, "gebf,g->ebf", ac, tv);
      Tensor cc = einsum(cx.dev, "ebf,e->fb", t1, tv);
      Tensor Cd = cx.Cv(e, c, s);
      pad3(cx.dev, cc.ptr, Cd.ptr, 1, D2, D2, chi, chi);
      Tensor ae = cx.av(cx.lat.shift(s, INIT_EDGE_SITE[c][0],
                                     INIT_EDGE_SITE[c][1]), c);
      Tensor tt = einsum(cx.dev, "gebf,e->gfb", ae, tv);
      Tensor Td = cx.Tv(e, c, s);
      pad3(cx.dev, tt.ptr, Td.ptr, D2, D2, D2, D2, chi);
    }
  cx.env = e;
  cx.have_env = true;
  cx.have_warm = false;
}

std::vector<Var> arot_fb(Tape& tp, const std::vector<Var>& arot) {
  std::vector<Var> r(arot.size());
  for (size_t i = 0; i < arot.size(); ++i)
    r[i] = tp.permute(arot[i], {0, 1, 3, 2});
  return r;
}

VEnv ctm_step_ad(Tape& tp, Context& cx, const VEnv& in,
                 const std::vector<Var>& arot,
                 const std::vector<Var>* arotf) {
  const int ns = cx.nsite(), chi = cx.chi, D2 = cx.D2, nc = cx.ncut();
  const int64_t n = cx.n;
  const Lattice& L = cx.lat;
  auto C = [&](int c, int s) { return in.C[c * ns + s]; };
  auto T = [&](int c, int s) { return in.T[c * ns + s]; };
  std::vector<Var> af_own;
  if (!arotf) af_own = arot_fb(tp, arot);
  const std::vector<Var>& afv = arotf ? *arotf : af_own;
  // a[g e f b]: columns (f, b) of the products with the double layer, b the
  // innermost output leg
  auto af = [&](int s, int c) { return afv[s * 4 + c]; };

  // enlarged corners Q_c(s)[(m f), (k b)], all corners of all sites in one
  // batched contraction per step
  std::vector<Var> Q(4 * ns);
  {
    std::vector<Var> Tl(4 * ns), Cc(4 * ns), Tc(4 * ns), ac(4 * ns);
    for (int c = 0; c < 4; ++c)
      for (int s = 0; s < ns; ++s) {
        Tl[c * ns + s] = T((c + 3) % 4, s);
        Cc[c * ns + s] = C(c, s);
        Tc[c * ns + s] = T(c, s);
        ac[c * ns + s] = af(s, c);
      }
    // X2 is written in the grouping the big contraction reads ([m k | g e]),
    // and Q in its cut-matrix layout, both from the GEMM epilogues; X2 (and
    // Y1 below) only ever enter products, which round them to FP32 in the
    // FP32 and BF16 arithmetics: they are stored in FP32 there
    std::vector<Var> X1 = tp.einsum_n("mgi,ij->mgj", Tl, Cc);
    std::vector<Var> X2 = tp.einsum_n("mgj,jek->mkge", X1, Tc, true);
    std::vector<Var> Qe = tp.einsum_n("mkge,gefb->mfkb", X2, ac);
    for (int i = 0; i < 4 * ns; ++i) Q[i] = tp.view(Qe[i], {n, n});
  }
  // projectors of every cut: cut index c*ns + p (plaquette p, cut c between
  // its corners c and c+1)
  std::vector<Var> Qa(nc), Qb(nc);
  for (int c = 0; c < 4; ++c)
    for (int p = 0; p < ns; ++p) {
      const int sa = L.shift(p, PLAQ_OFFSET[c][0], PLAQ_OFFSET[c][1]);
      const int sb = L.shift(p, PLAQ_OFFSET[(c + 1) % 4][0],
                             PLAQ_OFFSET[(c + 1) % 4][1]);
      Qa[c * ns + p] = Q[c * ns + sa];
      Qb[c * ns + p] = Q[((c + 1) % 4) * ns + sb];
    }
  auto proj = projector_op(tp, cx, Qa, Qb);
  const std::vector<Var>& P = proj.first;
  const std::vector<Var>& PtT = proj.second;

  // renormalised corners and edges, each contraction batched over all
  // corners of all sites
  VEnv out;
  out.C.resize(4 * ns);
  out.T.resize(4 * ns);
  const int m = 4 * ns;
  std::vector<Var> PtL(m), Qc(m), PR(m), Pt3(m), Tc(m), ac(m), P3(m);
  for (int c = 0; c < 4; ++c)
    for (int s = 0; s < ns; ++s) {
      const int i = c * ns + s;
      const int p = L.shift(s, -PLAQ_OFFSET[c][0], -PLAQ_OFFSET[c][1]);
      const int cutL = ((c + 3) % 4) * ns + p, cutR = c * ns + p;
      PtL[i] = PtT[cutL];
      Qc[i] = Q[i];
      PR[i] = P[cutR];
      const int pccw = L.shift(s, -PLAQ_OFFSET[(c + 1) % 4][0],
                               -PLAQ_OFFSET[(c + 1) % 4][1]);
      Pt3[i] = tp.view(PtT[c * ns + pccw], {chi, D2, chi});
      Tc[i] = T(c, s);
      ac[i] = af(s, c);
      P3[i] = tp.view(P[cutR], {chi, D2, chi});
    }
  std::vector<Var> Y = tp.einsum_n("rx,rq->xq", PtL, Qc);
  std::vector<Var> Cn = tp.einsum_n("xq,qy->xy", Y, PR);
  // intermediates written in the grouping of their consumers
  std::vector<Var> Y1 = tp.einsum_n("jgx,jek->xkge", Pt3, Tc, true);
  std::vector<Var> Y2 = tp.einsum_n("xkge,gefb->xfkb", Y1, ac);
  std::vector<Var> Tn = tp.einsum_n("xfkb,kby->xfy", Y2, P3);
  std::vector<Var> raw(Cn);
  raw.insert(raw.end(), Tn.begin(), Tn.end());
  std::vector<Var> nrm = tp.normalize_n(raw);
  for (int c = 0; c < 4; ++c)
    for (int s = 0; s < ns; ++s) {
      const int i = c * ns + s;
      out.C[c * ns + L.shift(s, CORNER_MOVE[c][0], CORNER_MOVE[c][1])] =
          nrm[i];
      out.T[c * ns + L.shift(s, EDGE_MOVE[c][0], EDGE_MOVE[c][1])] =
          nrm[m + i];
    }
  return out;
}

void ctm_step(Context& cx, const Env& in, Env& out) {
  Tape tp(cx.dev, false);
  VEnv v = ctm_step_ad(tp, cx, venv_leaves(tp, cx, in), arot_leaves(tp, cx));
  out = env_pack(cx, v);
}

// Singular values of every corner (two-pass tall-skinny SVD), sorted.
void corner_spectra(Context& cx, const Env& e, Tensor& S) {
  Device& dev = cx.dev;
  const int chi = cx.chi, nb = 4 * cx.nsite();
  const int b = chi + (chi % 2);
  Tensor W;
  if (b == chi) {
    W = e.C.view({nb, chi, chi});
  } else {
    W = dev.zeros({nb, chi, b});
    pad3(dev, e.C.ptr, W.ptr, nb, chi, chi, chi, b);
  }
  // Warm start: the singular values of W J are those of W for any
  // orthogonal J, and with J the right singular vectors of the previous
  // call's corners (which change little from one CTMRG iteration to the
  // next) the Gram matrices of the two Jacobi passes are nearly diagonal
  // already.  The rotation is the product of the calls' Jacobi rotations;
  // every 64 calls the solve starts cold, so that its rounding stays at
  // the level of a few products.
  const int64_t sW = (int64_t)chi * b, sJ = (int64_t)b * b;
  const bool warm = cx.spec_J.numel() == nb * sJ && cx.spec_J_age < 64;
  Tensor Wr = W;
  if (warm) {
    PrecScope f64(dev, PREC_FP64);
    Wr = dev.empty({nb, chi, b});
    gemm(dev, false, false, chi, b, b, 1.0, W.ptr, b, sW, cx.spec_J.ptr, b,
         sJ, 0.0, Wr.ptr, b, sW, nb);
  }
  Tensor U, J;
  svd_ts(dev, Wr, nb, chi, b, U, S, J, dev.cprec == PREC_FP64 ? 1e-15 : 1e-12);
  if (warm) {
    PrecScope f64(dev, PREC_FP64);
    Tensor Jn = dev.empty({nb, b, b});
    gemm(dev, false, false, b, b, b, 1.0, cx.spec_J.ptr, b, sJ, J.ptr, b, sJ,
         0.0, Jn.ptr, b, sJ, nb);
    cx.spec_J = Jn;
    ++cx.spec_J_age;
  } else {
    cx.spec_J = J;
    cx.spec_J_age = 0;
  }
}

int converge_env(Context& cx, double tol, int max_iter, int* n_iter,
                 double* delta) {
  int it = 0;
  double dl = INFINITY;
  const double svd_tol = cx.svd.tol;
  const bool injected = cx.env_injected;
  cx.env_injected = false;
  const long svd_bad0 = cx.stats.svd_unconverged;
  // the spectrum change cannot fall below the rounding of the contraction
  // arithmetic: tolerances under that floor are raised to it (with the
  // precision ladder, to the floor of the arithmetic of the last rung)
  const double tol_in = tol;
  auto eff_tol = [&]() {
    return tol_in > 0.0
               ? std::max(tol_in, prec_floors(cx.work_prec).spectra)
               : tol_in;
  };
  tol = eff_tol();
  // precision ladder: the BF16 rung ends when the spectrum change reaches
  // its floor or has not fallen below 0.9 of its smallest value for three
  // iterations; the iterations then continue in FP32
  double best = INFINITY;
  int flat = 0;
  // reduced-precision arithmetic: a state whose corner spectra hold values
  // near the rounding of the products (a small singular value kept at the
  // cut) leaves the change hovering above the floor, where more iterations
  // only redraw the rounding; once the change is within 100 times the floor
  // and has not set a new low (below 0.9 of the smallest) for 8 iterations
  // the iteration stops, reported as not converged
  double low = INFINITY;
  int stall = 0;
  struct RestoreTol {
    Context& c;
    double t;
    ~RestoreTol() { c.svd.tol = t; }
  } restore{cx, svd_tol};
  while (it < max_iter) {
    // the first projectors of an environment set from outside have no
    // subspace of an earlier iteration to start from: computed with FP32
    // products the subspace iteration levels off near its rounding floor
    // and the truncation moves the environment by ~1e-4 in the spectra,
    // which the next iterations then have to undo; that first iteration
    // runs in FP64
    PrecScope ps(cx.dev, it == 0 && injected ? (int)PREC_FP64 : cx.work_prec);
    // when iterating to a tolerance, the projector SVD of an iteration only
    // needs to be as accurate as the environment it produces: its tolerance
    // follows the last spectrum change (never looser than 1e-6, never
    // tighter than the configured one), so the final iterations and the
    // fixed point are computed at full accuracy; an environment set from
    // outside for these site tensors is taken to change by about the
    // tolerance, so its first projectors are as accurate as the last ones
    const double ref = it == 0 && injected ? tol : dl;
    if (tol > 0.0) cx.svd.tol = std::max(svd_tol, std::min(1e-6, 1e-2 * ref));
    Env next;
    ctm_step(cx, cx.env, next);
    cx.env = next;
    ++it;
    dl = corner_spectra_change(cx, cx.env);
    if (cx.ladder && cx.work_prec != PREC_FP32) {
      if (dl < 0.9 * best) {
        best = dl;
        flat = 0;
      } else {
        ++flat;
      }
      if (dl < prec_floors(cx.work_prec).spectra || flat >= 3) {
        cx.work_prec = PREC_FP32;
        tol = eff_tol();
        low = INFINITY;
        stall = 0;
        continue;
      }
    }
    if (tol > 0.0 && dl < tol) break;
    const double rounding = prec_floors(cx.work_prec).spectra;
    if (tol > 0.0 && rounding > 0.0) {
      if (dl < 0.9 * low) {
        low = dl;
        stall = 0;
      } else if (dl < 100.0 * rounding && ++stall >= 8) {
        break;
      }
    }
  }
  cx.converged_once = true;
  if (n_iter) *n_iter = it;
  if (delta) *delta = dl;
  if (tol > 0.0 && !(dl < tol)) return 1;
  // a projector SVD that stopped at svd_max_iter above its tolerance
  return cx.stats.svd_unconverged != svd_bad0 ? 1 : 0;
}

double corner_spectra_change(Context& cx, const Env& e) {
  Device& dev = cx.dev;
  const int chi = cx.chi, nb = 4 * cx.nsite();
  const int b = chi + (chi % 2);
  Tensor S;
  corner_spectra(cx, e, S);
  if (cx.spec_cur.numel() != (int64_t)nb * chi) {
    cx.spec_cur = dev.zeros({nb, chi});
    cx.spec_old = dev.zeros({nb, chi});
  }
  Tensor dl = dev.empty({1});
  spectra_update(dev, S.ptr, b, chi, nb, b, cx.spec_cur.ptr, cx.spec_old.ptr,
                 dl.ptr);
  double h = 0.0;
  dev.download(dl, &h);
  return h;
}

}  // namespace ipeps
