// CTMRG on the device: double layer, trace-boundary start, one simultaneous
// four-corner iteration with half-system SVD projectors, normalisation and
// the corner-spectrum convergence measure (Sec. III A: the environment of the
// energy network, Eq. (7)).
#include <algorithm>
#include <cmath>

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

static Tensor site_tensor(const Context& cx, const Tensor& A, int s) {
  Tensor t = A;
  const int64_t sz = (int64_t)cx.d * cx.D * cx.D * cx.D * cx.D;
  t.ptr = A.ptr + s * sz;
  t.shape = {cx.d, cx.D, cx.D, cx.D, cx.D};
  return t;
}

// a = sum_p A[p,l,u,r,d] A[p,l',u',r',d'], legs fused (k k') -> k*D + k',
// stored in the four clockwise rotations a_c.
void build_double_layer(Context& cx) {
  const int ns = cx.nsite(), D2 = cx.D2, D = cx.D;
  const int64_t a4 = (int64_t)D2 * D2 * D2 * D2;
  if (cx.a_rot.numel() != ns * 4 * a4) cx.a_rot = cx.dev.empty({ns, 4, D2, D2, D2, D2});
  for (int s = 0; s < ns; ++s) {
    Tensor As = site_tensor(cx, cx.A, s);
    Tensor a8 = einsum(cx.dev, "pabce,pfghi->afbgchei", As, As);
    Tensor a = a8.view({D2, D2, D2, D2});
    (void)D;
    for (int c = 0; c < 4; ++c) {
      Tensor dst = cx.av(s, c);
      permute(cx.dev, a, {c % 4, (c + 1) % 4, (c + 2) % 4, (c + 3) % 4}, dst);
    }
  }
}

static Tensor trace_vector(Context& cx) {
  std::vector<double> h((size_t)cx.D2, 0.0);
  for (int k = 0; k < cx.D; ++k) h[(size_t)k * cx.D + k] = 1.0;
  Tensor e = cx.dev.empty({cx.D2});
  cx.dev.upload(e, h.data());
  return e;
}

// Trace-boundary start: corners and edges are double layers whose outward
// legs are closed with delta_{k k'}; bond dimension D^2 zero padded to chi.
void init_env(Context& cx) {
  const int ns = cx.nsite(), chi = cx.chi, D2 = cx.D2;
  Env e;
  e.C = cx.dev.zeros({4, ns, chi, chi});
  e.T = cx.dev.zeros({4, ns, chi, D2, chi});
  Tensor tv = trace_vector(cx);
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

void ctm_step(Context& cx, const Env& in, Env& out, StepTape* tape) {
  Device& dev = cx.dev;
  const int ns = cx.nsite(), chi = cx.chi, D2 = cx.D2, nc = cx.ncut();
  const int64_t n = cx.n, nn = n * n;
  const Lattice& L = cx.lat;

  // enlarged corners Q_c(s)[(m f), (k b)]
  Tensor Q = dev.empty({4, ns, n, n});
  for (int c = 0; c < 4; ++c)
    for (int s = 0; s < ns; ++s) {
      Tensor X1 = einsum(dev, "mgi,ij->mgj", cx.Tv(in, (c + 3) % 4, s),
                         cx.Cv(in, c, s));
      Tensor X2 = einsum(dev, "mgj,jek->mgek", X1, cx.Tv(in, c, s));
      Tensor Qcs = Q;
      Qcs.ptr = Q.ptr + ((int64_t)c * ns + s) * nn;
      Qcs.shape = {chi, D2, chi, D2};
      einsum_into(dev, "mgek,gebf->mfkb", X2, cx.av(s, c), Qcs);
    }
  auto Qp = [&](int c, int s) { return Q.ptr + ((int64_t)c * ns + s) * nn; };

  // projectors of every cut: cut index c*ns + p (plaquette p, cut c between
  // its corners c and c+1)
  CutBatch cb;
  cb.ncut = nc;
  cb.n = n;
  cb.b = cx.b;
  cb.chi = chi;
  cb.Qa.resize(nc);
  cb.Qb.resize(nc);
  for (int c = 0; c < 4; ++c)
    for (int p = 0; p < ns; ++p) {
      const int sa = L.shift(p, PLAQ_OFFSET[c][0], PLAQ_OFFSET[c][1]);
      const int sb = L.shift(p, PLAQ_OFFSET[(c + 1) % 4][0],
                             PLAQ_OFFSET[(c + 1) % 4][1]);
      cb.Qa[c * ns + p] = Qp(c, sa);
      cb.Qb[c * ns + p] = Qp((c + 1) % 4, sb);
    }
  Tensor U, S, V, keep;
  projector_svd(dev, cb, cx.Xwarm, cx.have_warm, U, S, V, keep, cx.svd,
                &cx.stats);
  cx.have_warm = true;
  const int b = cx.b;
  const int64_t sUV = n * b;
  // P = Qb V_k S_k^-1/2 and Pt^T = Qa^T U_k S_k^-1/2, zero beyond k
  Tensor P = dev.empty({nc, n, chi});
  Tensor PtT = dev.empty({nc, n, chi});
  for (int i = 0; i < nc; ++i) {
    gemm(dev, false, false, n, chi, n, 1.0, cb.Qb[i], n, 0, V.ptr + i * sUV,
         b, 0, 0.0, P.ptr + i * n * chi, chi, 0);
    gemm(dev, true, false, n, chi, n, 1.0, cb.Qa[i], n, 0, U.ptr + i * sUV, b,
         0, 0.0, PtT.ptr + i * n * chi, chi, 0);
  }
  col_scale(dev, P.ptr, n, chi, S.ptr, 1, (const int*)keep.ptr, nc, n * chi,
            b);
  col_scale(dev, PtT.ptr, n, chi, S.ptr, 1, (const int*)keep.ptr, nc,
            n * chi, b);
  auto Pv = [&](const Tensor& T, int cut) {
    Tensor t = T;
    t.ptr = T.ptr + (int64_t)cut * n * chi;
    t.shape = {n, chi};
    return t;
  };

  Env raw;
  raw.C = dev.empty({4, ns, chi, chi});
  raw.T = dev.empty({4, ns, chi, D2, chi});
  for (int c = 0; c < 4; ++c)
    for (int s = 0; s < ns; ++s) {
      const int p = L.shift(s, -PLAQ_OFFSET[c][0], -PLAQ_OFFSET[c][1]);
      const int cutL = ((c + 3) % 4) * ns + p, cutR = c * ns + p;
      Tensor Qcs = Q;
      Qcs.ptr = Qp(c, s);
      Qcs.shape = {n, n};
      Tensor Y = einsum(dev, "rx,rq->xq", Pv(PtT, cutL), Qcs);
      Tensor Cd = cx.Cv(raw, c, L.shift(s, CORNER_MOVE[c][0],
                                        CORNER_MOVE[c][1]));
      einsum_into(dev, "xq,qy->xy", Y, Pv(P, cutR), Cd);
      const int pccw = L.shift(s, -PLAQ_OFFSET[(c + 1) % 4][0],
                               -PLAQ_OFFSET[(c + 1) % 4][1]);
      Tensor Pt3 = Pv(PtT, c * ns + pccw).view({chi, D2, chi});
      Tensor Y1 = einsum(dev, "jgx,jek->xgek", Pt3, cx.Tv(in, c, s));
      Tensor Y2 = einsum(dev, "xgek,gebf->xkbf", Y1, cx.av(s, c));
      Tensor P3 = Pv(P, cutR).view({chi, D2, chi});
      Tensor Td = cx.Tv(raw, c, L.shift(s, EDGE_MOVE[c][0], EDGE_MOVE[c][1]));
      einsum_into(dev, "xkbf,kby->xfy", Y2, P3, Td);
    }
  // normalise every tensor by its Frobenius norm
  Tensor norms = dev.empty({2, 4 * ns});
  out.C = dev.empty({4, ns, chi, chi});
  out.T = dev.empty({4, ns, chi, D2, chi});
  const int64_t cs = (int64_t)chi * chi, ts = (int64_t)chi * D2 * chi;
  for (int i = 0; i < 4 * ns; ++i) {
    nrm2(dev, raw.C.ptr + i * cs, cs, norms.ptr + i);
    nrm2(dev, raw.T.ptr + i * ts, ts, norms.ptr + 4 * ns + i);
  }
  axpby(dev, raw.C.numel(), 1.0, raw.C.ptr, 0.0, out.C.ptr);
  axpby(dev, raw.T.numel(), 1.0, raw.T.ptr, 0.0, out.T.ptr);
  for (int i = 0; i < 4 * ns; ++i) {
    scale_dev(dev, out.C.ptr + i * cs, cs, norms.ptr + i, true);
    scale_dev(dev, out.T.ptr + i * ts, ts, norms.ptr + 4 * ns + i, true);
  }
  if (tape) {
    tape->in = in;
    tape->Q = Q;
    tape->U = U;
    tape->S = S;
    tape->V = V;
    tape->keep = keep;
    tape->P = P;
    tape->PtT = PtT;
    tape->Craw = raw.C;
    tape->Traw = raw.T;
    tape->Cnorm = norms;
  }
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
  Tensor U, J;
  svd_ts(dev, W, nb, chi, b, U, S, J);
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
