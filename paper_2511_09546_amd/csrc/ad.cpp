// Reverse-mode tape over the device contraction engine.
#include <algorithm>

#include "ad.hpp"

namespace ipeps {

Tensor& Tape::grad(const Var& x) {
  if (!x->g.ptr) x->g = dev.zeros(x->v.shape);
  return x->g;
}

// Gradient of x as the target of a product: a first contribution is
// written (beta 0) into fresh memory instead of added to zeros, which saves
// the fill and the read of the zeros.
static Tensor& grad_target(Device& dev, Node* x, double& beta) {
  if (!x->g.ptr) {
    x->g = dev.empty(x->v.shape);
    beta = 0.0;
  } else {
    beta = 1.0;
  }
  return x->g;
}

static void parse3(const std::string& spec, std::string& a, std::string& b,
                   std::string& o) {
  const auto c = spec.find(','), ar = spec.find("->");
  a = spec.substr(0, c);
  b = spec.substr(c + 1, ar - c - 1);
  o = spec.substr(ar + 2);
}

// The two backward contractions of out = einsum(la, lb -> lo) read the
// incoming gradient with its labels grouped as [shared by la and lb | only
// in la | only in lb] (in lo's order within each group): the first reads it
// as [batch, free, contracted], the second as [batch, contracted, free].
// When lo interleaves the groups and both operands need their gradient, the
// gradient is permuted into that grouping once, instead of once by each
// contraction.  Returns lo when it is grouped already.
static std::string grad_grouping(const std::string& la, const std::string& lb,
                                 const std::string& lo) {
  std::string bt, ga, gb;
  for (char ch : lo) {
    const bool ia = la.find(ch) != std::string::npos;
    const bool ib = lb.find(ch) != std::string::npos;
    (ia && ib ? bt : (ia ? ga : gb)) += ch;
  }
  return bt + ga + gb;
}

static std::vector<int> label_perm(const std::string& from,
                                   const std::string& to) {
  std::vector<int> p;
  for (char ch : to) p.push_back((int)from.find(ch));
  return p;
}

Var Tape::einsum(const std::string& spec, const Var& a, const Var& b) {
  auto out = std::make_shared<Node>();
  out->v = ipeps::einsum(dev, spec, a->v, b->v);
  out->req = rec && (a->req || b->req);
  if (out->req) {
    std::string la, lb, lo;
    parse3(spec, la, lb, lo);
    push([this, a, b, out, la, lb, lo]() {
      if (!has_grad(out)) return;
      double beta;
      std::string lg = lo;
      Tensor g = out->g;
      if (a->req && b->req) {
        const std::string grp = grad_grouping(la, lb, lo);
        if (grp != lo) {
          g = permuted(dev, out->g, label_perm(lo, grp));
          lg = grp;
        }
      }
      if (a->req) {
        Tensor& ga = grad_target(dev, a.get(), beta);
        einsum_into(dev, lg + "," + lb + "->" + la, g, b->v, ga, 1.0, beta);
      }
      if (b->req) {
        Tensor& gb = grad_target(dev, b.get(), beta);
        einsum_into(dev, la + "," + lg + "->" + lb, a->v, g, gb, 1.0, beta);
      }
    });
  }
  return out;
}

// grad(target[i]) += einsum(spec, first[i], second[i]) for the listed
// items, in batched launches whose targets are distinct (an item whose
// target already occurs in the current launch goes to a later one); targets
// without a gradient yet are written (beta 0), the others accumulated
static void accumulate_n(Device& dev, const std::string& spec,
                         std::vector<Tensor> first, std::vector<Tensor> second,
                         std::vector<Node*> target) {
  while (!first.empty()) {
    std::vector<Tensor> f[2], s[2], t[2], f2, s2;
    std::vector<Node*> used, k2;
    for (size_t i = 0; i < first.size(); ++i) {
      bool dup = false;
      for (const Node* u : used) dup = dup || u == target[i];
      if (dup) {
        f2.push_back(first[i]);
        s2.push_back(second[i]);
        k2.push_back(target[i]);
      } else {
        double beta;
        Tensor& g = grad_target(dev, target[i], beta);
        const int j = beta != 0.0;
        f[j].push_back(first[i]);
        s[j].push_back(second[i]);
        t[j].push_back(g);
        used.push_back(target[i]);
      }
    }
    einsum_into_n(dev, spec, f[0], s[0], t[0], 1.0, 0.0);
    einsum_into_n(dev, spec, f[1], s[1], t[1], 1.0, 1.0);
    first.swap(f2);
    second.swap(s2);
    target.swap(k2);
  }
}

std::vector<Var> Tape::einsum_n(const std::string& spec,
                                const std::vector<Var>& a,
                                const std::vector<Var>& b, bool f32) {
  const size_t ni = a.size();
  std::vector<Tensor> av(ni), bv(ni);
  for (size_t i = 0; i < ni; ++i) {
    av[i] = a[i]->v;
    bv[i] = b[i]->v;
  }
  std::vector<Tensor> ov = ipeps::einsum_n(dev, spec, av, bv, f32);
  std::vector<Var> out(ni);
  bool any = false;
  for (size_t i = 0; i < ni; ++i) {
    out[i] = std::make_shared<Node>();
    out[i]->v = ov[i];
    out[i]->req = rec && (a[i]->req || b[i]->req);
    any = any || out[i]->req;
  }
  if (any) {
    std::string la, lb, lo;
    parse3(spec, la, lb, lo);
    push([this, a, b, out, la, lb, lo]() {
      // gradients grouped once when both sides need them (grad_grouping)
      const std::string grp = grad_grouping(la, lb, lo);
      bool both = grp != lo;
      for (size_t i = 0; i < out.size() && both; ++i)
        both = !has_grad(out[i]) || (a[i]->req && b[i]->req);
      const std::string lg = both ? grp : lo;
      std::vector<Tensor> g(out.size());
      for (size_t i = 0; i < out.size(); ++i)
        if (has_grad(out[i]))
          g[i] = both ? permuted(dev, out[i]->g, label_perm(lo, grp))
                      : out[i]->g;
      std::vector<Tensor> f, s;
      std::vector<Node*> k;
      for (size_t i = 0; i < out.size(); ++i)
        if (has_grad(out[i]) && a[i]->req) {
          f.push_back(g[i]);
          s.push_back(b[i]->v);
          k.push_back(a[i].get());
        }
      accumulate_n(dev, lg + "," + lb + "->" + la, f, s, k);
      f.clear();
      s.clear();
      k.clear();
      for (size_t i = 0; i < out.size(); ++i)
        if (has_grad(out[i]) && b[i]->req) {
          f.push_back(a[i]->v);
          s.push_back(g[i]);
          k.push_back(b[i].get());
        }
      accumulate_n(dev, la + "," + lg + "->" + lb, f, s, k);
    });
  }
  return out;
}

Var Tape::trace_dd(const Var& x) {
  const int r = x->v.rank();
  if (r < 2 || x->v.shape[r - 1] != x->v.shape[r - 2])
    throw ArgError("trace_dd: last two extents differ");
  const int d = (int)x->v.shape[r - 1];
  std::vector<int64_t> sh(x->v.shape.begin(), x->v.shape.end() - 2);
  if (sh.empty()) sh.push_back(1);
  auto out = std::make_shared<Node>();
  out->v = dev.empty(sh);
  const int64_t rows = out->v.numel();
  ipeps::trace_dd(dev, x->v.ptr, rows, d, out->v.ptr);
  out->req = rec && x->req;
  if (out->req)
    push([this, x, out, rows, d]() {
      if (!has_grad(out)) return;
      double beta;
      Tensor& gx = grad_target(dev, x.get(), beta);
      trace_dd_backward(dev, out->g.ptr, rows, d, gx.ptr, beta);
    });
  return out;
}

Var Tape::view(const Var& x, std::vector<int64_t> shape) {
  auto out = std::make_shared<Node>();
  out->v = x->v.view(std::move(shape));
  out->req = x->req;
  if (out->req)
    push([this, x, out]() {
      if (!has_grad(out)) return;
      Tensor& gx = grad(x);
      axpby(dev, gx.numel(), 1.0, out->g.ptr, 1.0, gx.ptr);
    });
  return out;
}

Var Tape::slice0(const Var& x, int64_t i) {
  auto out = std::make_shared<Node>();
  out->v = x->v.slice0(i);
  out->req = x->req;
  if (out->req) {
    const int64_t off = out->v.ptr - x->v.ptr;
    push([this, x, out, off]() {
      if (!has_grad(out)) return;
      Tensor& gx = grad(x);
      axpby(dev, out->v.numel(), 1.0, out->g.ptr, 1.0, gx.ptr + off);
    });
  }
  return out;
}

Var Tape::pad3(const Var& x, int a, int b, int c,
               std::vector<int64_t> shape) {
  auto out = std::make_shared<Node>();
  out->v = dev.zeros(shape);
  const int64_t tot = out->v.numel();
  const int C = (int)shape.back();
  const int B = (int)(shape.size() >= 2 ? shape[shape.size() - 2] : 1);
  if ((int64_t)a * B * C > tot || b > B || c > C ||
      x->v.numel() != (int64_t)a * b * c)
    throw ArgError("pad3: shapes do not fit");
  ipeps::pad3(dev, x->v.ptr, out->v.ptr, a, b, c, B, C);
  out->req = x->req;
  if (out->req) {
    push([this, x, out, a, b, c, B, C]() {
      if (!has_grad(out)) return;
      crop3_add(dev, out->g.ptr, grad(x).ptr, a, b, c, B, C);
    });
  }
  return out;
}

Var Tape::permute(const Var& x, const std::vector<int>& perm) {
  auto out = std::make_shared<Node>();
  out->v = permuted(dev, x->v, perm);
  out->req = x->req;
  if (out->req) {
    std::vector<int> inv(perm.size());
    for (size_t i = 0; i < perm.size(); ++i) inv[perm[i]] = (int)i;
    push([this, x, out, inv]() {
      if (!has_grad(out)) return;
      ipeps::permute(dev, out->g, inv, grad(x), 1.0, 1.0);
    });
  }
  return out;
}

Var Tape::normalize(const Var& x) {
  auto out = std::make_shared<Node>();
  const int64_t len = x->v.numel();
  Tensor nrm = dev.empty({1});
  nrm2(dev, x->v.ptr, len, nrm.ptr);
  out->v = dev.empty(x->v.shape);
  axpby(dev, len, 1.0, x->v.ptr, 0.0, out->v.ptr);
  scale_dev(dev, out->v.ptr, len, nrm.ptr, true);
  out->req = rec && x->req;
  if (out->req)
    push([this, x, out, nrm, len]() {
      if (!has_grad(out)) return;
      normalize_backward(dev, len, out->v.ptr, out->g.ptr, nrm.ptr,
                         grad(x).ptr);
    });
  return out;
}

std::vector<Var> Tape::normalize_n(const std::vector<Var>& xs) {
  std::vector<Var> out(xs.size());
  for (size_t b0 = 0; b0 < xs.size(); b0 += NB_MAX) {
    const int cnt = (int)std::min<size_t>(NB_MAX, xs.size() - b0);
    Tensor nrm = dev.empty({cnt});
    NormBatch p{};
    bool any = false;
    std::vector<Var> xi(cnt), yi(cnt);
    for (int k = 0; k < cnt; ++k) {
      const Var& x = xs[b0 + k];
      auto o = std::make_shared<Node>();
      o->v = dev.empty(x->v.shape);
      o->req = rec && x->req;
      any = any || o->req;
      p.a[k] = x->v.ptr;
      p.out[k] = o->v.ptr;
      p.n[k] = (long)x->v.numel();
      xi[k] = x;
      yi[k] = o;
      out[b0 + k] = o;
    }
    normalize_batch(dev, p, cnt, nrm.ptr);
    if (any)
      push([this, xi, yi, nrm, cnt]() {
        NormBatch q{};
        int m = 0;
        for (int k = 0; k < cnt; ++k)
          if (has_grad(yi[k]) && xi[k]->req) {
            q.a[m] = yi[k]->v.ptr;
            q.b[m] = yi[k]->g.ptr;
            q.out[m] = grad(xi[k]).ptr;
            q.nrm[m] = nrm.ptr + k;
            q.n[m] = (long)yi[k]->v.numel();
            ++m;
          }
        // distinct inputs only in one launch (each accumulates into its
        // own gradient)
        for (int k = 1; k < m; ++k)
          for (int j = 0; j < k; ++j)
            if (q.out[j] == q.out[k])
              throw ArgError("normalize_n: an input occurs twice");
        normalize_backward_batch(dev, q, m);
      });
  }
  return out;
}

void Tape::backward() {
  for (auto it = ops_.rbegin(); it != ops_.rend(); ++it) (*it)();
  ops_.clear();
}

}  // namespace ipeps
