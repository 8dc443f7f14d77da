// Reverse-mode differentiation over the device contraction engine.
//
// A Var holds a device tensor and, once a cotangent flows into it, its
// gradient buffer.  A Tape records one backward closure per differentiable
// operation when recording is on; backward() runs them in reverse order.
// With recording off the same forward code runs without keeping anything.
#pragma once

#include <functional>
#include <memory>
#include <string>
#include <vector>

#include "engine.hpp"

namespace ipeps {

struct Node {
  Tensor v;
  Tensor g;          // empty until a cotangent arrives
  bool req = false;  // needs a gradient
};
using Var = std::shared_ptr<Node>;

class Tape {
 public:
  Tape(Device& d, bool record) : dev(d), rec(record) {}
  Device& dev;
  bool rec;

  Var leaf(const Tensor& t, bool req) {
    auto n = std::make_shared<Node>();
    n->v = t;
    n->req = req && rec;
    return n;
  }
  // gradient buffer of x (zero-initialised on first use)
  Tensor& grad(const Var& x);
  bool has_grad(const Var& x) const { return x->g.ptr != nullptr; }

  Var einsum(const std::string& spec, const Var& a, const Var& b);
  // the same contraction for items of one shape, batched in one GEMM launch
  // forwards and backwards; f32: the outputs kept in FP32 storage when the
  // products are FP32 or BF16 (for intermediates that only products read)
  std::vector<Var> einsum_n(const std::string& spec, const std::vector<Var>& a,
                            const std::vector<Var>& b, bool f32 = false);
  Var view(const Var& x, std::vector<int64_t> shape);
  // i-th sub-tensor along the leading dimension (shares memory)
  Var slice0(const Var& x, int64_t i);
  Var permute(const Var& x, const std::vector<int>& perm);
  // y = x / ||x||_F
  Var normalize(const Var& x);
  // the same for several tensors, in batched launches forwards and backwards
  std::vector<Var> normalize_n(const std::vector<Var>& xs);
  // x [a][b][c] placed at the start of each row block of a zero tensor of
  // shape `shape` read as [*][B][C] (B, C its last two extents after a 3-d
  // view): out[l][j][k] = x[l][j][k] for l < a, j < b, k < c
  Var pad3(const Var& x, int a, int b, int c, std::vector<int64_t> shape);

  // Q of the thin QR Y = Q R (n x b, diag R > 0) by Cholesky QR in two
  // passes (FP64); a column whose R diagonal is below 1e-6 of the column
  // scale |Y|_F / sqrt(b) is dropped (a zero column of Q)
  Var qr_q(const Var& Y);
  // eigenvectors (columns) of a symmetric b x b matrix (b even, <= 128):
  // the k of largest |lambda| first, then the others, each group in
  // descending signed order; the derivative uses x / (x^2 + eta^2),
  // eta = 1e-12 max|lambda|, for 1 / (lambda_j - lambda_i)
  Var eig_kept(const Var& B, int k);
  // y[r] = sum_s x[r][s][s] over the last two (equal) extents of x
  Var trace_dd(const Var& x);
  // y = X diag(s) for an n x b X and a constant device vector s
  Var colscale(const Var& X, const Tensor& s);
  // y = (x + P x) / 2 for a permutation P that is its own inverse
  Var sym_pair(const Var& x, const std::vector<int>& perm);

  void push(std::function<void()> f) {
    if (rec) ops_.push_back(std::move(f));
  }
  void backward();
  size_t size() const { return ops_.size(); }

 private:
  std::vector<std::function<void()>> ops_;
};

// x_bar += (y_bar - y <y, y_bar>) / n  with n = ||x|| (device scalar)
void normalize_backward(Device& dev, int64_t len, const double* y,
                        const double* ybar, const double* nrm, double* xbar);

}  // namespace ipeps
