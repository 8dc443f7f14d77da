// Device memory pool, tensor views, and the pairwise contraction planner.
#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <limits>
#include <mutex>

#include "engine.hpp"

namespace ipeps {

// ------------------------------------------------------------------- Pool
static size_t round_bytes(size_t b) {
  const size_t g = 256;
  b = (b + g - 1) / g * g;
  if (b > (1u << 20)) {
    // coarser rounding for large blocks so that nearby sizes share blocks
    const size_t g2 = 1u << 16;
    b = (b + g2 - 1) / g2 * g2;
  }
  return b;
}

// Blocks of destroyed contexts, kept for later contexts of the process (a
// context is destroyed only after its stream has drained, so its blocks are
// idle).  Trimmed when hipMalloc runs out of memory.
namespace {
std::mutex g_idle_mu;
std::multimap<size_t, void*> g_idle;

bool take_idle(size_t bytes, void** p, size_t* got) {
  std::lock_guard<std::mutex> lock(g_idle_mu);
  auto it = g_idle.lower_bound(bytes);
  if (it == g_idle.end() || it->first > bytes + bytes / 8) return false;
  *p = it->second;
  *got = it->first;
  g_idle.erase(it);
  return true;
}

void trim_idle() {
  std::lock_guard<std::mutex> lock(g_idle_mu);
  for (auto& kv : g_idle) (void)hipFree(kv.second);
  g_idle.clear();
}
}  // namespace

size_t trim_idle_to(size_t keep_bytes) {
  std::lock_guard<std::mutex> lock(g_idle_mu);
  size_t total = 0;
  for (const auto& kv : g_idle) total += kv.first;
  // the largest blocks first
  while (total > keep_bytes && !g_idle.empty()) {
    auto it = std::prev(g_idle.end());
    IPEPS_HIP(hipFree(it->second));
    total -= it->first;
    g_idle.erase(it);
  }
  return total;
}

void Pool::begin_arena(void* base, size_t bytes) {
  arena_ = (char*)base;
  arena_size_ = bytes;
  arena_top_ = 0;
  arena_peak_ = 0;
  arena_lo_ = arena_;
  arena_hi_ = arena_ + bytes;
  arena_free_.clear();
}

void Pool::end_arena() {
  arena_ = nullptr;
  arena_free_.clear();
}

void* Pool::alloc(size_t bytes, size_t* got) {
  bytes = round_bytes(std::max<size_t>(bytes, 8));
  if (arena_) {
    auto it = arena_free_.lower_bound(bytes);
    if (it != arena_free_.end() && it->first <= bytes + bytes / 8) {
      void* p = it->second;
      *got = it->first;
      arena_free_.erase(it);
      return p;
    }
    if (bytes > arena_size_ - arena_top_)
      throw OomError("scratch area of " + std::to_string(arena_size_) +
                     " bytes exhausted");
    void* p = arena_ + arena_top_;
    arena_top_ += bytes;
    arena_peak_ = std::max(arena_peak_, arena_top_);
    *got = bytes;
    return p;
  }
  if (bytes > limit_ || live_ > limit_ - bytes)
    throw OomError("context memory budget of " + std::to_string(limit_) +
                   " bytes exceeded");
  auto it = free_.lower_bound(bytes);
  if (it != free_.end() && it->first <= bytes + bytes / 8) {
    void* p = it->second;
    *got = it->first;
    free_.erase(it);
    live_ += *got;
    peak_live_ = std::max(peak_live_, live_);
    return p;
  }
  void* p = nullptr;
  size_t size = bytes;
  if (!take_idle(bytes, &p, &size)) {
    hipError_t e = hipMalloc(&p, bytes);
    if (e != hipSuccess) {
      (void)hipGetLastError();
      // return cached blocks (this context's and the idle ones) to HIP and
      // retry once
      trim_idle();
      for (auto& kv : free_) {
        (void)hipFree(kv.second);
        for (auto a = all_.begin(); a != all_.end(); ++a)
          if (a->first == kv.second) {
            reserved_ -= a->second;
            all_.erase(a);
            break;
          }
      }
      free_.clear();
      e = hipMalloc(&p, bytes);
      if (e != hipSuccess) {
        (void)hipGetLastError();
        throw OomError("hipMalloc of " + std::to_string(bytes) + " bytes");
      }
    }
  }
  all_.emplace_back(p, size);
  reserved_ += size;
  *got = size;
  live_ += size;
  peak_live_ = std::max(peak_live_, live_);
  return p;
}

void Pool::release(void* p, size_t block_bytes) {
  const char* c = (const char*)p;
  if (arena_lo_ && c >= arena_lo_ && c < arena_hi_) {
    // a block of the scratch region: back to the arena while it is active,
    // dropped otherwise (never to HIP or the cached blocks)
    if (arena_) arena_free_.emplace(block_bytes, p);
    return;
  }
  live_ -= block_bytes;
  if (hold_) {
    held_.emplace_back(p, block_bytes);
    held_bytes_ += block_bytes;
  } else
    free_.emplace(block_bytes, p);
}

std::vector<std::pair<void*, size_t>> Pool::take_held() {
  std::vector<std::pair<void*, size_t>> r;
  r.swap(held_);
  held_bytes_ = 0;
  return r;
}

Pool::~Pool() {
  std::lock_guard<std::mutex> lock(g_idle_mu);
  for (auto& a : all_) g_idle.emplace(a.second, a.first);
}

// ----------------------------------------------------------------- Tensor
Tensor Tensor::view(std::vector<int64_t> s) const {
  Tensor t = *this;
  t.shape = std::move(s);
  if (t.numel() != numel()) throw ArgError("view: numel mismatch");
  return t;
}

Tensor Tensor::slice0(int64_t i) const {
  Tensor t = *this;
  t.shape.erase(t.shape.begin());
  t.ptr = f32 ? (double*)((float*)ptr + i * t.numel()) : ptr + i * t.numel();
  return t;
}

// --------------------------------------------------------------- Profiler
hipEvent_t Profiler::get() {
  if (!pool.empty()) {
    hipEvent_t e = pool.back();
    pool.pop_back();
    return e;
  }
  hipEvent_t e;
  IPEPS_HIP(hipEventCreate(&e));
  return e;
}

void Profiler::begin(hipStream_t s, int fam, double flop, double bytes,
                     bool wide) {
  Rec r{fam, get(), get(), flop, bytes, net, wide};
  IPEPS_HIP(hipEventRecord(r.a, s));
  recs.push_back(r);
}

void Profiler::end(hipStream_t s) { IPEPS_HIP(hipEventRecord(recs.back().b, s)); }

void Profiler::read(int fam, long* n, double* sec, double* flop,
                    double* bytes) {
  long cnt = 0;
  double t = 0.0, f = 0.0, by = 0.0;
  for (auto& r : recs) {
    const bool gemm =
        r.fam == PROF_GEMM || r.fam == PROF_GEMM32 || r.fam == PROF_GEMM16;
    if (fam == PROF_NET ? !(r.net && gemm)
                        : (fam == PROF_WIDE ? !r.wide : r.fam != fam))
      continue;
    IPEPS_HIP(hipEventSynchronize(r.b));
    float ms = 0.f;
    IPEPS_HIP(hipEventElapsedTime(&ms, r.a, r.b));
    ++cnt;
    t += ms * 1e-3;
    f += r.flop;
    by += r.bytes;
  }
  *n = cnt;
  *sec = t;
  *flop = f;
  *bytes = by;
}

void Profiler::clear() {
  for (auto& r : recs) {
    pool.push_back(r.a);
    pool.push_back(r.b);
  }
  recs.clear();
}

void Profiler::reserve(size_t n) {
  while (pool.size() < n) {
    hipEvent_t e;
    IPEPS_HIP(hipEventCreate(&e));
    pool.push_back(e);
  }
}

Profiler::~Profiler() {
  clear();
  for (auto e : pool) (void)hipEventDestroy(e);
}

// ----------------------------------------------------------------- Device
int memcheck_mode() {
  const char* v = std::getenv("IPEPS_MEMCHECK");
  return v ? std::atoi(v) : 0;
}

Tensor Device::empty(std::vector<int64_t> shape) {
  Tensor t;
  t.shape = std::move(shape);
  const size_t bytes = (size_t)std::max<int64_t>(t.numel(), 1) * 8;
  auto b = std::make_shared<Buffer>();
  size_t got = 0;
  if (memcheck > 0 && !pool.in_arena()) {
    // guard bands on both sides (pattern 0xa5), the tensor in between
    const size_t G = MEMCHECK_GUARD;
    pool.hold_released(true);
    if (pool.held_bytes() >= MEMCHECK_HOLD)
      memcheck_pending += memcheck_verify();
    b->p = pool.alloc(bytes + 2 * G, &got);
    b->bytes = got;
    b->pool = &pool;
    char* raw = (char*)b->p;
    IPEPS_HIP(hipMemsetAsync(raw, 0xa5, G, stream));
    IPEPS_HIP(hipMemsetAsync(raw + G + bytes, 0xa5, got - G - bytes, stream));
    if (memcheck >= 2) IPEPS_HIP(hipMemsetAsync(raw + G, 0xff, bytes, stream));
    guarded[raw] = {bytes, got};
    t.buf = b;
    t.ptr = (double*)(raw + G);
    return t;
  }
  b->p = pool.alloc(bytes, &got);
  b->bytes = got;
  b->pool = &pool;
  t.buf = b;
  t.ptr = (double*)b->p;
  return t;
}

long Device::memcheck_verify() {
  if (memcheck <= 0) return 0;
  IPEPS_HIP(hipStreamSynchronize(stream));
  const size_t G = MEMCHECK_GUARD;
  long bad = 0;
  std::vector<unsigned char> h;
  for (const auto& kv : guarded) {
    const char* raw = (const char*)kv.first;
    const size_t user = kv.second.first, block = kv.second.second;
    for (int tail = 0; tail < 2; ++tail) {
      const size_t n = tail ? block - G - user : G;
      h.resize(n);
      IPEPS_HIP(hipMemcpy(h.data(), tail ? raw + G + user : raw, n,
                          hipMemcpyDeviceToHost));
      size_t first = n, last = 0, cnt = 0;
      for (size_t i = 0; i < n; ++i)
        if (h[i] != 0xa5) {
          if (first == n) first = i;
          last = i;
          ++cnt;
        }
      if (!cnt) continue;
      ++bad;
      std::fprintf(stderr,
                   "memcheck: tensor of %zu bytes at %p: %zu bytes changed "
                   "%s it, the nearest %zu bytes away\n",
                   user, (const void*)(raw + G), cnt,
                   tail ? "after" : "before", tail ? first : G - 1 - last);
    }
  }
  // the held blocks are verified: reusable again
  for (const auto& hb : pool.take_held()) {
    guarded.erase(hb.first);
    pool.reissue(hb.first, hb.second);
  }
  return bad;
}

Tensor Device::empty_f32(std::vector<int64_t> shape) {
  int64_t n = 1;
  for (auto s : shape) n *= s;
  Tensor t = empty({(n + 1) / 2});
  t.shape = std::move(shape);
  t.f32 = true;
  return t;
}

Tensor Device::zeros(std::vector<int64_t> shape) {
  Tensor t = empty(std::move(shape));
  fill(*this, t.ptr, t.numel(), 0.0);
  return t;
}

Tensor Device::scalar_buffer(int n) { return empty({n}); }

void Device::upload(Tensor& t, const double* host) {
  IPEPS_HIP(hipMemcpyAsync(t.ptr, host, t.numel() * 8, hipMemcpyHostToDevice,
                           stream));
}

void Device::download(const Tensor& t, double* host) {
  IPEPS_HIP(hipMemcpyAsync(host, t.ptr, t.numel() * 8, hipMemcpyDeviceToHost,
                           stream));
  IPEPS_HIP(hipStreamSynchronize(stream));
}

void Device::sync() { IPEPS_HIP(hipStreamSynchronize(stream)); }

void prime_gemm_attributes();    // gemm.hip
void prime_kernel_attributes();  // kernels.hip

void prime_attributes() {
  static std::once_flag once;
  std::call_once(once, []() {
    prime_gemm_attributes();
    prime_kernel_attributes();
  });
}

// ---------------------------------------------------------------- einsum
namespace {

struct Spec {
  std::string a, b, o;
};

Spec parse(const std::string& spec) {
  Spec s;
  auto c = spec.find(',');
  auto ar = spec.find("->");
  if (c == std::string::npos || ar == std::string::npos || ar < c)
    throw ArgError("einsum: bad spec " + spec);
  s.a = spec.substr(0, c);
  s.b = spec.substr(c + 1, ar - c - 1);
  s.o = spec.substr(ar + 2);
  return s;
}

bool has(const std::string& s, char ch) {
  return s.find(ch) != std::string::npos;
}

std::vector<int> perm_of(const std::string& from, const std::string& to) {
  std::vector<int> p;
  for (char ch : to) p.push_back((int)from.find(ch));
  return p;
}

bool is_identity(const std::vector<int>& p) {
  for (size_t i = 0; i < p.size(); ++i)
    if (p[i] != (int)i) return false;
  return true;
}

// A candidate layout of the two GEMM operands and the output.
struct Plan {
  bool swap = false;       // first operand is B
  std::string first, second, out;  // label orders actually used
  bool tA = false, tB = false;
  bool perm_first = false, perm_second = false, perm_out = false;
  bool scatter = false;    // the GEMM writes the output layout directly
  int64_t cost = std::numeric_limits<int64_t>::max();
};

// Mixed-radix digits (least significant first) of an index that enumerates
// the labels `ls` row-major, each digit's stride that of its label in the
// row-major tensor with labels `o` and shape `shape`; adjacent digits that
// are contiguous in the output are merged.  False when more than
// CMAP_DIGITS digits remain.
bool cmap_digits(const std::string& ls, const std::string& o,
                 const std::vector<int64_t>& shape, int& n, int* ext,
                 int64_t* str) {
  std::vector<int64_t> e, st;
  for (int i = (int)ls.size() - 1; i >= 0; --i) {
    const size_t pos = o.find(ls[i]);
    int64_t stride = 1;
    for (size_t j = pos + 1; j < o.size(); ++j) stride *= shape[j];
    const int64_t ex = shape[pos];
    if (!e.empty() && st.back() * e.back() == stride) {
      e.back() *= ex;
    } else {
      e.push_back(ex);
      st.push_back(stride);
    }
  }
  if (e.empty()) {  // no label: a single index 0
    e.push_back(1);
    st.push_back(0);
  }
  if ((int)e.size() > CMAP_DIGITS) return false;
  n = (int)e.size();
  for (int i = 0; i < n; ++i) {
    ext[i] = (int)e[i];
    str[i] = st[i];
  }
  return true;
}

}  // namespace

static int64_t dim_of(char ch, const std::string& la, const Tensor& A,
                      const std::string& lb, const Tensor& B) {
  auto i = la.find(ch);
  if (i != std::string::npos) return A.shape[i];
  return B.shape[lb.find(ch)];
}

void einsum_into_n(Device& dev, const std::string& spec,
                   const std::vector<Tensor>& As,
                   const std::vector<Tensor>& Bs,
                   const std::vector<Tensor>& outs, double alpha,
                   double beta) {
  const size_t ni = As.size();
  if (ni == 0) return;
  if (Bs.size() != ni || outs.size() != ni)
    throw ArgError("einsum: operand counts differ in " + spec);
  for (size_t i = 1; i < ni; ++i)
    if (As[i].f32 != As[0].f32 || Bs[i].f32 != Bs[0].f32 ||
        outs[i].f32 != outs[0].f32)
      throw ArgError("einsum: batched items differ in storage in " + spec);
  // FP32-stored tensors take part directly only as operands of FP32 or
  // BF16 products: with FP64 products they are widened first, and an FP32
  // output is computed in FP64 and rounded
  if (dev.cprec == PREC_FP64 && (As[0].f32 || Bs[0].f32 || outs[0].f32)) {
    auto widen = [&](const std::vector<Tensor>& v) {
      std::vector<Tensor> r(v.size());
      for (size_t i = 0; i < v.size(); ++i) {
        if (!v[i].f32) {
          r[i] = v[i];
          continue;
        }
        r[i] = dev.empty(v[i].shape);
        to_f64(dev, (const float*)v[i].ptr, r[i].ptr, v[i].numel());
      }
      return r;
    };
    std::vector<Tensor> ow = outs;
    if (outs[0].f32) {
      if (beta != 0.0) {
        ow = widen(outs);
      } else {
        for (auto& o : ow) o = dev.empty(o.shape);
      }
    }
    einsum_into_n(dev, spec, widen(As), widen(Bs), ow, alpha, beta);
    if (outs[0].f32)
      for (size_t i = 0; i < ni; ++i)
        to_f32(dev, ow[i].ptr, (float*)outs[i].ptr, outs[i].numel());
    return;
  }
  NetScope net(dev.prof);
  for (size_t i = 1; i < ni; ++i)
    if (As[i].shape != As[0].shape || Bs[i].shape != Bs[0].shape ||
        outs[i].shape != outs[0].shape)
      throw ArgError("einsum: batched items differ in shape in " + spec);
  const Tensor& A = As[0];
  const Tensor& B = Bs[0];
  const Tensor& out = outs[0];
  Spec s = parse(spec);
  if ((int)s.a.size() != A.rank() || (int)s.b.size() != B.rank() ||
      (int)s.o.size() != out.rank())
    throw ArgError("einsum: rank mismatch in " + spec);
  for (size_t i = 0; i < s.a.size(); ++i)
    if (has(s.b, s.a[i]) && B.shape[s.b.find(s.a[i])] != A.shape[i])
      throw ArgError("einsum: dim mismatch in " + spec);
  for (size_t i = 0; i < s.o.size(); ++i)
    if (dim_of(s.o[i], s.a, A, s.b, B) != out.shape[i])
      throw ArgError("einsum: output dim mismatch in " + spec);
  for (char ch : s.a)
    if (!has(s.b, ch) && !has(s.o, ch))
      throw ArgError("einsum: summed free label unsupported in " + spec);
  for (char ch : s.b)
    if (!has(s.a, ch) && !has(s.o, ch))
      throw ArgError("einsum: summed free label unsupported in " + spec);

  // label classes
  std::string batch, contr_a, contr_b, free_a_o, free_b_o;
  for (char ch : s.o)
    if (has(s.a, ch) && has(s.b, ch)) batch += ch;
  for (char ch : s.a)
    if (has(s.b, ch) && !has(s.o, ch)) contr_a += ch;
  for (char ch : s.b)
    if (has(s.a, ch) && !has(s.o, ch)) contr_b += ch;
  for (char ch : s.o)
    if (has(s.a, ch) && !has(s.b, ch)) free_a_o += ch;
  for (char ch : s.o)
    if (has(s.b, ch) && !has(s.a, ch)) free_b_o += ch;
  auto own_order = [](const std::string& src, const std::string& sel) {
    std::string r;
    for (char ch : src)
      if (has(sel, ch)) r += ch;
    return r;
  };
  const std::string free_a_own = own_order(s.a, free_a_o);
  const std::string free_b_own = own_order(s.b, free_b_o);

  int64_t nA = A.numel(), nB = B.numel(), nO = out.numel();
  int64_t nbatch_all = 1;
  for (char ch : batch) nbatch_all *= dim_of(ch, s.a, A, s.b, B);
  // a scattered output needs the batch labels next to each other in the
  // output (one batch stride)
  bool batch_adjacent = true;
  if (!batch.empty()) {
    const size_t p0 = s.o.find(batch[0]);
    batch_adjacent = s.o.compare(p0, batch.size(), batch) == 0;
  }
  Plan best;
  for (int swap = 0; swap < 2; ++swap) {
    const std::string& L1 = swap ? s.b : s.a;
    const std::string& L2 = swap ? s.a : s.b;
    const int64_t n1 = swap ? nB : nA, n2 = swap ? nA : nB;
    const bool f1s = swap ? B.f32 : A.f32, f2s = swap ? A.f32 : B.f32;
    const std::string& f1o = swap ? free_b_o : free_a_o;
    const std::string& f2o = swap ? free_a_o : free_b_o;
    const std::string& f1own = swap ? free_b_own : free_a_own;
    const std::string& f2own = swap ? free_a_own : free_b_own;
    for (int co = 0; co < 2; ++co) {
      const std::string contr = co ? contr_b : contr_a;
      for (int f1c = 0; f1c < 2; ++f1c) {
        const std::string f1 = f1c ? f1own : f1o;
        for (int f2c = 0; f2c < 2; ++f2c) {
          const std::string f2 = f2c ? f2own : f2o;
          Plan p;
          p.swap = swap;
          // first operand: [batch f1 contr] (tA=0) or [batch contr f1]
          const std::string l1n = batch + f1 + contr;
          const std::string l1t = batch + contr + f1;
          if (L1 == l1n) {
            p.first = l1n;
          } else if (L1 == l1t) {
            p.first = l1t;
            p.tA = true;
          } else {
            p.first = l1n;
            p.perm_first = true;
          }
          const std::string l2n = batch + contr + f2;
          const std::string l2t = batch + f2 + contr;
          if (L2 == l2n) {
            p.second = l2n;
          } else if (L2 == l2t) {
            p.second = l2t;
            p.tB = true;
          } else {
            p.second = l2n;
            p.perm_second = true;
          }
          p.out = batch + f1 + f2;
          p.perm_out = (p.out != s.o);
          // an FP32-stored operand is read as it is by the products only
          // as the first one, unpermuted; elsewhere it is widened first
          const int64_t pin = (p.perm_first ? n1 : 0) +
                              (p.perm_second ? n2 : 0) +
                              (f1s && p.perm_first ? n1 : 0) +
                              (f2s ? n2 : 0) +
                              (f1s && nbatch_all > 1 ? n1 : 0);
          p.cost = pin + (p.perm_out ? 2 * nO : 0);
          // prefer no transposes on ties (slightly faster loads)
          auto take = [&](const Plan& q) {
            if (q.cost < best.cost ||
                (q.cost == best.cost &&
                 ((int)q.scatter > (int)best.scatter ||
                  ((int)q.scatter == (int)best.scatter &&
                   (int)q.tA + (int)q.tB < (int)best.tA + (int)best.tB))))
              best = q;
          };
          take(p);
          if (p.perm_out && batch_adjacent && dev.allow_scatter) {
            // the same GEMM writing the output layout from its epilogue: no
            // permute pass.  Its stores run along the fastest column digit,
            // coalesced when that is the output's innermost label (runs of
            // that label's extent); otherwise they are strided
            Plan q = p;
            q.perm_out = false;
            q.scatter = true;
            const char inner = s.o.back();
            const bool coal = !f2.empty() && f2.back() == inner;
            const int64_t ein = dim_of(inner, s.a, A, s.b, B);
            q.cost = pin + (coal ? (ein >= 8 ? 0 : nO / 2) : 4 * nO);
            take(q);
          }
        }
      }
    }
  }

  const std::string& L1 = best.swap ? s.b : s.a;
  const std::string& L2 = best.swap ? s.a : s.b;
  std::vector<Tensor> op1(ni), op2(ni);
  auto widened = [&](const Tensor& t) {
    if (!t.f32) return t;
    Tensor w = dev.empty(t.shape);
    to_f64(dev, (const float*)t.ptr, w.ptr, t.numel());
    return w;
  };
  // the first operand stays FP32 when the products can read it so (one
  // pointer batch, no permutation)
  const bool a32 = (best.swap ? B.f32 : A.f32) && !best.perm_first &&
                   nbatch_all == 1;
  for (size_t i = 0; i < ni; ++i) {
    const Tensor T1 = a32 ? (best.swap ? Bs[i] : As[i])
                          : widened(best.swap ? Bs[i] : As[i]);
    const Tensor T2 = widened(best.swap ? As[i] : Bs[i]);
    op1[i] = best.perm_first ? permuted(dev, T1, perm_of(L1, best.first))
                             : T1;
    op2[i] = best.perm_second ? permuted(dev, T2, perm_of(L2, best.second))
                              : T2;
  }

  auto prod = [&](const std::string& ls) {
    int64_t p = 1;
    for (char ch : ls) p *= dim_of(ch, s.a, A, s.b, B);
    return p;
  };
  const std::string f1 =
      best.out.substr(batch.size(), best.out.size() - batch.size());
  int64_t nbatch = prod(batch);
  // free labels of the first operand are those of out after batch that
  // belong to L1
  std::string lf1, lf2;
  for (char ch : f1) (has(L1, ch) ? lf1 : lf2) += ch;
  const int64_t M = prod(lf1), N = prod(lf2);
  std::string contr;
  for (char ch : best.first)
    if (has(L2, ch) && !has(batch, ch)) contr += ch;
  const int64_t K = prod(contr);

  std::vector<Tensor> dst(outs);
  double beta_g = beta;
  CMap cm;
  int64_t sC_out = M * N;
  if (best.scatter) {
    const std::vector<int64_t>& osh = out.shape;
    if (!cmap_digits(lf1, s.o, osh, cm.nr, cm.re, cm.rs) ||
        !cmap_digits(lf2, s.o, osh, cm.nc, cm.ce, cm.cs)) {
      // too many digits: write the GEMM's own order and permute
      best.scatter = false;
      best.perm_out = true;
    } else if (!batch.empty()) {
      const size_t pl = s.o.find(batch.back());
      sC_out = 1;
      for (size_t j = pl + 1; j < s.o.size(); ++j) sC_out *= osh[j];
    }
    if (best.scatter) {
      // every address the epilogue forms lies inside the output: the digit
      // extents multiply to M and N, and the largest offset of a batch item
      // plus the largest batch offset is below the element count
      int64_t pr = 1, pc = 1, top = (nbatch - 1) * sC_out;
      for (int i = 0; i < cm.nr; ++i) {
        pr *= cm.re[i];
        top += (cm.re[i] - 1) * cm.rs[i];
      }
      for (int i = 0; i < cm.nc; ++i) {
        pc *= cm.ce[i];
        top += (cm.ce[i] - 1) * cm.cs[i];
      }
      if (pr != M || pc != N || top >= out.numel() || top < 0)
        throw std::logic_error("einsum: scattered layout out of range");
    }
  }
  if (best.perm_out) {
    std::vector<int64_t> sh;
    for (char ch : best.out) sh.push_back(dim_of(ch, s.a, A, s.b, B));
    for (size_t i = 0; i < ni; ++i) dst[i] = dev.empty(sh);
    beta_g = 0.0;
  }
  const int64_t lda = best.tA ? M : K;
  const int64_t ldb = best.tB ? K : N;
  const double alpha_g = best.perm_out ? 1.0 : alpha;
  // an FP32 output written straight from the epilogue (after a permute
  // pass it is rounded below)
  cm.c32 = (out.f32 && !best.perm_out) ? 1 : 0;
  const CMap* cmp = (best.scatter || cm.c32) ? &cm : nullptr;
  if (best.scatter) ++dev.scatter_count;
  if (a32) {
    std::vector<const float*> pa(ni);
    std::vector<const double*> pb(ni);
    std::vector<double*> pc(ni);
    for (size_t i = 0; i < ni; ++i) {
      pa[i] = (const float*)op1[i].ptr;
      pb[i] = op2[i].ptr;
      pc[i] = dst[i].ptr;
    }
    gemm_ptrs_a32(dev, best.tA, best.tB, M, N, K, alpha_g, pa, lda, pb, ldb,
                  beta_g, pc, N, cmp);
  } else if (ni == 1 || nbatch > 1) {
    for (size_t i = 0; i < ni; ++i)
      gemm(dev, best.tA, best.tB, M, N, K, alpha_g, op1[i].ptr, lda, M * K,
           op2[i].ptr, ldb, K * N, beta_g, dst[i].ptr, N, sC_out, nbatch,
           cmp);
  } else {
    // the items are independent products of one shape: one pointer batch
    std::vector<const double*> pa(ni), pb(ni);
    std::vector<double*> pc(ni);
    for (size_t i = 0; i < ni; ++i) {
      pa[i] = op1[i].ptr;
      pb[i] = op2[i].ptr;
      pc[i] = dst[i].ptr;
    }
    gemm_ptrs(dev, best.tA, best.tB, M, N, K, alpha_g, pa, lda, pb, ldb,
              beta_g, pc, N, cmp);
  }
  if (best.perm_out)
    for (size_t i = 0; i < ni; ++i) {
      if (!out.f32) {
        Tensor o = outs[i];
        permute(dev, dst[i], perm_of(best.out, s.o), o, alpha, beta);
        continue;
      }
      Tensor o = dev.empty(outs[i].shape);
      if (beta != 0.0)
        to_f64(dev, (const float*)outs[i].ptr, o.ptr, o.numel());
      permute(dev, dst[i], perm_of(best.out, s.o), o, alpha, beta);
      to_f32(dev, o.ptr, (float*)outs[i].ptr, o.numel());
    }
}

void einsum_into(Device& dev, const std::string& spec, const Tensor& A,
                 const Tensor& B, Tensor& out, double alpha, double beta) {
  einsum_into_n(dev, spec, {A}, {B}, {out}, alpha, beta);
}

std::vector<Tensor> einsum_n(Device& dev, const std::string& spec,
                             const std::vector<Tensor>& A,
                             const std::vector<Tensor>& B, bool f32) {
  if (A.empty()) return {};
  Spec s = parse(spec);
  std::vector<int64_t> sh;
  for (char ch : s.o) sh.push_back(dim_of(ch, s.a, A[0], s.b, B[0]));
  std::vector<Tensor> out(A.size());
  const bool o32 = f32 && dev.cprec != PREC_FP64;
  for (auto& o : out) o = o32 ? dev.empty_f32(sh) : dev.empty(sh);
  einsum_into_n(dev, spec, A, B, out, 1.0, 0.0);
  return out;
}

Tensor einsum(Device& dev, const std::string& spec, const Tensor& A,
              const Tensor& B) {
  return einsum_n(dev, spec, {A}, {B})[0];
}

}  // namespace ipeps
