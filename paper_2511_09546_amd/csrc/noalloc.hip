// Allocation-free variant of precond_apply_dev (include/ipeps.h): every
// temporary of the call lives in one fixed scratch array per GPU instead of
// the context's memory pool, so the call makes no hipMalloc, hipFree or other
// allocating call.
//
// The array is a file-scope __device__ object.  Its host-side name is only a
// stand-in: the device address is looked up once per device with
// hipGetSymbolAddress (with that device current) and only that address is
// handed to the kernels.  All calls on one GPU share the array, so calls that
// overlap on one GPU race; the array keeps the last call's contents, and
// everything that must start at zero (the CG iterate, the scalars) is cleared
// by a fill kernel in the call.
#include <hip/hip_runtime.h>

#include <mutex>

#include "../../include/ipeps.h"
#include "ipeps_impl.hpp"

namespace {

constexpr size_t kScratchBytes = IPEPS_NOALLOC_SCRATCH_BYTES;
static_assert(kScratchBytes % 256 == 0, "scratch size");

__device__ __align__(256) char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void* g_ptr[kMaxDevices] = {};

// device address of this device's scratch array (looked up on first use)
void* scratch_ptr(int dev) {
  if (dev < 0 || dev >= kMaxDevices)
    throw ipeps::ArgError("device index out of range");
  std::lock_guard<std::mutex> lock(g_mu);
  if (!g_ptr[dev]) {
    void* p = nullptr;
    IPEPS_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p) throw ipeps::HipError("hipGetSymbolAddress returned null");
    g_ptr[dev] = p;
  }
  return g_ptr[dev];
}

// makes `dev` current for a scope and restores the caller's device
struct DeviceScope {
  int old = -1;
  explicit DeviceScope(int dev) {
    IPEPS_HIP(hipGetDevice(&old));
    if (old != dev) IPEPS_HIP(hipSetDevice(dev));
  }
  ~DeviceScope() {
    int cur = -1;
    if (hipGetDevice(&cur) == hipSuccess && cur != old) (void)hipSetDevice(old);
  }
};

// the pool of a context serves from the scratch array for a scope
struct ArenaScope {
  ipeps::Pool& pool;
  ArenaScope(ipeps::Pool& p, void* base, size_t bytes) : pool(p) {
    pool.begin_arena(base, bytes);
  }
  ~ArenaScope() { pool.end_arena(); }
};

}  // namespace

extern "C" {

size_t precond_noalloc_bytes(int Lx, int Ly, int d, int D, int chi) {
  if (Lx < 1 || Ly < 1 || d < 1 || D < 1 || chi < 1) return 0;
  return ipeps::precondition_lean_bytes(Lx * Ly, d, D, chi);
}

int precond_apply_dev_noalloc(ipeps_ctx* c, const double* d_g, double delta,
                              double cg_tol, int cg_maxiter, double* d_x,
                              int* n_iter, double* rel_resid) {
  if (!c || !d_g || !d_x || !(delta > 0.0) || !(delta < INFINITY) ||
      !(cg_tol >= 0.0) || cg_maxiter < 0)
    return IPEPS_EINVAL;
  ipeps::Context& cx = ipeps_context(c);
  if (!cx.converged_once) return IPEPS_ESTATE;
  if (ipeps::precondition_lean_bytes(cx.nsite(), cx.d, cx.D, cx.chi) >
      kScratchBytes)
    return IPEPS_ESCRATCH;
  try {
    DeviceScope ds(cx.device);
    void* base = scratch_ptr(cx.device);
    int res = 0;
    {
      ipeps::PrecScope ps(cx.dev, cx.ladder ? (int)ipeps::PREC_FP32 : cx.prec);
      ArenaScope as(cx.dev.pool, base, kScratchBytes);
      res = ipeps::precondition(cx, d_g, delta, cg_tol, cg_maxiter, d_x,
                                n_iter, rel_resid, true, true);
    }
    return res;
  } catch (const ipeps::OomError&) {
    return IPEPS_ESCRATCH;  // the estimate was short: nothing allocated
  } catch (const ipeps::ArgError&) {
    return IPEPS_EINVAL;
  } catch (...) {
    return IPEPS_EHIP;
  }
}

}  // extern "C"
