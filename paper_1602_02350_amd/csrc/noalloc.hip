// Full-gradient pass for callers that cannot allocate device memory (code under stream capture,
// serving loops, harnesses that forbid hipMalloc): the same kernels as scs_full_gradient, with all
// of their scratch (the transposed U~, gradient partials, FP64 column sums, solver state) carved
// from one file-scope device array instead of the context's workspace.
//
// The array's name is only a host-side stand-in in host code: its device address comes from
// hipGetSymbolAddress, taken once per device with that device current (at context creation), and
// only that address is ever handed to kernels. Every call on one device shares the array.
#include <hip/hip_runtime.h>

#include <mutex>

#include "scs_internal.h"

namespace scs {

namespace {

static __device__ __align__(256) unsigned char scratch[SCS_NOALLOC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;
void* g_scratch_ptr[kMaxDevices] = {};
std::mutex g_scratch_mu;

size_t up256(size_t b) { return (b + 255) / 256 * 256; }

}  // namespace

int noalloc_scratch_init(int device) {
  if (device < 0 || device >= kMaxDevices) {
    set_error("allocation-free scratch: device index out of range");
    return SCS_EINVAL;
  }
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (g_scratch_ptr[device]) return SCS_OK;
  void* p = nullptr;
  SCS_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
  if (!p) {
    set_error("allocation-free scratch: hipGetSymbolAddress returned a null address");
    return SCS_EDEVICE;
  }
  g_scratch_ptr[device] = p;
  return SCS_OK;
}

// Scratch bytes the pass needs for an n x d problem with k sketch vectors (each piece 256-aligned).
size_t noalloc_full_gradient_bytes(int64_t n, int64_t d, int k) {
  const int nwg = grad_num_workgroups(n, d);
  return up256(sizeof(float) * (size_t)k * d)      // U~^T
         + up256(sizeof(SolveState))                // state
         + up256(sizeof(float) * (size_t)d)         // w = P^{-1/2} w~
         + up256(sizeof(double) * (size_t)d)        // FP64 vector scratch
         + up256(sizeof(double) * 16 * (size_t)d)   // first-level column sums
         + up256(sizeof(float) * (size_t)nwg * d)   // per-workgroup gradient partials
         + up256(sizeof(double) * (size_t)nwg)      // per-workgroup residual sums
         + up256(sizeof(float) * (size_t)d);        // snapshot slot the finalizer may write
}

int full_gradient_noalloc(int device, hipStream_t st, const float* X, int64_t n, int64_t d, int64_t ldx,
                          const float* y, const float* U, const double* lam, int k, double lambda, const float* wt,
                          float* grad_out, double* obj_out) {
  if (device < 0 || device >= kMaxDevices || !g_scratch_ptr[device]) {
    set_error("allocation-free scratch: not initialised on this device");
    return SCS_EDEVICE;
  }
  const size_t need = noalloc_full_gradient_bytes(n, d, k);
  if (need > (size_t)SCS_NOALLOC_SCRATCH_BYTES) {
    set_error("scs_full_gradient_noalloc: the problem needs " + std::to_string(need) +
              " bytes of scratch, more than the fixed " + std::to_string((size_t)SCS_NOALLOC_SCRATCH_BYTES));
    return SCS_EINVAL;
  }
  char* p = static_cast<char*>(g_scratch_ptr[device]);
  auto carve = [&](size_t bytes) {
    char* q = p;
    p += up256(bytes);
    return q;
  };
  const int nwg = grad_num_workgroups(n, d);
  float* UT = reinterpret_cast<float*>(carve(sizeof(float) * (size_t)k * d));
  SolveState* state = reinterpret_cast<SolveState*>(carve(sizeof(SolveState)));
  float* w32 = reinterpret_cast<float*>(carve(sizeof(float) * (size_t)d));
  double* tmp = reinterpret_cast<double*>(carve(sizeof(double) * (size_t)d));
  double* g64 = reinterpret_cast<double*>(carve(sizeof(double) * 16 * (size_t)d));
  float* part = reinterpret_cast<float*>(carve(sizeof(float) * (size_t)nwg * d));
  double* rsq = reinterpret_cast<double*>(carve(sizeof(double) * (size_t)nwg));
  float* wcur = reinterpret_cast<float*>(carve(sizeof(float) * (size_t)d));

  // the state left by the previous call is cleared by a kernel (no memset node under capture)
  SCS_CHECK(launch_zero3(st, state, (int64_t)sizeof(SolveState), nullptr, 0, nullptr, 0));
  const float* UTc = nullptr;
  if (k > 0) {
    SCS_CHECK(launch_transpose_f32(st, U, d, k, UT));
    UTc = UT;
  }
  SCS_CHECK(launch_premap(st, UTc, U, lam, k, d, lambda, wt, w32, nullptr, tmp, state));
  SCS_CHECK(launch_grad_partial(st, X, n, d, ldx, y, w32, part, rsq, nwg, state));
  SCS_CHECK(launch_grad_finish(st, part, rsq, nwg, n, d, w32, lambda, UTc, U, lam, k, grad_out, g64, tmp, state,
                               SCS_STOP_EPOCHS, 0.0, 0.0, wcur, nullptr, 1, nullptr));
  if (!obj_out) return SCS_OK;
  SolveState hs;
  SCS_HIP(hipMemcpyAsync(&hs, state, sizeof(hs), hipMemcpyDeviceToHost, st));
  SCS_HIP(hipStreamSynchronize(st));
  *obj_out = hs.obj0;
  if (hs.status == SCS_ENONFINITE) {
    set_error("non-finite value in X or y");
    return SCS_ENONFINITE;
  }
  return SCS_OK;
}

}  // namespace scs
