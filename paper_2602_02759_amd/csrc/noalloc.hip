// nnef_mlp_gradient_noalloc: the gradient of the extrapolation network's
// training loss with no device allocation.  Same kernels as
// nnef_mlp_gradient; the per-workgroup gradient and loss partials live in a
// file-scope device array instead of the allocation that nnef_mlp_create
// makes, and the parameters come from a caller buffer instead of an MLP
// handle.
#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstring>
#include <mutex>
#include <string>

#include "../../include/nnef.h"
#include "nnef_internal.hpp"

namespace {

// Partials of at most kSlots workgroups: kSlots x kMlpParams floats, then
// kSlots doubles (18.2 MB in all).  mlp_grid never launches more than 256
// workgroups.
constexpr int kSlots = 256;
constexpr size_t kGradBytes = (size_t)kSlots * nnef::kMlpParams * sizeof(float);
constexpr size_t kLossOff = (kGradBytes + 255) / 256 * 256;
constexpr size_t kScratchBytes = kLossOff + kSlots * sizeof(double);

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void* g_ptr[kMaxDevices] = {};

// Device address of this device's copy of `scratch` (looked up once per
// device, with that device current).
hipError_t scratch_ptr(void** out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lk(g_mu);
  if (!g_ptr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_ptr[dev] = p;
  }
  *out = g_ptr[dev];
  return hipSuccess;
}

}  // namespace

namespace nnef {
nnef_status report_error(nnef_status st, const std::string& msg);
nnef_status report_hip_error(int e, const char* what);
}  // namespace nnef

extern "C" nnef_status nnef_mlp_gradient_noalloc(const float* d_params, const float* X, const float* tau,
                                                 const int32_t* idx, int64_t n_rows, float* d_grad,
                                                 double* d_loss, void* stream) {
  using namespace nnef;
  const auto fail = report_error;
  const auto hip_fail = report_hip_error;
  if (!d_params || !X || !tau || !d_grad) return fail(NNEF_E_ARG, "NULL argument");
  if (n_rows <= 0) return fail(NNEF_E_ARG, "n_rows must be positive");
  if (n_rows >= (int64_t(1) << 31)) return fail(NNEF_E_SHAPE, "n_rows must be below 2^31");
  const int grid = mlp_grid(n_rows);
  if (grid > kSlots)
    return fail(NNEF_E_SHAPE, "the gradient needs more partial slots than the static scratch holds");
  void* base = nullptr;
  const hipError_t e0 = scratch_ptr(&base);
  if (e0 != hipSuccess) return hip_fail((int)e0, "scratch address lookup");
  MlpArgs a;
  std::memset(&a, 0, sizeof(a));
  a.params = d_params;
  a.n_rows = n_rows;
  a.X = X;
  a.tau = tau;
  a.idx = idx;
  a.inv_n = (float)(1.0 / (double)n_rows);
  // every workgroup writes all of its partial slot, so nothing needs clearing
  a.gpart = reinterpret_cast<float*>(base);
  a.lpart = reinterpret_cast<double*>(reinterpret_cast<unsigned char*>(base) + kLossOff);
  int e = launch_mlp(a, 1, grid, stream);
  if (e) return hip_fail(e, "MLP gradient launch");
  e = launch_mlp_reduce(a.gpart, a.lpart, grid, a.inv_n, d_grad, d_loss, nullptr, nullptr, nullptr, 0.f,
                        0.9f, 0.999f, 1e-8f, 1.f, 1.f, 0, stream);
  return e ? hip_fail(e, "MLP reduction launch") : NNEF_OK;
}
