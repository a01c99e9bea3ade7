// noalloc.hip -- the relative residual norm for callers that cannot allocate device
// memory.  mg_residual_norm's kernels need scratch memory (the solve state and one
// partial sum per block of each norm pass); here that scratch is the file-scope device
// array `scratch`, located once per device with hipGetSymbolAddress, and the result is
// written to a caller-owned device double.  Nothing is allocated, nothing is waited for.
#include <hip/hip_runtime.h>

#include <mutex>
#include <string>

#include "batch.h"
#include "mg.h"
#include "mg_internal.h"

using mgk::DevState;

namespace {

constexpr size_t kScratchBytes = MG_NOALLOC_SCRATCH_BYTES;
// the solve state first, the partial sums from the next 256-byte boundary
constexpr size_t kPartialsOffset = (sizeof(DevState) + 255) / 256 * 256;
static_assert(kPartialsOffset < kScratchBytes, "the scratch holds the solve state");

// Host code must never pass `scratch` itself to a kernel or a copy: on the host the name
// is a stand-in, not a device address.  scratch_ptr() gives the device address.
__device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void *g_scratch[kMaxDevices];  // device address of `scratch` on each device, once looked up

mg_status fail(mg_status st, const std::string &msg) {
  mgb::set_error(msg);
  return st;
}

// Device address of this device's copy of `scratch` (the current device's).
mg_status scratch_ptr(int device, void **out) {
  if (device < 0 || device >= kMaxDevices) return fail(MG_EDEVICE, "device ordinal out of range");
  std::lock_guard<std::mutex> lock(g_mu);
  if (g_scratch[device] == nullptr) {
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || p == nullptr)
      return fail(MG_EDEVICE, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    g_scratch[device] = p;
  }
  *out = g_scratch[device];
  return MG_OK;
}

// The state of a two-check norm evaluation (no stopping test, no floor detection).
__global__ void k_noalloc_state(DevState *st) {
  if (threadIdx.x == 0) {
    st->done = 0;
    st->checks = 0;
    st->status = 0;
    st->stall = 0;
    st->max_checks = 2;
    st->floor_detect = 0;
    st->rtol = -1.0;
    st->fnorm2 = 0.0;
    st->best = 0.0;
    st->last_ratio = 0.0;
  }
}

__global__ void k_noalloc_result(const DevState *st, double *rel) {
  if (threadIdx.x == 0) *rel = st->hist[0];
}

bool pow2_plus_one(int n) {
  if (n < 9) return false;
  const int m = n - 1;
  return (m & (m - 1)) == 0;
}

}  // namespace

extern "C" mg_status mg_residual_norm_noalloc(int dim, int n, int order, const double *f,
                                              const double *u, double *rel, void *hip_stream) {
  if (dim != 2 && dim != 3) return fail(MG_EINVAL, "dim must be 2 or 3");
  if (order != 2 && order != 4 && order != 6) return fail(MG_EINVAL, "order must be 2, 4 or 6");
  if (!pow2_plus_one(n) || n > (dim == 2 ? 32769 : 2049)) return fail(MG_EINVAL, "n must be 2^k + 1, k >= 3");
  if (!f || !u || !rel) return fail(MG_EINVAL, "null f, u or rel");
  const size_t need = kPartialsOffset + (size_t)mgk::sweep_partials(dim, n) * sizeof(double);
  if (need > kScratchBytes)
    return fail(MG_EINVAL, "n = " + std::to_string(n) + " needs " + std::to_string(need) +
                               " scratch bytes, more than MG_NOALLOC_SCRATCH_BYTES (" +
                               std::to_string(kScratchBytes) + ")");
  int device = 0;
  if (hipGetDevice(&device) != hipSuccess) return fail(MG_EDEVICE, "no HIP device");
  void *base = nullptr;
  mg_status st = scratch_ptr(device, &base);
  if (st != MG_OK) return st;
  DevState *state = (DevState *)base;
  double *partials = (double *)((unsigned char *)base + kPartialsOffset);
  hipStream_t s = (hipStream_t)hip_stream;
  const mgk::LevelOp op = mgk::rediscretized_op(order, dim, 1.0 / (n - 1));
  // 3D: the LDS limits of the sweep kernels (an attribute call, no allocation)
  hipError_t e = dim == 3 ? mgk::prepare_3d() : hipSuccess;
  if (e == hipSuccess) {
    hipLaunchKernelGGL(k_noalloc_state, dim3(1), dim3(64), 0, s, state);
    e = hipGetLastError();
  }
  int np = 0;
  // ||f||_h (the residual of u = 0), then ||f - L u||_h: the passes of mg_residual_norm
  if (e == hipSuccess)
    e = mgk::launch_sweep<double, double>(dim, mgk::kNormOnly, op, 1.0, f, nullptr, (double *)nullptr, n,
                                          partials, &np, nullptr, s);
  if (e == hipSuccess) e = mgk::launch_check(state, partials, np, 0, s);
  if (e == hipSuccess)
    e = mgk::launch_sweep<double, double>(dim, mgk::kNormOnly, op, 1.0, f, u, (double *)nullptr, n,
                                          partials, &np, nullptr, s);
  if (e == hipSuccess) e = mgk::launch_check(state, partials, np, 1, s);
  if (e == hipSuccess) {
    hipLaunchKernelGGL(k_noalloc_result, dim3(1), dim3(64), 0, s, state, rel);
    e = hipGetLastError();
  }
  if (e != hipSuccess) return fail(MG_EDEVICE, std::string("kernel launch: ") + hipGetErrorString(e));
  return MG_OK;
}
