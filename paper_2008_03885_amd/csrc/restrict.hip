// restrict.hip -- the cubic-adjoint restriction of appendix A.4 (the operator
// I_h^H = (1/1024) [1 0 -9 -16 -9 0 1]^T [1 0 -9 -16 -9 0 1], with the printed equation
// labels of the two transfers swapped: this is the restriction, the 1/256 operator the
// interpolation).  Per axis the weights are 1/2 at the coarse point, 9/32 at +-1 and -1/32
// at +-3 fine points; in 3D the tensor product of three.  The input is a fine-grid defect
// with zero boundary values; fine points beyond the boundary are odd reflections.
//
// One thread per coarse point sums the 5^dim non-zero taps; neighbouring threads share
// their fine rows through the caches.  This pass runs after a separate defect pass (the
// fused defect + full weighting kernels have the radius-1 weights built in).
#include "mg_internal.h"

namespace mgk {
namespace {

__device__ __forceinline__ bool stopped(const int *done) { return done != nullptr && *done != 0; }

__device__ __forceinline__ int fold(int i, int n, int &sign) {
  if (i < 0) { i = -i; sign = -sign; }
  if (i > n - 1) { i = 2 * (n - 1) - i; sign = -sign; }
  return i;
}

constexpr int kTaps = 5;
__device__ __constant__ const int kOff[kTaps] = {-3, -1, 0, 1, 3};
__device__ __constant__ const double kW[kTaps] = {-1.0 / 32, 9.0 / 32, 0.5, 9.0 / 32, -1.0 / 32};

template <typename T, int DIM>
__global__ __launch_bounds__(256) void k_restrict_cubic(const T *__restrict__ r, T *__restrict__ fc, int n,
                                                        const int *__restrict__ done) {
  done = slot_done(done);
  if (stopped(done)) return;
  const int nc = (n - 1) / 2 + 1;
  const size_t nf = DIM == 2 ? (size_t)n * n : (size_t)n * n * n;
  const size_t ncp = DIM == 2 ? (size_t)nc * nc : (size_t)nc * nc * nc;
  r = slot_ptr(r, nf);
  fc = slot_ptr(fc, ncp);
  for (size_t id = (size_t)blockIdx.x * blockDim.x + threadIdx.x; id < ncp; id += (size_t)gridDim.x * blockDim.x) {
    const int I = (int)(id % nc), J = (int)((id / nc) % nc), K = DIM == 3 ? (int)(id / ((size_t)nc * nc)) : 0;
    const bool inner = I > 0 && I < nc - 1 && J > 0 && J < nc - 1 && (DIM == 2 || (K > 0 && K < nc - 1));
    double acc = 0.0;
    if (inner) {
      for (int c = 0; c < (DIM == 3 ? kTaps : 1); ++c) {
        int sz = 1, zf = 0;
        double wz = 1.0;
        if (DIM == 3) {
          zf = fold(2 * K + kOff[c], n, sz);
          if (zf == 0 || zf == n - 1) continue;
          wz = kW[c] * sz;
        }
        for (int b = 0; b < kTaps; ++b) {
          int sy = 1;
          const int yf = fold(2 * J + kOff[b], n, sy);
          if (yf == 0 || yf == n - 1) continue;
          const double wy = wz * kW[b] * sy;
          const size_t row = ((size_t)zf * n + yf) * n;
          double s = 0.0;
          for (int a = 0; a < kTaps; ++a) {
            int sx = 1;
            const int xf = fold(2 * I + kOff[a], n, sx);
            if (xf == 0 || xf == n - 1) continue;
            s += kW[a] * sx * (double)r[row + xf];
          }
          acc += wy * s;
        }
      }
    }
    fc[id] = (T)acc;
  }
}

}  // namespace

template <typename T>
hipError_t launch_restrict_cubic(int dim, const T *r, T *fc, int n, const int *done, hipStream_t s, int slots) {
  if (dim != 2 && dim != 3) return hipErrorInvalidValue;
  const int nc = (n - 1) / 2 + 1;
  const size_t ncp = dim == 2 ? (size_t)nc * nc : (size_t)nc * nc * nc;
  const int blocks = (int)std::min<size_t>((ncp + 255) / 256, 16384);
  if (dim == 2)
    hipLaunchKernelGGL((k_restrict_cubic<T, 2>), dim3(blocks, 1, slots), dim3(256), 0, s, r, fc, n, done);
  else
    hipLaunchKernelGGL((k_restrict_cubic<T, 3>), dim3(blocks, 1, slots), dim3(256), 0, s, r, fc, n, done);
  return hipGetLastError();
}

template hipError_t launch_restrict_cubic<double>(int, const double *, double *, int, const int *, hipStream_t,
                                                  int);
template hipError_t launch_restrict_cubic<float>(int, const float *, float *, int, const int *, hipStream_t, int);

}  // namespace mgk
