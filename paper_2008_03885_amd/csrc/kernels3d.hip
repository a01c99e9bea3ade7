// kernels3d.hip -- 3D hot-path kernels for gfx950 (not yet implemented).
#include "mg_internal.h"

namespace mgk {

int sweep_partials_3d(int n) { return 1; }

template <typename T, typename TO>
hipError_t launch_sweep_3d(int, const LevelOp &, double, const T *, const T *, TO *, int,
                           double *, int *, const int *, hipStream_t) {
  return hipErrorNotSupported;
}
template <typename T>
hipError_t launch_resid_restrict_3d(const LevelOp &, const T *, const T *, T *, int, const int *,
                                    hipStream_t) {
  return hipErrorNotSupported;
}
template <typename T>
hipError_t launch_prolong_correct_3d(int, const T *, const T *, T *, int, const int *,
                                     hipStream_t) {
  return hipErrorNotSupported;
}

template hipError_t launch_sweep_3d<double, double>(int, const LevelOp &, double, const double *,
                                                    const double *, double *, int, double *, int *,
                                                    const int *, hipStream_t);
template hipError_t launch_sweep_3d<float, float>(int, const LevelOp &, double, const float *,
                                                  const float *, float *, int, double *, int *,
                                                  const int *, hipStream_t);
template hipError_t launch_sweep_3d<double, float>(int, const LevelOp &, double, const double *,
                                                   const double *, float *, int, double *, int *,
                                                   const int *, hipStream_t);
template hipError_t launch_resid_restrict_3d<double>(const LevelOp &, const double *,
                                                     const double *, double *, int, const int *,
                                                     hipStream_t);
template hipError_t launch_resid_restrict_3d<float>(const LevelOp &, const float *, const float *,
                                                    float *, int, const int *, hipStream_t);
template hipError_t launch_prolong_correct_3d<double>(int, const double *, const double *,
                                                      double *, int, const int *, hipStream_t);
template hipError_t launch_prolong_correct_3d<float>(int, const float *, const float *, float *,
                                                     int, const int *, hipStream_t);
}  // namespace mgk
