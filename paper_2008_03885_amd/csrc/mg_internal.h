// mg_internal.h -- declarations shared by the kernels and the host runtime.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

#include "mg.h"

namespace mgk {

constexpr int kBlock = 256;      // threads per block of the streaming kernels
constexpr int kMaxRadius = 3;    // widest 1D operator factor (Galerkin coarse levels)
constexpr int kMaxHistory = MG_MAX_HISTORY;

// Level operator L = sum over axes of a (along that axis) times b (along the others),
// a and b symmetric 1D stencils of radius <= 3 stored at offsets -3..3.
// cross: b is the unit stencil, so L is the (2D 9-point / 3D 13-point) cross and the
// kernels use the difference form sum_{k != 0} w_k (u_0 - u_k) with w_k = -a_k.
struct LevelOp {
  double a[7];
  double b[7];
  bool cross;
  double diag;          // centre coefficient of L
  bool cross3 = false;  // b is the unit stencil and a has radius 3 (sixth order): the fused
                        // 2D kernels apply it as a radius-3 cross, the others as separable
};

// Coefficients as seen by a kernel, in its arithmetic type.
template <typename T>
struct KOp {
  T a[7];
  T b[7];
  T w1, w2;   // cross: weights of (u_0 - u_{+-1}) and (u_0 - u_{+-2})
  T w3;       // radius-3 cross: weight of (u_0 - u_{+-3})
  T om_d;     // omega / diag
  int colour; // sweeps: 0 relax every interior point; 1 only odd x+y(+z), 2 only even
};

// Fused 2D kernels with colour kColourRB run red-black stages: stage s (1-based) relaxes
// the red points (odd x+y) when s is odd and the black ones when s is even.
constexpr int kColourRB = 3;
template <typename T>
__device__ __forceinline__ T stage_om(const KOp<T> &k, int s, int xy) {
  return (k.colour != kColourRB || ((xy + s) & 1) == 0) ? k.om_d : T(0);
}

// Relaxation weight of a sweep at a point with coordinate sum xyz: omega/diag where the
// point's colour is relaxed, 0 (the value is kept) elsewhere.
template <typename T>
__device__ __forceinline__ T colour_om(const KOp<T> &k, int xyz) {
  return (k.colour == 0 || (xyz & 1) == (k.colour & 1)) ? k.om_d : T(0);
}

// Device-resident stopping state of a solve; every step kernel returns at once when
// done != 0, so a captured step can be replayed past convergence at no cost.
struct DevState {
  int done;
  int checks;      // number of residual checks recorded
  int status;      // 0 running, 1 converged, 2 cap, 3 floor, 4 non-finite, 5 growth
  int stall;
  int max_checks;  // stop after this many checks
  int floor_detect;
  double rtol;
  double fnorm2;   // sum of f^2 over interior points
  double best;
  double last_ratio;
  double hist[kMaxHistory];
};

// kSweepRB: a sweep relaxing one colour (KOp::colour), the 3D kernels' red-black step.
// kSweepZ2: two omega-Jacobi sweeps from a zero iterate in one pass (3D): the first
// sweep's result, omega / a0 * f, is formed on the fly wherever the second reads u.
enum SweepMode { kSweep = 0, kResidual = 1, kNormOnly = 2, kSweepRB = 3, kSweepZ2 = 4, kSweepCorr = 5 };

// Workgroups are dealt to the XCDs (8 on MI355X, each with its own L2) round-robin in
// linear dispatch order.  xcd_logical maps a linear id to a logical block id such that
// each XCD receives one contiguous range of logical ids; neighbouring tiles then run on
// the same XCD and share their halo lines in its L2.  A bijection on [0, nb).
constexpr unsigned kXcds = 8;
__device__ __forceinline__ unsigned xcd_logical(unsigned lid, unsigned nb) {
  const unsigned q = nb / kXcds, r = nb % kXcds;
  const unsigned x = lid % kXcds, local = lid / kXcds;
  return x < r ? x * (q + 1) + local : r * (q + 1) + (x - r) * q + local;
}
// Logical (x, y) block of a 2D grid (the third grid dimension is left alone).
struct Block2 {
  int x, y;
};
__device__ __forceinline__ Block2 block2() {
  const unsigned nb = gridDim.x * gridDim.y;
  const unsigned l = xcd_logical(blockIdx.y * gridDim.x + blockIdx.x, nb);
  return {(int)(l % gridDim.x), (int)(l / gridDim.x)};
}
// Logical (x, y, z) block of a 3D grid.
struct Block3 {
  int x, y, z;
};
__device__ __forceinline__ Block3 block3() {
  const unsigned nxy = gridDim.x * gridDim.y;
  const unsigned l = xcd_logical((blockIdx.z * gridDim.y + blockIdx.y) * gridDim.x + blockIdx.x,
                                 nxy * gridDim.z);
  const unsigned rxy = l % nxy;
  return {(int)(rxy % gridDim.x), (int)(rxy / gridDim.x), (int)(l / nxy)};
}

// Batched launches.  grid.z indexes independent problems of one size ("slots"): every
// per-problem array is dense [slot][points], partial sums are [slot][blocks of one slot]
// and each slot has its own DevState, so slot k of a batched launch computes exactly
// what an unbatched launch on slot k's arrays computes.  The 3D streaming kernels use
// grid.z for plane chunks and are never batched.
constexpr size_t kStateInts = sizeof(DevState) / sizeof(int);
static_assert(sizeof(DevState) % sizeof(int) == 0, "DevState packs whole ints");
__device__ __forceinline__ const int *slot_done(const int *done) {
  return done == nullptr ? nullptr : done + (size_t)blockIdx.z * kStateInts;
}
template <typename P>
__device__ __forceinline__ P *slot_ptr(P *p, size_t per_slot) {
  return p == nullptr ? p : p + (size_t)blockIdx.z * per_slot;
}

// The rediscretized operator of a level of spacing h (order 2, 4 or 6), as 1D factors
// (runtime.hip).
LevelOp rediscretized_op(int order, int dim, double h);

// ---- launchers (kernels.hip) ----------------------------------------------------
// All take the level side n, dense arrays, and an optional `done` flag.

// colour (kSweep): 0 relaxes every interior point, 1 the red points (odd x+y(+z)), 2 the
// black ones; the other points are copied.  One red-black sweep is colour 1, then 2.
template <typename T, typename TO>
hipError_t launch_sweep(int dim, int mode, const LevelOp &op, double omega, const T *f,
                        const T *u, TO *out, int n, double *partials, int *nparts,
                        const int *done, hipStream_t s, int slots = 1, int colour = 0);

template <typename T>
hipError_t launch_resid_restrict(int dim, const LevelOp &op, const T *f, const T *u, T *fc,
                                 int n, const int *done, hipStream_t s, int slots = 1);

template <typename T>
hipError_t launch_prolong_correct(int dim, int prolong, const T *v, const T *uin, T *uout,
                                  int n, const int *done, hipStream_t s, int slots = 1);

template <typename T>
hipError_t launch_coarsest(int dim, const double *ainv_t, const T *g, T *v, int nc,
                           const int *done, hipStream_t s, int slots = 1);

// nparts: partial sums per slot (slot k reads partials[k * nparts ...]).
hipError_t launch_check(DevState *st, const double *partials, int nparts, int record,
                        hipStream_t s, int slots = 1);

hipError_t launch_ir_correct(int dim, double *u, const float *e, int n, const int *done,
                             hipStream_t s, int slots = 1);

template <typename T>
hipError_t launch_fill(T *p, size_t count, T value, const int *done, hipStream_t s,
                       int slots = 1);

// Largest number of partial sums a level-0 sweep of side n produces.
int sweep_partials(int dim, int n);

// ---- launch geometry ----------------------------------------------------------------
// Blocks of kernel fn (`threads` per block, `smem` dynamic LDS bytes) the current device
// keeps resident at once: the occupancy calculator's blocks per CU times the CU count.
int resident_blocks(const void *fn, int threads, size_t smem);
// Rows (or planes) per band when a launch covers `total` rows in bands of `across`
// blocks each: as many bands as one round of `capacity` resident blocks holds, none
// shorter than cmin.  A launch of one round has no straggler blocks.
int band_rows(int total, int across, int capacity, int cmin);

// 3D variants (kernels3d.hip), called by the launchers above for dim == 3.
int sweep_partials_3d(int n);
bool sweep3d_z2_ok(const LevelOp &op);
hipError_t prepare_3d();  // enables the large dynamic LDS of the separable 3D kernels
template <typename T, typename TO>
hipError_t launch_sweep_3d(int mode, const LevelOp &op, double omega, const T *f, const T *u,
                           TO *out, int n, double *partials, int *nparts, const int *done,
                           hipStream_t s, int colour = 0);
// One red-black sweep (red, then black partial step) of a cross level in one pass;
// out != u.  hipErrorInvalidValue for a non-cross operator.
template <typename T>
hipError_t launch_rbsweep_3d(const LevelOp &op, double omega, const T *f, const T *u, T *out, int n,
                             double *partials, int *nparts, const int *done, hipStream_t s);
// The last FP32 sweep of a refinement step fused with the FP64 correction: one
// omega-Jacobi sweep of the cross on e (FP32), whose result e' (rounded to FP32) is added to
// u64 at every interior point, u64 += e'; e' itself is not stored.  Interior points only:
// u64's boundary is left as it is.
hipError_t launch_sweep_corr_3d(const LevelOp &op, double omega, const float *f, const float *e,
                                double *u64, int n, const int *done, hipStream_t s);
// two omega-Jacobi sweeps of the cross in one pass (out of place)
template <typename T>
hipError_t launch_x2sweep_3d(const LevelOp &op, double omega, const T *f, const T *u, T *out, int n,
                             double *partials, int *nparts, const int *done, hipStream_t s);
template <typename T>
hipError_t launch_resid_restrict_3d(const LevelOp &op, const T *f, const T *u, T *fc, int n,
                                    const int *done, hipStream_t s);
template <typename T>
hipError_t launch_prolong_correct_3d(int prolong, const T *v, const T *uin, T *uout, int n,
                                     const int *done, hipStream_t s);

// ---- cubic-adjoint restriction (restrict.hip) --------------------------------------
// fc = I_h^H r (appendix A.4, the 1/1024 operator) on the level (n-1)/2+1, r a fine defect
// with zero boundary; every coarse point written (boundary zeros).  dim 2 or 3.
template <typename T>
hipError_t launch_restrict_cubic(int dim, const T *r, T *fc, int n, const int *done, hipStream_t s,
                                 int slots = 1);

// ---- red-black Gauss-Seidel partial step, 2D (gs2d.hip) --------------------------
// The colour's points (1 red, 2 black) in lexicographic order from the current values
// (section 3.1 eq. S_GS), every other point copied; cross operators of radius 2 or 3 only
// (hipErrorInvalidValue otherwise).  uout != uin, both full n x n arrays (boundary zeros
// written).
template <typename T>
hipError_t launch_gs2d(const LevelOp &op, double omega, int colour, const T *f, const T *uin, T *uout,
                       int n, const int *done, hipStream_t s, int slots = 1);

// ---- fused 2D cycle kernels (fused2d.hip) ----------------------------------------
// Pre kernel modes (bit set): 1 write the smoothed iterate, 2 full-weight the defect,
// 4 write the defect.  Supported: WriteU|Restrict with nu <= 3 (the pre half of a cycle),
// WriteU with nu = 1 (one sweep), WriteR with nu = 0 (the defect), Restrict with nu = 0
// (defect and full weighting).  rb: the nu stages alternate red and black partial steps,
// red first (a red-black sweep is two stages); supported: WriteU|Restrict with nu = 0 or
// 2, WriteU with nu = 2.  launch_post2d with rb: nu2 = 0 or 2 stages.
constexpr int kPreWriteU = 1, kPreRestrict = 2, kPreWriteR = 4;
int pre2d_partials(int n);
template <typename T>
hipError_t launch_pre2d(const LevelOp &op, double omega, int nu, int mode, const T *f, const T *u,
                        T *uout, T *rout, T *fc, int n, double *partials, int *nparts,
                        const int *done, hipStream_t s, int slots = 1, bool rb = false);
template <typename T>
hipError_t launch_post2d(const LevelOp &op, double omega, int nu2, int prolong, const T *v,
                         const T *uin, const T *f, T *uout, int n, const int *done,
                         hipStream_t s, int slots = 1, bool rb = false);

// ---- tile kernels for small levels (tile2d.hip) -------------------------------------
// launch_pre2d / launch_post2d use them for sides up to tile2d_max_side() (the
// MG_TILE_N environment variable, default 513).
int tile2d_max_side();
int pre2d_tile_partials(int n);
template <typename T>
hipError_t launch_pre2d_tile(const LevelOp &op, double omega, int nu, int mode, const T *f, const T *u,
                             T *uout, T *rout, T *fc, int n, double *partials, int *nparts,
                             const int *done, hipStream_t s, int slots, bool rb);
template <typename T>
hipError_t launch_post2d_tile(const LevelOp &op, double omega, int nu2, int prolong, const T *v,
                              const T *uin, const T *f, T *uout, int n, const int *done,
                              hipStream_t s, int slots, bool rb);

// ---- LDS-resident tail (tail.hip) -------------------------------------------------
constexpr int kMaxTailLevels = 8;
struct TailLevel {
  int n;
  int ent_begin, ent_count;  // non-centre stencil entries of this level
  int cross;                 // rediscretized cross stencil (weights w1, w2)
  double om_d;               // omega / centre coefficient
  double w1, w2;
};
struct TailArgs {
  int levels, gamma, nu1, nu2, prolong, zero_init, m, lds_r;
  int repeats;               // cycles from the top level (the parent's gamma visits)
  int rb;                    // 1: red-black Jacobi sweeps, 0: omega-Jacobi
  int ent_first, ent_total;  // entries of the tail's levels in eoff/ecoef
  int lds_ent;               // byte offset of the entry table in LDS
  TailLevel lv[kMaxTailLevels];
  const int *eoff;       // (dx, dy, dz) per entry
  const double *ecoef;   // coefficient per entry
  const double *ainv_t;  // coarsest inverse, transposed, m x m
  const double *dst;     // coarsest sine table (S, then scaled inverse eigenvalues), or null
  const void *f_top;
  void *u_top;
  const int *done;
};
int tail_max_side(int dim);
size_t tail_scratch_offset(int dim, int G, const int *ns, int levels);
size_t tail_entry_offset(int dim, int G, const int *ns, int levels, size_t es);
size_t tail_lds_bytes(int dim, int G, const int *ns, int levels, int entries, size_t es);
template <typename T>
hipError_t tail_prepare(int dim, int G, size_t lds_bytes);
template <typename T>
hipError_t launch_tail(int dim, int G, const TailArgs &args, size_t lds_bytes, hipStream_t s,
                       int slots = 1);

// The 3D tail of line passes (tail3d.hip): a 17^3 level whose operator is given by its 1D
// factors, and the 9^3 coarsest level solved by sine transforms.
constexpr int kTail3Side = 17, kTail3Coarse = 9;
struct Tail3Args {
  int nu1, nu2, prolong, zero_init, repeats;
  int rb;                // 1: red-black Jacobi sweeps, 0: omega-Jacobi
  double om_d;           // omega / diagonal of the 17^3 operator
  double a[7], b[7];     // its 1D factors
  const double *dst;     // 9^3 sine table (7 x 7), then the 343 per-mode factors
  const void *f_top;
  void *u_top;
  const int *done;
};
size_t tail3_lds_bytes(size_t es);
template <typename T>
hipError_t tail3_prepare();
template <typename T>
hipError_t launch_tail3(const Tail3Args &args, hipStream_t s, int slots = 1);

}  // namespace mgk
