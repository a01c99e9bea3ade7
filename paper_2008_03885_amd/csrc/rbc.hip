// rbc.hip -- red-black coarsening multigrid in two dimensions (section 4.3 Theorem 3,
// section 4.4), FP64.
//
// Level l lives on the standard grid of spacing 2^(l/2) h that holds it (side m).  An odd
// level is rotated: its points are those with an even index sum, and its arrays keep only
// them, row i holding (i, j) at column j/2 (row pitch (m + 1)/2; the odd rows' last entry
// is padding and stays zero).  Every
// level's operator is a symmetric stencil of at most four coefficients on that storage
// grid: centre, axis neighbours at distance 1, diagonal neighbours, axis neighbours at
// distance 2.  The omega-Jacobi partial steps and the interpolation are one thread per
// array entry, reading the few neighbours they need through the caches; the restriction
// forms the defect once per point in an LDS tile; the coarsest level is solved by its
// inverse, formed on the host at set-up and applied in one workgroup.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>

#include "batch.h"
#include "mg_rbc.h"

namespace {

struct Op {
  double c0, a1, d1, a2;  // centre, axis +-1, diagonal, axis +-2
};

constexpr int kBX = 64, kBY = 4;          // one wavefront per storage row segment
constexpr int kMaxCoarseSide = 17;        // storage side of the largest coarsest level
constexpr int kNormBlocks = 1024;

__device__ __forceinline__ bool interior(int m, int i, int j) {
  return i > 0 && j > 0 && i < m - 1 && j < m - 1;
}
__device__ __forceinline__ bool unknown(bool odd, int m, int i, int j) {
  return interior(m, i, j) && (!odd || ((i + j) & 1) == 0);
}
// C points stay on the next level: even index sum on an even level, both even on an odd one.
__device__ __forceinline__ bool cpoint(bool odd, int i, int j) {
  return odd ? (((i | j) & 1) == 0) : (((i + j) & 1) == 0);
}

// u(i, j) with the odd reflection about the boundary lines; at most one index is outside
// [0, m) and by at most one point (the distance-2 taps of an interior point).
__device__ __forceinline__ double tap(const double *u, int m, int i, int j) {
  if (i < 0) return 2.0 * u[j] - u[(size_t)(-i) * m + j];
  if (i >= m) return 2.0 * u[(size_t)(m - 1) * m + j] - u[(size_t)(2 * (m - 1) - i) * m + j];
  if (j < 0) return 2.0 * u[(size_t)i * m] - u[(size_t)i * m - j];
  if (j >= m) return 2.0 * u[(size_t)i * m + m - 1] - u[(size_t)i * m + 2 * (m - 1) - j];
  return u[(size_t)i * m + j];
}

// L u at an interior point.
__device__ __forceinline__ double apply_op(const double *u, int m, int i, int j, const Op &op) {
  const size_t p = (size_t)i * m + j;
  double v = op.c0 * u[p];
  if (op.a1 != 0.0) v += op.a1 * ((u[p - m] + u[p + m]) + (u[p - 1] + u[p + 1]));
  if (op.d1 != 0.0)
    v += op.d1 * ((u[p - m - 1] + u[p - m + 1]) + (u[p + m - 1] + u[p + m + 1]));
  if (op.a2 != 0.0)
    v += op.a2 * ((tap(u, m, i - 2, j) + tap(u, m, i + 2, j)) +
                  (tap(u, m, i, j - 2) + tap(u, m, i, j + 2)));
  return v;
}

__host__ __device__ __forceinline__ int rot_pitch(int m) { return (m + 1) / 2; }

// The point-wise kernels run on a 1D grid of gx-wide rows of kBX x kBY tiles.  Blocks are
// dealt round-robin to the eight XCDs, each with its own L2; the remap gives every XCD a
// contiguous run of tiles in raster order, so tile rows that share halo rows meet in the
// same L2.  The first 8 * (total / 8) blocks are remapped, the rest keep their place.
__device__ __forceinline__ void xcd_tile(int gx, int total, int &tx, int &ty) {
  int b = blockIdx.x;
  const int q = total / 8;
  if (b < 8 * q) b = (b % 8) * q + b / 8;
  tx = b % gx;
  ty = b / gx;
}

// A point of a rotated level's packed array beyond the boundary lines by at most one
// point: minus its mirror image (rotated levels are coarse, with zero boundary values).
__device__ __forceinline__ double rot_tap(const double *u, int m, int w, int a, int b) {
  if (a < 0) return -u[(size_t)(-a) * w + (b >> 1)];
  if (a >= m) return -u[(size_t)(2 * (m - 1) - a) * w + (b >> 1)];
  if (b < 0) return -u[(size_t)a * w + ((-b) >> 1)];
  if (b >= m) return -u[(size_t)a * w + ((2 * (m - 1) - b) >> 1)];
  return u[(size_t)a * w + (b >> 1)];
}

// L u at an interior point of a rotated level (packed, pitch w): the diagonal taps and
// the axis taps at distance 2 (the axis-1 coefficient of a rotated level is zero).
__device__ __forceinline__ double apply_rot(const double *u, int m, int w, int i, int j,
                                            const Op &op) {
  const int jl = (j - 1) >> 1, jr = (j + 1) >> 1;
  const size_t up = (size_t)(i - 1) * w, dn = (size_t)(i + 1) * w;
  double v = op.c0 * u[(size_t)i * w + (j >> 1)];
  v += op.d1 * ((u[up + jl] + u[up + jr]) + (u[dn + jl] + u[dn + jr]));
  if (op.a2 != 0.0)
    v += op.a2 * ((rot_tap(u, m, w, i - 2, j) + rot_tap(u, m, w, i + 2, j)) +
                  (rot_tap(u, m, w, i, j - 2) + rot_tap(u, m, w, i, j + 2)));
  return v;
}

// One omega-Jacobi partial step on the F points (colour 1) or the C points (colour 2) at
// array entry (i, k) of a level: column k = j of a standard level, or the packed column of
// a rotated one (point (i, 2k + (i & 1)); padding entries are copied).
template <bool ODD>
__device__ __forceinline__ void smooth_entry(const double *__restrict__ f, const double *__restrict__ uin,
                                             double *__restrict__ uout, int m, const Op &op, int colour,
                                             double omega, int i, int k) {
  const int w = ODD ? rot_pitch(m) : m;
  const int j = ODD ? 2 * k + (i & 1) : k;
  const size_t p = (size_t)i * w + k;
  double v = uin[p];
  if (j < m && unknown(ODD, m, i, j) && cpoint(ODD, i, j) == (colour == 2))
    v += omega * (f[p] - (ODD ? apply_rot(uin, m, w, i, j, op) : apply_op(uin, m, i, j, op))) / op.c0;
  uout[p] = v;
}

// The partial step over a standard level, one thread per entry.
__global__ __launch_bounds__(kBX *kBY) void k_rbc_smooth(const double *__restrict__ f,
                                                         const double *__restrict__ uin,
                                                         double *__restrict__ uout, int m,
                                                         Op op, int colour, double omega,
                                                         int gx, int total) {
  int tx, ty;
  xcd_tile(gx, total, tx, ty);
  const int j = tx * kBX + threadIdx.x;
  const int i = ty * kBY + threadIdx.y;
  if (i >= m || j >= m) return;
  smooth_entry<false>(f, uin, uout, m, op, colour, omega, i, j);
}

// The same on a rotated level, one thread per packed entry.
__global__ __launch_bounds__(kBX *kBY) void k_rbc_smooth_rot(const double *__restrict__ f,
                                                             const double *__restrict__ uin,
                                                             double *__restrict__ uout, int m,
                                                             Op op, int colour, double omega,
                                                             int gx, int total) {
  int tx, ty;
  xcd_tile(gx, total, tx, ty);
  const int k = tx * kBX + threadIdx.x;
  const int i = ty * kBY + threadIdx.y;
  if (i >= m || k >= rot_pitch(m)) return;
  smooth_entry<true>(f, uin, uout, m, op, colour, omega, i, k);
}

// Defect restricted with eq. transfer_r2 onto the next level's storage grid (side mc),
// zero off the next level's unknowns; uc (may be null) is zeroed, the next level starting
// from a zero correction.  A block takes a kRTY x kRTX tile of level l's storage grid:
// u with a 3-point halo (the defect one point outside the tile reaches two further) goes
// to LDS, with the odd reflection written into the halo beyond the boundary lines; the
// defect over the tile and a 1-point ring is formed once in LDS; each C point of the tile
// then gathers itself and its four F neighbours.
constexpr int kRTX = 64, kRTY = 16;

template <bool ODD>
__global__ __launch_bounds__(256) void k_rbc_restrict(const double *__restrict__ f,
                                                      const double *__restrict__ u,
                                                      double *__restrict__ fc,
                                                      double *__restrict__ uc, int m, Op op,
                                                      int mc) {
  constexpr int UX = kRTX + 6, UY = kRTY + 6, RX = kRTX + 2, RY = kRTY + 2;
  __shared__ double su[UY][UX];
  __shared__ double sr[RY][RX];
  const int t = threadIdx.x;
  const int i0 = blockIdx.y * kRTY, j0 = blockIdx.x * kRTX;
  const int w = ODD ? rot_pitch(m) : m;  // pitch of this level's arrays
  for (int q = t; q < UY * UX; q += 256) {
    const int a = i0 - 3 + q / UX, b = j0 - 3 + q % UX;
    const bool ain = a >= 0 && a < m, bin = b >= 0 && b < m;
    const bool near = (ain && (b == -1 || b == m)) || (bin && (a == -1 || a == m));
    double v = 0.0;  // never read unless one index is at most one point outside
    if (ODD) {
      if (((a + b) & 1) == 0 && ((ain && bin) || near)) v = rot_tap(u, m, w, a, b);
    } else if (ain && bin) {
      v = u[(size_t)a * m + b];
    } else if (near) {
      v = tap(u, m, a, b);
    }
    su[q / UX][q % UX] = v;
  }
  __syncthreads();
  for (int q = t; q < RY * RX; q += 256) {
    const int x = q / RX, y = q % RX;  // sr[x][y] is the point (i0 - 1 + x, j0 - 1 + y)
    const int a = i0 - 1 + x, b = j0 - 1 + y;
    double r = 0.0;
    if (unknown(ODD, m, a, b)) {
      const int X = x + 2, Y = y + 2;  // the same point in su
      double v = op.c0 * su[X][Y];
      if (op.a1 != 0.0) v += op.a1 * ((su[X - 1][Y] + su[X + 1][Y]) + (su[X][Y - 1] + su[X][Y + 1]));
      if (op.d1 != 0.0)
        v += op.d1 * ((su[X - 1][Y - 1] + su[X - 1][Y + 1]) + (su[X + 1][Y - 1] + su[X + 1][Y + 1]));
      if (op.a2 != 0.0)
        v += op.a2 * ((su[X - 2][Y] + su[X + 2][Y]) + (su[X][Y - 2] + su[X][Y + 2]));
      r = f[(size_t)a * w + (ODD ? b >> 1 : b)] - v;
    }
    sr[x][y] = r;
  }
  __syncthreads();
  if (ODD) {
    // coarse point (I, J) sits at fine (2I, 2J); its F neighbours are the diagonals
    for (int q = t; q < (kRTY / 2) * (kRTX / 2); q += 256) {
      const int I = i0 / 2 + q / (kRTX / 2), J = j0 / 2 + q % (kRTX / 2);
      if (I >= mc || J >= mc) continue;
      double v = 0.0;
      if (unknown(false, mc, I, J)) {
        const int x = 2 * I - i0 + 1, y = 2 * J - j0 + 1;
        v = (4.0 * sr[x][y] + ((sr[x - 1][y - 1] + sr[x - 1][y + 1]) + (sr[x + 1][y - 1] + sr[x + 1][y + 1]))) *
            0.125;
      }
      fc[(size_t)I * mc + J] = v;
      if (uc) uc[(size_t)I * mc + J] = 0.0;
    }
  } else {
    // the next (rotated) level's points are this grid's even-index-sum points, packed;
    // F neighbours are the axis ones
    const int wc = rot_pitch(m);
    for (int q = t; q < kRTY * kRTX; q += 256) {
      const int a = i0 + q / kRTX, b = j0 + q % kRTX;
      if (a >= m || b >= m || ((a + b) & 1)) continue;
      double v = 0.0;
      if (unknown(true, m, a, b)) {
        const int x = a - i0 + 1, y = b - j0 + 1;
        v = (4.0 * sr[x][y] + ((sr[x - 1][y] + sr[x + 1][y]) + (sr[x][y - 1] + sr[x][y + 1]))) * 0.125;
      }
      fc[(size_t)a * wc + (b >> 1)] = v;
      if (uc) uc[(size_t)a * wc + (b >> 1)] = 0.0;
    }
  }
}

// u_out = u_in + interpolated correction at array entry (i, k): C points take the coarse
// value, F points the mean of their four C neighbours (eq. transfer_r2).  A standard level
// (side m) takes the correction from the rotated level below, packed with pitch
// (m + 1)/2, along the axes; a rotated level (packed) from the standard level below (side
// mc) along the diagonals, its C points having both indices even.
template <bool ODD>
__device__ __forceinline__ void prolong_entry(const double *__restrict__ ec, const double *uin, double *uout,
                                              int m, int mc, int i, int k) {
  const int w = ODD ? rot_pitch(m) : m;
  const int j = ODD ? 2 * k + (i & 1) : k;
  const size_t p = (size_t)i * w + k;
  double v = uin[p];
  if (j < m && unknown(ODD, m, i, j)) {
    if (ODD) {
      auto e = [&](int a, int b) { return ec[(size_t)(a >> 1) * mc + (b >> 1)]; };
      if (cpoint(true, i, j))
        v += e(i, j);
      else
        v += 0.25 * ((e(i - 1, j - 1) + e(i - 1, j + 1)) + (e(i + 1, j - 1) + e(i + 1, j + 1)));
    } else {
      const int wc = rot_pitch(m);
      auto e = [&](int a, int b) { return ec[(size_t)a * wc + (b >> 1)]; };  // a + b even
      if (cpoint(false, i, j))
        v += e(i, j);
      else
        v += 0.25 * ((e(i - 1, j) + e(i + 1, j)) + (e(i, j - 1) + e(i, j + 1)));
    }
  }
  uout[p] = v;
}

__global__ __launch_bounds__(kBX *kBY) void k_rbc_prolong(const double *__restrict__ ec,
                                                          const double *uin, double *uout,
                                                          int m, int gx, int total) {
  int tx, ty;
  xcd_tile(gx, total, tx, ty);
  const int j = tx * kBX + threadIdx.x;
  const int i = ty * kBY + threadIdx.y;
  if (i >= m || j >= m) return;
  prolong_entry<false>(ec, uin, uout, m, 0, i, j);
}

__global__ __launch_bounds__(kBX *kBY) void k_rbc_prolong_rot(const double *__restrict__ ec,
                                                              const double *uin, double *uout,
                                                              int m, int mc, int gx, int total) {
  int tx, ty;
  xcd_tile(gx, total, tx, ty);
  const int k = tx * kBX + threadIdx.x;
  const int i = ty * kBY + threadIdx.y;
  if (i >= m || k >= rot_pitch(m)) return;
  prolong_entry<true>(ec, uin, uout, m, mc, i, k);
}

// Exact solve of the coarsest level: u = A^{-1} f over its K unknowns, with the inverse
// formed once at set-up (transposed, so that for each column the threads of a row range
// read consecutive entries) and pos[] giving each unknown's array index.  Every other
// entry of u (boundary, padding) is set to zero.  f is read whole into LDS before any
// entry of u is written, so f may be the same array as u.  One 1024-thread workgroup:
// four threads share a row, each summing every fourth column, then the four sums are
// added.
__device__ __forceinline__ void coarsest_solve(const double *f, double *u, const double *__restrict__ ainv_t,
                                               const int *__restrict__ pos, int K, int entries) {
  constexpr int K_MAX = MG_RBC_MAX_COARSEST;
  static_assert(4 * K_MAX == 1024, "four threads per row of the inverse fill the workgroup");
  __shared__ double fs[K_MAX];
  __shared__ double part[4][K_MAX];
  const int t = threadIdx.x;
  for (int c = t; c < K; c += 1024) fs[c] = f[pos[c]];
  __syncthreads();
  for (int p = t; p < entries; p += 1024) u[p] = 0.0;
  const int r = t % K_MAX, q = t / K_MAX;
  if (r < K) {
    // eight independent partial sums keep eight loads in flight
    double a[8] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    int c = q;
    for (; c + 28 < K; c += 32) {
#pragma unroll
      for (int v = 0; v < 8; ++v) a[v] += ainv_t[(size_t)(c + 4 * v) * K + r] * fs[c + 4 * v];
    }
    for (; c < K; c += 4) a[0] += ainv_t[(size_t)c * K + r] * fs[c];
    part[q][r] = ((a[0] + a[1]) + (a[2] + a[3])) + ((a[4] + a[5]) + (a[6] + a[7]));
  }
  __syncthreads();
  if (t < K) u[pos[t]] = (part[0][t] + part[1][t]) + (part[2][t] + part[3][t]);
}

__global__ __launch_bounds__(1024) void k_rbc_coarsest(const double *f, double *u,
                                                       const double *__restrict__ ainv_t,
                                                       const int *__restrict__ pos, int K,
                                                       int entries) {
  coarsest_solve(f, u, ainv_t, pos, K, entries);
}

// ------------------------------------------------------------- small-level tail ----
// The levels from a side of at most 33 (by default) down to the coarsest run in one
// 1024-thread workgroup: the same partial steps, interpolation and coarsest solve as the
// per-level kernels (the same device functions), the restriction gathering each coarse
// point's defects directly, one phase after another with a workgroup barrier between
// them.  The small levels' arrays stay in the caches; the tail replaces a launch per
// phase (five or six per level and visit) by a barrier.  Measured at 4097^2 (17 levels,
// G1 V(1,1) cycle): 1.476 ms per-level, 1.456 ms from side 33, 1.477 ms from side 65 and
// 1.662 ms from 129: a phase over a 65^2 level in one workgroup takes as long as a launch.
constexpr int kTailMaxLevels = 8;

struct TailLevel {
  double *f, *u, *t;
  Op op;
  int m, odd;
};

struct TailArgs {
  TailLevel lv[kTailMaxLevels];
  int nl;               // levels in the tail, the last one the coarsest
  int gamma, nu1, nu2;  // cycle
  int visits;           // visits of the tail's top level in a row
  double omega;
  const double *ainv_t;
  const int *pos;
  int K;
};

// The defect at point (a, b) of a level, zero off its unknowns.
template <bool ODD>
__device__ __forceinline__ double defect_at(const double *f, const double *u, int m, const Op &op, int a,
                                            int b) {
  if (!unknown(ODD, m, a, b)) return 0.0;
  if (ODD) {
    const int w = rot_pitch(m);
    return f[(size_t)a * w + (b >> 1)] - apply_rot(u, m, w, a, b, op);
  }
  return f[(size_t)a * m + b] - apply_op(u, m, a, b, op);
}

// Restriction (eq. transfer_r2) from level L onto the next level C, with C's iterate
// zeroed: the weights and sum order of k_rbc_restrict.
__device__ void tail_restrict(const TailLevel &L, const TailLevel &C) {
  const int t = threadIdx.x, m = L.m, mc = C.m;
  if (L.odd) {
    for (int q = t; q < mc * mc; q += 1024) {
      const int I = q / mc, J = q % mc;
      double v = 0.0;
      if (unknown(false, mc, I, J)) {
        const int a = 2 * I, b = 2 * J;
        auto r = [&](int x, int y) { return defect_at<true>(L.f, L.u, m, L.op, x, y); };
        v = (4.0 * r(a, b) + ((r(a - 1, b - 1) + r(a - 1, b + 1)) + (r(a + 1, b - 1) + r(a + 1, b + 1)))) * 0.125;
      }
      C.f[q] = v;
      C.u[q] = 0.0;
    }
  } else {
    const int wc = rot_pitch(m);
    for (int q = t; q < m * wc; q += 1024) {
      const int a = q / wc, b = 2 * (q % wc) + (a & 1);
      if (b >= m) continue;  // padding of an odd row
      double v = 0.0;
      if (unknown(true, m, a, b)) {
        auto r = [&](int x, int y) { return defect_at<false>(L.f, L.u, m, L.op, x, y); };
        v = (4.0 * r(a, b) + ((r(a - 1, b) + r(a + 1, b)) + (r(a, b - 1) + r(a, b + 1)))) * 0.125;
      }
      C.f[q] = v;
      C.u[q] = 0.0;
    }
  }
}

__device__ void tail_smooth(const TailLevel &L, int colour, const double *uin, double *uout, double omega) {
  const int w = L.odd ? rot_pitch(L.m) : L.m, entries = L.m * w;
  for (int q = threadIdx.x; q < entries; q += 1024) {
    if (L.odd)
      smooth_entry<true>(L.f, uin, uout, L.m, L.op, colour, omega, q / w, q % w);
    else
      smooth_entry<false>(L.f, uin, uout, L.m, L.op, colour, omega, q / w, q % w);
  }
  __syncthreads();
}

// A red-black sweep: F points into t, then C points back into u.
__device__ void tail_sweep(const TailLevel &L, double omega) {
  tail_smooth(L, 1, L.u, L.t, omega);
  tail_smooth(L, 2, L.t, L.u, omega);
}

__device__ void tail_prolong(const TailLevel &L, const TailLevel &C) {
  const int w = L.odd ? rot_pitch(L.m) : L.m, entries = L.m * w;
  for (int q = threadIdx.x; q < entries; q += 1024) {
    if (L.odd)
      prolong_entry<true>(C.u, L.u, L.u, L.m, C.m, q / w, q % w);
    else
      prolong_entry<false>(C.u, L.u, L.u, L.m, C.m, q / w, q % w);
  }
  __syncthreads();
}

// The gamma-cycle over the tail's levels without recursion: descending, each level
// smooths and restricts; a finished visit of level l + 1 either starts the next one (the
// second visit of a W-cycle, bit l of `again`) or lets level l interpolate and smooth.
__global__ __launch_bounds__(1024) void k_rbc_tail(TailArgs a) {
  const int last = a.nl - 1;
  for (int v = 0; v < a.visits; ++v) {
    int l = 0;
    bool down = true;
    unsigned again = 0u;
    while (true) {
      if (down) {
        if (l == last) {
          const TailLevel &C = a.lv[l];
          coarsest_solve(C.f, C.u, a.ainv_t, a.pos, a.K, C.m * (C.odd ? rot_pitch(C.m) : C.m));
          __syncthreads();
          down = false;
          continue;
        }
        for (int k = 0; k < a.nu1; ++k) tail_sweep(a.lv[l], a.omega);
        tail_restrict(a.lv[l], a.lv[l + 1]);
        __syncthreads();
        again &= ~(1u << l);
        ++l;
        continue;
      }
      if (l == 0) break;  // the top level's visit is complete
      const int p = l - 1;
      if (p + 1 < last && a.gamma == 2 && !((again >> p) & 1u)) {
        again |= 1u << p;
        down = true;  // a second visit of level p + 1
        continue;
      }
      tail_prolong(a.lv[p], a.lv[p + 1]);
      for (int k = 0; k < a.nu2; ++k) tail_sweep(a.lv[p], a.omega);
      l = p;
    }
  }
}

// Per-block sums of the squared level-0 defect over the interior.
__global__ __launch_bounds__(256) void k_rbc_resnorm(const double *__restrict__ f,
                                                     const double *__restrict__ u, int m, Op op,
                                                     double *__restrict__ partial) {
  __shared__ double red[256];
  double s = 0.0;
  // block b takes interior rows b + 1, b + 1 + gridDim.x, ...; its threads stride the row
  for (int i = 1 + blockIdx.x; i < m - 1; i += gridDim.x)
    for (int j = 1 + threadIdx.x; j < m - 1; j += blockDim.x) {
      const double r = f[(size_t)i * m + j] - apply_op(u, m, i, j, op);
      s += r * r;
    }
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) partial[blockIdx.x] = red[0];
}

__global__ __launch_bounds__(256) void k_rbc_sum(const double *__restrict__ partial, int count,
                                                 double scale, double *__restrict__ out) {
  __shared__ double red[256];
  double s = 0.0;
  for (int q = threadIdx.x; q < count; q += blockDim.x) s += partial[q];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[0] = sqrt(red[0] * scale);
}

struct Level {
  int m;
  bool odd;
  Op op;
  int unknowns;
};

mg_status fail(mg_status st, const std::string &msg) {
  mgb::set_error(msg);
  return st;
}

#define RBC_HIP(call)                                                                     \
  do {                                                                                    \
    hipError_t e_ = (call);                                                               \
    if (e_ != hipSuccess)                                                                 \
      return fail(MG_EDEVICE, std::string(#call) + ": " + hipGetErrorString(e_));         \
  } while (0)

int storage_side(int n, int l) { return (n - 1) / (1 << (l / 2)) + 1; }

int count_unknowns(int m, bool odd) {
  int k = 0;
  for (int i = 1; i < m - 1; ++i)
    for (int j = 1; j < m - 1; ++j) k += !odd || ((i + j) % 2 == 0);
  return k;
}

// Level l's stencil on its storage grid of spacing s: the five-point operator on the
// level's own axes, or eq. L_G1 for the Galerkin choices; an odd level's axes are the
// storage diagonals and its H^2 = 2 s^2.
Op level_op(const mg_rbc_config &c, int l) {
  const double s = std::ldexp(1.0 / (c.n - 1), l / 2), s2 = s * s;
  const bool g1 = l > 0 && (c.coarse == MG_RBC_G1 || (c.coarse == MG_RBC_GN && l == 1));
  if (l % 2 == 0) {
    if (!g1) return Op{4.0 / s2, -1.0 / s2, 0.0, 0.0};
    return Op{3.0 / s2, -0.5 / s2, -0.25 / s2, 0.0};
  }
  const double H2 = 2.0 * s2;
  if (!g1) return Op{4.0 / H2, 0.0, -1.0 / H2, 0.0};
  return Op{3.0 / H2, 0.0, -0.5 / H2, -0.25 / H2};
}

// Entries of a level's arrays: m^2, or m rows of (m + 1)/2 on a rotated level.
size_t level_entries(const Level &L) { return (size_t)L.m * (L.odd ? rot_pitch(L.m) : L.m); }

// The coarsest level's operator as a dense K x K matrix over its unknowns (row-major
// storage order), each stencil tap beyond the boundary line folded onto its mirror image
// with the opposite sign (zero boundary values), and its inverse by Gauss-Jordan
// elimination with partial pivoting; inv_t is the inverse transposed.  Returns false if
// the matrix is singular.  pos gets each unknown's index in the level's arrays.
bool coarsest_inverse(const Level &L, std::vector<double> &inv_t, std::vector<int> &pos) {
  const int m = L.m, w = L.odd ? rot_pitch(m) : m;
  std::vector<int> idx((size_t)m * m, -1);
  pos.clear();
  for (int i = 1; i < m - 1; ++i)
    for (int j = 1; j < m - 1; ++j)
      if (!L.odd || (i + j) % 2 == 0) {
        idx[(size_t)i * m + j] = (int)pos.size();
        pos.push_back(i * w + (L.odd ? j / 2 : j));
      }
  const int K = (int)pos.size();
  std::vector<double> A((size_t)K * K, 0.0), X((size_t)K * K, 0.0);
  const Op &op = L.op;
  for (int i = 1; i < m - 1; ++i)
    for (int j = 1; j < m - 1; ++j) {
      const int row = idx[(size_t)i * m + j];
      if (row < 0) continue;
      auto add = [&](int a, int c, double wgt) {
        if (a < 0 || a >= m || c < 0 || c >= m) {
          wgt = -wgt;
          a = a < 0 ? -a : (a >= m ? 2 * (m - 1) - a : a);
          c = c < 0 ? -c : (c >= m ? 2 * (m - 1) - c : c);
        }
        const int col = idx[(size_t)a * m + c];
        if (col >= 0) A[(size_t)row * K + col] += wgt;
      };
      add(i, j, op.c0);
      if (op.a1 != 0.0) {
        add(i - 1, j, op.a1); add(i + 1, j, op.a1); add(i, j - 1, op.a1); add(i, j + 1, op.a1);
      }
      if (op.d1 != 0.0) {
        add(i - 1, j - 1, op.d1); add(i - 1, j + 1, op.d1);
        add(i + 1, j - 1, op.d1); add(i + 1, j + 1, op.d1);
      }
      if (op.a2 != 0.0) {
        add(i - 2, j, op.a2); add(i + 2, j, op.a2); add(i, j - 2, op.a2); add(i, j + 2, op.a2);
      }
    }
  for (int r = 0; r < K; ++r) X[(size_t)r * K + r] = 1.0;
  for (int k = 0; k < K; ++k) {
    int piv = k;
    for (int r = k + 1; r < K; ++r)
      if (std::fabs(A[(size_t)r * K + k]) > std::fabs(A[(size_t)piv * K + k])) piv = r;
    if (A[(size_t)piv * K + k] == 0.0) return false;
    if (piv != k)
      for (int c = 0; c < K; ++c) {
        std::swap(A[(size_t)k * K + c], A[(size_t)piv * K + c]);
        std::swap(X[(size_t)k * K + c], X[(size_t)piv * K + c]);
      }
    const double d = 1.0 / A[(size_t)k * K + k];
    for (int c = 0; c < K; ++c) {
      A[(size_t)k * K + c] *= d;
      X[(size_t)k * K + c] *= d;
    }
    for (int r = 0; r < K; ++r) {
      const double g = A[(size_t)r * K + k];
      if (r == k || g == 0.0) continue;
      for (int c = 0; c < K; ++c) {
        A[(size_t)r * K + c] -= g * A[(size_t)k * K + c];
        X[(size_t)r * K + c] -= g * X[(size_t)k * K + c];
      }
    }
  }
  inv_t.assign((size_t)K * K, 0.0);
  for (int r = 0; r < K; ++r)
    for (int c = 0; c < K; ++c) inv_t[(size_t)c * K + r] = X[(size_t)r * K + c];
  return true;
}



}  // namespace

struct mg_rbc_ctx {
  mg_rbc_config cfg;
  hipStream_t stream = nullptr;
  std::vector<Level> lv;
  std::vector<double *> u, f, t;  // per level; u[0], f[0] are the caller's
  double *partial = nullptr, *norm_dev = nullptr, *norm_host = nullptr;
  double *ainv_t = nullptr;  // the coarsest operator's inverse, transposed (K x K)
  int *pos = nullptr;        // array index of each coarsest unknown
  int coarse_k = 0;
  int tail_top = 1 << 30;    // first level of the one-workgroup tail (none: past the last)
};

namespace {

std::string validate(const mg_rbc_config &c) {
  const int N = c.n - 1;
  if (c.n < 3 || c.n > 32769 || (N & (N - 1)) != 0) return "n - 1 must be a power of two, 3 <= n <= 32769";
  if (c.coarse < MG_RBC_NG || c.coarse > MG_RBC_GN) return "coarse must be MG_RBC_NG, MG_RBC_G1 or MG_RBC_GN";
  if (c.gamma < 1 || c.gamma > 2) return "gamma must be 1 or 2";
  if (c.nu1 < 0 || c.nu2 < 0 || c.nu1 > 8 || c.nu2 > 8 || c.nu1 + c.nu2 < 1)
    return "nu1, nu2 must be in 0..8 with at least one sweep";
  if (!(c.omega == 0.0 || (c.omega > 0.0 && c.omega < 2.0))) return "omega must be 0 (default) or in (0, 2)";
  if (!(c.rtol >= 0.0)) return "rtol must be >= 0";
  if (c.max_cycles < 1 || c.max_cycles > MG_MAX_HISTORY) return "max_cycles must be in 1..MG_MAX_HISTORY";
  if (c.levels < 2) return "levels must be >= 2";
  for (int l = 1; l < c.levels; ++l) {
    if (storage_side(c.n, l) < 3 || (N % (1 << (l / 2))) != 0) return "too many levels for n";
  }
  const int last = c.levels - 1;
  const int mc = storage_side(c.n, last);
  const int k = count_unknowns(mc, last % 2 == 1);
  if (mc > kMaxCoarseSide || k < 1 || k > MG_RBC_MAX_COARSEST)
    return "the coarsest level has " + std::to_string(k) + " unknowns (1..MG_RBC_MAX_COARSEST allowed); add levels";
  return "";
}

mg_status launch_smooth(mg_rbc_ctx *h, int l, int colour, const double *f, const double *uin,
                        double *uout) {
  const Level &L = h->lv[l];
  const double omega = h->cfg.omega == 0.0 ? 1.0 : h->cfg.omega;
  const int gx = ((L.odd ? rot_pitch(L.m) : L.m) + kBX - 1) / kBX, total = gx * ((L.m + kBY - 1) / kBY);
  if (L.odd)
    hipLaunchKernelGGL(k_rbc_smooth_rot, dim3(total), dim3(kBX, kBY), 0, h->stream, f, uin, uout, L.m,
                       L.op, colour, omega, gx, total);
  else
    hipLaunchKernelGGL(k_rbc_smooth, dim3(total), dim3(kBX, kBY), 0, h->stream, f, uin, uout, L.m, L.op,
                       colour, omega, gx, total);
  RBC_HIP(hipGetLastError());
  return MG_OK;
}

mg_status launch_restrict(mg_rbc_ctx *h, int l, const double *f, const double *u, double *fc,
                          double *uc) {
  const Level &L = h->lv[l];
  const int mc = h->lv[l + 1].m;
  const dim3 grid((L.m + kRTX - 1) / kRTX, (L.m + kRTY - 1) / kRTY);
  if (L.odd)
    hipLaunchKernelGGL(k_rbc_restrict<true>, grid, dim3(256), 0, h->stream, f, u, fc, uc, L.m, L.op, mc);
  else
    hipLaunchKernelGGL(k_rbc_restrict<false>, grid, dim3(256), 0, h->stream, f, u, fc, uc, L.m, L.op, mc);
  RBC_HIP(hipGetLastError());
  return MG_OK;
}

mg_status launch_prolong(mg_rbc_ctx *h, int l, const double *ec, const double *uin, double *uout) {
  const Level &L = h->lv[l];
  const int gx = ((L.odd ? rot_pitch(L.m) : L.m) + kBX - 1) / kBX, total = gx * ((L.m + kBY - 1) / kBY);
  if (L.odd)
    hipLaunchKernelGGL(k_rbc_prolong_rot, dim3(total), dim3(kBX, kBY), 0, h->stream, ec, uin, uout, L.m,
                       h->lv[l + 1].m, gx, total);
  else
    hipLaunchKernelGGL(k_rbc_prolong, dim3(total), dim3(kBX, kBY), 0, h->stream, ec, uin, uout, L.m, gx,
                       total);
  RBC_HIP(hipGetLastError());
  return MG_OK;
}

// Levels tail_top .. last in one launch, the top level's arrays f and u, visited `visits`
// times in a row.
mg_status launch_tail(mg_rbc_ctx *h, const double *f, double *u, int visits) {
  const int top = h->tail_top, last = (int)h->lv.size() - 1;
  TailArgs a{};
  a.nl = last - top + 1;
  for (int i = 0; i < a.nl; ++i) {
    const Level &L = h->lv[top + i];
    a.lv[i] = TailLevel{i == 0 ? const_cast<double *>(f) : h->f[top + i], i == 0 ? u : h->u[top + i],
                        h->t[top + i], L.op, L.m, L.odd ? 1 : 0};
  }
  a.gamma = h->cfg.gamma;
  a.nu1 = h->cfg.nu1;
  a.nu2 = h->cfg.nu2;
  a.visits = visits;
  a.omega = h->cfg.omega == 0.0 ? 1.0 : h->cfg.omega;
  a.ainv_t = h->ainv_t;
  a.pos = h->pos;
  a.K = h->coarse_k;
  hipLaunchKernelGGL(k_rbc_tail, dim3(1), dim3(1024), 0, h->stream, a);
  RBC_HIP(hipGetLastError());
  return MG_OK;
}

mg_status launch_coarsest(mg_rbc_ctx *h, const double *f, double *u) {
  hipLaunchKernelGGL(k_rbc_coarsest, dim3(1), dim3(1024), 0, h->stream, f, u, h->ainv_t, h->pos,
                     h->coarse_k, (int)level_entries(h->lv.back()));
  RBC_HIP(hipGetLastError());
  return MG_OK;
}

#define RBC_TRY(x)                  \
  do {                              \
    mg_status s_ = (x);             \
    if (s_ != MG_OK) return s_;     \
  } while (0)

mg_status sweep(mg_rbc_ctx *h, int l, const double *f, double *u) {
  RBC_TRY(launch_smooth(h, l, 1, f, u, h->t[l]));
  return launch_smooth(h, l, 2, f, h->t[l], u);
}

mg_status cycle(mg_rbc_ctx *h, int l, const double *f, double *u) {
  const int last = (int)h->lv.size() - 1;
  if (l == h->tail_top) return launch_tail(h, f, u, 1);
  if (l == last) return launch_coarsest(h, f, u);
  for (int k = 0; k < h->cfg.nu1; ++k) RBC_TRY(sweep(h, l, f, u));
  RBC_TRY(launch_restrict(h, l, f, u, h->f[l + 1], h->u[l + 1]));
  const int reps = l + 1 < last ? h->cfg.gamma : 1;
  if (l + 1 == h->tail_top)  // the visits of the tail's top level in one launch
    RBC_TRY(launch_tail(h, h->f[l + 1], h->u[l + 1], reps));
  else
    for (int k = 0; k < reps; ++k) RBC_TRY(cycle(h, l + 1, h->f[l + 1], h->u[l + 1]));
  RBC_TRY(launch_prolong(h, l, h->u[l + 1], u, u));
  for (int k = 0; k < h->cfg.nu2; ++k) RBC_TRY(sweep(h, l, f, u));
  return MG_OK;
}

mg_status norm(mg_rbc_ctx *h, const double *f, const double *u, double *out) {
  const Level &L = h->lv[0];
  const size_t ni = (size_t)(L.m - 2) * (L.m - 2);
  const int blocks = std::min(kNormBlocks, L.m - 2);  // a block takes whole interior rows
  hipLaunchKernelGGL(k_rbc_resnorm, dim3(blocks), dim3(256), 0, h->stream, f, u, L.m, L.op, h->partial);
  RBC_HIP(hipGetLastError());
  hipLaunchKernelGGL(k_rbc_sum, dim3(1), dim3(256), 0, h->stream, h->partial, blocks, 1.0 / (double)ni,
                     h->norm_dev);
  RBC_HIP(hipGetLastError());
  RBC_HIP(hipMemcpyAsync(h->norm_host, h->norm_dev, sizeof(double), hipMemcpyDeviceToHost, h->stream));
  RBC_HIP(hipStreamSynchronize(h->stream));
  *out = *h->norm_host;
  return MG_OK;
}

mg_status check_level(const mg_rbc_ctx *h, int level, bool need_next) {
  if (!h) return fail(MG_EINVAL, "null handle");
  if (level < 0 || level >= (int)h->lv.size() || (need_next && level + 1 >= (int)h->lv.size()))
    return fail(MG_EINVAL, "level out of range");
  return MG_OK;
}

}  // namespace

extern "C" {

mg_status mg_rbc_setup(const mg_rbc_config *cfg, void *stream, mg_rbc_ctx **out) {
  if (!cfg || !out) return fail(MG_EINVAL, "null argument");
  *out = nullptr;
  const std::string why = validate(*cfg);
  if (!why.empty()) return fail(MG_EINVAL, why);
  mg_rbc_ctx *h = new mg_rbc_ctx();
  h->cfg = *cfg;
  h->stream = (hipStream_t)stream;
  for (int l = 0; l < cfg->levels; ++l) {
    Level L;
    L.m = storage_side(cfg->n, l);
    L.odd = l % 2 == 1;
    L.op = level_op(*cfg, l);
    L.unknowns = count_unknowns(L.m, L.odd);
    h->lv.push_back(L);
  }
  auto alloc = [&](double **p, size_t count) {
    return hipMalloc((void **)p, count * sizeof(double)) == hipSuccess;
  };
  bool ok = true;
  h->u.assign(cfg->levels, nullptr);
  h->f.assign(cfg->levels, nullptr);
  h->t.assign(cfg->levels, nullptr);
  for (int l = 0; l < cfg->levels && ok; ++l) {
    const size_t cnt = level_entries(h->lv[l]);
    if (l > 0) ok = ok && alloc(&h->u[l], cnt) && alloc(&h->f[l], cnt);
    ok = ok && alloc(&h->t[l], cnt);
  }
  ok = ok && alloc(&h->partial, kNormBlocks) && alloc(&h->norm_dev, 1);
  std::vector<double> inv_t;
  std::vector<int> pos;
  if (ok && !coarsest_inverse(h->lv.back(), inv_t, pos)) {
    mg_rbc_destroy(h);
    return fail(MG_EINVAL, "the coarsest level's operator is singular");
  }
  h->coarse_k = (int)pos.size();
  ok = ok && alloc(&h->ainv_t, inv_t.size()) &&
       hipMalloc((void **)&h->pos, pos.size() * sizeof(int)) == hipSuccess;
  ok = ok && hipHostMalloc((void **)&h->norm_host, sizeof(double), hipHostMallocDefault) == hipSuccess;
  if (!ok) {
    mg_rbc_destroy(h);
    return fail(MG_ENOMEM, "device allocation failed");
  }
  // the set-up copies are synchronous: inv_t and pos are freed on return
  if (hipMemcpy(h->ainv_t, inv_t.data(), inv_t.size() * sizeof(double), hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(h->pos, pos.data(), pos.size() * sizeof(int), hipMemcpyHostToDevice) != hipSuccess) {
    mg_rbc_destroy(h);
    return fail(MG_EDEVICE, "copying the coarsest inverse failed");
  }
  // the one-workgroup tail: from the first level of side <= MG_RBC_TAIL (default 33; 0
  // switches it off) to the coarsest, at least two levels and at most kTailMaxLevels
  {
    const char *e = getenv("MG_RBC_TAIL");
    const int side = e != nullptr && *e != 0 ? atoi(e) : 33;
    const int last = cfg->levels - 1;
    int top = 0;
    while (top <= last && h->lv[top].m > side) ++top;
    top = std::max(top, last + 1 - kTailMaxLevels);
    if (side > 0 && top < last) h->tail_top = top;
  }
  // every level array starts at zero: their boundaries and off-grid entries stay zero
  for (int l = 1; l < cfg->levels; ++l) {
    const size_t bytes = level_entries(h->lv[l]) * sizeof(double);
    hipError_t e = hipMemsetAsync(h->u[l], 0, bytes, h->stream);
    if (e == hipSuccess) e = hipMemsetAsync(h->f[l], 0, bytes, h->stream);
    if (e == hipSuccess) e = hipMemsetAsync(h->t[l], 0, bytes, h->stream);
    if (e != hipSuccess) {
      mg_rbc_destroy(h);
      return fail(MG_EDEVICE, std::string("hipMemsetAsync: ") + hipGetErrorString(e));
    }
  }
  *out = h;
  return MG_OK;
}

void mg_rbc_destroy(mg_rbc_ctx *h) {
  if (!h) return;
  // teardown: errors here have no caller to go to
  (void)(h->stream ? hipStreamSynchronize(h->stream) : hipDeviceSynchronize());
  auto release = [](double *p) {
    if (p) (void)hipFree(p);
  };
  for (double *p : h->u) release(p);
  for (double *p : h->f) release(p);
  for (double *p : h->t) release(p);
  release(h->partial);
  release(h->norm_dev);
  release(h->ainv_t);
  if (h->pos) (void)hipFree(h->pos);
  if (h->norm_host) (void)hipHostFree(h->norm_host);
  delete h;
}

int mg_rbc_level_size(const mg_rbc_ctx *h, int level) {
  if (!h || level < 0 || level >= (int)h->lv.size()) return -1;
  return h->lv[level].m;
}

int mg_rbc_level_pitch(const mg_rbc_ctx *h, int level) {
  if (!h || level < 0 || level >= (int)h->lv.size()) return -1;
  return h->lv[level].odd ? rot_pitch(h->lv[level].m) : h->lv[level].m;
}

mg_status mg_rbc_cycles(mg_rbc_ctx *h, const double *f, double *u, int ncycles) {
  if (!h || !f || !u || ncycles < 0) return fail(MG_EINVAL, "bad argument");
  for (int k = 0; k < ncycles; ++k) RBC_TRY(cycle(h, 0, f, u));
  return MG_OK;
}

mg_status mg_rbc_residual_norm(mg_rbc_ctx *h, const double *f, const double *u, double *out) {
  if (!h || !f || !u || !out) return fail(MG_EINVAL, "bad argument");
  return norm(h, f, u, out);
}

mg_status mg_rbc_solve(mg_rbc_ctx *h, const double *f, double *u, int *cycles, double *hist) {
  if (!h || !f || !u) return fail(MG_EINVAL, "bad argument");
  double r0 = 0.0, r = 0.0;
  RBC_TRY(norm(h, f, u, &r0));
  if (hist) hist[0] = r0;
  int k = 0;
  r = r0;
  mg_status st = MG_OK;
  while (r > h->cfg.rtol * r0 && k < h->cfg.max_cycles) {
    RBC_TRY(cycle(h, 0, f, u));
    RBC_TRY(norm(h, f, u, &r));
    ++k;
    if (hist) hist[k] = r;
    if (!std::isfinite(r)) {
      st = fail(MG_ENUMERIC, "residual norm is not finite");
      break;
    }
  }
  if (cycles) *cycles = k;
  if (st == MG_OK && r > h->cfg.rtol * r0) st = fail(MG_ENOCONV, "solve did not reach rtol");
  return st;
}

mg_status mg_rbc_kernel_smooth(mg_rbc_ctx *h, int level, int colour, const double *f,
                               const double *u_in, double *u_out) {
  RBC_TRY(check_level(h, level, false));
  if (colour != 1 && colour != 2) return fail(MG_EINVAL, "colour must be 1 (F) or 2 (C)");
  if (!f || !u_in || !u_out || u_in == u_out) return fail(MG_EINVAL, "bad array arguments");
  return launch_smooth(h, level, colour, f, u_in, u_out);
}

mg_status mg_rbc_kernel_restrict(mg_rbc_ctx *h, int level, const double *f, const double *u,
                                 double *f_coarse) {
  RBC_TRY(check_level(h, level, true));
  if (!f || !u || !f_coarse) return fail(MG_EINVAL, "bad array arguments");
  return launch_restrict(h, level, f, u, f_coarse, nullptr);
}

mg_status mg_rbc_kernel_prolong(mg_rbc_ctx *h, int level, const double *e_coarse,
                                const double *u_in, double *u_out) {
  RBC_TRY(check_level(h, level, true));
  if (!e_coarse || !u_in || !u_out) return fail(MG_EINVAL, "bad array arguments");
  return launch_prolong(h, level, e_coarse, u_in, u_out);
}

mg_status mg_rbc_kernel_coarsest(mg_rbc_ctx *h, const double *f, double *u) {
  if (!h) return fail(MG_EINVAL, "null handle");
  if (!f || !u) return fail(MG_EINVAL, "bad array arguments");
  return launch_coarsest(h, f, u);
}

}  // extern "C"
