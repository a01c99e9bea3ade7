// tile2d.hip -- the two fused 2D cycle passes on small levels, one LDS tile per block.
//
// On a level of a few hundred points per side the row-marching kernels of fused2d.hip are
// latency-bound: each block walks tens of rows one after another.  Here a block instead
// loads a tile of the grid with its halo into LDS once and runs every stage as a parallel
// pass over a shrinking region (a stage of radius R is exact R points inside the region
// of the previous one), with one barrier between stages:
//   pre:  nu omega-Jacobi sweeps, the defect, its full weighting onto the coarse tile;
//   post: interpolation of the coarse correction and correction, nu2 sweeps.
// With red-black smoothing the sweeps are partial steps, red and black in turn.
// Inputs are extended oddly across the Dirichlet boundary when loaded (u(-i) = -u(i),
// boundary values zero), and every stage evaluated on the extended region reproduces the
// odd extension of its output, exactly as in the row-marching kernels.
#include <algorithm>
#include <cmath>
#include <cstdlib>

#include "mg_internal.h"

namespace mgk {
namespace {

__device__ __forceinline__ bool stopped(const int *done) { return done != nullptr && *done != 0; }

__device__ __forceinline__ int floordiv2(int a) { return a >= 0 ? a / 2 : -((1 - a) / 2); }

// Odd extension of grid index i (at most two reflections); -1 when it lies further out.
__device__ __forceinline__ int fold(int i, int n, int &sign) {
  if (i < 0) { i = -i; sign = -sign; }
  if (i > n - 1) { i = 2 * (n - 1) - i; sign = -sign; }
  if (i < 0) { i = -i; sign = -sign; }
  return (i >= 0 && i <= n - 1) ? i : -1;
}

// Odd-extended value of a at grid point (x, y).
template <typename T>
__device__ __forceinline__ T load_odd(const T *a, int x, int y, int n) {
  int s = 1;
  const int xf = fold(x, n, s), yf = fold(y, n, s);
  if (xf <= 0 || xf >= n - 1 || yf <= 0 || yf >= n - 1) return T(0);
  return T(s) * a[(size_t)yf * n + xf];
}

__device__ double block_sum(double v) {
  __shared__ double ws[kBlock / 64];
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  if ((threadIdx.x & 63) == 0) ws[threadIdx.x >> 6] = v;
  __syncthreads();
  double t = 0.0;
  if (threadIdx.x == 0)
    for (int i = 0; i < kBlock / 64; ++i) t += ws[i];
  return t;
}

// L u at region point p (pitch PW) of buffer u.  Cross operator: difference form with
// weights w1, w2.  Separable operator: the y sums A, B of the same point's row were
// written to sa, sb by y_sums (pitch PW) and L u = sum_i a_i (B(x+i) - B) + b_i A(x+i).
template <typename T, int R, int PW>
__device__ __forceinline__ T lu_at(const T *u, const T *sa, const T *sb, int p, const KOp<T> &op) {
  if constexpr (R == 2) {
    const T c = u[p];
    const T d1 = ((c - u[p - 1]) + (c - u[p + 1])) + ((c - u[p - PW]) + (c - u[p + PW]));
    const T d2 = ((c - u[p - 2]) + (c - u[p + 2])) + ((c - u[p - 2 * PW]) + (c - u[p + 2 * PW]));
    return op.w1 * d1 + op.w2 * d2;
  } else {
    const T B = sb[p];
    T v = T(0);
#pragma unroll
    for (int i = 0; i < 2 * R + 1; ++i) {
      if (i != R) v += op.a[i] * (sb[p + i - R] - B);
      v += op.b[i] * sa[p + i - R];
    }
    return v;
  }
}

// Separable operator, first pass: A = sum_{k != 0} a_k (u(y+k) - u), B = sum_k b_k u(y+k)
// at every point of rows [r0, r1) and columns [c0, c1) of the region.
template <typename T, int R, int PW>
__device__ __forceinline__ void y_sums(const T *u, T *sa, T *sb, int r0, int r1, int c0, int c1,
                                       const KOp<T> &op) {
  const int w = c1 - c0;
  for (int e = threadIdx.x; e < (r1 - r0) * w; e += kBlock) {
    const int p = (r0 + e / w) * PW + c0 + e % w;
    const T c = u[p];
    T A = T(0), B = T(0);
#pragma unroll
    for (int k = 0; k < 2 * R + 1; ++k) {
      const T v = u[p + (k - R) * PW];
      if (k != R) A += op.a[k] * (v - c);
      B += op.b[k] * v;
    }
    sa[p] = A;
    sb[p] = B;
  }
}

// ------------------------------------------------------------------------- pre ----
// Restricting modes: the block owns a CX x CY tile of coarse points and the fine points
// 2I0 .. 2I0+2CX-1 (rows alike); the defect is formed on the full-weighting support of
// the coarse tile, (2CX+1) x (2CY+1) fine points.  Other modes: a TX x TY fine tile.
constexpr int kCX = 16, kCY = 8, kTX = 32, kTY = 16;

template <typename T, int R, int NU, int MODE, bool HAS_U>
__global__ __launch_bounds__(kBlock) void k_pre_tile(const T *__restrict__ f, const T *__restrict__ u,
                                                     T *__restrict__ uout, T *__restrict__ rout,
                                                     T *__restrict__ fc, int n, KOp<T> op,
                                                     double *__restrict__ partials,
                                                     const int *__restrict__ done) {
  constexpr bool RESTRICT = (MODE & kPreRestrict) != 0;
  constexpr bool WRITE_R = (MODE & kPreWriteR) != 0;
  constexpr bool WRITE_U = (MODE & kPreWriteU) != 0;
  constexpr bool RES = RESTRICT || WRITE_R;
  constexpr int K = NU + (RES ? 1 : 0);  // stencil stages
  constexpr int DW = RESTRICT ? 2 * kCX + 1 : kTX, DH = RESTRICT ? 2 * kCY + 1 : kTY;
  constexpr int E = K * R;               // halo of the loaded region
  constexpr int PW = DW + 2 * E, PH = DH + 2 * E, PS = PW * PH;
  constexpr bool SEP = R == 3;
  __shared__ T sf[PS];
  __shared__ T su[2][PS];
  __shared__ T sy[SEP ? 2 : 1][SEP ? PS : 1];
  done = slot_done(done);
  if (stopped(done)) return;
  const int nc = (n - 1) / 2 + 1;
  f = slot_ptr(f, (size_t)n * n);
  u = slot_ptr(u, (size_t)n * n);
  uout = slot_ptr(uout, (size_t)n * n);
  rout = slot_ptr(rout, (size_t)n * n);
  fc = slot_ptr(fc, (size_t)nc * nc);
  partials = slot_ptr(partials, (size_t)gridDim.x * gridDim.y);
  const Block2 blk = block2();
  // region origin: the defect region (restricting) or the tile, less the halo
  const int I0 = blk.x * kCX, J0 = blk.y * kCY;
  const int DX0 = RESTRICT ? 2 * I0 - 1 : blk.x * kTX, DY0 = RESTRICT ? 2 * J0 - 1 : blk.y * kTY;
  const int X0 = DX0 - E, Y0 = DY0 - E;
  // own fine points: written, and counted in the defect norm
  const int ox0 = RESTRICT ? 2 * I0 : DX0, oy0 = RESTRICT ? 2 * J0 : DY0;
  const int ox1 = min(ox0 + (RESTRICT ? 2 * kCX : kTX), n), oy1 = min(oy0 + (RESTRICT ? 2 * kCY : kTY), n);

  for (int e = threadIdx.x; e < PS; e += kBlock) {
    const int x = X0 + e % PW, y = Y0 + e / PW;
    sf[e] = load_odd(f, x, y, n);
    su[0][e] = HAS_U ? load_odd(u, x, y, n) : T(0);
  }
  __syncthreads();

  double acc = 0.0;
  // stage s (1..K) covers the loaded region less sR on every side; stage K the defect region
#pragma unroll
  for (int s = 1; s <= K; ++s) {
    const int m = s * R;  // margin of stage s's region
    const T *ui = su[(s - 1) & 1];
    if constexpr (SEP) {
      y_sums<T, R, PW>(ui, sy[0], sy[1], m, PH - m, m - R, PW - m + R, op);
      __syncthreads();
    }
    const int w = PW - 2 * m, h = PH - 2 * m;
    for (int e = threadIdx.x; e < w * h; e += kBlock) {
      const int i = m + e % w, j = m + e / w;
      const int p = j * PW + i;
      const T r = sf[p] - lu_at<T, R, PW>(ui, sy[0], sy[SEP ? 1 : 0], p, op);
      const int x = X0 + i, y = Y0 + j;
      if (s == 1 && partials != nullptr && x >= ox0 && x < ox1 && y >= oy0 && y < oy1 && x > 0 &&
          x < n - 1 && y > 0 && y < n - 1)
        acc += (double)r * (double)r;
      if (s <= NU)
        su[s & 1][p] = ui[p] + stage_om(op, s, x + y) * r;
      else
        su[s & 1][p] = r;  // the defect (stage K of a residual mode)
    }
    __syncthreads();
  }
  // outputs on the own fine points: the smoothed iterate (stage NU) and the defect
  const T *un = su[NU & 1];
  const T *rd = su[K & 1];
  for (int e = threadIdx.x; e < (ox1 - ox0) * (oy1 - oy0); e += kBlock) {
    const int x = ox0 + e % (ox1 - ox0), y = oy0 + e / (ox1 - ox0);
    const int p = (y - Y0) * PW + (x - X0);
    const bool inside = x > 0 && x < n - 1 && y > 0 && y < n - 1;
    const size_t id = (size_t)y * n + x;
    if (WRITE_U) uout[id] = inside ? un[p] : T(0);
    if (WRITE_R) rout[id] = inside ? rd[p] : T(0);
  }
  if (RESTRICT) {
    for (int e = threadIdx.x; e < kCX * kCY; e += kBlock) {
      const int I = I0 + e % kCX, J = J0 + e / kCX;
      if (I > nc - 1 || J > nc - 1) continue;
      T v = T(0);
      if (I > 0 && I < nc - 1 && J > 0 && J < nc - 1) {
        const int p = (2 * J - Y0) * PW + (2 * I - X0);
        const T *q = rd + p;
        const T ym = T(0.25) * q[-PW - 1] + T(0.5) * q[-PW] + T(0.25) * q[-PW + 1];
        const T y0 = T(0.25) * q[-1] + T(0.5) * q[0] + T(0.25) * q[1];
        const T yp = T(0.25) * q[PW - 1] + T(0.5) * q[PW] + T(0.25) * q[PW + 1];
        v = T(0.25) * ym + T(0.5) * y0 + T(0.25) * yp;
      }
      fc[(size_t)J * nc + I] = v;
    }
  }
  if (partials != nullptr) {
    const double tot = block_sum(acc);
    if (threadIdx.x == 0) partials[blockIdx.y * gridDim.x + blockIdx.x] = tot;
  }
}

// ------------------------------------------------------------------------ post ----
// A TX x TY fine tile: the corrected iterate on the tile plus an nu2 R halo, then nu2
// sweeps over shrinking regions.
template <typename T, int R, int NU2, int P>
__global__ __launch_bounds__(kBlock) void k_post_tile(const T *__restrict__ v, const T *__restrict__ uin,
                                                      const T *__restrict__ f, T *__restrict__ uout,
                                                      int n, KOp<T> op, const int *__restrict__ done) {
  constexpr int E = NU2 * R;
  constexpr int PW = kTX + 2 * E, PH = kTY + 2 * E, PS = PW * PH;
  constexpr int CW = PW / 2 + 5, CH = PH / 2 + 5, CS = CW * CH;  // coarse cover of the region
  constexpr bool SEP = R == 3;
  __shared__ T sf[NU2 > 0 ? PS : 1];
  __shared__ T su[2][PS];
  __shared__ T sv[CS];
  __shared__ T sy[SEP && NU2 > 0 ? 2 : 1][SEP && NU2 > 0 ? PS : 1];
  done = slot_done(done);
  if (stopped(done)) return;
  const int nc = (n - 1) / 2 + 1;
  v = slot_ptr(v, (size_t)nc * nc);
  uin = slot_ptr(uin, (size_t)n * n);
  f = slot_ptr(f, (size_t)n * n);
  uout = slot_ptr(uout, (size_t)n * n);
  const Block2 blk = block2();
  const int tx0 = blk.x * kTX, ty0 = blk.y * kTY;
  const int X0 = tx0 - E, Y0 = ty0 - E;
  const int C0 = floordiv2(X0) - 2, D0 = floordiv2(Y0) - 2;  // coarse cover origin

  for (int e = threadIdx.x; e < CS; e += kBlock) sv[e] = load_odd(v, C0 + e % CW, D0 + e / CW, nc);
  for (int e = threadIdx.x; e < PS; e += kBlock) {
    const int x = X0 + e % PW, y = Y0 + e / PW;
    su[0][e] = load_odd(uin, x, y, n);
    if (NU2 > 0) sf[e] = load_odd(f, x, y, n);
  }
  __syncthreads();
  // stage 0: u + I_H^h v on the whole region
  for (int e = threadIdx.x; e < PS; e += kBlock) {
    const int x = X0 + e % PW, y = Y0 + e / PW;
    T wx[4], wy[4];
    auto weights = [](int fine, T (&w)[4]) {  // coarse fine/2-1 .. fine/2+2 (floor)
      if ((fine & 1) == 0) {
        w[0] = T(0); w[1] = T(1); w[2] = T(0); w[3] = T(0);
      } else if (P == 3) {
        w[0] = T(-0.0625); w[1] = T(0.5625); w[2] = T(0.5625); w[3] = T(-0.0625);
      } else {
        w[0] = T(0); w[1] = T(0.5); w[2] = T(0.5); w[3] = T(0);
      }
    };
    weights(x, wx);
    weights(y, wy);
    const int ci = floordiv2(x) - 1 - C0, cj = floordiv2(y) - 1 - D0;
    T s = T(0);
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      T row = T(0);
#pragma unroll
      for (int a2 = 0; a2 < 4; ++a2) row += wx[a2] * sv[(cj + b) * CW + ci + a2];
      s += wy[b] * row;
    }
    su[0][e] += s;
  }
  __syncthreads();
#pragma unroll
  for (int s = 1; s <= NU2; ++s) {
    const int m = s * R;  // stage NU2 covers the tile
    const T *ui = su[(s - 1) & 1];
    if constexpr (SEP) {
      y_sums<T, R, PW>(ui, sy[0], sy[SEP && NU2 > 0 ? 1 : 0], m, PH - m, m - R, PW - m + R, op);
      __syncthreads();
    }
    const int w = PW - 2 * m, h = PH - 2 * m;
    for (int e = threadIdx.x; e < w * h; e += kBlock) {
      const int i = m + e % w, j = m + e / w;
      const int p = j * PW + i;
      const T r = sf[NU2 > 0 ? p : 0] - lu_at<T, R, PW>(ui, sy[0], sy[SEP && NU2 > 0 ? 1 : 0], p, op);
      su[s & 1][p] = ui[p] + stage_om(op, s, X0 + i + Y0 + j) * r;
    }
    __syncthreads();
  }
  const T *un = su[NU2 & 1];
  const int w = min(kTX, n - tx0), h = min(kTY, n - ty0);
  for (int e = threadIdx.x; e < w * h; e += kBlock) {
    const int x = tx0 + e % w, y = ty0 + e / w;
    const bool inside = x > 0 && x < n - 1 && y > 0 && y < n - 1;
    uout[(size_t)y * n + x] = inside ? un[(y - Y0) * PW + (x - X0)] : T(0);
  }
}

int cdiv(long a, long b) { return (int)((a + b - 1) / b); }

template <typename T>
KOp<T> to_kop(const LevelOp &op, double omega) {
  KOp<T> k;
  for (int i = 0; i < 7; ++i) {
    k.a[i] = (T)op.a[i];
    k.b[i] = (T)op.b[i];
  }
  k.w1 = (T)(-op.a[2]);
  k.w2 = (T)(-op.a[1]);
  k.w3 = (T)(-op.a[0]);
  k.om_d = (T)(omega / op.diag);
  k.colour = 0;
  return k;
}

template <typename T, int R, int NU, int MODE>
hipError_t pre_tile_dispatch(const T *f, const T *u, T *uout, T *rout, T *fc, int n, const KOp<T> &k,
                             double *partials, int *nparts, const int *done, hipStream_t s,
                             int slots) {
  constexpr bool RM = (MODE & kPreRestrict) != 0;
  const int nc = (n - 1) / 2 + 1;
  const dim3 grid = RM ? dim3(cdiv(nc, kCX), cdiv(nc, kCY), slots) : dim3(cdiv(n, kTX), cdiv(n, kTY), slots);
  if (nparts) *nparts = grid.x * grid.y;
  if (u != nullptr)
    hipLaunchKernelGGL((k_pre_tile<T, R, NU, MODE, true>), grid, dim3(kBlock), 0, s, f, u, uout, rout,
                       fc, n, k, partials, done);
  else
    hipLaunchKernelGGL((k_pre_tile<T, R, NU, MODE, false>), grid, dim3(kBlock), 0, s, f, u, uout, rout,
                       fc, n, k, partials, done);
  return hipGetLastError();
}

template <typename T, int R>
hipError_t pre_tile_r(int nu, int mode, const T *f, const T *u, T *uout, T *rout, T *fc, int n,
                      const KOp<T> &k, double *partials, int *nparts, const int *done, hipStream_t s,
                      int slots) {
  constexpr int WR = kPreWriteU | kPreRestrict;
  if (mode == WR) {
    switch (nu) {
      case 0: return pre_tile_dispatch<T, R, 0, WR>(f, u, uout, rout, fc, n, k, partials, nparts, done, s, slots);
      case 1: return pre_tile_dispatch<T, R, 1, WR>(f, u, uout, rout, fc, n, k, partials, nparts, done, s, slots);
      case 2: return pre_tile_dispatch<T, R, 2, WR>(f, u, uout, rout, fc, n, k, partials, nparts, done, s, slots);
      case 3: return pre_tile_dispatch<T, R, 3, WR>(f, u, uout, rout, fc, n, k, partials, nparts, done, s, slots);
      default: return hipErrorInvalidValue;
    }
  }
  if (mode == kPreWriteU && nu == 1)
    return pre_tile_dispatch<T, R, 1, kPreWriteU>(f, u, uout, rout, fc, n, k, partials, nparts, done, s, slots);
  if (mode == kPreWriteU && nu == 2)
    return pre_tile_dispatch<T, R, 2, kPreWriteU>(f, u, uout, rout, fc, n, k, partials, nparts, done, s, slots);
  if (mode == kPreWriteR && nu == 0)
    return pre_tile_dispatch<T, R, 0, kPreWriteR>(f, u, uout, rout, fc, n, k, partials, nparts, done, s, slots);
  if (mode == kPreRestrict && nu == 0)
    return pre_tile_dispatch<T, R, 0, kPreRestrict>(f, u, uout, rout, fc, n, k, partials, nparts, done, s, slots);
  return hipErrorInvalidValue;
}

template <typename T, int R, int NU2>
hipError_t post_tile_dispatch(int prolong, const T *v, const T *uin, const T *f, T *uout, int n,
                              const KOp<T> &k, const int *done, hipStream_t s, int slots) {
  const dim3 grid(cdiv(n, kTX), cdiv(n, kTY), slots);
  if (prolong == 3)
    hipLaunchKernelGGL((k_post_tile<T, R, NU2, 3>), grid, dim3(kBlock), 0, s, v, uin, f, uout, n, k, done);
  else
    hipLaunchKernelGGL((k_post_tile<T, R, NU2, 1>), grid, dim3(kBlock), 0, s, v, uin, f, uout, n, k, done);
  return hipGetLastError();
}

}  // namespace

int tile2d_max_side() {
  static const int side = [] {
    const char *e = std::getenv("MG_TILE_N");
    return e ? std::atoi(e) : 513;
  }();
  return side;
}

int pre2d_tile_partials(int n) {
  const int nc = (n - 1) / 2 + 1;
  return std::max(cdiv(nc, kCX) * cdiv(nc, kCY), cdiv(n, kTX) * cdiv(n, kTY));
}

template <typename T>
hipError_t launch_pre2d_tile(const LevelOp &op, double omega, int nu, int mode, const T *f, const T *u,
                             T *uout, T *rout, T *fc, int n, double *partials, int *nparts,
                             const int *done, hipStream_t s, int slots, bool rb) {
  KOp<T> k = to_kop<T>(op, omega);
  if (rb) k.colour = kColourRB;
  if (op.cross) return pre_tile_r<T, 2>(nu, mode, f, u, uout, rout, fc, n, k, partials, nparts, done, s, slots);
  return pre_tile_r<T, 3>(nu, mode, f, u, uout, rout, fc, n, k, partials, nparts, done, s, slots);
}

template <typename T>
hipError_t launch_post2d_tile(const LevelOp &op, double omega, int nu2, int prolong, const T *v,
                              const T *uin, const T *f, T *uout, int n, const int *done,
                              hipStream_t s, int slots, bool rb) {
  KOp<T> k = to_kop<T>(op, omega);
  if (rb) k.colour = kColourRB;
  if (op.cross) {
    switch (nu2) {
      case 0: return post_tile_dispatch<T, 2, 0>(prolong, v, uin, f, uout, n, k, done, s, slots);
      case 1: return post_tile_dispatch<T, 2, 1>(prolong, v, uin, f, uout, n, k, done, s, slots);
      case 2: return post_tile_dispatch<T, 2, 2>(prolong, v, uin, f, uout, n, k, done, s, slots);
      default: return hipErrorInvalidValue;
    }
  }
  switch (nu2) {
    case 0: return post_tile_dispatch<T, 3, 0>(prolong, v, uin, f, uout, n, k, done, s, slots);
    case 1: return post_tile_dispatch<T, 3, 1>(prolong, v, uin, f, uout, n, k, done, s, slots);
    case 2: return post_tile_dispatch<T, 3, 2>(prolong, v, uin, f, uout, n, k, done, s, slots);
    default: return hipErrorInvalidValue;
  }
}

template hipError_t launch_pre2d_tile<double>(const LevelOp &, double, int, int, const double *,
                                              const double *, double *, double *, double *, int,
                                              double *, int *, const int *, hipStream_t, int, bool);
template hipError_t launch_pre2d_tile<float>(const LevelOp &, double, int, int, const float *,
                                             const float *, float *, float *, float *, int, double *,
                                             int *, const int *, hipStream_t, int, bool);
template hipError_t launch_post2d_tile<double>(const LevelOp &, double, int, int, const double *,
                                               const double *, const double *, double *, int,
                                               const int *, hipStream_t, int, bool);
template hipError_t launch_post2d_tile<float>(const LevelOp &, double, int, int, const float *,
                                              const float *, const float *, float *, int, const int *,
                                              hipStream_t, int, bool);

}  // namespace mgk
