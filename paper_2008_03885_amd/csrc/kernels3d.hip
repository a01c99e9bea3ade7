// kernels3d.hip -- 3D hot-path kernels for gfx950.
//
// A block of 256 threads owns a 32 x 8 tile of (x, y) columns and marches along z over a
// chunk of planes.  LDS holds a ring of the last 2R+1 planes of the tile extended by
// its halo; each step loads one new plane cooperatively (the next plane's loads are
// issued one step ahead, branch-free, with the reflection sign applied at use), waits
// at one barrier and computes the outputs of one plane from LDS.  The odd extension
// across the Dirichlet boundary is applied to every load (u(-i) = -u(i), boundary
// values zero).
//
// Cross operator (rediscretized levels, R = 2): difference form with weights w1, w2 on
// the 12 neighbours.  Separable operator (Galerkin levels, R = 3):
// L = a_x b_y b_z + b_x a_y b_z + b_x b_y a_z, applied as a z pass, a y pass and an x
// pass through LDS with every a factor in difference form, so constants are annihilated
// exactly.
#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <type_traits>
#include <utility>

#include "mg_internal.h"

namespace mgk {
namespace {

constexpr int TX = 32, TY = 8;  // output tile per block (one column per thread)

__device__ __forceinline__ bool stopped(const int *done) { return done != nullptr && *done != 0; }

__device__ __forceinline__ int fold(int i, int n, int &sign) {
  if (i < 0) { i = -i; sign = -sign; }
  if (i > n - 1) { i = 2 * (n - 1) - i; sign = -sign; }
  if (i < 0) { i = -i; sign = -sign; }
  return (i >= 0 && i <= n - 1) ? i : -1;
}

__device__ __forceinline__ int round_up8(int a) { return (a + 7) / 8 * 8; }

// Sum over a block of NT threads (valid in thread 0).
template <int NT>
__device__ double block_sum(double v) {
  __shared__ double ws[NT / 64];
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  if ((threadIdx.x & 63) == 0) ws[threadIdx.x >> 6] = v;
  __syncthreads();
  double t = 0.0;
  if (threadIdx.x == 0)
    for (int w = 0; w < NT / 64; ++w) t += ws[w];
  return t;
}

// ----------------------------------------------- cross sweep, z windows in registers ----
// The radius-2 cross operator (rediscretized levels).  Each thread keeps the u values of
// its own column at planes z-2 .. z+5 in a ring of registers; only plane z of the tile and
// its halo goes through LDS (double-buffered, one barrier per plane).  The plane loop is
// unrolled by the ring length, so ring slots are fixed registers and loads issued four to
// six planes ahead stay in flight.

template <int N, typename F, int... I>
__device__ __forceinline__ void static_for_impl(F &&f, std::integer_sequence<int, I...>) {
  (f(std::integral_constant<int, I>{}), ...);
}
template <int N, typename F>
__device__ __forceinline__ void static_for(F &&f) {
  static_for_impl<N>(f, std::make_integer_sequence<int, N>{});
}

constexpr int kZR = 8;  // planes per loop turn (the u ring); f and halo rings hold 4

// Register rings: the loop of a kernel refills a ring slot right after consuming it, in an
// unrolled turn that addresses the slots at compile-time positions.  Two rules keep the
// refills in flight across the loop's back edge:
//  - a slot is consumed by arithmetic (a product, even by 1), never by a plain copy, so
//    that the old value is dead when the refill is issued and the refill can land in the
//    slot's own register (a copy would be tied up in a register move and a wait);
//  - the prologue's loads are pinned before the loop (hold_regs), so that the loop header
//    does not wait for loads the compiler would otherwise sink to the loop entry.
template <typename T, int N>
__device__ __forceinline__ void hold_regs(T (&r)[N]) {
#pragma unroll
  for (int k = 0; k < N; ++k) asm volatile("" : "+v"(r[k]));
}

// A grid column (x, y): folded address and the sign of the odd extension (0 on and
// beyond the boundary).
template <typename T>
struct Col3 {
  int off;
  T mul;
  __device__ void init(int x, int y, int n) {
    int s = 1;
    const int xf = fold(x, n, s), yf = fold(y, n, s);
    const bool ok = xf > 0 && xf < n - 1 && yf > 0 && yf < n - 1;
    off = ok ? yf * n + xf : n + 1;
    mul = ok ? T(s) : T(0);
  }
};

// Address of plane z (folded into the grid) and the factor of its odd extension.
__device__ __forceinline__ size_t plane_base(int z, int n) {
  int s = 1;
  int zf = fold(z, n, s);
  zf = (zf > 0 && zf < n - 1) ? zf : 1;
  return (size_t)zf * n * n;
}
template <typename T>
__device__ __forceinline__ T plane_mul(int z, int n) {
  int s = 1;
  const int zf = fold(z, n, s);
  return (zf > 0 && zf < n - 1) ? T(s) : T(0);
}

// RR = 3: the radius-3 cross of the sixth-order operator (weights w1, w2, w3), with a u
// ring of 16 planes.  YS = 2: each thread owns two columns, rows ty and ty + TY, so a
// block covers an XW x 2TY tile and the y halo (2R rows) is shared by twice the rows.
template <typename T, typename TO, int MODE, bool HAS_U, int XW, int RR = 2, int YS = 1>
__global__ __launch_bounds__(XW * TY) void k_xsweep3d(const T *__restrict__ f, const T *__restrict__ u,
                                                  TO *__restrict__ out, int n, int zchunk, KOp<T> op,
                                                  double *__restrict__ partials,
                                                  const int *__restrict__ done) {
  constexpr int NT = XW * TY, R = RR, TYB = TY * YS, PX = XW + 2 * R, PY = TYB + 2 * R, PS = PX * PY;
  constexpr int ZR = RR == 2 ? kZR : 16;  // u ring length = planes per loop turn
  constexpr int NH = PS - NT * YS;  // halo cells of a plane
  static_assert(NH <= NT, "one halo cell per thread");
  __shared__ T plane[2][PS];
  if (stopped(done)) return;
  const Block3 blk = block3();
  // tiles and plane chunks start at row, column and plane 1: for n = 2^k + 1 the points
  // 1 .. n-1 fill whole tiles and chunks, and no block is left with the boundary column,
  // row or plane n-1 alone.  Column 0 and row 0 are stored by the halo lanes of the
  // first tiles, plane 0 by the first chunks.
  const int x0 = 1 + blk.x * XW, y0 = 1 + blk.y * TYB;
  const int z0 = 1 + blk.z * zchunk, z1 = min(z0 + zchunk, n);
  const int tx = threadIdx.x % XW, ty = threadIdx.x / XW;
  const int x = x0 + tx;
  int yv[YS], pown[YS];
  bool own[YS], xin[YS];
  Col3<T> cu[YS];
  size_t fcol[YS];
#pragma unroll
  for (int sr = 0; sr < YS; ++sr) {
    yv[sr] = y0 + ty + sr * TY;
    own[sr] = x <= n - 1 && yv[sr] <= n - 1;
    xin[sr] = x > 0 && x < n - 1 && yv[sr] > 0 && yv[sr] < n - 1;
    cu[sr].init(x, yv[sr], n);
    pown[sr] = (ty + sr * TY + R) * PX + tx + R;
    fcol[sr] = (size_t)(xin[sr] ? yv[sr] : 1) * n + (xin[sr] ? x : 1);
  }
  // this thread's halo cell (threads 0 .. NH-1): R rows above, R below, R columns on
  // each side of the middle rows
  Col3<T> ch;
  int hx = 0, hy = 0;
  const bool has_halo = threadIdx.x < NH;
  {
    const int h = threadIdx.x;
    if (h < R * PX) {
      hy = h / PX;
      hx = h % PX;
    } else if (h < 2 * R * PX) {
      hy = PY - R + (h - R * PX) / PX;
      hx = (h - R * PX) % PX;
    } else {
      const int hh = h - 2 * R * PX;
      hy = R + hh / (2 * R);
      const int c = hh % (2 * R);
      hx = c < R ? c : PX - 2 * R + c;
    }
  }
  // threads without a halo cell load their own column again (a line already in cache)
  if (has_halo)
    ch.init(x0 - R + hx, y0 - R + hy, n);
  else
    ch = cu[0];
  const int phal = hy * PX + hx;
  // halo lanes on column 0 beside the tile's rows, on row 0 above its columns, and the
  // corner (0, 0) store those boundary points (0)
  const int xe = x0 - R + hx, ye = y0 - R + hy;
  const bool edge = has_halo && ((xe == 0 && ye >= y0 && ye < y0 + TYB) || (ye == 0 && xe >= x0 && xe < x0 + XW) ||
                                 (xe == 0 && ye == 0));
  const size_t ide = (size_t)min(max(ye, 0), n - 1) * n + min(max(xe, 0), n - 1);
  constexpr bool STORES = MODE == kSweep || MODE == kSweepRB || MODE == kSweepZ2 || MODE == kResidual;
  constexpr bool CORR = MODE == kSweepCorr;  // out is the FP64 iterate: out += the sweep's result
  if (STORES && blk.z == 0) {  // plane 0
#pragma unroll
    for (int sr = 0; sr < YS; ++sr) out[(size_t)min(yv[sr], n - 1) * n + min(x, n - 1)] = (TO)0;
    if (edge) out[ide] = (TO)0;
  }
  // u is read from f (scaled by omega / a0 when consumed) for two sweeps from zero
  const T *up = (HAS_U && MODE != kSweepZ2) ? u : f;  // a valid address when there is no u
  const int zlast = z0 + (z1 - z0 + ZR - 1) / ZR * ZR - 1;
  const bool fast = z0 - R > 0 && zlast + ZR - R < n - 1;

  double acc = 0.0;
  auto run = [&](auto fast_tag) {
    constexpr bool FAST = decltype(fast_tag)::value;
    auto base = [&](int z) -> size_t { return FAST ? (size_t)z * n * n : plane_base(z, n); };
    // ring refills past the planes this chunk consumes re-read the last one it needs (an
    // L2 hit) instead of fetching planes it never uses: 1025^3 FP32 sweep 3582 -> 3478 us
    auto basec = [&](int z, int cap) -> size_t { return FAST ? (size_t)min(z, cap) * n * n : plane_base(z, n); };
    auto zm = [&](int z) -> T { return FAST ? T(1) : plane_mul<T>(z, n); };
    // raw loads: u of the own columns at z-R+k, f of the own columns and the halo at z+k
    T ur[YS][ZR], fr[YS][4], hr[4];
#pragma unroll
    for (int sr = 0; sr < YS; ++sr) {
#pragma unroll
      for (int k = 0; k < ZR; ++k) ur[sr][k] = HAS_U ? up[base(z0 - R + k) + cu[sr].off] : T(0);
#pragma unroll
      for (int k = 0; k < 4; ++k) fr[sr][k] = f[(FAST ? (size_t)(z0 + k) * n * n : base(z0 + k)) + fcol[sr]];
      hold_regs(ur[sr]);
      hold_regs(fr[sr]);
    }
#pragma unroll
    for (int k = 0; k < 4; ++k) hr[k] = HAS_U ? up[base(z0 + k) + ch.off] : T(0);
    hold_regs(hr);
    // CORR: the FP64 iterate of the own columns at the current plane, loaded one step
    // ahead (refilled right after its use)
    TO gr[YS];
    if constexpr (CORR) {
#pragma unroll
      for (int sr = 0; sr < YS; ++sr)
        gr[sr] = out[((size_t)min(z0, n - 1) * n + min(yv[sr], n - 1)) * n + min(x, n - 1)];
    }
    const KOp<T> kop = op;
    const T uscale = MODE == kSweepZ2 ? kop.om_d : T(1);
    auto step = [&](const int z, auto pc) {
      constexpr int P = decltype(pc)::value;
      // plane z+d sits in slot (P + R + d) mod ZR
      T um3[YS], um2[YS], um1[YS], uc[YS], up1[YS], up2[YS], up3[YS], fz[YS];
#pragma unroll
      for (int sr = 0; sr < YS; ++sr) {
        const T m = cu[sr].mul * uscale;
        um3[sr] = RR == 3 ? ur[sr][P % ZR] * (m * zm(z - 3)) : T(0);
        um2[sr] = ur[sr][(P + R - 2) % ZR] * (m * zm(z - 2));
        um1[sr] = ur[sr][(P + R - 1) % ZR] * (m * zm(z - 1));
        uc[sr] = ur[sr][(P + R) % ZR] * (m * zm(z));
        up1[sr] = ur[sr][(P + R + 1) % ZR] * (m * zm(z + 1));
        up2[sr] = ur[sr][(P + R + 2) % ZR] * (m * zm(z + 2));
        up3[sr] = RR == 3 ? ur[sr][(P + R + 3) % ZR] * (m * zm(z + 3)) : T(0);
        fz[sr] = fr[sr][P % 4] * (xin[sr] ? T(1) : T(0));
        if constexpr (RR == 3)
          asm volatile("" : "+v"(um3[sr]), "+v"(fz[sr]));
        else
          asm volatile("" : "+v"(um2[sr]), "+v"(fz[sr]));
        if constexpr (MODE == kSweepZ2)  // the products omega / a0 * f rounded as stored
          asm volatile("" : "+v"(um2[sr]), "+v"(um1[sr]), "+v"(uc[sr]), "+v"(up1[sr]), "+v"(up2[sr]),
                       "+v"(um3[sr]), "+v"(up3[sr]));
      }
      T hz = hr[P % 4] * ((ch.mul * uscale) * zm(z));
      asm volatile("" : "+v"(hz));
      __builtin_amdgcn_sched_barrier(0);
#pragma unroll
      for (int sr = 0; sr < YS; ++sr) {
        if (HAS_U) ur[sr][P % ZR] = up[basec(z - R + ZR, z1 - 1 + R) + cu[sr].off];  // the slot of plane z-R
        fr[sr][P % 4] = f[basec(z + 4, z1 - 1) + fcol[sr]];
      }
      if (HAS_U) hr[P % 4] = up[basec(z + 4, z1 - 1) + ch.off];
      T *pl = plane[P & 1];
#pragma unroll
      for (int sr = 0; sr < YS; ++sr) pl[pown[sr]] = uc[sr];
      if (has_halo) pl[phal] = hz;
      __syncthreads();
#pragma unroll
      for (int sr = 0; sr < YS; ++sr) {
        const int po = pown[sr];
        const T c = uc[sr];
        T lu = HAS_U ? kop.w1 * (((c - pl[po - 1]) + (c - pl[po + 1])) +
                                 ((c - pl[po - PX]) + (c - pl[po + PX])) + ((c - um1[sr]) + (c - up1[sr]))) +
                           kop.w2 * (((c - pl[po - 2]) + (c - pl[po + 2])) +
                                     ((c - pl[po - 2 * PX]) + (c - pl[po + 2 * PX])) +
                                     ((c - um2[sr]) + (c - up2[sr])))
                     : T(0);
        if constexpr (RR == 3)
          if (HAS_U)
            lu += kop.w3 * (((c - pl[po - 3]) + (c - pl[po + 3])) +
                            ((c - pl[po - 3 * PX]) + (c - pl[po + 3 * PX])) + ((c - um3[sr]) + (c - up3[sr])));
        const bool inside = own[sr] && xin[sr] && z > 0 && z < n - 1;
        const T r = inside ? fz[sr] - lu : T(0);
        if (partials != nullptr && inside && z < z1) acc += (double)r * (double)r;
        // Every lane stores, so no store sits under a branch.  A lane past the grid, or a
        // step past the last plane, lands on the boundary (clamped address) and stores its
        // value there, 0; a step past this block's planes stores the value the owning
        // block stores too (same inputs, same arithmetic).
        const size_t id = ((size_t)min(z, n - 1) * n + min(yv[sr], n - 1)) * n + min(x, n - 1);
        if (MODE == kSweep || MODE == kSweepRB || MODE == kSweepZ2)
          out[id] = (TO)(inside ? c + (MODE == kSweepRB ? colour_om(kop, x + yv[sr] + z) : kop.om_d) * r : T(0));
        if (MODE == kResidual) out[id] = (TO)r;
        if constexpr (CORR) {
          // e' rounded to T as a stored sweep result would be, then added in TO
          T e1 = c + kop.om_d * r;
          asm volatile("" : "+v"(e1));
          const TO unew = gr[sr] + (TO)e1;
          if (inside) out[id] = unew;
          gr[sr] = out[((size_t)min(z + 1, n - 1) * n + min(yv[sr], n - 1)) * n + min(x, n - 1)];
        }
      }
      if (STORES && edge) out[(size_t)min(z, n - 1) * n * n + ide] = (TO)0;
    };
    for (int z = z0; z < z1; z += ZR)
      static_for<ZR>([&](auto pc) { step(z + decltype(pc)::value, pc); });
  };
  if (fast)
    run(std::true_type{});
  else
    run(std::false_type{});
  if (partials != nullptr) {
    const double tot = block_sum<NT>(acc);
    if (threadIdx.x == 0)
      partials[((size_t)blockIdx.z * gridDim.y + blockIdx.y) * gridDim.x + blockIdx.x] = tot;
  }
}

// --------------------------------------- red-black sweep of the cross, one pass ----
// One red-black sweep of the radius-2 cross (section 3.1 eq. S_rb) in one pass: the red
// partial step (odd x+y+z) on plane z, the black one two planes behind.  The black step
// of an XW x YW tile needs red results two columns around it, so the block has one thread
// per column of the tile plus a two-column frame, (XW+4) x (YW+4) threads (60 x 8: twelve
// whole wavefronts); all of them take
// the red step, the tile's threads the black step.  Per plane, u of the frame region and
// a further two-column halo goes through LDS (double-buffered) for the red step; the red
// results go through an LDS ring of four planes for the black step's in-plane
// neighbours; z neighbours of u, f and the red results stay in register rings (same
// register-ring rules as the cross sweep).  One barrier per plane.  Every value is the
// odd extension across the Dirichlet boundary (reflection keeps a point's colour), so
// frame columns outside the grid hold the odd extension of the red results.
// J2: the same pass with both steps over every point, i.e. two omega-Jacobi sweeps (the
// first on plane z and the frame, the second two planes behind on the tile).
template <typename T, bool HAS_U, int XW, int YW, bool J2 = false>
__global__ __launch_bounds__((XW + 4) * (YW + 4)) void k_rbxsweep3d(const T *__restrict__ f, const T *__restrict__ u,
                                                                     T *__restrict__ out, int n, int zchunk,
                                                                     KOp<T> op, double *__restrict__ partials,
                                                                     const int *__restrict__ done) {
  constexpr int R = 2, EX = XW + 2 * R, EY = YW + 2 * R, NT = EX * EY;
  constexpr int PX = EX + 2 * R, PY = EY + 2 * R, PS = PX * PY;
  constexpr int NH = PS - NT;  // halo cells of a plane
  static_assert(NH <= NT, "one halo cell per thread");
  static_assert(NT % 64 == 0, "whole wavefronts (block_sum)");
  __shared__ T plane[2][PS];
  __shared__ T red[4][NT];
  if (stopped(done)) return;
  const Block3 blk = block3();
  const int x0 = blk.x * XW, y0 = blk.y * YW;
  const int z0 = blk.z * zchunk, z1 = min(z0 + zchunk, n);
  const int tid = threadIdx.x;
  const int ex = tid % EX, ey = tid / EX;
  const int x = x0 - R + ex, y = y0 - R + ey;
  // the tile's columns (black step and output); clamped neighbour slots for the others
  const bool tile = ex >= R && ex < XW + R && ey >= R && ey < YW + R;
  const bool own = tile && x <= n - 1 && y <= n - 1;
  const bool xin = x > 0 && x < n - 1 && y > 0 && y < n - 1;
  const int qm1 = max(tid - 1, 0), qp1 = min(tid + 1, NT - 1), qm2 = max(tid - 2, 0), qp2 = min(tid + 2, NT - 1);
  const int qmy = max(tid - EX, 0), qpy = min(tid + EX, NT - 1), qmy2 = max(tid - 2 * EX, 0), qpy2 = min(tid + 2 * EX, NT - 1);
  Col3<T> cu, ch;
  cu.init(x, y, n);
  int hx = 0, hy = 0;
  const bool has_halo = tid < NH;
  {
    const int h = tid;
    if (h < 2 * PX) {
      hy = h / PX;
      hx = h % PX;
    } else if (h < 4 * PX) {
      hy = PY - R + (h - 2 * PX) / PX;
      hx = (h - 2 * PX) % PX;
    } else {
      const int hh = h - 4 * PX;
      hy = R + hh / (2 * R);
      const int c = hh % (2 * R);
      hx = c < R ? c : PX - 2 * R + c;
    }
  }
  if (has_halo)
    ch.init(x - ex - R + hx, y - ey - R + hy, n);
  else
    ch = cu;
  const int pown = (ey + R) * PX + ex + R, phal = hy * PX + hx;
  const T *up = HAS_U ? u : f;
  // red steps on planes z0-2 .. z1+1, black steps two planes behind
  const int zs = z0 - 2, zlast = zs + round_up8(z1 - z0 + 4) - 1;
  const bool fast = zs - R > 0 && zlast + 6 < n - 1;
  double acc = 0.0;
  auto run = [&](auto fast_tag) {
    constexpr bool FAST = decltype(fast_tag)::value;
    auto base = [&](int z) -> size_t { return FAST ? (size_t)z * n * n : plane_base(z, n); };
    auto zm = [&](int z) -> T { return FAST ? T(1) : plane_mul<T>(z, n); };
    T ur[kZR], fr[kZR], hr[4], vr[kZR];  // u and f of this column at z-2+k; halo at z+k; red results
#pragma unroll
    for (int k = 0; k < kZR; ++k) {
      ur[k] = HAS_U ? up[base(zs - 2 + k) + cu.off] : T(0);
      fr[k] = f[base(zs - 2 + k) + cu.off];
      vr[k] = T(0);
    }
#pragma unroll
    for (int k = 0; k < 4; ++k) hr[k] = HAS_U ? up[base(zs + k) + ch.off] : T(0);
    hold_regs(ur);
    hold_regs(fr);
    hold_regs(hr);
    const KOp<T> kop = op;
    auto step = [&](const int z, auto pc) {  // red step on plane z, black step on plane z-2
      constexpr int P = decltype(pc)::value;
      const T m = cu.mul;
      T um2 = ur[P % kZR] * (m * zm(z - 2)), um1 = ur[(P + 1) % kZR] * (m * zm(z - 1));
      T uc = ur[(P + 2) % kZR] * (m * zm(z)), up1 = ur[(P + 3) % kZR] * (m * zm(z + 1));
      T up2 = ur[(P + 4) % kZR] * (m * zm(z + 2));
      T fb = fr[P % kZR] * (m * zm(z - 2)), fz = fr[(P + 2) % kZR] * (m * zm(z));
      T hz = hr[P % 4] * (ch.mul * zm(z));
      asm volatile("" : "+v"(um2), "+v"(fb), "+v"(hz));
      __builtin_amdgcn_sched_barrier(0);
      if (HAS_U) ur[P % kZR] = up[base(z + 6) + cu.off];  // the slot of plane z-2
      fr[P % kZR] = f[base(z + 6) + cu.off];
      if (HAS_U) hr[P % 4] = up[base(z + 4) + ch.off];
      T *pl = plane[P & 1];
      pl[pown] = uc;
      if (has_halo) pl[phal] = hz;
      __syncthreads();
      // red step on plane z (every frame column), odd extension included
      const T lu = HAS_U ? kop.w1 * (((uc - pl[pown - 1]) + (uc - pl[pown + 1])) +
                                     ((uc - pl[pown - PX]) + (uc - pl[pown + PX])) + ((uc - um1) + (uc - up1))) +
                               kop.w2 * (((uc - pl[pown - 2]) + (uc - pl[pown + 2])) +
                                         ((uc - pl[pown - 2 * PX]) + (uc - pl[pown + 2 * PX])) +
                                         ((uc - um2) + (uc - up2)))
                         : T(0);
      const T r = fz - lu;
      if (partials != nullptr && own && xin && z >= z0 && z < z1 && z > 0 && z < n - 1)
        acc += (double)r * (double)r;
      const T v = uc + ((J2 || ((x + y + z) & 1) != 0) ? kop.om_d : T(0)) * r;
      vr[(P + 4) % kZR] = v;
      red[(z % 4 + 4) % 4][tid] = v;
      // black step on plane z-2 from the red results (in-plane: written two planes ago)
      const int zb = z - 2;
      const T *rp = red[(zb % 4 + 4) % 4];
      const T vc = vr[(P + 2) % kZR];
      const T lb = kop.w1 * (((vc - rp[qm1]) + (vc - rp[qp1])) + ((vc - rp[qmy]) + (vc - rp[qpy])) +
                             ((vc - vr[(P + 1) % kZR]) + (vc - vr[(P + 3) % kZR]))) +
                   kop.w2 * (((vc - rp[qm2]) + (vc - rp[qp2])) + ((vc - rp[qmy2]) + (vc - rp[qpy2])) +
                             ((vc - vr[P % kZR]) + (vc - vr[(P + 4) % kZR])));
      const bool inside = xin && zb > 0 && zb < n - 1;
      const T w = inside ? vc + ((J2 || ((x + y + zb) & 1) == 0) ? kop.om_d : T(0)) * (fb - lb) : T(0);
      if (own && zb >= z0 && zb < z1) out[((size_t)zb * n + y) * n + x] = w;
    };
    for (int z = zs; z <= zlast; z += kZR)
      static_for<kZR>([&](auto pc) { step(z + decltype(pc)::value, pc); });
  };
  if (fast)
    run(std::true_type{});
  else
    run(std::false_type{});
  if (partials != nullptr) {
    const double tot = block_sum<NT>(acc);
    if (tid == 0) partials[((size_t)blockIdx.z * gridDim.y + blockIdx.y) * gridDim.x + blockIdx.x] = tot;
  }
}

// Values of the neighbouring lanes across the whole wavefront (DPP wavefront shifts):
// lane_prev gives lane L the value of lane L-1, lane_next that of lane L+1; the lane with
// no neighbour gets 0.
__device__ __forceinline__ int dpp_prev(int v) { return __builtin_amdgcn_mov_dpp(v, 0x138, 0xf, 0xf, true); }
__device__ __forceinline__ int dpp_next(int v) { return __builtin_amdgcn_mov_dpp(v, 0x130, 0xf, 0xf, true); }
__device__ __forceinline__ float lane_prev(float v) { return __int_as_float(dpp_prev(__float_as_int(v))); }
__device__ __forceinline__ float lane_next(float v) { return __int_as_float(dpp_next(__float_as_int(v))); }
__device__ __forceinline__ double lane_prev(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = dpp_prev((int)(b & 0xffffffffLL)), hi = dpp_prev((int)(b >> 32));
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}
__device__ __forceinline__ double lane_next(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = dpp_next((int)(b & 0xffffffffLL)), hi = dpp_next((int)(b >> 32));
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// ------------------------------- separable (Galerkin) sweep, wavefront pencils ----
// Coarse Galerkin operators are sums of three tensor products of 1D stencils of radius 3,
// L = a_x b_y b_z + b_x a_y b_z + b_x b_y a_z, applied as
//   L u(z) = sum_k b_k P1(z+k) + sum_{k != 0} a_k (P2(z+k) - P2(z)),
//   P1 = a_x (b_y u) + b_x (a_y u),  P2 = b_x (b_y u)   (in-plane, per plane),
// each a-stencil in difference form (its coefficients sum to zero).  This kernel applies
// it without LDS and without barriers: every wavefront works alone on a pencil of YR rows
// and 64 columns, of which the middle 58 are its outputs (three columns of x halo on
// each side).  Per plane a lane loads its column at the YR rows and three rows of y halo
// on each side, applies b_y and a_y in registers, and takes the x neighbours of b_y u and
// a_y u from the lanes beside it (cross-lane shuffles); P1 and P2 enter register rings of
// eight planes, the z pass runs over the rings.  Symmetric factors: with
// t_j = (v_{+j} - v_0) + (v_{-j} - v_0), a v = sum_j a_j t_j (difference form) and
// b v = (sum_i b_i) v_0 + sum_j b_j t_j.  Four wavefronts per block take neighbouring row
// groups of the same columns and planes.  Register rings as in the cross sweep: the u
// window of a plane is loaded two planes ahead, f four planes ahead.
template <typename T, typename TO, int MODE, int YR>
__global__ __launch_bounds__(256) void k_gpen3d(const T *__restrict__ f, const T *__restrict__ u,
                                                TO *__restrict__ out, int n, int zchunk, KOp<T> op,
                                                double *__restrict__ partials, const int *__restrict__ done) {
  constexpr int R = 3, OUT = 64 - 2 * R, WIN = YR + 2 * R;
  if (stopped(done)) return;
  const Block3 blk = block3();
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int x = blk.x * OUT + lane - R;  // this lane's column (beyond the grid: folded)
  const int y0 = (blk.y * 4 + wave) * YR;
  const int z0 = blk.z * zchunk, z1 = min(z0 + zchunk, n);
  // column: folded offset and the factor of the odd extension (0 on the boundary)
  int sx = 1;
  const int xf = fold(x, n, sx);
  const bool xok = xf > 0 && xf < n - 1;
  const int xoff = xok ? xf : 1;
  const T xmul = xok ? T(sx) : T(0);
  // rows of the window (uniform over the wavefront): offsets y*n and factors
  int yoff[WIN];
  T ymul[WIN];
#pragma unroll
  for (int i = 0; i < WIN; ++i) {
    int sy = 1;
    const int yf = fold(y0 - R + i, n, sy);
    const bool ok = yf > 0 && yf < n - 1;
    yoff[i] = (ok ? yf : 1) * n;
    ymul[i] = ok ? T(sy) : T(0);
  }
  const bool lane_out = lane >= R && lane < 64 - R;
  const bool xin = lane_out && x > 0 && x < n - 1;
  const KOp<T> kop = op;
  T bsum = kop.b[3];
#pragma unroll
  for (int j = 1; j <= 3; ++j) bsum += T(2) * kop.b[3 + j];
  auto pbase = [&](int z) -> size_t {
    int sz = 1;
    int zf = fold(z, n, sz);
    zf = (zf > 0 && zf < n - 1) ? zf : 1;
    return (size_t)zf * n * n;
  };
  auto pmul = [&](int z) -> T {
    int sz = 1;
    const int zf = fold(z, n, sz);
    return (zf > 0 && zf < n - 1) ? T(sz) : T(0);
  };
  double acc = 0.0;
  // rings: u windows by (plane - (z0-3)) mod 2, P and the window centres by the same
  // mod 8 / 4, f by (plane - z0) mod 4
  T win[2][WIN], p1r[YR][8], p2r[YR][8], ucr[YR][4], fr[YR][4];
  // loads from a plane base that is uniform over the wavefront plus a 32-bit offset
  const T *ub = MODE == kSweepZ2 ? f : u;  // two sweeps from zero: u = omega / a0 * f
  auto load_win = [&](int slot, int q) {
    const T *pl = ub + pbase(q);
#pragma unroll
    for (int i = 0; i < WIN; ++i) win[slot][i] = pl[(unsigned)(xoff + yoff[i])];
  };
  load_win(0, z0 - R);
  load_win(1, z0 - R + 1);
  unsigned foff[YR];  // f of the own rows within a plane
#pragma unroll
  for (int r = 0; r < YR; ++r) foff[r] = (unsigned)(min(max(y0 + r, 0), n - 1) * n + (xin ? x : 1));
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const T *pl = f + pbase(min(z0 + k, n - 1));
#pragma unroll
    for (int r = 0; r < YR; ++r) fr[r][k] = pl[foff[r]];
  }
  hold_regs(win[0]);
  hold_regs(win[1]);
  // P1, P2 of plane q from its window (slot ws), into ring slot ps; the window centres
  // into the centre ring slot cs
  auto inplane = [&](int q, int ws, int ps, int cs) {
    __builtin_amdgcn_sched_barrier(0);  // one plane at a time (register pressure)
    const T m = (MODE == kSweepZ2 ? xmul * kop.om_d : xmul) * pmul(q);
    T v[WIN];
#pragma unroll
    for (int i = 0; i < WIN; ++i) {
      v[i] = win[ws][i] * (m * ymul[i]);
      if constexpr (MODE == kSweepZ2) asm volatile("" : "+v"(v[i]));  // rounded as stored
    }
    __builtin_amdgcn_sched_barrier(0);
    load_win(ws, q + 2);
#pragma unroll
    for (int r = 0; r < YR; ++r) {
      const T c = v[r + R];
      ucr[r][cs] = c;
      T ay = T(0), by = bsum * c;
#pragma unroll
      for (int j = 1; j <= 3; ++j) {
        const T t = (v[r + R + j] - c) + (v[r + R - j] - c);
        ay += kop.a[3 + j] * t;
        by += kop.b[3 + j] * t;
      }
      // x pass: neighbours from the lanes beside, shifted in j steps of one lane (the
      // lanes at the strip edges take values of no use: they produce no output)
      T p1 = kop.b[3] * ay, p2 = bsum * by;
      T bl = by, br = by, al = ay, ar = ay;
#pragma unroll
      for (int j = 1; j <= 3; ++j) {
        bl = lane_prev(bl);  // by of column x - j
        br = lane_next(br);  // by of column x + j
        al = lane_prev(al);
        ar = lane_next(ar);
        const T tb = (br - by) + (bl - by);
        p1 += kop.a[3 + j] * tb + kop.b[3 + j] * (ar + al);
        p2 += kop.b[3 + j] * tb;
      }
      p1r[r][ps] = p1;
      p2r[r][ps] = p2;
    }
  };
  // Step s (s = 0, 1, ...; P = s mod 8) computes P1, P2 of plane z0-3+s into ring slot P
  // and, from s = 6 on, the output plane z = z0-6+s from the slots P+2 .. P+8 (mod 8).
  // The first six steps only fill the rings (a uniform branch skips the z pass).
  auto step = [&](const int z, auto pc) {
    constexpr int P = decltype(pc)::value;  // (z - (z0-6)) mod 8
    inplane(z + R, P % 2, P, P % 4);
    if (z < z0) return;
    T fz[YR];
#pragma unroll
    for (int r = 0; r < YR; ++r) fz[r] = fr[r][(P + 2) % 4] * (xin ? T(1) : T(0));
    asm volatile("" : "+v"(fz[0]));
    {
      const T *pl = f + pbase(min(z + 4, n - 1));
#pragma unroll
      for (int r = 0; r < YR; ++r) fr[r][(P + 2) % 4] = pl[foff[r]];
    }
#pragma unroll
    for (int r = 0; r < YR; ++r) {
      // z pass: planes z-3 .. z+3 sit in slots P+2 .. P+8
      const T c2 = p2r[r][(P + 5) % 8];
      T lu = kop.b[3] * p1r[r][(P + 5) % 8];
#pragma unroll
      for (int j = 1; j <= 3; ++j)
        lu += kop.b[3 + j] * (p1r[r][(P + 5 + j) % 8] + p1r[r][(P + 5 - j) % 8]) +
              kop.a[3 + j] * ((p2r[r][(P + 5 + j) % 8] - c2) + (p2r[r][(P + 5 - j) % 8] - c2));
      const int y = y0 + r;
      const bool inside = xin && y > 0 && y < n - 1 && z > 0 && z < n - 1;
      const T rr = inside ? fz[r] - lu : T(0);
      if (partials != nullptr && inside && z < z1) acc += (double)rr * (double)rr;
      // every lane stores: the x-halo lanes store the value of the nearest output lane
      // at its address (same value), lanes past the grid the boundary's 0 (clamped)
      const T uc = ucr[r][(P + 1) % 4];
      T v = T(0);
      if (MODE == kSweep || MODE == kSweepRB || MODE == kSweepZ2)
        v = inside ? uc + (MODE == kSweepRB ? colour_om(kop, x + y + z) : kop.om_d) * rr : T(0);
      if (MODE == kResidual) v = rr;
      if (MODE != kNormOnly) {
        const int src = lane < R ? R : (lane >= 64 - R ? 63 - R : lane);
        const T vs = __shfl(v, src, 64);
        const int xs = min(max(blk.x * OUT + src - R, 0), n - 1);
        const size_t id = ((size_t)min(z, n - 1) * n + min(y, n - 1)) * n + xs;
        out[id] = (TO)vs;
      }
    }
  };
  for (int z = z0 - 6; z < z1; z += 8)
    static_for<8>([&](auto pc) { step(z + decltype(pc)::value, pc); });
  if (partials != nullptr) {
    const double tot = block_sum<256>(acc);
    if (threadIdx.x == 0)
      partials[((size_t)blockIdx.z * gridDim.y + blockIdx.y) * gridDim.x + blockIdx.x] = tot;
  }
}

// ------------------------------------- cross defect + full weighting, z rings ----
// The radius-2 cross operator.  A block owns a CX x CY tile of coarse columns and coarse
// planes [K0, K1).  The full-weighting support of the tile is (2CX+1) x (2CY+1) fine
// columns, one per thread; each keeps its u values at planes z-2 .. z+5 in a ring of
// registers and its last four defects in another, while plane z of the support plus a
// two-point halo goes through LDS.  After every odd fine plane 2K+1 the z-weighted
// defects of planes 2K-1 .. 2K+1 are weighted in x and y through LDS.
// RR = 3: the radius-3 cross of the sixth-order operator, with a u ring of 16 planes.
template <typename T, bool HAS_U, int CX, int CY, int NT, int RR = 2>
__global__ __launch_bounds__(NT) void k_xrr3d(const T *__restrict__ f, const T *__restrict__ u,
                                              T *__restrict__ fc, int n, int kchunk, KOp<T> op,
                                              const int *__restrict__ done) {
  constexpr int kRDX = 2 * CX + 1, kRDY = 2 * CY + 1;
  constexpr int R = RR, PX = kRDX + 2 * R, PY = kRDY + 2 * R, PS = PX * PY;
  constexpr int ZR = RR == 2 ? kZR : 16;  // u ring length = planes per loop turn (even)
  constexpr int ND = kRDX * kRDY, NH = PS - ND;  // defect columns, halo cells
  static_assert(ND <= NT && NH <= NT, "one column and one halo cell per thread");
  __shared__ T plane[2][PS];
  __shared__ T dz[ND];
  if (stopped(done)) return;
  const int nc = (n - 1) / 2 + 1;
  const Block3 blk = block3();
  // coarse tiles start at column 1 (for n = 2^k + 1 the nc - 1 columns 1 .. nc-1 fill
  // whole tiles); column 0 is stored by edge lanes of the first tiles
  const int I0 = 1 + blk.x * CX, J0 = blk.y * CY;
  const int X0 = 2 * I0 - 1, Y0 = 2 * J0 - 1;  // defect support origin
  const int K0 = blk.z * kchunk, K1 = min(K0 + kchunk, nc);
  const int t = threadIdx.x;
  const bool has_col = t < ND;
  const int dx = has_col ? t % kRDX : 0, dy = has_col ? t / kRDX : 0;
  Col3<T> cu, ch;
  cu.init(X0 + dx, Y0 + dy, n);
  int hx = 0, hy = 0;
  const bool has_halo = t < NH;
  if (t < R * PX) {
    hy = t / PX;
    hx = t % PX;
  } else if (t < 2 * R * PX) {
    hy = PY - R + (t - R * PX) / PX;
    hx = (t - R * PX) % PX;
  } else {
    const int hh = t - 2 * R * PX;
    hy = R + hh / (2 * R);
    const int c = hh % (2 * R);
    hx = c < R ? c : PX - 2 * R + c;
  }
  if (has_halo)
    ch.init(X0 - R + hx, Y0 - R + hy, n);
  else
    ch = cu;
  const int pown = (dy + R) * PX + dx + R, phal = hy * PX + hx;
  const int fx = X0 + dx, fy = Y0 + dy;
  const bool fin = has_col && fx > 0 && fx < n - 1 && fy > 0 && fy < n - 1;
  const size_t fcol = (size_t)(fin ? fy : 1) * n + (fin ? fx : 1);
  // boundary coarse planes of this block
  const int ci = t % CX, cj = t / CX;
  const int I = I0 + ci, J = J0 + cj;
  const bool cown = t < CX * CY && I <= nc - 1 && J <= nc - 1;
  const bool cin = cown && I > 0 && I < nc - 1 && J > 0 && J < nc - 1;
  // edge lanes: coarse column 0 beside the tile's rows
  static_assert(CX * CY + CY <= NT, "edge lanes");
  const int je = J0 + t - CX * CY;
  const bool edge = blk.x == 0 && t >= CX * CY && t < CX * CY + CY && je <= nc - 1;
  const size_t ide = (size_t)min(je, nc - 1) * nc;
  if (cown) {
    if (K0 == 0) fc[(size_t)J * nc + I] = T(0);
    if (K1 == nc) fc[((size_t)(nc - 1) * nc + J) * nc + I] = T(0);
  }
  if (edge)
    for (int K = K0; K < K1; ++K) fc[(size_t)K * nc * nc + ide] = T(0);
  const int Klo = max(K0, 1), Khi = min(K1, nc - 1);
  if (Klo >= Khi) return;
  const int zs = 2 * Klo - 1;                                        // odd
  const int ze = zs + (2 * (Khi - Klo) + ZR) / ZR * ZR - 1;          // whole turns of the ring
  const T *up = HAS_U ? u : f;
  const bool fast = zs - R > 0 && ze + ZR - R < n - 1;

  auto run = [&](auto fast_tag) {
    constexpr bool FAST = decltype(fast_tag)::value;
    auto base = [&](int z) -> size_t { return FAST ? (size_t)z * n * n : plane_base(z, n); };
    // refills past the last fine plane of the chunk re-read that plane (see the sweep)
    auto basec = [&](int z, int cap) -> size_t { return FAST ? (size_t)min(z, cap) * n * n : plane_base(z, n); };
    const int zl = 2 * Khi - 1;  // last fine plane of the chunk's supports
    auto zm = [&](int z) -> T { return FAST ? T(1) : plane_mul<T>(z, n); };
    T ur[ZR], fr[4], hr[4], dr[4];
#pragma unroll
    for (int k = 0; k < ZR; ++k) ur[k] = HAS_U ? up[base(zs - R + k) + cu.off] : T(0);
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      fr[k] = f[base(zs + k) + fcol];
      hr[k] = HAS_U ? up[base(zs + k) + ch.off] : T(0);
      dr[k] = T(0);
    }
    hold_regs(ur);
    hold_regs(fr);
    hold_regs(hr);
    const KOp<T> kop = op;
    const T fmask = fin ? T(1) : T(0);
    auto step = [&](const int z, auto pc) {
      constexpr int P = decltype(pc)::value;  // z - zs mod ZR; z odd exactly when P is even
      const T m = cu.mul;
      // plane z+d sits in slot (P + R + d) mod ZR
      T um3 = RR == 3 ? ur[P % ZR] * (m * zm(z - 3)) : T(0);
      T um2 = ur[(P + R - 2) % ZR] * (m * zm(z - 2)), um1 = ur[(P + R - 1) % ZR] * (m * zm(z - 1));
      T uc = ur[(P + R) % ZR] * (m * zm(z)), up1 = ur[(P + R + 1) % ZR] * (m * zm(z + 1));
      T up2 = ur[(P + R + 2) % ZR] * (m * zm(z + 2));
      T up3 = RR == 3 ? ur[(P + R + 3) % ZR] * (m * zm(z + 3)) : T(0);
      T fz = fr[P % 4] * fmask, hz = hr[P % 4] * (ch.mul * zm(z));
      if constexpr (RR == 3)
        asm volatile("" : "+v"(um3), "+v"(fz), "+v"(hz));
      else
        asm volatile("" : "+v"(um2), "+v"(fz), "+v"(hz));
      __builtin_amdgcn_sched_barrier(0);
      if (HAS_U) ur[P % ZR] = up[basec(z - R + ZR, zl + R) + cu.off];
      fr[P % 4] = f[basec(z + 4, zl) + fcol];
      if (HAS_U) hr[P % 4] = up[basec(z + 4, zl) + ch.off];
      T *pl = plane[P & 1];
      if (has_col) pl[pown] = uc;
      if (has_halo) pl[phal] = hz;
      __syncthreads();
      T lu = HAS_U ? kop.w1 * (((uc - pl[pown - 1]) + (uc - pl[pown + 1])) +
                               ((uc - pl[pown - PX]) + (uc - pl[pown + PX])) + ((uc - um1) + (uc - up1))) +
                         kop.w2 * (((uc - pl[pown - 2]) + (uc - pl[pown + 2])) +
                                   ((uc - pl[pown - 2 * PX]) + (uc - pl[pown + 2 * PX])) +
                                   ((uc - um2) + (uc - up2)))
                   : T(0);
      if constexpr (RR == 3)
        if (HAS_U)
          lu += kop.w3 * (((uc - pl[pown - 3]) + (uc - pl[pown + 3])) +
                          ((uc - pl[pown - 3 * PX]) + (uc - pl[pown + 3 * PX])) + ((uc - um3) + (uc - up3)));
      dr[P % 4] = fz - lu;  // defect of plane z at this column (used on interior supports only)
      if constexpr ((P & 1) == 0) {
        if (z >= zs + 2) {  // z = 2K+1 completes coarse plane K
          const int K = (z - 1) >> 1;
          if (has_col)
            dz[t] = T(0.25) * dr[(P + 2) % 4] + T(0.5) * dr[(P + 3) % 4] + T(0.25) * dr[P % 4];
          __syncthreads();
          if (cown && K < Khi) {
            T sum = T(0);
            if (cin) {
#pragma unroll
              for (int oy = -1; oy <= 1; ++oy)
#pragma unroll
                for (int ox = -1; ox <= 1; ++ox) {
                  const T w = (ox == 0 ? T(0.5) : T(0.25)) * (oy == 0 ? T(0.5) : T(0.25));
                  sum += w * dz[(2 * cj + 1 + oy) * kRDX + 2 * ci + 1 + ox];
                }
            }
            fc[((size_t)K * nc + J) * nc + I] = sum;
          }
        }
      }
    };
    for (int z = zs; z <= ze; z += ZR)
      static_for<ZR>([&](auto pc) { step(z + decltype(pc)::value, pc); });
  };
  if (fast)
    run(std::true_type{});
  else
    run(std::false_type{});
}

// ----------------------- separable (Galerkin) defect + full weighting, z rings ----
// The defect of the separable operator (the P1/P2 form of the pencil sweep, in-plane
// passes through LDS) on the full-weighting support of a CX x CY coarse tile, restricted
// as in the cross kernel: support columns one per thread, P1/P2 and defect rings in
// registers, z weighting per column, x and y weighting through LDS after every odd fine
// plane.
template <typename T, int CX, int CY, int NT>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(sizeof(T) == 4 ? 4 : 1)))
void k_grr3d(const T *__restrict__ f, const T *__restrict__ u, T *__restrict__ fc, int n,
             int kchunk, KOp<T> op, const int *__restrict__ done) {
  constexpr int SX = 2 * CX + 1, SY = 2 * CY + 1, ND = SX * SY;  // support
  constexpr int R = 3, PX = SX + 2 * R, PY = SY + 2 * R, PS = PX * PY, NH = PS - ND;
  constexpr int NYO = PX * SY;
  static_assert(ND <= NT && NH <= NT && NYO <= 2 * NT, "thread mapping");
  __shared__ T upl[PS];
  __shared__ T yb[NYO], ya[NYO];
  __shared__ T dz[ND];
  if (stopped(done)) return;
  const int nc = (n - 1) / 2 + 1;
  const Block3 blk = block3();
  const int I0 = blk.x * CX, J0 = blk.y * CY;
  const int X0 = 2 * I0 - 1, Y0 = 2 * J0 - 1;  // support origin
  const int K0 = blk.z * kchunk, K1 = min(K0 + kchunk, nc);
  const int t = threadIdx.x;
  const bool has_col = t < ND;
  const int dx = has_col ? t % SX : 0, dy = has_col ? t / SX : 0;
  Col3<T> cu, ch;
  cu.init(X0 + dx, Y0 + dy, n);
  int hx = 0, hy = 0;
  const bool has_halo = t < NH;
  if (t < R * PX) {
    hy = t / PX;
    hx = t % PX;
  } else if (t < 2 * R * PX) {
    hy = PY - R + (t - R * PX) / PX;
    hx = (t - R * PX) % PX;
  } else {
    const int hh = t - 2 * R * PX;
    hy = R + hh / (2 * R);
    const int c = hh % (2 * R);
    hx = c < R ? c : PX - 2 * R + c;
  }
  if (has_halo)
    ch.init(X0 - R + hx, Y0 - R + hy, n);
  else
    ch = cu;
  const int pown = (dy + R) * PX + dx + R, phal = hy * PX + hx;
  const int fx = X0 + dx, fy = Y0 + dy;
  const bool fin = has_col && fx > 0 && fx < n - 1 && fy > 0 && fy < n - 1;
  const size_t fcol = (size_t)(fin ? fy : 1) * n + (fin ? fx : 1);
  const bool y2 = t + NT < NYO;
  const int ye0 = t < NYO ? (t / PX + R) * PX + t % PX : R * PX;
  const int ye1 = y2 ? ((t + NT) / PX + R) * PX + (t + NT) % PX : ye0;
  const int xo = dy * PX + dx + R;
  // coarse points of this block
  const int ci = t % CX, cj = t / CX;
  const int I = I0 + ci, J = J0 + cj;
  const bool cown = t < CX * CY && I <= nc - 1 && J <= nc - 1;
  const bool cin = cown && I > 0 && I < nc - 1 && J > 0 && J < nc - 1;
  if (cown) {
    if (K0 == 0) fc[(size_t)J * nc + I] = T(0);
    if (K1 == nc) fc[((size_t)(nc - 1) * nc + J) * nc + I] = T(0);
  }
  const int Klo = max(K0, 1), Khi = min(K1, nc - 1);
  if (Klo >= Khi) return;
  const int zs = 2 * Klo - 1;                              // odd
  const int ze = zs + round_up8(2 * (Khi - Klo) + 1) - 1;  // whole turns of the rings
  const bool fast = zs - R > 0 && ze + 8 < n - 1;

  auto run = [&](auto fast_tag) {
    constexpr bool FAST = decltype(fast_tag)::value;
    auto base = [&](int z) -> size_t { return FAST ? (size_t)z * n * n : plane_base(z, n); };
    auto zm = [&](int z) -> T { return FAST ? T(1) : plane_mul<T>(z, n); };
    const KOp<T> kop = op;
    // ring slots: u and P by (plane - (zs-3)) mod 8, halo by the same mod 4, f and the
    // defects by (plane - zs) mod 4
    T ur[8], hr[4], fr[4], dr[4], p1r[8], p2r[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) ur[k] = u[base(zs - R + k) + cu.off];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      hr[k] = u[base(zs - R + k) + ch.off];
      fr[k] = f[base(zs + k) + fcol];
      dr[k] = T(0);
    }
    hold_regs(ur);
    hold_regs(hr);
    hold_regs(fr);
    auto inplane = [&](T uq, T hq, T &p1, T &p2) {
      if (has_col) upl[pown] = uq;
      if (has_halo) upl[phal] = hq;
      __syncthreads();
      if (t < NYO) {
        const T c = upl[ye0];
        T sb = T(0), sa = T(0);
#pragma unroll
        for (int j = 0; j < 7; ++j) {
          const T v = upl[ye0 + (j - 3) * PX];
          sb += kop.b[j] * v;
          if (j != 3) sa += kop.a[j] * (v - c);
        }
        yb[t] = sb;
        ya[t] = sa;
      }
      __builtin_amdgcn_sched_barrier(0);
      if (y2) {
        const T c = upl[ye1];
        T sb = T(0), sa = T(0);
#pragma unroll
        for (int j = 0; j < 7; ++j) {
          const T v = upl[ye1 + (j - 3) * PX];
          sb += kop.b[j] * v;
          if (j != 3) sa += kop.a[j] * (v - c);
        }
        yb[t + NT] = sb;
        ya[t + NT] = sa;
      }
      __syncthreads();
      const T c1 = yb[xo];
      T s1 = T(0), s2 = T(0);
#pragma unroll
      for (int i = 0; i < 7; ++i) {
        const T vb = yb[xo + i - 3];
        if (i != 3) s1 += kop.a[i] * (vb - c1);
        s1 += kop.b[i] * ya[xo + i - 3];
        s2 += kop.b[i] * vb;
      }
      p1 = s1;
      p2 = s2;
    };
    static_for<6>([&](auto kc) {
      constexpr int K = decltype(kc)::value;
      const int q = zs - R + K;
      T uq = ur[K] * (cu.mul * zm(q)), hq = hr[K % 4] * (ch.mul * zm(q));
      asm volatile("" : "+v"(uq), "+v"(hq));
      __builtin_amdgcn_sched_barrier(0);
      if constexpr (K < 3) ur[K] = u[base(q + 8) + cu.off];
      hr[K % 4] = u[base(q + 4) + ch.off];
      inplane(uq, hq, p1r[K], p2r[K]);
    });
    hold_regs(ur);
    hold_regs(hr);
    const T fmask = fin ? T(1) : T(0);
    auto step = [&](const int z, auto pc) {
      constexpr int P = decltype(pc)::value;  // z - zs mod 8; z odd exactly when P is even
      constexpr int SQ = (P + 6) % 8, SZ = (P + 3) % 8, SH = (P + 2) % 4, SF = P % 4;
      T uq = ur[SQ] * (cu.mul * zm(z + R)), hq = hr[SH] * (ch.mul * zm(z + R));
      T fz = fr[SF] * fmask;
      asm volatile("" : "+v"(uq), "+v"(hq), "+v"(fz));
      __builtin_amdgcn_sched_barrier(0);
      ur[SZ] = u[base(z + 8) + cu.off];  // plane z: used by no later step
      hr[SH] = u[base(z + R + 4) + ch.off];
      fr[SF] = f[base(z + 4) + fcol];
      inplane(uq, hq, p1r[SQ], p2r[SQ]);
      const T c2 = p2r[SZ];
      T lu = T(0);
#pragma unroll
      for (int k = 0; k < 7; ++k) {
        lu += kop.b[k] * p1r[(P + k) % 8];
        if (k != 3) lu += kop.a[k] * (p2r[(P + k) % 8] - c2);
      }
      dr[SF] = fz - lu;  // defect of plane z (used on interior supports only)
      if constexpr ((P & 1) == 0) {
        if (z >= zs + 2) {  // z = 2K+1 completes coarse plane K
          const int K = (z - 1) >> 1;
          if (has_col)
            dz[t] = T(0.25) * dr[(P + 2) % 4] + T(0.5) * dr[(P + 3) % 4] + T(0.25) * dr[P % 4];
          __syncthreads();
          if (cown && K < Khi) {
            T sum = T(0);
            if (cin) {
#pragma unroll
              for (int oy = -1; oy <= 1; ++oy)
#pragma unroll
                for (int ox = -1; ox <= 1; ++ox) {
                  const T w = (ox == 0 ? T(0.5) : T(0.25)) * (oy == 0 ? T(0.5) : T(0.25));
                  sum += w * dz[(2 * cj + 1 + oy) * SX + 2 * ci + 1 + ox];
                }
            }
            fc[((size_t)K * nc + J) * nc + I] = sum;
          }
        }
      }
    };
    for (int z = zs; z <= ze; z += 8)
      static_for<8>([&](auto pc) { step(z + decltype(pc)::value, pc); });
  };
  if (fast)
    run(std::true_type{});
  else
    run(std::false_type{});
}

// ---------------------------------------------- interpolation + correction ----
// Fine tile XW x TY at planes [z0, z1), one column per thread.  Each coarse plane of the
// region around the tile goes through LDS once and is interpolated in x and y at every
// fine column; the four coarse planes around the current fine plane stay in registers
// for the z interpolation.  Coarse planes are loaded four planes (eight fine steps) and
// the fine u eight planes ahead, into register rings that a fully unrolled turn of eight
// fine planes addresses at compile-time positions.
//
// Every lane stores every step, so that no store sits under a branch: lanes past the grid
// and steps past the last plane land on the boundary (clamped address) and store 0 there.
// Bands other than the last are whole turns (the host rounds the band to 8 planes), so no
// block stores outside its own planes and uout may be uin.
template <typename T, int P, int XW>
__global__ __launch_bounds__(XW * TY) void k_prolong3d(const T *__restrict__ v, const T *uin, T *uout,
                                                      int n, int zchunk, const int *__restrict__ done) {
  constexpr int NT = XW * TY, CX = XW / 2 + 4, CY = TY / 2 + 4, CS = CX * CY;
  static_assert(CS + TY + XW + 1 <= NT, "one coarse point or edge point per thread");
  __shared__ T cpl[2][CS + 1];  // the last slot takes the stores of threads past CS
  if (stopped(done)) return;
  const int nc = (n - 1) / 2 + 1;
  const Block3 blk = block3();
  // tiles start at row and column 1 (for n = 2^k + 1 the n - 1 points 1 .. n-1 fill whole
  // tiles); the last band also takes the planes past the last whole band
  const int x0 = 1 + blk.x * XW, y0 = 1 + blk.y * TY;
  const int z0 = blk.z * zchunk;  // even (zchunk is)
  const int z1 = blk.z == gridDim.z - 1 ? n : min(z0 + zchunk, n);
  const int tx = threadIdx.x % XW, ty = threadIdx.x / XW;
  // edge lanes (threads past the coarse points): column 0 beside the tile's rows, row 0
  // above its columns and the corner (0, 0) store those boundary points (0)
  int xe = -1, ye = -1;
  {
    const int e = (int)threadIdx.x - CS;
    if (blk.x == 0 && e >= 0 && e < TY) {
      xe = 0;
      ye = y0 + e;
    } else if (blk.y == 0 && e >= TY && e < TY + XW) {
      ye = 0;
      xe = x0 + e - TY;
    } else if (blk.x == 0 && blk.y == 0 && e == TY + XW) {
      xe = 0;
      ye = 0;
    }
  }
  const bool edge = xe >= 0;
  const size_t ide = (size_t)min(max(ye, 0), n - 1) * n + min(max(xe, 0), n - 1);
  const int x = x0 + tx, y = y0 + ty;
  const int Ib = x0 / 2 - 1, Jb = y0 / 2 - 1;  // coarse region origin
  const bool xyin = x > 0 && x < n - 1 && y > 0 && y < n - 1;
  const size_t col = (size_t)min(y, n - 1) * n + min(x, n - 1);
  // this thread's coarse point of the region (threads below CS)
  const bool has_c = threadIdx.x < CS;
  const int cslot = has_c ? (int)threadIdx.x : CS;
  int coff = nc + 1;
  T cmul = T(0);
  if (has_c) {
    int s = 1;
    const int xf = fold(Ib + (int)threadIdx.x % CX, nc, s), yf = fold(Jb + (int)threadIdx.x / CX, nc, s);
    const bool ok = xf > 0 && xf < nc - 1 && yf > 0 && yf < nc - 1;
    coff = ok ? yf * nc + xf : nc + 1;
    cmul = ok ? T(s) : T(0);
  }
  auto cbase = [&](int K) -> size_t {
    int s = 1;
    int kf = fold(K, nc, s);
    kf = (kf > 0 && kf < nc - 1) ? kf : 1;
    return (size_t)kf * nc * nc;
  };
  auto cmulz = [&](int K) -> T {
    int s = 1;
    const int kf = fold(K, nc, s);
    return (kf > 0 && kf < nc - 1) ? T(s) : T(0);
  };
  // 1D weights of coarse points fine/2-1 .. fine/2+2 for an odd fine index
  constexpr T c0 = P == 3 ? T(-0.0625) : T(0), c1 = P == 3 ? T(0.5625) : T(0.5);
  T wx[4], wy[4];
  {
    const bool ox = x & 1, oy = y & 1;
    wx[0] = ox ? c0 : T(0); wx[1] = ox ? c1 : T(1); wx[2] = ox ? c1 : T(0); wx[3] = ox ? c0 : T(0);
    wy[0] = oy ? c0 : T(0); wy[1] = oy ? c1 : T(1); wy[2] = oy ? c1 : T(0); wy[3] = oy ? c0 : T(0);
  }
  const int lx = (x >> 1) - 1 - Ib, ly = (y >> 1) - 1 - Jb;  // local start of the 4 x 4 window
  auto interp_xy = [&](const T *pl) -> T {
    T s = T(0);
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      T row = T(0);
#pragma unroll
      for (int a = 0; a < 4; ++a) row += wx[a] * pl[(ly + b) * CX + lx + a];
      s += wy[b] * row;
    }
    return s;
  };
  const int kb0 = z0 / 2 - 1;  // first coarse plane of the window
  const int zlast = z0 + round_up8(z1 - z0) - 1;
  T pw[4], cr[4], ur[8];
  // prologue: coarse planes kb0 .. kb0+2 into the window (the first advance brings
  // kb0+3), kb0+3 .. kb0+6 into the coarse ring, fine planes z0 .. z0+7 into the u ring
#pragma unroll
  for (int k = 0; k < 4; ++k) cr[k] = v[cbase(kb0 + 3 + k) + coff];
#pragma unroll
  for (int k = 0; k < 8; ++k) ur[k] = uin[(size_t)min(z0 + k, n - 1) * n * n + col];
  pw[0] = T(0);
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    T c = v[cbase(kb0 + k) + coff];
    const T m = cmul * cmulz(kb0 + k);
    cpl[k & 1][cslot] = m != T(0) ? c * m : T(0);
    __syncthreads();
    pw[k + 1] = interp_xy(cpl[k & 1]);
  }
  __syncthreads();  // the first advance writes cpl[0] again
  hold_regs(cr);
  hold_regs(ur);
  auto step = [&](const int z, auto pc) {
    constexpr int Q = decltype(pc)::value;  // z - z0 mod 8; z even exactly when Q is
    // A ring slot is consumed by arithmetic before its refill is issued, so that the
    // refill can land in the same register (a plain copy would keep the old value alive
    // across the load and cost a register move, and a wait, at the loop's back edge).
    if constexpr ((Q & 1) == 0) {
      // advance the window to coarse planes z/2-1 .. z/2+2
      const int K = z / 2 + 2;
      constexpr int S = Q / 2;  // ring slot of plane K
      const T m = cmul * cmulz(K);
      const T cv = m != T(0) ? cr[S] * m : T(0);
      __builtin_amdgcn_sched_barrier(0);
      cr[S] = v[cbase(K + 4) + coff];
      cpl[S & 1][cslot] = cv;
      __syncthreads();
      const T nv = interp_xy(cpl[S & 1]);
      pw[0] = pw[1];
      pw[1] = pw[2];
      pw[2] = pw[3];
      pw[3] = nv;
    }
    const T val = (Q & 1) == 0 ? pw[1] : c0 * pw[0] + c1 * pw[1] + c1 * pw[2] + c0 * pw[3];
    const bool inside = xyin && z > 0 && z < n - 1;
    const T res = inside ? ur[Q] + val : T(0);
    __builtin_amdgcn_sched_barrier(0);
    ur[Q] = uin[(size_t)min(z + 8, n - 1) * n * n + col];
    uout[(size_t)min(z, n - 1) * n * n + col] = res;
    if (edge) uout[(size_t)min(z, n - 1) * n * n + ide] = T(0);
  };
  for (int z = z0; z <= zlast; z += 8)
    static_for<8>([&](auto pc) { step(z + decltype(pc)::value, pc); });
}

int cdiv(long a, long b) { return (int)((a + b - 1) / b); }

template <typename T>
KOp<T> to_kop3(const LevelOp &op, double omega) {
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

// Plane bands of the 3D kernels: 8..64 fine planes (4..32 coarse), about four rounds of
// resident blocks per launch (the plane loop of a block is latency-bound, so several
// blocks per CU in flight beat one long march each).
constexpr int kMinPlanes = 8, kMaxPlanes = 64, kRounds3d = 4;

// Whether a level takes the wide tiles (64 fine columns) in the cross kernels: rows of
// 256 bytes and more keep the HBM pages of a plane busy on the large levels, while the
// narrow tiles give more blocks on the small ones.  Environment variable `var` = 0 or 1
// forces the choice.
template <typename T>
bool wide_tiles(int n, const char *var) {
  const char *e = getenv(var);
  if (e != nullptr && *e != 0) return atoi(e) != 0;
  return (size_t)n * n * n * sizeof(T) >= ((size_t)96 << 20);
}

template <typename T, typename TO, int XW, int RR = 2, int YS = 1>
const void *xsweep3d_fn(int mode, bool has_u) {
  if (mode == kSweepZ2) return (const void *)k_xsweep3d<T, TO, kSweepZ2, true, XW, RR, YS>;
  if (mode == kSweep) return has_u ? (const void *)k_xsweep3d<T, TO, kSweep, true, XW, RR, YS> : (const void *)k_xsweep3d<T, TO, kSweep, false, XW, RR, YS>;
  if (mode == kSweepRB) return has_u ? (const void *)k_xsweep3d<T, TO, kSweepRB, true, XW, RR, YS> : (const void *)k_xsweep3d<T, TO, kSweepRB, false, XW, RR, YS>;
  if (mode == kResidual) return has_u ? (const void *)k_xsweep3d<T, TO, kResidual, true, XW, RR, YS> : (const void *)k_xsweep3d<T, TO, kResidual, false, XW, RR, YS>;
  return has_u ? (const void *)k_xsweep3d<T, TO, kNormOnly, true, XW, RR, YS> : (const void *)k_xsweep3d<T, TO, kNormOnly, false, XW, RR, YS>;
}

// Rows per thread of the wide cross-sweep tiles: 2 (a 64 x 16 tile per block; FP32 117
// VGPRs, FP64 187: 1025^3 FP64 sweep 6632 -> 6269 us, FP64 residual cast to FP32 5543 ->
// 5328 us against one row), except the FP64 norm-only pass, which spills with two rows;
// MG_X3_YS = 1 or 2 sets every case.
template <typename T>
int x3_ys(int mode) {
  const char *e = getenv("MG_X3_YS");
  const int env = e != nullptr ? atoi(e) : 0;
  if (env == 1 || env == 2) return env;
  return sizeof(T) == 8 && mode == kNormOnly ? 1 : 2;
}

// FP32 wide cross-sweep tiles of 128 columns (MG_X3_W128 = 0: 64 columns).
inline bool wide128() {
  const char *e = getenv("MG_X3_W128");
  return e == nullptr || atoi(e) != 0;
}

// Rows per wavefront of the pencil sweep: 2 (FP32 126 VGPRs, four wavefronts per SIMD;
// FP64 209), doubled for FP32 levels from 513^3 up.  Measured at 513^3: FP32 two rows
// 571 us, four 540 us, but four rows lose on the smaller levels (257^3: 81 against
// 94 us); FP64 one row (147 VGPRs) was slower than two in the whole solve (316 against
// 308 ms).  MG_GPEN_ROWS = 1 or 2 sets the factor on every level.
template <typename T>
constexpr int gpen_rows() { return 2; }
template <typename T>
int gpen_rows_scale(int n) {
  const char *e = getenv("MG_GPEN_ROWS");
  if (e != nullptr && *e != 0) return atoi(e) == 2 ? 2 : 1;
  return sizeof(T) == 4 && n >= 513 ? 2 : 1;
}
template <typename T, typename TO, int YR>
const void *gpen3d_fn_rows(int mode) {
  if (mode == kSweepZ2) return (const void *)k_gpen3d<T, TO, kSweepZ2, YR>;
  if (mode == kSweep) return (const void *)k_gpen3d<T, TO, kSweep, YR>;
  if (mode == kSweepRB) return (const void *)k_gpen3d<T, TO, kSweepRB, YR>;
  if (mode == kResidual) return (const void *)k_gpen3d<T, TO, kResidual, YR>;
  return (const void *)k_gpen3d<T, TO, kNormOnly, YR>;
}
}  // namespace

bool x3_r3();

// Whether two sweeps from zero run in one pass on a level of this operator: the cross
// kernels (radius 2 and 3) and the pencil kernel all have the mode.
bool sweep3d_z2_ok(const LevelOp &op) {
  (void)op;
  return true;
}

namespace {

template <typename T, typename TO>
const void *sweep3d_fn(int mode, bool has_u, int xw, int ys = 1) {
  if constexpr (sizeof(T) == 4)
    if (xw == 128) return xsweep3d_fn<T, TO, 128, 2, 2>(mode, has_u);
  return xw == 64 ? (ys == 2 ? xsweep3d_fn<T, TO, 64, 2, 2>(mode, has_u) : xsweep3d_fn<T, TO, 64>(mode, has_u))
                  : xsweep3d_fn<T, TO, 32>(mode, has_u);
}

}  // namespace

int sweep_partials_3d(int n) {
  const long tiles = (long)cdiv(n, TX) * cdiv(n, TY);
  // the pencil sweep: 58 columns x 4 wavefronts of gpen_rows rows per block
  const long pencils = (long)cdiv(n, 58) * cdiv(n, 4 * std::min(gpen_rows<float>(), gpen_rows<double>()));
  return (int)(std::max(tiles, pencils) * cdiv(n, kMinPlanes));
}

// The sixth-order radius-3 cross runs the cross kernels with R = 3 (MG_X3_R3=0: the
// separable kernels of the Galerkin levels instead).
bool x3_r3() {
  static const bool on = [] {
    const char *e = getenv("MG_X3_R3");
    return e == nullptr || atoi(e) != 0;
  }();
  return on;
}

template <typename T, typename TO>
hipError_t launch_sweep_3d(int mode, const LevelOp &op, double omega, const T *f, const T *u,
                           TO *out, int n, double *partials, int *nparts, const int *done,
                           hipStream_t s, int colour) {
  if (colour != 0) {  // one colour of a red-black sweep: the kSweepRB instances
    if (mode != kSweep || !std::is_same<T, TO>::value) return hipErrorInvalidValue;
    mode = kSweepRB;
  }
  if (mode == kSweepZ2) {  // two sweeps from zero: the kernels read u from f
    if (!std::is_same<T, TO>::value || !sweep3d_z2_ok(op)) return hipErrorInvalidValue;
    u = f;
  }
  // a zero initial guess needs no operator: the cross kernel's u-free path serves every
  // operator (it uses om_d only); radius-3 crosses (sixth order) take the cross kernel
  // with R = 3 unless MG_X3_R3 = 0; every other operator the separable pencil kernel
  const bool xpath = op.cross || u == nullptr;
  const bool x3path = !xpath && op.cross3 && x3_r3();
  KOp<T> k = to_kop3<T>(op, omega);
  k.colour = colour;
  if (!xpath && !x3path) {
    constexpr int Y1 = gpen_rows<T>(), Y2 = 2 * gpen_rows<T>();
    const int yr = Y1 * gpen_rows_scale<T>(n);
    const void *fn = yr == Y1 ? gpen3d_fn_rows<T, TO, Y1>(mode) : gpen3d_fn_rows<T, TO, Y2>(mode);
    const int ptiles = cdiv(n, 58) * cdiv(n, 4 * yr);
    const int pzc = (std::min(kMaxPlanes, band_rows(n, ptiles, kRounds3d * resident_blocks(fn, 256, 0), kMinPlanes)) + 7) / 8 * 8;
    const dim3 pgrid(cdiv(n, 58), cdiv(n, 4 * yr), cdiv(n, pzc));
    if (nparts) *nparts = pgrid.x * pgrid.y * pgrid.z;
#define MG_GP(MODE, YR) hipLaunchKernelGGL((k_gpen3d<T, TO, MODE, YR>), pgrid, dim3(256), 0, s, f, u, out, n, pzc, k, partials, done)
#define MG_GPM(YR)                          \
    if (mode == kSweepZ2) MG_GP(kSweepZ2, YR);      \
    else if (mode == kSweep) MG_GP(kSweep, YR);     \
    else if (mode == kSweepRB) MG_GP(kSweepRB, YR); \
    else if (mode == kResidual) MG_GP(kResidual, YR); \
    else MG_GP(kNormOnly, YR);
    if (yr == Y1) {
      MG_GPM(Y1)
    } else {
      MG_GPM(Y2)
    }
#undef MG_GPM
#undef MG_GP
    return hipGetLastError();
  }
  int xw = (xpath && wide_tiles<T>(n, "MG_X3_W")) || x3path ? 64 : TX;
  const int ys = xpath && xw == 64 ? x3_ys<T>(mode) : 1;  // rows per thread of the cross sweep
  // FP32 wide tiles: 128 x 16 points, 1024 threads (121 VGPRs; FP64 would spill).  Half
  // the x halo and row-alignment bytes of 64-column tiles: 1025^3 sweep 3472 -> 3198 us
  if (xpath && xw == 64 && ys == 2 && sizeof(T) == 4 && wide128()) xw = 128;
  const int nt = xw * TY;
  // tiles and chunks cover points 1 .. n-1 (the kernel stores row, column and plane 0)
  const int tiles = cdiv(n - 1, xw) * cdiv(n - 1, TY * ys);
  const void *occ_fn = x3path ? xsweep3d_fn<T, TO, 64, 3>(mode, true) : sweep3d_fn<T, TO>(mode, u != nullptr, xw, ys);
  const int zr = x3path ? 16 : kZR;  // planes per loop turn of the kernel
  const int zc = (std::min(kMaxPlanes, band_rows(n, tiles, kRounds3d * resident_blocks(occ_fn, nt, 0),
                                                 kMinPlanes)) + zr - 1) / zr * zr;
  const dim3 grid(cdiv(n - 1, xw), cdiv(n - 1, TY * ys), cdiv(n - 1, zc));
  if (nparts) *nparts = grid.x * grid.y * grid.z;
  if (x3path) {
#define MG_X33(MODE) hipLaunchKernelGGL((k_xsweep3d<T, TO, MODE, true, 64, 3>), grid, dim3(nt), 0, s, f, u, out, n, zc, k, partials, done)
    if (mode == kSweepZ2) MG_X33(kSweepZ2);
    else if (mode == kSweep) MG_X33(kSweep);
    else if (mode == kSweepRB) MG_X33(kSweepRB);
    else if (mode == kResidual) MG_X33(kResidual);
    else MG_X33(kNormOnly);
#undef MG_X33
    return hipGetLastError();
  }
#define MG_X3(MODE, XW, YS)                                                                  \
  if (u != nullptr)                                                                          \
    hipLaunchKernelGGL((k_xsweep3d<T, TO, MODE, true, XW, 2, YS>), grid, dim3(nt), 0, s, f, u, out, n, zc, k, partials, done); \
  else                                                                                       \
    hipLaunchKernelGGL((k_xsweep3d<T, TO, MODE, false, XW, 2, YS>), grid, dim3(nt), 0, s, f, u, out, n, zc, k, partials, done);
  if (mode == kSweepZ2) {
#define MG_XZ(XW, YS) hipLaunchKernelGGL((k_xsweep3d<T, TO, kSweepZ2, true, XW, 2, YS>), grid, dim3(nt), 0, s, f, u, out, n, zc, k, partials, done)
    if constexpr (sizeof(T) == 4)
      if (xw == 128) {
        MG_XZ(128, 2);
        return hipGetLastError();
      }
    if (xw == 64 && ys == 2) MG_XZ(64, 2);
    else if (xw == 64) MG_XZ(64, 1);
    else MG_XZ(32, 1);
#undef MG_XZ
    return hipGetLastError();
  }
  if constexpr (sizeof(T) == 4)
    if (xw == 128) {
      if (mode == kSweep) { MG_X3(kSweep, 128, 2) }
      else if (mode == kSweepRB) { MG_X3(kSweepRB, 128, 2) }
      else if (mode == kResidual) { MG_X3(kResidual, 128, 2) }
      else { MG_X3(kNormOnly, 128, 2) }
      return hipGetLastError();
    }
  if (xw == 64 && ys == 2) {
    if (mode == kSweep) { MG_X3(kSweep, 64, 2) }
    else if (mode == kSweepRB) { MG_X3(kSweepRB, 64, 2) }
    else if (mode == kResidual) { MG_X3(kResidual, 64, 2) }
    else { MG_X3(kNormOnly, 64, 2) }
  } else if (xw == 64) {
    if (mode == kSweep) { MG_X3(kSweep, 64, 1) }
    else if (mode == kSweepRB) { MG_X3(kSweepRB, 64, 1) }
    else if (mode == kResidual) { MG_X3(kResidual, 64, 1) }
    else { MG_X3(kNormOnly, 64, 1) }
  } else {
    if (mode == kSweep) { MG_X3(kSweep, 32, 1) }
    else if (mode == kSweepRB) { MG_X3(kSweepRB, 32, 1) }
    else if (mode == kResidual) { MG_X3(kResidual, 32, 1) }
    else { MG_X3(kNormOnly, 32, 1) }
  }
#undef MG_X3
  return hipGetLastError();
}

template <typename T>
hipError_t launch_rbsweep_3d(const LevelOp &op, double omega, const T *f, const T *u, T *out, int n,
                             double *partials, int *nparts, const int *done, hipStream_t s) {
  if (!op.cross) return hipErrorInvalidValue;
  // 60 x 8 tiles, 768 threads (measured at 513^3 against 28 x 16 tiles, 640 threads:
  // 56.4 against 57.8 ms per FP64 red-black solve)
  constexpr int xw = 60, yw = 8, nt = (xw + 4) * (yw + 4);
  const void *fn = u != nullptr ? (const void *)k_rbxsweep3d<T, true, xw, yw> : (const void *)k_rbxsweep3d<T, false, xw, yw>;
  const int tiles = cdiv(n, xw) * cdiv(n, yw);
  // bands of at least 32 planes: every band takes four extra red planes
  const int zc = std::min(kMaxPlanes, band_rows(n, tiles, kRounds3d * resident_blocks(fn, nt, 0), 32));
  const dim3 grid(cdiv(n, xw), cdiv(n, yw), cdiv(n, zc));
  if (nparts) *nparts = grid.x * grid.y * grid.z;
  const KOp<T> k = to_kop3<T>(op, omega);
#define MG_RB3(HU, W, H) hipLaunchKernelGGL((k_rbxsweep3d<T, HU, W, H>), grid, dim3(nt), 0, s, f, u, out, n, zc, k, partials, done)
  if (u != nullptr)
    MG_RB3(true, xw, yw);
  else
    MG_RB3(false, xw, yw);
#undef MG_RB3
  return hipGetLastError();
}

// Two omega-Jacobi sweeps of the cross in one pass (the red-black pass with both steps over
// every point).
template <typename T>
hipError_t launch_x2sweep_3d(const LevelOp &op, double omega, const T *f, const T *u, T *out, int n,
                             double *partials, int *nparts, const int *done, hipStream_t s) {
  if (!op.cross) return hipErrorInvalidValue;
  // the red-black pass's 60 x 8 tiles, 768 threads
  constexpr int xw = 60, yw = 8, nt = (xw + 4) * (yw + 4);
  const void *fn = u != nullptr ? (const void *)k_rbxsweep3d<T, true, xw, yw, true> : (const void *)k_rbxsweep3d<T, false, xw, yw, true>;
  const int tiles = cdiv(n, xw) * cdiv(n, yw);
  // bands of at least 32 planes: every band takes four extra first-sweep planes
  const int zc = std::min(kMaxPlanes, band_rows(n, tiles, kRounds3d * resident_blocks(fn, nt, 0), 32));
  const dim3 grid(cdiv(n, xw), cdiv(n, yw), cdiv(n, zc));
  if (nparts) *nparts = grid.x * grid.y * grid.z;
  const KOp<T> k = to_kop3<T>(op, omega);
#define MG_RB3(HU, W, H) hipLaunchKernelGGL((k_rbxsweep3d<T, HU, W, H, true>), grid, dim3(nt), 0, s, f, u, out, n, zc, k, partials, done)
  if (u != nullptr)
    MG_RB3(true, xw, yw);
  else
    MG_RB3(false, xw, yw);
#undef MG_RB3
  return hipGetLastError();
}

hipError_t launch_sweep_corr_3d(const LevelOp &op, double omega, const float *f, const float *e,
                                double *u64, int n, const int *done, hipStream_t s) {
  if (!op.cross || op.cross3) return hipErrorInvalidValue;
  // the FP32 sweep's tiles: 128 x 16 points (two rows per thread) on the large levels
  const bool wide = wide_tiles<float>(n, "MG_X3_W");
  const int xw = wide ? (wide128() ? 128 : 64) : TX, ys = wide ? 2 : 1, nt = xw * TY;
  const void *fn = xw == 128 ? (const void *)k_xsweep3d<float, double, kSweepCorr, true, 128, 2, 2>
                 : xw == 64  ? (const void *)k_xsweep3d<float, double, kSweepCorr, true, 64, 2, 2>
                             : (const void *)k_xsweep3d<float, double, kSweepCorr, true, TX, 2, 1>;
  const int tiles = cdiv(n - 1, xw) * cdiv(n - 1, TY * ys);
  const int zc = (std::min(kMaxPlanes, band_rows(n, tiles, kRounds3d * resident_blocks(fn, nt, 0), kMinPlanes)) +
                  kZR - 1) / kZR * kZR;
  const dim3 grid(cdiv(n - 1, xw), cdiv(n - 1, TY * ys), cdiv(n - 1, zc));
  const KOp<float> k = to_kop3<float>(op, omega);
  if (xw == 128)
    hipLaunchKernelGGL((k_xsweep3d<float, double, kSweepCorr, true, 128, 2, 2>), grid, dim3(nt), 0, s, f, e, u64, n,
                       zc, k, nullptr, done);
  else if (xw == 64)
    hipLaunchKernelGGL((k_xsweep3d<float, double, kSweepCorr, true, 64, 2, 2>), grid, dim3(nt), 0, s, f, e, u64, n,
                       zc, k, nullptr, done);
  else
    hipLaunchKernelGGL((k_xsweep3d<float, double, kSweepCorr, true, TX, 2, 1>), grid, dim3(nt), 0, s, f, e, u64, n,
                       zc, k, nullptr, done);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_resid_restrict_3d(const LevelOp &op, const T *f, const T *u, T *fc, int n,
                                    const int *done, hipStream_t s) {
  const int nc = (n - 1) / 2 + 1;
  // the cross kernel also serves every operator on a zero u (the defect is f)
  if (op.cross || u == nullptr) {
    // 16 x 3 coarse columns per 256-thread block on the small levels, 16 x 7 per 512
    // threads from 257^3 up (support 33 x 15, 90% of it owned; wider or larger tiles
    // measured slower).  MG_XRR_TALL = 0 or 1 forces the choice.
    bool tall = n >= 257;
    if (const char *e = getenv("MG_XRR_TALL")) {
      if (*e != 0) tall = atoi(e) != 0;
    }
    const int cx = 16, cy = tall ? 7 : 3, nt = tall ? 512 : 256;
    // coarse tiles cover columns 1 .. nc-1 (the kernel stores column 0)
    const int ctiles = cdiv(nc - 1, cx) * cdiv(nc, cy);
    const void *fx = tall ? (u != nullptr ? (const void *)k_xrr3d<T, true, 16, 7, 512> : (const void *)k_xrr3d<T, false, 16, 7, 512>)
                          : (u != nullptr ? (const void *)k_xrr3d<T, true, 16, 3, 256> : (const void *)k_xrr3d<T, false, 16, 3, 256>);
    // coarse planes per band: 4m-1, so that the 8m-1 fine planes of a band fill m turns
    // of the plane ring but one plane
    const int kb = std::min(kMaxPlanes / 2, band_rows(nc, ctiles, kRounds3d * resident_blocks(fx, nt, 0), kMinPlanes / 2));
    const int kc = std::max(3, (kb + 1) / 4 * 4 - 1);
    const dim3 grid(cdiv(nc - 1, cx), cdiv(nc, cy), cdiv(nc, kc));
    const KOp<T> k = to_kop3<T>(op, 1.0);
#define MG_XRR(CX, CY, NT)                                                                  \
  if (u != nullptr)                                                                         \
    hipLaunchKernelGGL((k_xrr3d<T, true, CX, CY, NT>), grid, dim3(nt), 0, s, f, u, fc, n, kc, k, done); \
  else                                                                                      \
    hipLaunchKernelGGL((k_xrr3d<T, false, CX, CY, NT>), grid, dim3(nt), 0, s, f, u, fc, n, kc, k, done);
    if (tall) {
      MG_XRR(16, 7, 512)
    } else {
      MG_XRR(16, 3, 256)
    }
#undef MG_XRR
    return hipGetLastError();
  }
  if (op.cross3 && x3_r3()) {
    // the radius-3 cross: 16 x 7 coarse columns per 512 threads; coarse planes per band
    // 8m-1, so that the 16m-1 fine planes of a band fill m turns of the 16-plane ring
    const int ctiles = cdiv(nc - 1, 16) * cdiv(nc, 7);
    const void *fx = (const void *)k_xrr3d<T, true, 16, 7, 512, 3>;
    const int kb = std::min(kMaxPlanes / 2, band_rows(nc, ctiles, kRounds3d * resident_blocks(fx, 512, 0), kMinPlanes / 2));
    const int kc = std::max(7, (kb + 1) / 8 * 8 - 1);
    const dim3 grid(cdiv(nc - 1, 16), cdiv(nc, 7), cdiv(nc, kc));
    hipLaunchKernelGGL((k_xrr3d<T, true, 16, 7, 512, 3>), grid, dim3(512), 0, s, f, u, fc, n, kc, to_kop3<T>(op, 1.0), done);
    return hipGetLastError();
  }
  // every other operator: the separable defect kernel
  const int ctiles = cdiv(nc, 16) * cdiv(nc, 7);
  const void *fx = (const void *)k_grr3d<T, 16, 7, 512>;
  const int kb = std::min(kMaxPlanes / 2, band_rows(nc, ctiles, kRounds3d * resident_blocks(fx, 512, 0), kMinPlanes / 2));
  const int kc = std::max(3, (kb + 1) / 4 * 4 - 1);
  const dim3 grid(cdiv(nc, 16), cdiv(nc, 7), cdiv(nc, kc));
  hipLaunchKernelGGL((k_grr3d<T, 16, 7, 512>), grid, dim3(512), 0, s, f, u, fc, n, kc, to_kop3<T>(op, 1.0), done);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_prolong_correct_3d(int prolong, const T *v, const T *uin, T *uout, int n,
                                     const int *done, hipStream_t s) {
  const int xw = wide_tiles<T>(n, "MG_P3_W") ? 64 : TX, nt = xw * TY;
  // tiles cover points 1 .. n-1 (the kernel stores row and column 0)
  const int tiles = cdiv(n - 1, xw) * cdiv(n - 1, TY);
  const void *fn = xw == 64 ? (prolong == 3 ? (const void *)k_prolong3d<T, 3, 64> : (const void *)k_prolong3d<T, 1, 64>)
                            : (prolong == 3 ? (const void *)k_prolong3d<T, 3, TX> : (const void *)k_prolong3d<T, 1, TX>);
  // bands of whole turns (8 planes): no block stores outside its planes; the last band
  // takes the remainder (for n = 2^k + 1 the boundary plane)
  const int zc = (std::min(kMaxPlanes, band_rows(n, tiles, kRounds3d * resident_blocks(fn, nt, 0), kMinPlanes)) + 7) / 8 * 8;
  const dim3 grid(cdiv(n - 1, xw), cdiv(n - 1, TY), std::max(1, (n - 1) / zc));
#define MG_P3(PP, XW) hipLaunchKernelGGL((k_prolong3d<T, PP, XW>), grid, dim3(nt), 0, s, v, uin, uout, n, zc, done)
  if (xw == 64) {
    if (prolong == 3) MG_P3(3, 64);
    else MG_P3(1, 64);
  } else {
    if (prolong == 3) MG_P3(3, TX);
    else MG_P3(1, TX);
  }
#undef MG_P3
  return hipGetLastError();
}

// Set-up of the 3D kernels before their first launch (none of them needs dynamic LDS).
hipError_t prepare_3d() { return hipSuccess; }

template hipError_t launch_sweep_3d<double, double>(int, const LevelOp &, double, const double *,
                                                    const double *, double *, int, double *, int *,
                                                    const int *, hipStream_t, int);
template hipError_t launch_sweep_3d<float, float>(int, const LevelOp &, double, const float *,
                                                  const float *, float *, int, double *, int *,
                                                  const int *, hipStream_t, int);
template hipError_t launch_sweep_3d<double, float>(int, const LevelOp &, double, const double *,
                                                   const double *, float *, int, double *, int *,
                                                   const int *, hipStream_t, int);
template hipError_t launch_rbsweep_3d<double>(const LevelOp &, double, const double *, const double *,
                                              double *, int, double *, int *, const int *, hipStream_t);
template hipError_t launch_rbsweep_3d<float>(const LevelOp &, double, const float *, const float *,
                                             float *, int, double *, int *, const int *, hipStream_t);
template hipError_t launch_x2sweep_3d<double>(const LevelOp &, double, const double *, const double *,
                                              double *, int, double *, int *, const int *, hipStream_t);
template hipError_t launch_x2sweep_3d<float>(const LevelOp &, double, const float *, const float *,
                                             float *, int, double *, int *, const int *, hipStream_t);
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
