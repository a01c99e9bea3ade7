// gs2d.hip -- the omega red-black Gauss-Seidel partial step (section 3.1 eqs. S_rb and
// S_GS) on 2D levels whose operator is a cross of radius 2 (fourth order) or 3 (sixth
// order).
//
// A partial step updates the points of one colour in lexicographic order (x fastest), each
// from the current values: its same-colour neighbours at -2 e_x and -2 e_y are already new,
// every other value it reads is old.  Along a row the new values of the colour obey the
// first-order recurrence
//   x_i = A x_{i-2} + B_i,   A = -omega c_2 / a_0   (c_2 the coefficient at +-2 e_x),
// where B_i holds the old values and the new value two rows below; across rows each point
// depends on the point two rows below.  |A| is about 1/50, and an error in a starting value
// shrinks by about |A| / (1 - |A|) per same-colour step, left to right and bottom to top, so
// after ten steps (twenty columns or rows) it is below 1e-16 of the values.
//
// Layout.  A wave owns a strip of 128 columns, two per lane, so each lane holds one point
// of each colour per row.  The leftmost kHaloCols columns are recomputed from an approximate
// start (old values in place of new ones left of the strip) and not stored; so are the
// rightmost lanes whose neighbours would lie beyond the strip.  The wave marches up a band
// of rows starting kHaloRows rows below it (row 1, exactly, for the first band).  Per row
// each lane forms B for its point of the colour from a register ring of rows (the new value
// two rows below is already there; the loads run several rows ahead), the recurrence runs
// as a 64-lane inclusive scan of the affine maps x -> A x + B (six shuffle steps), and the
// finished row is stored.
// Beyond the boundary, values are odd reflections of the current ones; at the first two
// points of a row the -2 e_x neighbour is such a reflection of an old value or a boundary
// zero, and the chain restarts there (A = 0).  No LDS, no barriers.
#include <algorithm>
#include <utility>

#include "mg_internal.h"

namespace mgk {
namespace {

constexpr int kLanes = 64;
constexpr int kWaves = 4;           // waves per block, independent of each other
constexpr int kHaloCols = 20;       // columns recomputed left of a strip (ten steps)
constexpr int kHaloRows = 20;       // rows recomputed below a band (ten steps)
constexpr int kMinBandRows = 64;

__device__ __forceinline__ bool stopped(const int *done) { return done != nullptr && *done != 0; }

template <typename F, int... I>
__device__ __forceinline__ void static_for_impl(F &&f, std::integer_sequence<int, I...>) {
  (f(std::integral_constant<int, I>{}), ...);
}
template <int N, typename F>
__device__ __forceinline__ void static_for(F &&f) {
  static_for_impl(f, std::make_integer_sequence<int, N>{});
}

__device__ __forceinline__ int fold(int i, int n, int &sign) {
  if (i < 0) { i = -i; sign = -sign; }
  if (i > n - 1) { i = 2 * (n - 1) - i; sign = -sign; }
  return i;
}

// lanes of a strip whose results are stored: after the halo, before the lanes whose
// right neighbours (up to R columns) would be past the strip
template <int R>
constexpr int out_lanes() { return kLanes - kHaloCols / 2 - (R + 1) / 2; }

template <typename T>
struct GsCoef {
  T c[4];   // c[d]: coefficient of the entries at +-d (d = 1..3) along either axis
  T om_d;   // omega / a_0
};

template <typename T, int R>
__global__ __launch_bounds__(kLanes * kWaves) void k_gs2d(const T *__restrict__ f, const T *__restrict__ uin,
                                                      T *__restrict__ uout, int n, int colour,
                                                      int strips, int bands, int band_rows,
                                                      GsCoef<T> k, const int *__restrict__ done) {
  done = slot_done(done);
  if (stopped(done)) return;
  const size_t np = (size_t)n * n;
  f = slot_ptr(f, np);
  uin = slot_ptr(uin, np);
  uout = slot_ptr(uout, np);
  const int lane = threadIdx.x & (kLanes - 1);
  const int wave = blockIdx.x * kWaves + (int)(threadIdx.x / kLanes);
  if (wave >= strips * bands) return;  // the whole wave leaves
  constexpr int OUT = 2 * out_lanes<R>();
  const int strip = wave % strips, band = wave / strips;
  const int x0 = 1 - kHaloCols + strip * OUT + 2 * lane;  // odd: columns x0 and x0 + 1
  const int jo0 = 1 + band * band_rows;                  // first stored row
  const int jo1 = min(jo0 + band_rows, n - 1);           // one past the last stored row
  const int js = max(1, jo0 - kHaloRows);                // first row marched
  // columns: folded index and the odd-reflection factor (0 on the boundary)
  int sg0 = 1, sg1 = 1;
  const int c0 = fold(x0, n, sg0), c1 = fold(x0 + 1, n, sg1);
  const bool in0 = c0 > 0 && c0 < n - 1, in1 = c1 > 0 && c1 < n - 1;
  const T m0 = in0 ? T(sg0) : T(0), m1 = in1 ? T(sg1) : T(0);
  const int a0 = in0 ? c0 : 1, a1 = in1 ? c1 : 1;
  auto load = [&](int y, T &v0, T &v1) {
    int sy = 1;
    const int yf = fold(y, n, sy);
    const bool ok = yf > 0 && yf < n - 1;
    const size_t base = (size_t)(ok ? yf : 1) * n;
    const T my = ok ? T(sy) : T(0);
    v0 = uin[base + a0] * (m0 * my);
    v1 = uin[base + a1] * (m1 * my);
  };
  const bool out_lane = lane >= kHaloCols / 2 && lane < kHaloCols / 2 + out_lanes<R>();
  const bool st0 = out_lane && x0 >= 0 && x0 <= n - 1;
  const bool st1 = (out_lane || x0 + 1 == 0) && x0 + 1 >= 0 && x0 + 1 <= n - 1;
  auto store = [&](int y, T v0, T v1) {
    const size_t base = (size_t)y * n;
    if (st0) uout[base + x0] = v0;
    if (st1) uout[base + x0 + 1] = v1;
  };
  if (band == 0) store(0, T(0), T(0));
  if (jo1 == n - 1) store(n - 1, T(0), T(0));

  // Register rings, addressed at compile-time slots in a loop turn unrolled to the ring
  // length UL: row y of the lane's two columns sits in slot (y - js + R) mod UL, f of row y
  // in slot (y - js) mod 4.  A slot is refilled right after its last use, so the loads run
  // UL - 2R rows (u) and four rows (f) ahead of their use.
  constexpr int UL = R == 2 ? 8 : 12;
  T w0[UL], w1[UL], g0[4], g1[4];
#pragma unroll
  for (int r = 0; r < UL; ++r) load(js - R + r, w0[r], w1[r]);
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const size_t row = (size_t)min(js + r, n - 2) * n;
    g0[r] = f[row + a0];
    g1[r] = f[row + a1];
  }
  const T A_link = -k.om_d * k.c[2];
  auto step = [&](const int j, auto pc) {
    constexpr int P = decltype(pc)::value;
    if (j >= jo1) return;  // past the band (the same for the whole wave)
    const int sel = colour == 1 ? (j & 1) : ((j & 1) ^ 1);  // the colour's column: x0 + sel
    const int xc = x0 + sel;
    constexpr int S0 = (P + R) % UL;  // slot of row j
    // row j at columns x0 - 4 .. x0 + 5 from lanes l-2 .. l+2 (beyond the wave: unused)
    T col[10];
    col[4] = w0[S0];
    col[5] = w1[S0];
    col[2] = __shfl_up(w0[S0], 1, kLanes);
    col[3] = __shfl_up(w1[S0], 1, kLanes);
    col[6] = __shfl_down(w0[S0], 1, kLanes);
    col[7] = __shfl_down(w1[S0], 1, kLanes);
    if (R == 3) {
      col[0] = __shfl_up(w0[S0], 2, kLanes);
      col[1] = __shfl_up(w1[S0], 2, kLanes);
      col[8] = __shfl_down(w0[S0], 2, kLanes);
      col[9] = __shfl_down(w1[S0], 2, kLanes);
    } else {
      col[0] = col[1] = col[8] = col[9] = T(0);
    }
    auto ux = [&](int d) { return sel ? col[5 + d] : col[4 + d]; };  // row j at xc + d
    auto uy = [&](int d) {                                         // column xc at row j + d
      return sel ? w1[(P + R + d + UL) % UL] : w0[(P + R + d + UL) % UL];
    };
    const T up = ux(0);
    const T fs = sel ? g1[P % 4] : g0[P % 4];
    const bool active = xc >= 1 && xc <= n - 2;
    const bool start = xc <= 2;  // the -2 e_x neighbour is beyond the boundary or on it
    // the defect without the -2 e_x term (which the recurrence supplies), difference form
    T lu = T(0);
#pragma unroll
    for (int d = 1; d <= R; ++d) {
      lu += k.c[d] * ((uy(d) - up) + (uy(-d) - up));
      lu += k.c[d] * (ux(d) - up);
      if (d != 2) lu += k.c[d] * (ux(-d) - up);
    }
    T A, B;
    if (!active) {
      A = T(0);
      B = T(0);
    } else if (start) {
      A = T(0);
      B = up + k.om_d * (fs - (lu + k.c[2] * (ux(-2) - up)));
    } else {
      A = A_link;
      B = up + k.om_d * ((fs - lu) + k.c[2] * up);
    }
    // inclusive scan of x -> A x + B over the lanes (lane l composes lanes <= l)
#pragma unroll
    for (int s = 1; s < kLanes; s <<= 1) {
      const T Ap = __shfl_up(A, s, kLanes), Bp = __shfl_up(B, s, kLanes);
      if (lane >= s) {
        B = A * Bp + B;
        A = A * Ap;
      }
    }
    if (active) {
      if (sel)
        w1[S0] = B;
      else
        w0[S0] = B;
    }
    if (j >= jo0) store(j, w0[S0], w1[S0]);
    // refill: row j-R (its last use was this step) with row j-R+UL; f of row j with row j+4
    load(j - R + UL, w0[P % UL], w1[P % UL]);
    const size_t row = (size_t)min(j + 4, n - 2) * n;
    g0[P % 4] = f[row + a0];
    g1[P % 4] = f[row + a1];
  };
  for (int j = js; j < jo1; j += UL)
    static_for<UL>([&](auto pc) { step(j + decltype(pc)::value, pc); });
}

}  // namespace

template <typename T>
hipError_t launch_gs2d(const LevelOp &op, double omega, int colour, const T *f, const T *uin, T *uout,
                       int n, const int *done, hipStream_t s, int slots) {
  if (colour != 1 && colour != 2) return hipErrorInvalidValue;
  const int R = op.cross3 ? 3 : (op.cross && op.a[1] != 0.0 ? 2 : 0);
  if (R == 0 || op.b[3] != 1.0) return hipErrorInvalidValue;  // cross stencils of radius 2 or 3
  GsCoef<T> k;
  k.c[0] = T(0);
  for (int d = 1; d <= 3; ++d) k.c[d] = (T)op.a[3 + d];
  k.om_d = (T)(omega / op.diag);
  const int out = R == 3 ? 2 * out_lanes<3>() : 2 * out_lanes<2>();
  const int strips = (n - 1 + out - 1) / out;  // stored columns cover 1 .. n-1
  // bands: about ten waves per CU, none shorter than kMinBandRows (each band recomputes
  // kHaloRows rows below it)
  int cus = 256, dev = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
    cus = 256;
  const int want = std::max(1, 10 * cus / strips);
  const int band_rows = std::max(kMinBandRows, (n - 2 + want - 1) / want);
  const int bands = (n - 2 + band_rows - 1) / band_rows;
  const int blocks = (strips * bands + kWaves - 1) / kWaves;
  const dim3 grid(blocks, 1, slots), block(kLanes * kWaves);
  if (R == 3)
    hipLaunchKernelGGL((k_gs2d<T, 3>), grid, block, 0, s, f, uin, uout, n, colour, strips, bands, band_rows, k,
                       done);
  else
    hipLaunchKernelGGL((k_gs2d<T, 2>), grid, block, 0, s, f, uin, uout, n, colour, strips, bands, band_rows, k,
                       done);
  return hipGetLastError();
}

template hipError_t launch_gs2d<double>(const LevelOp &, double, int, const double *, const double *, double *,
                                        int, const int *, hipStream_t, int);
template hipError_t launch_gs2d<float>(const LevelOp &, double, int, const float *, const float *, float *, int,
                                       const int *, hipStream_t, int);

}  // namespace mgk
