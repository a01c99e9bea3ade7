// fused2d.hip -- temporally blocked 2D cycle kernels for gfx950.
//
// Every wave (64 lanes) owns one strip of grid columns and marches down a chunk of rows
// on its own: no block-wide barrier inside the row loop, so the u/f loads of the next
// rows stay in flight while the current rows are computed.  y neighbours live in
// per-lane register windows; x neighbours are exchanged through a wave-private LDS row
// (one write and two paired reads per stencil stage; waves of a block never wait for
// each other).  Each stencil stage shrinks the valid lanes by the stencil radius R, so
// a strip carries a halo of H columns on each side that are computed but not written.
//
// Pre kernel (k_pre2d):  NU omega-Jacobi sweeps, then the defect f - L u, then full
//   weighting, in one pass: reads u and f once, writes the smoothed u and the coarse
//   right-hand side.  Stage s of the pipeline lags stage s-1 by R rows.  With red-black
//   smoothing the sweeps are partial steps, red and black in turn.
// Post kernel (k_post2d): interpolation of the coarse correction (cubic or linear),
//   correction, then NU2 sweeps, in one pass: reads u, f and the coarse v once, writes u.
//
// Dirichlet closure: all inputs are extended oddly across the boundary (u(-i) = -u(i),
// boundary values read as zero), and every stage is evaluated with the same formula on
// the extended rows and columns, which reproduces the odd extension of its output.
// Blocks whose rows all lie inside the grid take a path without row reflection.
//
// Loads are issued unconditionally from a valid address and the reflection sign / zero
// is applied when the value is consumed: a branch around a load would make the compiler
// wait for it at once and serialise the row loop on memory latency.
#include <cmath>
#include <type_traits>
#include <utility>

#include "mg_internal.h"

namespace mgk {
namespace {

constexpr int kWave = 64;
constexpr int kWavesPerBlock = kBlock / kWave;
constexpr int kPad = 4;              // LDS row padding on each side (>= R + 1)
constexpr int kRowLen = kWave + 2 * kPad;
constexpr int kPF = 4;               // rows of u and f loaded ahead

__device__ __forceinline__ bool stopped(const int *done) { return done != nullptr && *done != 0; }

__device__ __forceinline__ int round_up(int a, int m) { return (a + m - 1) / m * m; }

// Slot of an offset in a ring of length L (compile time).
template <int L>
__host__ __device__ constexpr int ring(int a) {
  return ((a % L) + L) % L;
}

// f(integral_constant<int, i>) for i = 0 .. N-1, unrolled.
template <int N, typename F, int... I>
__device__ __forceinline__ void static_for_impl(F &&f, std::integer_sequence<int, I...>) {
  (f(std::integral_constant<int, I>{}), ...);
}
template <int N, typename F>
__device__ __forceinline__ void static_for(F &&f) {
  static_for_impl<N>(f, std::make_integer_sequence<int, N>{});
}

__device__ __forceinline__ int floordiv2(int a) { return a >= 0 ? a / 2 : -((1 - a) / 2); }

// Odd extension: fold index i into 0..n-1 (at most two reflections), sign flips per
// reflection; returns -1 when i lies further out.
__device__ __forceinline__ int fold(int i, int n, int &sign) {
  if (i < 0) { i = -i; sign = -sign; }
  if (i > n - 1) { i = 2 * (n - 1) - i; sign = -sign; }
  if (i < 0) { i = -i; sign = -sign; }
  return (i >= 0 && i <= n - 1) ? i : -1;
}

__device__ __forceinline__ void wave_sync() { __builtin_amdgcn_wave_barrier(); }

// L u at the centre of window w (rows c-R..c+R of this lane's column); x neighbours
// through the wave's LDS rows (ra, rb point at this lane's slot).  Cross operator
// (R = 2, or R = 3 with XC): difference form with weights w1, w2 (, w3).  Separable
// operator (R = 3): L = a_x b_y + b_x a_y with the a factors in difference form.
template <typename T, int R, bool XC = false>
__device__ __forceinline__ T apply_op(const T (&w)[2 * R + 1], const KOp<T> &op, T *ra, T *rb) {
  const T c = w[R];
  if constexpr (XC) {
    ra[0] = c;
    wave_sync();
    const T xm1 = ra[-1], xp1 = ra[1], xm2 = ra[-2], xp2 = ra[2], xm3 = ra[-3], xp3 = ra[3];
    wave_sync();
    return op.w1 * (((c - xm1) + (c - xp1)) + ((c - w[R - 1]) + (c - w[R + 1]))) +
           op.w2 * (((c - xm2) + (c - xp2)) + ((c - w[R - 2]) + (c - w[R + 2]))) +
           op.w3 * (((c - xm3) + (c - xp3)) + ((c - w[R - 3]) + (c - w[R + 3])));
  } else if constexpr (R == 2) {
    ra[0] = c;
    wave_sync();
    const T xm1 = ra[-1], xp1 = ra[1], xm2 = ra[-2], xp2 = ra[2];
    wave_sync();
    return op.w1 * (((c - xm1) + (c - xp1)) + ((c - w[R - 1]) + (c - w[R + 1]))) +
           op.w2 * (((c - xm2) + (c - xp2)) + ((c - w[R - 2]) + (c - w[R + 2])));
  } else {
    T A = T(0), B = T(0);
#pragma unroll
    for (int k = 0; k < 2 * R + 1; ++k) {
      if (k != R) A += op.a[k] * (w[k] - c);
      B += op.b[k] * w[k];
    }
    ra[0] = A;
    rb[0] = B;
    wave_sync();
    T lu = T(0);
#pragma unroll
    for (int i = 0; i < 2 * R + 1; ++i) {
      if (i != R) lu += op.a[i] * (rb[i - R] - B);
      lu += op.b[i] * ra[i - R];
    }
    wave_sync();
    return lu;
  }
}

template <typename T, int N>
__device__ __forceinline__ void push(T (&w)[N], T v) {
#pragma unroll
  for (int k = 0; k < N - 1; ++k) w[k] = w[k + 1];
  w[N - 1] = v;
}

__device__ double block_sum(double v) {
  __shared__ double ws[kWavesPerBlock];
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  if (lane == 0) ws[wid] = v;
  __syncthreads();
  double tot = 0.0;
  if (threadIdx.x == 0)
    for (int i = 0; i < kWavesPerBlock; ++i) tot += ws[i];
  return tot;
}

// Row access for one lane's column: raw loads from a valid address and the factor that
// turns them into the odd extension (sign, or zero on and beyond the boundary).
template <typename T>
struct Column {
  int n;
  int xs;       // address column (valid even when the lane lies outside)
  bool xin;     // the lane's column is an interior column
  T xsign;      // reflection sign of the column
  T xmul;       // xin ? xsign : 0
  __device__ void init(int x, int n_) {
    n = n_;
    int sx = 1;
    const int xf = fold(x, n, sx);
    xin = xf > 0 && xf < n - 1;
    xs = xin ? xf : 1;
    xsign = T(sx);
    xmul = xin ? xsign : T(0);
  }
  template <bool FAST>
  __device__ __forceinline__ size_t addr(int y) const {
    if (FAST) return (size_t)y * n + xs;
    int s = 1;
    int ys = fold(y, n, s);
    ys = (ys > 0 && ys < n - 1) ? ys : 1;
    return (size_t)ys * n + xs;
  }
  template <bool FAST>
  __device__ __forceinline__ T fix(T v, int y) const {
    if (FAST) return v * xmul;
    int s = 1;
    const int ys = fold(y, n, s);
    const bool ok = xin && ys > 0 && ys < n - 1;
    return ok ? v * (xsign * T(s)) : T(0);
  }
};

// Pre-kernel modes.
constexpr int kWriteU = 1;    // write the smoothed iterate
constexpr int kRestrict = 2;  // full-weight the defect onto the coarse grid
constexpr int kWriteR = 4;    // write the defect itself

template <typename T>
struct PreArgs {
  const T *f;
  const T *u;  // nullptr: zero initial guess
  T *uout;
  T *rout;
  T *fc;
  int n;
  int chunk;  // coarse rows (kRestrict) or fine rows per block
  KOp<T> op;
  double *partials;  // sum of squares of the first defect (f - L u), per block
  const int *done;
};

// Stage s (1 <= s <= K) of the pipeline works on row t - (s-1)(R+1) at row step t: one
// row more than the stencil radius behind stage s-1, so every stage reads only values
// that earlier row steps produced.  All stages of a row step are then independent: their
// x neighbours go through LDS in one batched exchange and their arithmetic overlaps.
// The full weighting of the defect lags one more row for the same reason.
// RBS: the stages are red-black partial steps (stage_om), else omega-Jacobi sweeps.
// XC: the R = 3 operator is a cross (sixth order), exchanged and applied as one.
template <typename T, int R, int NU, int MODE, bool HAS_U, bool RBS = false, bool XC = false>
__global__ __launch_bounds__(kBlock) void k_pre2d(PreArgs<T> a) {
  constexpr bool RESTRICT = (MODE & kRestrict) != 0;
  constexpr bool WRITE_R = (MODE & kWriteR) != 0;
  constexpr bool WRITE_U = (MODE & kWriteU) != 0;
  constexpr bool RES = RESTRICT || WRITE_R;
  constexpr int K = NU + (RES ? 1 : 0);            // stencil stages (sweeps, then the defect)
  constexpr int H = K * R + (RESTRICT ? 1 : 0);    // halo columns of a strip
  constexpr int S = kWave - 2 * H;
  constexpr int W = 2 * R + 1;
  constexpr int LAG = R + 1;                       // rows between consecutive stages
  constexpr int FQ = (K - 1) * LAG + 1;            // f rows kept (stage s reads row t-(s-1)LAG)
  constexpr bool CROSS = R == 2 || XC;
  constexpr int XV = CROSS ? 1 : 2;                // values one stage exchanges across lanes
  constexpr int NX = K * XV + (RESTRICT ? 1 : 0);  // LDS rows per wave
  constexpr int LR = FQ <= 8 ? 8 : 16;            // ring length = row steps per loop turn
  static_assert(K >= 1, "the pre kernel runs at least one stencil stage");
  static_assert(2 * R + 1 < LR && LR % kPF == 0, "rings hold a stencil window; queue divides");
  __shared__ T lrow[kWavesPerBlock][NX][kRowLen];
  a.done = slot_done(a.done);
  if (stopped(a.done)) return;
  {
    const size_t ps = (size_t)a.n * a.n, ncs = (size_t)((a.n - 1) / 2 + 1);
    a.f = slot_ptr(a.f, ps);
    a.u = slot_ptr(a.u, ps);
    a.uout = slot_ptr(a.uout, ps);
    a.rout = slot_ptr(a.rout, ps);
    a.fc = slot_ptr(a.fc, ncs * ncs);
    a.partials = slot_ptr(a.partials, (size_t)gridDim.x * gridDim.y);
  }
  const int n = a.n;
  const int lane = threadIdx.x & (kWave - 1);
  const int wv = threadIdx.x >> 6;
  const Block2 blk = block2();
  const int strip = blk.x * kWavesPerBlock + wv;
  const int x = strip * S - H + lane;
  const bool active = strip * S < n;  // wave-uniform
  const bool useful = lane >= H && lane < H + S && x <= n - 1;
  T *const lds0 = &lrow[wv][0][kPad + lane];  // LDS row k of this wave at lds0 + k * kRowLen
  Column<T> col;
  col.init(x, n);

  // Rows: the last stage emits rows ya..yb; rows [own_a, own_b) belong to this block for
  // writes and for the defect norm.
  int ya, yb, own_a, own_b, Jlo = 0, Jhi = 0;
  const int nc = (n - 1) / 2 + 1;
  if (RESTRICT) {
    const int J0 = blk.y * a.chunk, J1 = min(J0 + a.chunk, nc);
    ya = 2 * J0 - 1;
    yb = 2 * J1 - 1;
    own_a = 2 * J0;
    own_b = min(2 * J1, n);
    Jlo = max(J0, 1);
    Jhi = min(J1, nc - 1);
    if (active && useful && (x & 1) == 0) {
      const int I = x >> 1;
      if (J0 == 0) a.fc[I] = T(0);
      if (J1 == nc) a.fc[(size_t)(nc - 1) * nc + I] = T(0);
    }
  } else {
    const int y0 = blk.y * a.chunk;
    ya = y0;
    yb = min(y0 + a.chunk, n) - 1;
    own_a = y0;
    own_b = yb + 1;
  }
  // stage 1 starts (K-1)R rows early so that stage K is exact from row ya on; the row
  // loop runs whole groups of kPF steps (extra steps emit nothing: their rows are past yb)
  const int ts = ya - (K - 1) * R;
  const int te = ts + round_up(yb + (K - 1) * LAG + (RESTRICT ? 1 : 0) - ts + 1, LR) - 1;
  const bool fast = ts - R > 0 && te + R + kPF < n - 1;
  const T *up = HAS_U ? a.u : a.f;

  double acc = 0.0;
  auto run = [&](auto fast_tag) {
    constexpr bool FAST = decltype(fast_tag)::value;
    // Every array carried from one row step to the next is a ring whose slot for row r is
    // (r - ts) mod its length, known at compile time once the loop is unrolled by LR row
    // steps; no value ever moves between registers, so loads in flight across the loop
    // back edge stay in flight.
    T w[K][LR];  // w[s][ring(r - ts)]: stage-s value of row r (s = 0: the input u)
    T fr[LR];    // f of row r
    T uq[kPF], fq[kPF];  // loads in flight: u of row t + R, f of row t, slot (t - ts) mod kPF
    T dr[4];     // defect of row r, slot (r - ts) mod 4
#pragma unroll
    for (int s = 0; s < K; ++s)
#pragma unroll
      for (int k = 0; k < LR; ++k) w[s][k] = T(0);
#pragma unroll
    for (int k = 0; k < LR; ++k) fr[k] = T(0);
#pragma unroll
    for (int k = 0; k < 4; ++k) dr[k] = T(0);
    if (HAS_U) {
#pragma unroll
      for (int k = 0; k < 2 * R; ++k)
        w[0][ring<LR>(k - R)] = col.template fix<FAST>(up[col.template addr<FAST>(ts - R + k)], ts - R + k);
    }
#pragma unroll
    for (int p = 0; p < kPF; ++p) {
      if (HAS_U) uq[p] = up[col.template addr<FAST>(ts + R + p)];
      fq[p] = a.f[col.template addr<FAST>(ts + p)];
    }
    const KOp<T> op = a.op;

    // Row step t = ts + (multiple of LR) + P.
    auto step = [&](const int t, auto pc) {
      constexpr int P = decltype(pc)::value;
      constexpr int Q = P % kPF;
      T unew = HAS_U ? col.template fix<FAST>(uq[Q], t + R) : T(0);
      T fnew = col.template fix<FAST>(fq[Q], t);
      // Materialise both values here (an empty asm that only pins them in registers) and
      // keep the refill below: the slot's raw value dies before its register is reloaded.
      asm volatile("" : "+v"(unew), "+v"(fnew));
      __builtin_amdgcn_sched_barrier(0);
      if (HAS_U) uq[Q] = up[col.template addr<FAST>(t + R + kPF)];
      fq[Q] = a.f[col.template addr<FAST>(t + kPF)];
      w[0][ring<LR>(P + R)] = unew;  // row t + R
      fr[ring<LR>(P)] = fnew;        // row t
      const int cK = t - (K - 1) * LAG;  // row of stage K

      // one exchange for every stage: the centre (cross) or the y sums (separable) of
      // stage s+1's input, stage s around row t - s LAG
      T ya_[K], yb_[K];
#pragma unroll
      for (int s = 0; s < K; ++s) {
        if constexpr (CROSS) {
          ya_[s] = w[s][ring<LR>(P - s * LAG)];
          lds0[s * kRowLen] = ya_[s];
        } else {
          const T c = w[s][ring<LR>(P - s * LAG)];
          T A = T(0), B = T(0);
#pragma unroll
          for (int k = 0; k < W; ++k) {
            const T v = w[s][ring<LR>(P - s * LAG + k - R)];
            if (k != R) A += op.a[k] * (v - c);
            B += op.b[k] * v;
          }
          ya_[s] = A;
          yb_[s] = B;
          lds0[(2 * s) * kRowLen] = A;
          lds0[(2 * s + 1) * kRowLen] = B;
        }
      }
      T ry = T(0);
      if (RESTRICT) {
        constexpr int D = ring<4>(P - (K - 1) * LAG);  // slot of row cK
        ry = T(0.25) * dr[(D + 1) % 4] + T(0.5) * dr[(D + 2) % 4] + T(0.25) * dr[(D + 3) % 4];
        lds0[(NX - 1) * kRowLen] = ry;
      }
      wave_sync();
      T lu[K];
#pragma unroll
      for (int s = 0; s < K; ++s) {
        if constexpr (R == 2) {
          const T *row = lds0 + s * kRowLen;
          const T c = ya_[s];
          const T ym1 = w[s][ring<LR>(P - s * LAG - 1)], yp1 = w[s][ring<LR>(P - s * LAG + 1)];
          const T ym2 = w[s][ring<LR>(P - s * LAG - 2)], yp2 = w[s][ring<LR>(P - s * LAG + 2)];
          const T xm1 = row[-1], xp1 = row[1], xm2 = row[-2], xp2 = row[2];
          lu[s] = op.w1 * (((c - xm1) + (c - xp1)) + ((c - ym1) + (c - yp1))) +
                  op.w2 * (((c - xm2) + (c - xp2)) + ((c - ym2) + (c - yp2)));
        } else if constexpr (XC) {
          const T *row = lds0 + s * kRowLen;
          const T c = ya_[s];
          T v = T(0);
#pragma unroll
          for (int k = 1; k <= 3; ++k) {
            const T ym = w[s][ring<LR>(P - s * LAG - k)], yp = w[s][ring<LR>(P - s * LAG + k)];
            const T wk = k == 1 ? op.w1 : k == 2 ? op.w2 : op.w3;
            v += wk * (((c - row[-k]) + (c - row[k])) + ((c - ym) + (c - yp)));
          }
          lu[s] = v;
        } else {
          const T *ra = lds0 + (2 * s) * kRowLen;
          const T *rb = lds0 + (2 * s + 1) * kRowLen;
          const T B = yb_[s];
          T v = T(0);
#pragma unroll
          for (int i = 0; i < W; ++i) {
            if (i != R) v += op.a[i] * (rb[i - R] - B);
            v += op.b[i] * ra[i - R];
          }
          lu[s] = v;
        }
      }
      T left = T(0), right = T(0);
      if (RESTRICT) {
        left = lds0[(NX - 1) * kRowLen - 1];
        right = lds0[(NX - 1) * kRowLen + 1];
      }
      wave_sync();

      // sweeps: stage s at row t - (s-1)LAG
      T nv[NU > 0 ? NU : 1];
#pragma unroll
      for (int s = 1; s <= NU; ++s) {
        const int row = t - (s - 1) * LAG;
        const T r = fr[ring<LR>(P - (s - 1) * LAG)] - lu[s - 1];
        if (s == 1 && a.partials != nullptr && useful && col.xin && row >= own_a && row < own_b &&
            row > 0 && row < n - 1)
          acc += (double)r * (double)r;
        nv[s - 1] = w[s - 1][ring<LR>(P - (s - 1) * LAG)] + (RBS ? stage_om(op, s, x + row) : op.om_d) * r;
      }
      // defect of the smoothed iterate at row cK
      T rd = T(0);
      if (RES) {
        rd = fr[ring<LR>(P - (K - 1) * LAG)] - lu[K - 1];
        if (NU == 0 && a.partials != nullptr && useful && col.xin && cK >= own_a && cK < own_b &&
            cK > 0 && cK < n - 1)
          acc += (double)rd * (double)rd;
      }
      if (useful && cK >= own_a && cK < own_b && cK >= 0 && cK <= n - 1) {
        const bool inside = col.xin && cK > 0 && cK < n - 1;
        const size_t id = (size_t)cK * n + x;
        T uval;
        if constexpr (RES)
          uval = w[NU][ring<LR>(P - NU * LAG)];
        else
          uval = nv[NU > 0 ? NU - 1 : 0];
        if (WRITE_U) a.uout[id] = inside ? uval : T(0);
        if (WRITE_R) a.rout[id] = inside ? rd : T(0);
      }
      // full weighting of the defect rows cK-3 .. cK-1 onto coarse row J
      if (RESTRICT && (cK & 1) == 0) {
        const int J = (cK >> 1) - 1;
        if (J >= Jlo && J < Jhi && useful && (x & 1) == 0) {
          const int I = x >> 1;
          const bool inside = I > 0 && I < nc - 1;
          a.fc[(size_t)J * nc + I] = inside ? T(0.25) * left + T(0.5) * ry + T(0.25) * right : T(0);
        }
      }
#pragma unroll
      for (int s = 1; s < K; ++s) w[s][ring<LR>(P - (s - 1) * LAG)] = nv[s - 1];
      if (RES) dr[ring<4>(P - (K - 1) * LAG)] = rd;
    };
    for (int t = ts; t <= te; t += LR)
      static_for<LR>([&](auto pc) { step(t + decltype(pc)::value, pc); });
  };
  if (active) {
    if (fast)
      run(std::true_type{});
    else
      run(std::false_type{});
  }
  if (a.partials != nullptr) {
    const double tot = block_sum(acc);
    if (threadIdx.x == 0) a.partials[blockIdx.y * gridDim.x + blockIdx.x] = tot;
  }
}

template <typename T>
struct PostArgs {
  const T *v;    // coarse correction, side nc
  const T *uin;  // iterate before the correction
  const T *f;
  T *uout;
  int n;
  int chunk;  // fine rows per block
  KOp<T> op;
  const int *done;
};

template <typename T, int R, int NU2, int P, bool RBS = false, bool XC = false>
__global__ __launch_bounds__(kBlock) void k_post2d(PostArgs<T> a) {
  constexpr int H = NU2 * R;
  constexpr int S = kWave - 2 * H;
  constexpr int W = 2 * R + 1;
  constexpr int FQ = NU2 > 0 ? (NU2 - 1) * R + 1 : 1;
  __shared__ T lrow[kWavesPerBlock][2][kRowLen];
  a.done = slot_done(a.done);
  if (stopped(a.done)) return;
  const int n = a.n, nc = (n - 1) / 2 + 1;
  a.v = slot_ptr(a.v, (size_t)nc * nc);
  a.uin = slot_ptr(a.uin, (size_t)n * n);
  a.f = slot_ptr(a.f, (size_t)n * n);
  a.uout = slot_ptr(a.uout, (size_t)n * n);
  const int lane = threadIdx.x & (kWave - 1);
  const int wv = threadIdx.x >> 6;
  const Block2 blk = block2();
  const int strip = blk.x * kWavesPerBlock + wv;
  const int x0 = strip * S - H;
  const int x = x0 + lane;
  if (strip * S >= n) return;  // whole wave idle; no block barrier follows
  const bool useful = lane >= H && lane < H + S && x <= n - 1;
  T *ra = &lrow[wv][0][kPad + lane];
  T *rb = &lrow[wv][1][kPad + lane];
  Column<T> col;
  col.init(x, n);
  // coarse column loaded by this lane (lanes 0..35 cover the strip and its stencil)
  const int Ib = floordiv2(x0) - 1;
  Column<T> ccol;
  ccol.init(Ib + lane, nc);
  // LDS slots of this fine column's coarse neighbours (relative to the lane's own slot)
  const int src0 = floordiv2(x) - Ib - lane;
  T *crow = &lrow[wv][1][kPad + lane];

  const int y0 = blk.y * a.chunk;
  const int y1 = min(y0 + a.chunk, n);
  const int ts = y0 - NU2 * R, te = y1 - 1 + NU2 * R;
  const int jb0 = floordiv2(ts) - 1;
  const bool fast = ts - R > 0 && te + kPF < n - 1 && jb0 - 1 > 0 && floordiv2(te) + 4 < nc - 1;
  const T *fp = NU2 > 0 ? a.f : a.uin;  // f is not read without post-smoothing

  auto run = [&](auto fast_tag) {
    constexpr bool FAST = decltype(fast_tag)::value;
    // x-interpolation of a coarse row at this lane's fine column
    auto interp = [&](T cv) -> T {
      crow[0] = cv;
      wave_sync();
      const T c0 = crow[src0], c1 = crow[src0 + 1];
      T out;
      if (P == 3) {
        const T cm = crow[src0 - 1], c2 = crow[src0 + 2];
        out = (x & 1) == 0 ? c0 : (T(9) * (c0 + c1) - (cm + c2)) * T(0.0625);
      } else {
        out = (x & 1) == 0 ? c0 : T(0.5) * (c0 + c1);
      }
      wave_sync();
      return out;
    };
    T pw[4];
    int jb = jb0;
    // coarse rows jb..jb+3 now, and the next one ahead
#pragma unroll
    for (int k = 0; k < 4; ++k) pw[k] = interp(ccol.template fix<FAST>(a.v[ccol.template addr<FAST>(jb + k)], jb + k));
    T cnext = a.v[ccol.template addr<FAST>(jb + 4)];
    T w[NU2 + 1][W];
#pragma unroll
    for (int s = 0; s <= NU2; ++s)
#pragma unroll
      for (int k = 0; k < W; ++k) w[s][k] = T(0);
    T fw[FQ];
#pragma unroll
    for (int k = 0; k < FQ; ++k) fw[k] = T(0);
    T uq[kPF], fq[kPF];
#pragma unroll
    for (int p = 0; p < kPF; ++p) {
      uq[p] = a.uin[col.template addr<FAST>(ts + p)];
      if (NU2 > 0) fq[p] = fp[col.template addr<FAST>(ts - R + p)];
    }
    const KOp<T> op = a.op;

    for (int t = ts; t <= te; ++t) {
      const int Jc = floordiv2(t);
      if (jb < Jc - 1) {  // the stencil moved down one coarse row (every other fine row)
        const T nv = interp(ccol.template fix<FAST>(cnext, jb + 4));
        cnext = a.v[ccol.template addr<FAST>(jb + 5)];
        push(pw, nv);
        ++jb;
      }
      const T pv = ((t & 1) == 0) ? pw[1]
                   : (P == 3 ? (T(9) * (pw[1] + pw[2]) - (pw[0] + pw[3])) * T(0.0625)
                             : T(0.5) * (pw[1] + pw[2]));
      const T unew = col.template fix<FAST>(uq[0], t);
      push(uq, a.uin[col.template addr<FAST>(t + kPF)]);
      const T ut = unew + pv;  // corrected iterate at row t
      T out = ut;
      int c = t;
      if (NU2 > 0) {
        const T fnew = col.template fix<FAST>(fq[0], t - R);
        push(fq, fp[col.template addr<FAST>(t - R + kPF)]);
        push(fw, fnew);
        push(w[0], ut);
#pragma unroll
        for (int s = 1; s <= NU2; ++s) {
          // stage s: sweep at row t - s R, the centre of w[s-1]
          const T fv = fw[FQ - 1 - (s - 1) * R];
          const T r = fv - apply_op<T, R, XC>(w[s - 1], op, ra, rb);
          push(w[s], w[s - 1][R] + (RBS ? stage_om(op, s, x + t - s * R) : op.om_d) * r);
        }
        out = w[NU2][W - 1];
        c = t - NU2 * R;
      }
      if (useful && c >= y0 && c < y1) {
        const bool inside = col.xin && c > 0 && c < n - 1;
        a.uout[(size_t)c * n + x] = inside ? out : T(0);
      }
    }
  };
  if (fast)
    run(std::true_type{});
  else
    run(std::false_type{});
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

// Shortest band of a fused launch: coarse rows (pre kernel with restriction) or fine rows.
constexpr int kMinCoarseRows = 4, kMinFineRows = 8;

// Rows of a pre launch and its bands.  grid.x (blocks across) is set by the caller; the
// band height fills at most one round of resident blocks of the kernel fn.
int pre_bands(const void *fn, int n, bool restrict_mode, dim3 *grid) {
  const int rows_total = restrict_mode ? (n - 1) / 2 + 1 : n;
  const int c = band_rows(rows_total, grid->x, resident_blocks(fn, kBlock, 0),
                          restrict_mode ? kMinCoarseRows : kMinFineRows);
  grid->y = cdiv(rows_total, c);
  return c;
}

template <typename T, int R, int NU, int MODE, bool RBS = false, bool XC = false>
hipError_t pre_dispatch(PreArgs<T> args, dim3 grid, bool restrict_mode, int *nparts, hipStream_t s) {
  const void *fn = args.u != nullptr ? (const void *)k_pre2d<T, R, NU, MODE, true, RBS, XC>
                                     : (const void *)k_pre2d<T, R, NU, MODE, false, RBS, XC>;
  args.chunk = pre_bands(fn, args.n, restrict_mode, &grid);
  if (nparts) *nparts = grid.x * grid.y;
  if (args.u != nullptr)
    hipLaunchKernelGGL((k_pre2d<T, R, NU, MODE, true, RBS, XC>), grid, dim3(kBlock), 0, s, args);
  else
    hipLaunchKernelGGL((k_pre2d<T, R, NU, MODE, false, RBS, XC>), grid, dim3(kBlock), 0, s, args);
  return hipGetLastError();
}

template <typename T, int R, int MODE, bool XC>
hipError_t pre_nu(int nu, const PreArgs<T> &args, dim3 grid, int *nparts, hipStream_t s) {
  constexpr bool RM = (MODE & kRestrict) != 0;
  constexpr bool RES = (MODE & (kRestrict | kWriteR)) != 0;
  switch (nu) {
    case 0:
      if constexpr (RES) return pre_dispatch<T, R, 0, MODE, false, XC>(args, grid, RM, nparts, s);
      return hipErrorInvalidValue;  // nothing to compute
    case 1: return pre_dispatch<T, R, 1, MODE, false, XC>(args, grid, RM, nparts, s);
    case 2: return pre_dispatch<T, R, 2, MODE, false, XC>(args, grid, RM, nparts, s);
    case 3: return pre_dispatch<T, R, 3, MODE, false, XC>(args, grid, RM, nparts, s);
    default: return hipErrorInvalidValue;
  }
}

// The pre passes of one operator shape: R = 2 cross, R = 3 separable or (XC) cross.
template <typename T, int R, bool XC>
hipError_t pre_shape(int nu, int mode, bool rb, PreArgs<T> &args, dim3 grid, int *nparts, hipStream_t s) {
  constexpr int WR = kWriteU | kRestrict;
  if (rb) {
    // red-black passes: two stages (one sweep), or none before the defect
    args.op.colour = kColourRB;
    if (mode == WR && nu == 0) return pre_dispatch<T, R, 0, WR, false, XC>(args, grid, true, nparts, s);
    if (mode == WR && nu == 2) return pre_dispatch<T, R, 2, WR, true, XC>(args, grid, true, nparts, s);
    if (mode == kWriteU && nu == 2) return pre_dispatch<T, R, 2, kWriteU, true, XC>(args, grid, false, nparts, s);
    return hipErrorInvalidValue;
  }
  if (mode == WR) return pre_nu<T, R, WR, XC>(nu, args, grid, nparts, s);
  if (mode == kWriteU && nu == 1) return pre_dispatch<T, R, 1, kWriteU, false, XC>(args, grid, false, nparts, s);
  if (mode == kWriteR && nu == 0) return pre_dispatch<T, R, 0, kWriteR, false, XC>(args, grid, false, nparts, s);
  if (mode == kRestrict && nu == 0) return pre_dispatch<T, R, 0, kRestrict, false, XC>(args, grid, true, nparts, s);
  return hipErrorInvalidValue;
}

template <typename T, int R, int NU2, bool RBS = false, bool XC = false>
hipError_t post_dispatch(int prolong, PostArgs<T> args, dim3 grid, hipStream_t s) {
  const void *fn = prolong == 3 ? (const void *)k_post2d<T, R, NU2, 3, RBS, XC>
                                : (const void *)k_post2d<T, R, NU2, 1, RBS, XC>;
  args.chunk = band_rows(args.n, grid.x, resident_blocks(fn, kBlock, 0), kMinFineRows);
  grid.y = cdiv(args.n, args.chunk);
  if (prolong == 3)
    hipLaunchKernelGGL((k_post2d<T, R, NU2, 3, RBS, XC>), grid, dim3(kBlock), 0, s, args);
  else
    hipLaunchKernelGGL((k_post2d<T, R, NU2, 1, RBS, XC>), grid, dim3(kBlock), 0, s, args);
  return hipGetLastError();
}

template <typename T, int R, bool XC>
hipError_t post_shape(int nu2, int prolong, bool rb, PostArgs<T> &args, dim3 grid, hipStream_t s) {
  if (rb) {
    args.op.colour = kColourRB;
    if (nu2 == 0) return post_dispatch<T, R, 0, false, XC>(prolong, args, grid, s);
    if (nu2 == 2) return post_dispatch<T, R, 2, true, XC>(prolong, args, grid, s);
    return hipErrorInvalidValue;
  }
  switch (nu2) {
    case 0: return post_dispatch<T, R, 0, false, XC>(prolong, args, grid, s);
    case 1: return post_dispatch<T, R, 1, false, XC>(prolong, args, grid, s);
    case 2: return post_dispatch<T, R, 2, false, XC>(prolong, args, grid, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace

int pre2d_partials(int n) {
  // the largest grid any pre launch uses at side n (smallest strip width S = 64 - 2H)
  int best = pre2d_tile_partials(n);
  for (int R = 2; R <= 3; ++R)
    for (int nu = 0; nu <= 3; ++nu)
      for (int restrict_mode = 0; restrict_mode <= 1; ++restrict_mode) {
        const int H = (nu + 1) * R + restrict_mode;
        const int S = kWave - 2 * H;
        if (S <= 0) continue;
        const int bx = cdiv(cdiv(n, S), kWavesPerBlock);
        const int rows_total = restrict_mode ? (n - 1) / 2 + 1 : n;
        const int nb = bx * cdiv(rows_total, restrict_mode ? kMinCoarseRows : kMinFineRows);
        best = nb > best ? nb : best;
      }
  return best;
}

template <typename T>
hipError_t launch_pre2d(const LevelOp &op, double omega, int nu, int mode, const T *f, const T *u,
                        T *uout, T *rout, T *fc, int n, double *partials, int *nparts,
                        const int *done, hipStream_t s, int slots, bool rb) {
  if (n <= tile2d_max_side())
    return launch_pre2d_tile<T>(op, omega, nu, mode, f, u, uout, rout, fc, n, partials, nparts, done,
                                s, slots, rb);
  const int R = op.cross ? 2 : 3;
  const bool restrict_mode = (mode & kRestrict) != 0;
  const bool res = restrict_mode || (mode & kWriteR) != 0;
  const int K = nu + (res ? 1 : 0);
  const int H = K * R + (restrict_mode ? 1 : 0);
  const int S = kWave - 2 * H;
  if (S <= 0 || nu < 0 || nu > 3) return hipErrorInvalidValue;
  PreArgs<T> args{f, u, uout, rout, fc, n, 0, to_kop<T>(op, omega), partials, done};
  const dim3 grid(cdiv(cdiv(n, S), kWavesPerBlock), 1, slots);
  if (R == 2) return pre_shape<T, 2, false>(nu, mode, rb, args, grid, nparts, s);
  if (op.cross3) return pre_shape<T, 3, true>(nu, mode, rb, args, grid, nparts, s);
  return pre_shape<T, 3, false>(nu, mode, rb, args, grid, nparts, s);
}

template <typename T>
hipError_t launch_post2d(const LevelOp &op, double omega, int nu2, int prolong, const T *v,
                         const T *uin, const T *f, T *uout, int n, const int *done,
                         hipStream_t s, int slots, bool rb) {
  if (nu2 < 0 || nu2 > 2) return hipErrorInvalidValue;
  if (n <= tile2d_max_side())
    return launch_post2d_tile<T>(op, omega, nu2, prolong, v, uin, f, uout, n, done, s, slots, rb);
  const int R = op.cross ? 2 : 3;
  const int H = nu2 * R;
  const int S = kWave - 2 * H;
  PostArgs<T> args{v, uin, f, uout, n, 0, to_kop<T>(op, omega), done};
  const dim3 grid(cdiv(cdiv(n, S), kWavesPerBlock), 1, slots);
  if (R == 2) return post_shape<T, 2, false>(nu2, prolong, rb, args, grid, s);
  if (op.cross3) return post_shape<T, 3, true>(nu2, prolong, rb, args, grid, s);
  return post_shape<T, 3, false>(nu2, prolong, rb, args, grid, s);
}

template hipError_t launch_pre2d<double>(const LevelOp &, double, int, int, const double *,
                                         const double *, double *, double *, double *, int,
                                         double *, int *, const int *, hipStream_t, int, bool);
template hipError_t launch_pre2d<float>(const LevelOp &, double, int, int, const float *,
                                        const float *, float *, float *, float *, int, double *,
                                        int *, const int *, hipStream_t, int, bool);
template hipError_t launch_post2d<double>(const LevelOp &, double, int, int, const double *,
                                          const double *, const double *, double *, int,
                                          const int *, hipStream_t, int, bool);
template hipError_t launch_post2d<float>(const LevelOp &, double, int, int, const float *,
                                         const float *, const float *, float *, int, const int *,
                                         hipStream_t, int, bool);

}  // namespace mgk
