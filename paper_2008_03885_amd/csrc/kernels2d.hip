// kernels2d.hip -- 2D hot-path kernels for gfx950 and the dimension-independent ones
// (coarsest solve, residual checks, refinement correction, fills).
//
// Streaming pattern of the 2D stencil kernels: a block of 256 threads owns 256
// consecutive grid columns and marches down a strip of rows.  Each thread keeps the
// 2R+1 values of its own column around the current row in registers (the y
// neighbours) and publishes one value per row to a double-buffered LDS row, from which
// the x neighbours are read: one barrier per row, every u value read from HBM once
// per strip, and the x halo (R columns on each side) costs 2R/256 extra loads.  Grid
// functions are extended across the Dirichlet boundary by odd reflection.
#include <algorithm>
#include <cmath>
#include <map>
#include <mutex>
#include <tuple>

#include "mg_internal.h"

namespace mgk {
namespace {

__device__ __forceinline__ bool stopped(const int *done) { return done != nullptr && *done != 0; }

// Reflect index i into 0..n-1 (odd extension); flips sign for each reflection.
__device__ __forceinline__ int fold(int i, int n, int &sign) {
  if (i < 0) { i = -i; sign = -sign; }
  if (i > n - 1) { i = 2 * (n - 1) - i; sign = -sign; }
  return i;
}

// Sum over a 1D block of kBlock threads; result valid in thread 0.  Fixed order.
__device__ double block_sum(double v) {
  __shared__ double ws[kBlock / 64];
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  if (lane == 0) ws[wid] = v;
  __syncthreads();
  double tot = 0.0;
  if (threadIdx.x == 0)
    for (int i = 0; i < kBlock / 64; ++i) tot += ws[i];
  return tot;
}

// ---------------------------------------------------------------- 2D sweep ----
// MODE kSweep: out = u + omega/diag (f - L u); kResidual: out = f - L u;
// kNormOnly: nothing written.  partials (optional) receives sum (f - L u)^2 per block.
// u == nullptr means u = 0.
template <typename T, typename TO, int MODE, bool CROSS>
__global__ __launch_bounds__(kBlock) void k_sweep2d(const T *__restrict__ f,
                                                    const T *__restrict__ u,
                                                    TO *__restrict__ out, int n, int rows,
                                                    KOp<T> op, double *__restrict__ partials,
                                                    const int *__restrict__ done) {
  constexpr int R = CROSS ? 2 : 3;
  constexpr int W = 2 * R + 1;
  constexpr int NP = CROSS ? 1 : 2;
  __shared__ T pub[2][NP][kBlock];
  done = slot_done(done);
  if (stopped(done)) return;
  f = slot_ptr(f, (size_t)n * n);
  u = slot_ptr(u, (size_t)n * n);
  out = slot_ptr(out, (size_t)n * n);
  partials = slot_ptr(partials, (size_t)gridDim.x * gridDim.y);
  const int t = threadIdx.x;
  const Block2 blk = block2();
  const int x = blk.x * (kBlock - 2 * R) - R + t;
  const int y0 = blk.y * rows;
  const int y1 = min(y0 + rows, n);
  int sx = 1;
  const int xs = fold(x, n, sx);
  const bool col_ok = xs >= 0 && xs <= n - 1;
  const bool own = t >= R && t < kBlock - R && x <= n - 1;
  const bool zero_u = (u == nullptr);

  auto load_u = [&](int y) -> T {
    int s = sx;
    const int ys = fold(y, n, s);
    if (zero_u || !col_ok || ys < 0 || ys > n - 1) return T(0);
    const T v = u[(size_t)ys * n + xs];
    return s > 0 ? v : -v;
  };

  T w[W];
#pragma unroll
  for (int k = 0; k < W; ++k) w[k] = load_u(y0 - R + k);
  double acc = 0.0;
  int buf = 0;
  for (int y = y0; y < y1; ++y) {
    const T un = load_u(y + R + 1);
    const bool interior = own && x >= 1 && x <= n - 2 && y >= 1 && y <= n - 2;
    const T fv = interior ? f[(size_t)y * n + x] : T(0);
    if (CROSS) {
      pub[buf][0][t] = w[R];
    } else {
      // column sums A = a_y u (difference form: a annihilates constants) and B = b_y u
      T A = T(0), B = T(0);
#pragma unroll
      for (int k = 0; k < W; ++k) {
        if (k != R) A += op.a[k] * (w[k] - w[R]);
        B += op.b[k] * w[k];
      }
      pub[buf][0][t] = A;
      pub[buf][NP - 1][t] = B;
    }
    __syncthreads();
    if (own) {
      T r = T(0), val = T(0);
      if (interior) {
        T lu;
        if (CROSS) {
          const T u0 = w[R];
          const T *row = pub[buf][0];
          lu = op.w1 * (((u0 - row[t - 1]) + (u0 - row[t + 1])) + ((u0 - w[R - 1]) + (u0 - w[R + 1]))) +
               op.w2 * (((u0 - row[t - 2]) + (u0 - row[t + 2])) + ((u0 - w[R - 2]) + (u0 - w[R + 2])));
        } else {
          // L u = a_x (b_y u) + b_x (a_y u), a_x in difference form
          const T *Bs = pub[buf][NP - 1];
          const T *As = pub[buf][0];
          lu = T(0);
#pragma unroll
          for (int i = 0; i < W; ++i) {
            if (i != R) lu += op.a[i] * (Bs[t + i - R] - Bs[t]);
            lu += op.b[i] * As[t + i - R];
          }
        }
        r = fv - lu;
        val = w[R] + colour_om(op, x + y) * r;
        acc += (double)r * (double)r;
      }
      if (MODE == kSweep) out[(size_t)y * n + x] = (TO)val;
      if (MODE == kResidual) out[(size_t)y * n + x] = (TO)r;
    }
#pragma unroll
    for (int k = 0; k < W - 1; ++k) w[k] = w[k + 1];
    w[W - 1] = un;
    buf ^= 1;
  }
  if (partials != nullptr) {
    const double tot = block_sum(acc);
    if (t == 0) partials[blockIdx.y * gridDim.x + blockIdx.x] = tot;
  }
}

// --------------------------------------------------- 2D defect + full weighting ----
// fc = I_h^H (f - L u) on the coarse grid (nc = (n-1)/2+1).  Thread t owns fine column
// x = 2*CB*bx - (R+1) + t; even-offset threads emit coarse column I = CB*bx + (t-R-1)/2.
// The defect of a fine row is combined in y (weights 1/4,1/2,1/4) in registers, then
// in x through LDS.  u == nullptr means u = 0.
template <typename T, bool CROSS>
__global__ __launch_bounds__(kBlock) void k_resid_restrict2d(const T *__restrict__ f,
                                                             const T *__restrict__ u,
                                                             T *__restrict__ fc, int n, int crows,
                                                             KOp<T> op,
                                                             const int *__restrict__ done) {
  constexpr int R = CROSS ? 2 : 3;
  constexpr int W = 2 * R + 1;
  constexpr int NP = CROSS ? 1 : 2;
  constexpr int CB = (kBlock - 2 * R - 2) / 2;
  __shared__ T pub[2][NP][kBlock];
  __shared__ T rrow[kBlock];
  done = slot_done(done);
  if (stopped(done)) return;
  const int nc = (n - 1) / 2 + 1;
  f = slot_ptr(f, (size_t)n * n);
  u = slot_ptr(u, (size_t)n * n);
  fc = slot_ptr(fc, (size_t)nc * nc);
  const int t = threadIdx.x;
  const Block2 blk = block2();
  const int x = 2 * blk.x * CB - (R + 1) + t;
  int sx = 1;
  const int xs = fold(x, n, sx);
  const bool col_ok = xs >= 0 && xs <= n - 1;
  const bool own = t >= R && t < kBlock - R;
  const bool emits = t >= R + 1 && ((t - R - 1) & 1) == 0 && t <= 2 * CB + R - 1;
  const int I = blk.x * CB + (t - R - 1) / 2;
  const bool I_ok = emits && I <= nc - 1;
  const bool I_int = I_ok && I >= 1 && I <= nc - 2;
  const bool zero_u = (u == nullptr);
  const int J0 = blk.y * crows;
  const int J1 = min(J0 + crows, nc);
  if (I_ok) {
    if (J0 == 0) fc[I] = T(0);
    if (J1 == nc) fc[(size_t)(nc - 1) * nc + I] = T(0);
  }
  const int Jlo = max(J0, 1), Jhi = min(J1, nc - 1);
  if (Jlo >= Jhi) return;

  auto load_u = [&](int y) -> T {
    int s = sx;
    const int ys = fold(y, n, s);
    if (zero_u || !col_ok || ys < 0 || ys > n - 1) return T(0);
    const T v = u[(size_t)ys * n + xs];
    return s > 0 ? v : -v;
  };

  const int ys0 = 2 * Jlo - 1, ye = 2 * (Jhi - 1) + 1;
  T w[W];
#pragma unroll
  for (int k = 0; k < W; ++k) w[k] = load_u(ys0 - R + k);
  T r0 = T(0), r1 = T(0), r2 = T(0);
  int buf = 0;
  for (int y = ys0; y <= ye; ++y) {
    const T un = load_u(y + R + 1);
    const bool interior = own && x >= 1 && x <= n - 2;
    const T fv = interior ? f[(size_t)y * n + x] : T(0);
    if (CROSS) {
      pub[buf][0][t] = w[R];
    } else {
      // column sums A = a_y u (difference form: a annihilates constants) and B = b_y u
      T A = T(0), B = T(0);
#pragma unroll
      for (int k = 0; k < W; ++k) {
        if (k != R) A += op.a[k] * (w[k] - w[R]);
        B += op.b[k] * w[k];
      }
      pub[buf][0][t] = A;
      pub[buf][NP - 1][t] = B;
    }
    __syncthreads();
    T r = T(0);
    if (interior) {
      T lu;
      if (CROSS) {
        const T u0 = w[R];
        const T *row = pub[buf][0];
        lu = op.w1 * (((u0 - row[t - 1]) + (u0 - row[t + 1])) + ((u0 - w[R - 1]) + (u0 - w[R + 1]))) +
             op.w2 * (((u0 - row[t - 2]) + (u0 - row[t + 2])) + ((u0 - w[R - 2]) + (u0 - w[R + 2])));
      } else {
        const T *Bs = pub[buf][NP - 1];
        const T *As = pub[buf][0];
        lu = T(0);
#pragma unroll
        for (int i = 0; i < W; ++i) {
          if (i != R) lu += op.a[i] * (Bs[t + i - R] - Bs[t]);
          lu += op.b[i] * As[t + i - R];
        }
      }
      r = fv - lu;
    }
    r0 = r1;
    r1 = r2;
    r2 = r;
    if (((y - ys0) & 1) == 0 && y > ys0) {
      rrow[t] = T(0.25) * r0 + T(0.5) * r1 + T(0.25) * r2;
      __syncthreads();
      if (I_ok) {
        const int J = (y - 1) / 2;
        fc[(size_t)J * nc + I] =
            I_int ? T(0.25) * rrow[t - 1] + T(0.5) * rrow[t] + T(0.25) * rrow[t + 1] : T(0);
      }
    }
#pragma unroll
    for (int k = 0; k < W - 1; ++k) w[k] = w[k + 1];
    w[W - 1] = un;
    buf ^= 1;
  }
}

// ------------------------------------------- 2D interpolation + correction ----
// uout = uin + I_H^h v.  Coarse rows are staged in LDS one at a time, interpolated in x
// for this thread's fine column, and kept in a 4-row register window from which the
// y interpolation is formed.  P = 3 cubic (weights -1,9,9,-1 over 16), P = 1 linear.
template <typename T, int P>
__global__ __launch_bounds__(kBlock) void k_prolong2d(const T *__restrict__ v,
                                                      const T *uin, T *uout, int n, int rows,
                                                      const int *__restrict__ done) {
  constexpr int NCOL = kBlock / 2 + 4;
  __shared__ T crow[2][NCOL];
  done = slot_done(done);
  if (stopped(done)) return;
  const int nc = (n - 1) / 2 + 1;
  v = slot_ptr(v, (size_t)nc * nc);
  uin = slot_ptr(uin, (size_t)n * n);
  uout = slot_ptr(uout, (size_t)n * n);
  const int t = threadIdx.x;
  const Block2 blk = block2();
  const int xb = blk.x * kBlock;
  const int x = xb + t;
  const int Ib = xb / 2 - 1;
  int sc = 1;
  const int Ic = fold(Ib + t, nc, sc);
  const bool cok = t < NCOL && Ic >= 0 && Ic <= nc - 1;
  const int y0 = blk.y * rows;
  const int y1 = min(y0 + rows, n);

  auto load_row = [&](int J, int b) {
    int s = sc;
    const int Js = fold(J, nc, s);
    T val = T(0);
    if (cok && Js >= 0 && Js <= nc - 1) {
      val = v[(size_t)Js * nc + Ic];
      if (s < 0) val = -val;
    }
    if (t < NCOL) crow[b][t] = val;
  };
  auto interp_x = [&](int b) -> T {
    if ((x & 1) == 0) return crow[b][x / 2 - Ib];
    const int i = (x - 1) / 2 - Ib;
    if (P == 3)
      return (T(9) * (crow[b][i] + crow[b][i + 1]) - (crow[b][i - 1] + crow[b][i + 2])) * T(0.0625);
    return T(0.5) * (crow[b][i] + crow[b][i + 1]);
  };

  T pw[4];
  int jb = (y0 >> 1) - 1;
  int b = 0;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    load_row(jb + k, b);
    __syncthreads();
    pw[k] = interp_x(b);
    b ^= 1;
  }
  for (int y = y0; y < y1; ++y) {
    const int Jc = y >> 1;
    while (jb < Jc - 1) {
      load_row(jb + 4, b);
      __syncthreads();
      const T nv = interp_x(b);
      b ^= 1;
      pw[0] = pw[1];
      pw[1] = pw[2];
      pw[2] = pw[3];
      pw[3] = nv;
      ++jb;
    }
    T val;
    if ((y & 1) == 0)
      val = pw[1];
    else if (P == 3)
      val = (T(9) * (pw[1] + pw[2]) - (pw[0] + pw[3])) * T(0.0625);
    else
      val = T(0.5) * (pw[1] + pw[2]);
    if (x <= n - 1) {
      const size_t id = (size_t)y * n + x;
      const bool interior = x >= 1 && x <= n - 2 && y >= 1 && y <= n - 2;
      uout[id] = interior ? uin[id] + val : T(0);
    }
  }
}

// ------------------------------------------------------- coarsest exact solve ----
// v = A^{-1} g on the coarsest level with the inverse precomputed on the host (FP64,
// stored transposed so that threads of a wave read consecutive entries).
template <typename T>
__global__ __launch_bounds__(kBlock) void k_coarsest(const double *__restrict__ ainv_t,
                                                     const T *__restrict__ g,
                                                     T *__restrict__ v, int nc, int dim,
                                                     const int *__restrict__ done) {
  extern __shared__ double gs[];
  done = slot_done(done);
  if (stopped(done)) return;
  const size_t per = dim == 2 ? (size_t)nc * nc : (size_t)nc * nc * nc;
  g = slot_ptr(g, per);
  v = slot_ptr(v, per);
  const int q = nc - 2;
  const int m = dim == 2 ? q * q : q * q * q;
  for (int p = threadIdx.x; p < m; p += kBlock) {
    const int i = 1 + p % q, j = 1 + (p / q) % q, k = dim == 3 ? 1 + p / (q * q) : 0;
    gs[p] = (double)g[((size_t)k * nc + j) * nc + i];
  }
  const int total = dim == 2 ? nc * nc : nc * nc * nc;
  for (int id = threadIdx.x; id < total; id += kBlock) {
    const int i = id % nc, j = (id / nc) % nc, k = id / (nc * nc);
    const bool bd = i == 0 || i == nc - 1 || j == 0 || j == nc - 1 ||
                    (dim == 3 && (k == 0 || k == nc - 1));
    if (bd) v[id] = T(0);
  }
  __syncthreads();
  for (int r = threadIdx.x; r < m; r += kBlock) {
    double s = 0.0;
    for (int c = 0; c < m; ++c) s += ainv_t[(size_t)c * m + r] * gs[c];
    const int i = 1 + r % q, j = 1 + (r / q) % q, k = dim == 3 ? 1 + r / (q * q) : 0;
    v[((size_t)k * nc + j) * nc + i] = (T)s;
  }
}

// -------------------------------------------------------------- residual check ----
// record = 0: store sum f^2 (the partials of a zero-u residual pass).  record = 1:
// relative residual of the latest pass into the history and the stopping decision.
__global__ __launch_bounds__(kBlock) void k_check(DevState *st, const double *__restrict__ partials,
                                                  int np, int record) {
  st += blockIdx.z;
  partials += (size_t)blockIdx.z * np;
  if (record && st->done) return;
  double s = 0.0;
  for (int i = threadIdx.x; i < np; i += kBlock) s += partials[i];
  const double tot = block_sum(s);
  if (threadIdx.x != 0) return;
  if (!record) {
    st->fnorm2 = tot;
    return;
  }
  const double rel = st->fnorm2 > 0.0 ? sqrt(tot / st->fnorm2) : sqrt(tot);
  const int c = st->checks;
  if (c < kMaxHistory) st->hist[c] = rel;
  st->checks = c + 1;
  if (c > 0) st->last_ratio = rel / st->hist[min(c - 1, kMaxHistory - 1)];
  int status = 0;
  if (!isfinite(rel)) {
    status = 4;
  } else if (rel <= st->rtol) {
    status = 1;
  } else if (c + 1 >= st->max_checks) {
    status = 2;
  } else if (c > 0 && rel > 1e3 * st->hist[0]) {
    status = 5;
  } else if (st->floor_detect) {
    if (c >= 2 && rel > 0.9 * st->best)
      st->stall += 1;
    else
      st->stall = 0;
    if (st->stall >= 2) status = 3;
  }
  if (c == 0 || rel < st->best) st->best = rel;
  if (status != 0) {
    st->status = status;
    st->done = 1;
  }
}

// u += e over the whole grid (the boundary of e is zero).  Four consecutive points per
// thread and step (16-byte loads of e, two of u when the arrays are 16-byte aligned), the
// last total % 4 points one by one.
__global__ __launch_bounds__(kBlock) void k_ir_correct(double *__restrict__ u,
                                                       const float *__restrict__ e, size_t total,
                                                       const int *__restrict__ done) {
  done = slot_done(done);
  if (stopped(done)) return;
  u = slot_ptr(u, total);
  e = slot_ptr(e, total);
  const size_t step = (size_t)gridDim.x * kBlock;
  const bool vec = ((reinterpret_cast<uintptr_t>(u) | reinterpret_cast<uintptr_t>(e)) & 15) == 0;
  const size_t quads = vec ? total / 4 : 0;
  for (size_t q = (size_t)blockIdx.x * kBlock + threadIdx.x; q < quads; q += step) {
    const float4 ev = reinterpret_cast<const float4 *>(e)[q];
    double2 *up = reinterpret_cast<double2 *>(u) + 2 * q;
    double2 a = up[0], b = up[1];
    a.x += (double)ev.x;
    a.y += (double)ev.y;
    b.x += (double)ev.z;
    b.y += (double)ev.w;
    up[0] = a;
    up[1] = b;
  }
  for (size_t i = quads * 4 + (size_t)blockIdx.x * kBlock + threadIdx.x; i < total; i += step)
    u[i] += (double)e[i];
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_fill(T *__restrict__ p, size_t count, T value,
                                                 const int *__restrict__ done) {
  done = slot_done(done);
  if (stopped(done)) return;
  p = slot_ptr(p, count);
  for (size_t i = (size_t)blockIdx.x * kBlock + threadIdx.x; i < count;
       i += (size_t)gridDim.x * kBlock)
    p[i] = value;
}

int cdiv(long a, long b) { return (int)((a + b - 1) / b); }

int clampi(long v, int lo, int hi) { return (int)(v < lo ? lo : (v > hi ? hi : v)); }

template <typename T, typename TO>
const void *sweep2d_fn(int mode, bool cross) {
  if (cross) {
    if (mode == kSweep) return (const void *)k_sweep2d<T, TO, kSweep, true>;
    if (mode == kResidual) return (const void *)k_sweep2d<T, TO, kResidual, true>;
    return (const void *)k_sweep2d<T, TO, kNormOnly, true>;
  }
  if (mode == kSweep) return (const void *)k_sweep2d<T, TO, kSweep, false>;
  if (mode == kResidual) return (const void *)k_sweep2d<T, TO, kResidual, false>;
  return (const void *)k_sweep2d<T, TO, kNormOnly, false>;
}

constexpr int kMinRows = 4;  // rows per band of the unfused 2D kernels, at least

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

// For R = 3 kernels the a/b arrays are used at offsets -3..3 directly.
}  // namespace

int resident_blocks(const void *fn, int threads, size_t smem) {
  static std::mutex mu;
  static std::map<std::tuple<int, const void *, int, size_t>, int> cache;
  int dev = 0;
  (void)hipGetDevice(&dev);
  const auto key = std::make_tuple(dev, fn, threads, smem);
  std::lock_guard<std::mutex> g(mu);
  const auto it = cache.find(key);
  if (it != cache.end()) return it->second;
  int per_cu = 0, cus = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, threads, smem) != hipSuccess ||
      per_cu < 1) {
    (void)hipGetLastError();
    per_cu = 1;
  }
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
      cus < 1) {
    (void)hipGetLastError();
    cus = 1;
  }
  return cache[key] = per_cu * cus;
}

int band_rows(int total, int across, int capacity, int cmin) {
  const int per = std::max(1, capacity / std::max(1, across));
  return std::max(cmin, cdiv(total, per));
}

int sweep_partials(int dim, int n) {
  if (dim == 2) {
    int best = 0;
    for (int R = 2; R <= 3; ++R) {
      const int np = cdiv(n, kBlock - 2 * R) * cdiv(n, kMinRows);
      best = np > best ? np : best;
    }
    return best;
  }
  return sweep_partials_3d(n);
}

template <typename T, typename TO>
hipError_t launch_sweep(int dim, int mode, const LevelOp &op, double omega, const T *f,
                        const T *u, TO *out, int n, double *partials, int *nparts,
                        const int *done, hipStream_t s, int slots, int colour) {
  if (colour < 0 || colour > 2) return hipErrorInvalidValue;
  if (dim == 2 && mode == kSweepZ2) return hipErrorInvalidValue;  // a 3D pass
  if (dim == 3) {
    if (slots != 1) return hipErrorInvalidValue;
    return launch_sweep_3d<T, TO>(mode, op, omega, f, u, out, n, partials, nparts, done, s, colour);
  }
  const int R = op.cross ? 2 : 3;
  const int nbx = cdiv(n, kBlock - 2 * R);
  const int rows =
      band_rows(n, nbx, resident_blocks(sweep2d_fn<T, TO>(mode, op.cross), kBlock, 0), kMinRows);
  const dim3 grid(nbx, cdiv(n, rows), slots);
  if (nparts) *nparts = grid.x * grid.y;
  KOp<T> k = to_kop<T>(op, omega);
  k.colour = colour;
#define MG_SWEEP2D(MODE, CROSS) \
  hipLaunchKernelGGL((k_sweep2d<T, TO, MODE, CROSS>), grid, dim3(kBlock), 0, s, f, u, out, n, rows, k, partials, done)
  if (op.cross) {
    if (mode == kSweep) MG_SWEEP2D(kSweep, true);
    else if (mode == kResidual) MG_SWEEP2D(kResidual, true);
    else MG_SWEEP2D(kNormOnly, true);
  } else {
    if (mode == kSweep) MG_SWEEP2D(kSweep, false);
    else if (mode == kResidual) MG_SWEEP2D(kResidual, false);
    else MG_SWEEP2D(kNormOnly, false);
  }
#undef MG_SWEEP2D
  return hipGetLastError();
}

template <typename T>
hipError_t launch_resid_restrict(int dim, const LevelOp &op, const T *f, const T *u, T *fc,
                                 int n, const int *done, hipStream_t s, int slots) {
  if (dim == 3) {
    if (slots != 1) return hipErrorInvalidValue;
    return launch_resid_restrict_3d<T>(op, f, u, fc, n, done, s);
  }
  const int nc = (n - 1) / 2 + 1;
  const int R = op.cross ? 2 : 3;
  const int CB = (kBlock - 2 * R - 2) / 2;
  const int nbx = cdiv(nc, CB);
  const void *fn = op.cross ? (const void *)k_resid_restrict2d<T, true>
                            : (const void *)k_resid_restrict2d<T, false>;
  const int crows = band_rows(nc, nbx, resident_blocks(fn, kBlock, 0), 2);
  const dim3 grid(nbx, cdiv(nc, crows), slots);
  const KOp<T> k = to_kop<T>(op, 1.0);
  if (op.cross)
    hipLaunchKernelGGL((k_resid_restrict2d<T, true>), grid, dim3(kBlock), 0, s, f, u, fc, n, crows, k, done);
  else
    hipLaunchKernelGGL((k_resid_restrict2d<T, false>), grid, dim3(kBlock), 0, s, f, u, fc, n, crows, k, done);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_prolong_correct(int dim, int prolong, const T *v, const T *uin, T *uout,
                                  int n, const int *done, hipStream_t s, int slots) {
  if (dim == 3) {
    if (slots != 1) return hipErrorInvalidValue;
    return launch_prolong_correct_3d<T>(prolong, v, uin, uout, n, done, s);
  }
  const int nbx = cdiv(n, kBlock);
  const void *fn = prolong == 3 ? (const void *)k_prolong2d<T, 3> : (const void *)k_prolong2d<T, 1>;
  const int rows = band_rows(n, nbx, resident_blocks(fn, kBlock, 0), kMinRows);
  const dim3 grid(nbx, cdiv(n, rows), slots);
  if (prolong == 3)
    hipLaunchKernelGGL((k_prolong2d<T, 3>), grid, dim3(kBlock), 0, s, v, uin, uout, n, rows, done);
  else
    hipLaunchKernelGGL((k_prolong2d<T, 1>), grid, dim3(kBlock), 0, s, v, uin, uout, n, rows, done);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_coarsest(int dim, const double *ainv_t, const T *g, T *v, int nc,
                           const int *done, hipStream_t s, int slots) {
  const int q = nc - 2;
  const int m = dim == 2 ? q * q : q * q * q;
  hipLaunchKernelGGL((k_coarsest<T>), dim3(1, 1, slots), dim3(kBlock), sizeof(double) * m, s, ainv_t, g, v,
                     nc, dim, done);
  return hipGetLastError();
}

hipError_t launch_check(DevState *st, const double *partials, int nparts, int record,
                        hipStream_t s, int slots) {
  hipLaunchKernelGGL(k_check, dim3(1, 1, slots), dim3(kBlock), 0, s, st, partials, nparts, record);
  return hipGetLastError();
}

hipError_t launch_ir_correct(int dim, double *u, const float *e, int n, const int *done,
                             hipStream_t s, int slots) {
  const size_t total = dim == 2 ? (size_t)n * n : (size_t)n * n * n;
  const int blocks = clampi(cdiv((long)(total / 4 + 1), kBlock), 1, 16384);
  hipLaunchKernelGGL(k_ir_correct, dim3(blocks, 1, slots), dim3(kBlock), 0, s, u, e, total, done);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_fill(T *p, size_t count, T value, const int *done, hipStream_t s, int slots) {
  const int blocks = clampi(cdiv((long)count, kBlock), 1, 8192);
  hipLaunchKernelGGL((k_fill<T>), dim3(blocks, 1, slots), dim3(kBlock), 0, s, p, count, value, done);
  return hipGetLastError();
}

// explicit instantiations
template hipError_t launch_sweep<double, double>(int, int, const LevelOp &, double, const double *,
                                                 const double *, double *, int, double *, int *,
                                                 const int *, hipStream_t, int, int);
template hipError_t launch_sweep<float, float>(int, int, const LevelOp &, double, const float *,
                                               const float *, float *, int, double *, int *,
                                               const int *, hipStream_t, int, int);
template hipError_t launch_sweep<double, float>(int, int, const LevelOp &, double, const double *,
                                                const double *, float *, int, double *, int *,
                                                const int *, hipStream_t, int, int);
template hipError_t launch_resid_restrict<double>(int, const LevelOp &, const double *,
                                                  const double *, double *, int, const int *,
                                                  hipStream_t, int);
template hipError_t launch_resid_restrict<float>(int, const LevelOp &, const float *, const float *,
                                                 float *, int, const int *, hipStream_t, int);
template hipError_t launch_prolong_correct<double>(int, int, const double *, const double *,
                                                   double *, int, const int *, hipStream_t, int);
template hipError_t launch_prolong_correct<float>(int, int, const float *, const float *, float *,
                                                  int, const int *, hipStream_t, int);
template hipError_t launch_coarsest<double>(int, const double *, const double *, double *, int,
                                            const int *, hipStream_t, int);
template hipError_t launch_coarsest<float>(int, const double *, const float *, float *, int,
                                           const int *, hipStream_t, int);
template hipError_t launch_fill<double>(double *, size_t, double, const int *, hipStream_t, int);
template hipError_t launch_fill<float>(float *, size_t, float, const int *, hipStream_t, int);

}  // namespace mgk
