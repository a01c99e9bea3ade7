// tail.hip -- the coarse end of a cycle in one workgroup, resident in LDS.
//
// Below a few thousand points per level, a multigrid level costs a few microseconds of
// launch latency per kernel and almost no memory traffic.  This kernel runs the whole
// gamma-cycle from a given level down to the coarsest one (pre-smoothing, defect and
// full weighting, the exact coarsest solve, interpolation and correction,
// post-smoothing; gamma recursive visits per level) inside one workgroup of 1024
// threads, with barriers between the steps.
//
// LDS layout per level: the iterate u with a ghost frame of G points on every side
// that holds the odd reflection across the Dirichlet boundary (refreshed after every
// update, so stencil reads need no index folding), and the right-hand side f without a
// frame.  One defect scratch array of the top level's size is shared by all levels.
// Rediscretized levels use the cross stencil directly; Galerkin levels walk a list of
// non-centre stencil entries in the difference form sum_e c_e (u(x + o_e) - u(x)).
#include <algorithm>
#include <cmath>
#include <cstdint>

#include "mg_internal.h"

namespace mgk {
namespace {

constexpr int kTailThreads = 1024;
// Points per thread of a sweep at the largest tail side (65^2 = 4225, 17^3 = 4913).
constexpr int kSlots = 5;
static_assert(65 * 65 <= kSlots * kTailThreads && 17 * 17 * 17 <= kSlots * kTailThreads,
              "tail sides must fit kSlots points per thread");
// Ghost frame G: a stencil of radius R reaches R-1 points past the boundary, cubic
// interpolation one coarse point; G = 1 when every tail level is the radius-2 cross,
// G = 2 otherwise.

// Thread tiling of a level (NT threads): TX x TY (x TZ) threads stride over the level.
template <int DIM, int NT>
struct Tiling;
template <>
struct Tiling<2, 1024> {
  static constexpr int TX = 64, TY = 16, TZ = 1;
};
template <>
struct Tiling<3, 1024> {
  static constexpr int TX = 16, TY = 8, TZ = 8;
};

struct LevelInfo {
  int n, pp;       // side and padded pitch (n + 2G)
  int u, u2, f;    // element offsets in LDS: the two framed iterates, the right-hand side
  int e0, ne;      // entries of this level in the LDS entry table
  double om_d;
  double w1, w2;   // cross weights (rediscretized levels)
  int cross;
};

template <typename T, int DIM, int G, int NT>
struct Tail {
  using TL = Tiling<DIM, NT>;
  const LevelInfo *lv;
  T *lds;
  const int *edelta;  // entry offsets as index deltas in the padded layout of their level
  const T *ecoef;
  const double *ainv_t;
  const double *dst;  // sine table of the coarsest solve, or null (dense inverse)
  int m, levels, gamma, nu1, nu2, prolong, scratch;
  int rb;  // red-black smoothing: a sweep is the red, then the black partial step
  int tx, ty, tz;
  // Each level keeps two framed iterates: a smoothing step reads one and writes the
  // other, so it needs one barrier; bit l tells which is current (uniform over threads).
  unsigned cur = 0u;

  __device__ __forceinline__ int ubase(int l) const { return ((cur >> l) & 1u) ? lv[l].u2 : lv[l].u; }
  __device__ __forceinline__ int obase(int l) const { return ((cur >> l) & 1u) ? lv[l].u : lv[l].u2; }
  __device__ __forceinline__ int pidx_in(int base, int l, int i, int j, int k) const {
    const int pp = lv[l].pp;
    return base + (DIM == 3 ? ((k + G) * pp + (j + G)) * pp : (j + G) * pp) + (i + G);
  }
  // element of the current iterate of level l
  __device__ __forceinline__ int pidx(int l, int i, int j, int k) const { return pidx_in(ubase(l), l, i, j, k); }
  __device__ __forceinline__ int didx(int l, int i, int j, int k) const {
    const int n = lv[l].n;
    return (DIM == 3 ? (k * n + j) * n : j * n) + i;
  }
  template <typename F>
  __device__ __forceinline__ void each(int n, F fn) const {
    for (int k = (DIM == 3 ? tz : 0); k < (DIM == 3 ? n : 1); k += TL::TZ)
      for (int j = ty; j < n; j += TL::TY)
        for (int i = tx; i < n; i += TL::TX) fn(i, j, k);
  }
  __device__ __forceinline__ bool interior(int n, int i, int j, int k) const {
    return i > 0 && i < n - 1 && j > 0 && j < n - 1 && (DIM == 2 || (k > 0 && k < n - 1));
  }
  // Point p of an n^DIM level in x-fastest order.
  __device__ __forceinline__ void decode(int p, int n, int &i, int &j, int &k) const {
    i = p % n;
    const int t = p / n;
    if (DIM == 3) {
      j = t % n;
      k = t / n;
    } else {
      j = t;
      k = 0;
    }
  }
  // The points threadIdx.x + r NT (r = 0, 1, ...) of an n^DIM level in x-fastest order,
  // walked without a division per point: start at the thread's point, then add NT's
  // coordinates (d) with carries.
  struct Walk {
    int i, j, k, di, dj, dk, n;
    __device__ __forceinline__ void next() {
      i += di;
      j += dj;
      if (i >= n) {
        i -= n;
        ++j;
      }
      if (DIM == 3) {
        k += dk;
        if (j >= n) {
          j -= n;
          ++k;
        }
      }
    }
  };
  __device__ __forceinline__ Walk walk(int n) const {
    Walk w;
    w.n = n;
    decode((int)threadIdx.x, n, w.i, w.j, w.k);
    decode(NT, n, w.di, w.dj, w.dk);
    return w;
  }
  // Stores the value v of interior point (i, j, k) of level l together with its odd
  // images in the ghost frame (points within G of the boundary have one image per such
  // axis, and the products of those for corners).  Frame cells whose source is a
  // boundary point hold 0 from the start and are never written.
  __device__ __forceinline__ void put(int l, int i, int j, int k, T v) const { put_in(ubase(l), l, i, j, k, v); }
  __device__ __forceinline__ void put_in(int base, int l, int i, int j, int k, T v) const {
    const int n = lv[l].n;
    int xs[2] = {i, i}, ys[2] = {j, j}, zs[2] = {k, k};
    int nx = 1, ny = 1, nz = 1;
    if (i <= G) { xs[1] = -i; nx = 2; } else if (i >= n - 1 - G) { xs[1] = 2 * (n - 1) - i; nx = 2; }
    if (j <= G) { ys[1] = -j; ny = 2; } else if (j >= n - 1 - G) { ys[1] = 2 * (n - 1) - j; ny = 2; }
    if (DIM == 3) {
      if (k <= G) { zs[1] = -k; nz = 2; } else if (k >= n - 1 - G) { zs[1] = 2 * (n - 1) - k; nz = 2; }
    }
    for (int c = 0; c < nz; ++c)
      for (int b = 0; b < ny; ++b)
        for (int a = 0; a < nx; ++a) {
          const bool odd = (a + b + c) & 1;
          lds[pidx_in(base, l, xs[a], ys[b], zs[c])] = odd ? -v : v;
        }
  }
  __device__ __forceinline__ T lu(int l, int p, T c) const {
    const LevelInfo &L = lv[l];
    if (L.cross) {
      const int sy = L.pp, sz = L.pp * L.pp;
      T d1 = (c - lds[p - 1]) + (c - lds[p + 1]);
      T d2 = (c - lds[p - 2]) + (c - lds[p + 2]);
      d1 += (c - lds[p - sy]) + (c - lds[p + sy]);
      d2 += (c - lds[p - 2 * sy]) + (c - lds[p + 2 * sy]);
      if (DIM == 3) {
        d1 += (c - lds[p - sz]) + (c - lds[p + sz]);
        d2 += (c - lds[p - 2 * sz]) + (c - lds[p + 2 * sz]);
      }
      return T(L.w1) * d1 + T(L.w2) * d2;
    }
    T s = T(0);
    for (int e = L.e0; e < L.e0 + L.ne; ++e) s += ecoef[e] * (lds[p + edelta[e]] - c);
    return s;
  }
  // refresh the ghost frame of u on level l with the odd reflection
  __device__ __forceinline__ void ghosts(int l) const {
    const int n = lv[l].n;
    for (int k = (DIM == 3 ? tz - G : 0); k < (DIM == 3 ? n + G : 1); k += TL::TZ)
      for (int j = ty - G; j < n + G; j += TL::TY)
        for (int i = tx - G; i < n + G; i += TL::TX) {
          const bool in = i >= 0 && i < n && j >= 0 && j < n && (DIM == 2 || (k >= 0 && k < n));
          if (in) continue;
          T sgn = T(1);
          int si = i, sj = j, sk = k;
          if (si < 0) { si = -si; sgn = -sgn; }
          if (si > n - 1) { si = 2 * (n - 1) - si; sgn = -sgn; }
          if (sj < 0) { sj = -sj; sgn = -sgn; }
          if (sj > n - 1) { sj = 2 * (n - 1) - sj; sgn = -sgn; }
          if (DIM == 3) {
            if (sk < 0) { sk = -sk; sgn = -sgn; }
            if (sk > n - 1) { sk = 2 * (n - 1) - sk; sgn = -sgn; }
          }
          lds[pidx(l, i, j, k)] = sgn * lds[pidx(l, si, sj, sk)];
        }
    __syncthreads();
  }
  // One omega-Jacobi step on level l: every thread computes its points (at most kSlots,
  // x-fastest order) from the current iterate and stores them, with their ghost images,
  // into the other one, which then becomes current.  colour 0 updates every interior
  // point, 1 those with odd i+j(+k), 2 the even ones; the others keep their value
  // (relaxation weight 0, stored as well).
  __device__ __forceinline__ void step(int l, bool zero, int colour) {
    const int n = lv[l].n;
    const int total = DIM == 3 ? n * n * n : n * n;
    const T om_all = T(lv[l].om_d);
    const int ob = obase(l);
    Walk wk = walk(n);
#pragma unroll
    for (int r = 0; r < kSlots; ++r) {
      const int p = (int)threadIdx.x + r * NT;
      if (p < total) {
        const int i = wk.i, j = wk.j, k = wk.k;
        if (interior(n, i, j, k)) {
          const int q = pidx(l, i, j, k);
          const T u0 = zero ? T(0) : lds[q];
          const T rr = lds[lv[l].f + p] - (zero ? T(0) : lu(l, q, u0));
          const T om = (colour == 0 || ((i + j + k) & 1) == (colour & 1)) ? om_all : T(0);
          put_in(ob, l, i, j, k, u0 + om * rr);
        }
      }
      wk.next();
    }
    cur ^= 1u << l;
    __syncthreads();
  }
  // One smoothing sweep: omega-Jacobi, or red then black (section 3.1 eq. S_rb).
  __device__ __forceinline__ void smooth(int l, bool zero) {
    if (rb) {
      step(l, zero, 1);
      step(l, false, 2);
    } else {
      step(l, zero, 0);
    }
  }
  __device__ __forceinline__ void zero_level(int l) const {
    const int n = lv[l].n;
    each(n, [&](int i, int j, int k) { lds[pidx(l, i, j, k)] = T(0); });
    __syncthreads();
    ghosts(l);
  }
  // defect of level l into the scratch array, then full weighting into f of level l+1
  __device__ __forceinline__ void resid_restrict(int l) const {
    const int n = lv[l].n;
    T *r = lds + scratch;
    each(n, [&](int i, int j, int k) {
      T v = T(0);
      if (interior(n, i, j, k)) {
        const int p = pidx(l, i, j, k);
        v = lds[lv[l].f + didx(l, i, j, k)] - lu(l, p, lds[p]);
      }
      r[didx(l, i, j, k)] = v;
    });
    __syncthreads();
    const int nc = lv[l + 1].n;
    T *fc = lds + lv[l + 1].f;
    each(nc, [&](int I, int J, int K) {
      T s = T(0);
      if (interior(nc, I, J, K)) {
        for (int oz = (DIM == 3 ? -1 : 0); oz <= (DIM == 3 ? 1 : 0); ++oz)
          for (int oy = -1; oy <= 1; ++oy)
            for (int ox = -1; ox <= 1; ++ox) {
              T w = (ox == 0 ? T(0.5) : T(0.25)) * (oy == 0 ? T(0.5) : T(0.25));
              if (DIM == 3) w *= (oz == 0 ? T(0.5) : T(0.25));
              s += w * r[didx(l, 2 * I + ox, 2 * J + oy, DIM == 3 ? 2 * K + oz : 0)];
            }
      }
      fc[didx(l + 1, I, J, K)] = s;
    });
    __syncthreads();
  }
  // Coarse points and weights of the interpolation along one axis at fine index x
  // (interior): four consecutive points from c0 for cubic interpolation, two for linear;
  // an even x takes its coarse point alone (weight 1, the others 0).  Every point read
  // lies inside the ghost-framed coarse array.
  template <int NP>
  __device__ __forceinline__ int axis_weights(int x, T (&w)[NP]) const {
    if (NP == 4) {
      const bool odd = x & 1;
      w[0] = odd ? T(-0.0625) : T(0);
      w[1] = odd ? T(0.5625) : T(1);
      w[2] = odd ? T(0.5625) : T(0);
      w[3] = odd ? T(-0.0625) : T(0);
      return odd ? (x - 3) >> 1 : (x >> 1) - 1;
    }
    const bool odd = x & 1;
    w[0] = odd ? T(0.5) : T(1);
    w[NP - 1] = odd ? T(0.5) : T(0);
    return x >> 1;
  }
  // u(l) += I_H^h u(l+1), coarse values read from the ghost-framed array
  template <int NP>
  __device__ __forceinline__ void prolong_np(int l) const {
    const int n = lv[l].n, ppc = lv[l + 1].pp;
    each(n, [&](int i, int j, int k) {
      if (!interior(n, i, j, k)) return;
      T wx[NP], wy[NP], wz[NP];
      const int i0 = axis_weights<NP>(i, wx), j0 = axis_weights<NP>(j, wy);
      const int k0 = DIM == 3 ? axis_weights<NP>(k, wz) : 0;
      const int base = pidx(l + 1, i0, j0, k0);
      T s = T(0);
#pragma unroll
      for (int c = 0; c < (DIM == 3 ? NP : 1); ++c) {
        const T zc = DIM == 3 ? wz[c] : T(1);
#pragma unroll
        for (int b = 0; b < NP; ++b) {
#pragma unroll
          for (int a = 0; a < NP; ++a)
            s += wx[a] * wy[b] * zc * lds[base + (DIM == 3 ? c * ppc * ppc : 0) + b * ppc + a];
        }
      }
      put(l, i, j, k, lds[pidx(l, i, j, k)] + s);
    });
    __syncthreads();
  }
  __device__ __forceinline__ void prolong_correct(int l) const {
    if (prolong == 3)
      prolong_np<4>(l);
    else
      prolong_np<2>(l);
  }
  // v = A^{-1} f on the coarsest level by sine transforms (FP64): the interior right-hand
  // side goes to a double array in the defect scratch, is transformed along each axis
  // (w(.., a, ..) = sum_i S(a, i) w(.., i, ..), one pass per axis), scaled per mode by
  // (2/N)^d / lambda, and transformed back.  A few KB of LDS, no matrix to stream.
  __device__ __forceinline__ void coarsest_dst(int l) const {
    const int n = lv[l].n, q = n - 2;
    double *w0 = reinterpret_cast<double *>((reinterpret_cast<uintptr_t>(lds + scratch) + 7) & ~uintptr_t(7));
    double *w1 = w0 + m, *S = w0 + 2 * m;
    const double *scale = dst + q * q;
    // interior point (1 + a, 1 + b, 1 + c) of element e in x-fastest order
    auto coords = [&](int e, int &ci, int &cj, int &ck) {
      ci = 1 + e % q;
      cj = 1 + (e / q) % q;
      ck = DIM == 3 ? 1 + e / (q * q) : 0;
    };
    // the first pass (along x) reads the right-hand side in place, with the table from
    // global memory, and copies the table to LDS for the other passes
    for (int e = threadIdx.x; e < q * q; e += NT) S[e] = dst[e];
    for (int c = threadIdx.x; c < m; c += NT) {
      const int a = c % q, b0 = c - a;
      int ci, cj, ck;
      coords(b0, ci, cj, ck);
      double acc = 0.0;
      for (int i = 0; i < q; ++i) acc += dst[a * q + i] * (double)lds[lv[l].f + didx(l, 1 + i, cj, ck)];
      w1[c] = acc;
    }
    __syncthreads();
    auto pass = [&](const double *in, double *out, int stride, bool scaled) {
      for (int c = threadIdx.x; c < m; c += NT) {
        const int a = (c / stride) % q, b0 = c - a * stride;
        double acc = 0.0;
        for (int i = 0; i < q; ++i) acc += S[a * q + i] * in[b0 + i * stride];
        out[c] = scaled ? acc * scale[c] : acc;
      }
      __syncthreads();
    };
    // forward along x (above), y (, z), the last forward pass scaled; then back along x,
    // y (, z), the last backward pass storing the solution into the iterate
    if (DIM == 3) {
      pass(w1, w0, q, false);
      pass(w0, w1, q * q, true);
      pass(w1, w0, 1, false);
      pass(w0, w1, q, false);
    } else {
      pass(w1, w0, q, true);
      pass(w0, w1, 1, false);
    }
    const int stride = DIM == 3 ? q * q : q;
    for (int c = threadIdx.x; c < m; c += NT) {
      const int a = (c / stride) % q, b0 = c - a * stride;
      double acc = 0.0;
      for (int i = 0; i < q; ++i) acc += S[a * q + i] * w1[b0 + i * stride];
      int ci, cj, ck;
      coords(c, ci, cj, ck);
      put(l, ci, cj, ck, (T)acc);
    }
    __syncthreads();
  }
  // v = A^{-1} f on the coarsest level, by sine transforms when the table is there, else
  // by the dense inverse (FP64 sums): the interior right-hand side is packed into the
  // defect scratch (row-major interior order, the order of A's unknowns); two adjacent
  // lanes share a row of A^{-1}, each summing one half of the columns, and add their
  // halves with a lane shuffle.  The result goes to the second half of the scratch.
  __device__ __forceinline__ void coarsest(int l) const {
    if (dst != nullptr) {
      coarsest_dst(l);
      return;
    }
    const int n = lv[l].n, q = n - 2;
    T *fv = lds + scratch, *v = fv + m;
    for (int c = threadIdx.x; c < m; c += NT) {
      const int ci = 1 + c % q, cj = 1 + (c / q) % q, ck = DIM == 3 ? 1 + c / (q * q) : 0;
      fv[c] = lds[lv[l].f + didx(l, ci, cj, ck)];
    }
    __syncthreads();
    const int half = (m + 1) / 2, h = threadIdx.x & 1;
    const int c0 = h * half, c1 = h ? m : half;
    for (int r0 = 0; r0 < m; r0 += NT / 2) {
      const int r = r0 + (threadIdx.x >> 1);
      const int rr = r < m ? r : m - 1;  // lanes past the last row repeat it (result unused)
      const double *col = ainv_t + rr;
      double val = 0.0;
#pragma unroll 8
      for (int c = c0; c < c1; ++c) val += col[(size_t)c * m] * (double)fv[c];
      val += __shfl_xor(val, 1);
      if (h == 0 && r < m) v[r] = (T)val;
    }
    __syncthreads();  // v complete
    for (int r = threadIdx.x; r < m; r += NT) {
      const int ri = 1 + r % q, rj = 1 + (r / q) % q, rk = DIM == 3 ? 1 + r / (q * q) : 0;
      put(l, ri, rj, rk, v[r]);
    }
    __syncthreads();
  }
};

// The gamma-cycle from level 0 of the tail, without recursion: a visit of level l
// pre-smooths, restricts and descends; the way back up interpolates, post-smooths and
// either repeats level l (gamma > 1, second visit from the same parent, non-zero guess)
// or returns to the parent.  Bit l of `visited` records a finished visit of level l.
template <typename T, int DIM, int G, int NT>
__device__ __forceinline__ void run_cycle(Tail<T, DIM, G, NT> &c, bool zero0) {
  const int last = c.levels - 1;
  if (last == 0) {
    c.coarsest(0);
    return;
  }
  int l = 0;
  bool zero = zero0;
  unsigned visited = 0u;
  for (;;) {
    // down: pre-smoothing and restriction of level l
    if (zero && c.nu1 == 0) c.zero_level(l);
    for (int s = 0; s < c.nu1; ++s) c.smooth(l, zero && s == 0);
    c.resid_restrict(l);
    if (l + 1 < last) {
      visited &= ~(1u << (l + 1));
      ++l;
      zero = true;
      continue;
    }
    c.coarsest(l + 1);
    // up: interpolation, correction and post-smoothing, as far as the visits allow
    for (;;) {
      c.prolong_correct(l);
      for (int s = 0; s < c.nu2; ++s) c.smooth(l, false);
      if (l == 0) return;
      if (c.gamma > 1 && !(visited & (1u << l))) {
        visited |= 1u << l;  // the parent's second visit of level l follows
        zero = false;
        break;
      }
      --l;
    }
  }
}

template <typename T, int DIM, int G, int NT>
__global__ __launch_bounds__(NT) void k_tail(TailArgs a) {
  extern __shared__ __align__(16) unsigned char tail_lds[];
  __shared__ LevelInfo lvt[kMaxTailLevels];
  const int *done = slot_done(a.done);
  if (done != nullptr && *done != 0) return;
  // level table: padded pitches and LDS offsets (u framed, f dense)
  if (threadIdx.x == 0) {
    int off = 0;
    for (int l = 0; l < a.levels; ++l) {
      LevelInfo &L = lvt[l];
      L.n = a.lv[l].n;
      L.pp = L.n + 2 * G;
      L.u = off;
      off += DIM == 3 ? L.pp * L.pp * L.pp : L.pp * L.pp;
      L.u2 = off;
      off += DIM == 3 ? L.pp * L.pp * L.pp : L.pp * L.pp;
      L.f = off;
      off += DIM == 3 ? L.n * L.n * L.n : L.n * L.n;
      L.e0 = a.lv[l].ent_begin - a.ent_first;
      L.ne = a.lv[l].ent_count;
      L.om_d = a.lv[l].om_d;
      L.cross = a.lv[l].cross;
      L.w1 = a.lv[l].w1;
      L.w2 = a.lv[l].w2;
    }
  }
  __syncthreads();
  T *lds = reinterpret_cast<T *>(tail_lds);
  int *edelta = reinterpret_cast<int *>(tail_lds + a.lds_ent);
  T *ecoef = reinterpret_cast<T *>(tail_lds + a.lds_ent + sizeof(int) * a.ent_total +
                                   (sizeof(T) - (sizeof(int) * a.ent_total) % sizeof(T)) % sizeof(T));
  for (int e = threadIdx.x; e < a.ent_total; e += NT) {
    const int g = a.ent_first + e;
    int l = 0;
    while (l + 1 < a.levels && e >= lvt[l + 1].e0) ++l;
    const int pp = lvt[l].pp;
    edelta[e] = (a.eoff[3 * g + 2] * pp + a.eoff[3 * g + 1]) * pp + a.eoff[3 * g];
    ecoef[e] = (T)a.ecoef[g];
  }
  using TL = Tiling<DIM, NT>;
  Tail<T, DIM, G, NT> c;
  c.lv = lvt;
  c.lds = lds;
  c.edelta = edelta;
  c.ecoef = ecoef;
  c.ainv_t = a.ainv_t;
  c.dst = a.dst;
  c.m = a.m;
  c.levels = a.levels;
  c.gamma = a.gamma;
  c.nu1 = a.nu1;
  c.nu2 = a.nu2;
  c.prolong = a.prolong;
  c.rb = a.rb;
  c.scratch = a.lds_r;
  c.tx = threadIdx.x % TL::TX;
  c.ty = (threadIdx.x / TL::TX) % TL::TY;
  c.tz = threadIdx.x / (TL::TX * TL::TY);
  const int n = lvt[0].n;
  const size_t per = DIM == 3 ? (size_t)n * n * n : (size_t)n * n;
  const T *fg = slot_ptr(static_cast<const T *>(a.f_top), per);
  T *ug = slot_ptr(static_cast<T *>(a.u_top), per);
  // the framed iterates start at zero (both of every level; level 0's current one is
  // loaded below): boundary points and the frame cells that mirror them are never
  // written afterwards
  for (int l = 0; l < a.levels; ++l) {
    const int pp = lvt[l].pp, tot = DIM == 3 ? pp * pp * pp : pp * pp;
    for (int e = threadIdx.x; e < tot; e += NT) {
      if (l > 0) lds[lvt[l].u + e] = T(0);
      lds[lvt[l].u2 + e] = T(0);
    }
  }
  c.each(n, [&](int i, int j, int k) {
    const int d = c.didx(0, i, j, k);
    lds[lvt[0].f + d] = fg[d];
    const bool bd = !c.interior(n, i, j, k);
    lds[c.pidx(0, i, j, k)] = (a.zero_init || bd) ? T(0) : ug[d];
  });
  __syncthreads();
  c.ghosts(0);
  for (int r = 0; r < a.repeats; ++r) run_cycle<T, DIM, G, NT>(c, r == 0 && a.zero_init != 0);
  c.each(n, [&](int i, int j, int k) { ug[c.didx(0, i, j, k)] = lds[c.pidx(0, i, j, k)]; });
}

}  // namespace

int tail_max_side(int dim) { return dim == 2 ? 65 : 17; }

// Element offset of the defect scratch (after every level's two framed iterates and dense f).
size_t tail_scratch_offset(int dim, int G, const int *ns, int levels) {
  size_t pts = 0;
  for (int l = 0; l < levels; ++l) {
    const size_t n = ns[l], pp = n + 2 * G;
    pts += dim == 3 ? 2 * pp * pp * pp + n * n * n : 2 * pp * pp + n * n;
  }
  return pts;
}

// Byte offset of the entry table.  The scratch holds the top level's defect, and on the
// coarsest level the packed right-hand side and the solution (two interior vectors), or
// the sine-transform work arrays (two FP64 interior vectors and the q x q table).
size_t tail_entry_offset(int dim, int G, const int *ns, int levels, size_t es) {
  const size_t n0 = ns[0], q = ns[levels - 1] - 2;
  const size_t top = dim == 3 ? n0 * n0 * n0 : n0 * n0, m = dim == 3 ? q * q * q : q * q;
  const size_t dst = ((2 * m + q * q) * 8 + 8 + es - 1) / es;  // sine-transform work arrays
  return (tail_scratch_offset(dim, G, ns, levels) + std::max(std::max(top, 2 * m), dst)) * es;
}

size_t tail_lds_bytes(int dim, int G, const int *ns, int levels, int entries, size_t es) {
  size_t bytes = tail_entry_offset(dim, G, ns, levels, es) + sizeof(int) * (size_t)entries;
  bytes = (bytes + es - 1) / es * es;
  return bytes + (size_t)entries * es;
}

template <typename T>
const void *tail_fn(int dim, int G) {
  if (dim == 2) return G == 1 ? (const void *)k_tail<T, 2, 1, kTailThreads> : (const void *)k_tail<T, 2, 2, kTailThreads>;
  return G == 1 ? (const void *)k_tail<T, 3, 1, kTailThreads> : (const void *)k_tail<T, 3, 2, kTailThreads>;
}

template <typename T>
hipError_t tail_prepare(int dim, int G, size_t lds_bytes) {
  return hipFuncSetAttribute(tail_fn<T>(dim, G), hipFuncAttributeMaxDynamicSharedMemorySize,
                             (int)lds_bytes);
}

template <typename T>
hipError_t launch_tail(int dim, int G, const TailArgs &args, size_t lds_bytes, hipStream_t s,
                       int slots) {
  const dim3 grid(1, 1, slots);
  if (dim == 2 && G == 1)
    hipLaunchKernelGGL((k_tail<T, 2, 1, kTailThreads>), grid, dim3(kTailThreads), lds_bytes, s, args);
  else if (dim == 2)
    hipLaunchKernelGGL((k_tail<T, 2, 2, kTailThreads>), grid, dim3(kTailThreads), lds_bytes, s, args);
  else if (G == 1)
    hipLaunchKernelGGL((k_tail<T, 3, 1, kTailThreads>), grid, dim3(kTailThreads), lds_bytes, s, args);
  else
    hipLaunchKernelGGL((k_tail<T, 3, 2, kTailThreads>), grid, dim3(kTailThreads), lds_bytes, s, args);
  return hipGetLastError();
}

template hipError_t tail_prepare<double>(int, int, size_t);
template hipError_t tail_prepare<float>(int, int, size_t);
template hipError_t launch_tail<double>(int, int, const TailArgs &, size_t, hipStream_t, int);
template hipError_t launch_tail<float>(int, int, const TailArgs &, size_t, hipStream_t, int);

}  // namespace mgk
