// tail3d.hip -- the coarse end of a 3D cycle in one workgroup: a 17^3 level (any operator
// given by its 1D factors: the rediscretized cross, the sixth-order cross or a Galerkin
// product) and the 9^3 coarsest level, resident in LDS.
//
// The level operator is L = a_x b_y b_z + b_x a_y b_z + b_x b_y a_z with symmetric 1D
// factors a, b of radius 3 (a in difference form: a u(i) = sum_{j != 0} a_j (u(i+j) - u(i))).
// It is applied as three line passes over the interior:
//   y pass:  BY = b_y u,  AY = a_y u            (per (x, z) line)
//   x pass:  P2 = b_x BY, P1 = a_x BY + b_x AY  (per (y, z) line, in place of BY, AY)
//   z pass:  L u = b_z P1 + a_z P2              (per (x, y) line)
// about 60 multiply-adds per point instead of a walk over the 343 entries of the assembled
// Galerkin stencil.  Each line pass gives four threads to a line of 15 points (four
// outputs each, a window of ten inputs in registers).  Values beyond the boundary are the
// odd reflection of the Dirichlet closure (u, and every partial product, vanishes on the
// boundary planes and is odd across them), so every pass folds its indices instead of
// keeping ghost frames.
//
// The 9^3 level is solved exactly by sine transforms (FP64), as in the general tail.  One
// launch runs the parent's gamma visits of the 17^3 level (repeats), each: nu1 sweeps,
// defect and full weighting, the coarsest solve, interpolation and correction, nu2 sweeps.
#include <cstdint>

#include "mg_internal.h"

namespace mgk {
namespace {

constexpr int kT3N = 17, kT3NC = 9;
// FP32: 1024 threads, four outputs of a line each; FP64: 512 threads (more registers per
// thread for the wider windows), eight outputs each
template <typename T>
constexpr int t3_threads() { return sizeof(T) == 8 ? 512 : 1024; }
template <typename T>
constexpr int t3_outputs() { return sizeof(T) == 8 ? 8 : 4; }

// Index p of a line of side N folded into [0, N-1] by odd reflection; s = +-1, or 0 on
// the boundary (where every stored quantity is 0).
template <int N>
__device__ __forceinline__ int fold_line(int p, int &s) {
  s = 1;
  if (p < 0) { p = -p; s = -s; }
  if (p > N - 1) { p = 2 * (N - 1) - p; s = -s; }
  if (p == 0 || p == N - 1) s = 0;
  return p;
}

// LDS layout (elements of T): u and f (N^3 each, dense, zero on the boundary), g0 and g1
// (Q^3 each, interior points: BY and AY, then P2 and P1; the defect in g0), fc and uc
// (NC^3 each, dense), then the coefficients a_1..a_3, b_0..b_3 and omega / diagonal.
// The sine-transform work arrays (FP64) live in g1, which is free during the coarsest
// solve.  Every array sits at a compile-time offset from the one base register.
template <typename T>
struct T3 {
  static constexpr int N = kT3N, Q = N - 2, NC = kT3NC, QC = NC - 2;
  static constexpr int NT = t3_threads<T>(), OPT = t3_outputs<T>(), WIN = OPT + 6;
  static constexpr int TPL = (Q + OPT - 1) / OPT;  // threads per line
  static constexpr int NTH = Q * Q * TPL;          // threads of a line pass
  static_assert(NTH <= NT, "a line pass fits the workgroup");
  static constexpr int OU = 0, OF = N * N * N, OG0 = 2 * N * N * N, OG1 = OG0 + Q * Q * Q,
                       OFC = OG1 + Q * Q * Q, OUC = OFC + NC * NC * NC, OCOEF = OUC + NC * NC * NC,
                       TOTAL = OCOEF + 8;
  // the sine-transform arrays start at the first 8-byte boundary in g1
  static constexpr int OG1D = (OG1 * (int)sizeof(T) + 7) / 8;
  static_assert((OG1D + 2 * QC * QC * QC + QC * QC) * 8 <= OFC * (int)sizeof(T), "sine arrays fit in g1");
  T *base;
  const double *dst;  // global: the sine table, then the per-mode factors (2/N)^3 / lambda
  int nu1, nu2, prolong, rb;

  __device__ T *u() const { return base + OU; }
  __device__ T *f() const { return base + OF; }
  __device__ T *g0() const { return base + OG0; }
  __device__ T *g1() const { return base + OG1; }
  __device__ T *fc() const { return base + OFC; }
  __device__ T *uc() const { return base + OUC; }
  __device__ T *coef() const { return base + OCOEF; }
  __device__ double *g1d() const { return reinterpret_cast<double *>(base) + OG1D; }
  __device__ static int di(int x, int y, int z) { return (z * N + y) * N + x; }
  __device__ static int ii(int x, int y, int z) { return ((z - 1) * Q + (y - 1)) * Q + (x - 1); }

  // The WIN values at positions p0-3 .. p0+OPT+2 of a line whose position p sits at
  // b[p * stride]: plain loads when all of them lie in [LO, HI], else folded by the odd
  // reflection (positions 0 and N-1 give 0).  DENSE: the array stores positions 0 .. N-1
  // (u, zero on the boundary); otherwise 1 .. Q, and b points one stride before position 1.
  template <bool DENSE>
  __device__ static void window(const T *b, int stride, int p0, T (&w)[WIN]) {
    constexpr int LO = DENSE ? 0 : 1, HI = DENSE ? N - 1 : Q;
    if (p0 - 3 >= LO && p0 + OPT + 2 <= HI) {
#pragma unroll
      for (int i = 0; i < WIN; ++i) w[i] = b[(p0 - 3 + i) * stride];
    } else {
#pragma unroll
      for (int i = 0; i < WIN; ++i) {
        int s;
        const int p = fold_line<N>(p0 - 3 + i, s);
        w[i] = s == 0 ? T(0) : T(s) * b[p * stride];
      }
    }
  }
  // Line-pass thread layout: part-major (a wavefront mostly shares its part, so the
  // folding branch of window() is mostly uniform): line = t % (Q*Q), part = t / (Q*Q).
  static constexpr int LINES = Q * Q;

  // y pass: BY, AY of every interior point from u
  __device__ void pass_y() const {
    const int t = threadIdx.x;
    if (t < NTH) {
      const int line = t % LINES, part = t / LINES;
      const int x = 1 + line % Q, z = 1 + line / Q, y0 = 1 + OPT * part;
      const T *cf = coef();
      T *g0 = this->g0(), *g1 = this->g1();
      const T A[4] = {T(0), cf[0], cf[1], cf[2]}, B[4] = {cf[3], cf[4], cf[5], cf[6]};
      T w[WIN];
      window<true>(u() + di(x, 0, z), N, y0, w);
#pragma unroll
      for (int o = 0; o < OPT; ++o) {
        const int y = y0 + o;
        if (y > Q) break;
        const T c = w[o + 3];
        T sb = B[0] * c, sa = T(0);
#pragma unroll
        for (int j = 1; j <= 3; ++j) {
          sb += B[j] * (w[o + 3 + j] + w[o + 3 - j]);
          sa += A[j] * ((w[o + 3 + j] - c) + (w[o + 3 - j] - c));
        }
        g0[ii(x, y, z)] = sb;
        g1[ii(x, y, z)] = sa;
      }
    }
    __syncthreads();
  }
  // x pass: P2 = b_x BY into g0, P1 = a_x BY + b_x AY into g1 (in place: the windows are
  // read before any thread writes)
  __device__ void pass_x() const {
    const int t = threadIdx.x;
    T wb[WIN], wa[WIN];
    int y = 0, z = 0, x0 = 0;
    T *g0 = this->g0(), *g1 = this->g1();
    if (t < NTH) {
      const int line = t % LINES, part = t / LINES;
      y = 1 + line % Q;
      z = 1 + line / Q;
      x0 = 1 + OPT * part;
      const int r = ii(1, y, z) - 1;
      window<false>(g0 + r, 1, x0, wb);
      window<false>(g1 + r, 1, x0, wa);
    }
    __syncthreads();
    if (t < NTH) {
      const T *cf = coef();
      const T A[4] = {T(0), cf[0], cf[1], cf[2]}, B[4] = {cf[3], cf[4], cf[5], cf[6]};
#pragma unroll
      for (int o = 0; o < OPT; ++o) {
        const int x = x0 + o;
        if (x > Q) break;
        const T c = wb[o + 3];
        T p2 = B[0] * c, p1 = B[0] * wa[o + 3];
#pragma unroll
        for (int j = 1; j <= 3; ++j) {
          p2 += B[j] * (wb[o + 3 + j] + wb[o + 3 - j]);
          p1 += A[j] * ((wb[o + 3 + j] - c) + (wb[o + 3 - j] - c)) + B[j] * (wa[o + 3 + j] + wa[o + 3 - j]);
        }
        g0[ii(x, y, z)] = p2;
        g1[ii(x, y, z)] = p1;
      }
    }
    __syncthreads();
  }
  // z pass: L u = b_z P1 + a_z P2, then a Jacobi update of u (mode 0; colour 1 / 2: only
  // the points with odd / even x+y+z move) or the defect f - L u into g0 (mode 1)
  __device__ void pass_z(int mode, int colour) const {
    const int t = threadIdx.x;
    T w1v[WIN], w2v[WIN];
    int x = 0, y = 0, z0 = 0;
    T *g0 = this->g0(), *g1 = this->g1();
    if (t < NTH) {
      const int line = t % LINES, part = t / LINES;
      x = 1 + line % Q;
      y = 1 + line / Q;
      z0 = 1 + OPT * part;
      const int r = ii(x, y, 1) - Q * Q;
      window<false>(g1 + r, Q * Q, z0, w1v);
      window<false>(g0 + r, Q * Q, z0, w2v);
    }
    if (mode == 1) __syncthreads();  // the defect overwrites g0, which others still read
    if (t < NTH) {
      const T *cf = coef(), *f = this->f();
      T *u = this->u();
      const T A[4] = {T(0), cf[0], cf[1], cf[2]}, B[4] = {cf[3], cf[4], cf[5], cf[6]}, om = cf[7];
#pragma unroll
      for (int o = 0; o < OPT; ++o) {
        const int z = z0 + o;
        if (z > Q) break;
        const T c = w2v[o + 3];
        T lu = B[0] * w1v[o + 3];
#pragma unroll
        for (int j = 1; j <= 3; ++j)
          lu += B[j] * (w1v[o + 3 + j] + w1v[o + 3 - j]) + A[j] * ((w2v[o + 3 + j] - c) + (w2v[o + 3 - j] - c));
        const int d = di(x, y, z);
        const T r = f[d] - lu;
        if (mode == 1) {
          g0[ii(x, y, z)] = r;
        } else {
          const T w = (colour == 0 || ((x + y + z) & 1) == (colour & 1)) ? om : T(0);
          u[d] = u[d] + w * r;
        }
      }
    }
    __syncthreads();
  }
  __device__ void apply(int mode, int colour) const {
    pass_y();
    pass_x();
    pass_z(mode, colour);
  }
  // one Jacobi step from a zero iterate: u = om f (on the colour's points)
  __device__ void step_from_zero(int colour) const {
    T *u = this->u();
    const T *f = this->f();
    const T om = coef()[7];
    for (int p = threadIdx.x; p < Q * Q * Q; p += NT) {
      const int x = 1 + p % Q, y = 1 + (p / Q) % Q, z = 1 + p / (Q * Q);
      const T w = (colour == 0 || ((x + y + z) & 1) == (colour & 1)) ? om : T(0);
      u[di(x, y, z)] = w * f[di(x, y, z)];
    }
    __syncthreads();
  }
  // one smoothing sweep: omega-Jacobi, or red then black (section 3.1 eq. S_rb)
  __device__ void smooth(bool zero) const {
    if (rb) {
      if (zero)
        step_from_zero(1);
      else
        apply(0, 1);
      apply(0, 2);
    } else if (zero) {
      step_from_zero(0);
    } else {
      apply(0, 0);
    }
  }
  __device__ void zero_u() const {
    T *u = this->u();
    for (int p = threadIdx.x; p < N * N * N; p += NT) u[p] = T(0);
    __syncthreads();
  }
  // full weighting of the defect in g0 into fc (coarse interior; the fine points 2X +- 1
  // of an interior coarse point are all interior)
  __device__ void restrict_fw() const {
    const T *g0 = this->g0();
    T *fc = this->fc();
    for (int p = threadIdx.x; p < QC * QC * QC; p += NT) {
      const int X = 1 + p % QC, Y = 1 + (p / QC) % QC, Z = 1 + p / (QC * QC);
      T s = T(0);
#pragma unroll
      for (int oz = -1; oz <= 1; ++oz)
#pragma unroll
        for (int oy = -1; oy <= 1; ++oy)
#pragma unroll
          for (int ox = -1; ox <= 1; ++ox) {
            const T w = (ox == 0 ? T(0.5) : T(0.25)) * (oy == 0 ? T(0.5) : T(0.25)) * (oz == 0 ? T(0.5) : T(0.25));
            s += w * g0[ii(2 * X + ox, 2 * Y + oy, 2 * Z + oz)];
          }
      fc[(Z * NC + Y) * NC + X] = s;
    }
    __syncthreads();
  }
  // uc = A_c^{-1} fc by sine transforms along x, y, z, a per-mode scaling, and back (FP64)
  __device__ void coarsest() const {
    constexpr int q = QC, m = QC * QC * QC;
    double *a0 = g1d(), *a1 = a0 + m, *S = a1 + m;
    const T *fc = this->fc();
    T *uc = this->uc();
    const double *scale = dst + q * q;
    for (int p = threadIdx.x; p < m; p += NT) {
      const int X = 1 + p % q, Y = 1 + (p / q) % q, Z = 1 + p / (q * q);
      a0[p] = (double)fc[(Z * NC + Y) * NC + X];
    }
    for (int e = threadIdx.x; e < q * q; e += NT) S[e] = dst[e];
    __syncthreads();
    auto pass = [&](const double *in, double *out, int stride, bool scaled) {
      for (int c = threadIdx.x; c < m; c += NT) {
        const int k = (c / stride) % q, b0 = c - k * stride;
        double acc = 0.0;
#pragma unroll
        for (int i = 0; i < q; ++i) acc += S[k * q + i] * in[b0 + i * stride];
        out[c] = scaled ? acc * scale[c] : acc;
      }
      __syncthreads();
    };
    pass(a0, a1, 1, false);
    pass(a1, a0, q, false);
    pass(a0, a1, q * q, true);
    pass(a1, a0, 1, false);
    pass(a0, a1, q, false);
    pass(a1, a0, q * q, false);
    for (int p = threadIdx.x; p < m; p += NT) {
      const int X = 1 + p % q, Y = 1 + (p / q) % q, Z = 1 + p / (q * q);
      uc[(Z * NC + Y) * NC + X] = (T)a0[p];
    }
    __syncthreads();
  }
  // u += I_H^h uc at the fine interior points, one axis at a time: x into g0 (coarse
  // rows Y, Z interior, fine x), y into g1 (coarse planes Z, fine y, x), z into u.  A fine
  // point at even index takes the coarse value below it; at odd index the cubic weights
  // -1/16, 9/16, 9/16, -1/16 at coarse distances 3, 1, 1, 3 (linear: 1/2, 1/2), coarse
  // values beyond the boundary by odd reflection.
  __device__ T interp(const T *v, int stride, int i) const {
    // v(X) at coarse index X of a line with zero ends, i the fine index in [1, Q]
    auto at = [&](int X) -> T {
      int s;
      const int k = fold_line<NC>(X, s);
      return T(s) * v[k * stride];
    };
    if ((i & 1) == 0) return v[(i >> 1) * stride];
    const int lo = i >> 1;  // coarse points lo and lo + 1 at fine distance 1
    if (prolong == 3)
      return T(0.5625) * (at(lo) + at(lo + 1)) - T(0.0625) * (at(lo - 1) + at(lo + 2));
    return T(0.5) * (at(lo) + at(lo + 1));
  }
  __device__ void prolong_correct() const {
    const T *uc = this->uc();
    T *t1 = g0(), *t2 = g1(), *u = this->u();
    constexpr int A1 = QC * QC * Q, A2 = QC * Q * Q;
    // x: t1[Z-1][Y-1][x-1]
    for (int p = threadIdx.x; p < A1; p += NT) {
      const int x = 1 + p % Q, Y = 1 + (p / Q) % QC, Z = 1 + p / (Q * QC);
      t1[p] = interp(uc + (Z * NC + Y) * NC, 1, x);
    }
    __syncthreads();
    // y: t2[Z-1][y-1][x-1] from t1 (coarse rows 0 and NC-1 are zero: a zero row of t1 is
    // emulated by folding to the boundary index, which interp maps to zero)
    for (int p = threadIdx.x; p < A2; p += NT) {
      const int x = 1 + p % Q, y = 1 + (p / Q) % Q, Z = 1 + p / (Q * Q);
      const T *col = t1 + (Z - 1) * QC * Q + (x - 1);  // t1 at (Z, Y, x) = col[(Y-1) * Q]
      auto at = [&](int Y) -> T {
        int s;
        const int k = fold_line<NC>(Y, s);
        return s == 0 ? T(0) : T(s) * col[(k - 1) * Q];
      };
      T v;
      if ((y & 1) == 0) {
        v = at(y >> 1);
      } else {
        const int lo = y >> 1;
        v = prolong == 3 ? T(0.5625) * (at(lo) + at(lo + 1)) - T(0.0625) * (at(lo - 1) + at(lo + 2))
                         : T(0.5) * (at(lo) + at(lo + 1));
      }
      t2[p] = v;
    }
    __syncthreads();
    // z: u += from t2
    for (int p = threadIdx.x; p < Q * Q * Q; p += NT) {
      const int x = 1 + p % Q, y = 1 + (p / Q) % Q, z = 1 + p / (Q * Q);
      const T *col = t2 + (y - 1) * Q + (x - 1);  // t2 at (Z, y, x) = col[(Z-1) * Q * Q]
      auto at = [&](int Z) -> T {
        int s;
        const int k = fold_line<NC>(Z, s);
        return s == 0 ? T(0) : T(s) * col[(k - 1) * Q * Q];
      };
      T v;
      if ((z & 1) == 0) {
        v = at(z >> 1);
      } else {
        const int lo = z >> 1;
        v = prolong == 3 ? T(0.5625) * (at(lo) + at(lo + 1)) - T(0.0625) * (at(lo - 1) + at(lo + 2))
                         : T(0.5) * (at(lo) + at(lo + 1));
      }
      u[di(x, y, z)] += v;
    }
    __syncthreads();
  }
  // one visit of the 17^3 level
  __device__ void visit(bool zero) const {
    if (zero && nu1 == 0) zero_u();
    for (int s = 0; s < nu1; ++s) smooth(zero && s == 0);
    apply(1, 0);
    restrict_fw();
    coarsest();
    prolong_correct();
    for (int s = 0; s < nu2; ++s) smooth(false);
  }
};

template <typename T>
__global__ __launch_bounds__(t3_threads<T>()) void k_tail3(Tail3Args a) {
  extern __shared__ __align__(16) unsigned char t3_lds[];
  const int *done = slot_done(a.done);
  if (done != nullptr && *done != 0) return;
  using C = T3<T>;
  constexpr int N = C::N, NC = C::NC;
  C c;
  c.base = reinterpret_cast<T *>(t3_lds);
  c.dst = a.dst;
  c.nu1 = a.nu1;
  c.nu2 = a.nu2;
  c.prolong = a.prolong;
  c.rb = a.rb;
  if (threadIdx.x < 8) {
    const int k = threadIdx.x;  // a_1..a_3, b_0..b_3, omega / diagonal
    c.coef()[k] = (T)(k < 3 ? a.a[4 + k] : (k < 7 ? a.b[k] : a.om_d));
  }
  const size_t per = (size_t)N * N * N;
  const T *fg = slot_ptr(static_cast<const T *>(a.f_top), per);
  T *ug = slot_ptr(static_cast<T *>(a.u_top), per);
  constexpr int NT = C::NT;
  for (int i = threadIdx.x; i < N * N * N; i += NT) {
    const int x = i % N, y = (i / N) % N, z = i / (N * N);
    const bool in = x > 0 && x < N - 1 && y > 0 && y < N - 1 && z > 0 && z < N - 1;
    c.f()[i] = in ? fg[i] : T(0);
    c.u()[i] = (a.zero_init || !in) ? T(0) : ug[i];
  }
  for (int i = threadIdx.x; i < NC * NC * NC; i += NT) {
    c.fc()[i] = T(0);
    c.uc()[i] = T(0);
  }
  __syncthreads();
  for (int r = 0; r < a.repeats; ++r) c.visit(r == 0 && a.zero_init != 0);
  for (int i = threadIdx.x; i < N * N * N; i += NT) ug[i] = c.u()[i];
}

}  // namespace

static_assert(kT3N == 17 && kT3NC == 9 && kTail3Side == kT3N && kTail3Coarse == kT3NC, "tail sides");

size_t tail3_lds_bytes(size_t es) {
  return es == sizeof(float) ? T3<float>::TOTAL * sizeof(float) : T3<double>::TOTAL * sizeof(double);
}

template <typename T>
hipError_t tail3_prepare() {
  return hipFuncSetAttribute((const void *)k_tail3<T>, hipFuncAttributeMaxDynamicSharedMemorySize,
                             (int)tail3_lds_bytes(sizeof(T)));
}

template <typename T>
hipError_t launch_tail3(const Tail3Args &args, hipStream_t s, int slots) {
  hipLaunchKernelGGL((k_tail3<T>), dim3(1, 1, slots), dim3(t3_threads<T>()), tail3_lds_bytes(sizeof(T)), s, args);
  return hipGetLastError();
}

template hipError_t tail3_prepare<double>();
template hipError_t tail3_prepare<float>();
template hipError_t launch_tail3<double>(const Tail3Args &, hipStream_t, int);
template hipError_t launch_tail3<float>(const Tail3Args &, hipStream_t, int);

}  // namespace mgk
