// runtime.hip -- host runtime and C ABI of the multigrid library.
//
// Hierarchy: standard coarsening n_{l+1} = (n_l - 1)/2 + 1 down to n_coarsest (eq. G_H_d).
// Level operators are kept as 1D factors (a along an axis, b along the others):
//   rediscretized: a = the 1D fourth- (or second-) order second difference at h_l, b = unit
//   (eq. L_H_4n_2d);
//   Galerkin: a_{l+1} = R a_l P and b_{l+1} = R b_l P in 1D, which is exactly R L_l P for the
//   tensor-product transfers (eqs. L_H_G, L_H_4G).
// A solve step is one gamma-cycle (FP64) or one refinement step (MIXED); it is captured
// once into a HIP graph and replayed.  The residual check runs on the device and sets a
// flag that makes every later kernel of the step return at once, so the host can launch
// replays in chunks and read the flag one chunk behind without stalling the GPU.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstddef>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <type_traits>
#include <vector>

#include "batch.h"
#include "mg.h"
#include "mg_internal.h"

using mgk::DevState;
using mgk::LevelOp;

namespace mgk {

// The rediscretized operator of a level of spacing h as 1D factors: a = the 1D second
// difference of the given order, b = unit (eqs. L_h_2d_4o, L_H_4n_2d, L_H_2d; section 3.3
// eq. LhOrder6).
LevelOp rediscretized_op(int order, int dim, double h) {
  LevelOp op{};
  const double s = 1.0 / (h * h);
  if (order == 6) {
    // section 3.3 eq. LhOrder6: radius 3, applied by the separable (Galerkin-level) kernels
    const double c[7] = {-2.0 / 180, 27.0 / 180, -270.0 / 180, 490.0 / 180, -270.0 / 180, 27.0 / 180, -2.0 / 180};
    for (int i = 0; i < 7; ++i) op.a[i] = c[i] * s;
  } else if (order == 4) {
    const double c[7] = {0.0, 1.0 / 12, -16.0 / 12, 30.0 / 12, -16.0 / 12, 1.0 / 12, 0.0};
    for (int i = 0; i < 7; ++i) op.a[i] = c[i] * s;
  } else {
    const double c[7] = {0.0, 0.0, -1.0, 2.0, -1.0, 0.0, 0.0};
    for (int i = 0; i < 7; ++i) op.a[i] = c[i] * s;
  }
  op.b[3] = 1.0;
  op.cross = order != 6;
  op.cross3 = order == 6;
  op.diag = dim * op.a[3];
  return op;
}

}  // namespace mgk

using mgk::rediscretized_op;

namespace {

thread_local std::string g_error;

mg_status fail(mg_status st, const std::string &msg) {
  g_error = msg;
  return st;
}

#define MG_HIP(call)                                                                      \
  do {                                                                                    \
    hipError_t e_ = (call);                                                               \
    if (e_ != hipSuccess)                                                                 \
      return fail(MG_EDEVICE, std::string(#call) + ": " + hipGetErrorString(e_));         \
  } while (0)

struct Buffers {
  void *u = nullptr, *f = nullptr, *t = nullptr;
  void *t2 = nullptr;  // second sweep target (fused red-black passes, see rb_passes)
};

__global__ void k_state_init(DevState *st, double rtol, int max_checks, int floor_detect) {
  if (threadIdx.x == 0) {
    st->done = 0;
    st->checks = 0;
    st->status = 0;
    st->stall = 0;
    st->max_checks = max_checks;
    st->floor_detect = floor_detect;
    st->rtol = rtol;
    st->fnorm2 = 0.0;
    st->best = 0.0;
    st->last_ratio = 0.0;
  }
}

int num_levels(int n, int nc) {
  if (nc < 5 || n < nc) return 0;
  int L = 1;
  while (n > nc) {
    if ((n - 1) % 2) return 0;
    n = (n - 1) / 2 + 1;
    ++L;
  }
  return n == nc ? L : 0;
}

// 1D restriction weight (full weighting) and interpolation weight at fine offset o.
double fw1(int o) { return o == 0 ? 0.5 : (o == 1 || o == -1 ? 0.25 : 0.0); }
double p1(int prolong, int o) {
  o = o < 0 ? -o : o;
  if (prolong == 3) return o == 0 ? 1.0 : (o == 1 ? 9.0 / 16.0 : (o == 3 ? -1.0 / 16.0 : 0.0));
  return o == 0 ? 1.0 : (o == 1 ? 0.5 : 0.0);
}

// c' = R c P in 1D (coarse offsets -3..3): c'_J = sum_o r(o) sum_k c_k p(o + k - 2J).
void galerkin_1d(const double c[7], int prolong, double out[7]) {
  // c, the weighting and the interpolation are all symmetric, so the product is: the
  // entries at -J are those at +J (taken from one sum, so that the factor is symmetric to
  // the last bit and the sine transforms diagonalize the assembled coarsest matrix)
  for (int J = 0; J <= 3; ++J) {
    double s = 0.0;
    for (int o = -1; o <= 1; ++o)
      for (int k = -3; k <= 3; ++k) s += fw1(o) * c[k + 3] * p1(prolong, o + k - 2 * J);
    out[3 + J] = s;
    out[3 - J] = s;
  }
}

LevelOp galerkin(const LevelOp &fine, int dim, int prolong) {
  LevelOp op{};
  galerkin_1d(fine.a, prolong, op.a);
  galerkin_1d(fine.b, prolong, op.b);
  op.cross = false;
  op.diag = dim * op.a[3] * std::pow(op.b[3], dim - 1);
  return op;
}

// Dense matrix of the level operator over interior points (odd reflection folded in),
// inverted by Gauss-Jordan elimination with partial pivoting; returned transposed.
// The coarsest operator as a dense m x m matrix over the interior points (x fastest),
// with the odd reflection of the Dirichlet closure folded in.
std::vector<double> coarsest_matrix(const LevelOp &op, int dim, int n) {
  const int q = n - 2;
  const int m = dim == 2 ? q * q : q * q * q;
  std::vector<double> A((size_t)m * m, 0.0);
  auto coef = [&](int ox, int oy, int oz) {
    // sum over axes of a along the axis times b along the others
    double c = op.a[ox + 3] * op.b[oy + 3];
    double d = op.b[ox + 3] * op.a[oy + 3];
    if (dim == 3) {
      c *= op.b[oz + 3];
      d *= op.b[oz + 3];
      return c + d + op.b[ox + 3] * op.b[oy + 3] * op.a[oz + 3];
    }
    return c + d;
  };
  auto fold = [&](int i, double &sign) {
    if (i < 0) { i = -i; sign = -sign; }
    if (i > n - 1) { i = 2 * (n - 1) - i; sign = -sign; }
    return i;
  };
  const int zr = dim == 3 ? 3 : 0;
  for (int row = 0; row < m; ++row) {
    const int i = 1 + row % q, j = 1 + (row / q) % q, k = dim == 3 ? 1 + row / (q * q) : 0;
    for (int oz = -zr; oz <= zr; ++oz)
      for (int oy = -3; oy <= 3; ++oy)
        for (int ox = -3; ox <= 3; ++ox) {
          const double c = coef(ox, oy, oz);
          if (c == 0.0) continue;
          double sign = 1.0;
          const int ti = fold(i + ox, sign), tj = fold(j + oy, sign);
          const int tk = dim == 3 ? fold(k + oz, sign) : 0;
          if (ti == 0 || ti == n - 1 || tj == 0 || tj == n - 1) continue;
          if (dim == 3 && (tk == 0 || tk == n - 1)) continue;
          const int col = (ti - 1) + q * ((tj - 1) + (dim == 3 ? q * (tk - 1) : 0));
          A[(size_t)row * m + col] += sign * c;
        }
  }
  return A;
}

bool coarsest_inverse(const LevelOp &op, int dim, int n, std::vector<double> &inv_t) {
  const int q = n - 2;
  const int m = dim == 2 ? q * q : q * q * q;
  std::vector<double> A = coarsest_matrix(op, dim, n), B((size_t)m * m, 0.0);
  for (int r = 0; r < m; ++r) B[(size_t)r * m + r] = 1.0;
  for (int c = 0; c < m; ++c) {
    int p = c;
    for (int r = c + 1; r < m; ++r)
      if (std::fabs(A[(size_t)r * m + c]) > std::fabs(A[(size_t)p * m + c])) p = r;
    if (A[(size_t)p * m + c] == 0.0) return false;
    if (p != c)
      for (int k = 0; k < m; ++k) {
        std::swap(A[(size_t)p * m + k], A[(size_t)c * m + k]);
        std::swap(B[(size_t)p * m + k], B[(size_t)c * m + k]);
      }
    const double piv = 1.0 / A[(size_t)c * m + c];
    for (int k = 0; k < m; ++k) {
      A[(size_t)c * m + k] *= piv;
      B[(size_t)c * m + k] *= piv;
    }
    for (int r = 0; r < m; ++r) {
      if (r == c) continue;
      const double l = A[(size_t)r * m + c];
      if (l == 0.0) continue;
      for (int k = 0; k < m; ++k) {
        A[(size_t)r * m + k] -= l * A[(size_t)c * m + k];
        B[(size_t)r * m + k] -= l * B[(size_t)c * m + k];
      }
    }
  }
  inv_t.assign((size_t)m * m, 0.0);
  for (int r = 0; r < m; ++r)
    for (int c = 0; c < m; ++c) inv_t[(size_t)c * m + r] = B[(size_t)r * m + c];
  return true;
}

// Sine-transform form of the coarsest solve.  Under the odd-reflection closure every
// level operator is a symmetric stencil applied alike at every interior point, so the
// sine modes sin(pi i k / N) (N = n - 1) are its eigenvectors, and with the 1D factors
// a, b of radius <= 3 the eigenvalue of mode (kx, ky, kz) is
//   lambda = a^(kx) b^(ky) b^(kz) + b^(kx) a^(ky) b^(kz) + b^(kx) b^(ky) a^(kz),
//   c^(k) = c_0 + 2 sum_j c_j cos(pi j k / N).
// Then L^{-1} = (2/N)^d S diag(1/lambda) S with S_ik = sin(pi i k / N) per axis.  The
// table holds S (q x q) followed by (2/N)^d / lambda for every mode (x fastest).  Each
// eigenpair is checked against the assembled matrix; false if any fails.
bool coarsest_dst(const LevelOp &op, int dim, int n, std::vector<double> &tab) {
  const int q = n - 2, N = n - 1;
  const int m = dim == 2 ? q * q : q * q * q;
  const double pi = 3.14159265358979323846;
  std::vector<double> S((size_t)q * q), ah(q), bh(q);
  for (int i = 0; i < q; ++i)
    for (int k = 0; k < q; ++k) S[(size_t)i * q + k] = std::sin(pi * (i + 1) * (k + 1) / N);
  for (int k = 0; k < q; ++k) {
    double sa = op.a[3], sb = op.b[3];
    for (int j = 1; j <= 3; ++j) {
      if (op.a[3 + j] != op.a[3 - j] || op.b[3 + j] != op.b[3 - j]) return false;  // not symmetric
      sa += 2.0 * op.a[3 + j] * std::cos(pi * j * (k + 1) / N);
      sb += 2.0 * op.b[3 + j] * std::cos(pi * j * (k + 1) / N);
    }
    ah[k] = sa;
    bh[k] = sb;
  }
  const std::vector<double> A = coarsest_matrix(op, dim, n);
  const double norm = std::pow(2.0 / N, dim);
  tab.assign((size_t)q * q + m, 0.0);
  std::copy(S.begin(), S.end(), tab.begin());
  std::vector<double> v(m), Av(m);
  for (int mode = 0; mode < m; ++mode) {
    const int kx = mode % q, ky = (mode / q) % q, kz = dim == 3 ? mode / (q * q) : 0;
    double lam = ah[kx] * bh[ky] + bh[kx] * ah[ky];
    if (dim == 3) lam = ah[kx] * bh[ky] * bh[kz] + bh[kx] * ah[ky] * bh[kz] + bh[kx] * bh[ky] * ah[kz];
    if (!(std::fabs(lam) > 0.0)) return false;
    double vmax = 0.0;
    for (int p = 0; p < m; ++p) {
      const int i = p % q, j = (p / q) % q, k = dim == 3 ? p / (q * q) : 0;
      v[p] = S[(size_t)i * q + kx] * S[(size_t)j * q + ky] * (dim == 3 ? S[(size_t)k * q + kz] : 1.0);
      vmax = std::max(vmax, std::fabs(v[p]));
    }
    double err = 0.0;
    for (int r = 0; r < m; ++r) {
      double acc = 0.0;
      for (int c2 = 0; c2 < m; ++c2) acc += A[(size_t)r * m + c2] * v[c2];
      err = std::max(err, std::fabs(acc - lam * v[r]));
    }
    if (err > 1e-10 * std::fabs(lam) * vmax) return false;
    tab[(size_t)q * q + mode] = norm / lam;
  }
  return true;
}

size_t points(int dim, int n) { return dim == 2 ? (size_t)n * n : (size_t)n * n * n; }

mg_status validate(const mg_config *c, int *levels) {
  if (!c) return fail(MG_EINVAL, "null config");
  if (c->dim != 2 && c->dim != 3) return fail(MG_EINVAL, "dim must be 2 or 3");
  if (c->order != 2 && c->order != 4 && c->order != 6) return fail(MG_EINVAL, "order must be 2, 4 or 6");
  if (c->coarse != MG_COARSE_NG && c->coarse != MG_COARSE_GALERKIN && c->coarse != MG_COARSE_NG2 &&
      c->coarse != MG_COARSE_G2)
    return fail(MG_EINVAL, "unknown coarse operator");
  if (c->smoother != MG_SMOOTH_JACOBI && c->smoother != MG_SMOOTH_RBJ && c->smoother != MG_SMOOTH_RBGS)
    return fail(MG_EINVAL, "unknown smoother");
  if (c->smoother == MG_SMOOTH_RBGS &&
      (c->dim != 2 || (c->coarse != MG_COARSE_NG && c->coarse != MG_COARSE_NG2)))
    return fail(MG_EINVAL, "red-black Gauss-Seidel needs dim 2 and rediscretized (cross-stencil) coarse operators");
  if (c->nu1 < 0 || c->nu2 < 0 || c->nu1 + c->nu2 < 1 || c->nu1 > 16 || c->nu2 > 16)
    return fail(MG_EINVAL, "need 0 <= nu1, nu2 <= 16 and nu1 + nu2 >= 1");
  if (c->gamma != 1 && c->gamma != 2) return fail(MG_EINVAL, "gamma must be 1 (V) or 2 (W)");
  if (c->prolong != 1 && c->prolong != 3) return fail(MG_EINVAL, "prolong must be 1 or 3");
  if (c->restrict_op != 1 && c->restrict_op != 3)
    return fail(MG_EINVAL, "restrict_op must be 1 (full weighting) or 3 (cubic adjoint)");
  if (c->restrict_op == 3 && c->coarse != MG_COARSE_NG && c->coarse != MG_COARSE_NG2)
    return fail(MG_EINVAL, "the cubic-adjoint restriction needs rediscretized coarse operators (its Galerkin "
                           "products would have stencils wider than radius 3)");
  if (c->precision != MG_PREC_FP64 && c->precision != MG_PREC_MIXED)
    return fail(MG_EINVAL, "unknown precision");
  if (c->omega > 0.0 && c->omega >= 2.0) return fail(MG_EINVAL, "omega must be in (0, 2)");
  if (c->max_cycles < 1 || c->max_cycles > MG_MAX_HISTORY - 2)
    return fail(MG_EINVAL, "max_cycles out of range");
  if (c->precision == MG_PREC_MIXED && (c->inner_cycles < 1 || c->inner_cycles > 64))
    return fail(MG_EINVAL, "inner_cycles must be in 1..64 for mixed precision");
  if (!(c->rtol >= 0.0)) return fail(MG_EINVAL, "rtol must be >= 0");
  const int maxn = c->dim == 2 ? 32769 : 2049;
  if (c->n > maxn) return fail(MG_EINVAL, "n too large");
  if (c->n_coarsest > (c->dim == 2 ? 33 : 9)) return fail(MG_EINVAL, "n_coarsest too large");
  const int L = num_levels(c->n, c->n_coarsest);
  if (L <= 0) return fail(MG_EINVAL, "n must be 2^k+1 coarsening to n_coarsest >= 5");
  *levels = L;
  return MG_OK;
}

double default_omega(int dim, int order, int smoother, int coarse) {
  // Red-black smoothers: the minimiser of the Fourier-analysis two-grid factor of the V(2,1)
  // cycle with cubic interpolation, to two decimals, per fine order and coarse operator
  // (section 3.1 tunes omega per coarse operator).  Coarse index: NG, GALERKIN, NG2, G2.
  if (smoother == MG_SMOOTH_RBGS) {  // 2D, NG or NG2
    if (order == 2) return 1.0;
    const bool ng2 = coarse == MG_COARSE_NG2;
    return order == 6 ? (ng2 ? 1.0 : 1.18) : (ng2 ? 0.98 : 1.16);
  }
  if (smoother == MG_SMOOTH_RBJ) {
    static const double t2[3][4] = {{1.0, 0.98, 1.0, 0.98}, {1.13, 1.0, 0.98, 0.97}, {1.13, 1.02, 0.99, 0.99}};
    static const double t3[3][4] = {{1.13, 1.09, 1.13, 1.09}, {1.17, 1.09, 1.09, 1.08}, {1.15, 1.1, 1.09, 1.08}};
    const int oi = order == 2 ? 0 : (order == 4 ? 1 : 2);
    return dim == 2 ? t2[oi][coarse] : t3[oi][coarse];
  }
  // omega-Jacobi: equioscillation of the symbol over the high frequencies (the two-grid
  // factor is smoothing-limited and the same for every coarse operator).
  if (order == 6) return dim == 2 ? 490.0 / 653.0 : 147.0 / 185.0;
  if (order == 4) return dim == 2 ? 10.0 / 13.0 : 9.0 / 11.0;
  return dim == 2 ? 4.0 / 5.0 : 6.0 / 7.0;
}

}  // namespace

struct mg_ctx {
  mg_config cfg{};
  double omega = 0.0;
  int dim = 2, L = 0;
  std::vector<int> ns;
  std::vector<LevelOp> ops;
  std::vector<Buffers> b64, b32;
  int device = 0;
  hipStream_t stream = nullptr, cap = nullptr;
  double *ainv_t = nullptr;
  double *dst = nullptr;    // sine-transform table of the coarsest solve (tail), or null
  double *partials = nullptr;
  int np_max = 0;
  DevState *st = nullptr;
  int *poll = nullptr;  // pinned host: 2 x {done, checks}
  hipEvent_t ev[2] = {nullptr, nullptr};
  hipEvent_t ev_async = nullptr;
  bool async_pending = false;
  hipGraph_t graph = nullptr;
  hipGraphExec_t gexec = nullptr;
  const double *gf = nullptr;
  double *gu = nullptr;
  bool use_graph = true;
  bool fused = true;       // temporally blocked 2D kernels
  int tail_top = 0;        // first level handled by the LDS-resident tail (L: none)
  size_t tail_lds = 0;     // dynamic LDS bytes of the tail
  bool tail3 = false;      // 3D: the tail is 17^3 + 9^3 in the line-pass kernel
  int *eoff = nullptr;     // stencil entry lists of every level (tail kernel)
  double *ecoef = nullptr;
  std::vector<int> ent_begin, ent_count;
  int chunk = 0;          // steps per replay chunk; 0: chosen from the measured step time
  int slots = 1;         // independent problems of this size (batched launches, grid.z)
  bool own_top = false;  // level-0 FP64 f and u are the handle's (batches), not the caller's
  std::vector<void *> allocs;
  size_t footprint = 0;
};

namespace {

mg_status dev_alloc(mg_ctx *c, void **p, size_t bytes) {
  *p = nullptr;
  if (bytes == 0) return MG_OK;
  hipError_t e = hipMalloc(p, bytes);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    *p = nullptr;
    return fail(MG_ENOMEM, std::string("hipMalloc failed: ") + hipGetErrorString(e));
  }
  c->allocs.push_back(*p);
  c->footprint += bytes;
  return MG_OK;
}

int partials_needed(int dim, int n) {
  int np = mgk::sweep_partials(dim, n);
  if (dim == 2) np = std::max(np, mgk::pre2d_partials(n));
  return np;
}

// Upper bound of the stencil entry lists (non-centre entries of every level).
size_t entries_bytes(const mg_config *cfg, int L) {
  const int w = 7;
  const size_t per = cfg->dim == 2 ? (size_t)w * w : (size_t)w * w * w;
  return (size_t)L * per * (3 * sizeof(int) + sizeof(double));
}

// Fused 2D red-black cycles run one pass per red-black sweep: max(1, nu1) pre passes (the
// last one also forms and restricts the defect) and max(1, nu2) post passes (the first one
// also interpolates and corrects).  Passes alternate between u and t and must end in u;
// with an odd number of passes the first one writes a third array t2.
int rb_passes(const mg_config *cfg) { return std::max(1, cfg->nu1) + std::max(1, cfg->nu2); }
// 3D red-black sweeps of FP64 cross levels in one pass (k_rbxsweep3d); MG_RB3_FUSED=0
// runs the two partial steps as separate launches.  Measured at 513^3: FP64 solves 56.4
// against 60.9 ms; FP32 cycles are faster as two launches (mixed 44.0 against 39.8 ms).
bool rb3_fused() {
  static const bool on = [] {
    const char *e = std::getenv("MG_RB3_FUSED");
    return e == nullptr || std::atoi(e) != 0;
  }();
  return on;
}

bool needs_t2(const mg_config *cfg) {
  return cfg->dim == 2 && cfg->smoother == MG_SMOOTH_RBJ && rb_passes(cfg) % 2 == 1;
}

// Device bytes of a handle: per-problem arrays times `slots`, plus the shared tables.
// own_top: the handle also holds level-0 FP64 f and u (batches copy requests in).
size_t footprint_of(const mg_config *cfg, int L, int slots = 1, bool own_top = false) {
  size_t per = 0;
  int n = cfg->n;
  const size_t es = cfg->precision == MG_PREC_MIXED ? 4 : 8;
  const bool mixed = cfg->precision == MG_PREC_MIXED;
  for (int l = 0; l < L; ++l) {
    const size_t np = points(cfg->dim, n);
    int arrays = (l > 0 || mixed) ? 2 : 0;  // u and f (level 0 FP64 uses the caller's)
    if (L > 1 && l < L - 1) arrays += needs_t2(cfg) ? 2 : 1;  // sweep targets
    per += arrays * np * es;
    if (l == 0 && own_top) per += 2 * np * 8;
    n = (n - 1) / 2 + 1;
  }
  per += (size_t)partials_needed(cfg->dim, cfg->n) * 8;
  per += sizeof(DevState);
  const int q = cfg->n_coarsest - 2;
  const size_t m = cfg->dim == 2 ? (size_t)q * q : (size_t)q * q * q;
  return per * (size_t)slots + m * m * 8 + ((size_t)q * q + m) * 8 + entries_bytes(cfg, L);
}

// Ghost width of a tail starting at level l: 1 if every tail level is the cross.
int tail_ghost(const mg_ctx *c, int l) {
  for (int k = l; k < c->L; ++k)
    if (!c->ops[k].cross) return 2;
  return 1;
}

int tail_entries(const mg_ctx *c, int l) {
  return c->ent_begin[c->L - 1] + c->ent_count[c->L - 1] - c->ent_begin[l];
}

// Dynamic LDS of a tail starting at level l.
size_t tail_bytes(const mg_ctx *c, int l, size_t es) {
  return mgk::tail_lds_bytes(c->dim, tail_ghost(c, l), &c->ns[l], c->L - l, tail_entries(c, l), es);
}

template <typename T>
hipError_t launch_tail_at(mg_ctx *c, int l, T *u, const T *f, bool zero_u, const int *done,
                          hipStream_t s, int repeats = 1) {
  if (c->tail3 && l == c->L - 2) {
    mgk::Tail3Args a{};
    a.nu1 = c->cfg.nu1;
    a.nu2 = c->cfg.nu2;
    a.prolong = c->cfg.prolong;
    a.zero_init = zero_u ? 1 : 0;
    a.repeats = repeats;
    a.rb = c->cfg.smoother == MG_SMOOTH_RBJ ? 1 : 0;
    a.om_d = c->omega / c->ops[l].diag;
    for (int k = 0; k < 7; ++k) {
      a.a[k] = c->ops[l].a[k];
      a.b[k] = c->ops[l].b[k];
    }
    a.dst = c->dst;
    a.f_top = f;
    a.u_top = u;
    a.done = done;
    return mgk::launch_tail3<T>(a, s, c->slots);
  }
  mgk::TailArgs a{};
  // a tail holding only the coarsest level solves it exactly: a repeated visit with the
  // same right-hand side gives the same values, so it runs once
  a.repeats = l == c->L - 1 ? 1 : repeats;
  a.levels = c->L - l;
  a.gamma = c->cfg.gamma;
  a.nu1 = c->cfg.nu1;
  a.nu2 = c->cfg.nu2;
  a.prolong = c->cfg.prolong;
  a.rb = c->cfg.smoother == MG_SMOOTH_RBJ ? 1 : 0;
  a.zero_init = zero_u ? 1 : 0;
  const int q = c->ns[c->L - 1] - 2;
  a.m = c->dim == 2 ? q * q : q * q * q;
  for (int k = l; k < c->L; ++k) {
    mgk::TailLevel &tl = a.lv[k - l];
    tl.n = c->ns[k];
    tl.ent_begin = c->ent_begin[k];
    tl.ent_count = c->ent_count[k];
    tl.cross = c->ops[k].cross ? 1 : 0;
    tl.om_d = c->omega / c->ops[k].diag;
    tl.w1 = -c->ops[k].a[2];
    tl.w2 = -c->ops[k].a[1];
  }
  const int G = tail_ghost(c, l);
  a.lds_r = (int)mgk::tail_scratch_offset(c->dim, G, &c->ns[l], c->L - l);
  a.lds_ent = (int)mgk::tail_entry_offset(c->dim, G, &c->ns[l], c->L - l, sizeof(T));
  a.eoff = c->eoff;
  a.ecoef = c->ecoef;
  a.ainv_t = c->ainv_t;
  a.dst = c->dst;
  a.f_top = f;
  a.u_top = u;
  a.done = done;
  a.ent_first = c->ent_begin[l];
  a.ent_total = tail_entries(c, l);
  return mgk::launch_tail<T>(c->dim, G, a, tail_bytes(c, l, sizeof(T)), s, c->slots);
}

template <typename T>
hipError_t cycle(mg_ctx *c, std::vector<Buffers> &B, int l, T *u, const T *f, bool zero_u,
                 bool check, hipStream_t s, double *corr = nullptr);

// fc = I_h^H (f - L_l u) on level l+1.  Full weighting: one fused pass, or on 3D separable
// levels the defect into scratch (a free level-l array) and then its restriction.  Cubic
// adjoint (appendix A.4): the defect into scratch, then the restriction.
template <typename T>
hipError_t resid_restrict(mg_ctx *c, int l, const T *f, const T *u, T *scratch, T *fc, const int *done,
                          hipStream_t s) {
  // 3D separable (Galerkin) levels: the pencil kernel's defect into scratch, then full
  // weighting of it by the cross kernel's zero-iterate form (C5 FP64 278.6 -> 272.8 ms,
  // mixed 431.3 -> 430.2 ms against the fused k_grr3d, which waits at its barriers);
  // MG_GRR_2PASS=0 keeps the fused kernel.
  const LevelOp &op = c->ops[l];
  const char *two = std::getenv("MG_GRR_2PASS");
  if (c->cfg.restrict_op != 3 && c->dim == 3 && !op.cross && !op.cross3 && u != nullptr &&
      !(two != nullptr && *two != 0 && std::atoi(two) == 0)) {
    hipError_t e = mgk::launch_sweep<T, T>(3, mgk::kResidual, op, c->omega, f, u, scratch, c->ns[l], nullptr,
                                           nullptr, done, s, c->slots);
    if (e != hipSuccess) return e;
    return mgk::launch_resid_restrict<T>(3, op, scratch, nullptr, fc, c->ns[l], done, s, c->slots);
  }
  if (c->cfg.restrict_op != 3)
    return mgk::launch_resid_restrict<T>(c->dim, c->ops[l], f, u, fc, c->ns[l], done, s, c->slots);
  hipError_t e = mgk::launch_sweep<T, T>(c->dim, mgk::kResidual, c->ops[l], c->omega, f, u, scratch, c->ns[l],
                                         nullptr, nullptr, done, s, c->slots);
  if (e != hipSuccess) return e;
  return mgk::launch_restrict_cubic<T>(c->dim, scratch, fc, c->ns[l], done, s, c->slots);
}

// Two omega-Jacobi sweeps of a 3D cross level in one pass: FP64 by default; MG_X2=0 or 1
// sets both precisions.
template <typename T>
bool x2_enabled() {
  const char *e = std::getenv("MG_X2");
  if (e != nullptr && *e != 0) return std::atoi(e) != 0;
  return sizeof(T) == 8;
}

// Two omega-Jacobi sweeps from a zero iterate in one 3D pass unless MG_Z2=0.
bool z2_enabled() {
  const char *e = std::getenv("MG_Z2");
  return !(e != nullptr && std::atoi(e) == 0);
}

// Cross levels of radius 2 or 3 (where Gauss-Seidel partial steps differ from Jacobi ones).
bool gs_level(const LevelOp &op) { return op.cross3 || (op.cross && op.a[1] != 0.0); }

// One partial step of the red-black smoother on level l, colour 1 (red) or 2 (black):
// Gauss-Seidel (section 3.1 eq. S_GS) on radius-2/3 cross levels with MG_SMOOTH_RBGS, else
// the Jacobi partial step (for the five-point operator the two coincide).  partials: the
// defect norm partials of u_in (Jacobi steps only), or null.
template <typename T>
hipError_t partial_step(mg_ctx *c, int l, int colour, const T *f, const T *uin, T *uout, double *partials,
                        int *np, hipStream_t s) {
  const LevelOp &op = c->ops[l];
  if (c->cfg.smoother == MG_SMOOTH_RBGS && gs_level(op)) {
    if (uin == nullptr || partials != nullptr) return hipErrorInvalidValue;
    return mgk::launch_gs2d<T>(op, c->omega, colour, f, uin, uout, c->ns[l], &c->st->done, s, c->slots);
  }
  return mgk::launch_sweep<T, T>(c->dim, mgk::kSweep, op, c->omega, f, uin, uout, c->ns[l], partials, np,
                                 &c->st->done, s, c->slots, colour);
}

// The fused 2D cycle on level l with red-black smoothing (rb_passes): every pass is one
// pre or post kernel whose stages alternate red and black partial steps.
template <typename T>
hipError_t cycle_rb2d(mg_ctx *c, std::vector<Buffers> &B, int l, T *u, const T *f, bool zero_u,
                      bool check, hipStream_t s) {
  const int *done = &c->st->done;
  const int n = c->ns[l];
  const LevelOp &op = c->ops[l];
  T *t = (T *)B[l].t, *t2 = (T *)B[l].t2;
  T *uc = (T *)B[l + 1].u;
  T *fc = (T *)B[l + 1].f;
  const int pre = std::max(1, c->cfg.nu1), total = rb_passes(&c->cfg);
  int k = 0;  // passes done
  const T *in = zero_u ? nullptr : u;
  // pass k writes u when total - 1 - k is even, else t; a first pass that would write its
  // own input u writes t2 instead
  auto target = [&](int kk) -> T * {
    T *o = ((total - 1 - kk) % 2 == 0) ? u : t;
    return (o == in) ? t2 : o;
  };
  hipError_t e;
  for (; k < pre; ++k) {
    const bool last = k == pre - 1;
    const int stages = c->cfg.nu1 == 0 ? 0 : 2;
    T *o = target(k);
    if (o == nullptr) return hipErrorInvalidValue;
    int np = 0;
    e = mgk::launch_pre2d<T>(op, c->omega, stages, last ? (mgk::kPreWriteU | mgk::kPreRestrict) : mgk::kPreWriteU,
                             f, in, o, nullptr, last ? fc : nullptr, n,
                             check && k == 0 ? c->partials : nullptr, &np, done, s, c->slots, true);
    if (e != hipSuccess) return e;
    if (check && k == 0) {
      e = mgk::launch_check(c->st, c->partials, np, 1, s, c->slots);
      if (e != hipSuccess) return e;
    }
    in = o;
  }
  if (l + 1 >= c->tail_top) {
    e = launch_tail_at<T>(c, l + 1, uc, fc, true, done, s, c->cfg.gamma);
  } else if (l + 1 == c->L - 1) {
    e = mgk::launch_coarsest<T>(c->dim, c->ainv_t, fc, uc, c->ns[l + 1], done, s, c->slots);
  } else {
    e = hipSuccess;
    for (int g = 0; g < c->cfg.gamma && e == hipSuccess; ++g)
      e = cycle<T>(c, B, l + 1, uc, fc, g == 0, false, s);
  }
  if (e != hipSuccess) return e;
  for (int j = 0; k < total; ++k, ++j) {
    T *o = target(k);
    if (o == nullptr || o == in) return hipErrorInvalidValue;
    if (j == 0)
      e = mgk::launch_post2d<T>(op, c->omega, c->cfg.nu2 == 0 ? 0 : 2, c->cfg.prolong, uc, in, f, o, n,
                                done, s, c->slots, true);
    else
      e = mgk::launch_pre2d<T>(op, c->omega, 2, mgk::kPreWriteU, f, in, o, nullptr, nullptr, n, nullptr,
                               nullptr, done, s, c->slots, true);
    if (e != hipSuccess) return e;
    in = o;
  }
  return in == u ? hipSuccess : hipErrorInvalidValue;
}

// Whether the last FP32 cycle of a refinement step ends in the fused sweep + correction
// (3D cross level 0 run by the streaming kernels with omega-Jacobi sweeps, one sweep per
// pass after the interpolation); MG_FUSE_CORR=0 keeps the separate correction.
bool fuse_corr(const mg_ctx *c) {
  const char *e = std::getenv("MG_FUSE_CORR");
  const bool on = !(e != nullptr && std::atoi(e) == 0);
  const LevelOp &op = c->ops[0];
  return on && c->cfg.precision == MG_PREC_MIXED && c->dim == 3 && c->L > 1 && c->tail_top > 0 &&
         op.cross && !op.cross3 && c->cfg.smoother == MG_SMOOTH_JACOBI && c->cfg.nu2 >= 1 &&
         !x2_enabled<float>() && c->slots == 1;
}

template <typename T>
hipError_t cycle(mg_ctx *c, std::vector<Buffers> &B, int l, T *u, const T *f, bool zero_u,
                 bool check, hipStream_t s, double *corr) {
  const int *done = &c->st->done;
  const int dim = c->dim;
  const int n = c->ns[l];
  const LevelOp &op = c->ops[l];
  hipError_t e;
  if (l >= c->tail_top) {
    if (check) {
      int np = 0;
      e = mgk::launch_sweep<T, T>(dim, mgk::kNormOnly, op, c->omega, f, zero_u ? nullptr : u,
                                  (T *)nullptr, n, c->partials, &np, done, s, c->slots);
      if (e != hipSuccess) return e;
      e = mgk::launch_check(c->st, c->partials, np, 1, s, c->slots);
      if (e != hipSuccess) return e;
    }
    return launch_tail_at<T>(c, l, u, f, zero_u, done, s);
  }
  if (c->fused && dim == 2 && c->L > 1 && c->cfg.smoother == MG_SMOOTH_RBJ)
    return cycle_rb2d<T>(c, B, l, u, f, zero_u, check, s);
  if (c->fused && dim == 2 && c->L > 1) {
    T *t = (T *)B[l].t;
    T *uc = (T *)B[l + 1].u;
    T *fc = (T *)B[l + 1].f;
    int np = 0;
    e = mgk::launch_pre2d<T>(op, c->omega, c->cfg.nu1, mgk::kPreWriteU | mgk::kPreRestrict, f,
                             zero_u ? nullptr : u, t, nullptr, fc, n,
                             check ? c->partials : nullptr, &np, done, s, c->slots);
    if (e != hipSuccess) return e;
    if (check) {
      e = mgk::launch_check(c->st, c->partials, np, 1, s, c->slots);
      if (e != hipSuccess) return e;
    }
    if (l + 1 >= c->tail_top) {
      // the gamma visits of the tail's top level in one launch
      e = launch_tail_at<T>(c, l + 1, uc, fc, true, done, s, c->cfg.gamma);
      if (e != hipSuccess) return e;
    } else if (l + 1 == c->L - 1) {
      e = mgk::launch_coarsest<T>(dim, c->ainv_t, fc, uc, c->ns[l + 1], done, s, c->slots);
      if (e != hipSuccess) return e;
    } else {
      for (int g = 0; g < c->cfg.gamma; ++g) {
        e = cycle<T>(c, B, l + 1, uc, fc, g == 0, false, s);
        if (e != hipSuccess) return e;
      }
    }
    return mgk::launch_post2d<T>(op, c->omega, c->cfg.nu2, c->cfg.prolong, uc, t, f, u, n, done, s, c->slots);
  }
  if (c->L == 1) {  // a single level: the exact solve is the whole cycle
    if (check) {
      int np = 0;
      e = mgk::launch_sweep<T, T>(dim, mgk::kNormOnly, op, c->omega, f, zero_u ? nullptr : u,
                                  (T *)nullptr, n, c->partials, &np, done, s, c->slots);
      if (e != hipSuccess) return e;
      e = mgk::launch_check(c->st, c->partials, np, 1, s, c->slots);
      if (e != hipSuccess) return e;
    }
    return mgk::launch_coarsest<T>(dim, c->ainv_t, f, u, n, done, s, c->slots);
  }
  T *t = (T *)B[l].t;
  T *cur = u, *other = t;
  bool zero = zero_u;
  if (check && c->cfg.nu1 == 0) {
    int np = 0;
    e = mgk::launch_sweep<T, T>(dim, mgk::kNormOnly, op, c->omega, f, zero ? nullptr : u,
                                (T *)nullptr, n, c->partials, &np, done, s, c->slots);
    if (e != hipSuccess) return e;
    e = mgk::launch_check(c->st, c->partials, np, 1, s, c->slots);
    if (e != hipSuccess) return e;
  }
  if (zero && c->cfg.nu1 == 0) {
    e = mgk::launch_fill<T>(u, points(dim, n), T(0), done, s, c->slots);
    if (e != hipSuccess) return e;
    zero = false;
  }
  // a red-black sweep is two steps: the red points (colour 1), then the black ones (2);
  // on 3D cross levels one launch does both
  const bool rb = c->cfg.smoother == MG_SMOOTH_RBJ || c->cfg.smoother == MG_SMOOTH_RBGS;
  const bool rb3 = c->cfg.smoother == MG_SMOOTH_RBJ && dim == 3 && op.cross && sizeof(T) == 8 && rb3_fused();
  const int steps = rb && !rb3 ? 2 : 1;
  // Gauss-Seidel steps do not form the defect norm: the stopping check gets its own pass
  const bool gs_check = check && c->cfg.smoother == MG_SMOOTH_RBGS && gs_level(op) && c->cfg.nu1 > 0;
  if (gs_check) {
    int np = 0;
    e = mgk::launch_sweep<T, T>(dim, mgk::kNormOnly, op, c->omega, f, zero ? nullptr : u, (T *)nullptr, n,
                                c->partials, &np, done, s, c->slots);
    if (e != hipSuccess) return e;
    e = mgk::launch_check(c->st, c->partials, np, 1, s, c->slots);
    if (e != hipSuccess) return e;
  }
  if (zero && c->cfg.smoother == MG_SMOOTH_RBGS && gs_level(op) && c->cfg.nu1 > 0) {
    // a Gauss-Seidel step reads the new values it has just written: start from stored zeros
    e = mgk::launch_fill<T>(cur, points(dim, n), T(0), done, s, c->slots);
    if (e != hipSuccess) return e;
    zero = false;
  }
  int k0 = 0;
  if (zero && !rb && !rb3 && !check && dim == 3 && c->cfg.nu1 >= 2 && z2_enabled() && mgk::sweep3d_z2_ok(op)) {
    // the first two sweeps from the zero iterate in one pass, into the array the second
    // sweep would have written (the ping-pong order of the sweeps that follow is kept)
    e = mgk::launch_sweep<T, T>(dim, mgk::kSweepZ2, op, c->omega, f, (const T *)nullptr, cur, n, nullptr,
                                nullptr, done, s, c->slots, 0);
    if (e != hipSuccess) return e;
    zero = false;
    k0 = 2;
  }
  // two omega-Jacobi sweeps of a 3D cross level in one pass where two remain (FP64: 1025^3
  // 10.8 ms against two sweeps of 6.27; in FP32 the pass takes 7.74 ms against 2 x 3.58)
  const bool x2 = !rb && !rb3 && dim == 3 && op.cross && x2_enabled<T>();
  for (int k = k0; k < c->cfg.nu1 * steps; ++k) {
    const bool first_check = check && k == 0 && !gs_check;
    int np = 0;
    if (x2 && c->cfg.nu1 * steps - k >= 2) {
      e = mgk::launch_x2sweep_3d<T>(op, c->omega, f, zero ? nullptr : cur, other, n,
                                    first_check ? c->partials : nullptr, &np, done, s);
      ++k;  // the pass took two sweeps
    } else if (rb3)
      e = mgk::launch_rbsweep_3d<T>(op, c->omega, f, zero ? nullptr : cur, other, n,
                                    first_check ? c->partials : nullptr, &np, done, s);
    else if (rb)
      e = partial_step<T>(c, l, 1 + k % 2, f, zero ? nullptr : cur, other, first_check ? c->partials : nullptr,
                          &np, s);
    else
      e = mgk::launch_sweep<T, T>(dim, mgk::kSweep, op, c->omega, f, zero ? nullptr : cur, other, n,
                                  first_check ? c->partials : nullptr, &np, done, s, c->slots, 0);
    if (e != hipSuccess) return e;
    if (first_check) {
      e = mgk::launch_check(c->st, c->partials, np, 1, s, c->slots);
      if (e != hipSuccess) return e;
    }
    zero = false;
    std::swap(cur, other);
  }
  T *uc = (T *)B[l + 1].u;
  T *fc = (T *)B[l + 1].f;
  e = resid_restrict<T>(c, l, f, cur, other, fc, done, s);
  if (e != hipSuccess) return e;
  if (l + 1 == c->L - 1 && l + 1 < c->tail_top) {
    e = mgk::launch_coarsest<T>(dim, c->ainv_t, fc, uc, c->ns[l + 1], done, s, c->slots);
    if (e != hipSuccess) return e;
  } else if (l + 1 >= c->tail_top) {
    // the gamma visits of the tail's top level in one launch
    e = launch_tail_at<T>(c, l + 1, uc, fc, true, done, s, c->cfg.gamma);
    if (e != hipSuccess) return e;
  } else {
    for (int g = 0; g < c->cfg.gamma; ++g) {
      e = cycle<T>(c, B, l + 1, uc, fc, g == 0, false, s);
      if (e != hipSuccess) return e;
    }
  }
  // the passes of the post-smoothing alternate between t and u and end in u
  const int npost = c->cfg.nu2 * steps, passes = x2 ? npost / 2 + npost % 2 : npost;
  T *dst = (passes % 2 == 0) ? u : t;
  e = mgk::launch_prolong_correct<T>(dim, c->cfg.prolong, uc, cur, dst, n, done, s, c->slots);
  if (e != hipSuccess) return e;
  cur = dst;
  other = (dst == u) ? t : u;
  for (int k = 0; k < npost; ++k) {
    if (x2 && npost - k >= 2) {
      e = mgk::launch_x2sweep_3d<T>(op, c->omega, f, cur, other, n, nullptr, nullptr, done, s);
      ++k;
    } else if (corr != nullptr && k == npost - 1) {
      // the last sweep of the step's last cycle adds its result to the FP64 iterate
      if constexpr (std::is_same<T, float>::value)
        e = mgk::launch_sweep_corr_3d(op, c->omega, f, cur, corr, n, done, s);
      else
        e = hipErrorInvalidValue;
    } else if (rb3)
      e = mgk::launch_rbsweep_3d<T>(op, c->omega, f, cur, other, n, nullptr, nullptr, done, s);
    else if (rb)
      e = partial_step<T>(c, l, 1 + k % 2, f, cur, other, nullptr, nullptr, s);
    else
      e = mgk::launch_sweep<T, T>(dim, mgk::kSweep, op, c->omega, f, cur, other, n, nullptr, nullptr,
                                  done, s, c->slots, 0);
    if (e != hipSuccess) return e;
    std::swap(cur, other);
  }
  return hipSuccess;
}

// One solve step on stream s: an FP64 cycle, or a mixed-precision refinement step.
hipError_t record_step(mg_ctx *c, const double *f, double *u, hipStream_t s) {
  if (c->cfg.precision == MG_PREC_FP64) return cycle<double>(c, c->b64, 0, u, f, false, true, s);
  const int *done = &c->st->done;
  int np = 0;
  float *r32 = (float *)c->b32[0].f;
  float *e32 = (float *)c->b32[0].u;
  hipError_t e = mgk::launch_sweep<double, float>(c->dim, mgk::kResidual, c->ops[0], c->omega, f, u,
                                                  r32, c->ns[0], c->partials, &np, done, s, c->slots);
  if (e != hipSuccess) return e;
  e = mgk::launch_check(c->st, c->partials, np, 1, s, c->slots);
  if (e != hipSuccess) return e;
  const bool fuse = fuse_corr(c);
  for (int i = 0; i < c->cfg.inner_cycles; ++i) {
    const bool last = i == c->cfg.inner_cycles - 1;
    e = cycle<float>(c, c->b32, 0, e32, r32, i == 0, false, s, fuse && last ? u : nullptr);
    if (e != hipSuccess) return e;
  }
  if (fuse) return hipSuccess;  // the last sweep added e to u
  return mgk::launch_ir_correct(c->dim, u, e32, c->ns[0], done, s, c->slots);
}

mg_status ensure_graph(mg_ctx *c, const double *f, double *u) {
  if (!c->use_graph) return MG_OK;
  if (c->gexec && c->gf == f && c->gu == u) return MG_OK;
  if (c->gexec) {
    MG_HIP(hipGraphExecDestroy(c->gexec));
    c->gexec = nullptr;
  }
  if (c->graph) {
    MG_HIP(hipGraphDestroy(c->graph));
    c->graph = nullptr;
  }
  MG_HIP(hipStreamBeginCapture(c->cap, hipStreamCaptureModeThreadLocal));
  hipError_t e = record_step(c, f, u, c->cap);
  hipGraph_t g = nullptr;
  hipError_t e2 = hipStreamEndCapture(c->cap, &g);
  if (e != hipSuccess) {
    if (g) (void)hipGraphDestroy(g);
    return fail(MG_EDEVICE, std::string("kernel launch during capture: ") + hipGetErrorString(e));
  }
  if (e2 != hipSuccess) return fail(MG_EDEVICE, std::string("hipStreamEndCapture: ") + hipGetErrorString(e2));
  c->graph = g;
  MG_HIP(hipGraphInstantiate(&c->gexec, c->graph, nullptr, nullptr, 0));
  c->gf = f;
  c->gu = u;
  return MG_OK;
}

mg_status launch_step(mg_ctx *c, const double *f, double *u) {
  if (c->use_graph) {
    MG_HIP(hipGraphLaunch(c->gexec, c->stream));
  } else {
    MG_HIP(record_step(c, f, u, c->stream));
  }
  return MG_OK;
}

mg_status begin_solve(mg_ctx *c, const double *f, double *u, double rtol, int max_steps,
                      int floor_detect) {
  if (!f || !u) return fail(MG_EINVAL, "null f or u");
  if (c->async_pending) return fail(MG_EBUSY, "an asynchronous solve is still pending");
  MG_HIP(hipSetDevice(c->device));
  mg_status st = ensure_graph(c, f, u);
  if (st != MG_OK) return st;
  hipLaunchKernelGGL(k_state_init, dim3(1), dim3(64), 0, c->stream, c->st, rtol, max_steps + 1,
                     floor_detect);
  MG_HIP(hipGetLastError());
  int np = 0;
  MG_HIP((mgk::launch_sweep<double, double>(c->dim, mgk::kNormOnly, c->ops[0], c->omega, f,
                                            nullptr, (double *)nullptr, c->ns[0], c->partials,
                                            &np, nullptr, c->stream)));
  MG_HIP(mgk::launch_check(c->st, c->partials, np, 0, c->stream));
  return MG_OK;
}

void result_from_state(const mg_ctx *c, const DevState &hs, mg_result *res, mg_status *outcome) {
  const int checks = std::min(hs.checks, mgk::kMaxHistory);
  const double final_rel = checks > 0 ? hs.hist[checks - 1] : 0.0;
  if (res) {
    std::memset(res, 0, sizeof(*res));
    const int steps = std::max(0, hs.checks - 1);
    if (c->cfg.precision == MG_PREC_MIXED) {
      res->outer_steps = steps;
      res->cycles = steps * c->cfg.inner_cycles;
    } else {
      res->cycles = steps;
    }
    res->status = hs.status;
    res->floor_hit = hs.status == 3;
    res->rel_residual = final_rel;
    res->conv_factor = hs.last_ratio;
    res->history_len = checks;
    for (int i = 0; i < checks; ++i) res->history[i] = hs.hist[i];
  }
  switch (hs.status) {
    case 1: *outcome = MG_OK; break;
    case 4: *outcome = MG_ENUMERIC; break;
    // 2 cycle cap, 3 rounding floor above rtol (floor_hit), 5 growth: rtol not reached

    default: *outcome = MG_ENOCONV; break;
  }
}

mg_status fill_result(mg_ctx *c, mg_result *res, mg_status *outcome) {
  DevState hs;
  MG_HIP(hipMemcpyAsync(&hs, c->st, sizeof(DevState), hipMemcpyDeviceToHost, c->stream));
  MG_HIP(hipStreamSynchronize(c->stream));
  result_from_state(c, hs, res, outcome);
  return MG_OK;
}

// Replay policy.  Steps are replayed in chunks, and the host reads the stopping flag of
// chunk k-1 while chunk k runs, so the device never waits for the host.  Every step
// replayed after convergence still launches its kernels, which return at once (a few
// microseconds each: a W-cycle on eight levels is some two thousand launches).  So the
// chunk is sized from the measured step time to about kChunkSeconds, and steps longer
// than kSyncStepSeconds are run one at a time with no lookahead: the host turnaround
// (tens of microseconds) then costs less than one replay past convergence.
constexpr double kChunkSeconds = 3e-4, kSyncStepSeconds = 2e-3;

double wall_seconds() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

mg_status run(mg_ctx *c, const double *f, double *u, double rtol, int max_steps, int floor_detect,
              mg_result *res) {
  mg_status st = begin_solve(c, f, u, rtol, max_steps, floor_detect);
  if (st != MG_OK) return st;
  const int total = max_steps + 1;
  int launched = 0, k = 0, chunk = c->chunk > 0 ? c->chunk : 1, prev_cnt = 0;
  bool lookahead = true;
  double t_prev = wall_seconds();
  while (launched < total) {
    const int cnt = std::min(chunk, total - launched);
    for (int i = 0; i < cnt; ++i) {
      st = launch_step(c, f, u);
      if (st != MG_OK) return st;
    }
    launched += cnt;
    MG_HIP(hipMemcpyAsync(&c->poll[2 * (k & 1)], &c->st->done, 2 * sizeof(int),
                          hipMemcpyDeviceToHost, c->stream));
    MG_HIP(hipEventRecord(c->ev[k & 1], c->stream));
    if (!lookahead) {  // wait for this chunk (one step) at once
      MG_HIP(hipEventSynchronize(c->ev[k & 1]));
      if (c->poll[2 * (k & 1)] != 0) break;
    } else if (k > 0) {
      MG_HIP(hipEventSynchronize(c->ev[(k - 1) & 1]));
      if (c->poll[2 * ((k - 1) & 1)] != 0) break;
      // chunk k-1 ran from the end of chunk k-2 (or the start) to now
      const double t = wall_seconds(), step_s = (t - t_prev) / std::max(prev_cnt, 1);
      t_prev = t;
      if (c->chunk == 0) {
        if (step_s > kSyncStepSeconds) {
          lookahead = false;
          chunk = 1;
        } else {
          chunk = std::min(8, std::max(1, (int)std::ceil(kChunkSeconds / step_s)));
        }
      }
    }
    prev_cnt = cnt;
    ++k;
  }
  mg_status outcome = MG_OK;
  st = fill_result(c, res, &outcome);
  if (st != MG_OK) return st;
  if (outcome == MG_ENOCONV && rtol < 0.0) outcome = MG_OK;  // fixed cycle count requested
  if (outcome != MG_OK)
    g_error = res && res->floor_hit ? "solve stopped at the rounding floor above rtol"
                                    : "solve did not reach rtol";
  return outcome;
}

template <typename T>
mg_status check_level(mg_ctx *c, int level, bool needs_coarse) {
  if (!c) return fail(MG_EINVAL, "null handle");
  if (level < 0 || level >= c->L || (needs_coarse && level >= c->L - 1))
    return fail(MG_EINVAL, "level out of range");
  MG_HIP(hipSetDevice(c->device));
  return MG_OK;
}

}  // namespace

extern "C" {

const char *mg_last_error(void) { return g_error.c_str(); }

size_t mg_footprint_bytes(const mg_config *cfg) {
  int L = 0;
  if (validate(cfg, &L) != MG_OK) return 0;
  return footprint_of(cfg, L);
}

mg_status mg_destroy(mg_handle h) {
  if (!h) return MG_OK;
  (void)hipSetDevice(h->device);
  if (h->stream) (void)hipStreamSynchronize(h->stream);
  if (h->gexec) (void)hipGraphExecDestroy(h->gexec);
  if (h->graph) (void)hipGraphDestroy(h->graph);
  for (void *p : h->allocs) (void)hipFree(p);
  if (h->poll) (void)hipHostFree(h->poll);
  for (auto &e : h->ev)
    if (e) (void)hipEventDestroy(e);
  if (h->ev_async) (void)hipEventDestroy(h->ev_async);
  if (h->cap) (void)hipStreamDestroy(h->cap);
  delete h;
  return MG_OK;
}

namespace {

// Builds a handle for `slots` independent problems of the configured size.
mg_status setup_ctx(const mg_config *cfg, void *hip_stream, int slots, bool own_top, mg_ctx **out) {
  *out = nullptr;
  int L = 0;
  mg_status st = validate(cfg, &L);
  if (st != MG_OK) return st;
  if (slots < 1 || (slots > 1 && cfg->dim != 2)) return fail(MG_EINVAL, "batches are 2D only");
  mg_ctx *c = new mg_ctx();
  c->cfg = *cfg;
  c->slots = slots;
  c->own_top = own_top;
  c->dim = cfg->dim;
  c->L = L;
  c->omega = cfg->omega > 0.0 ? cfg->omega : default_omega(cfg->dim, cfg->order, cfg->smoother, cfg->coarse);
  c->stream = (hipStream_t)hip_stream;
  if (const char *g = std::getenv("MG_GRAPH")) c->use_graph = std::atoi(g) != 0;
  if (const char *k = std::getenv("MG_CHUNK")) c->chunk = std::max(1, std::atoi(k));
  if (const char *fz = std::getenv("MG_FUSED")) c->fused = std::atoi(fz) != 0;
  if (cfg->smoother == MG_SMOOTH_JACOBI && (cfg->nu1 > 3 || cfg->nu2 > 2)) c->fused = false;
  // Gauss-Seidel partial steps and the cubic-adjoint restriction run as their own kernels on
  // every level (no fused passes, no LDS-resident tail)
  if (cfg->smoother == MG_SMOOTH_RBGS || cfg->restrict_op == 3) c->fused = false;
  auto bail = [&](mg_status s) {
    std::string msg = g_error;
    mg_destroy(c);
    g_error = msg;
    return s;
  };
  if (hipGetDevice(&c->device) != hipSuccess) return bail(fail(MG_EDEVICE, "no HIP device"));
  int n = cfg->n;
  for (int l = 0; l < L; ++l) {
    c->ns.push_back(n);
    const double h = 1.0 / (n - 1);
    if (l == 0 || cfg->coarse == MG_COARSE_NG)
      c->ops.push_back(rediscretized_op(cfg->order, cfg->dim, h));
    else if (cfg->coarse == MG_COARSE_NG2)
      c->ops.push_back(rediscretized_op(2, cfg->dim, h));
    else if (cfg->coarse == MG_COARSE_G2 && l == 1)  // R L_h^(2) P, second order at the finest spacing
      c->ops.push_back(galerkin(rediscretized_op(2, cfg->dim, 1.0 / (cfg->n - 1)), cfg->dim, cfg->prolong));
    else
      c->ops.push_back(galerkin(c->ops[l - 1], cfg->dim, cfg->prolong));
    n = (n - 1) / 2 + 1;
  }
  std::vector<double> inv;
  if (!coarsest_inverse(c->ops[L - 1], c->dim, c->ns[L - 1], inv))
    return bail(fail(MG_EINVAL, "coarsest operator is singular"));
  if ((st = dev_alloc(c, (void **)&c->ainv_t, inv.size() * sizeof(double))) != MG_OK) return bail(st);
  const bool mixed = cfg->precision == MG_PREC_MIXED;
  c->b64.resize(L);
  c->b32.resize(L);
  for (int l = 0; l < L; ++l) {
    const size_t np = points(c->dim, c->ns[l]) * (size_t)slots;
    if (l == 0 && own_top) {
      Buffers &b = c->b64[0];
      if ((st = dev_alloc(c, &b.u, np * 8)) != MG_OK) return bail(st);
      if ((st = dev_alloc(c, &b.f, np * 8)) != MG_OK) return bail(st);
    }
    if (!mixed) {
      Buffers &b = c->b64[l];
      if (l > 0) {
        if ((st = dev_alloc(c, &b.u, np * 8)) != MG_OK) return bail(st);
        if ((st = dev_alloc(c, &b.f, np * 8)) != MG_OK) return bail(st);
      }
      if (L > 1 && l < L - 1) {
        if ((st = dev_alloc(c, &b.t, np * 8)) != MG_OK) return bail(st);
        if (needs_t2(cfg) && (st = dev_alloc(c, &b.t2, np * 8)) != MG_OK) return bail(st);
      }
    } else {
      Buffers &b = c->b32[l];
      if ((st = dev_alloc(c, &b.u, np * 4)) != MG_OK) return bail(st);
      if ((st = dev_alloc(c, &b.f, np * 4)) != MG_OK) return bail(st);
      if (L > 1 && l < L - 1) {
        if ((st = dev_alloc(c, &b.t, np * 4)) != MG_OK) return bail(st);
        if (needs_t2(cfg) && (st = dev_alloc(c, &b.t2, np * 4)) != MG_OK) return bail(st);
      }
    }
  }
  // Stencil entry lists (non-centre, non-zero) of every level, for the tail kernel.
  {
    std::vector<int> off;
    std::vector<double> coef;
    for (int l = 0; l < L; ++l) {
      const LevelOp &op = c->ops[l];
      c->ent_begin.push_back((int)coef.size());
      const int zr = c->dim == 3 ? 3 : 0;
      for (int oz = -zr; oz <= zr; ++oz)
        for (int oy = -3; oy <= 3; ++oy)
          for (int ox = -3; ox <= 3; ++ox) {
            if (ox == 0 && oy == 0 && oz == 0) continue;
            double v = op.a[ox + 3] * op.b[oy + 3] + op.b[ox + 3] * op.a[oy + 3];
            if (c->dim == 3)
              v = (op.a[ox + 3] * op.b[oy + 3] + op.b[ox + 3] * op.a[oy + 3]) * op.b[oz + 3] +
                  op.b[ox + 3] * op.b[oy + 3] * op.a[oz + 3];
            if (v == 0.0) continue;
            off.push_back(ox);
            off.push_back(oy);
            off.push_back(oz);
            coef.push_back(v);
          }
      c->ent_count.push_back((int)coef.size() - c->ent_begin[l]);
    }
    if ((st = dev_alloc(c, (void **)&c->eoff, off.size() * sizeof(int))) != MG_OK) return bail(st);
    if ((st = dev_alloc(c, (void **)&c->ecoef, coef.size() * sizeof(double))) != MG_OK) return bail(st);
    if (hipMemcpy(c->eoff, off.data(), off.size() * sizeof(int), hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(c->ecoef, coef.data(), coef.size() * sizeof(double), hipMemcpyHostToDevice) != hipSuccess)
      return bail(fail(MG_EDEVICE, "upload of the stencil entries failed"));
  }
  // The coarse end of the hierarchy runs in one LDS-resident workgroup when it fits.
  {
    int lds_limit = 0;
    if (hipDeviceGetAttribute(&lds_limit, hipDeviceAttributeMaxSharedMemoryPerBlock, c->device) != hipSuccess)
      lds_limit = 65536;
    // Largest level side in the tail, by measurement: in 3D one workgroup's pass over a
    // 17^3 level costs more than the streaming kernels' launches, so only the coarsest
    // solve runs there; in 2D the tail takes the levels up to 33^2.
    int cap = c->dim == 2 ? 33 : 9;
    if (const char *tn = std::getenv("MG_TAIL_N")) cap = std::atoi(tn);
    if (cfg->smoother == MG_SMOOTH_RBGS || cfg->restrict_op == 3) cap = 0;
    const size_t es = mixed ? sizeof(float) : sizeof(double);
    c->tail_top = L;
    for (int l = L - 1; l >= 0 && L - l <= mgk::kMaxTailLevels; --l) {
      const size_t np = points(c->dim, c->ns[l]);
      const size_t need = tail_bytes(c, l, es);
      if (c->ns[l] > cap || c->ns[l] > mgk::tail_max_side(c->dim) || need > (size_t)lds_limit) break;
      (void)np;
      c->tail_top = l;
      c->tail_lds = need;
    }
    if (c->tail_top < L) {
      const int G = tail_ghost(c, c->tail_top);
      hipError_t e = mixed ? mgk::tail_prepare<float>(c->dim, G, c->tail_lds)
                           : mgk::tail_prepare<double>(c->dim, G, c->tail_lds);
      if (e != hipSuccess) return bail(fail(MG_EDEVICE, std::string("tail setup: ") + hipGetErrorString(e)));
    }
  }
  if (c->dim == 3) {
    hipError_t e = mgk::prepare_3d();
    if (e != hipSuccess) return bail(fail(MG_EDEVICE, std::string("3D kernel setup: ") + hipGetErrorString(e)));
  }
  c->np_max = partials_needed(c->dim, cfg->n);
  if ((st = dev_alloc(c, (void **)&c->partials, (size_t)c->np_max * 8 * slots)) != MG_OK) return bail(st);
  if ((st = dev_alloc(c, (void **)&c->st, sizeof(DevState) * slots)) != MG_OK) return bail(st);
  if (hipMemcpy(c->ainv_t, inv.data(), inv.size() * sizeof(double), hipMemcpyHostToDevice) != hipSuccess)
    return bail(fail(MG_EDEVICE, "upload of the coarsest inverse failed"));
  {
    // the tail solves the coarsest level by sine transforms unless MG_COARSE_DST=0 (or
    // the operator fails the eigenpair check): no matrix to stream per visit
    const char *e = std::getenv("MG_COARSE_DST");
    const int q = c->ns[L - 1] - 2;
    const size_t tab_len = (size_t)q * q + (c->dim == 2 ? (size_t)q * q : (size_t)q * q * q);
    double *table = nullptr;  // allocated in any case, so that the footprint is exact
    if ((st = dev_alloc(c, (void **)&table, tab_len * sizeof(double))) != MG_OK) return bail(st);
    std::vector<double> tab;
    if (!(e != nullptr && std::atoi(e) == 0) && coarsest_dst(c->ops[L - 1], c->dim, c->ns[L - 1], tab)) {
      if (hipMemcpy(table, tab.data(), tab_len * sizeof(double), hipMemcpyHostToDevice) != hipSuccess)
        return bail(fail(MG_EDEVICE, "upload of the coarsest sine table failed"));
      c->dst = table;
    }
  }
  {
    // 3D: the levels 17^3 and 9^3 in one workgroup of line passes (tail3d.hip) when the
    // coarsest solve has its sine table and the LDS holds both levels; MG_TAIL3=0, or an
    // explicit MG_TAIL_N, keeps the general tail
    const char *e3 = std::getenv("MG_TAIL3");
    const bool want = !(e3 != nullptr && std::atoi(e3) == 0) && std::getenv("MG_TAIL_N") == nullptr;
    int lds_limit = 0;
    if (hipDeviceGetAttribute(&lds_limit, hipDeviceAttributeMaxSharedMemoryPerBlock, c->device) != hipSuccess)
      lds_limit = 65536;
    const size_t need = mgk::tail3_lds_bytes(mixed ? sizeof(float) : sizeof(double));
    if (want && c->dim == 3 && L >= 2 && c->ns[L - 2] == mgk::kTail3Side && c->ns[L - 1] == mgk::kTail3Coarse &&
        c->dst != nullptr && cfg->smoother != MG_SMOOTH_RBGS && cfg->restrict_op == 1 &&
        need <= (size_t)lds_limit) {
      hipError_t e = mixed ? mgk::tail3_prepare<float>() : mgk::tail3_prepare<double>();
      if (e != hipSuccess) return bail(fail(MG_EDEVICE, std::string("tail setup: ") + hipGetErrorString(e)));
      c->tail3 = true;
      c->tail_top = L - 2;
    }
  }
  {
    // slots of a batch start parked (done = 1) until a problem is admitted
    std::vector<DevState> init(slots);
    std::memset(init.data(), 0, sizeof(DevState) * slots);
    if (slots > 1)
      for (auto &d : init) d.done = 1;
    if (hipMemcpy(c->st, init.data(), sizeof(DevState) * slots, hipMemcpyHostToDevice) != hipSuccess)
      return bail(fail(MG_EDEVICE, "upload of the solve state failed"));
  }
  if (hipHostMalloc((void **)&c->poll, 4 * sizeof(int), hipHostMallocDefault) != hipSuccess)
    return bail(fail(MG_ENOMEM, "pinned host allocation failed"));
  if (hipStreamCreateWithFlags(&c->cap, hipStreamNonBlocking) != hipSuccess)
    return bail(fail(MG_EDEVICE, "stream creation failed"));
  for (auto &e : c->ev)
    if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess)
      return bail(fail(MG_EDEVICE, "event creation failed"));
  if (hipEventCreateWithFlags(&c->ev_async, hipEventDisableTiming) != hipSuccess)
    return bail(fail(MG_EDEVICE, "event creation failed"));
  *out = c;
  return MG_OK;
}

}  // namespace

mg_status mg_setup(const mg_config *cfg, void *hip_stream, mg_handle *out) {
  if (!out) return fail(MG_EINVAL, "null output handle");
  return setup_ctx(cfg, hip_stream, 1, false, out);
}

mg_status mg_solve(mg_handle h, const double *f, double *u, mg_result *res) {
  if (!h) return fail(MG_EINVAL, "null handle");
  return run(h, f, u, h->cfg.rtol, h->cfg.max_cycles, 1, res);
}

mg_status mg_run_cycles(mg_handle h, const double *f, double *u, int ncycles, mg_result *res) {
  if (!h) return fail(MG_EINVAL, "null handle");
  if (ncycles < 0 || ncycles > MG_MAX_HISTORY - 2) return fail(MG_EINVAL, "ncycles out of range");
  return run(h, f, u, -1.0, ncycles, 0, res);
}

mg_status mg_solve_async(mg_handle h, const double *f, double *u) {
  if (!h) return fail(MG_EINVAL, "null handle");
  mg_status st = begin_solve(h, f, u, h->cfg.rtol, h->cfg.max_cycles, 1);
  if (st != MG_OK) return st;
  for (int i = 0; i < h->cfg.max_cycles + 1; ++i) {
    st = launch_step(h, f, u);
    if (st != MG_OK) return st;
  }
  MG_HIP(hipEventRecord(h->ev_async, h->stream));
  h->async_pending = true;
  return MG_OK;
}

mg_status mg_query(mg_handle h, mg_result *res) {
  if (!h) return fail(MG_EINVAL, "null handle");
  if (!h->async_pending) return fail(MG_EINVAL, "no asynchronous solve pending");
  hipError_t e = hipEventQuery(h->ev_async);
  if (e == hipErrorNotReady) return MG_EBUSY;
  if (e != hipSuccess) return fail(MG_EDEVICE, hipGetErrorString(e));
  h->async_pending = false;
  mg_status outcome = MG_OK;
  mg_status st = fill_result(h, res, &outcome);
  return st != MG_OK ? st : outcome;
}

mg_status mg_residual_norm(mg_handle h, const double *f, const double *u, double *rel) {
  if (!h || !f || !u || !rel) return fail(MG_EINVAL, "null argument");
  MG_HIP(hipSetDevice(h->device));
  hipLaunchKernelGGL(k_state_init, dim3(1), dim3(64), 0, h->stream, h->st, -1.0, 2, 0);
  int np = 0;
  MG_HIP((mgk::launch_sweep<double, double>(h->dim, mgk::kNormOnly, h->ops[0], h->omega, f, nullptr,
                                            (double *)nullptr, h->ns[0], h->partials, &np, nullptr,
                                            h->stream)));
  MG_HIP(mgk::launch_check(h->st, h->partials, np, 0, h->stream));
  MG_HIP((mgk::launch_sweep<double, double>(h->dim, mgk::kNormOnly, h->ops[0], h->omega, f, u,
                                            (double *)nullptr, h->ns[0], h->partials, &np, nullptr,
                                            h->stream)));
  MG_HIP(mgk::launch_check(h->st, h->partials, np, 1, h->stream));
  DevState hs;
  MG_HIP(hipMemcpyAsync(&hs, h->st, sizeof(DevState), hipMemcpyDeviceToHost, h->stream));
  MG_HIP(hipStreamSynchronize(h->stream));
  *rel = hs.hist[0];
  return MG_OK;
}

int mg_level_size(mg_handle h, int level) {
  if (!h || level < 0 || level >= h->L) return -1;
  return h->ns[level];
}

mg_status mg_level_operator(mg_handle h, int level, double a[7], double b[7]) {
  if (!h || level < 0 || level >= h->L || !a || !b) return fail(MG_EINVAL, "bad argument");
  for (int i = 0; i < 7; ++i) {
    a[i] = h->ops[level].a[i];
    b[i] = h->ops[level].b[i];
  }
  return MG_OK;
}

mg_status mg_kernel_smooth(mg_handle h, int level, int fp32, const void *f, const void *u_in,
                           void *u_out) {
  mg_status st = fp32 ? check_level<float>(h, level, false) : check_level<double>(h, level, false);
  if (st != MG_OK) return st;
  if (!f || !u_out || u_in == u_out) return fail(MG_EINVAL, "bad buffers");
  if (h->dim == 2) {
    if (fp32)
      MG_HIP(mgk::launch_pre2d<float>(h->ops[level], h->omega, 1, mgk::kPreWriteU, (const float *)f,
                                      (const float *)u_in, (float *)u_out, nullptr, nullptr,
                                      h->ns[level], nullptr, nullptr, nullptr, h->stream));
    else
      MG_HIP(mgk::launch_pre2d<double>(h->ops[level], h->omega, 1, mgk::kPreWriteU, (const double *)f,
                                       (const double *)u_in, (double *)u_out, nullptr, nullptr,
                                       h->ns[level], nullptr, nullptr, nullptr, h->stream));
    return MG_OK;
  }
  if (fp32)
    MG_HIP((mgk::launch_sweep<float, float>(h->dim, mgk::kSweep, h->ops[level], h->omega,
                                            (const float *)f, (const float *)u_in, (float *)u_out,
                                            h->ns[level], nullptr, nullptr, nullptr, h->stream)));
  else
    MG_HIP((mgk::launch_sweep<double, double>(h->dim, mgk::kSweep, h->ops[level], h->omega,
                                              (const double *)f, (const double *)u_in,
                                              (double *)u_out, h->ns[level], nullptr, nullptr,
                                              nullptr, h->stream)));
  return MG_OK;
}

mg_status mg_kernel_smooth_colour(mg_handle h, int level, int fp32, int colour, const void *f,
                                  const void *u_in, void *u_out) {
  mg_status st = fp32 ? check_level<float>(h, level, false) : check_level<double>(h, level, false);
  if (st != MG_OK) return st;
  if (!f || !u_out || u_in == u_out) return fail(MG_EINVAL, "bad buffers");
  if (colour < 0 || colour > 3) return fail(MG_EINVAL, "colour must be 0, 1, 2 or 3");
  if (h->cfg.smoother == MG_SMOOTH_RBGS && gs_level(h->ops[level])) {  // section 3.1 eq. S_GS
    if (colour != 1 && colour != 2) return fail(MG_EINVAL, "Gauss-Seidel partial steps take colour 1 or 2");
    if (!u_in) return fail(MG_EINVAL, "Gauss-Seidel partial steps need u_in");
    if (fp32)
      MG_HIP(mgk::launch_gs2d<float>(h->ops[level], h->omega, colour, (const float *)f, (const float *)u_in,
                                     (float *)u_out, h->ns[level], nullptr, h->stream));
    else
      MG_HIP(mgk::launch_gs2d<double>(h->ops[level], h->omega, colour, (const double *)f, (const double *)u_in,
                                      (double *)u_out, h->ns[level], nullptr, h->stream));
    return MG_OK;
  }
  if (colour == 3) {  // a whole red-black sweep in one pass
    const LevelOp &op = h->ops[level];
    const int n = h->ns[level];
    if (h->dim == 3) {
      if (!op.cross) return fail(MG_EINVAL, "one-pass 3D red-black sweeps need the cross operator");
      if (fp32)
        MG_HIP(mgk::launch_rbsweep_3d<float>(op, h->omega, (const float *)f, (const float *)u_in,
                                             (float *)u_out, n, nullptr, nullptr, nullptr, h->stream));
      else
        MG_HIP(mgk::launch_rbsweep_3d<double>(op, h->omega, (const double *)f, (const double *)u_in,
                                              (double *)u_out, n, nullptr, nullptr, nullptr, h->stream));
      return MG_OK;
    }
    if (fp32)
      MG_HIP(mgk::launch_pre2d<float>(op, h->omega, 2, mgk::kPreWriteU, (const float *)f, (const float *)u_in,
                                      (float *)u_out, nullptr, nullptr, n, nullptr, nullptr, nullptr,
                                      h->stream, 1, true));
    else
      MG_HIP(mgk::launch_pre2d<double>(op, h->omega, 2, mgk::kPreWriteU, (const double *)f,
                                       (const double *)u_in, (double *)u_out, nullptr, nullptr, n, nullptr,
                                       nullptr, nullptr, h->stream, 1, true));
    return MG_OK;
  }
  if (fp32)
    MG_HIP((mgk::launch_sweep<float, float>(h->dim, mgk::kSweep, h->ops[level], h->omega,
                                            (const float *)f, (const float *)u_in, (float *)u_out,
                                            h->ns[level], nullptr, nullptr, nullptr, h->stream, 1,
                                            colour)));
  else
    MG_HIP((mgk::launch_sweep<double, double>(h->dim, mgk::kSweep, h->ops[level], h->omega,
                                              (const double *)f, (const double *)u_in,
                                              (double *)u_out, h->ns[level], nullptr, nullptr,
                                              nullptr, h->stream, 1, colour)));
  return MG_OK;
}

mg_status mg_kernel_residual(mg_handle h, int level, int fp32, const void *f, const void *u,
                             void *r) {
  mg_status st = check_level<double>(h, level, false);
  if (st != MG_OK) return st;
  if (!f || !u || !r) return fail(MG_EINVAL, "bad buffers");
  if (h->dim == 2) {
    if (fp32)
      MG_HIP(mgk::launch_pre2d<float>(h->ops[level], h->omega, 0, mgk::kPreWriteR, (const float *)f,
                                      (const float *)u, nullptr, (float *)r, nullptr, h->ns[level],
                                      nullptr, nullptr, nullptr, h->stream));
    else
      MG_HIP(mgk::launch_pre2d<double>(h->ops[level], h->omega, 0, mgk::kPreWriteR, (const double *)f,
                                       (const double *)u, nullptr, (double *)r, nullptr,
                                       h->ns[level], nullptr, nullptr, nullptr, h->stream));
    return MG_OK;
  }
  if (fp32)
    MG_HIP((mgk::launch_sweep<float, float>(h->dim, mgk::kResidual, h->ops[level], h->omega,
                                            (const float *)f, (const float *)u, (float *)r,
                                            h->ns[level], nullptr, nullptr, nullptr, h->stream)));
  else
    MG_HIP((mgk::launch_sweep<double, double>(h->dim, mgk::kResidual, h->ops[level], h->omega,
                                              (const double *)f, (const double *)u, (double *)r,
                                              h->ns[level], nullptr, nullptr, nullptr, h->stream)));
  return MG_OK;
}

mg_status mg_kernel_residual_restrict(mg_handle h, int level, int fp32, const void *f,
                                      const void *u, void *fc) {
  mg_status st = check_level<double>(h, level, true);
  if (st != MG_OK) return st;
  if (!f || !fc) return fail(MG_EINVAL, "bad buffers");
  if (h->cfg.restrict_op == 3) {  // the defect goes through the level's sweep target
    if (!u) return fail(MG_EINVAL, "the cubic-adjoint restriction needs u");
    const bool mixed = h->cfg.precision == MG_PREC_MIXED;
    if (mixed && !fp32) return fail(MG_EINVAL, "a mixed-precision handle holds FP32 level arrays only");
    void *scratch = mixed ? h->b32[level].t : h->b64[level].t;
    if (fp32)
      MG_HIP(resid_restrict<float>(h, level, (const float *)f, (const float *)u, (float *)scratch, (float *)fc,
                                   nullptr, h->stream));
    else
      MG_HIP(resid_restrict<double>(h, level, (const double *)f, (const double *)u, (double *)scratch,
                                    (double *)fc, nullptr, h->stream));
    return MG_OK;
  }
  if (h->dim == 2) {
    if (fp32)
      MG_HIP(mgk::launch_pre2d<float>(h->ops[level], h->omega, 0, mgk::kPreRestrict, (const float *)f,
                                      (const float *)u, nullptr, nullptr, (float *)fc, h->ns[level],
                                      nullptr, nullptr, nullptr, h->stream));
    else
      MG_HIP(mgk::launch_pre2d<double>(h->ops[level], h->omega, 0, mgk::kPreRestrict,
                                       (const double *)f, (const double *)u, nullptr, nullptr,
                                       (double *)fc, h->ns[level], nullptr, nullptr, nullptr,
                                       h->stream));
    return MG_OK;
  }
  if (fp32)
    MG_HIP(mgk::launch_resid_restrict<float>(h->dim, h->ops[level], (const float *)f,
                                             (const float *)u, (float *)fc, h->ns[level], nullptr,
                                             h->stream));
  else
    MG_HIP(mgk::launch_resid_restrict<double>(h->dim, h->ops[level], (const double *)f,
                                              (const double *)u, (double *)fc, h->ns[level],
                                              nullptr, h->stream));
  return MG_OK;
}

mg_status mg_kernel_prolong_correct(mg_handle h, int level, int fp32, const void *v,
                                    const void *u_in, void *u_out) {
  mg_status st = check_level<double>(h, level, true);
  if (st != MG_OK) return st;
  if (!v || !u_in || !u_out) return fail(MG_EINVAL, "bad buffers");
  if (h->dim == 2) {
    if (fp32)
      MG_HIP(mgk::launch_post2d<float>(h->ops[level], h->omega, 0, h->cfg.prolong, (const float *)v,
                                       (const float *)u_in, nullptr, (float *)u_out, h->ns[level],
                                       nullptr, h->stream));
    else
      MG_HIP(mgk::launch_post2d<double>(h->ops[level], h->omega, 0, h->cfg.prolong,
                                        (const double *)v, (const double *)u_in, nullptr,
                                        (double *)u_out, h->ns[level], nullptr, h->stream));
    return MG_OK;
  }
  if (fp32)
    MG_HIP(mgk::launch_prolong_correct<float>(h->dim, h->cfg.prolong, (const float *)v,
                                              (const float *)u_in, (float *)u_out, h->ns[level],
                                              nullptr, h->stream));
  else
    MG_HIP(mgk::launch_prolong_correct<double>(h->dim, h->cfg.prolong, (const double *)v,
                                               (const double *)u_in, (double *)u_out,
                                               h->ns[level], nullptr, h->stream));
  return MG_OK;
}

mg_status mg_kernel_presmooth_restrict(mg_handle h, int level, int fp32, const void *f,
                                       const void *u_in, void *u_out, void *fc) {
  mg_status st = check_level<double>(h, level, true);
  if (st != MG_OK) return st;
  const bool rb = h->cfg.smoother == MG_SMOOTH_RBJ;
  if (h->cfg.smoother == MG_SMOOTH_RBGS) return fail(MG_EINVAL, "no fused pass for Gauss-Seidel smoothing");
  if (h->cfg.restrict_op == 3) return fail(MG_EINVAL, "no fused pass for the cubic-adjoint restriction");
  if (h->dim != 2 || (!rb && h->cfg.nu1 > 3))
    return fail(MG_EINVAL, "fused pre-smoothing needs dim 2, nu1 <= 3");
  if (!f || !u_out || !fc || u_in == u_out) return fail(MG_EINVAL, "bad buffers");
  const int mode = mgk::kPreWriteU | mgk::kPreRestrict;
  const int stages = rb ? 2 * std::min(1, h->cfg.nu1) : h->cfg.nu1;
  if (fp32)
    MG_HIP(mgk::launch_pre2d<float>(h->ops[level], h->omega, stages, mode, (const float *)f,
                                    (const float *)u_in, (float *)u_out, nullptr, (float *)fc,
                                    h->ns[level], nullptr, nullptr, nullptr, h->stream, 1, rb));
  else
    MG_HIP(mgk::launch_pre2d<double>(h->ops[level], h->omega, stages, mode, (const double *)f,
                                     (const double *)u_in, (double *)u_out, nullptr, (double *)fc,
                                     h->ns[level], nullptr, nullptr, nullptr, h->stream, 1, rb));
  return MG_OK;
}

mg_status mg_kernel_prolong_postsmooth(mg_handle h, int level, int fp32, const void *v,
                                       const void *u_in, const void *f, void *u_out) {
  mg_status st = check_level<double>(h, level, true);
  if (st != MG_OK) return st;
  const bool rb = h->cfg.smoother == MG_SMOOTH_RBJ;
  if (h->cfg.smoother == MG_SMOOTH_RBGS) return fail(MG_EINVAL, "no fused pass for Gauss-Seidel smoothing");
  if (h->dim != 2 || (!rb && h->cfg.nu2 > 2))
    return fail(MG_EINVAL, "fused post-smoothing needs dim 2, nu2 <= 2");
  if (!v || !u_in || !f || !u_out || u_in == u_out) return fail(MG_EINVAL, "bad buffers");
  const int stages = rb ? 2 * std::min(1, h->cfg.nu2) : h->cfg.nu2;
  if (fp32)
    MG_HIP(mgk::launch_post2d<float>(h->ops[level], h->omega, stages, h->cfg.prolong,
                                     (const float *)v, (const float *)u_in, (const float *)f,
                                     (float *)u_out, h->ns[level], nullptr, h->stream, 1, rb));
  else
    MG_HIP(mgk::launch_post2d<double>(h->ops[level], h->omega, stages, h->cfg.prolong,
                                      (const double *)v, (const double *)u_in, (const double *)f,
                                      (double *)u_out, h->ns[level], nullptr, h->stream, 1, rb));
  return MG_OK;
}

mg_status mg_kernel_coarsest_solve(mg_handle h, int fp32, const void *g, void *v) {
  if (!h || !g || !v) return fail(MG_EINVAL, "bad argument");
  MG_HIP(hipSetDevice(h->device));
  const int nc = h->ns[h->L - 1];
  if (fp32)
    MG_HIP(mgk::launch_coarsest<float>(h->dim, h->ainv_t, (const float *)g, (float *)v, nc, nullptr,
                                       h->stream));
  else
    MG_HIP(mgk::launch_coarsest<double>(h->dim, h->ainv_t, (const double *)g, (double *)v, nc,
                                        nullptr, h->stream));
  return MG_OK;
}

mg_status mg_synchronize(mg_handle h) {
  if (!h) return fail(MG_EINVAL, "null handle");
  MG_HIP(hipStreamSynchronize(h->stream));
  return MG_OK;
}

}  // extern "C"

// ------------------------------------------------------------------ batches ----
namespace mgb {

static_assert(offsetof(DevState, done) == 0 && offsetof(DevState, checks) == 4 &&
                  offsetof(DevState, status) == 8 && offsetof(DevState, stall) == 12,
              "SlotFlags mirrors the leading fields of DevState");

size_t footprint(const mg_config *cfg, int slots) {
  int L = 0;
  if (validate(cfg, &L) != MG_OK) return 0;
  return footprint_of(cfg, L, slots, true);
}

mg_status create(const mg_config *cfg, int slots, hipStream_t stream, mg_ctx **out) {
  mg_status st = setup_ctx(cfg, stream, slots, true, out);
  if (st != MG_OK) return st;
  mg_ctx *c = *out;
  st = ensure_graph(c, (const double *)c->b64[0].f, (double *)c->b64[0].u);
  if (st != MG_OK) {
    mg_destroy(c);
    *out = nullptr;
  }
  return st;
}

void destroy(mg_ctx *c) { mg_destroy(c); }

mg_status admit(mg_ctx *c, int k, const double *f) {
  if (k < 0 || k >= c->slots || !f) return fail(MG_EINVAL, "bad slot or buffer");
  const size_t np = points(c->dim, c->ns[0]);
  double *fk = (double *)c->b64[0].f + (size_t)k * np;
  double *uk = (double *)c->b64[0].u + (size_t)k * np;
  DevState *sk = c->st + k;
  double *pk = c->partials + (size_t)k * c->np_max;
  MG_HIP(hipMemcpyAsync(fk, f, np * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
  MG_HIP(mgk::launch_fill<double>(uk, np, 0.0, nullptr, c->stream));
  hipLaunchKernelGGL(k_state_init, dim3(1), dim3(64), 0, c->stream, sk, c->cfg.rtol,
                     c->cfg.max_cycles + 1, 1);
  MG_HIP(hipGetLastError());
  int nparts = 0;
  MG_HIP((mgk::launch_sweep<double, double>(c->dim, mgk::kNormOnly, c->ops[0], c->omega, fk,
                                            nullptr, (double *)nullptr, c->ns[0], pk, &nparts,
                                            nullptr, c->stream)));
  MG_HIP(mgk::launch_check(sk, pk, nparts, 0, c->stream));
  return MG_OK;
}

mg_status step(mg_ctx *c, int count) {
  for (int i = 0; i < count; ++i) {
    mg_status st = launch_step(c, (const double *)c->b64[0].f, (double *)c->b64[0].u);
    if (st != MG_OK) return st;
  }
  return MG_OK;
}

mg_status read_flags(mg_ctx *c, SlotFlags *host) {
  MG_HIP(hipMemcpy2DAsync(host, sizeof(SlotFlags), c->st, sizeof(DevState), sizeof(SlotFlags),
                          c->slots, hipMemcpyDeviceToHost, c->stream));
  return MG_OK;
}

mg_status retire(mg_ctx *c, int k, double *u_dst, DevState *host_state) {
  if (k < 0 || k >= c->slots || !u_dst) return fail(MG_EINVAL, "bad slot or buffer");
  const size_t np = points(c->dim, c->ns[0]);
  const double *uk = (const double *)c->b64[0].u + (size_t)k * np;
  MG_HIP(hipMemcpyAsync(u_dst, uk, np * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
  MG_HIP(hipMemcpyAsync(host_state, c->st + k, sizeof(DevState), hipMemcpyDeviceToHost, c->stream));
  return MG_OK;
}

void result(const mg_ctx *c, const DevState &hs, mg_result *res, mg_status *outcome) {
  result_from_state(c, hs, res, outcome);
}

void set_error(const std::string &msg) { g_error = msg; }

}  // namespace mgb
