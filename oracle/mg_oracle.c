/*
 * mg_oracle.c -- plain FP64 CPU reference multigrid (TEST INFRASTRUCTURE ONLY).
 *
 * Written for readability against the paper, not for speed: every operator is the
 * plain sum its stencil defines, evaluated point by point, with the odd reflection
 * of grid functions across the Dirichlet boundary.  No fusion, no blocking, no
 * reduced precision.  OpenMP only splits the outermost grid loop; every norm is
 * summed in a fixed order so results do not depend on the thread count.
 *
 * Citations name sections and equation labels of Liu & Henshaw, "Multigrid with
 * Nonstandard Coarsening".
 */
#include "mg_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

int or_num_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

void or_set_num_threads(int threads) {
#ifdef _OPENMP
  if (threads > 0) omp_set_num_threads(threads);
#else
  (void)threads;
#endif
}

/* ------------------------------------------------------------------ grids -- */

static long npts(int dim, int n) { return dim == 2 ? (long)n * n : (long)n * n * n; }

static long at(int n, int i, int j, int k) { return ((long)k * n + j) * n + i; }

/* Range of the outermost loop over interior points: z = 1..n-2 in 3D, the single
 * plane z = 0 in 2D. */
static int k_first(int dim) { return dim == 3 ? 1 : 0; }
static int k_end(int dim, int n) { return dim == 3 ? n - 1 : 1; }

/* Value of the odd extension of u at (i, j, k): each coordinate outside 0..n-1 is
 * reflected about the boundary point it crossed and flips the sign. */
static double ext(const double *u, int dim, int n, int i, int j, int k) {
  double sign = 1.0;
  if (i < 0) { i = -i; sign = -sign; }
  if (i > n - 1) { i = 2 * (n - 1) - i; sign = -sign; }
  if (j < 0) { j = -j; sign = -sign; }
  if (j > n - 1) { j = 2 * (n - 1) - j; sign = -sign; }
  if (dim == 3) {
    if (k < 0) { k = -k; sign = -sign; }
    if (k > n - 1) { k = 2 * (n - 1) - k; sign = -sign; }
  } else {
    k = 0;
  }
  return sign * u[at(n, i, j, k)];
}

int or_num_levels(int n, int n_coarsest) {
  int levels = 1;
  if (n_coarsest < 3 || n < n_coarsest) return 0;
  while (n > n_coarsest) {
    if ((n - 1) % 2 != 0) return 0;
    n = (n - 1) / 2 + 1;
    ++levels;
  }
  return n == n_coarsest ? levels : 0;
}

/* --------------------------------------------------------------- stencils -- */

static int swidth(int R) { return 2 * R + 1; }

static long sidx(int dim, int R, int ox, int oy, int oz) {
  int w = swidth(R);
  return dim == 2 ? (long)(oy + R) * w + (ox + R) : ((long)(oz + R) * w + (oy + R)) * w + (ox + R);
}

/* 1D second difference -u'' of order 2 (eq. L_h_2), 4 (eq. L_h_2d_4o) or 6 (section 3.3
 * eq. LhOrder6, one axis of the printed 2D stencil), times h^2. */
static void second_difference_1d(int order, double *c /* 2R+1 */) {
  if (order == 2) {
    c[0] = -1.0; c[1] = 2.0; c[2] = -1.0;
  } else if (order == 4) {
    c[0] = 1.0 / 12.0; c[1] = -16.0 / 12.0; c[2] = 30.0 / 12.0;
    c[3] = -16.0 / 12.0; c[4] = 1.0 / 12.0;
  } else {
    c[0] = -2.0 / 180.0; c[1] = 27.0 / 180.0; c[2] = -270.0 / 180.0; c[3] = 490.0 / 180.0;
    c[4] = -270.0 / 180.0; c[5] = 27.0 / 180.0; c[6] = -2.0 / 180.0;
  }
}

int or_fine_stencil(int dim, int order, double h, double *s) {
  int R = order / 2, w = swidth(R);
  double c[7];
  long total = dim == 2 ? (long)w * w : (long)w * w * w;
  second_difference_1d(order, c);
  memset(s, 0, sizeof(double) * total);
  /* -Delta_h is the sum over axes of the 1D operator along that axis. */
  for (int o = -R; o <= R; ++o) {
    double v = c[o + R] / (h * h);
    s[sidx(dim, R, o, 0, 0)] += v;
    s[sidx(dim, R, 0, o, 0)] += v;
    if (dim == 3) s[sidx(dim, R, 0, 0, o)] += v;
  }
  return R;
}

/* 1D restriction weights at fine offset o from the coarse point (section 3.1 eq.
 * transfer_2d per axis: (1,2,1)/4; appendix A.4 per axis: (1,0,-9,-16,-9,0,1)/(-32)). */
static int restrict_radius(int op) { return op == OR_RESTRICT_CUBIC ? 3 : 1; }
static double restrict_w1(int op, int o) {
  if (o < 0) o = -o;
  if (op == OR_RESTRICT_CUBIC) {
    switch (o) {
      case 0: return 16.0 / 32.0;
      case 1: return 9.0 / 32.0;
      case 3: return -1.0 / 32.0;
      default: return 0.0;
    }
  }
  switch (o) {
    case 0: return 0.5;
    case 1: return 0.25;
    default: return 0.0;
  }
}

/* 1D interpolation weight of a coarse value at fine distance o (in fine points)
 * (section 3.1 linear: ]1 2 1[/2 per axis; appendix A.4 cubic: ]-1 0 9 16 9 0 -1[/16). */
static int prolong_radius(int op) { return op == OR_PROLONG_CUBIC ? 3 : 1; }
static double prolong_w1(int op, int o) {
  if (o < 0) o = -o;
  if (op == OR_PROLONG_CUBIC) {
    switch (o) {
      case 0: return 1.0;
      case 1: return 9.0 / 16.0;
      case 3: return -1.0 / 16.0;
      default: return 0.0;
    }
  }
  switch (o) {
    case 0: return 1.0;
    case 1: return 0.5;
    default: return 0.0;
  }
}

int or_galerkin_stencil(int dim, int Rf, const double *sf, int restrict_op, int prolong,
                        double *sc) {
  int rP = prolong_radius(prolong), rR = restrict_radius(restrict_op);
  int Rc = (Rf + rP + rR) / 2;
  int W = 2 * Rc + rP;
  if (rR + Rf > W) W = rR + Rf;
  int ww = 2 * W + 1;
  int kz_lo = dim == 3 ? -Rc : 0, kz_hi = dim == 3 ? Rc : 0;
  int fz = dim == 3 ? Rf : 0, rz = dim == 3 ? rR : 0, wz = dim == 3 ? W : 0;
  long wsize = dim == 3 ? (long)ww * ww * ww : (long)ww * ww;
  double *w = (double *)malloc(sizeof(double) * wsize);
  for (int Jz = kz_lo; Jz <= kz_hi; ++Jz)
    for (int Jy = -Rc; Jy <= Rc; ++Jy)
      for (int Jx = -Rc; Jx <= Rc; ++Jx) {
        /* w = I_H^h applied to the coarse unit function at J, on the fine window. */
        for (int z = -wz; z <= wz; ++z)
          for (int y = -W; y <= W; ++y)
            for (int x = -W; x <= W; ++x) {
              double v = prolong_w1(prolong, x - 2 * Jx) * prolong_w1(prolong, y - 2 * Jy);
              if (abs(x - 2 * Jx) > rP || abs(y - 2 * Jy) > rP) v = 0.0;
              if (dim == 3) {
                if (abs(z - 2 * Jz) > rP) v = 0.0;
                else v *= prolong_w1(prolong, z - 2 * Jz);
              }
              w[((long)(z + wz) * ww + (y + W)) * ww + (x + W)] = v;
            }
        /* c_J = sum_o r(o) * (L_h w)(o). */
        double c = 0.0;
        for (int oz = -rz; oz <= rz; ++oz)
          for (int oy = -rR; oy <= rR; ++oy)
            for (int ox = -rR; ox <= rR; ++ox) {
              double r = restrict_w1(restrict_op, ox) * restrict_w1(restrict_op, oy);
              if (dim == 3) r *= restrict_w1(restrict_op, oz);
              if (r == 0.0) continue;
              double lw = 0.0;
              for (int kz = -fz; kz <= fz; ++kz)
                for (int ky = -Rf; ky <= Rf; ++ky)
                  for (int kx = -Rf; kx <= Rf; ++kx) {
                    double a = sf[sidx(dim, Rf, kx, ky, kz)];
                    if (a == 0.0) continue;
                    lw += a * w[((long)(oz + kz + wz) * ww + (oy + ky + W)) * ww + (ox + kx + W)];
                  }
              c += r * lw;
            }
        sc[sidx(dim, Rc, Jx, Jy, Jz)] = c;
      }
  free(w);
  return Rc;
}

/* Non-zero stencil entries as an offset list (keeps the loops below readable). */
typedef struct {
  int count;
  int *ox, *oy, *oz;
  double *c;
} entries;

static entries list_entries(int dim, int R, const double *s) {
  entries e;
  int w = swidth(R);
  long total = dim == 2 ? (long)w * w : (long)w * w * w;
  e.count = 0;
  e.ox = (int *)malloc(sizeof(int) * total);
  e.oy = (int *)malloc(sizeof(int) * total);
  e.oz = (int *)malloc(sizeof(int) * total);
  e.c = (double *)malloc(sizeof(double) * total);
  for (int oz = (dim == 3 ? -R : 0); oz <= (dim == 3 ? R : 0); ++oz)
    for (int oy = -R; oy <= R; ++oy)
      for (int ox = -R; ox <= R; ++ox) {
        double v = s[sidx(dim, R, ox, oy, oz)];
        if (v == 0.0) continue;
        e.ox[e.count] = ox; e.oy[e.count] = oy; e.oz[e.count] = oz; e.c[e.count] = v;
        ++e.count;
      }
  return e;
}

static void free_entries(entries *e) {
  free(e->ox); free(e->oy); free(e->oz); free(e->c);
}

/* (L u)(x) = sum_k c_k u(x+k).  Every operator of the method annihilates constants (its
 * coefficients sum to zero: -Delta_h of either order, and R L P with transfers that
 * preserve constants), so the sum equals sum_{k != 0} c_k (u(x+k) - u(x)).  That form is
 * used here: with the plain form, the rounding of coefficients such as -16/12 leaves a
 * non-zero row sum of order eps/h^2, i.e. a spurious term (eps/h^2) u that shifts the
 * discrete solution by about eps/(h^2 lambda_min) relative, 1e-10 at h = 1/4096. */
static double apply_at(const entries *e, int dim, int n, const double *u, int i, int j, int k) {
  const double u0 = ext(u, dim, n, i, j, k);
  double sum = 0.0;
  for (int q = 0; q < e->count; ++q) {
    if (e->ox[q] == 0 && e->oy[q] == 0 && e->oz[q] == 0) continue;
    sum += e->c[q] * (ext(u, dim, n, i + e->ox[q], j + e->oy[q], k + e->oz[q]) - u0);
  }
  return sum;
}

/* True when the stencil annihilates constants up to rounding (the relative row sum of a
 * computed Galerkin stencil grows like 4^l * eps over l levels: 2e-12 at l = 9). */
static int annihilates_constants(int dim, int R, const double *s) {
  int w = swidth(R);
  long total = dim == 2 ? (long)w * w : (long)w * w * w;
  double sum = 0.0, mag = 0.0;
  for (long q = 0; q < total; ++q) {
    sum += s[q];
    mag += fabs(s[q]);
  }
  return fabs(sum) <= 1e-9 * mag;
}

/* -------------------------------------------------------- grid operators -- */

void or_apply(int dim, int n, int R, const double *s, const double *u, double *out) {
  entries e = list_entries(dim, R, s);
  memset(out, 0, sizeof(double) * npts(dim, n));
#pragma omp parallel for schedule(static)
  for (int k = k_first(dim); k < k_end(dim, n); ++k) {
    for (int j = 1; j < n - 1; ++j)
      for (int i = 1; i < n - 1; ++i) out[at(n, i, j, k)] = apply_at(&e, dim, n, u, i, j, k);
  }
  free_entries(&e);
}

void or_residual(int dim, int n, int R, const double *s, const double *f, const double *u,
                 double *d) {
  entries e = list_entries(dim, R, s);
  memset(d, 0, sizeof(double) * npts(dim, n));
#pragma omp parallel for schedule(static)
  for (int k = k_first(dim); k < k_end(dim, n); ++k) {
    for (int j = 1; j < n - 1; ++j)
      for (int i = 1; i < n - 1; ++i) {
        long p = at(n, i, j, k);
        d[p] = f[p] - apply_at(&e, dim, n, u, i, j, k);
      }
  }
  free_entries(&e);
}

void or_jacobi_colour(int dim, int n, int R, const double *s, double omega, int colour,
                      const double *f, const double *u, double *u_out) {
  entries e = list_entries(dim, R, s);
  double a0 = s[sidx(dim, R, 0, 0, 0)];
  memcpy(u_out, u, sizeof(double) * npts(dim, n));
#pragma omp parallel for schedule(static)
  for (int k = k_first(dim); k < k_end(dim, n); ++k) {
    for (int j = 1; j < n - 1; ++j)
      for (int i = 1; i < n - 1; ++i) {
        int odd = (i + j + k) % 2;  /* k = 0 in 2D */
        if (colour == 1 && !odd) continue;
        if (colour == 2 && odd) continue;
        long p = at(n, i, j, k);
        u_out[p] = u[p] + omega / a0 * (f[p] - apply_at(&e, dim, n, u, i, j, k));
      }
  }
  free_entries(&e);
}

void or_gs_colour(int dim, int n, int R, const double *s, double omega, int colour,
                  const double *f, const double *u, double *u_out) {
  entries e = list_entries(dim, R, s);
  double a0 = s[sidx(dim, R, 0, 0, 0)];
  memcpy(u_out, u, sizeof(double) * npts(dim, n));
  /* sequential on purpose: each point sees the new values of the points before it */
  for (int k = k_first(dim); k < k_end(dim, n); ++k)
    for (int j = 1; j < n - 1; ++j)
      for (int i = 1; i < n - 1; ++i) {
        int odd = (i + j + k) % 2;
        if (colour == 1 && !odd) continue;
        if (colour == 2 && odd) continue;
        long p = at(n, i, j, k);
        u_out[p] += omega / a0 * (f[p] - apply_at(&e, dim, n, u_out, i, j, k));
      }
  free_entries(&e);
}

void or_jacobi(int dim, int n, int R, const double *s, double omega, const double *f,
               const double *u, double *u_out) {
  or_jacobi_colour(dim, n, R, s, omega, 0, f, u, u_out);
}

void or_restrict(int dim, int nf, int restrict_op, const double *d, double *fc) {
  int nc = (nf - 1) / 2 + 1;
  int rR = restrict_radius(restrict_op);
  int rz = dim == 3 ? rR : 0;
  memset(fc, 0, sizeof(double) * npts(dim, nc));
#pragma omp parallel for schedule(static)
  for (int K = k_first(dim); K < k_end(dim, nc); ++K) {
    for (int J = 1; J < nc - 1; ++J)
      for (int I = 1; I < nc - 1; ++I) {
        double sum = 0.0;
        for (int oz = -rz; oz <= rz; ++oz)
          for (int oy = -rR; oy <= rR; ++oy)
            for (int ox = -rR; ox <= rR; ++ox) {
              double w = restrict_w1(restrict_op, ox) * restrict_w1(restrict_op, oy);
              if (dim == 3) w *= restrict_w1(restrict_op, oz);
              if (w == 0.0) continue;
              sum += w * ext(d, dim, nf, 2 * I + ox, 2 * J + oy, dim == 3 ? 2 * K + oz : 0);
            }
        fc[at(nc, I, J, dim == 3 ? K : 0)] = sum;
      }
  }
}

/* Smallest coarse index whose interpolation stencil reaches fine index x. */
static int floor_div2(int a) { return a >= 0 ? a / 2 : -((-a + 1) / 2); }

void or_prolong_add(int dim, int nf, int prolong, const double *v, double *u) {
  int nc = (nf - 1) / 2 + 1;
  int rP = prolong_radius(prolong);
#pragma omp parallel for schedule(static)
  for (int k = k_first(dim); k < k_end(dim, nf); ++k) {
    for (int j = 1; j < nf - 1; ++j)
      for (int i = 1; i < nf - 1; ++i) {
        double sum = 0.0;
        int kz_lo = dim == 3 ? floor_div2(k - rP + 1) : 0, kz_hi = dim == 3 ? floor_div2(k + rP) : 0;
        for (int Kc = kz_lo; Kc <= kz_hi; ++Kc)
          for (int Jc = floor_div2(j - rP + 1); Jc <= floor_div2(j + rP); ++Jc)
            for (int Ic = floor_div2(i - rP + 1); Ic <= floor_div2(i + rP); ++Ic) {
              if (abs(i - 2 * Ic) > rP || abs(j - 2 * Jc) > rP) continue;
              if (dim == 3 && abs(k - 2 * Kc) > rP) continue;
              double w = prolong_w1(prolong, i - 2 * Ic) * prolong_w1(prolong, j - 2 * Jc);
              if (dim == 3) w *= prolong_w1(prolong, k - 2 * Kc);
              if (w == 0.0) continue;
              sum += w * ext(v, dim, nc, Ic, Jc, Kc);
            }
        u[at(nf, i, j, k)] += sum;
      }
  }
}

double or_norm(int dim, int n, const double *v) {
  int nk = dim == 3 ? n : 1;
  double h = 1.0 / (n - 1);
  double *part = (double *)calloc(nk, sizeof(double));
#pragma omp parallel for schedule(static)
  for (int k = k_first(dim); k < k_end(dim, n); ++k) {
    double s = 0.0;
    for (int j = 1; j < n - 1; ++j)
      for (int i = 1; i < n - 1; ++i) {
        double x = v[at(n, i, j, k)];
        s += x * x;
      }
    part[k] = s;
  }
  double total = 0.0;
  for (int k = 0; k < nk; ++k) total += part[k];
  free(part);
  return sqrt(pow(h, dim) * total);
}

double or_residual_norm_ld(int dim, int n, int R, const double *s, const double *f,
                           const double *u) {
  entries e = list_entries(dim, R, s);
  int nk = dim == 3 ? n : 1;
  long double *part = (long double *)calloc(nk, sizeof(long double));
#pragma omp parallel for schedule(static)
  for (int k = k_first(dim); k < k_end(dim, n); ++k) {
    long double acc = 0.0L;
    for (int j = 1; j < n - 1; ++j)
      for (int i = 1; i < n - 1; ++i) {
        const long double u0 = ext(u, dim, n, i, j, k);
        long double lu = 0.0L;
        for (int q = 0; q < e.count; ++q) {
          if (e.ox[q] == 0 && e.oy[q] == 0 && e.oz[q] == 0) continue;
          lu += (long double)e.c[q] *
                ((long double)ext(u, dim, n, i + e.ox[q], j + e.oy[q], k + e.oz[q]) - u0);
        }
        long double r = (long double)f[at(n, i, j, k)] - lu;
        acc += r * r;
      }
    part[k] = acc;
  }
  long double total = 0.0L;
  for (int k = 0; k < nk; ++k) total += part[k];
  free(part);
  free_entries(&e);
  double h = 1.0 / (n - 1);
  return (double)sqrtl((long double)pow(h, dim) * total);
}

/* -------------------------------------------------------------- hierarchy -- */

typedef struct {
  int n, R;
  double *s;        /* stencil (2R+1)^dim */
  double *u, *f;    /* iterate and right-hand side (levels >= 1) */
  double *d, *t;    /* defect and Jacobi target */
} or_level;

struct or_mg {
  or_config cfg;
  int L;
  or_level lev[OR_MAX_LEVELS];
  /* coarsest-level dense LU factors */
  int m;
  double *lu;
  int *piv;
};

static double *alloc_grid(int dim, int n) { return (double *)calloc(npts(dim, n), sizeof(double)); }

static void factor_coarsest(or_mg *mg) {
  or_level *c = &mg->lev[mg->L - 1];
  int dim = mg->cfg.dim, n = c->n;
  int q = n - 2;
  int m = dim == 2 ? q * q : q * q * q;
  double *e = alloc_grid(dim, n), *col = alloc_grid(dim, n);
  mg->m = m;
  mg->lu = (double *)malloc(sizeof(double) * (size_t)m * m);
  mg->piv = (int *)malloc(sizeof(int) * m);
  /* Column p of the matrix is L applied to the p-th interior unit function. */
  for (int p = 0; p < m; ++p) {
    int i = 1 + p % q, j = 1 + (p / q) % q, k = dim == 3 ? 1 + p / (q * q) : 0;
    memset(e, 0, sizeof(double) * npts(dim, n));
    e[at(n, i, j, k)] = 1.0;
    or_apply(dim, n, c->R, c->s, e, col);
    for (int r = 0; r < m; ++r) {
      int ri = 1 + r % q, rj = 1 + (r / q) % q, rk = dim == 3 ? 1 + r / (q * q) : 0;
      mg->lu[(size_t)r * m + p] = col[at(n, ri, rj, rk)];
    }
  }
  free(e);
  free(col);
  /* LU factorisation with partial pivoting, row-major, in place. */
  double *a = mg->lu;
  for (int kcol = 0; kcol < m; ++kcol) {
    int best = kcol;
    for (int r = kcol + 1; r < m; ++r)
      if (fabs(a[(size_t)r * m + kcol]) > fabs(a[(size_t)best * m + kcol])) best = r;
    mg->piv[kcol] = best;
    if (best != kcol)
      for (int cidx = 0; cidx < m; ++cidx) {
        double tmp = a[(size_t)kcol * m + cidx];
        a[(size_t)kcol * m + cidx] = a[(size_t)best * m + cidx];
        a[(size_t)best * m + cidx] = tmp;
      }
    for (int r = kcol + 1; r < m; ++r) {
      double l = a[(size_t)r * m + kcol] / a[(size_t)kcol * m + kcol];
      a[(size_t)r * m + kcol] = l;
      for (int cidx = kcol + 1; cidx < m; ++cidx) a[(size_t)r * m + cidx] -= l * a[(size_t)kcol * m + cidx];
    }
  }
}

void or_mg_coarsest_solve(or_mg *mg, const double *g, double *v) {
  or_level *c = &mg->lev[mg->L - 1];
  int dim = mg->cfg.dim, n = c->n, q = n - 2, m = mg->m;
  double *b = (double *)malloc(sizeof(double) * m);
  for (int p = 0; p < m; ++p) {
    int i = 1 + p % q, j = 1 + (p / q) % q, k = dim == 3 ? 1 + p / (q * q) : 0;
    b[p] = g[at(n, i, j, k)];
  }
  for (int kcol = 0; kcol < m; ++kcol) {
    int pr = mg->piv[kcol];
    if (pr != kcol) { double t = b[kcol]; b[kcol] = b[pr]; b[pr] = t; }
  }
  for (int r = 0; r < m; ++r)
    for (int cidx = 0; cidx < r; ++cidx) b[r] -= mg->lu[(size_t)r * m + cidx] * b[cidx];
  for (int r = m - 1; r >= 0; --r) {
    for (int cidx = r + 1; cidx < m; ++cidx) b[r] -= mg->lu[(size_t)r * m + cidx] * b[cidx];
    b[r] /= mg->lu[(size_t)r * m + r];
  }
  memset(v, 0, sizeof(double) * npts(dim, n));
  for (int p = 0; p < m; ++p) {
    int i = 1 + p % q, j = 1 + (p / q) % q, k = dim == 3 ? 1 + p / (q * q) : 0;
    v[at(n, i, j, k)] = b[p];
  }
  free(b);
}

or_mg *or_mg_create(const or_config *cfg) {
  int L = or_num_levels(cfg->n, cfg->n_coarsest);
  if (L <= 0 || L > OR_MAX_LEVELS || (cfg->dim != 2 && cfg->dim != 3)) return NULL;
  if (cfg->order != 2 && cfg->order != 4 && cfg->order != 6) return NULL;
  if (cfg->coarse < OR_COARSE_NG || cfg->coarse > OR_COARSE_G2) return NULL;
  if (cfg->smoother != OR_SMOOTH_JACOBI && cfg->smoother != OR_SMOOTH_RBJ &&
      cfg->smoother != OR_SMOOTH_RBGS)
    return NULL;
  or_mg *mg = (or_mg *)calloc(1, sizeof(or_mg));
  int dim = cfg->dim;
  int w = swidth(OR_MAX_RADIUS);
  long smax = dim == 2 ? (long)w * w : (long)w * w * w;
  mg->cfg = *cfg;
  mg->L = L;
  int n = cfg->n;
  for (int l = 0; l < L; ++l) {
    or_level *lv = &mg->lev[l];
    lv->n = n;
    lv->s = (double *)calloc(smax, sizeof(double));
    double h = 1.0 / (n - 1);
    if (l == 0 || cfg->coarse == OR_COARSE_NG) {
      lv->R = or_fine_stencil(dim, cfg->order, h, lv->s);
    } else if (cfg->coarse == OR_COARSE_NG2) {
      lv->R = or_fine_stencil(dim, 2, h, lv->s);
    } else if (cfg->coarse == OR_COARSE_G2 && l == 1) {
      /* R L_h^(2) P with the second-order operator at the finest spacing */
      double *s2 = (double *)calloc(smax, sizeof(double));
      const int R2 = or_fine_stencil(dim, 2, 1.0 / (cfg->n - 1), s2);
      lv->R = or_galerkin_stencil(dim, R2, s2, cfg->restrict_op, cfg->prolong, lv->s);
      free(s2);
    } else {
      or_level *fl = &mg->lev[l - 1];
      lv->R = or_galerkin_stencil(dim, fl->R, fl->s, cfg->restrict_op, cfg->prolong, lv->s);
    }
    if (!annihilates_constants(dim, lv->R, lv->s)) {
      or_mg_destroy(mg);
      return NULL;
    }
    if (l > 0) {
      lv->u = alloc_grid(dim, n);
      lv->f = alloc_grid(dim, n);
    }
    lv->d = alloc_grid(dim, n);
    lv->t = alloc_grid(dim, n);
    n = (n - 1) / 2 + 1;
  }
  factor_coarsest(mg);
  return mg;
}

void or_mg_destroy(or_mg *mg) {
  if (!mg) return;
  for (int l = 0; l < mg->L; ++l) {
    free(mg->lev[l].s); free(mg->lev[l].u); free(mg->lev[l].f);
    free(mg->lev[l].d); free(mg->lev[l].t);
  }
  free(mg->lu);
  free(mg->piv);
  free(mg);
}

int or_mg_levels(const or_mg *mg) { return mg->L; }

int or_mg_level_stencil(const or_mg *mg, int l, int *n_out, double *s) {
  const or_level *lv = &mg->lev[l];
  int w = swidth(lv->R);
  long total = mg->cfg.dim == 2 ? (long)w * w : (long)w * w * w;
  if (n_out) *n_out = lv->n;
  if (s) memcpy(s, lv->s, sizeof(double) * total);
  return lv->R;
}

static void smooth(or_mg *mg, int l, double *u, const double *f, int sweeps) {
  or_level *lv = &mg->lev[l];
  int dim = mg->cfg.dim;
  /* omega-Jacobi: one partial step on every point; red-black: red points, then black
   * points from the updated red values (S = S^B S^R, section 3.1 eq. S_rb), each partial
   * step a Jacobi step (RBJ) or a Gauss-Seidel step (RBGS, eq. S_GS) on its colour */
  const int rb = mg->cfg.smoother != OR_SMOOTH_JACOBI;
  for (int s = 0; s < sweeps; ++s) {
    for (int c = rb ? 1 : 0; c <= (rb ? 2 : 0); ++c) {
      if (mg->cfg.smoother == OR_SMOOTH_RBGS)
        or_gs_colour(dim, lv->n, lv->R, lv->s, mg->cfg.omega, c, f, u, lv->t);
      else
        or_jacobi_colour(dim, lv->n, lv->R, lv->s, mg->cfg.omega, c, f, u, lv->t);
      memcpy(u, lv->t, sizeof(double) * npts(dim, lv->n));
    }
  }
}

/* The gamma-cycle of section 2.2 on level l: pre-smooth, defect, restrict, coarse
 * solve (exact on the coarsest level, else gamma cycles from a zero guess), interpolate
 * and correct, post-smooth. */
static void cycle(or_mg *mg, int l, double *u, const double *f) {
  int dim = mg->cfg.dim;
  or_level *lv = &mg->lev[l], *cv = &mg->lev[l + 1];
  smooth(mg, l, u, f, mg->cfg.nu1);
  or_residual(dim, lv->n, lv->R, lv->s, f, u, lv->d);
  or_restrict(dim, lv->n, mg->cfg.restrict_op, lv->d, cv->f);
  if (l + 1 == mg->L - 1) {
    or_mg_coarsest_solve(mg, cv->f, cv->u);
  } else {
    memset(cv->u, 0, sizeof(double) * npts(dim, cv->n));
    for (int g = 0; g < mg->cfg.gamma; ++g) cycle(mg, l + 1, cv->u, cv->f);
  }
  or_prolong_add(dim, lv->n, mg->cfg.prolong, cv->u, u);
  smooth(mg, l, u, f, mg->cfg.nu2);
}

void or_mg_cycle(or_mg *mg, double *u, const double *f) {
  if (mg->L == 1) {
    or_mg_coarsest_solve(mg, f, u);
    return;
  }
  cycle(mg, 0, u, f);
}

int or_mg_solve(or_mg *mg, double *u, const double *f, double rtol, int max_cycles, double *hist) {
  or_level *lv = &mg->lev[0];
  int dim = mg->cfg.dim;
  double fn = or_norm(dim, lv->n, f);
  int c = 0;
  for (;;) {
    or_residual(dim, lv->n, lv->R, lv->s, f, u, lv->d);
    double rel = fn > 0.0 ? or_norm(dim, lv->n, lv->d) / fn : 0.0;
    if (hist) hist[c] = rel;
    if (rel <= rtol || c == max_cycles) break;
    or_mg_cycle(mg, u, f);
    ++c;
  }
  return c;
}
