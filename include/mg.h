/*
 * mg.h -- C ABI of the MI355X multigrid library for fourth-order finite-difference
 * Poisson problems.
 *
 * Method: K. Liu, W. D. Henshaw, "Multigrid with Nonstandard Coarsening".  The library
 * solves L_h u = f for L_h = -Delta_h on [0,1]^dim (section 2.1 problem statement;
 * section 2.3 eq. L_h_2d_4o for the fourth-order operator, its 3D analogue the sum of
 * the three axis operators) with homogeneous Dirichlet boundary values, by the
 * (lmax+1)-level gamma-cycle of section 2.2: omega-Jacobi smoothing, full-weighting
 * restriction of the defect (section 3.1 eq. transfer_2d), exact solve on the coarsest
 * level, cubic (appendix A.4) or linear interpolation of the correction, and either
 * rediscretized coarse operators (eq. L_H_4n_2d) or Galerkin coarse operators
 * R * L * P (eqs. L_H_G, L_H_4G).  Coarse grids come from standard coarsening
 * (eq. G_H_d).
 *
 * Grids.  A level of side n holds n points per axis including both boundary points,
 * x_i = i h, h = 1/(n-1), n = 2^k + 1.  Arrays are dense, x fastest:
 * index (k*n + j)*n + i (2D: j*n + i).  Boundary entries are the (zero) Dirichlet data.
 * The width-5 stencils reach one point past the boundary; the library reads that
 * value as the odd reflection u(-i) = -u(i) (the paper's analysis is on periodic or
 * infinite grids and gives no closure for wide stencils at a Dirichlet boundary).
 *
 * Memory.  Every pointer named "device" is GPU memory of the device current when the
 * handle was set up (for instance a torch tensor's data_ptr()).  The caller owns f and
 * u; the handle owns every hierarchy buffer.  All work is ordered on the HIP stream
 * given to mg_setup.  No entry point allocates memory except mg_setup.
 *
 * Errors.  Every entry point returns an mg_status; on failure mg_last_error() gives a
 * message (per calling thread).  A handle is used by one thread at a time.
 */
#ifndef MG_H
#define MG_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct mg_ctx *mg_handle;

typedef enum {
  MG_OK = 0,
  MG_EINVAL = 1,    /* bad configuration or argument */
  MG_ENOMEM = 2,    /* device allocation failed or the footprint exceeds the budget */
  MG_EDEVICE = 3,   /* a HIP runtime call failed */
  MG_ENOCONV = 4,   /* rtol not reached: max_cycles reached, the residual grew, or it stopped
                       decreasing at the rounding floor (floor_hit); result still filled */
  MG_ENUMERIC = 5,  /* the residual norm is NaN or Inf */
  MG_EBUSY = 6      /* an asynchronous solve on the handle has not finished */
} mg_status;

typedef enum {
  MG_COARSE_NG = 0,        /* rediscretized: the fine stencil at the coarse spacing (eq. L_H_4n_2d) */
  MG_COARSE_GALERKIN = 1,  /* R * L_l * P built at setup, level by level (eq. L_H_4G) */
  /* Second-order coarse operators for a fourth-order fine operator (section 3.1): */
  MG_COARSE_NG2 = 2,       /* the second-order operator at every coarse spacing (eq. L_H_2d) */
  MG_COARSE_G2 = 3         /* level 1: R * L_h^(2) * P with the second-order operator at the finest
                            * spacing (eq. L_H_2G_2d); below it R * L_l * P, level by level */
} mg_coarse;

typedef enum {
  MG_SMOOTH_JACOBI = 0,  /* omega-Jacobi: every interior point relaxed at once (section 5.3) */
  MG_SMOOTH_RBJ = 1,     /* omega red-black Jacobi (section 3.1 eq. S_rb with the Jacobi partial
                          * step; the smoother of appendix A.4.1): the red points (odd index sum
                          * i+j(+k)) take an omega-Jacobi step, then the black points from the
                          * updated red values; one such pair counts once in nu1, nu2 */
  MG_SMOOTH_RBGS = 2     /* omega red-black Gauss-Seidel (section 3.1 eqs. S_rb, S_GS): each
                          * partial step sweeps its colour in lexicographic order (x fastest),
                          * a point reading the new values of the same-colour points before it
                          * (L+ = a_0/omega plus the entries at -2 e_x, -2 e_y); 2D only, with
                          * rediscretized coarse operators (MG_COARSE_NG or MG_COARSE_NG2, cross
                          * stencils on every level), else MG_EINVAL */
} mg_smoother;

typedef enum {
  MG_PREC_FP64 = 0,   /* every step in FP64 */
  MG_PREC_MIXED = 1   /* FP32 cycles inside FP64 iterative refinement (FP64 outer residual,
                         correction and coarsest solve) */
} mg_precision;

typedef struct {
  int dim;             /* 2 or 3 */
  int n;               /* points per axis incl. boundary, 2^k + 1, reaching n_coarsest */
  int order;           /* 4 (fourth order, width-5 stencil), 2 (5-/7-point) or 6 (sixth order,
                          width-7 stencil, section 3.3 eq. LhOrder6) */
  int coarse;          /* mg_coarse */
  int smoother;        /* mg_smoother */
  double omega;        /* relaxation; <= 0 selects the Fourier-analysis optimum:
                          omega-Jacobi (any coarse operator) 10/13 in 2D, 9/11 in 3D for order
                          4 (4/5, 6/7 for order 2; 490/653, 147/185 for order 6), by
                          equioscillation; the red-black smoothers the minimiser of the
                          two-grid factor of V(2,1) with cubic interpolation, per coarse
                          operator (NG, GALERKIN, NG2, G2): red-black Jacobi, order 4:
                          2D 1.13, 1.00, 0.98, 0.97; 3D 1.17, 1.09, 1.09, 1.08 (order 6: 2D
                          1.13, 1.02, 0.99, 0.99; 3D 1.15, 1.10, 1.09, 1.08; order 2: 2D 1.00,
                          0.98; 3D 1.13, 1.09); red-black Gauss-Seidel (2D): NG 1.16, NG2 0.98
                          for order 4 (1.18, 1.00 for order 6; 1.00 for order 2) */
  int nu1, nu2;        /* pre- and post-smoothing sweeps per cycle (nu1 + nu2 >= 1) */
  int gamma;           /* 1 = V cycle, 2 = W cycle */
  int prolong;         /* 3 = cubic interpolation, 1 = (bi/tri)linear */
  int restrict_op;     /* 1 = full weighting (section 3.1 eq. transfer_2d); 3 = the cubic
                          interpolation's adjoint (appendix A.4, the 1/1024 operator), with
                          rediscretized coarse operators only (MG_COARSE_NG, MG_COARSE_NG2) */
  int n_coarsest;      /* side of the coarsest level (exact dense solve), e.g. 9 */
  int precision;       /* mg_precision */
  double rtol;         /* stop when ||f - L u||_h <= rtol ||f||_h */
  int max_cycles;      /* FP64: cycle cap; MIXED: cap on refinement steps */
  int inner_cycles;    /* MIXED: FP32 cycles per refinement step */
} mg_config;

#define MG_MAX_HISTORY 512

typedef struct {
  int cycles;          /* multigrid cycles run (MIXED: FP32 inner cycles) */
  int outer_steps;     /* MIXED: refinement steps run; FP64: 0 */
  int status;          /* 1 converged, 2 cycle cap, 3 rounding floor, 4 non-finite, 5 growth */
  int floor_hit;       /* 1 when the residual stopped decreasing above rtol */
  double rel_residual; /* final ||f - L u||_h / ||f||_h (FP64, difference form) */
  double conv_factor;  /* last residual ratio between successive checks */
  int history_len;     /* entries in history */
  double history[MG_MAX_HISTORY]; /* relative residual before each cycle (FP64) or each
                                     refinement step (MIXED), and after the last */
} mg_result;

/* Set-up of the multigrid hierarchy (section 2.2, the levels l = 0..lmax of standard
 * coarsening, eq. G_H_d): validates cfg, forms every level's operator (rediscretized,
 * eq. L_H_4n_2d / L_H_2d, or the Galerkin product R L_l P of eqs. L_H_G, L_H_4G,
 * L_H_2G_2d, kept as 1D factors), the relaxation weight (the Fourier-analysis optimum
 * of section 5.3 unless cfg->omega > 0), the exact coarsest-level solve, and allocates
 * every device buffer on the current device.  hip_stream: a hipStream_t (NULL = the
 * default stream); all later work of the handle is ordered on it.  On failure *out is
 * NULL and nothing is leaked (MG_EINVAL for a bad cfg, MG_ENOMEM, MG_EDEVICE). */
mg_status mg_setup(const mg_config *cfg, void *hip_stream, mg_handle *out);

/* Device bytes a handle for cfg allocates: the per-level arrays of the section 2.2
 * hierarchy (u, f and a sweep target per level; level 0 FP64 u and f are the caller's),
 * the coarsest-level solve tables and the reduction partials.  Exact, so a caller can
 * admit work by HBM footprint.  0 for an invalid cfg. */
size_t mg_footprint_bytes(const mg_config *cfg);

/* Solves L u = f by repeated gamma-cycles (section 2.2, the multigrid algorithm; its
 * loop read as "while ||f - L u||_h / ||f||_h > rtol and fewer than max_cycles"), or,
 * for MIXED precision, by FP64 refinement steps around FP32 cycles.  f, u: device FP64
 * arrays of n^dim values (caller-owned); u holds the initial guess on entry and the
 * solution on exit; f is read only.  The relative residual is checked on the device
 * before every cycle (step).  Stops at rtol (MG_OK), at max_cycles, on growth, or at the
 * FP64 rounding floor above rtol (two checks in a row above 0.9 x the best so far:
 * res->floor_hit = 1); all three return MG_ENOCONV with res filled.  A NaN or Inf
 * residual returns MG_ENUMERIC.  res may be NULL.  Returns after the solve finished. */
mg_status mg_solve(mg_handle h, const double *f, double *u, mg_result *res);

/* Runs exactly ncycles gamma-cycles of section 2.2 (MIXED: ncycles refinement steps)
 * with no stopping test, recording the residual before each and after the last.  For
 * measurement and parity checks at a fixed cycle count.  MG_OK unless an argument is
 * bad (MG_EINVAL), a HIP call fails, or the residual is not finite (MG_ENUMERIC). */
mg_status mg_run_cycles(mg_handle h, const double *f, double *u, int ncycles, mg_result *res);

/* Stream-ordered form of mg_solve (the same section 2.2 iteration and stopping rule):
 * enqueues max_cycles + 1 steps on the handle's stream, each returning at once on the
 * device after the stopping test has fired, and returns without waiting.  f and u must
 * stay valid until mg_query reports completion.  MG_EBUSY if a previous asynchronous
 * solve on the handle has not been collected by mg_query. */
mg_status mg_solve_async(mg_handle h, const double *f, double *u);

/* After mg_solve_async: MG_EBUSY while running, else the solve's status and res. */
mg_status mg_query(mg_handle h, mg_result *res);

/* rel = ||f - L u||_h / ||f||_h in FP64 on the device (difference form). */
mg_status mg_residual_norm(mg_handle h, const double *f, const double *u, double *rel);

/* ---- for callers that cannot allocate device memory ----
 * Code under HIP graph capture, tight serving loops and harnesses that forbid hipMalloc.
 * The library's static scratch (a solve state and per-block partial sums) has this many
 * bytes, one copy per device, held from the library's load to the end of the process. */
#define MG_NOALLOC_SCRATCH_BYTES (8u << 20)

/* mg_residual_norm without a handle and without allocating: *rel = ||f - L_h u||_h /
 * ||f||_h (||f - L_h u||_h when f = 0), L_h the order-`order` operator at spacing
 * 1/(n-1), on the current device, ordered on hip_stream (a hipStream_t, NULL = default
 * stream), not waited for.  f, u: device FP64 arrays of n^dim values; rel: device pointer
 * to one double, written when the stream reaches it.  The same kernels and summation
 * order as mg_residual_norm, so the same value bit for bit.  Limits: n = 2^k + 1, k >= 3,
 * and the partial sums of the norm passes must fit the scratch: n <= 16385 in 2D,
 * n <= 1025 in 3D; beyond them MG_EINVAL, before any device work.  Calls on one device
 * share its scratch, which keeps the last call's contents: calls that overlap on a
 * device (other streams or threads) race; calls ordered on one stream do not. */
mg_status mg_residual_norm_noalloc(int dim, int n, int order, const double *f, const double *u,
                                   double *rel, void *hip_stream);

/* Releases every buffer of the handle (waits for its stream first). */
mg_status mg_destroy(mg_handle h);

/* Message of the last failure on this thread ("" if none). */
const char *mg_last_error(void);

/* ---- component entry points: one hot-path step on level `level` of a handle ----
 * Arrays are the level's dense n_l^dim layout; fp32 = 1 selects float arrays (the FP32
 * kernels of MIXED precision), else double.  They launch on the handle's stream and
 * return without waiting. */

/* Side n_l of level l (0 = finest), or -1. */
int mg_level_size(mg_handle h, int level);

/* One omega-Jacobi sweep u_out = u_in + omega/a_0 (f - L_l u_in) (section 5.3 smoother
 * with a_0 the centre coefficient of L_l).  u_in == NULL means u_in = 0.
 * u_out != u_in. */
mg_status mg_kernel_smooth(mg_handle h, int level, int fp32, const void *f, const void *u_in,
                           void *u_out);

/* One partial step of red-black smoothing (section 3.1 eq. S_rb): the points of one colour
 * take the omega-Jacobi step of mg_kernel_smooth, every other point copies u_in.  On a
 * MG_SMOOTH_RBGS handle's radius-2/3 cross levels the step is the Gauss-Seidel one of eq.
 * S_GS instead (colour 1 or 2 only, u_in not NULL).
 * colour 1 = red (odd index sum i+j(+k)), 2 = black (even), 0 = every point.  A red-black
 * sweep is colour 1 into a second array, then colour 2 back; colour 3 runs the whole
 * red-black sweep in one pass (2D: every level; 3D: levels with the cross operator, else
 * MG_EINVAL).  u_in == NULL means u_in = 0.  u_out != u_in. */
mg_status mg_kernel_smooth_colour(mg_handle h, int level, int fp32, int colour, const void *f,
                                  const void *u_in, void *u_out);

/* r = f - L_l u (the defect of section 2.2), zero on the boundary. */
mg_status mg_kernel_residual(mg_handle h, int level, int fp32, const void *f, const void *u,
                             void *r);

/* fc = I_h^H (f - L_l u) on level l+1: defect and full weighting in one pass; with the
 * cubic-adjoint restriction (restrict_op = 3) the defect first goes to the handle's level-l
 * sweep target (a mixed-precision handle then takes fp32 = 1 only). */
mg_status mg_kernel_residual_restrict(mg_handle h, int level, int fp32, const void *f,
                                      const void *u, void *fc);

/* u_out = u_in + I_H^h v, v on level l+1 (interpolation and correction in one pass);
 * u_out may equal u_in. */
mg_status mg_kernel_prolong_correct(mg_handle h, int level, int fp32, const void *v,
                                    const void *u_in, void *u_out);

/* The pre-coarse half of a cycle on level l in one pass (2D): u_out = nu1 omega-Jacobi
 * sweeps of u_in (NULL = zero guess), fc = I_h^H (f - L_l u_out) on level l+1.
 * u_out != u_in.  With red-black smoothing the pass holds min(1, nu1) red-black sweeps:
 * the last pass of the cycle's pre-coarse half (the cycle runs max(1, nu1) passes). */
mg_status mg_kernel_presmooth_restrict(mg_handle h, int level, int fp32, const void *f,
                                       const void *u_in, void *u_out, void *fc);

/* The post-coarse half of a cycle on level l in one pass (2D): u_out = nu2 omega-Jacobi
 * sweeps of (u_in + I_H^h v).  u_out != u_in.  With red-black smoothing the pass holds
 * min(1, nu2) red-black sweeps: the first pass of the cycle's post-coarse half. */
mg_status mg_kernel_prolong_postsmooth(mg_handle h, int level, int fp32, const void *v,
                                       const void *u_in, const void *f, void *u_out);

/* v = L_c^{-1} g on the coarsest level (FP64 arithmetic for either storage type). */
mg_status mg_kernel_coarsest_solve(mg_handle h, int fp32, const void *g, void *v);

/* Level-l operator as 1D factors: L_l = sum over axes of a (along the axis) times b
 * (along every other axis).  Writes 7 coefficients each (offsets -3..3). */
mg_status mg_level_operator(mg_handle h, int level, double a[7], double b[7]);

/* Blocks until the handle's stream is idle. */
mg_status mg_synchronize(mg_handle h);

#ifdef __cplusplus
}
#endif
#endif
