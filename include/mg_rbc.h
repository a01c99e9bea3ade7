/* mg_rbc.h -- red-black coarsening multigrid for the two-dimensional Poisson equation.
 *
 * Liu & Henshaw, Multigrid with Nonstandard Coarsening, section 4.3 (Theorem 3: red-black
 * smoothing, red-black coarsening with the transfers of eq. transfer_r2 and the Galerkin
 * coarse operator of eq. L_G1 make a two-level direct solver) and section 4.4 (the
 * multi-level cycle with the G1 and Gn coarse operators).
 *
 * Problem: the second-order five-point operator (1/h^2)[-1; -1 4 -1; -1] (eq. L_h_2) on the
 * unit square with n x n points, n - 1 a power of two, h = 1/(n - 1), Dirichlet values on
 * the boundary.  Every grid function is an n x n row-major array of doubles in device
 * memory (index i*n + j); the boundary entries of u hold the Dirichlet values and are
 * never changed, those of f are ignored.
 *
 * Levels: level 0 is the fine grid; the coarse grid of a level is its black points, so
 * level 1 is the rotated grid of spacing sqrt(2) h (the level-0 points with an even index
 * sum), level 2 the standard grid of spacing 2h, and so on.  Level l is stored on the
 * standard grid of spacing 2^(l/2) h that holds it: mg_rbc_level_size(l) = (n - 1)/2^(l/2)
 * + 1 points a side.  An odd (rotated) level's points are those with an even index sum,
 * and its arrays keep only them: m rows of pitch mg_rbc_level_pitch(l) = (m + 1)/2, point
 * (i, j) at i*pitch + j/2 (the last entry of an odd row is padding, kept zero).  An even
 * level's arrays are m x m (pitch m).  Within a level the C points
 * (black) are those kept on the next level (even index sum on an even level, both indices
 * even on an odd one) and the F points (red) the others.
 *
 * Coarse operators (stencils on a level's own axes; on an odd level these are the
 * storage diagonals, H^2 = 2 s^2 for storage spacing s):
 *   MG_RBC_NG  the five-point operator rediscretized on every coarse level;
 *   MG_RBC_G1  the first Galerkin stencil (1/4H^2)[-1 -2 -1; -2 12 -2; -1 -2 -1]
 *              (eq. L_G1) on every coarse level;
 *   MG_RBC_GN  eq. L_G1 on level 1, the rediscretized operator below.
 * Beyond the boundary a coarse-level stencil takes the odd reflection of the grid
 * function about the boundary line (the Galerkin product of the bounded grid).
 *
 * Cycle (levels >= 2): nu1 red-black sweeps (omega-Jacobi on the F points, then on the C
 * points), the defect restricted with (1/8)[. 1 .; 1 4 1; . 1 .] onto the C points,
 * gamma cycles on the next level from a zero guess (on the last level one exact solve by
 * the inverse formed at set-up), the correction interpolated with (1/4)]. 1 .; 1 4 1; . 1 .[ (C points copy, F
 * points take the mean of their four C neighbours) and added, nu2 sweeps.  The levels of
 * side <= 33 (environment MG_RBC_TAIL: another side, 0 for none) run in one workgroup
 * launch per visit, with the same arithmetic as the per-level kernels.
 *
 * Status codes and mg_last_error() are those of mg.h.  Every call is asynchronous on the
 * handle's stream unless it returns a host value.  Calls on one handle must not overlap.
 */
#ifndef MG_RBC_H
#define MG_RBC_H

#include "mg.h"

#ifdef __cplusplus
extern "C" {
#endif

enum { MG_RBC_NG = 0, MG_RBC_G1 = 1, MG_RBC_GN = 2 };

/* Most unknowns of the coarsest level, whose inverse is formed at set-up and applied in
 * one workgroup. */
#define MG_RBC_MAX_COARSEST 256

typedef struct mg_rbc_config {
  int n;           /* points a side, n - 1 a power of two, n >= 3 */
  int levels;      /* >= 2; the last level must have 1..MG_RBC_MAX_COARSEST unknowns */
  int coarse;      /* MG_RBC_NG, MG_RBC_G1 or MG_RBC_GN */
  int gamma;       /* 1 = V-cycle, 2 = W-cycle */
  int nu1, nu2;    /* red-black sweeps before and after the coarse-level correction, 0..8 */
  double omega;    /* relaxation of both partial steps; 0 selects 1 (Theorem 3) */
  double rtol;     /* mg_rbc_solve stops when ||f - L u|| <= rtol ||f - L u0|| */
  int max_cycles;  /* mg_rbc_solve's cycle limit, 1..MG_MAX_HISTORY */
} mg_rbc_config;

typedef struct mg_rbc_ctx mg_rbc_ctx;

/* Validates cfg (MG_EINVAL with a message), allocates the level arrays (MG_ENOMEM) on the
 * current device and binds the handle to `stream` (a hipStream_t, 0 = default). */
mg_status mg_rbc_setup(const mg_rbc_config *cfg, void *stream, mg_rbc_ctx **out);
void mg_rbc_destroy(mg_rbc_ctx *h);

/* Side m of level l's storage grid, or -1 if l is out of range. */
int mg_rbc_level_size(const mg_rbc_ctx *h, int level);
/* Row pitch of level l's arrays (m, or (m + 1)/2 on a rotated level), or -1. */
int mg_rbc_level_pitch(const mg_rbc_ctx *h, int level);

/* `ncycles` cycles on u (device, n*n, updated in place) for right-hand side f. */
mg_status mg_rbc_cycles(mg_rbc_ctx *h, const double *f, double *u, int ncycles);

/* Cycles until the relative residual reaches rtol or max_cycles; blocks.  hist (host,
 * max_cycles + 1 entries, may be NULL) receives the residual norm before each cycle and
 * after the last; *cycles the number run.  MG_ENOCONV if rtol was not reached,
 * MG_ENUMERIC on a NaN or Inf norm. */
mg_status mg_rbc_solve(mg_rbc_ctx *h, const double *f, double *u, int *cycles, double *hist);

/* sqrt(mean over the interior of (f - L_0 u)^2) into *out (host); blocks. */
mg_status mg_rbc_residual_norm(mg_rbc_ctx *h, const double *f, const double *u, double *out);

/* Single steps on the arrays of one level (device, m x pitch doubles), for testing.
 * smooth: one omega-Jacobi partial step on the F points (colour 1) or the C points
 *   (colour 2) from u_in into u_out (every other entry copied); u_in != u_out.
 * restrict: the defect f - L_l u restricted onto level l + 1's grid into f_coarse (zero
 *   off its unknowns; the padding of a packed f_coarse is left as it is, zero in the
 *   handle's own arrays); l < levels - 1.
 * prolong: u_out = u_in + the interpolated level l + 1 correction e_coarse; in place
 *   allowed; l < levels - 1.
 * coarsest: the exact solve of the last level's equation into u (zero off the unknowns);
 *   f may be the same array as u. */
mg_status mg_rbc_kernel_smooth(mg_rbc_ctx *h, int level, int colour, const double *f,
                               const double *u_in, double *u_out);
mg_status mg_rbc_kernel_restrict(mg_rbc_ctx *h, int level, const double *f, const double *u,
                                 double *f_coarse);
mg_status mg_rbc_kernel_prolong(mg_rbc_ctx *h, int level, const double *e_coarse,
                                const double *u_in, double *u_out);
mg_status mg_rbc_kernel_coarsest(mg_rbc_ctx *h, const double *f, double *u);

#ifdef __cplusplus
}
#endif

#endif /* MG_RBC_H */
