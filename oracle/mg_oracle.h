/*
 * mg_oracle.h -- plain FP64 CPU reference multigrid (TEST INFRASTRUCTURE ONLY).
 *
 * This library exists to check the GPU library against the paper.  Only the
 * test suite, the smoke check and the CPU-baseline leg of the benchmark may
 * load it; the GPU product path never calls, links or includes anything here,
 * and nothing here includes anything from the GPU library.
 *
 * Paper: K. Liu, W. D. Henshaw, "Multigrid with Nonstandard Coarsening".
 *
 * Grids (section 2.4, eq. G_h_N, read for Dirichlet problems): a level holds
 * n points per axis including both boundary points, x_i = i*h, h = 1/(n-1),
 * stored dense with x fastest (index = (k*n + j)*n + i in 3D).  Interior points
 * are 1..n-2 on every axis; boundary values are the homogeneous Dirichlet data
 * (zero).  Wide stencils reach one point past the boundary; those values are
 * the odd reflection u(-i) = -u(i) of the grid function (a reading: the paper
 * computes with periodic grids and gives no closure for wide stencils).
 *
 * Stencils are dense arrays of (2R+1)^dim coefficients in the paper's
 * [a_j] notation (section 2.1, eq. bra): (L u)(x) = sum_j a_j u(x + j h),
 * offset index ((jz+R)*(2R+1) + (jy+R))*(2R+1) + (jx+R).
 */
#ifndef MG_ORACLE_H
#define MG_ORACLE_H

#ifdef __cplusplus
extern "C" {
#endif

#define OR_MAX_RADIUS 6
#define OR_MAX_LEVELS 16

/* Transfer operator identifiers. */
#define OR_RESTRICT_FW 1    /* full weighting, section 3.1 eq. transfer_2d (tensor product in 3D) */
#define OR_RESTRICT_CUBIC 3 /* adjoint of cubic interpolation, appendix A.4 (the 1/1024 operator) */
#define OR_PROLONG_LINEAR 1 /* (bi/tri)linear interpolation, section 3.1 eq. transfer_2d */
#define OR_PROLONG_CUBIC 3  /* cubic interpolation, appendix A.4 (the 1/256 operator) */

#define OR_COARSE_NG 0       /* rediscretized: same stencil at the coarse spacing (eq. L_H_4n_2d) */
#define OR_COARSE_GALERKIN 1 /* L_{l+1} = R L_l P, built recursively (eq. L_H_4G, section 2.4) */
#define OR_COARSE_NG2 2      /* second-order operator at every coarse spacing (section 3.1, eq. L_H_2d) */
#define OR_COARSE_G2 3       /* L_1 = R L_h^(2) P from the second-order operator at the finest
                              * spacing (section 3.1, eq. L_H_2G_2d), then L_{l+1} = R L_l P */

/* Smoother identifiers. */
#define OR_SMOOTH_JACOBI 0 /* omega-Jacobi (section 5.3) */
#define OR_SMOOTH_RBJ 1    /* omega red-black Jacobi: section 3.1 eq. S_rb, S = S^B S^R, with the
                            * Jacobi partial step on each colour (the smoother appendix A.4.1
                            * uses); red = odd index sum i+j(+k), black = even */
#define OR_SMOOTH_RBGS 2   /* omega red-black Gauss-Seidel: section 3.1 eqs. S_rb and S_GS, the
                            * partial step on a colour -(L+)^{-1} L- with L+ the centre over
                            * omega plus the same-colour entries that precede the point in
                            * lexicographic order (x fastest): an in-place sweep of the colour's
                            * points in that order */

typedef struct {
  int dim;          /* 2 or 3 */
  int n;            /* finest points per axis incl. boundary, 2^k+1 */
  int order;        /* 2, 4 or 6: order of the finest-level operator */
  int coarse;       /* OR_COARSE_NG, OR_COARSE_GALERKIN, OR_COARSE_NG2 or OR_COARSE_G2 */
  int restrict_op;  /* OR_RESTRICT_FW or OR_RESTRICT_CUBIC */
  int prolong;      /* OR_PROLONG_LINEAR or OR_PROLONG_CUBIC */
  int nu1, nu2;     /* pre- and post-smoothing sweeps */
  int gamma;        /* 1 = V cycle, 2 = W cycle */
  int n_coarsest;   /* points per axis of the coarsest level, e.g. 9 */
  double omega;     /* omega-Jacobi relaxation parameter, same on every level */
  int smoother;     /* OR_SMOOTH_JACOBI, OR_SMOOTH_RBJ or OR_SMOOTH_RBGS; a sweep (both colours
                     * of a red-black one) counts once in nu */
} or_config;

/* Number of levels n, (n-1)/2+1, ... down to n_coarsest; 0 if n does not reach it. */
int or_num_levels(int n, int n_coarsest);

/* Finest-level operator -Delta_h of the given order (2: eq. L_h_2, 4: eq. L_h_2d_4o,
 * 6: section 3.3 eq. LhOrder6), in dim dimensions as the sum of the 1D operators along
 * each axis.  Writes (2R+1)^dim coefficients with R = order/2 and returns R. */
int or_fine_stencil(int dim, int order, double h, double *s);

/* Galerkin coarse stencil R * L * P on the infinite grid (eq. L_H_G), computed by its
 * definition: for every coarse offset J, interpolate the coarse unit function at J,
 * apply the fine stencil, restrict at coarse point 0.  Returns the coarse radius and
 * writes (2Rc+1)^dim coefficients to sc (caller provides (2*OR_MAX_RADIUS+1)^dim). */
int or_galerkin_stencil(int dim, int Rf, const double *sf, int restrict_op, int prolong,
                        double *sc);

/* The operator functions below require a stencil whose coefficients sum to zero (true
 * for every operator of the method) and evaluate L u = sum_{k != 0} c_k (u(x+k) - u(x)).
 * out = L u on interior points, 0 on the boundary. */
void or_apply(int dim, int n, int R, const double *s, const double *u, double *out);
/* d = f - L u on interior points (the defect of section 2.2), 0 on the boundary. */
void or_residual(int dim, int n, int R, const double *s, const double *f, const double *u,
                 double *d);
/* One omega-Jacobi sweep u_out = u + omega/a_0 * (f - L u), a_0 = centre coefficient
 * (section 5.3 smoother with the diagonal of the operator in use). */
void or_jacobi(int dim, int n, int R, const double *s, double omega, const double *f,
               const double *u, double *u_out);
/* One omega-Jacobi partial step on one colour: at interior points whose index sum
 * i+j(+k) is odd (colour 1, red) or even (colour 2, black) u_out = u + omega/a_0 (f - L u);
 * every other point keeps u.  Colour 0 updates every interior point (or_jacobi). */
void or_jacobi_colour(int dim, int n, int R, const double *s, double omega, int colour,
                      const double *f, const double *u, double *u_out);
/* One omega Gauss-Seidel partial step on one colour (section 3.1 eq. S_GS): u_out = u, then
 * the interior points of the colour, in lexicographic order (x fastest, then y, then z),
 * are replaced in u_out one at a time by u_out + omega/a_0 (f - L u_out), L evaluated on
 * the current u_out (values beyond the boundary are odd reflections of current values).
 * Points of the other colour are not changed.  Colour 0: every interior point. */
void or_gs_colour(int dim, int n, int R, const double *s, double omega, int colour,
                  const double *f, const double *u, double *u_out);
/* fc = I_h^H d on the coarse grid of nc = (nf-1)/2+1 points (standard coarsening). */
void or_restrict(int dim, int nf, int restrict_op, const double *d, double *fc);
/* u += I_H^h v, v on the coarse grid of nc = (nf-1)/2+1 points. */
void or_prolong_add(int dim, int nf, int prolong, const double *v, double *u);
/* Discrete norm ||v||_h = sqrt(h^dim * sum over interior points of v^2) (section 2.1). */
double or_norm(int dim, int n, const double *v);
/* ||f - L u||_h evaluated with long-double accumulation of every term; a reference
 * for residual norms near the FP64 rounding floor. */
double or_residual_norm_ld(int dim, int n, int R, const double *s, const double *f,
                           const double *u);

/* Multigrid hierarchy and the (lmax+1)-level gamma-cycle of section 2.2. */
typedef struct or_mg or_mg;
or_mg *or_mg_create(const or_config *cfg);
void or_mg_destroy(or_mg *m);
int or_mg_levels(const or_mg *m);
/* Level l: returns n_l and R_l and copies the (2R_l+1)^dim stencil to s (if non-null). */
int or_mg_level_stencil(const or_mg *m, int l, int *n_out, double *s);
/* One cycle on the finest level, u updated in place. */
void or_mg_cycle(or_mg *m, double *u, const double *f);
/* Exact solve on the coarsest level: v = L^{-1} g (dense LU with partial pivoting). */
void or_mg_coarsest_solve(or_mg *m, const double *g, double *v);
/* Cycle until ||f - L u||_h <= rtol ||f||_h or max_cycles cycles were done.
 * hist (size max_cycles+1, may be null) receives the relative residual before every
 * cycle and after the last one.  Returns the number of cycles performed. */
int or_mg_solve(or_mg *m, double *u, const double *f, double rtol, int max_cycles, double *hist);

/* Number of OpenMP threads the loops above use. */
int or_num_threads(void);
/* Threads of the OpenMP loops from now on (3D grids split their outermost loop). */
void or_set_num_threads(int threads);

#ifdef __cplusplus
}
#endif
#endif
