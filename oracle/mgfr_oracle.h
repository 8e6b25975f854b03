/*
 * mgfr_oracle.h -- TEST INFRASTRUCTURE, not part of the product.
 *
 * A plain, slow, double-precision CPU implementation of the multigrid solve of the
 * nonlinear f(R) scalar-field equation of Li, Zhao, Teyssier & Koyama, "ECOSMOG: An
 * Efficient Code for Simulating Modified Gravity" (arXiv:1110.1379).  It exists only to
 * check the GPU library: only the test suite, the smoke check and the CPU-baseline leg
 * of the benchmark load it.  It shares no code, header or table with the GPU library.
 *
 * All arrays are host arrays of doubles in C order [i][j][k] (k fastest), i = x.
 * Return codes: 0 ok, -1 invalid argument, -2 non-finite input, -3 not converged
 * (the last iterate and the residual history are still written).
 */
#ifndef MGFR_ORACLE_H
#define MGFR_ORACLE_H

#ifdef __cplusplus
extern "C" {
#endif

/* Model and box (Sec. II and Sec. III.A): Hu-Sawicki n, |f_R0|, Omega_m, Omega_Lambda
 * (negative -> 1 - Omega_m), scale factor a, box side B in Mpc/h. */
typedef struct {
    double omega_m, omega_l, a, n, fr0_abs, box_mpc_h;
} orc_model;

typedef struct {
    double tol;           /* stop when the rms residual of the finest grid <= tol        */
    int pre, post;        /* Newton-Gauss-Seidel sweeps before / after the coarse step   */
    int coarsest_n;       /* side of the coarsest multigrid level                        */
    int coarsest_sweeps;  /* cap on the sweeps of the coarsest level                     */
    int max_cycles;       /* V-cycle cap                                                 */
    int subtract_mean;    /* 1: density contrast rho - mean(rho); 0: rho - 1              */
    int warm_start;       /* 1: start from the u passed in; 0: from the background u     */
    double max_step;      /* > 0: bound |Newton step| per visit; 0: the plain Newton step */
    double coarsest_rtol; /* coarsest level: stop once its rms residual <= rtol x initial
                             or reaches the rounding floor; 0: always coarsest_sweeps   */
} orc_opts;

/* Derived constants, in this order:
 * [0] xi, [1] c~, [2] K=(n a^2 xi)^(1/(n+1)), [3] A=(1/3) Om a^4 K, [4] Sbar=Om a^4 (a^-3+4 OL/Om),
 * [5] D=Om a, [6] u_bar, [7] C=c~^2/(2h^2) with h=1/N. */
int orc_constants(const orc_model* m, int N, double* out8);

/* Operator and its diagonal derivative on an n^3 grid of spacing h.
 * ub == NULL: periodic grid.  ub != NULL: cube patch, ub[6][n][n] boundary values on the
 * faces (-x,+x,-y,+y,-z,+z), ghost mask ratio r (=-1 for a cube patch).
 * rho != NULL: finest-level operator with the density source, contrast rho - rho_ref.
 * rho == NULL: flux + curvature term only (coarse levels).  L or dL may be NULL. */
int orc_operator(int n, double h, const double* u, const double* rho, double rho_ref,
                 const double* ub, double r, const orc_model* m, double* L, double* dL);

/* Same, at a list of cell indices only (flat C-order indices). */
int orc_operator_at(int n, double h, const double* u, const double* rho, double rho_ref,
                    const double* ub, double r, const orc_model* m,
                    long long ncell, const long long* idx, double* L);

/* Periodic domain grid: FAS V-cycles until rms(L) <= tol.  hist has max_cycles+1 slots. */
int orc_solve(const double* rho, int N, const orc_model* m, const orc_opts* o,
              double* u, double* hist, int* nhist);

/* One cube patch of side n and spacing h with fixed boundary values ub[6][n][n]. */
int orc_solve_patch(const double* rho, int n, double h, const double* ub,
                    const orc_model* m, const orc_opts* o, double* u, double* hist, int* nhist);

/* Boundary set-up of a patch from its parent-level solution (trilinear interpolation of
 * the parent u, cell-centred 27/9/3/1 weights).  parent: side pn, origin porigin (in
 * parent-level cells), periodic flag.  child: origin (child-level cells, even), side n.
 * Writes ub[6][n][n] and the initial guess u0[n^3]. */
int orc_patch_boundary(const double* parent_u, int pn, const int* porigin, int parent_periodic,
                       const int* origin, int n, double* ub, double* u0);

/* Single-grid Newton-Gauss-Seidel (no coarse levels), for the convergence comparison.
 * Runs nsweeps red-black sweeps; hist[s] = rms residual after s sweeps (nsweeps+1 slots). */
int orc_single_grid(const double* rho, int N, const orc_model* m, int subtract_mean, double max_step,
                    double* u, int nsweeps, double* hist);

/* A refinement level with the mask scheme (Sec. V): the periodic N^3 grid of the level's
 * resolution (h = 1/N); mask[q] in [-1, 1], active (relaxed) where > 0; on entry u holds the
 * initial guess in active cells and the fixed values interpolated from the coarser level in
 * the others, and both are kept as w for the boundary values.  FAS V-cycles over coarse
 * levels with 8-child-mean masks until the rms residual over the active cells <= tol.
 * Only active cells of u change. */
int orc_solve_masked(const double* rho, const double* mask, int N, const orc_model* m, const orc_opts* o,
                     double* u, double* hist, int* nhist);

/* L and dL/du of the masked operator at active cells (0 elsewhere), with fixed values w;
 * rho == NULL: no density and background terms (coarse levels); h = 1/n. */
int orc_masked_operator(int n, const double* u, const double* w, const double* mask, const double* rho,
                        double rho_ref, const orc_model* m, double* L, double* dL);

/* Smoother cell visits (all levels) of the last solve; for timing reports only. */
long long orc_last_cell_updates(void);

/* Host threads the loops may use (OpenMP; 1 when built without it), and a new count (> 0).
 * Results do not depend on it: sums are formed per plane and added in plane order. */
int orc_threads(void);
void orc_set_threads(int nthreads);

#ifdef __cplusplus
}
#endif
#endif
