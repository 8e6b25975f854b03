/*
 * mgfr_oracle.c -- TEST INFRASTRUCTURE, not part of the product.
 *
 * Plain, slow, double-precision CPU reference for the multigrid solve of the nonlinear
 * f(R) equation of Li, Zhao, Teyssier & Koyama (ECOSMOG, arXiv:1110.1379).  Only the
 * test suite, the smoke check and the benchmark's CPU-baseline leg may load it; the GPU
 * library shares nothing with it.  Every loop is written for a reader checking it
 * against the paper, not for speed: one cell at a time, exp() evaluated where the
 * formula has it, no blocking, no fusion.  Loops whose cells do not depend on each other
 * (one colour of a red-black sweep, a residual, a restriction, a prolongation) run on
 * several host threads (OpenMP) when the grid has at least 32 planes; their sums are formed
 * per plane and the planes added in order, so every result is the same whatever the thread
 * count.
 *
 * What is computed (the paper's notation, code units, tildes dropped):
 *   f_R = -exp(u), b = exp(u)                                      (Sec. III.C)
 *   L_i(u) = c^2/(2h^2) sum_nb (b_nb + b_i)(u_nb - u_i)
 *          + (1/3) Om a^4 (n a^2 xi)^(1/(n+1)) exp(-u_i/(n+1))
 *          - Om a (rho_i - 1) - Om a^4 (a^-3 + 4 OL/Om)               (eq. discrete_fR times c^2,
 *                                                                     = eq. bc_modified_fR_op)
 *   Newton-Gauss-Seidel: u_i <- u_i - (L_i - f_i) / (dL_i/du_i)       (Sec. V.B.1)
 *   FAS: L^H(u^H) = L^H(R u^h) - R d^h,  u^h += P(u^H - R u^h)        (Sec. V.B.2, V.B.3)
 * Readings where the paper is silent (each is listed in the design notes of the repo):
 *   - density coefficient Om a, not Om a / 3 (the sine and Gaussian test solutions of
 *     Sec. VI.A and the Poisson equation of Sec. III.B fix it);
 *   - R = mean of the 8 children; P = cell-centred trilinear, weights 27/9/3/1 /64;
 *   - red cells (i+j+k even) first, then black; one Newton step per visit, no damping;
 *   - coarse levels carry no density or constant term (they cancel in the FAS equation);
 *   - convergence: rms of L over the finest cells <= tol (absolute, Sec. VI.E);
 *   - patch boundary: ghost u from trilinear interpolation of the parent u; coarse-level
 *     boundary value = mean of the four fine boundary values on that face.
 */
#include "mgfr_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_EINVAL (-1)
#define ORC_ENONFINITE (-2)
#define ORC_ENOTCONV (-3)

/* Mask ratio m_ghost / m_active of a cube patch: active cells +1, all others -1 (Sec. V). */
#define CUBE_PATCH_R (-1.0)

typedef struct {
    double xi, ct, K, A, Sbar, D, ubar, n;
} consts;

static int derive(const orc_model* m, consts* c)
{
    if (!m) return ORC_EINVAL;
    double om = m->omega_m, a = m->a, n = m->n;
    double ol = m->omega_l < 0.0 ? 1.0 - om : m->omega_l;
    if (!(om > 0.0) || !(a > 0.0) || !(n > 0.0) || !(m->fr0_abs > 0.0) || !(m->box_mpc_h > 0.0) ||
        !(ol >= 0.0) || !isfinite(om + a + n + m->fr0_abs + m->box_mpc_h + ol))
        return ORC_EINVAL;
    /* Sec. II: f_R ~ -n xi (m^2 / -R)^(n+1), -Rbar = 3 m^2 (a^-3 + 4 OL/Om); at a = 1 this is f_R0. */
    c->xi = m->fr0_abs * pow(3.0 * (1.0 + 4.0 * ol / om), n + 1.0) / n;
    /* Sec. III.A: c~ = c / (B H0) with c in km/s, H0 = 100 h km/s/Mpc, B in Mpc/h. */
    c->ct = 299792.458 / (100.0 * m->box_mpc_h);
    double q = pow(a, -3.0) + 4.0 * ol / om;
    c->K = pow(n * a * a * c->xi, 1.0 / (n + 1.0));
    c->A = om * pow(a, 4.0) * c->K / 3.0;
    c->Sbar = om * pow(a, 4.0) * q;
    c->D = om * a;
    /* Sec. VI.A.1: background f~_R = -n a^2 xi / [3 (a^-3 + 4 OL/Om)]^(n+1) = -exp(u_bar). */
    c->ubar = log(n * a * a * c->xi / pow(3.0 * q, n + 1.0));
    c->n = n;
    return 0;
}

int orc_constants(const orc_model* m, int N, double* out8)
{
    consts c;
    if (derive(m, &c) != 0 || N < 1 || !out8) return ORC_EINVAL;
    double h = 1.0 / N;
    out8[0] = c.xi;
    out8[1] = c.ct;
    out8[2] = c.K;
    out8[3] = c.A;
    out8[4] = c.Sbar;
    out8[5] = c.D;
    out8[6] = c.ubar;
    out8[7] = c.ct * c.ct / (2.0 * h * h);
    return 0;
}

/* ----------------------------------------------------------------------------------- */
/* One grid: a periodic box (ub == NULL) or a cube patch with boundary values ub.       */

typedef struct {
    int n;
    double h, C;          /* spacing and c~^2 / (2 h^2) */
    const double* ub;     /* [6][n][n] or NULL */
    double r;             /* ghost mask ratio */
    const double* rho;    /* finest level only */
    double rho_ref;
} grid;

static long long at(int n, int i, int j, int k) { return ((long long)i * n + j) * n + k; }

static const int DI[6] = {-1, 1, 0, 0, 0, 0};
static const int DJ[6] = {0, 0, -1, 1, 0, 0};
static const int DK[6] = {0, 0, 0, 0, -1, 1};

/* Boundary value stored for face f of face cell (i,j,k); faces -x,+x,-y,+y,-z,+z. */
static double face_value(const grid* g, int f, int i, int j, int k)
{
    int n = g->n, p, q;
    if (f < 2) { p = j; q = k; }
    else if (f < 4) { p = i; q = k; }
    else { p = i; q = j; }
    return g->ub[((long long)f * n + p) * n + q];
}

/* L_i and dL_i/du_i at one cell (eq. bc_modified_fR_op and eq. bc_modified_fR_dop). */
static double cell_op(const grid* g, const consts* c, const double* u, int i, int j, int k,
                      double* dop)
{
    int n = g->n;
    double ui = u[at(n, i, j, k)];
    double bi = exp(ui);
    double L = 0.0, dL = 0.0;
    for (int f = 0; f < 6; ++f) {
        int ii = i + DI[f], jj = j + DJ[f], kk = k + DK[f];
        int outside = ii < 0 || ii >= n || jj < 0 || jj >= n || kk < 0 || kk >= n;
        if (outside && g->ub) {
            /* Ghost cell beyond a refinement boundary (eq. u_i-1jk):
               u_g = u_b - r u_b + r u_i, and b_g = exp(u_g) (b is not interpolated). */
            double ubv = face_value(g, f, i, j, k);
            double ug = (1.0 - g->r) * ubv + g->r * ui;
            double bg = exp(ug);
            L += g->C * (bg + bi) * (ug - ui);
            /* chain rule with du_g/du_i = r and db_g/du_i = r b_g */
            dL += g->C * ((g->r * bg + bi) * (ug - ui) + (bg + bi) * (g->r - 1.0));
        } else {
            /* stored neighbour; the domain grid is periodic */
            ii = (ii + n) % n;
            jj = (jj + n) % n;
            kk = (kk + n) % n;
            double un = u[at(n, ii, jj, kk)];
            double bn = exp(un);
            /* face coefficient b_{i+1/2} = (b_nb + b_i)/2 (Sec. IV), times c~^2/h^2 */
            L += g->C * (bn + bi) * (un - ui);
            dL += g->C * (bi * (un - ui) - bn - bi);
        }
    }
    double S = c->A * exp(-ui / (c->n + 1.0));
    L += S;
    dL -= S / (c->n + 1.0);
    if (g->rho) L -= c->D * (g->rho[at(n, i, j, k)] - g->rho_ref) + c->Sbar;
    if (dop) *dop = dL;
    return L;
}

/* Cell visits of the smoother since the last solve started (reported for timing only). */
static long long g_updates = 0;

long long orc_last_cell_updates(void) { return g_updates; }

int orc_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

void orc_set_threads(int nthreads)
{
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#else
    (void)nthreads;
#endif
}

/* Sum of per-plane partial sums, planes in order. */
static double sum_planes(const double* plane, int n)
{
    double s = 0.0;
    for (int i = 0; i < n; ++i) s += plane[i];
    return s;
}

/* Red-black Newton-Gauss-Seidel sweep: red (i+j+k even) first (Sec. V.B.1). */
static void ngs_sweep(const grid* g, const consts* c, double* u, const double* f, double max_step)
{
    int n = g->n;
    g_updates += (long long)n * n * n;
    /* a cell of one colour reads only cells of the other colour: its colour's cells can be
       visited in any order */
    for (int colour = 0; colour < 2; ++colour)
#pragma omp parallel for schedule(static) if (n >= 32)
        for (int i = 0; i < n; ++i)
            for (int j = 0; j < n; ++j)
                for (int k = 0; k < n; ++k) {
                    if (((i + j + k) & 1) != colour) continue;
                    double d;
                    double L = cell_op(g, c, u, i, j, k, &d);
                    if (f) L -= f[at(n, i, j, k)];
                    double step = -L / d;
                    /* optional bound on the Newton step (max_step > 0); the fixed point is
                       unchanged because the bound is inactive once |step| is small */
                    if (max_step > 0.0) step = fmax(-max_step, fmin(max_step, step));
                    u[at(n, i, j, k)] += step;
                }
}

/* d = L(u) - f over the grid; returns sum of d^2. */
static double residual(const grid* g, const consts* c, const double* u, const double* f, double* d)
{
    int n = g->n;
    double* plane = (double*)malloc((size_t)n * sizeof(double));
#pragma omp parallel for schedule(static) if (n >= 32)
    for (int i = 0; i < n; ++i) {
        double s = 0.0;
        for (int j = 0; j < n; ++j)
            for (int k = 0; k < n; ++k) {
                double v = cell_op(g, c, u, i, j, k, NULL);
                if (f) v -= f[at(n, i, j, k)];
                if (d) d[at(n, i, j, k)] = v;
                s += v * v;
            }
        plane[i] = s;
    }
    double s = sum_planes(plane, n);
    free(plane);
    return s;
}

/* Size of the double-precision rounding noise of rms(L - f): per cell, one unit in the last
   place of u times |dL/du| (u is only known to that granularity) plus one of the sum of the
   magnitudes of the terms, C (b_nb + b_i)|u_nb - u_i| per face, the curvature term and |f|
   (rms over the grid).  Sweeps cannot push the residual much below it. */
static double rounding_floor(const grid* g, const consts* c, const double* u, const double* f)
{
    const double eps = 2.220446049250313e-16;
    int n = g->n;
    double* plane = (double*)malloc((size_t)n * sizeof(double));
#pragma omp parallel for schedule(static) if (n >= 32)
    for (int i = 0; i < n; ++i) {
        double s = 0.0;
        for (int j = 0; j < n; ++j)
            for (int k = 0; k < n; ++k) {
                double dL;
                cell_op(g, c, u, i, j, k, &dL);
                double ui = u[at(n, i, j, k)], bi = exp(ui), t = 0.0;
                for (int q = 0; q < 6; ++q) {
                    int ii = (i + DI[q] + n) % n, jj = (j + DJ[q] + n) % n, kk = (k + DK[q] + n) % n;
                    double un = u[at(n, ii, jj, kk)];
                    t += g->C * (exp(un) + bi) * fabs(un - ui);
                }
                t += c->A * exp(-ui / (c->n + 1.0)) + (f ? fabs(f[at(n, i, j, k)]) : 0.0);
                double fl = eps * (fabs(dL) * fabs(ui) + t);
                s += fl * fl;
            }
        plane[i] = s;
    }
    double s = sum_planes(plane, n);
    free(plane);
    return sqrt(s / ((double)n * n * n));
}

/* Restriction: each coarse cell gets the mean of its 8 children. */
static void restrict_mean(int n, const double* fine, double* coarse)
{
    int nc = n / 2;
#pragma omp parallel for schedule(static) if (nc >= 32)
    for (int I = 0; I < nc; ++I)
        for (int J = 0; J < nc; ++J)
            for (int K = 0; K < nc; ++K) {
                double s = 0.0;
                for (int a = 0; a < 2; ++a)
                    for (int b = 0; b < 2; ++b)
                        for (int e = 0; e < 2; ++e) s += fine[at(n, 2 * I + a, 2 * J + b, 2 * K + e)];
                coarse[at(nc, I, J, K)] = s / 8.0;
            }
}

/* Coarse value for prolongation: periodic wrap on the domain; on a patch a coarse cell
   outside the patch is not a valid multigrid cell and contributes zero (Sec. V.A.3). */
static double coarse_val(int nc, const double* v, int periodic, int I, int J, int K)
{
    if (periodic) {
        I = (I + nc) % nc;
        J = (J + nc) % nc;
        K = (K + nc) % nc;
    } else if (I < 0 || I >= nc || J < 0 || J >= nc || K < 0 || K >= nc) {
        return 0.0;
    }
    return v[at(nc, I, J, K)];
}

/* u_fine += P(v): each fine cell takes 27/64 of the coarse cell containing it, 9/64 of the
   three sharing a face with it, 3/64 of the three sharing an edge, 1/64 of the one sharing
   a vertex (Sec. V.A.3). */
static void prolong_add(int nc, const double* v, int periodic, double* ufine)
{
    int n = 2 * nc;
#pragma omp parallel for schedule(static) if (n >= 32)
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j)
            for (int k = 0; k < n; ++k) {
                int I = i >> 1, J = j >> 1, K = k >> 1;
                int si = (i & 1) ? 1 : -1, sj = (j & 1) ? 1 : -1, sk = (k & 1) ? 1 : -1;
                double p = 27.0 / 64.0 * coarse_val(nc, v, periodic, I, J, K) +
                           9.0 / 64.0 * (coarse_val(nc, v, periodic, I + si, J, K) +
                                         coarse_val(nc, v, periodic, I, J + sj, K) +
                                         coarse_val(nc, v, periodic, I, J, K + sk)) +
                           3.0 / 64.0 * (coarse_val(nc, v, periodic, I + si, J + sj, K) +
                                         coarse_val(nc, v, periodic, I + si, J, K + sk) +
                                         coarse_val(nc, v, periodic, I, J + sj, K + sk)) +
                           1.0 / 64.0 * coarse_val(nc, v, periodic, I + si, J + sj, K + sk);
                ufine[at(n, i, j, k)] += p;
            }
}

/* Coarse-level boundary values of a patch: mean of the four fine ones on the same face. */
static void restrict_faces(int n, const double* ub, double* ubc)
{
    int nc = n / 2;
    for (int f = 0; f < 6; ++f)
        for (int P = 0; P < nc; ++P)
            for (int Q = 0; Q < nc; ++Q) {
                double s = 0.0;
                for (int a = 0; a < 2; ++a)
                    for (int b = 0; b < 2; ++b) s += ub[((long long)f * n + 2 * P + a) * n + 2 * Q + b];
                ubc[((long long)f * nc + P) * nc + Q] = s / 4.0;
            }
}

/* ----------------------------------------------------------------------------------- */
/* Multigrid hierarchy and V-cycle.                                                      */

typedef struct {
    grid g;
    double *u, *f, *uhat, *d;
    double* ubuf; /* coarse patch boundary values (owned) */
} level;

static void vcycle(level* lv, int m, int nlev, const consts* c, const orc_opts* o)
{
    level* F = &lv[m];
    if (m == nlev - 1) {
        /* coarsest level: sweep until its residual has dropped by coarsest_rtol (or, with
           coarsest_rtol = 0, exactly coarsest_sweeps times) */
        long long nc3 = (long long)F->g.n * F->g.n * F->g.n;
        double r0 = sqrt(residual(&F->g, c, F->u, F->f, NULL) / (double)nc3);
        for (int s = 0; s < o->coarsest_sweeps; ++s) {
            if (o->coarsest_rtol > 0.0) {
                /* stop once reduced by coarsest_rtol or down to the rounding floor */
                double r = sqrt(residual(&F->g, c, F->u, F->f, NULL) / (double)nc3);
                if (r <= o->coarsest_rtol * r0 || r <= rounding_floor(&F->g, c, F->u, F->f)) break;
            }
            ngs_sweep(&F->g, c, F->u, F->f, o->max_step);
        }
        return;
    }
    for (int s = 0; s < o->pre; ++s) ngs_sweep(&F->g, c, F->u, F->f, o->max_step);
    /* residual d^h = L^h(u^) - f^h */
    residual(&F->g, c, F->u, F->f, F->d);
    level* H = &lv[m + 1];
    int nc = H->g.n;
    long long ncell = (long long)nc * nc * nc;
    restrict_mean(F->g.n, F->u, H->uhat);
    restrict_mean(F->g.n, F->d, H->f);
    /* FAS coarse equation L^H(u^H) = L^H(R u^h) - R d^h, started from R u^h */
#pragma omp parallel for schedule(static) if (nc >= 32)
    for (int I = 0; I < nc; ++I)
        for (int J = 0; J < nc; ++J)
            for (int K = 0; K < nc; ++K) {
                long long q = at(nc, I, J, K);
                H->f[q] = cell_op(&H->g, c, H->uhat, I, J, K, NULL) - H->f[q];
            }
    memcpy(H->u, H->uhat, (size_t)ncell * sizeof(double));
    vcycle(lv, m + 1, nlev, c, o);
    /* u^h <- u^h + P(u^H - R u^h) */
    for (long long q = 0; q < ncell; ++q) H->d[q] = H->u[q] - H->uhat[q];
    prolong_add(nc, H->d, F->g.ub == NULL, F->u);
    for (int s = 0; s < o->post; ++s) ngs_sweep(&F->g, c, F->u, F->f, o->max_step);
}

static int is_pow2(int x) { return x > 0 && (x & (x - 1)) == 0; }

static int check_opts(const orc_opts* o)
{
    if (!o || o->pre < 0 || o->post < 0 || o->coarsest_sweeps < 0 || o->max_cycles < 0 ||
        !is_pow2(o->coarsest_n) || o->coarsest_n < 2 || !(o->tol >= 0.0) || !(o->max_step >= 0.0) ||
        !(o->coarsest_rtol >= 0.0))
        return ORC_EINVAL;
    return 0;
}

/* Builds levels n, n/2, ..., coarsest_n on top of the caller's u (level 0). */
static int build_levels(level* lv, int n, double h, const double* ub, double r, const double* rho,
                        double rho_ref, const consts* c, const orc_opts* o, double* u)
{
    int nlev = 0;
    for (int nm = n; nlev < 30; nm /= 2) {
        level* L = &lv[nlev];
        memset(L, 0, sizeof(*L));
        long long ncell = (long long)nm * nm * nm;
        double hm = h * (double)(n / nm);
        L->g.n = nm;
        L->g.h = hm;
        L->g.C = c->ct * c->ct / (2.0 * hm * hm);
        L->g.r = r;
        L->g.rho = nlev == 0 ? rho : NULL;
        L->g.rho_ref = rho_ref;
        if (ub && nlev == 0) {
            L->g.ub = ub;
        } else if (ub) {
            /* coarse patch level: boundary values restricted from the level above */
            L->ubuf = (double*)calloc((size_t)6 * nm * nm, sizeof(double));
            restrict_faces(2 * nm, lv[nlev - 1].g.ub, L->ubuf);
            L->g.ub = L->ubuf;
        }
        L->u = nlev == 0 ? u : (double*)calloc((size_t)ncell, sizeof(double));
        L->f = nlev == 0 ? NULL : (double*)calloc((size_t)ncell, sizeof(double));
        L->uhat = nlev == 0 ? NULL : (double*)calloc((size_t)ncell, sizeof(double));
        L->d = (double*)calloc((size_t)ncell, sizeof(double));
        ++nlev;
        if (nm <= o->coarsest_n || nm % 2) break;
    }
    return nlev;
}

static void free_levels(level* lv, int nlev)
{
    for (int m = 0; m < nlev; ++m) {
        if (m > 0) {
            free(lv[m].u);
            free(lv[m].f);
            free(lv[m].uhat);
        }
        free(lv[m].d);
        free(lv[m].ubuf);
    }
}

static int run_cycles(level* lv, int nlev, const consts* c, const orc_opts* o, double* hist,
                      int* nhist)
{
    g_updates = 0;
    long long ncell = (long long)lv[0].g.n * lv[0].g.n * lv[0].g.n;
    double rms = sqrt(residual(&lv[0].g, c, lv[0].u, NULL, NULL) / (double)ncell);
    int k = 0;
    if (hist) hist[0] = rms;
    while (isfinite(rms) && rms > o->tol && k < o->max_cycles) {
        vcycle(lv, 0, nlev, c, o);
        rms = sqrt(residual(&lv[0].g, c, lv[0].u, NULL, NULL) / (double)ncell);
        ++k;
        if (hist) hist[k] = rms;
    }
    if (nhist) *nhist = k + 1;
    if (!isfinite(rms)) return ORC_ENONFINITE;
    return rms <= o->tol ? 0 : ORC_ENOTCONV;
}

int orc_solve(const double* rho, int N, const orc_model* m, const orc_opts* o, double* u,
              double* hist, int* nhist)
{
    consts c;
    if (derive(m, &c) != 0 || check_opts(o) != 0 || !rho || !u || !is_pow2(N) || N < o->coarsest_n)
        return ORC_EINVAL;
    long long ncell = (long long)N * N * N;
    double mean = 0.0;
    for (long long q = 0; q < ncell; ++q) {
        if (!isfinite(rho[q])) return ORC_ENONFINITE;
        mean += rho[q];
    }
    mean /= (double)ncell;
    if (!o->warm_start)
        for (long long q = 0; q < ncell; ++q) u[q] = c.ubar;
    for (long long q = 0; q < ncell; ++q)
        if (!isfinite(u[q])) return ORC_ENONFINITE;
    level lv[32];
    memset(lv, 0, sizeof(lv));
    int nlev = build_levels(lv, N, 1.0 / N, NULL, 0.0, rho, o->subtract_mean ? mean : 1.0, &c, o, u);
    int st = run_cycles(lv, nlev, &c, o, hist, nhist);
    free_levels(lv, nlev);
    return st;
}

int orc_solve_patch(const double* rho, int n, double h, const double* ub, const orc_model* m,
                    const orc_opts* o, double* u, double* hist, int* nhist)
{
    consts c;
    if (derive(m, &c) != 0 || check_opts(o) != 0 || !rho || !u || !ub || !is_pow2(n) ||
        n < o->coarsest_n || !(h > 0.0))
        return ORC_EINVAL;
    long long ncell = (long long)n * n * n;
    for (long long q = 0; q < ncell; ++q)
        if (!isfinite(rho[q]) || !isfinite(u[q])) return ORC_ENONFINITE;
    for (long long q = 0; q < 6LL * n * n; ++q)
        if (!isfinite(ub[q])) return ORC_ENONFINITE;
    level lv[32];
    memset(lv, 0, sizeof(lv));
    int nlev = build_levels(lv, n, h, ub, CUBE_PATCH_R, rho, 1.0, &c, o, u);
    int st = run_cycles(lv, nlev, &c, o, hist, nhist);
    free_levels(lv, nlev);
    return st;
}

/* ----------------------------------------------------------------------------------- */
/* Patch boundary set-up from the parent level (Sec. V.A.1, V.B.1; Sec. VI.B).          */

static int floor_half(int x) { return x >= 0 ? x / 2 : -((-x + 1) / 2); }

/* Parent u at parent-local cell (I,J,K); NAN when outside a non-periodic parent. */
static double parent_val(const double* pu, int pn, int periodic, int I, int J, int K)
{
    if (periodic) {
        I = ((I % pn) + pn) % pn;
        J = ((J % pn) + pn) % pn;
        K = ((K % pn) + pn) % pn;
    } else if (I < 0 || I >= pn || J < 0 || J >= pn || K < 0 || K >= pn) {
        return NAN;
    }
    return pu[at(pn, I, J, K)];
}

/* Trilinear (27/9/3/1) interpolation of the parent u at child-level global cell (x,y,z). */
static double parent_interp(const double* pu, int pn, const int* po, int periodic, int x, int y, int z)
{
    int I = floor_half(x) - po[0], J = floor_half(y) - po[1], K = floor_half(z) - po[2];
    int si = (x & 1) ? 1 : -1, sj = (y & 1) ? 1 : -1, sk = (z & 1) ? 1 : -1;
    return 27.0 / 64.0 * parent_val(pu, pn, periodic, I, J, K) +
           9.0 / 64.0 * (parent_val(pu, pn, periodic, I + si, J, K) + parent_val(pu, pn, periodic, I, J + sj, K) +
                         parent_val(pu, pn, periodic, I, J, K + sk)) +
           3.0 / 64.0 * (parent_val(pu, pn, periodic, I + si, J + sj, K) +
                         parent_val(pu, pn, periodic, I + si, J, K + sk) +
                         parent_val(pu, pn, periodic, I, J + sj, K + sk)) +
           1.0 / 64.0 * parent_val(pu, pn, periodic, I + si, J + sj, K + sk);
}

int orc_patch_boundary(const double* parent_u, int pn, const int* porigin, int parent_periodic,
                       const int* origin, int n, double* ub, double* u0)
{
    if (!parent_u || !porigin || !origin || !ub || !u0 || pn < 1 || n < 2 || (n & 1)) return ORC_EINVAL;
    for (int d = 0; d < 3; ++d)
        if (origin[d] & 1) return ORC_EINVAL;
    const int* o = origin;
    /* initial guess inside: the interpolated parent solution */
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j)
            for (int k = 0; k < n; ++k)
                u0[at(n, i, j, k)] = parent_interp(parent_u, pn, porigin, parent_periodic, o[0] + i, o[1] + j, o[2] + k);
    /* ghost u by interpolation, then u_b from eq. u_i-1jk: u_b = (u_g - r u_i) / (1 - r) */
    const double r = CUBE_PATCH_R;
    for (int f = 0; f < 6; ++f)
        for (int p = 0; p < n; ++p)
            for (int q = 0; q < n; ++q) {
                int ci, cj, ck, gi, gj, gk;
                if (f < 2) { ci = f == 0 ? 0 : n - 1; cj = p; ck = q; }
                else if (f < 4) { ci = p; cj = f == 2 ? 0 : n - 1; ck = q; }
                else { ci = p; cj = q; ck = f == 4 ? 0 : n - 1; }
                gi = ci + DI[f];
                gj = cj + DJ[f];
                gk = ck + DK[f];
                double ug = parent_interp(parent_u, pn, porigin, parent_periodic, o[0] + gi, o[1] + gj, o[2] + gk);
                double ui = u0[at(n, ci, cj, ck)];
                ub[((long long)f * n + p) * n + q] = (ug - r * ui) / (1.0 - r);
            }
    for (long long q = 0; q < (long long)n * n * n; ++q)
        if (!isfinite(u0[q])) return ORC_EINVAL;
    for (long long q = 0; q < 6LL * n * n; ++q)
        if (!isfinite(ub[q])) return ORC_EINVAL;
    return 0;
}

/* ----------------------------------------------------------------------------------- */

int orc_operator(int n, double h, const double* u, const double* rho, double rho_ref,
                 const double* ub, double r, const orc_model* m, double* L, double* dL)
{
    consts c;
    if (derive(m, &c) != 0 || n < 1 || !u || !(h > 0.0)) return ORC_EINVAL;
    grid g = {n, h, c.ct * c.ct / (2.0 * h * h), ub, r, rho, rho_ref};
#pragma omp parallel for schedule(static) if (n >= 32)
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j)
            for (int k = 0; k < n; ++k) {
                double d;
                double v = cell_op(&g, &c, u, i, j, k, &d);
                if (L) L[at(n, i, j, k)] = v;
                if (dL) dL[at(n, i, j, k)] = d;
            }
    return 0;
}

int orc_operator_at(int n, double h, const double* u, const double* rho, double rho_ref,
                    const double* ub, double r, const orc_model* m, long long ncell,
                    const long long* idx, double* L)
{
    consts c;
    if (derive(m, &c) != 0 || n < 1 || !u || !idx || !L || !(h > 0.0)) return ORC_EINVAL;
    grid g = {n, h, c.ct * c.ct / (2.0 * h * h), ub, r, rho, rho_ref};
    long long tot = (long long)n * n * n;
    for (long long s = 0; s < ncell; ++s)
        if (idx[s] < 0 || idx[s] >= tot) return ORC_EINVAL;
#pragma omp parallel for schedule(static) if (ncell >= 4096)
    for (long long s = 0; s < ncell; ++s) {
        long long q = idx[s];
        int k = (int)(q % n), j = (int)((q / n) % n), i = (int)(q / ((long long)n * n));
        L[s] = cell_op(&g, &c, u, i, j, k, NULL);
    }
    return 0;
}

int orc_single_grid(const double* rho, int N, const orc_model* m, int subtract_mean, double max_step,
                    double* u, int nsweeps, double* hist)
{
    consts c;
    if (derive(m, &c) != 0 || !rho || !u || N < 2 || nsweeps < 0) return ORC_EINVAL;
    long long ncell = (long long)N * N * N;
    double mean = 0.0;
    for (long long q = 0; q < ncell; ++q) mean += rho[q];
    mean /= (double)ncell;
    double h = 1.0 / N;
    grid g = {N, h, c.ct * c.ct / (2.0 * h * h), NULL, 0.0, rho, subtract_mean ? mean : 1.0};
    if (hist) hist[0] = sqrt(residual(&g, &c, u, NULL, NULL) / (double)ncell);
    for (int s = 1; s <= nsweeps; ++s) {
        ngs_sweep(&g, &c, u, NULL, max_step);
        if (hist) hist[s] = sqrt(residual(&g, &c, u, NULL, NULL) / (double)ncell);
    }
    return 0;
}

/* ----------------------------------------------------------------------------------- */
/* A refinement level with the mask scheme (Sec. V, Sec. V.A.1-2, Sec. V.B.1-2).         */
/*                                                                                       */
/* The level is held as the periodic N^3 grid of its resolution.  mask[q] > 0 marks an   */
/* active cell (relaxed); mask <= 0 a cell outside the refinement, whose value is fixed.  */
/* Readings (listed in the design notes of the repo):                                   */
/*   - w = the field on entry, kept for the whole solve: in masked cells the values      */
/*     interpolated from the coarser level, in active cells the initial guess;           */
/*   - boundary value between active i and masked nb, where the linearly interpolated    */
/*     mask vanishes: u_b = (m_i w_nb - m_nb w_i) / (m_i - m_nb) (eq. phi_b, fixed);     */
/*   - ghost u_nb = (1 - r) u_b + r u_i, r = m_nb / m_i, and b_nb = exp(u_nb)            */
/*     (eq. u_i-1jk; b is not interpolated);                                             */
/*   - coarse levels: mask and w are the 8-child means of the finer level's;             */
/*   - R d: mean of the 8 children with d = 0 in masked children, into active coarse     */
/*     cells only; R u: mean of all 8 children (masked ones at their fixed value), into  */
/*     active coarse cells only; masked coarse cells hold their w;                       */
/*   - P: the coarse correction u^H - R u is zero in masked coarse cells (no             */
/*     renormalisation of the weights) and is added to active fine cells only;           */
/*   - the stop test is the rms of d over the active cells of the level.                 */

typedef struct {
    int n;
    double h, C;
    const double* mask;
    const double* w;
    const double* rho; /* finest level only */
    double rho_ref;
} mgrid;

/* L_i and dL_i/du_i at an active cell (eq. bc_modified_fR_op, eq. bc_modified_fR_dop
   with the ghost of each masked neighbour substituted). */
static double masked_op(const mgrid* g, const consts* c, const double* u, int i, int j, int k,
                        double* dop)
{
    int n = g->n;
    long long q = at(n, i, j, k);
    double mi = g->mask[q];
    double ui = u[q], bi = exp(ui);
    double L = 0.0, dL = 0.0;
    for (int f = 0; f < 6; ++f) {
        int ii = (i + DI[f] + n) % n, jj = (j + DJ[f] + n) % n, kk = (k + DK[f] + n) % n;
        long long p = at(n, ii, jj, kk);
        double mn = g->mask[p];
        if (mn > 0.0) {
            double un = u[p], bn = exp(un);
            L += g->C * (bn + bi) * (un - ui);
            dL += g->C * (bi * (un - ui) - bn - bi);
        } else {
            double r = mn / mi;
            double ubv = (mi * g->w[p] - mn * g->w[q]) / (mi - mn);
            double ug = (1.0 - r) * ubv + r * ui;
            double bg = exp(ug);
            L += g->C * (bg + bi) * (ug - ui);
            dL += g->C * ((r * bg + bi) * (ug - ui) + (bg + bi) * (r - 1.0));
        }
    }
    double S = c->A * exp(-ui / (c->n + 1.0));
    L += S;
    dL -= S / (c->n + 1.0);
    if (g->rho) L -= c->D * (g->rho[q] - g->rho_ref) + c->Sbar;
    if (dop) *dop = dL;
    return L;
}

static void masked_sweep(const mgrid* g, const consts* c, double* u, const double* f, double max_step)
{
    int n = g->n;
    for (long long q = 0; q < (long long)n * n * n; ++q)
        if (g->mask[q] > 0.0) ++g_updates;
    /* as ngs_sweep: the cells of one colour can be visited in any order */
    for (int colour = 0; colour < 2; ++colour)
#pragma omp parallel for schedule(static) if (n >= 32)
        for (int i = 0; i < n; ++i)
            for (int j = 0; j < n; ++j)
                for (int k = 0; k < n; ++k) {
                    if (((i + j + k) & 1) != colour) continue;
                    long long q = at(n, i, j, k);
                    if (!(g->mask[q] > 0.0)) continue;
                    double d;
                    double L = masked_op(g, c, u, i, j, k, &d);
                    if (f) L -= f[q];
                    double step = -L / d;
                    if (max_step > 0.0) step = fmax(-max_step, fmin(max_step, step));
                    u[q] += step;
                }
}

/* d = L(u) - f at active cells, 0 elsewhere; returns the sum of d^2 and the number of
   active cells in *nact. */
static double masked_residual(const mgrid* g, const consts* c, const double* u, const double* f,
                              double* d, long long* nact)
{
    int n = g->n;
    double* plane = (double*)malloc((size_t)n * sizeof(double));
    long long na = 0;
#pragma omp parallel for schedule(static) if (n >= 32) reduction(+ : na)
    for (int i = 0; i < n; ++i) {
        double s = 0.0;
        for (int j = 0; j < n; ++j)
            for (int k = 0; k < n; ++k) {
                long long q = at(n, i, j, k);
                double v = 0.0;
                if (g->mask[q] > 0.0) {
                    v = masked_op(g, c, u, i, j, k, NULL);
                    if (f) v -= f[q];
                    ++na;
                }
                if (d) d[q] = v;
                s += v * v;
            }
        plane[i] = s;
    }
    double s = sum_planes(plane, n);
    free(plane);
    if (nact) *nact = na;
    return s;
}

typedef struct {
    mgrid g;
    double *u, *f, *uhat, *d;
    double *mbuf, *wbuf; /* owned mask and w (coarse levels; w on level 0 too) */
} mlevel;

static double masked_rms(const mlevel* L, const consts* c, const double* f)
{
    long long na = 0;
    double s = masked_residual(&L->g, c, L->u, f, NULL, &na);
    return na > 0 ? sqrt(s / (double)na) : 0.0;
}

/* Rounding noise of the rms residual over the active cells, as rounding_floor() for the
   periodic grid: per active cell one unit in the last place of u times |dL/du| plus one of
   the summed magnitudes of the terms (C (b_nb + b_i)|u_nb - u_i| per face, the ghost's for a
   masked neighbour, the curvature term and |f|). */
static double masked_floor(const mlevel* L, const consts* c, const double* f)
{
    const double eps = 2.220446049250313e-16;
    const mgrid* g = &L->g;
    int n = g->n;
    double* plane = (double*)malloc((size_t)n * sizeof(double));
    long long na = 0;
#pragma omp parallel for schedule(static) if (n >= 32) reduction(+ : na)
    for (int i = 0; i < n; ++i) {
        double s = 0.0;
        for (int j = 0; j < n; ++j)
            for (int k = 0; k < n; ++k) {
                long long q = at(n, i, j, k);
                double mi = g->mask[q];
                if (!(mi > 0.0)) continue;
                double dL;
                masked_op(g, c, L->u, i, j, k, &dL);
                double ui = L->u[q], bi = exp(ui), t = 0.0;
                for (int e = 0; e < 6; ++e) {
                    long long p = at(n, (i + DI[e] + n) % n, (j + DJ[e] + n) % n, (k + DK[e] + n) % n);
                    double mn = g->mask[p], un;
                    if (mn > 0.0) {
                        un = L->u[p];
                    } else {
                        double r = mn / mi;
                        un = (1.0 - r) * ((mi * g->w[p] - mn * g->w[q]) / (mi - mn)) + r * ui;
                    }
                    t += g->C * (exp(un) + bi) * fabs(un - ui);
                }
                t += c->A * exp(-ui / (c->n + 1.0)) + (f ? fabs(f[q]) : 0.0);
                double fl = eps * (fabs(dL) * fabs(ui) + t);
                s += fl * fl;
                ++na;
            }
        plane[i] = s;
    }
    double s = sum_planes(plane, n);
    free(plane);
    return na > 0 ? sqrt(s / (double)na) : 0.0;
}

static void masked_vcycle(mlevel* lv, int m, int nlev, const consts* c, const orc_opts* o)
{
    mlevel* F = &lv[m];
    if (m == nlev - 1) {
        /* coarsest level: sweep until its residual has dropped by coarsest_rtol or reached
           the rounding floor (with coarsest_rtol = 0, exactly coarsest_sweeps times) */
        double r0 = masked_rms(F, c, F->f);
        for (int s = 0; s < o->coarsest_sweeps; ++s) {
            if (o->coarsest_rtol > 0.0) {
                double r = masked_rms(F, c, F->f);
                if (r <= o->coarsest_rtol * r0 || r <= masked_floor(F, c, F->f)) break;
            }
            masked_sweep(&F->g, c, F->u, F->f, o->max_step);
        }
        return;
    }
    for (int s = 0; s < o->pre; ++s) masked_sweep(&F->g, c, F->u, F->f, o->max_step);
    masked_residual(&F->g, c, F->u, F->f, F->d, NULL);
    mlevel* H = &lv[m + 1];
    int nc = H->g.n;
    long long ncell = (long long)nc * nc * nc;
    double* Ru = (double*)calloc((size_t)ncell, sizeof(double));
    double* Rd = (double*)calloc((size_t)ncell, sizeof(double));
    restrict_mean(F->g.n, F->u, Ru);
    restrict_mean(F->g.n, F->d, Rd); /* d is zero in masked fine cells */
    for (long long q = 0; q < ncell; ++q) {
        if (H->g.mask[q] > 0.0) {
            H->uhat[q] = Ru[q];
            H->u[q] = Ru[q];
        } else {
            H->uhat[q] = H->g.w[q];
            H->u[q] = H->g.w[q];
        }
    }
    /* FAS coarse equation at active coarse cells: L^H(u^H) = L^H(R u^h) - R d^h */
#pragma omp parallel for schedule(static) if (nc >= 32)
    for (int I = 0; I < nc; ++I)
        for (int J = 0; J < nc; ++J)
            for (int K = 0; K < nc; ++K) {
                long long q = at(nc, I, J, K);
                H->f[q] = H->g.mask[q] > 0.0 ? masked_op(&H->g, c, H->uhat, I, J, K, NULL) - Rd[q] : 0.0;
            }
    free(Ru);
    free(Rd);
    masked_vcycle(lv, m + 1, nlev, c, o);
    /* u^h += P(u^H - R u^h) at active fine cells; zero correction from masked coarse cells */
    for (long long q = 0; q < ncell; ++q) H->d[q] = H->g.mask[q] > 0.0 ? H->u[q] - H->uhat[q] : 0.0;
    int n = F->g.n;
    double* corr = (double*)calloc((size_t)n * n * n, sizeof(double));
    prolong_add(nc, H->d, 1, corr);
    for (long long q = 0; q < (long long)n * n * n; ++q)
        if (F->g.mask[q] > 0.0) F->u[q] += corr[q];
    free(corr);
    for (int s = 0; s < o->post; ++s) masked_sweep(&F->g, c, F->u, F->f, o->max_step);
}

static void free_mlevels(mlevel* lv, int nlev)
{
    for (int m = 0; m < nlev; ++m) {
        if (m > 0) {
            free(lv[m].u);
            free(lv[m].f);
            free(lv[m].uhat);
        }
        free(lv[m].d);
        free(lv[m].mbuf);
        free(lv[m].wbuf);
    }
}

int orc_solve_masked(const double* rho, const double* mask, int N, const orc_model* m, const orc_opts* o,
                     double* u, double* hist, int* nhist)
{
    consts c;
    if (derive(m, &c) != 0 || check_opts(o) != 0 || !rho || !mask || !u || !is_pow2(N) || N < 2)
        return ORC_EINVAL;
    long long ncell = (long long)N * N * N;
    double mean = 0.0;
    for (long long q = 0; q < ncell; ++q) {
        if (!isfinite(rho[q]) || !isfinite(u[q])) return ORC_ENONFINITE;
        if (!(mask[q] >= -1.0 && mask[q] <= 1.0)) return ORC_EINVAL;
        mean += rho[q];
    }
    mean /= (double)ncell;
    mlevel lv[32];
    memset(lv, 0, sizeof(lv));
    int nlev = 0;
    for (int nm = N; nlev < 30; nm /= 2) {
        mlevel* L = &lv[nlev];
        long long nc = (long long)nm * nm * nm;
        double hm = 1.0 / nm;
        L->g.n = nm;
        L->g.h = hm;
        L->g.C = c.ct * c.ct / (2.0 * hm * hm);
        L->g.rho = nlev == 0 ? rho : NULL;
        L->g.rho_ref = o->subtract_mean ? mean : 1.0;
        L->wbuf = (double*)calloc((size_t)nc, sizeof(double));
        if (nlev == 0) {
            memcpy(L->wbuf, u, (size_t)nc * sizeof(double));
            L->g.mask = mask;
        } else {
            L->mbuf = (double*)calloc((size_t)nc, sizeof(double));
            restrict_mean(2 * nm, lv[nlev - 1].g.mask, L->mbuf);
            restrict_mean(2 * nm, lv[nlev - 1].g.w, L->wbuf);
            L->g.mask = L->mbuf;
        }
        L->g.w = L->wbuf;
        L->u = nlev == 0 ? u : (double*)calloc((size_t)nc, sizeof(double));
        L->f = nlev == 0 ? NULL : (double*)calloc((size_t)nc, sizeof(double));
        L->uhat = nlev == 0 ? NULL : (double*)calloc((size_t)nc, sizeof(double));
        L->d = (double*)calloc((size_t)nc, sizeof(double));
        ++nlev;
        if (nm <= o->coarsest_n || nm % 2) break;
    }
    g_updates = 0;
    double rms = masked_rms(&lv[0], &c, NULL);
    int k = 0;
    if (hist) hist[0] = rms;
    while (isfinite(rms) && rms > o->tol && k < o->max_cycles) {
        masked_vcycle(lv, 0, nlev, &c, o);
        rms = masked_rms(&lv[0], &c, NULL);
        ++k;
        if (hist) hist[k] = rms;
    }
    if (nhist) *nhist = k + 1;
    free_mlevels(lv, nlev);
    if (!isfinite(rms)) return ORC_ENONFINITE;
    return rms <= o->tol ? 0 : ORC_ENOTCONV;
}

int orc_masked_operator(int n, const double* u, const double* w, const double* mask, const double* rho,
                        double rho_ref, const orc_model* m, double* L, double* dL)
{
    consts c;
    if (derive(m, &c) != 0 || n < 1 || !u || !w || !mask) return ORC_EINVAL;
    double h = 1.0 / n;
    mgrid g = {n, h, c.ct * c.ct / (2.0 * h * h), mask, w, rho, rho_ref};
#pragma omp parallel for schedule(static) if (n >= 32)
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j)
            for (int k = 0; k < n; ++k) {
                long long q = at(n, i, j, k);
                double d = 0.0, v = 0.0;
                if (mask[q] > 0.0) v = masked_op(&g, &c, u, i, j, k, &d);
                if (L) L[q] = v;
                if (dL) dL[q] = d;
            }
    return 0;
}
