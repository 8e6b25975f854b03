/*
 * mgfr.h -- C ABI of libmgfr.so, the MI355X (gfx950) multigrid solver of the nonlinear
 * f(R) scalar-field equation of ECOSMOG (Li, Zhao, Teyssier & Koyama, arXiv:1110.1379).
 *
 * Problem (Sec. III.C, Sec. IV): given the code-unit density rho~ on a periodic N^3 grid
 * (box side 1, h = 1/N) and the Hu-Sawicki model, find u with f~_R = -exp(u) such that at
 * every cell
 *
 *   L_i(u) = c~^2/(2h^2) sum_nb (b_nb + b_i)(u_nb - u_i)          b = exp(u)
 *          + (1/3) Om a^4 (n a^2 xi)^(1/(n+1)) exp(-u_i/(n+1))
 *          - Om a (rho~_i - 1) - Om a^4 (a^-3 + 4 OL/Om)  = 0
 *
 * (eq. discrete_fR multiplied by c~^2, i.e. the scaling of eq. bc_modified_fR_op).  The
 * solver runs FAS V-cycles (Sec. V.B.2) with a red-black Newton-Gauss-Seidel smoother
 * (Sec. V.B.1) until the rms of L over the grid is <= tol.  Refinement patches (Sec. V,
 * Sec. VI.B) are cube sub-grids whose boundary values come from the parent solution.
 *
 * Conventions for every entry point:
 *   - Arrays of cells are C order [i][j][k] with k fastest; i is x.  Doubles unless noted.
 *   - "device" pointers are HIP device memory of the context's device; "host" pointers are
 *     ordinary host memory.  The caller owns every buffer passed in; the context owns its
 *     internal scratch (multigrid hierarchy, reductions), which it keeps between calls.
 *   - stream: a hipStream_t (NULL = the default stream).  Work is queued on it; calls that
 *     return residual histories synchronise it before returning.
 *   - Return value: MGFR_OK or a negative MGFR_E* code; mgfr_last_error() then holds a
 *     message.  No C++ exception crosses this interface.  A context is not thread-safe.
 */
#ifndef MGFR_H
#define MGFR_H

#ifdef __cplusplus
extern "C" {
#endif

#define MGFR_OK 0
#define MGFR_EINVAL (-1)     /* invalid argument (sizes, pointers, options, patch layout)   */
#define MGFR_ENONFINITE (-2) /* non-finite density or start field, or the iteration overflowed */
#define MGFR_ENOTCONV (-3)   /* max_cycles reached; u and the history are still written     */
#define MGFR_EDEVICE (-4)    /* HIP runtime error                                            */
#define MGFR_ENOMEM (-5)     /* device allocation failed                                     */

/* opts.precision */
#define MGFR_FP64 0          /* every level and sweep in double precision                   */
#define MGFR_MIXED 1         /* FP32 correction-form V-cycles inside an FP64 defect-correction loop */

/* opts.flags */
#define MGFR_SUBTRACT_MEAN 1 /* density contrast rho~ - mean(rho~) instead of rho~ - 1       */
#define MGFR_WARM_START 2    /* start from the u passed in instead of the background u      */
#define MGFR_PROFILE 4       /* time every finest-level smoother launch with HIP events
                                (batched solves: every sweep of the finest level of every
                                unit, both colour launches, when MGFR_GRAPH is not set)      */
#define MGFR_GRAPH 8         /* batched solves: capture one cycle's launches in a HIP graph
                                on first use and replay it for every later cycle of the call.
                                mg_fr_solve: capture two cycles, each ending in the stop test
                                on the device, once per context and storage (kept until the
                                hierarchy changes or the context is destroyed), replay them
                                until the device test stops the solve (every kernel of a cycle
                                returns at once after it) and read one flag per replay.  Only
                                with pre + post even and without MGFR_PROFILE and tau_alpha
                                (otherwise the cycles run eagerly); the results are the same
                                bits as eager cycles.  mg_fr_solve_noalloc rejects it.      */
#define MGFR_PER_PHASE 16    /* batched solves: the per-phase engine (every phase of every
                                level one launch over all units, per-unit norms read back by
                                the host after every cycle) instead of the default engine
                                (units of side <= unit_n solved whole by one workgroup each in
                                one persistent launch; larger units' fine levels launched per
                                phase, their coarse levels in one workgroup per unit; stop
                                tests on the device)                                          */

/* Model (Sec. II, Sec. III.A): Om, OL (< 0 means 1 - Om), scale factor a, Hu-Sawicki n,
 * |f_R0| (the present background f_R), box side B in Mpc/h. */
typedef struct mgfr_params {
    double omega_m, omega_l, a, n, fr0_abs, box_mpc_h;
} mgfr_params;

/* Solver options.  mgfr_default_opts() fills the defaults listed here. */
typedef struct mgfr_opts {
    double tol;           /* stop when rms(L) over the finest cells <= tol          [1e-8]   */
    int pre, post;        /* Newton-Gauss-Seidel sweeps before/after the coarse step [2, 2] */
    int coarsest_n;       /* side of the coarsest level, power of two >= 2          [4]      */
    int coarsest_sweeps;  /* cap on the sweeps of the coarsest level                [400]    */
    int max_cycles;       /* cap on V-cycles (mixed: on FP64 outer iterations)      [60]     */
    int precision;        /* MGFR_FP64 or MGFR_MIXED                                [FP64]   */
    int flags;            /* MGFR_SUBTRACT_MEAN | MGFR_WARM_START                   [0]      */
    int inner_cycles;     /* mixed: FP32 V-cycles per FP64 outer iteration          [1]      */
    double max_step;      /* > 0: bound |Newton step| per visit; 0: plain Newton    [1.0]    */
    double coarsest_rtol; /* coarsest level sweeps until rms <= rtol x initial or down to
                             its rounding floor; 0: always coarsest_sweeps            [1e-3]   */
    int planes;           /* planes per workgroup of the finest-level fused sweeps (N >= 64):
                             0 = automatic, else a power of two in [4, N]            [0]      */
    double tau_alpha;     /* > 0: also stop once rms(L) <= tau_alpha x rms(tau), tau the
                             truncation-error estimate of the current field (Sec. V.B;
                             the stop test is rms(L) <= max(tol, tau_alpha rms(tau)));
                             mg_fr_solve only: the batched and masked solves reject it
                             with MGFR_EINVAL                                      [0]      */
    int unit_n;           /* batched solves (default engine): units, and the levels of larger
                             units, of side <= unit_n are relaxed by one workgroup each (up
                             to 16 with every level in LDS); 0 = 16; rounded down to a power
                             of two; values below coarsest_n count as coarsest_n    [0]      */
    int tile;             /* tile of the finest level's fused sweeps (N >= 64).  FP64: 0 =
                             automatic (16 x 64), 1 = 16 x 64, 2 = 8 x 64 (column pairs over
                             the tile and its halo; 3 - 5 as 0).  Mixed, the single-precision
                             correction sweep: 0 = automatic (16 x 32), 1 = 16 x 32, 2 = 32 x
                             32, 3 = 16 x 64, 5 = 32 x 64 (one tile column pair per thread),
                             4 = 8 x 32 (column pairs over the tile and its halo).
                             Batched solves, launched sweeps of unit levels of side >=
                             32: 0 = automatic: periodic boxes walk 16 x 32 column tiles
                             (16 planes per workgroup), a mixed solve in pairs of fused
                             two-colour sweeps, double precision one colour per launch,
                             at multigrid depths with at least 256 such tiles in the
                             batch (one thread per cell of the colour at the others);
                             patches run one thread per cell of the colour; 1 = one
                             thread per cell everywhere; 2 = column tiles one colour per
                             launch everywhere; 3 = fused pairs at every depth, for
                             patches too (8 planes per workgroup) in mixed solves; 4, 5
                             as 0 (all give the same results, bit for bit)        [0]      */
} mgfr_opts;

/* One refinement patch: a cube of n^3 cells at refinement level `level` >= 1 (cell size
 * 1 / (N0 2^level)), with `origin` its first cell in level-`level` cells of the whole box.
 * `parent` is -1 for level 1 (the parent is the periodic N0^3 domain grid) and otherwise the
 * index of the enclosing level-1 patch.  `offset` is the element offset of its n^3 block in
 * the packed density and solution arrays. */
typedef struct mgfr_patch {
    int level;
    int parent;
    int origin[3];
    int n;
    long long offset;
} mgfr_patch;

/* Counters of the last solve on a context (mgfr_get_stats). */
typedef struct mgfr_stats {
    int cycles;                /* V-cycles (FP64) or FP64 outer iterations (mixed)             */
    int inner_cycles;          /* mixed: FP32 V-cycles in total; FP64: 0                       */
    long long cell_updates;    /* Newton-Gauss-Seidel cell visits on all levels                */
    long long finest_updates;  /* of which on the finest level                                 */
    int sweep_launches;        /* MGFR_PROFILE: finest-level smoother kernel launches timed    */
    double sweep_ms;           /* MGFR_PROFILE: their summed duration (HIP events, same stream) */
    double sweep_bytes;        /* algorithmic bytes of those launches: per cell the field
                                  read and written and its right-hand side read, in the
                                  sweep's precision: 24 B in FP64 (read u, read rho, write
                                  u), 12 B in the single-precision correction sweep (read
                                  and write e, read the rhs; the fixed base ub it also reads
                                  is not credited), counted once per fused launch (also for
                                  the two-sweep pass
                                  of mg_poisson_solve, which moves them once for both
                                  sweeps) or per pair of colour launches                    */
    double solve_ms;           /* host wall time of the last solve call                        */
    double tau_rms;            /* tau_alpha > 0: rms of tau at the last stop test; else 0    */
} mgfr_stats;

typedef struct mgfr_ctx mgfr_ctx;

/* Creates a context bound to HIP device `device`.  Returns MGFR_OK or MGFR_EDEVICE. */
int mgfr_create(mgfr_ctx** ctx, int device);

/* Frees the context and its device scratch (waits for its work to finish). */
void mgfr_destroy(mgfr_ctx* ctx);

/* Message of the last failed call on ctx ("" if none).  Owned by ctx. */
const char* mgfr_last_error(const mgfr_ctx* ctx);

/* Copies the counters of the last solve on ctx into *out. */
int mgfr_get_stats(const mgfr_ctx* ctx, mgfr_stats* out);

/* Autotuner: times complete solves of this problem (rho, N, params as for mg_fr_solve,
 * starting from the background) over candidate settings of the tunable options -- sweeps
 * before/after the coarse step, planes per workgroup and tile of the fused sweep, and for
 * MGFR_MIXED the single-precision V-cycles per outer iteration -- and writes the fastest
 * (by host wall time, best of two solves each) into *best (other fields copied from *base).
 * u_scratch: device, N^3, overwritten.  best_ms (host, may be NULL) gets its solve time.
 * Candidates that do not converge within base->max_cycles are skipped.  Synchronises. */
int mgfr_autotune(mgfr_ctx* ctx, const double* rho, int N, const mgfr_params* params,
                  const mgfr_opts* base, double* u_scratch, mgfr_opts* best, double* best_ms,
                  void* stream);

/* Writes the defaults into *opts. */
void mgfr_default_opts(mgfr_opts* opts);

/* Derived constants of the model on an N^3 domain grid (Sec. II, III, VI.A.1), host only:
 * out8 = {xi, c~, K = (n a^2 xi)^(1/(n+1)), A = (1/3) Om a^4 K,
 *         Sbar = Om a^4 (a^-3 + 4 OL/Om), D = Om a, u_bar, C = c~^2 / (2 h^2), h = 1/N}. */
int mgfr_constants(const mgfr_params* params, int N, double* out8);

/* Residual of a given field (device): d_i = L_i(u) for every cell of the periodic N^3
 * grid, the operator above with contrast rho~ - 1 (or rho~ - mean with
 * MGFR_SUBTRACT_MEAN in flags).  rho, u, d: device, N^3.  Does not synchronise. */
int mgfr_residual(mgfr_ctx* ctx, const double* rho, const double* u, int N,
                  const mgfr_params* params, int flags, double* d, void* stream);

/* Single-grid relaxation (Sec. VI.D.1's comparison; also the smoother on its own):
 * nsweeps red-black Newton-Gauss-Seidel sweeps of the periodic N^3 grid, in place on u
 * (device, N^3), with opts->max_step and opts->flags (MGFR_SUBTRACT_MEAN, MGFR_PROFILE).
 * variant: 0 = the kernel the solver uses for this N, 1 = one kernel per colour (in place),
 * 2 = the fused red-black sweep (N >= 64; out of place through context scratch).
 * Does not synchronise unless MGFR_PROFILE is set. */
int mgfr_smooth(mgfr_ctx* ctx, const double* rho, double* u, int N, const mgfr_params* params,
                const mgfr_opts* opts, int nsweeps, int variant, void* stream);

/* Single-grid relaxation of the single-precision correction equation of the mixed solver:
 * Sec. V.B.1's red-black Newton-Gauss-Seidel applied to N(e) = L(ub + e) - L(ub) = f, the
 * operator of eq. discrete_fR (times c~^2) differenced exactly about the base ub, on the
 * periodic N^3 grid (h = 1/N), every term written proportional to e:
 *   N_i(e) = C sum_nb [(M_nb + M_i)(ub_nb - ub_i) + (B_nb + B_i)(e_nb - e_i)]
 *          + A exp(-ub_i/(n+1)) expm1(-e_i/(n+1)),   b = exp(ub), M = b expm1(e), B = b + M.
 * nsweeps sweeps in place on e (device, N^3 float); ub and f (device, N^3 float) are read.
 * variant: 0 = the kernel the mixed solver uses on its finest level for this N, 1 = one kernel
 * per colour (in place), 2 = the fused red-black sweep (N >= 64, out of place through context
 * scratch), opts->planes planes per workgroup (0: the mixed solver's automatic choice; else a
 * multiple of 4 that is <= N).  opts->max_step bounds each step; MGFR_PROFILE times every
 * launch (12 B per cell: read ub and f, read and write e).  Returns MGFR_EINVAL for other N,
 * variants or planes.  Does not synchronise unless MGFR_PROFILE is set. */
int mgfr_smooth32(mgfr_ctx* ctx, const float* ub, float* e, const float* f, int N, const mgfr_params* params,
                  const mgfr_opts* opts, int nsweeps, int variant, void* stream);

/* The domain-grid solve (Sec. V.B, Sec. VI.A).
 * rho      device, N^3: code-unit density (mean 1 in the paper's units; negative values
 *          are allowed, non-finite ones are rejected with MGFR_ENONFINITE).
 * N        power of two, opts->coarsest_n <= N <= 1024.
 * u        device, N^3: output; with MGFR_WARM_START also the starting field.
 * res_hist host, max_cycles + 1 doubles (may be NULL): rms(L) before the first cycle and
 *          after every cycle (mixed: after every FP64 outer iteration).
 * n_hist   host (may be NULL): number of entries written to res_hist.
 * Returns MGFR_OK when rms(L) <= tol (or, with opts->tau_alpha > 0, when rms(L) <=
 * tau_alpha x rms(tau), rms(tau) then reported in the stats), MGFR_ENOTCONV when max_cycles
 * was reached first (u holds the last iterate).  Synchronises the stream. */
int mg_fr_solve(mgfr_ctx* ctx, const double* rho, int N, const mgfr_params* params,
                const mgfr_opts* opts, double* u, double* res_hist, int* n_hist, void* stream);

/* mg_fr_solve for callers that cannot allocate device memory (code being captured into a HIP
 * graph, tight serving loops, harnesses that forbid allocation): the same solve, same
 * arguments, results and errors, but every scratch buffer (multigrid levels, single-precision
 * levels, reduction partials) is carved from one fixed 72 MiB device array that the library
 * holds on each GPU it runs on until the process ends; the call itself allocates nothing
 * (device or host).  Limits: N a power of two in [coarsest_n, 128]; MGFR_PROFILE (its events
 * would be allocated) and MGFR_GRAPH (it keeps a graph and device state in the context) are
 * rejected.  Larger N gives MGFR_EINVAL.  The array is shared by every
 * call on the same GPU and keeps the last call's contents (everything a solve reads is written
 * by that solve first): calls that overlap on one GPU, from any context or stream, race and
 * must be serialised by the caller.  Returns MGFR_EDEVICE if the array's device address could
 * not be resolved when the context was created.  Synchronises the stream. */
int mg_fr_solve_noalloc(mgfr_ctx* ctx, const double* rho, int N, const mgfr_params* params,
                        const mgfr_opts* opts, double* u, double* res_hist, int* n_hist, void* stream);

/* Refinement patches, level by level (Sec. V, Sec. VI.B; the paper solves every refinement
 * level with its own V-cycles after the coarser level, with boundary values from it).
 * For each refinement level, in increasing order: every patch of that level gets its ghost
 * values by trilinear (27/9/3/1) interpolation of its parent's solution (u_domain for level
 * 1, the already solved parent patch otherwise), boundary values u_b = (u_g + u_i)/2 on its
 * faces (eq. u_i-1jk with mask ratio -1) and the interpolated parent solution as initial
 * guess; then all patches of the level run batched FAS V-cycles with the BC-modified
 * operator (eq. bc_modified_fR_op) until each has rms(L) <= tol or max_cycles.
 * u_domain    device, N0^3: the solved domain grid (read only).
 * patches     host, npatch entries.  Rules (else MGFR_EINVAL): n a power of two in
 *             [coarsest_n, 128]; origin even (aligned to parent cells) with the cube inside the
 *             level's box; a level >= 2 patch lies inside its parent with a margin of at least
 *             one parent cell on every side; patches of one level do not overlap; blocks
 *             [offset, offset + n^3) do not overlap and lie in [0, packed_cells).
 * rho_packed  device, packed_cells: the density of every patch cell (code units).
 * u_packed    device, packed_cells: output.
 * res_hist    host, npatch x (max_cycles + 1) (may be NULL); n_hist host, npatch (may be NULL).
 * opts->precision: MGFR_FP64 runs the V-cycles in double precision; MGFR_MIXED runs, per
 * cycle, opts->inner_cycles single-precision correction V-cycles (ghost faces in correction
 * form) followed by u += e and the double-precision residual, as in mg_fr_solve.  Histories
 * hold the double-precision rms per cycle.  MGFR_SUBTRACT_MEAN is rejected (the contrast is
 * rho - 1).  Returns MGFR_ENOTCONV if any patch missed tol (all patches are still written).
 * Synchronises. */
int mg_fr_solve_patches(mgfr_ctx* ctx, const double* u_domain, int N0, const mgfr_patch* patches,
                        int npatch, const double* rho_packed, double* u_packed, long long packed_cells,
                        const mgfr_params* params, const mgfr_opts* opts, double* res_hist,
                        int* n_hist, void* stream);

/* Independent periodic boxes solved together (Sec. V.B: the nonlinear multigrid solve of
 * the discrete equation eq. discrete_fR on a periodic grid, Sec. V.B.1 smoother, Sec. V.B.2
 * FAS coarse-grid correction, Sec. VI.A.1 code units per box; each box is the domain-grid
 * problem of mg_fr_solve with its own parameters).  Box b has side N[b] (power of two in
 * [coarsest_n, 1024]), density rho[b] and output u[b] (device arrays of N[b]^3, pointers
 * given in host arrays), and its own model per_box[b] (box size, |f_R0|, ...).  Every box
 * runs the domain-grid FAS V-cycles of mg_fr_solve batched with the others until
 * rms(L) <= tol or max_cycles, in double precision or (MGFR_MIXED) as single-precision
 * correction V-cycles inside the double-precision defect-correction loop.  MGFR_WARM_START
 * keeps the given u as the start; MGFR_SUBTRACT_MEAN is rejected.  res_hist host
 * nbox x (max_cycles + 1), n_hist host nbox (both may be NULL).  Returns MGFR_ENOTCONV if
 * any box missed tol.  Synchronises. */
int mg_fr_solve_batch(mgfr_ctx* ctx, int nbox, const int* N, const double* const* rho,
                      const mgfr_params* per_box, const mgfr_opts* opts, double* const* u,
                      double* res_hist, int* n_hist, void* stream);

/* Truncation-error estimate (Sec. V.B): tau = L^H(R u) - R L^h(u) on the level with N/2 cells
 * per side, R the 8-child mean, each operator with its own level's density (R rho~) and
 * spacing, on the periodic N^3 grid; the density and background terms cancel, so tau is the
 * FAS coarse right-hand side L^H(R u) - R d minus the restricted source.  rho, u: device N^3
 * (read); flags: MGFR_SUBTRACT_MEAN as in mgfr_residual.  tau: device (N/2)^3 (written; may
 * be NULL); rms: host (may be NULL), rms of tau.  N a power of two in [4, 1024].
 * Synchronises. */
int mgfr_tau(mgfr_ctx* ctx, const double* rho, const double* u, int N, const mgfr_params* params, int flags,
             double* tau, double* rms, void* stream);

/* The modified Poisson equation (eq. discrete_poisson; Sec. II, Sec. III.B): the Newtonian
 * potential phi of the density and of delta R of the scalaron f~_R = -exp(u), on the periodic
 * N^3 grid (box side 1, h = 1/N):
 *   (1/h^2) [sum of the 6 neighbours of phi - 6 phi] = S - mean(S),
 *   S = 2 Om a (rho~ - 1) - (1/6) Om a^4 [(n a^2 xi)^(1/(n+1)) exp(-u/(n+1)) - 3 (a^-3 + 4 OL/Om)].
 * The periodic system fixes phi up to a constant and needs a source of zero mean: the mean of
 * S is removed and phi is returned with zero mean.  Linear multigrid V-cycles (Sec. V.A.3):
 * red-black Gauss-Seidel (opts->pre / post sweeps), the residual restricted by 8-child means,
 * the coarse correction prolongated 27/9/3/1, the coarsest level (opts->coarsest_n) relaxed
 * as in mg_fr_solve; until rms(residual) <= opts->tol x rms(S - mean S) (a relative
 * criterion: the equation is linear) or opts->max_cycles.
 * rho, u   device, N^3 (read): the density and the scalaron, e.g. the solution of mg_fr_solve.
 * phi      device, N^3: output (with MGFR_WARM_START in opts->flags, also the start).
 * N        power of two in [2 coarsest_n, 1024].  opts->precision must be MGFR_FP64.
 * res_hist host, max_cycles + 1 (may be NULL): rms residual before each cycle and at the end;
 * n_hist   host (may be NULL): entries written.
 * Returns MGFR_ENONFINITE for a non-finite source, MGFR_ENOTCONV if tol was not reached (phi
 * still written).  Synchronises. */
int mg_poisson_solve(mgfr_ctx* ctx, const double* rho, const double* u, int N, const mgfr_params* params,
                     const mgfr_opts* opts, double* phi, double* res_hist, int* n_hist, void* stream);

/* Single-grid red-black Gauss-Seidel sweeps of the modified Poisson equation (Sec. V.A.3),
 * the smoother of mg_poisson_solve on its own: nsweeps sweeps of phi in place against the
 * source of rho and u (its mean removed), with no coarse levels.
 * variant 0: per-colour kernels (any N); 1: the one-sweep fused kernel; 2: the two-sweep
 * temporally blocked kernel (nsweeps even).  Variants 1 and 2 need N >= 256 and give the same
 * bits; variant 0 sums each cell's neighbours in another order.
 * rho, u device, N^3 (read); phi device, N^3 (read and written).  N power of two in
 * [4, 1024].  Returns MGFR_EINVAL for other N, variants or an odd nsweeps with variant 2,
 * MGFR_ENONFINITE for a non-finite source.  Synchronises. */
int mg_poisson_smooth(mgfr_ctx* ctx, const double* rho, const double* u, int N, const mgfr_params* params,
                      int nsweeps, int variant, double* phi, void* stream);

/* A refinement level of irregular shape solved with the mask scheme (Sec. V; eq. phi_b,
 * eq. u_i-1jk, eq. bc_modified_fR_op, eq. bc_modified_fR_dop; restriction and prolongation
 * rules of Sec. V.A.2, V.A.3, V.B.2).  The level is held as the periodic N^3 grid of its
 * resolution (h = 1/N).  A cell with mask > 0 is active and is solved for; a cell with
 * mask <= 0 keeps the value u holds on entry (the coarser level's solution interpolated
 * there).  A masked neighbour of an active cell i enters the operator through the boundary
 * value u_b = (m_i w_nb - m_nb w_i) / (m_i - m_nb), w = u on entry, fixed where the linearly
 * interpolated mask vanishes, and the ghost u_g = (1 - r) u_b + r u_i, r = m_nb / m_i, with
 * b_g = exp(u_g).  Coarse multigrid levels carry the 8-child means of the masks (fractional
 * values) and of w; the residual is restricted from active children into active coarse cells,
 * R u from all 8 children, and the coarse correction is prolongated (27/9/3/1) from active
 * coarse cells into active fine cells only.  FAS V-cycles until the rms residual over the
 * active finest cells <= opts->tol, or opts->max_cycles.
 * rho      device, N^3 (read): density rho~ (contrast rho - 1, or rho - mean with
 *          MGFR_SUBTRACT_MEAN in opts->flags).
 * mask     device, N^3 float in [-1, 1] (read); +1 / -1 on an adaptive level.
 * u        device, N^3, read and written: on entry the initial guess in active cells and the
 *          fixed values elsewhere (always read: MGFR_WARM_START is implied); on return the
 *          active cells hold the solution and the others are bit-for-bit unchanged.
 * N        power of two in [coarsest_n, 1024].  opts->precision must be MGFR_FP64 and
 *          opts->tau_alpha 0.  res_hist, n_hist: as mg_fr_solve (rms over active cells).
 *          A finest level of N >= 64 whose mask holds only +1 and -1 is swept both colours in
 *          one pass (opts->planes planes per workgroup, 0: automatic), out of place between
 *          u and a context buffer; opts->tile = 1 keeps one launch per colour (the same
 *          results, bit for bit).
 * Returns MGFR_EINVAL for a mask outside [-1, 1], MGFR_ENONFINITE for non-finite rho or u,
 * MGFR_ENOTCONV if tol was not reached (u still written).  Synchronises. */
int mg_fr_solve_masked(mgfr_ctx* ctx, const double* rho, const float* mask, int N, const mgfr_params* params,
                       const mgfr_opts* opts, double* u, double* res_hist, int* n_hist, void* stream);

/* Triangle-shaped-cloud density assignment (Sec. VI.C): the density of np particles on the
 * periodic N^3 grid of the unit box.  A particle at x (box units; taken modulo 1) with
 * s = x N, nearest cell floor(s) and offset d = s - floor(s) - 1/2 gives the cells floor(s)-1,
 * floor(s), floor(s)+1 the weights (1/2 - d)^2/2, 3/4 - d^2, (1/2 + d)^2/2 per axis, times
 * mass, the product over the three axes (mass N^3 / np gives mean density 1, the code-unit
 * normalisation of rho~).
 * The particles are sorted by nearest cell on the device and every cell sums the
 * contributions of the particles in its 27 neighbouring cells in a fixed order: the result is
 * the same bits on every call (no atomics).
 * pos   device, np x 3 doubles (x, y, z per particle), read; finite; np < 2^31.
 * rho   device, N^3 doubles, written.
 * N     power of two in [4, 1024].  Scratch (about 40 B per particle + 4 B per cell) is kept
 * in the context.  Returns MGFR_ENONFINITE for a non-finite coordinate (rho untouched).
 * Synchronises once (the coordinate check). */
int mgfr_tsc_density(mgfr_ctx* ctx, const double* pos, long long np, int N, double mass, double* rho, void* stream);

/* TSC force interpolation (Sec. VI.C): the acceleration -grad phi at np particles, the cell
 * values -(phi[i+1] - phi[i-1]) N / 2 per axis (central differences, periodic) weighted with
 * the same 27 TSC weights as mgfr_tsc_density, which makes the pair momentum conserving.
 * phi   device, N^3 doubles (e.g. from mg_poisson_solve), read.
 * pos   device, np x 3 doubles, read; acc: device, np x 3 doubles, written.
 * Returns MGFR_ENONFINITE for a non-finite coordinate.  Synchronises once. */
int mgfr_tsc_force(mgfr_ctx* ctx, const double* phi, int N, const double* pos, long long np, double* acc,
                   void* stream);

#ifdef __cplusplus
}
#endif
#endif /* MGFR_H */
