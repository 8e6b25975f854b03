// Internal interface between the host driver and the HIP kernels of libmgfr.so.
// Not installed; the public interface is include/mgfr.h.
#pragma once

#include <hip/hip_runtime.h>

#include "kernel_types.h"

namespace mgfr {

// ---- modified Poisson solve (poisson_kernels.hip) -----------------------------------------
// Number of block partials the grid-stride reductions below write for n elements.
int poisson_partials(long long n);
// S at every cell, and block partials (sum S, max |S|) for fold_partials.
hipError_t poisson_source(const PoissonSource& c, long long n3, const double* rho, const double* u, double* S,
                          double* partial, hipStream_t s);
// Block partials (sum r^2, max |r|) of r = b - bmean - lap x (x null: r = b - bmean); their
// number (at most 8192) in *nparts.
hipError_t poisson_resid_norm(const PGrid& g, const double* x, const double* b, double bmean, double* partial,
                              int* nparts, hipStream_t s);
// One red-black Gauss-Seidel sweep in place (one launch per colour).
hipError_t poisson_ngs(const PGrid& g, double* x, const double* b, double bmean, hipStream_t s);
// One red-black sweep from xin into xout (distinct arrays), n >= poisson_fused_min_n().
int poisson_fused_min_n();
hipError_t poisson_ngs_fused(const PGrid& g, const double* xin, double* xout, const double* b, double bmean, int ti,
                             hipStream_t s);
// Two red-black sweeps from xin into xout in one pass (the same bits as two one-sweep calls),
// and its planes per workgroup when the options leave them automatic.
int poisson_fused2_planes(int n);
hipError_t poisson_ngs_fused2(const PGrid& g, const double* xin, double* xout, const double* b, double bmean, int ti,
                              hipStream_t s);
// bc = R (b - bmean - lap x) on the level below.
hipError_t poisson_resid_restrict(const PGrid& g, const double* x, const double* b, double bmean, double* bc,
                                  hipStream_t s);
// Coarsest level (n <= 8) in one workgroup: x relaxed against b - bmean until rms <= rtol x
// initial (or its rounding floor, or cap sweeps).
hipError_t poisson_coarsest(const PGrid& g, double* x, const double* b, double bmean, int cap, double rtol,
                            hipStream_t s);
// x += v.
hipError_t poisson_add(double* x, double v, long long n, hipStream_t s);

// ---- refinement level with the mask scheme (masked.hip) ------------------------------------
// Active cells: mask > 0; w: fixed values (masked cells) and initial values (active cells).
// Block partials (number of active cells, max |mask|) of n masks; their number in *nparts.
hipError_t masked_count(const float* mask, long long n, double* partial, int* nparts, hipStream_t s);
// Coarse mask and w of level gc: 8-child means of the finer level's.
hipError_t masked_restrict_setup(const Grid& gc, const float* maskf, const double* wf, float* maskc, double* wc,
                                 hipStream_t s);
// Byte flags of a mask (1 where > 0), and block partials (first of each pair) of the number
// of cells whose mask is neither +1 nor -1; their number in *nparts.
hipError_t masked_flags(const float* mask, long long n, unsigned char* flags, double* partial, int* nparts,
                        hipStream_t s);
// One red-black Newton-Gauss-Seidel sweep of the active cells (one launch per colour).  The
// byte-flag forms take a +1 / -1 mask as flags (1: active).
hipError_t masked_ngs(const Grid& g, const float* mask, const double* w, double* u, const double* src, hipStream_t s);
hipError_t masked_ngs(const Grid& g, const unsigned char* flags, const double* w, double* u, const double* src,
                      hipStream_t s);
// One red-black sweep of a level read as byte flags in one pass (n >= 64, the domain's fused
// tiling with the mask scheme), out of place: uin to uout (never the same array; masked
// cells copied unchanged), ti planes per workgroup (a multiple of 4 dividing n).  The same
// values, bit for bit, as masked_ngs on the flags.
hipError_t masked_ngs_fused(const Grid& g, const unsigned char* flags, const double* w, const double* uin,
                            double* uout, const double* src, int ti, hipStream_t s);
// Into the level below: uc = uhat = R u and fc = R d at active coarse cells (w, w and 0 at
// masked ones).
hipError_t masked_resid_restrict(const Grid& g, const float* mask, const double* w, const double* u,
                                 const double* src, const float* maskc, const double* wc, double* uc, double* uhat,
                                 double* fc, hipStream_t s);
hipError_t masked_resid_restrict(const Grid& g, const unsigned char* flags, const double* w, const double* u,
                                 const double* src, const float* maskc, const double* wc, double* uc, double* uhat,
                                 double* fc, hipStream_t s);
// f = L^H(uhat) - f at active cells of the coarse level gc.
hipError_t masked_fas_rhs(const Grid& gc, const float* maskc, const double* wc, const double* uhat, double* f,
                          hipStream_t s);
// uf += P(uc - uhat) at active fine cells; zero correction from masked coarse cells.  uhat is
// overwritten with the coarse correction.
hipError_t masked_prolong(const Grid& gc, const float* maskc, const double* uc, double* uhat, const float* maskf,
                          double* uf, hipStream_t s);
// Block partials (sum d^2, max |d|) over active cells, one pair per 2048 cells (partial holds
// masked_norm_partials(n) pairs); their number in *nparts.
long long masked_norm_partials(const Grid& g);
hipError_t masked_norm(const Grid& g, const float* mask, const double* w, const double* u, const double* src,
                       double* partial, int* nparts, hipStream_t s);
hipError_t masked_norm(const Grid& g, const unsigned char* flags, const double* w, const double* u,
                       const double* src, double* partial, int* nparts, hipStream_t s);
// Coarsest level (n <= 8), one workgroup: sweeps until rms <= rtol x initial, or the rounding
// floor, or cap;
// the sweep count is added to *sweeps.
hipError_t masked_coarsest(const Grid& g, const float* mask, const double* w, double* u, const double* f, int cap,
                           double rtol, long long* sweeps, hipStream_t s);

// ---- batched units (batch_fp64.hip) ------------------------------------------------------
// One multigrid level of one unit (a cube refinement patch or a periodic box).
struct BGrid {
    int n, lg;
    int periodic;      // 1: periodic box; 0: patch with ghost faces from ub
    int unit;          // index of the unit (for the active flags)
    double C, A, inv_np1, max_step;
    double fscale, sref, fshift;  // f = fscale (src - sref) + fshift
    double u0;         // value that batch_fill writes
    double* u;
    double* uhat;      // coarse levels: R u of the finer level, then e = u - R u
    double* f;         // coarse levels: FAS right-hand side
    const double* src; // finest: the density; coarse: == f
    double* ub;        // patch: boundary values [6][n][n]
    // single-precision correction levels of a mixed solve (null in double precision)
    float* ub32;       // base: finest = u rounded, coarse = R ub
    float* e32;        // correction e
    float* eh32;       // coarse: R e of the finer level, then e - R e
    float* f32;        // finest: r = -d; coarse: the FAS right-hand side
    float* e32b;       // level swept by pairs of fused sweeps: their second buffer of e, or null
};

// Workgroup table: blk[b] = (index into grids, block number within that grid).
struct BTable {
    const BGrid* grids;
    const int2* blk;
    const int* active;  // per-unit flags, or null (all active)
};

// Every unit of a batch for the workgroup-per-unit kernels: the descriptors of all levels of
// all units (unit by unit, finest first), where each unit's start, how many levels it has,
// and the units solved whole by one workgroup in the order the queue hands them out.
struct UnitSet {
    const BGrid* grids;
    const int* first;
    const int* nlev;
    const int* order;
};

// Per-unit results on the device: residual history (H doubles per unit), cycles done, and
// status (0 converged, 1 not converged, 2 non-finite).
struct UnitOut {
    double* hist;
    int* ncyc;
    int* status;
    int H;
};

// Solver settings the workgroup-per-unit kernels need.
struct UnitCfg {
    double tol, rtol;
    int pre, post, max_cycles, inner, cap;
};

// Parent of a patch for the boundary set-up: the parent level's u (side n, periodic for the
// domain grid), its origin in parent-level cells, and the child's origin in child cells.
struct PatchParent {
    const double* u;
    int n, lg, periodic;
    int origin[3];
    int child[3];
};

int batch_block();
hipError_t batch_ngs(const BTable& t, int nblk, hipStream_t s);
// The same sweep over column tiles (batch_col.hip): blk[b] = (grid, tile), tiles of 16 x 32
// cells by 16 planes; batch_col_tiles(n) is the number of tiles of a grid of side n, 0 where
// the side does not allow them (n < 32).  Same results, bit for bit, as batch_ngs / batch_ngs32.
long long batch_col_tiles(int n);
hipError_t batch_ngs_col(const BTable& t, int nblk, hipStream_t s);
// d = L(u) - f of every cell over the same column tiles, with one (sum d^2, max |d|) pair per
// tile in partial (as batch_norm's blocks); cast: also r = -d, ub = u and e = 0 in single
// precision (as batch_resid_cast).  d is the same, bit for bit, as theirs.
hipError_t batch_resid_col(const BTable& t, int nblk, double* partial, bool cast, hipStream_t s);
// Residual and restriction over the same column tiles (coarse: the coarse grids, same order):
// as batch_resid_restrict (single: batch_resid_restrict32), the same results bit for bit.
hipError_t batch_resid_restrict_col(const BTable& t, int nblk, const BGrid* coarse, bool single, hipStream_t s);
hipError_t batch_ngs32_col(const BTable& t, int nblk, hipStream_t s);
// Two single-precision sweeps of unit levels (side >= 32, e32b set), each with both colours
// in one pass over the same column tiles (the fused tile sweep of the domain solve): e32 into
// e32b, then back.  Same results, bit for bit, as two batch_ngs32 sweeps.
// Its table: blk[b] = (grid, tile), tiles of 16 x 32 cells by 16 planes (periodic) or 8 planes
// (patch), every grid of the table periodic or every one a patch, as `periodic` says;
// batch_pair_tiles gives their number, 0 where the side does not allow them.  add_u
// (periodic tables only, else hipErrorInvalidValue): the second sweep ends a correction solve
// and adds its e to the grids' u (double precision) instead of writing e32 (as a
// batch_add_correction of those grids after it would, bit for bit); e32 keeps the first
// sweep's input.
hipError_t batch_ngs32_pair(const BTable& t, int nblk, bool periodic, bool add_u, hipStream_t s);
long long batch_pair_tiles(int n, int periodic);
hipError_t batch_resid_restrict(const BTable& t, int nblk, const BGrid* coarse, hipStream_t s);
hipError_t batch_fas_rhs(const BTable& t, int nblk, hipStream_t s);
hipError_t batch_coarse_diff(const BTable& t, int nblk, hipStream_t s);
// Fine u += P(coarse uhat) (trilinear 27/9/3/1; outside a patch a coarse cell contributes
// zero), over a table of coarse cells (blocks of the fine grids' cells / 8, the coarse grids
// in the same order): one thread per coarse cell and its eight fine cells.
// batch_prolong_add8_32: the same in single precision, e32 += P(coarse eh32).
hipError_t batch_prolong_add8(const BTable& t, int nblk, const BGrid* coarse, hipStream_t s);
hipError_t batch_prolong_add8_32(const BTable& t, int nblk, const BGrid* coarse, hipStream_t s);
// n: side of every grid in the list (the coarsest side, <= 8)
hipError_t batch_coarsest(const BGrid* grids, int ngrid, int n, const int* active, int cap, double rtol,
                          hipStream_t s);
hipError_t batch_norm(const BTable& t, int nblk, double* partial, const int* first, const int* count, int ngrid,
                      double* out, hipStream_t s);
// The blocks' (sum d^2, max |d|) of batch_norm only, without the fold.
hipError_t batch_norm_blocks(const BTable& t, int nblk, double* partial, hipStream_t s);
hipError_t batch_fold(const double* partial, const int* first, const int* count, int ngrid, double* out,
                      hipStream_t s);
hipError_t batch_setup(const BTable& t, int nblk, const PatchParent* parents, hipStream_t s);
hipError_t batch_restrict_faces(const BTable& t, int nblk, const BGrid* fine, hipStream_t s);
hipError_t batch_fill(const BTable& t, int nblk, hipStream_t s);
hipError_t batch_nonfinite(const BTable& t, int nblk, double* partial, hipStream_t s);

// ---- workgroup-per-unit kernels (unit.hip) ------------------------------------------------
// Sides up to which a unit, or the levels below a tail, are solved with every level in LDS.
constexpr int kUnitResidentMax = 16;
inline bool unit_resident(int side) { return side <= kUnitResidentMax; }
// The whole units us.order[begin, end), all of side `side`, solved completely by at most
// max_wg persistent workgroups taking units from the device counter *queue (reset here);
// results into out.
hipError_t unit_whole(const UnitSet& us, int begin, int end, int side, int* queue, const UnitOut& out,
                      const UnitCfg& cfg, bool mixed, int max_wg, hipStream_t s);
// One workgroup per tails[b] = (index of a large unit's tail level, of side `side`, in
// us.grids; levels from there): the rest of its V-cycle (the single-precision correction
// cycle when mixed, with the coarse bases below the tail level).
hipError_t unit_tail(const UnitSet& us, const int2* tails, int ntail, int side, const int* active, const UnitCfg& cfg,
                     bool mixed, hipStream_t s);
// Coarse bases R ub of the tail levels (from each tail level down), for tails the resident
// kernels do not take.
hipError_t unit_tail_base32(const UnitSet& us, const int2* tails, int ntail, const int* active, hipStream_t s);
// Device-side stop test of the large units after a cycle (first: before the first cycle).
hipError_t unit_judge(const double* sums, const int* ids, const double* ncell, int nl, int* active, const UnitOut& out,
                      double tol, int max_cycles, bool first, int* any, hipStream_t s);
hipError_t unit_fill_int(int* p, int v, int n, hipStream_t s);

// ---- batched mixed-precision solves (batch_fp32.hip; the double-precision parts in
// batch_fp64.hip) ------------------------------------------------------------------------------
// Finest grids (double precision): d = L(u) - f with ghost faces; r = -d, ub = u in single
// precision, e = 0; block partials of (sum d^2, max |d|) as batch_norm.
hipError_t batch_resid_cast(const BTable& t, int nblk, double* partial, hipStream_t s);
// Finest grids: u += e.
hipError_t batch_add_correction(const BTable& t, int nblk, hipStream_t s);
// Coarse base R ub (table over the coarse cells, indexed by the fine grids).
hipError_t batch_restrict_base32(const BTable& t, int nblk, const BGrid* coarse, hipStream_t s);
hipError_t batch_ngs32(const BTable& t, int nblk, hipStream_t s);
hipError_t batch_resid_restrict32(const BTable& t, int nblk, const BGrid* coarse, hipStream_t s);
hipError_t batch_fas_rhs32(const BTable& t, int nblk, hipStream_t s);
hipError_t batch_coarse_diff32(const BTable& t, int nblk, hipStream_t s);
hipError_t batch_coarsest32(const BGrid* grids, int ngrid, int n, const int* active, int cap, double rtol,
                            hipStream_t s);

// ---- FP64 kernels (kernels_fp64.hip) -----------------------------------------------
// All launchers queue work on `s` and return the hipError_t of the launch.

// One red-black Newton-Gauss-Seidel sweep: red (i+j+k even) cells, then black.
hipError_t ngs_sweep(const Grid& g, double* u, const double* src, hipStream_t s);

// Fine residual d = L(u) - f, restricted by 8-child means: uc = uhat = R u, fc = R d.
hipError_t resid_restrict(const Grid& g, const double* u, const double* src, double* uc,
                          double* uhat, double* fc, hipStream_t s);

// FAS right-hand side on a coarse level: f = L^H(uhat) - f (f holds R d on entry).
hipError_t fas_rhs(const Grid& gc, const double* uhat, double* f, hipStream_t s);

// Coarse-grid correction uf += P(uc - uhat), cell-centred trilinear 27/9/3/1 over 64,
// periodic; gc is the coarse level, 2 <= gc.n <= 512 (prolong.hip).
hipError_t prolong_correct(const Grid& gc, double* uf, const double* uc, const double* uhat, hipStream_t s);
hipError_t prolong_correct32(const Grid& gc, float* ef, const float* ec, const float* ehat, hipStream_t s);
// uf += P(ec), the correction itself on the coarse level (linear correction scheme).
hipError_t prolong_add_direct(const Grid& gc, double* uf, const double* ec, hipStream_t s);
// uf += P ec at the fine cells whose mask is positive (the others unchanged).
hipError_t prolong_add_masked(const Grid& gc, double* uf, const double* ec, const float* maskf, hipStream_t s);

// Coarsest level in one workgroup: sweeps until rms(L - f) <= rtol x initial or `cap`
// sweeps (rtol = 0: exactly cap sweeps).  n <= 8.  Adds the sweeps done to *sweeps_done
// (may be null).
hipError_t coarsest_solve(const Grid& g, double* u, const double* src, int cap, double rtol,
                          long long* sweeps_done, hipStream_t s);

// d = L(u) - f at every cell.
hipError_t residual_field(const Grid& g, const double* u, const double* src, double* d,
                          hipStream_t s);

// Block partial sums of d^2 and of max|d| (non-finite d -> NaN), then one workgroup folds
// them in a fixed order into out[0] = sum d^2, out[1] = max |d|.
hipError_t residual_norm(const Grid& g, const double* u, const double* src, double* partial,
                         double* out, hipStream_t s);

// out[0] = sum of x, out[1] = number of non-finite x (deterministic order).
hipError_t sum_and_count_nonfinite(const double* x, long long n, double* partial, double* out,
                                   hipStream_t s);

hipError_t fill(double* x, double v, long long n, hipStream_t s);

// ---- fused sweep (sweep_fp64.hip) --------------------------------------------------
// Smallest n the fused sweep supports, and its default planes per workgroup.
int fused_sweep_min_n();
int fused_sweep_planes(int n);

// One red-black sweep from uin into uout (distinct arrays), on 16 x 64 tiles (kTile64x16x64)
// or 8 x 64 tiles (kTile64x8x64).
constexpr int kTile64x16x64 = 1, kTile64x8x64 = 2;
hipError_t ngs_sweep_fused(const Grid& g, const double* uin, double* uout, const double* src, int ti, int tile,
                           hipStream_t s);

// ---- streaming residual (resid_fp64.hip), n >= 64 --------------------------------------
int resid_stream_planes(int n);
long long resid_stream_blocks(int n);
hipError_t resid_stream(const Grid& g, const double* uin, const double* src, ResidStream a, hipStream_t s);

// ---- small-grid helpers of the mixed loop (kernels_fp64.hip) ----------------------------
// u += e (single-precision correction); nothing once *halt is set (halt may be null).
hipError_t add_correction(double* u, const float* e, long long n, hipStream_t s, const int* halt = nullptr);
// Stop test of a graph-captured domain solve (red[0] = sum of d^2 after a cycle; state = {cycles
// done, stopped}), and a fill of up to 64 ints, both single-workgroup kernels.
hipError_t domain_stop(const double* red, long long ncell, double tol, int max_cycles, double* hist, int* state,
                       hipStream_t s);
hipError_t fill_int(int* p, int v, int n, hipStream_t s);
// r = -d, ub = u in single precision, and block partials of (sum d^2, max |d|) folded into
// out[0..1].
hipError_t residual_cast(const Grid& g, const double* u, const double* src, float* r32, float* ub32,
                         double* partial, double* out, hipStream_t s);
// out[0..1] from `nb` partial pairs (sum, max).
hipError_t fold_partials(const double* partial, int nb, double* out, hipStream_t s);

// tau = fH - R f_src on the level below the fine grid g (fH = L^H(R u) - R d there), written
// to tau if not null; block partials (sum tau^2, max |tau|).  Returns their number, or -1 if
// the launch failed.
int tau_finish(const Grid& g, const double* rho, const double* fH, double* tau, double* partial, hipStream_t s);

// ---- single-precision correction multigrid (kernels_fp32.hip) --------------------------
hipError_t ngs_sweep32(const Grid& g, const float* ub, float* e, const float* f, hipStream_t s);
// Tiles of the single-precision fused sweep: one tile column pair per thread on 16 x 32,
// 32 x 32 or 16 x 64 tiles (the last two: 512 threads), or the 8 x 32 tile whose pairs cover
// the tile and its halo.
constexpr int kTile16x32 = 1, kTile32x32 = 2, kTile16x64 = 3, kTile32Paired = 4, kTile32x64 = 5;
hipError_t ngs_sweep32_fused(const Grid& g, const float* ub, const float* ein, float* eout, const float* f,
                             int ti, int tile, hipStream_t s);
hipError_t resid_restrict32(const Grid& g, const float* ub, const float* e, const float* f, float* ec,
                            float* ehat, float* fc, hipStream_t s);
hipError_t fas_rhs32(const Grid& gc, const float* ubc, const float* ehat, float* f, hipStream_t s);
hipError_t restrict_mean32(const Grid& gc, const float* fine, float* coarse, hipStream_t s);
hipError_t coarsest_solve32(const Grid& g, const float* ub, float* e, const float* f, int cap, double rtol,
                            hipStream_t s);
hipError_t fill32(float* x, float v, long long n, hipStream_t s);

// Number of doubles the partial-sum scratch of the reductions needs.
long long reduction_scratch();

}  // namespace mgfr
