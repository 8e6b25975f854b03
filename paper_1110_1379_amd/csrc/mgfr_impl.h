// Internal interface between the host driver and the HIP kernels of libmgfr.so.
// Not installed; the public interface is include/mgfr.h.
#pragma once

#include <hip/hip_runtime.h>

namespace mgfr {

// One periodic multigrid level, passed to kernels by value.
//   L_i(u) = C sum_nb (b_nb + b_i)(u_nb - u_i) + A exp(-u_i/(n+1)) - f_i,   b = exp(u)
// with f_i = fscale * (src_i - sref) + fshift: on the finest level src = rho~,
// fscale = Om a, sref = rho_ref (1 or the mean), fshift = Sbar (eq. discrete_fR x c~^2);
// on coarse levels src = the FAS right-hand side and (fscale, sref, fshift) = (1, 0, 0).
struct Grid {
    int n;            // cells per side, a power of two >= 2
    int lg;           // log2(n)
    double C;         // c~^2 / (2 h^2)
    double A;         // (1/3) Om a^4 (n a^2 xi)^(1/(n+1))
    double inv_np1;   // 1 / (n_HS + 1)
    double max_step;  // > 0: bound on |Newton step|
    double fscale, sref, fshift;
};

inline long long cells(const Grid& g) { return 1LL << (3 * g.lg); }

// ---- FP64 kernels (kernels_fp64.hip) -----------------------------------------------
// All launchers queue work on `s` and return the hipError_t of the launch.

// One red-black Newton-Gauss-Seidel sweep: red (i+j+k even) cells, then black.
hipError_t ngs_sweep(const Grid& g, double* u, const double* src, hipStream_t s);

// Fine residual d = L(u) - f, restricted by 8-child means: uc = uhat = R u, fc = R d.
hipError_t resid_restrict(const Grid& g, const double* u, const double* src, double* uc,
                          double* uhat, double* fc, hipStream_t s);

// FAS right-hand side on a coarse level: f = L^H(uhat) - f (f holds R d on entry).
hipError_t fas_rhs(const Grid& gc, const double* uhat, double* f, hipStream_t s);

// uf += P(uc - uhat), cell-centred trilinear 27/9/3/1 over 64, periodic.
hipError_t prolong_correct(const Grid& gc, double* uf, const double* uc, const double* uhat,
                           hipStream_t s);

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

// Number of doubles the partial-sum scratch of the reductions needs.
long long reduction_scratch();

}  // namespace mgfr
