// Types that the HIP kernels take by value: the level descriptors and launch geometries of
// the domain, streaming and Poisson kernels.  Kept apart from the launcher declarations so
// that a change to those does not touch what the kernels are compiled from.
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
    int half_power;   // 1 when n_HS = 1: exp(-u/2) is taken as 1/sqrt(exp(u))
    double max_step;  // > 0: bound on |Newton step|
    double fscale, sref, fshift;
    const int* halt;  // device flag, or null: when it is set the kernels of a level return at once
};

inline long long cells(const Grid& g) { return 1LL << (3 * g.lg); }

// Launch geometry of the single-precision fused sweep (kernels_fp32.hip).
struct FusedSweep32 {
    int ti, ntj, ntk;
};

// Outputs of the streaming residual (resid_fp64.hip); null pointers switch parts off.
struct ResidStream {
    int ti, ntj, ntk;              // planes per workgroup (even); tiles (set by the launcher)
    double* partial;               // NORM: 2 doubles per workgroup (sum d^2, max |d|)
    double *uc, *uhat, *fc;        // RESTRICT: coarse R u (twice) and R d
    const float* e32;              // UPDATE: correction added to every loaded u ...
    double* uout;                  // ... and the updated u of the tile written here
    float *r32, *ub32;             // CAST: -d and u in single precision
};

// Launch geometry of the fused sweep (sweep_fp64.hip).
struct FusedSweep {
    int ti;            // planes per workgroup chunk
    int ntj, ntk;      // tiles along j and k (set by the launcher)
};

// ---- modified Poisson solve (poisson_kernels.hip) -----------------------------------------
// One periodic level of the linear solve: side n = 2^lg, h^2 and 1/h^2 (h = 1/n on the box).
struct PGrid {
    int n, lg;
    double hh, inv_hh;
};

// Constants of the source S = 2 D (rho~ - 1) - (A exp(-u inv_np1) - Sbar) / 2.
struct PoissonSource {
    double D, A, inv_np1, Sbar;
};

}  // namespace mgfr
