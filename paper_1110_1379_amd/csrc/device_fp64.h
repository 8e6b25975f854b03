// Device helpers of the double-precision kernels: the cell operator of the f(R) equation
// in the variable u (f~_R = -exp(u)), eq. discrete_fR times c~^2 (= eq. bc_modified_fR_op
// for a cell with no ghost neighbour) and its diagonal derivative (eq. bc_modified_fR_dop).
#pragma once

#include "mgfr_impl.h"

namespace mgfr {
namespace dev {

struct OpVal {
    double L, dL;
};

// Curvature term S = A exp(-u/(n+1)).  For n = 1 it is A / sqrt(b) with b = exp(u) already
// at hand: the hardware reciprocal square root refined by two Newton steps (each doubles
// the correct bits), instead of a second double-precision exponential.
__device__ __forceinline__ double curvature(const Grid& g, double ui, double bi)
{
    if (g.half_power) {
        double y = __builtin_amdgcn_rsq(bi);
        double e = fma(-bi * y, y, 1.0);
        y = fma(0.5 * y, e, y);
        e = fma(-bi * y, y, 1.0);
        y = fma(0.5 * y, e, y);
        return g.A * y;
    }
    return g.A * exp(-ui * g.inv_np1);
}

// L_i - f_i and dL_i/du_i from the cell value, its six neighbours and their b = exp(u).
__device__ __forceinline__ OpVal cell_op_b(const Grid& g, double ui, double bi, const double (&un)[6],
                                           const double (&bn)[6], double f)
{
    double su = 0.0, sb = 0.0, sbu = 0.0;
#pragma unroll
    for (int q = 0; q < 6; ++q) {
        const double du = un[q] - ui;
        su += du;
        sb += bn[q];
        sbu = fma(bn[q], du, sbu);
    }
    const double S = curvature(g, ui, bi);
    OpVal r;
    // sum_nb (b_nb + b_i)(u_nb - u_i) = sum b_nb du + b_i sum du
    r.L = g.C * fma(bi, su, sbu) + S - f;
    // sum_nb [b_i (u_nb - u_i) - b_nb - b_i]
    r.dL = g.C * (fma(bi, su, -sb) - 6.0 * bi) - S * g.inv_np1;
    return r;
}

__device__ __forceinline__ OpVal cell_op(const Grid& g, double ui, const double (&un)[6], double f)
{
    double bn[6];
#pragma unroll
    for (int q = 0; q < 6; ++q) bn[q] = exp(un[q]);
    return cell_op_b(g, ui, exp(ui), un, bn, f);
}

__device__ __forceinline__ double rhs_value(const Grid& g, double src)
{
    return fma(g.fscale, src - g.sref, g.fshift);
}

__device__ __forceinline__ long long at(const Grid& g, int i, int j, int k)
{
    return ((((long long)i << g.lg) + j) << g.lg) + k;
}

// Newton step, bounded to [-ms, ms] when ms > 0; comparisons (not fmin/fmax) keep a NaN step NaN.
__device__ __forceinline__ double bounded(double step, double ms)
{
    if (ms > 0.0) {
        if (step > ms) step = ms;
        if (step < -ms) step = -ms;
    }
    return step;
}

}  // namespace dev
}  // namespace mgfr
