// Device helpers of the single-precision correction solves (domain and batched): the
// correction form of the f(R) operator.  With the base ub (u rounded to single precision)
// fixed, the correction e solves
//   N_i(e) = L_i(ub + e) - L_i(ub) = r_i,
// written with every term proportional to e so that corrections far below the single-
// precision spacing of u are still resolved:
//   N_i(e) = C sum_nb [(M_nb + M_i)(ub_nb - ub_i) + (B_nb + B_i)(e_nb - e_i)]
//          + S_i expm1(-e_i/(n+1))
//   b = exp(ub),  M = b expm1(e),  B = b + M = b exp(e),  S_i = A exp(-ub_i/(n+1)),
// i.e. the flux and curvature terms of eq. discrete_fR (times c~^2) differenced exactly.
#pragma once

#include "mgfr_impl.h"

namespace mgfr {
namespace dev32 {

struct Op32 {
    float C, A, inv_np1, max_step;
};

__device__ __forceinline__ Op32 op32(const Grid& g)
{
    return Op32{(float)g.C, (float)g.A, (float)g.inv_np1, (float)g.max_step};
}

__device__ __forceinline__ Op32 op32(const BGrid& g)
{
    return Op32{(float)g.C, (float)g.A, (float)g.inv_np1, (float)g.max_step};
}

// expm1 in single precision: Taylor series to x^5 for |x| < 1/8 (the first omitted term,
// x^6/720, is below 4.3e-8 of x: under half the single-precision spacing), exp(x) - 1
// above.  Corrections are small once the outer loop has started to converge, so the
// exponential is a branch that whole wavefronts skip.
__device__ __forceinline__ float em1f(float x)
{
    float r = x * (1.0f + x * (0.5f + x * (1.0f / 6.0f + x * (1.0f / 24.0f + x * (1.0f / 120.0f)))));
    if (__builtin_expect(!(fabsf(x) < 0.125f), 0)) r = __expf(x) - 1.0f;
    return r;
}

// Per-cell values a neighbour needs: base, correction, B = b e^e, M = b (e^e - 1).
struct V32 {
    float ub, e, B, M;
};

__device__ __forceinline__ V32 make_v(float ub, float e)
{
    V32 v;
    v.ub = ub;
    v.e = e;
    const float b = __expf(ub);
    v.M = b * em1f(e);
    v.B = b + v.M;
    return v;
}

// The same values after the correction changed to e: b = B - M recovers exp(ub) without a
// second exponential (to the rounding of B).
__device__ __forceinline__ V32 remake_v(const V32& v, float e)
{
    V32 r;
    r.ub = v.ub;
    r.e = e;
    const float b = v.B - v.M;
    r.M = b * em1f(e);
    r.B = b + r.M;
    return r;
}

struct Res32 {
    float N, dN;
};

// N_i - f_i and dN_i/de_i.  The flux sum (M_nb + M_i) du + (B_nb + B_i) de is split into
// the neighbour parts and M_i sum(du) + B_i sum(de).
__device__ __forceinline__ Res32 corr_op(const Op32& o, const V32& c, const V32 (&nb)[6], float f)
{
    float t1 = 0.0f, t2 = 0.0f, su = 0.0f, se = 0.0f, sB = 0.0f;
#pragma unroll
    for (int q = 0; q < 6; ++q) {
        const float du = nb[q].ub - c.ub, de = nb[q].e - c.e;
        t1 = fmaf(nb[q].M, du, t1);
        t2 = fmaf(nb[q].B, de, t2);
        su += du;
        se += de;
        sB += nb[q].B;
    }
    const float S = o.A * __expf(-c.ub * o.inv_np1);
    const float x = em1f(-c.e * o.inv_np1);
    Res32 r;
    r.N = o.C * (fmaf(c.M, su, t1) + fmaf(c.B, se, t2)) + S * x - f;
    r.dN = o.C * (c.B * (su + se) - sB - 6.0f * c.B) - S * o.inv_np1 * (1.0f + x);
    return r;
}

// Newton step -N/dN through the hardware reciprocal (about 1 ulp), bounded to [-ms, ms]
// when ms > 0; a NaN step stays NaN.
__device__ __forceinline__ float newton32(const Res32& r, float ms)
{
    float step = -r.N * __builtin_amdgcn_rcpf(r.dN);
    if (ms > 0.0f) {
        if (step > ms) step = ms;
        if (step < -ms) step = -ms;
    }
    return step;
}

}  // namespace dev32
}  // namespace mgfr
