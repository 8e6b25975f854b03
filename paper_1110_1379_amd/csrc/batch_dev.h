// Device code shared by the batched kernels (one launch per multigrid depth over many units)
// and the workgroup-per-unit kernels (a unit's whole solve, or the coarse levels of its
// V-cycle, in one workgroup): the cell operators of a unit grid and the coarsest-level
// solves, in both precisions.
//
// A patch is a cube of active cells whose outside neighbours are ghost cells (Sec. V): for a
// ghost with mask ratio r = m_ghost/m_i = -1 (all cells of a cube patch are active) the ghost
// value is u_g = u_b - r u_b + r u_i = 2 u_b - u_i with the boundary value u_b fixed before
// the relaxation (eq. u_i-1jk), b_g = exp(u_g) (not interpolated), and the face term of
// eq. bc_modified_fR_op is C (b_g + b_i)(u_g - u_i).  A box is periodic.
//
// Single precision (mixed solves): the correction equation N(e) = r of device_fp32.h.  On a
// patch the ghost's double-precision value u_g = (1 - r) u_b + r u_i splits, with
// u_i = ub_i + e_i, into the base (1 - r) u_b + r ub_i and the correction r e_i, so the face
// term of N is (M_g + M_i)(ub_g - ub_i) + (B_g + B_i)(e_g - e_i), the correction form of the
// face term of eq. bc_modified_fR_op, with derivative in e_i
//   (r B_g + B_i)(ub_g - ub_i + e_g - e_i) + (B_g + B_i)(r - 1).
#pragma once

#include "device_fp32.h"
#include "device_fp64.h"

#include <type_traits>

namespace mgfr {
namespace bdev {

constexpr double kR = -1.0;    // ghost mask ratio of a cube patch
constexpr float kR32 = -1.0f;

using dev::OpVal;
using dev32::em1f;
using dev32::make_v;
using dev32::newton32;
using dev32::Op32;
using dev32::op32;
using dev32::Res32;
using dev32::V32;

__device__ __forceinline__ long long idx3(int lg, int i, int j, int k)
{
    return ((((long long)i << lg) + j) << lg) + k;
}

// element of the boundary values [6][n][n] (n = 2^lg) next to cell (i, j, k) through face f
__device__ __forceinline__ int face_index(int lg, int f, int i, int j, int k)
{
    int p, q;
    if (f < 2) { p = j; q = k; }
    else if (f < 4) { p = i; q = k; }
    else { p = i; q = j; }
    return (((f << lg) + p) << lg) + q;
}

__device__ __forceinline__ double face_ub(const BGrid& g, int f, int i, int j, int k)
{
    return g.ub[face_index(g.lg, f, i, j, k)];
}

// boundary value u_b of face f next to cell (i, j, k), rounded to single precision
__device__ __forceinline__ float face_ub32(const BGrid& g, int f, int i, int j, int k)
{
    return (float)face_ub(g, f, i, j, k);
}

// L_i - f_i and dL_i/du_i with ghost faces on the outside of a patch.
__device__ inline OpVal bcell(const BGrid& g, const double* __restrict__ u, int i, int j, int k, double f)
{
    const int n = g.n, m = n - 1;
    const double ui = u[idx3(g.lg, i, j, k)];
    const double bi = exp(ui);
    double su = 0.0, sb = 0.0, sbu = 0.0, lg_ = 0.0, dlg = 0.0;
    int nreg = 0;
    const int di[6] = {-1, 1, 0, 0, 0, 0}, dj[6] = {0, 0, -1, 1, 0, 0}, dk[6] = {0, 0, 0, 0, -1, 1};
#pragma unroll
    for (int q = 0; q < 6; ++q) {
        int ii = i + di[q], jj = j + dj[q], kk = k + dk[q];
        const bool out = ii < 0 || ii > m || jj < 0 || jj > m || kk < 0 || kk > m;
        if (out && !g.periodic) {
            const double ug = (1.0 - kR) * face_ub(g, q, i, j, k) + kR * ui;
            const double bg = exp(ug);
            lg_ += (bg + bi) * (ug - ui);
            dlg += (kR * bg + bi) * (ug - ui) + (bg + bi) * (kR - 1.0);
        } else {
            const double un = u[idx3(g.lg, ii & m, jj & m, kk & m)];
            const double bn = exp(un), du = un - ui;
            su += du;
            sb += bn;
            sbu = fma(bn, du, sbu);
            ++nreg;
        }
    }
    const double S = g.A * exp(-ui * g.inv_np1);
    OpVal r;
    r.L = g.C * (fma(bi, su, sbu) + lg_) + S - f;
    r.dL = g.C * (fma(bi, su, -sb) - nreg * bi + dlg) - S * g.inv_np1;
    return r;
}

__device__ __forceinline__ double brhs(const BGrid& g, long long q) { return fma(g.fscale, g.src[q] - g.sref, g.fshift); }

__device__ __forceinline__ bool live(const BTable& t, const BGrid& g) { return t.active == nullptr || t.active[g.unit]; }

// N_i - f_i and dN_i/de_i of cell (i, j, k), base ub and correction e, ghost faces on the
// outside of a patch.
__device__ inline Res32 bcell32(const BGrid& g, const Op32& o, const float* __restrict__ ub,
                                const float* __restrict__ e, int i, int j, int k, float f)
{
    const int m = g.n - 1;
    const V32 c = make_v(ub[idx3(g.lg, i, j, k)], e[idx3(g.lg, i, j, k)]);
    float t1 = 0.0f, t2 = 0.0f, su = 0.0f, se = 0.0f, sB = 0.0f, nreg = 0.0f, lgh = 0.0f, dgh = 0.0f;
    const int di[6] = {-1, 1, 0, 0, 0, 0}, dj[6] = {0, 0, -1, 1, 0, 0}, dk[6] = {0, 0, 0, 0, -1, 1};
#pragma unroll
    for (int q = 0; q < 6; ++q) {
        const int ii = i + di[q], jj = j + dj[q], kk = k + dk[q];
        const bool out = ii < 0 || ii > m || jj < 0 || jj > m || kk < 0 || kk > m;
        if (out && !g.periodic) {
            const float ubg = (1.0f - kR32) * face_ub32(g, q, i, j, k) + kR32 * c.ub;
            const float eg = kR32 * c.e;
            const float bg = __expf(ubg);
            const float Mg = bg * em1f(eg), Bg = bg + Mg;
            const float du = ubg - c.ub, de = eg - c.e;
            lgh += (Mg + c.M) * du + (Bg + c.B) * de;
            dgh += (kR32 * Bg + c.B) * (du + de) + (Bg + c.B) * (kR32 - 1.0f);
        } else {
            const long long qn = idx3(g.lg, ii & m, jj & m, kk & m);
            const V32 nb = make_v(ub[qn], e[qn]);
            const float du = nb.ub - c.ub, de = nb.e - c.e;
            t1 = fmaf(nb.M, du, t1);
            t2 = fmaf(nb.B, de, t2);
            su += du;
            se += de;
            sB += nb.B;
            nreg += 1.0f;
        }
    }
    const float S = o.A * __expf(-c.ub * o.inv_np1);
    const float x = em1f(-c.e * o.inv_np1);
    Res32 r;
    r.N = o.C * (fmaf(c.M, su, t1) + fmaf(c.B, se, t2) + lgh) + S * x - f;
    r.dN = o.C * (c.B * (su + se) - sB - nreg * c.B + dgh) - S * o.inv_np1 * (1.0f + x);
    return r;
}

// Orders the LDS accesses of one wavefront before and after it (its lanes run in lockstep and
// the LDS serves a wavefront's accesses in order; this keeps the compiler from moving them).
__device__ __forceinline__ void wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// ---- coarsest level in one workgroup of NT threads (n <= 8) -------------------------------
// LDS of the double-precision solve: u, b = exp(u), the curvature term S and the right-hand
// side of every cell, and the reduction buffers.
template <int NT>
struct Coarse64 {
    double su[512], sb[512], sS[512], sf[512];
    double ra[NT], rb[NT];
};

// The arrays of a double-precision coarsest solve in LDS: u, b = exp(u), S = A exp(-u/(n+1))
// and the right-hand side of every cell, and two reduction buffers of NT entries.
struct C64 {
    double *su, *sb, *sS;
    const double* sf;
    double *ra, *rb;
};

// Double precision: b = exp(u) and S of every cell stay in LDS and are refreshed when the
// cell is updated, so a visit evaluates exponentials only for its ghost faces.  The
// arithmetic is that of bcell, in the same order.  Sweeps until rms <= rtol x initial, or its
// rounding floor, or cap sweeps (rtol = 0: exactly cap).  Every thread of the workgroup calls
// it, with (su, sb, sS, sf) filled and visible to all.  A level of at most 64 cells is relaxed
// by the first wavefront alone (one cell per lane), with the same sums in the same order:
// its sweeps then cost no workgroup barriers.
template <int NT, class FaceFn>
__device__ void coarsest64_core(const BGrid& g, int cap, double rtol, const C64& sm, FaceFn face)
{
    const int nc = 1 << (3 * g.lg), m = g.n - 1;
    const int di[6] = {-1, 1, 0, 0, 0, 0}, dj[6] = {0, 0, -1, 1, 0, 0}, dk[6] = {0, 0, 0, 0, -1, 1};
    auto cell = [&](int q) -> OpVal {
        const int i = q >> (2 * g.lg), j = (q >> g.lg) & m, k = q & m;
        const double ui = sm.su[q], bi = sm.sb[q];
        double s_u = 0.0, s_b = 0.0, sbu = 0.0, lg_ = 0.0, dlg = 0.0;
        int nreg = 0;
#pragma unroll
        for (int f = 0; f < 6; ++f) {
            const int ii = i + di[f], jj = j + dj[f], kk = k + dk[f];
            const bool out = ii < 0 || ii > m || jj < 0 || jj > m || kk < 0 || kk > m;
            if (out && !g.periodic) {
                const double ug = (1.0 - kR) * face(f, i, j, k) + kR * ui;
                const double bg = exp(ug);
                lg_ += (bg + bi) * (ug - ui);
                dlg += (kR * bg + bi) * (ug - ui) + (bg + bi) * (kR - 1.0);
            } else {
                const int qn = ((ii & m) << (2 * g.lg)) + ((jj & m) << g.lg) + (kk & m);
                const double bn = sm.sb[qn], du = sm.su[qn] - ui;
                s_u += du;
                s_b += bn;
                sbu = fma(bn, du, sbu);
                ++nreg;
            }
        }
        const double S = sm.sS[q];
        OpVal r;
        r.L = g.C * (fma(bi, s_u, sbu) + lg_) + S - sm.sf[q];
        r.dL = g.C * (fma(bi, s_u, -s_b) - nreg * bi + dlg) - S * g.inv_np1;
        return r;
    };
    // Sums over the workgroup by the tree ra[t] += ra[t + w], w = NT/2 .. 1; in one wavefront
    // (WAVE) the same tree by lane shuffles (threads 64 .. NT - 1 would only add zeros).
    auto solve = [&](auto W) {
        constexpr bool WAVE = decltype(W)::value;
        auto reduce = [&](double a, double b, double& ta, double& tb) {
            if constexpr (WAVE) {
                for (int w = 32; w > 0; w >>= 1) {
                    a += __shfl_down(a, w);
                    b += __shfl_down(b, w);
                }
                ta = __shfl(a, 0);
                tb = __shfl(b, 0);
            } else {
                sm.ra[threadIdx.x] = a;
                sm.rb[threadIdx.x] = b;
                __syncthreads();
                for (int w = NT / 2; w > 0; w >>= 1) {
                    if (threadIdx.x < w) {
                        sm.ra[threadIdx.x] += sm.ra[threadIdx.x + w];
                        sm.rb[threadIdx.x] += sm.rb[threadIdx.x + w];
                    }
                    __syncthreads();
                }
                ta = sm.ra[0];
                tb = sm.rb[0];
                __syncthreads();
            }
        };
        // rms of L - f and its rounding floor (one unit in the last place of |dL||u| + |f| + S)
        auto rms = [&](double& floor) {
            double s = 0.0, fl = 0.0;
            for (int q = threadIdx.x; q < nc; q += NT) {
                const OpVal r = cell(q);
                s += r.L * r.L;
                const double f1 = 2.220446049250313e-16 * (fabs(r.dL) * fabs(sm.su[q]) + fabs(sm.sf[q]) + sm.sS[q]);
                fl += f1 * f1;
            }
            double ts, tf;
            reduce(s, fl, ts, tf);
            floor = sqrt(tf / nc);
            return sqrt(ts / nc);
        };
        double fl0;
        const double r0 = rtol > 0.0 ? rms(fl0) : 0.0;
        for (int sweep = 0; sweep < cap; ++sweep) {
            if (rtol > 0.0) {
                double fl;
                const double r = rms(fl);
                if (r <= rtol * r0 || r <= fl) break;
            }
            for (int colour = 0; colour < 2; ++colour) {
                for (int q = threadIdx.x; q < nc; q += NT) {
                    const int i = q >> (2 * g.lg), j = (q >> g.lg) & m, k = q & m;
                    if (((i + j + k) & 1) != colour) continue;
                    const OpVal r = cell(q);
                    const double u = sm.su[q] + dev::bounded(-r.L / r.dL, g.max_step);
                    sm.su[q] = u;
                    sm.sb[q] = exp(u);
                    sm.sS[q] = g.A * exp(-u * g.inv_np1);
                }
                if constexpr (WAVE) wave_sync();
                else __syncthreads();
            }
        }
    };
    if (NT >= 64 && nc <= 64) {
        // a level of at most 64 cells is relaxed by the first wavefront alone, without
        // workgroup barriers; the others wait for it at the one barrier below
        if (threadIdx.x < 64) solve(std::true_type{});
        __syncthreads();
    } else {
        solve(std::false_type{});
    }
}

// The coarsest level of a unit held in device memory: loaded into sm, solved, u written back.
template <int NT>
__device__ void coarsest64(const BGrid& g, int cap, double rtol, Coarse64<NT>& sm)
{
    const int nc = 1 << (3 * g.lg);
    for (int q = threadIdx.x; q < nc; q += NT) {
        sm.su[q] = g.u[q];
        sm.sb[q] = exp(sm.su[q]);
        sm.sS[q] = g.A * exp(-sm.su[q] * g.inv_np1);
        sm.sf[q] = brhs(g, q);
    }
    __syncthreads();
    coarsest64_core<NT>(g, cap, rtol, C64{sm.su, sm.sb, sm.sS, sm.sf, sm.ra, sm.rb},
                        [&](int f, int i, int j, int k) { return face_ub(g, f, i, j, k); });
    for (int q = threadIdx.x; q < nc; q += NT) g.u[q] = sm.su[q];
    __syncthreads();
}

// LDS of the single-precision solve: per cell the base, b = exp(ub), the correction and its
// (B, M), the right-hand side and S; per ghost face ub_g - ub_i and b_g.
template <int NT>
struct Coarse32 {
    float sub[512], sb[512], se[512], sB[512], sM[512], sf[512], sS[512];
    float gdu[6][512], gbb[6][512];
    float ra[NT], rb[NT];
};

// The arrays of a single-precision coarsest solve in LDS: per cell the base ub, b = exp(ub),
// the correction e and its (B, M), the right-hand side and S; per ghost face (stride 512)
// ub_g - ub_i and b_g; two reduction buffers of NT entries.
struct C32 {
    float *sub, *sb, *se, *sB, *sM, *sS;
    const float* sf;
    float *gdu, *gbb;
    float *ra, *rb;
};

// Single precision: everything that depends only on the base stays in LDS for the whole
// solve; per sweep only the correction-dependent parts (M, B) of the updated cells are
// recomputed.  The arithmetic is that of bcell32, in the same order.  Every thread of the
// workgroup calls it, with every array filled and visible to all; a level of at most 64 cells
// is relaxed by the first wavefront alone, as in coarsest64_core.
template <int NT>
__device__ void coarsest32_core(const BGrid& g, int cap, float rtol, const C32& sm)
{
    const Op32 o = op32(g);
    const int nc = 1 << (3 * g.lg), m = g.n - 1;
    const int di[6] = {-1, 1, 0, 0, 0, 0}, dj[6] = {0, 0, -1, 1, 0, 0}, dk[6] = {0, 0, 0, 0, -1, 1};
    auto ghost = [&](int q, int f) {
        const int i = q >> (2 * g.lg), j = (q >> g.lg) & m, k = q & m;
        const int ii = i + di[f], jj = j + dj[f], kk = k + dk[f];
        return !g.periodic && (ii < 0 || ii > m || jj < 0 || jj > m || kk < 0 || kk > m);
    };
    auto cell = [&](int q, float& dN) -> float {
        const int i = q >> (2 * g.lg), j = (q >> g.lg) & m, k = q & m;
        const float cub = sm.sub[q], ce = sm.se[q], cB = sm.sB[q], cM = sm.sM[q];
        float t1 = 0.0f, t2 = 0.0f, su = 0.0f, sE = 0.0f, sBn = 0.0f, nreg = 0.0f, lgh = 0.0f, dgh = 0.0f;
#pragma unroll
        for (int f = 0; f < 6; ++f) {
            if (ghost(q, f)) {
                const float eg = kR32 * ce;
                const float bg = sm.gbb[f * 512 + q];
                const float Mg = bg * em1f(eg), Bg = bg + Mg;
                const float du = sm.gdu[f * 512 + q], de = eg - ce;
                lgh += (Mg + cM) * du + (Bg + cB) * de;
                dgh += (kR32 * Bg + cB) * (du + de) + (Bg + cB) * (kR32 - 1.0f);
            } else {
                const int qn = (((i + di[f]) & m) << (2 * g.lg)) + (((j + dj[f]) & m) << g.lg) + ((k + dk[f]) & m);
                const float du = sm.sub[qn] - cub, de = sm.se[qn] - ce;
                t1 = fmaf(sm.sM[qn], du, t1);
                t2 = fmaf(sm.sB[qn], de, t2);
                su += du;
                sE += de;
                sBn += sm.sB[qn];
                nreg += 1.0f;
            }
        }
        const float S = sm.sS[q];
        const float x = em1f(-ce * o.inv_np1);
        dN = o.C * (cB * (su + sE) - sBn - nreg * cB + dgh) - S * o.inv_np1 * (1.0f + x);
        return o.C * (fmaf(cM, su, t1) + fmaf(cB, sE, t2) + lgh) + S * x - sm.sf[q];
    };
    // Sums as in coarsest64_core: the LDS tree over the workgroup, or in one wavefront (WAVE)
    // the same tree by lane shuffles.
    auto solve = [&](auto W) {
        constexpr bool WAVE = decltype(W)::value;
        // rms of N - f and its single-precision rounding floor (|dN||e| + |f|)
        auto rms = [&](float& floor) {
            float s = 0.0f, fl = 0.0f;
            for (int q = threadIdx.x; q < nc; q += NT) {
                float dN;
                const float N = cell(q, dN);
                s += N * N;
                const float f1 = 1.1920929e-7f * (fabsf(dN) * fabsf(sm.se[q]) + fabsf(sm.sf[q]));
                fl += f1 * f1;
            }
            float tot, tf;
            if constexpr (WAVE) {
                for (int w = 32; w > 0; w >>= 1) {
                    s += __shfl_down(s, w);
                    fl += __shfl_down(fl, w);
                }
                tot = __shfl(s, 0);
                tf = __shfl(fl, 0);
            } else {
                sm.ra[threadIdx.x] = s;
                sm.rb[threadIdx.x] = fl;
                __syncthreads();
                for (int w = NT / 2; w > 0; w >>= 1) {
                    if (threadIdx.x < w) {
                        sm.ra[threadIdx.x] += sm.ra[threadIdx.x + w];
                        sm.rb[threadIdx.x] += sm.rb[threadIdx.x + w];
                    }
                    __syncthreads();
                }
                tot = sm.ra[0];
                tf = sm.rb[0];
                __syncthreads();
            }
            floor = sqrtf(tf / nc);
            return sqrtf(tot / nc);
        };
        float fl0;
        const float r0 = rtol > 0.0f ? rms(fl0) : 0.0f;
        for (int sweep = 0; sweep < cap; ++sweep) {
            if (rtol > 0.0f) {
                float fl;
                const float r = rms(fl);
                if (r <= rtol * r0 || r <= fl) break;
            }
            for (int colour = 0; colour < 2; ++colour) {
                for (int q = threadIdx.x; q < nc; q += NT) {
                    const int i = q >> (2 * g.lg), j = (q >> g.lg) & m, k = q & m;
                    if (((i + j + k) & 1) != colour) continue;
                    Res32 r;
                    r.N = cell(q, r.dN);
                    const float e = sm.se[q] + newton32(r, o.max_step);
                    const float M = sm.sb[q] * em1f(e);
                    sm.se[q] = e;
                    sm.sM[q] = M;
                    sm.sB[q] = sm.sb[q] + M;
                }
                if constexpr (WAVE) wave_sync();
                else __syncthreads();
            }
        }
    };
    if (NT >= 64 && nc <= 64) {
        if (threadIdx.x < 64) solve(std::true_type{});
        __syncthreads();
    } else {
        solve(std::false_type{});
    }
}

// The ghost-face terms of the coarsest solve that depend only on the base (cell q of g with
// base ub): ub_g - ub and b_g per ghost face, zero elsewhere; face(f, i, j, k) gives the
// boundary value in single precision.
template <class FaceFn>
__device__ inline void coarse_ghosts32(const BGrid& g, int q, float ub, float* gdu, float* gbb, FaceFn face)
{
    const int m = g.n - 1;
    const int i = q >> (2 * g.lg), j = (q >> g.lg) & m, k = q & m;
    const int di[6] = {-1, 1, 0, 0, 0, 0}, dj[6] = {0, 0, -1, 1, 0, 0}, dk[6] = {0, 0, 0, 0, -1, 1};
    for (int f = 0; f < 6; ++f) {
        gdu[f * 512 + q] = 0.0f;
        gbb[f * 512 + q] = 0.0f;
        const int ii = i + di[f], jj = j + dj[f], kk = k + dk[f];
        if (!g.periodic && (ii < 0 || ii > m || jj < 0 || jj > m || kk < 0 || kk > m)) {
            const float ubg = (1.0f - kR32) * face(f, i, j, k) + kR32 * ub;
            gdu[f * 512 + q] = ubg - ub;
            gbb[f * 512 + q] = __expf(ubg);
        }
    }
}

// The coarsest level of a unit held in device memory: loaded into sm, solved, e written back.
template <int NT>
__device__ void coarsest32(const BGrid& g, int cap, float rtol, Coarse32<NT>& sm)
{
    const Op32 o = op32(g);
    const int nc = 1 << (3 * g.lg);
    for (int q = threadIdx.x; q < nc; q += NT) {
        const V32 v = make_v(g.ub32[q], g.e32[q]);
        sm.sub[q] = v.ub;
        sm.sb[q] = __expf(v.ub);
        sm.se[q] = v.e;
        sm.sB[q] = v.B;
        sm.sM[q] = v.M;
        sm.sf[q] = g.f32[q];
        sm.sS[q] = o.A * __expf(-v.ub * o.inv_np1);
        coarse_ghosts32(g, q, v.ub, &sm.gdu[0][0], &sm.gbb[0][0],
                        [&](int f, int i, int j, int k) { return face_ub32(g, f, i, j, k); });
    }
    __syncthreads();
    coarsest32_core<NT>(g, cap, rtol,
                        C32{sm.sub, sm.sb, sm.se, sm.sB, sm.sM, sm.sS, sm.sf, &sm.gdu[0][0], &sm.gbb[0][0], sm.ra, sm.rb});
    for (int q = threadIdx.x; q < nc; q += NT) g.e32[q] = sm.se[q];
    __syncthreads();
}

}  // namespace bdev
}  // namespace mgfr
