// Batched single-precision correction kernels of the mixed-precision patch and box solves.
//
// Same batching as batch_fp64.hip (one launch per multigrid depth over every unit, a block
// table of (unit grid, block) pairs, per-unit active flags), applied to the correction
// equation N(e) = r of device_fp32.h.  On a patch, a ghost cell outside face f has the
// double-precision value u_g = (1 - r) u_b + r u_i with u_b fixed (eq. u_i-1jk, r = -1 for a
// cube patch).  Splitting u_i = ub_i + e_i, the ghost's base is (1 - r) u_b + r ub_i and its
// correction r e_i, so the face term of N is
//   (M_g + M_i)(ub_g - ub_i) + (B_g + B_i)(e_g - e_i),
// the correction form of the face term of eq. bc_modified_fR_op, and its derivative in e_i
//   (r B_g + B_i)(ub_g - ub_i + e_g - e_i) + (B_g + B_i)(r - 1).
#include "device_fp32.h"

namespace mgfr {
namespace {

using dev32::em1f;
using dev32::make_v;
using dev32::newton32;
using dev32::Op32;
using dev32::op32;
using dev32::Res32;
using dev32::V32;

constexpr int kB = 256;
constexpr float kR = -1.0f;  // ghost mask ratio of a cube patch

__device__ __forceinline__ long long idx3(int lg, int i, int j, int k)
{
    return ((((long long)i << lg) + j) << lg) + k;
}

// boundary value u_b of face f next to cell (i, j, k), rounded to single precision
__device__ __forceinline__ float face_ub32(const BGrid& g, int f, int i, int j, int k)
{
    int p, q;
    if (f < 2) { p = j; q = k; }
    else if (f < 4) { p = i; q = k; }
    else { p = i; q = j; }
    return (float)g.ub[((((long long)f << g.lg) + p) << g.lg) + q];
}

__device__ __forceinline__ bool live(const BTable& t, const BGrid& g) { return t.active == nullptr || t.active[g.unit]; }

// N_i - f_i and dN_i/de_i of cell (i, j, k), base ub and correction e, ghost faces on the
// outside of a patch.
__device__ Res32 bcell32(const BGrid& g, const Op32& o, const float* __restrict__ ub, const float* __restrict__ e,
                         int i, int j, int k, float f)
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
            const float ubg = (1.0f - kR) * face_ub32(g, q, i, j, k) + kR * c.ub;
            const float eg = kR * c.e;
            const float bg = __expf(ubg);
            const float Mg = bg * em1f(eg), Bg = bg + Mg;
            const float du = ubg - c.ub, de = eg - c.e;
            lgh += (Mg + c.M) * du + (Bg + c.B) * de;
            dgh += (kR * Bg + c.B) * (du + de) + (Bg + c.B) * (kR - 1.0f);
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

// ---- smoother: one colour per launch, one thread per cell of that colour ------------------
__global__ void __launch_bounds__(kB) kb32_ngs(BTable t, int colour)
{
    const int2 b = t.blk[blockIdx.x];
    const BGrid g = t.grids[b.x];
    if (!live(t, g)) return;
    const long long half = 1LL << (3 * g.lg - 1);
    const long long tt = (long long)b.y * kB + threadIdx.x;
    if (tt >= half) return;
    const int hk = g.n >> 1;
    const int s = (int)(tt & (hk - 1));
    const long long row = tt >> (g.lg - 1);
    const int i = (int)(row >> g.lg), j = (int)(row & (g.n - 1));
    const int k = 2 * s + ((i + j + colour) & 1);
    const long long q = idx3(g.lg, i, j, k);
    const Op32 o = op32(g);
    const Res32 r = bcell32(g, o, g.ub32, g.e32, i, j, k, g.f32[q]);
    g.e32[q] = g.e32[q] + newton32(r, o.max_step);
}

// ---- residual + restriction (table over the coarse cells; tc = coarse grids) -------------
__global__ void __launch_bounds__(kB) kb32_resid_restrict(BTable t, const BGrid* __restrict__ tc)
{
    const int2 b = t.blk[blockIdx.x];
    const BGrid g = t.grids[b.x];
    if (!live(t, g)) return;
    const BGrid c = tc[b.x];
    const long long qc = (long long)b.y * kB + threadIdx.x;
    if (qc >= (1LL << (3 * c.lg))) return;
    const int I = (int)(qc >> (2 * c.lg)), J = (int)((qc >> c.lg) & (c.n - 1)), K = (int)(qc & (c.n - 1));
    const Op32 o = op32(g);
    float se = 0.0f, sd = 0.0f;
    for (int a = 0; a < 2; ++a)
        for (int bb = 0; bb < 2; ++bb)
            for (int z = 0; z < 2; ++z) {
                const int i = 2 * I + a, j = 2 * J + bb, k = 2 * K + z;
                const long long q = idx3(g.lg, i, j, k);
                se += g.e32[q];
                sd += bcell32(g, o, g.ub32, g.e32, i, j, k, g.f32[q]).N;
            }
    c.e32[qc] = 0.125f * se;
    c.eh32[qc] = 0.125f * se;
    c.f32[qc] = 0.125f * sd;
}

// coarse base R ub (table over the coarse cells; tc = coarse grids)
__global__ void __launch_bounds__(kB) kb32_restrict_base(BTable t, const BGrid* __restrict__ tc)
{
    const int2 b = t.blk[blockIdx.x];
    const BGrid g = t.grids[b.x];
    if (!live(t, g)) return;
    const BGrid c = tc[b.x];
    const long long qc = (long long)b.y * kB + threadIdx.x;
    if (qc >= (1LL << (3 * c.lg))) return;
    const int I = (int)(qc >> (2 * c.lg)), J = (int)((qc >> c.lg) & (c.n - 1)), K = (int)(qc & (c.n - 1));
    float s = 0.0f;
    for (int a = 0; a < 2; ++a)
        for (int bb = 0; bb < 2; ++bb)
            for (int z = 0; z < 2; ++z) s += g.ub32[idx3(g.lg, 2 * I + a, 2 * J + bb, 2 * K + z)];
    c.ub32[qc] = 0.125f * s;
}

// f = N^H(eh) - f on coarse grids (f holds R d on entry)
__global__ void __launch_bounds__(kB) kb32_fas_rhs(BTable t)
{
    const int2 b = t.blk[blockIdx.x];
    const BGrid c = t.grids[b.x];
    if (!live(t, c)) return;
    const long long q = (long long)b.y * kB + threadIdx.x;
    if (q >= (1LL << (3 * c.lg))) return;
    const int i = (int)(q >> (2 * c.lg)), j = (int)((q >> c.lg) & (c.n - 1)), k = (int)(q & (c.n - 1));
    c.f32[q] = bcell32(c, op32(c), c.ub32, c.eh32, i, j, k, 0.0f).N - c.f32[q];
}

__global__ void __launch_bounds__(kB) kb32_coarse_diff(BTable t)
{
    const int2 b = t.blk[blockIdx.x];
    const BGrid c = t.grids[b.x];
    if (!live(t, c)) return;
    const long long q = (long long)b.y * kB + threadIdx.x;
    if (q >= (1LL << (3 * c.lg))) return;
    c.eh32[q] = c.e32[q] - c.eh32[q];
}

// e += P(coarse difference) on fine grids; outside a patch a coarse cell contributes zero
// (Sec. V.A.3)
__global__ void __launch_bounds__(kB) kb32_prolong_add(BTable t, const BGrid* __restrict__ tc)
{
    const int2 b = t.blk[blockIdx.x];
    const BGrid g = t.grids[b.x];
    if (!live(t, g)) return;
    const BGrid c = tc[b.x];
    const long long q = (long long)b.y * kB + threadIdx.x;
    if (q >= (1LL << (3 * g.lg))) return;
    const int i = (int)(q >> (2 * g.lg)), j = (int)((q >> g.lg) & (g.n - 1)), k = (int)(q & (g.n - 1));
    const int I = i >> 1, J = j >> 1, K = k >> 1;
    const int si = (i & 1) ? 1 : -1, sj = (j & 1) ? 1 : -1, sk = (k & 1) ? 1 : -1;
    const int mc = c.n - 1;
    auto E = [&](int a, int bb, int z) -> float {
        if (c.periodic) return c.eh32[idx3(c.lg, a & mc, bb & mc, z & mc)];
        if (a < 0 || a > mc || bb < 0 || bb > mc || z < 0 || z > mc) return 0.0f;
        return c.eh32[idx3(c.lg, a, bb, z)];
    };
    const float p = (27.0f / 64.0f) * E(I, J, K) +
                    (9.0f / 64.0f) * (E(I + si, J, K) + E(I, J + sj, K) + E(I, J, K + sk)) +
                    (3.0f / 64.0f) * (E(I + si, J + sj, K) + E(I + si, J, K + sk) + E(I, J + sj, K + sk)) +
                    (1.0f / 64.0f) * E(I + si, J + sj, K + sk);
    g.e32[q] += p;
}

// ---- coarsest level: one workgroup per grid (n <= 8) --------------------------------------
// Everything that depends only on the base stays in LDS for the whole solve: ub, b = exp(ub),
// the curvature coefficient S, and per ghost face ub_g - ub_i and b_g; per sweep only the
// correction-dependent parts (M, B) of the updated cells are recomputed.  The arithmetic is
// that of bcell32, in the same order.
template <int NT>
__global__ void __launch_bounds__(NT) kb32_coarsest(const BGrid* __restrict__ grids, const int* __restrict__ active,
                                                   int cap, float rtol)
{
    __shared__ float sub[512], sb[512], se[512], sB[512], sM[512], sf[512], sS[512];
    __shared__ float gdu[6][512], gbb[6][512];
    __shared__ float ra[NT], rb[NT];
    const BGrid g = grids[blockIdx.x];
    if (active && !active[g.unit]) return;
    const Op32 o = op32(g);
    const int nc = 1 << (3 * g.lg), m = g.n - 1;
    const int di[6] = {-1, 1, 0, 0, 0, 0}, dj[6] = {0, 0, -1, 1, 0, 0}, dk[6] = {0, 0, 0, 0, -1, 1};
    auto ghost = [&](int q, int f) {
        const int i = q >> (2 * g.lg), j = (q >> g.lg) & m, k = q & m;
        const int ii = i + di[f], jj = j + dj[f], kk = k + dk[f];
        return !g.periodic && (ii < 0 || ii > m || jj < 0 || jj > m || kk < 0 || kk > m);
    };
    for (int q = threadIdx.x; q < nc; q += NT) {
        const V32 v = make_v(g.ub32[q], g.e32[q]);
        sub[q] = v.ub;
        sb[q] = __expf(v.ub);
        se[q] = v.e;
        sB[q] = v.B;
        sM[q] = v.M;
        sf[q] = g.f32[q];
        sS[q] = o.A * __expf(-v.ub * o.inv_np1);
        const int i = q >> (2 * g.lg), j = (q >> g.lg) & m, k = q & m;
        for (int f = 0; f < 6; ++f) {
            gdu[f][q] = 0.0f;
            gbb[f][q] = 0.0f;
            if (ghost(q, f)) {
                const float ubg = (1.0f - kR) * face_ub32(g, f, i, j, k) + kR * v.ub;
                gdu[f][q] = ubg - v.ub;
                gbb[f][q] = __expf(ubg);
            }
        }
    }
    __syncthreads();
    auto cell = [&](int q, float& dN) -> float {
        const int i = q >> (2 * g.lg), j = (q >> g.lg) & m, k = q & m;
        const float cub = sub[q], ce = se[q], cB = sB[q], cM = sM[q];
        float t1 = 0.0f, t2 = 0.0f, su = 0.0f, sE = 0.0f, sBn = 0.0f, nreg = 0.0f, lgh = 0.0f, dgh = 0.0f;
#pragma unroll
        for (int f = 0; f < 6; ++f) {
            if (ghost(q, f)) {
                const float eg = kR * ce;
                const float bg = gbb[f][q];
                const float Mg = bg * em1f(eg), Bg = bg + Mg;
                const float du = gdu[f][q], de = eg - ce;
                lgh += (Mg + cM) * du + (Bg + cB) * de;
                dgh += (kR * Bg + cB) * (du + de) + (Bg + cB) * (kR - 1.0f);
            } else {
                const int qn = (((i + di[f]) & m) << (2 * g.lg)) + (((j + dj[f]) & m) << g.lg) + ((k + dk[f]) & m);
                const float du = sub[qn] - cub, de = se[qn] - ce;
                t1 = fmaf(sM[qn], du, t1);
                t2 = fmaf(sB[qn], de, t2);
                su += du;
                sE += de;
                sBn += sB[qn];
                nreg += 1.0f;
            }
        }
        const float S = sS[q];
        const float x = em1f(-ce * o.inv_np1);
        dN = o.C * (cB * (su + sE) - sBn - nreg * cB + dgh) - S * o.inv_np1 * (1.0f + x);
        return o.C * (fmaf(cM, su, t1) + fmaf(cB, sE, t2) + lgh) + S * x - sf[q];
    };
    // rms of N - f and its single-precision rounding floor (|dN||e| + |f|)
    auto rms = [&](float& floor) {
        float s = 0.0f, fl = 0.0f;
        for (int q = threadIdx.x; q < nc; q += NT) {
            float dN;
            const float N = cell(q, dN);
            s += N * N;
            const float f1 = 1.1920929e-7f * (fabsf(dN) * fabsf(se[q]) + fabsf(sf[q]));
            fl += f1 * f1;
        }
        ra[threadIdx.x] = s;
        rb[threadIdx.x] = fl;
        __syncthreads();
        for (int w = NT / 2; w > 0; w >>= 1) {
            if (threadIdx.x < w) {
                ra[threadIdx.x] += ra[threadIdx.x + w];
                rb[threadIdx.x] += rb[threadIdx.x + w];
            }
            __syncthreads();
        }
        const float tot = ra[0], tf = rb[0];
        __syncthreads();
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
                const float e = se[q] + newton32(r, o.max_step);
                const float M = sb[q] * em1f(e);
                se[q] = e;
                sM[q] = M;
                sB[q] = sb[q] + M;
            }
            __syncthreads();
        }
    }
    for (int q = threadIdx.x; q < nc; q += NT) g.e32[q] = se[q];
}

}  // namespace

hipError_t batch_restrict_base32(const BTable& t, int nblk, const BGrid* coarse, hipStream_t s)
{
    hipLaunchKernelGGL(kb32_restrict_base, dim3(nblk), dim3(kB), 0, s, t, coarse);
    return hipGetLastError();
}
hipError_t batch_ngs32(const BTable& t, int nblk, hipStream_t s)
{
    for (int colour = 0; colour < 2; ++colour) hipLaunchKernelGGL(kb32_ngs, dim3(nblk), dim3(kB), 0, s, t, colour);
    return hipGetLastError();
}
hipError_t batch_resid_restrict32(const BTable& t, int nblk, const BGrid* coarse, hipStream_t s)
{
    hipLaunchKernelGGL(kb32_resid_restrict, dim3(nblk), dim3(kB), 0, s, t, coarse);
    return hipGetLastError();
}
hipError_t batch_fas_rhs32(const BTable& t, int nblk, hipStream_t s)
{
    hipLaunchKernelGGL(kb32_fas_rhs, dim3(nblk), dim3(kB), 0, s, t);
    return hipGetLastError();
}
hipError_t batch_coarse_diff32(const BTable& t, int nblk, hipStream_t s)
{
    hipLaunchKernelGGL(kb32_coarse_diff, dim3(nblk), dim3(kB), 0, s, t);
    return hipGetLastError();
}
hipError_t batch_prolong_add32(const BTable& t, int nblk, const BGrid* coarse, hipStream_t s)
{
    hipLaunchKernelGGL(kb32_prolong_add, dim3(nblk), dim3(kB), 0, s, t, coarse);
    return hipGetLastError();
}
hipError_t batch_coarsest32(const BGrid* grids, int ngrid, int n, const int* active, int cap, double rtol,
                            hipStream_t s)
{
    // one wavefront per grid when it fits (barriers and reductions stay within the wave)
    if (n <= 4)
        hipLaunchKernelGGL((kb32_coarsest<64>), dim3(ngrid), dim3(64), 0, s, grids, active, cap, (float)rtol);
    else
        hipLaunchKernelGGL((kb32_coarsest<kB>), dim3(ngrid), dim3(kB), 0, s, grids, active, cap, (float)rtol);
    return hipGetLastError();
}

}  // namespace mgfr
