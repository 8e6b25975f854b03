// Streaming residual of a double-precision level, for n >= 64.
//
// d_i = L_i(u) - f_i (the operator of device_fp64.h).  Each workgroup owns a TJ x 64 tile of
// (j,k) columns and a chunk of planes; per plane it stages u and b = exp(u) of the tile plus
// a one-cell in-plane halo in LDS, and keeps the i-neighbours in registers, so every cell's
// exponential is evaluated once.  What is done with d is chosen at compile time:
//   NORM      per-workgroup partial sum of d^2 and max |d| (NaN-propagating)
//   RESTRICT  8-child means of u and d into the coarse level: uc = uhat = R u, fc = R d
//   UPDATE    u = uin + e (e single precision, the correction of the defect-correction
//             loop) for every loaded cell; the updated tile is written to uout
//   CAST      r = -d and ub = u rounded to single precision (right-hand side and base of
//             the next single-precision correction solve)
#include "device_fp64.h"

namespace mgfr {
namespace {

constexpr int kTK = 64;

template <int TJ, int NT, bool NORM, bool RESTRICT, bool UPDATE, bool CAST>
__global__ void __launch_bounds__(NT) k_resid_stream(Grid g, const double* __restrict__ uin,
                                                     const double* __restrict__ src, ResidStream a)
{
    if (g.halt && *g.halt) return;
    constexpr int LJ = TJ + 2, LK = kTK + 2, NL = LJ * LK;
    constexpr int NS = (NL + NT - 1) / NT;
    __shared__ double lu[2][NL];
    __shared__ double lb[2][NL];
    __shared__ double ru[RESTRICT ? TJ * kTK : 1];
    __shared__ double rd[RESTRICT ? TJ * kTK : 1];
    __shared__ double red_s[NT], red_m[NT];

    const int nb = gridDim.x;
    int lid = blockIdx.x;
    if ((nb & 7) == 0) lid = (lid & 7) * (nb >> 3) + (lid >> 3);
    const int tk = lid % a.ntk;
    lid /= a.ntk;
    const int tj = lid % a.ntj;
    const int ci = lid / a.ntj;
    const int i0 = ci * a.ti, j0 = tj * TJ, k0 = tk * kTK;
    const int lg = g.lg, m = g.n - 1;
    const int last = i0 + a.ti;  // last plane read

    unsigned col[NS];
    int fl[NS], li[NS];
#pragma unroll
    for (int s = 0; s < NS; ++s) {
        const int c = threadIdx.x + s * NT;
        col[s] = 0;
        fl[s] = 0;
        li[s] = 0;
        if (c < NL) {
            const int jj = c / LK, kk = c - jj * LK;
            col[s] = (unsigned)((((j0 - 1 + jj) & m) << lg) | ((k0 - 1 + kk) & m));
            fl[s] = 1;
            if (jj >= 1 && jj <= TJ && kk >= 1 && kk <= kTK) {
                fl[s] |= 2;
                li[s] = (jj - 1) * kTK + (kk - 1);
            }
        }
    }
    // element offsets fit in 32 bits (n <= 1024)
    auto offset = [&](int p, int s) -> unsigned { return ((unsigned)(p & m) << (2 * lg)) + col[s]; };
    auto load_u = [&](int p, int s) -> double {
        double v = uin[offset(p, s)];
        if (UPDATE) v += (double)a.e32[offset(p, s)];
        return v;
    };
    // the correction of a prefetched plane is kept apart and added when the plane is used,
    // so that issuing the loads does not wait for them
    auto load_e = [&](int p, int s) -> float { return UPDATE ? a.e32[offset(p, s)] : 0.0f; };

    // u of planes p-1, p, p+1 in registers while planes p+2 and p+3 (and f of p+1) are in flight
    double um1[NS], u0[NS], up1[NS], bm1[NS], b0[NS], bp1[NS], un2[NS];
    float en2[NS];
    double uprev[NS], dprev[NS], f0[NS];
#pragma unroll
    for (int s = 0; s < NS; ++s) {
        um1[s] = u0[s] = up1[s] = bm1[s] = b0[s] = bp1[s] = un2[s] = f0[s] = 0.0;
        en2[s] = 0.0f;
        uprev[s] = dprev[s] = 0.0;
        if (fl[s] & 2) f0[s] = src[offset(i0, s)];
        if (fl[s]) {
            um1[s] = load_u(i0 - 1, s);
            u0[s] = load_u(i0, s);
            up1[s] = load_u(i0 + 1, s);
            un2[s] = uin[offset(i0 + 2, s)];
            en2[s] = load_e(i0 + 2, s);
            bm1[s] = exp(um1[s]);
            b0[s] = exp(u0[s]);
            bp1[s] = exp(up1[s]);
            lu[0][threadIdx.x + s * NT] = u0[s];
            lb[0][threadIdx.x + s * NT] = b0[s];
        }
    }
    __syncthreads();
    double acc = 0.0, mx = 0.0;
    for (int p = i0; p < i0 + a.ti; ++p) {
        const bool more3 = p + 3 <= last, moref = p + 1 < last;
        double un3[NS], f1[NS];
        float en3[NS];
#pragma unroll
        for (int s = 0; s < NS; ++s) {
            un3[s] = 0.0;
            en3[s] = 0.0f;
            f1[s] = 0.0;
            if (fl[s] && more3) {
                un3[s] = uin[offset(p + 3, s)];
                en3[s] = load_e(p + 3, s);
            }
            if ((fl[s] & 2) && moref) f1[s] = src[offset(p + 1, s)];
        }
        const double* LU = lu[(p - i0) & 1];
        const double* LB = lb[(p - i0) & 1];
        const bool second = RESTRICT && ((p - i0) & 1);
#pragma unroll
        for (int s = 0; s < NS; ++s) {
            const int c = threadIdx.x + s * NT;
            if (fl[s] & 2) {
                const double un[6] = {um1[s], up1[s], LU[c - LK], LU[c + LK], LU[c - 1], LU[c + 1]};
                const double bn[6] = {bm1[s], bp1[s], LB[c - LK], LB[c + LK], LB[c - 1], LB[c + 1]};
                const double d = dev::cell_op_b(g, u0[s], b0[s], un, bn, dev::rhs_value(g, f0[s])).L;
                const unsigned q = offset(p, s);
                if (NORM) {
                    acc += d * d;
                    const double ad = fabs(d);
                    if (!(mx >= ad)) mx = ad;
                }
                if (UPDATE) a.uout[q] = u0[s];
                if (CAST) {
                    a.r32[q] = (float)(-d);
                    a.ub32[q] = (float)u0[s];
                }
                if (RESTRICT) {
                    if (second) {
                        ru[li[s]] = uprev[s] + u0[s];
                        rd[li[s]] = dprev[s] + d;
                    } else {
                        uprev[s] = u0[s];
                        dprev[s] = d;
                    }
                }
            }
        }
        if (second) {
            __syncthreads();
            const int lgc = lg - 1;
            for (int t = threadIdx.x; t < (TJ / 2) * (kTK / 2); t += NT) {
                const int cj = t / (kTK / 2), ck = t - cj * (kTK / 2);
                const int b0i = (2 * cj) * kTK + 2 * ck;
                const double su = ru[b0i] + ru[b0i + 1] + ru[b0i + kTK] + ru[b0i + kTK + 1];
                const double sd = rd[b0i] + rd[b0i + 1] + rd[b0i + kTK] + rd[b0i + kTK + 1];
                const long long qc = ((((long long)((p & m) >> 1) << lgc) + ((j0 >> 1) + cj)) << lgc) + (k0 >> 1) + ck;
                a.uc[qc] = 0.125 * su;
                a.uhat[qc] = 0.125 * su;
                a.fc[qc] = 0.125 * sd;
            }
        }
        // stage plane p+1 into the other buffer and shift the registers
        double* NU = lu[(p + 1 - i0) & 1];
        double* NB = lb[(p + 1 - i0) & 1];
        const bool more2 = p + 2 <= last;
#pragma unroll
        for (int s = 0; s < NS; ++s) {
            if (fl[s]) {
                NU[threadIdx.x + s * NT] = up1[s];
                NB[threadIdx.x + s * NT] = bp1[s];
            }
            um1[s] = u0[s];
            bm1[s] = b0[s];
            u0[s] = up1[s];
            b0[s] = bp1[s];
            if (more2 && fl[s]) {
                up1[s] = UPDATE ? un2[s] + (double)en2[s] : un2[s];
                bp1[s] = exp(up1[s]);
            }
            un2[s] = un3[s];
            en2[s] = en3[s];
            f0[s] = f1[s];
        }
        __syncthreads();
    }
    if (NORM) {
        const int t = threadIdx.x;
        red_s[t] = acc;
        red_m[t] = mx;
        __syncthreads();
        for (int w = NT / 2; w > 0; w >>= 1) {
            if (t < w) {
                red_s[t] += red_s[t + w];
                const double o = red_m[t + w];
                if (!(red_m[t] >= o)) red_m[t] = o;
            }
            __syncthreads();
        }
        if (t == 0) {
            a.partial[2 * blockIdx.x] = red_s[0];
            a.partial[2 * blockIdx.x + 1] = red_m[0];
        }
    }
}

constexpr int kTJ = 8, kNT = 256;

template <bool NORM, bool RESTRICT, bool UPDATE, bool CAST>
hipError_t launch(const Grid& g, const double* uin, const double* src, ResidStream a, hipStream_t s)
{
    a.ntj = g.n / kTJ;
    a.ntk = g.n / kTK;
    const unsigned nb = (unsigned)((g.n / a.ti) * a.ntj * a.ntk);
    hipLaunchKernelGGL((k_resid_stream<kTJ, kNT, NORM, RESTRICT, UPDATE, CAST>), dim3(nb), dim3(kNT), 0, s, g,
                       uin, src, a);
    return hipGetLastError();
}

}  // namespace

int resid_stream_planes(int n)
{
    // even, dividing n, and few enough workgroups for the partial-sum scratch
    const long long tiles = (long long)(n / kTJ) * (n / kTK);
    int ti = 8;
    while (ti < n && tiles * (n / ti) > 8192) ti *= 2;
    return ti;
}

long long resid_stream_blocks(int n) { return (long long)(n / resid_stream_planes(n)) * (n / kTJ) * (n / kTK); }

hipError_t resid_stream(const Grid& g, const double* uin, const double* src, ResidStream a, hipStream_t s)
{
    if (g.n < kTK || g.n > 1024 || a.ti < 2 || (a.ti & 1) || g.n % a.ti) return hipErrorInvalidValue;
    const bool norm = a.partial != nullptr, restr = a.uc != nullptr, upd = a.e32 != nullptr,
               cast = a.r32 != nullptr;
    if (upd && (a.uout == nullptr || a.uout == uin)) return hipErrorInvalidValue;
    if (norm && !restr && !upd && !cast) return launch<true, false, false, false>(g, uin, src, a, s);
    if (!norm && restr && !upd && !cast) return launch<false, true, false, false>(g, uin, src, a, s);
    if (norm && !restr && upd && cast) return launch<true, false, true, true>(g, uin, src, a, s);
    if (norm && !restr && !upd && cast) return launch<true, false, false, true>(g, uin, src, a, s);
    return hipErrorInvalidValue;
}

}  // namespace mgfr
