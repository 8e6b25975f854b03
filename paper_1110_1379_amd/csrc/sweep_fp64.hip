// Fused red-black Newton-Gauss-Seidel sweep, double precision, for levels with n >= 64.
//
// One sweep (red cells, then black cells, Sec. V.B.1) in one pass over HBM: each workgroup
// owns a TJ x 64 tile of (j,k) columns and a chunk of planes i, and streams the planes in
// order.  Per plane it stages u and b = exp(u) of the tile plus an in-plane halo of two
// cells in LDS; the i-neighbours of a column stay in the registers of the thread that owns
// the column.  At step p it updates the red cells of plane p (tile + 1-cell ring) and then
// the black cells of plane p-1 (tile only), whose red neighbours are all final by then:
//   red(p)   needs black(p-1), black(p+1), black in-plane            (all old)
//   black(p-1) needs red(p-2), red(p), red in-plane incl. the ring  (all new)
// The ring's red values are recomputed from the same old values by both tiles that see
// them, so they are bit-identical to the owner's, and the sweep equals the two-pass
// red-then-black sweep cell for cell.  The sweep reads `uin` and writes `uout` (never the
// same array) so that halo reads always see the values from before the sweep.
//
// With a coarse correction e (CORR), every loaded u is first increased by the trilinear
// prolongation of e (27/9/3/1 over 64, Sec. V.A.3), which fuses the coarse-grid
// correction u <- u + P(u^H - R u^h) (Sec. V.B.3) into the first post-smoothing sweep.
#include "device_fp64.h"

namespace mgfr {
namespace {

using dev::OpVal;

constexpr int kTK = 64;  // tile width along k (contiguous)

__device__ __forceinline__ double prolong_e(const double* __restrict__ e, int lgc, int i, int j, int k)
{
    const int mc = (1 << lgc) - 1;
    const int I = i >> 1, J = j >> 1, K = k >> 1;
    const int Ip = (I + ((i & 1) ? 1 : -1)) & mc;
    const int Jp = (J + ((j & 1) ? 1 : -1)) & mc;
    const int Kp = (K + ((k & 1) ? 1 : -1)) & mc;
    auto E = [&](int a, int b, int c) { return e[((((long long)a << lgc) + b) << lgc) + c]; };
    return (27.0 / 64.0) * E(I, J, K) + (9.0 / 64.0) * (E(Ip, J, K) + E(I, Jp, K) + E(I, J, Kp)) +
           (3.0 / 64.0) * (E(Ip, Jp, K) + E(Ip, J, Kp) + E(I, Jp, Kp)) + (1.0 / 64.0) * E(Ip, Jp, Kp);
}

template <int TJ, int NT, bool CORR>
__global__ void __launch_bounds__(NT) k_ngs_fused(Grid g, const double* __restrict__ uin,
                                                  double* __restrict__ uout,
                                                  const double* __restrict__ src, FusedSweep a)
{
    constexpr int LJ = TJ + 4, LK = kTK + 4, NL = LJ * LK;
    constexpr int NS = (NL + NT - 1) / NT;
    __shared__ double lu[2][NL];
    __shared__ double lb[2][NL];

    // workgroup -> (plane chunk, j tile, k tile); consecutive workgroups go to different
    // XCDs, so hand each XCD a contiguous range of tiles (their halos share its L2)
    const int nb = gridDim.x;
    int lid = blockIdx.x;
    if ((nb & 7) == 0) lid = (lid & 7) * (nb >> 3) + (lid >> 3);
    const int tk = lid % a.ntk;
    lid /= a.ntk;
    const int tj = lid % a.ntj;
    const int ci = lid / a.ntj;
    const int i0 = ci * a.ti, j0 = tj * TJ, k0 = tk * kTK;
    const int lg = g.lg, m = g.n - 1;

    int col[NS], par[NS], fl[NS];
#pragma unroll
    for (int s = 0; s < NS; ++s) {
        const int c = threadIdx.x + s * NT;
        col[s] = 0;
        par[s] = 0;
        fl[s] = 0;
        if (c < NL) {
            const int jj = c / LK, kk = c - jj * LK;
            const int gj = (j0 - 2 + jj) & m, gk = (k0 - 2 + kk) & m;
            col[s] = (gj << lg) | gk;
            par[s] = (gj + gk) & 1;
            fl[s] = 1;
            if (jj >= 1 && jj <= LJ - 2 && kk >= 1 && kk <= LK - 2) fl[s] |= 2;  // red ring + tile
            if (jj >= 2 && jj <= LJ - 3 && kk >= 2 && kk <= LK - 3) fl[s] |= 4;  // tile
        }
    }

    auto offset = [&](int p, int s) -> long long { return ((long long)(p & m) << (2 * lg)) + col[s]; };
    auto load_u = [&](int p, int s) -> double {
        double v = uin[offset(p, s)];
        if (CORR) v += prolong_e(a.e, lg - 1, p & m, col[s] >> lg, col[s] & m);
        return v;
    };

    // registers of plane p-2, p-1, p, p+1 for each column slot
    double um2[NS], um1[NS], u0[NS], up1[NS];
    double bm2[NS], bm1[NS], b0[NS], bp1[NS];
    double fm1[NS], f0[NS], fp1[NS];
#pragma unroll
    for (int s = 0; s < NS; ++s) {
        um2[s] = bm2[s] = 0.0;
        um1[s] = bm1[s] = u0[s] = b0[s] = up1[s] = bp1[s] = 0.0;
        fm1[s] = f0[s] = fp1[s] = 0.0;
        if (fl[s]) {
            um1[s] = load_u(i0 - 2, s);
            u0[s] = load_u(i0 - 1, s);
            up1[s] = load_u(i0, s);
            fm1[s] = dev::rhs_value(g, src[offset(i0 - 2, s)]);
            f0[s] = dev::rhs_value(g, src[offset(i0 - 1, s)]);
            fp1[s] = dev::rhs_value(g, src[offset(i0, s)]);
            bm1[s] = exp(um1[s]);
            b0[s] = exp(u0[s]);
            bp1[s] = exp(up1[s]);
        }
    }

    const double ms = g.max_step;
    for (int p = i0 - 1; p <= i0 + a.ti; ++p) {
        // issue the loads of plane p+2 early
        const bool more = p + 2 <= i0 + a.ti + 1;
        double un2[NS], fn2[NS];
#pragma unroll
        for (int s = 0; s < NS; ++s) {
            un2[s] = 0.0;
            fn2[s] = 0.0;
            if (more && fl[s]) {
                un2[s] = load_u(p + 2, s);
                fn2[s] = dev::rhs_value(g, src[offset(p + 2, s)]);
            }
        }
        double* LA = lu[p & 1];
        double* BA = lb[p & 1];
        __syncthreads();  // the previous step is done reading this buffer
#pragma unroll
        for (int s = 0; s < NS; ++s) {
            const int c = threadIdx.x + s * NT;
            if (fl[s]) {
                LA[c] = u0[s];
                BA[c] = b0[s];
            }
        }
        __syncthreads();
        // red cells of plane p (tile + ring)
#pragma unroll
        for (int s = 0; s < NS; ++s) {
            const int c = threadIdx.x + s * NT;
            if ((fl[s] & 2) && ((p + par[s]) & 1) == 0) {
                const double un[6] = {um1[s], up1[s], LA[c - LK], LA[c + LK], LA[c - 1], LA[c + 1]};
                const double bn[6] = {bm1[s], bp1[s], BA[c - LK], BA[c + LK], BA[c - 1], BA[c + 1]};
                const OpVal r = dev::cell_op_b(g, u0[s], b0[s], un, bn, f0[s]);
                const double v = u0[s] + dev::bounded(-r.L / r.dL, ms);
                const double bv = exp(v);
                u0[s] = v;
                b0[s] = bv;
                LA[c] = v;
                BA[c] = bv;
            }
        }
        // black cells of plane p-1 (tile), then plane p-1 is final
        if (p - 1 >= i0) {
            const double* LB = lu[(p - 1) & 1];
            const double* BB = lb[(p - 1) & 1];
#pragma unroll
            for (int s = 0; s < NS; ++s) {
                const int c = threadIdx.x + s * NT;
                if (fl[s] & 4) {
                    if (((p - 1 + par[s]) & 1) == 1) {
                        const double un[6] = {um2[s], u0[s], LB[c - LK], LB[c + LK], LB[c - 1], LB[c + 1]};
                        const double bn[6] = {bm2[s], b0[s], BB[c - LK], BB[c + LK], BB[c - 1], BB[c + 1]};
                        const OpVal r = dev::cell_op_b(g, um1[s], bm1[s], un, bn, fm1[s]);
                        um1[s] = um1[s] + dev::bounded(-r.L / r.dL, ms);
                    }
                    uout[offset(p - 1, s)] = um1[s];
                }
            }
        }
#pragma unroll
        for (int s = 0; s < NS; ++s) {
            um2[s] = um1[s];
            bm2[s] = bm1[s];
            um1[s] = u0[s];
            bm1[s] = b0[s];
            fm1[s] = f0[s];
            u0[s] = up1[s];
            b0[s] = bp1[s];
            f0[s] = fp1[s];
            if (more && fl[s]) {
                up1[s] = un2[s];
                bp1[s] = exp(un2[s]);
                fp1[s] = fn2[s];
            }
        }
    }
}

// e = uc - uhat on the coarse level (in place in uhat).
__global__ void __launch_bounds__(256) k_coarse_diff(const double* __restrict__ uc, double* __restrict__ e,
                                                     long long n)
{
    const long long q = (long long)blockIdx.x * 256 + threadIdx.x;
    if (q < n) e[q] = uc[q] - e[q];
}

template <int TJ, int NT>
hipError_t launch(const Grid& g, const double* uin, double* uout, const double* src, FusedSweep a,
                  hipStream_t s)
{
    a.ntj = g.n / TJ;
    a.ntk = g.n / kTK;
    const int nti = g.n / a.ti;
    const unsigned nb = (unsigned)(nti * a.ntj * a.ntk);
    if (a.e)
        hipLaunchKernelGGL((k_ngs_fused<TJ, NT, true>), dim3(nb), dim3(NT), 0, s, g, uin, uout, src, a);
    else
        hipLaunchKernelGGL((k_ngs_fused<TJ, NT, false>), dim3(nb), dim3(NT), 0, s, g, uin, uout, src, a);
    return hipGetLastError();
}

}  // namespace

int fused_sweep_min_n() { return kTK; }

int fused_sweep_planes(int n)
{
    // planes per workgroup: long enough to amortise the 4 halo planes, short enough to
    // give >= 1024 workgroups
    const int tiles = (n / 16) * (n / kTK);
    int ti = 64;
    while (ti > 8 && (long long)tiles * (n / ti) < 1024) ti /= 2;
    return ti > n ? n : ti;
}

hipError_t ngs_sweep_fused(const Grid& g, const double* uin, double* uout, const double* src,
                           const double* e, int ti, hipStream_t s)
{
    if (g.n < kTK || uin == uout || ti < 1 || ti > g.n || (g.n % ti) != 0) return hipErrorInvalidValue;
    FusedSweep a{};
    a.ti = ti;
    a.e = e;
    return launch<16, 512>(g, uin, uout, src, a, s);
}

hipError_t coarse_difference(const Grid& gc, const double* uc, double* uhat_to_e, hipStream_t s)
{
    const long long n = cells(gc);
    hipLaunchKernelGGL(k_coarse_diff, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, uc, uhat_to_e, n);
    return hipGetLastError();
}

}  // namespace mgfr
