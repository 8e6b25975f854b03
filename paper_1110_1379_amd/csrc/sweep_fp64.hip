// Fused red-black Newton-Gauss-Seidel sweep, double precision, for levels with n >= 64.
//
// One sweep (red cells, then black cells, Sec. V.B.1) in one pass over HBM: each workgroup
// owns a TJ x 64 tile of (j,k) columns and a chunk of planes i, and streams the planes in
// order.  Per plane it stages u and b = exp(u) of the tile plus an in-plane halo of two
// cells in LDS (three plane buffers, so one barrier per plane suffices); the i-neighbours of
// a column stay in the registers of the thread that owns the column.  At step p it updates
// the red cells of plane p (tile + 1-cell ring), then the black cells of plane p-1 (tile
// only), whose red neighbours are all final by then, and stages plane p+1:
//   red(p)   needs black(p-1), black(p+1), black in-plane            (all old)
//   black(p-1) needs red(p-2), red(p), red in-plane incl. the ring  (all new)
// The ring's red values are recomputed from the same old values by both tiles that see
// them, so they are bit-identical to the owner's, and the sweep equals the two-pass
// red-then-black sweep cell for cell.  The sweep reads `uin` and writes `uout` (never the
// same array) so that halo reads always see the values from before the sweep.
#include "device_fp64.h"

namespace mgfr {
namespace {

using dev::OpVal;

constexpr int kTK = 64;  // tile width along k (contiguous)

template <int TJ, int NT>
__global__ void __launch_bounds__(NT) k_ngs_fused(Grid g, const double* __restrict__ uin,
                                                  double* __restrict__ uout,
                                                  const double* __restrict__ src, FusedSweep a)
{
    constexpr int LJ = TJ + 4, LK = kTK + 4, NL = LJ * LK;
    constexpr int NS = (NL + NT - 1) / NT;
    // three plane buffers: plane p (red update), plane p-1 (black update), plane p+1 (staged)
    __shared__ double lu[3][NL];
    __shared__ double lb[3][NL];

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
    const int last = i0 + a.ti + 1;  // last plane read

    unsigned col[NS];
    int par[NS], fl[NS];
#pragma unroll
    for (int s = 0; s < NS; ++s) {
        const int c = threadIdx.x + s * NT;
        col[s] = 0;
        par[s] = 0;
        fl[s] = 0;
        if (c < NL) {
            const int jj = c / LK, kk = c - jj * LK;
            const int gj = (j0 - 2 + jj) & m, gk = (k0 - 2 + kk) & m;
            col[s] = (unsigned)((gj << lg) | gk);
            par[s] = (gj + gk) & 1;
            fl[s] = 1;
            if (jj >= 1 && jj <= LJ - 2 && kk >= 1 && kk <= LK - 2) fl[s] |= 2;  // red ring + tile
            if (jj >= 2 && jj <= LJ - 3 && kk >= 2 && kk <= LK - 3) fl[s] |= 4;  // tile
        }
    }

    // element offsets fit in 32 bits (n <= 1024)
    auto offset = [&](int p, int s) -> unsigned { return ((unsigned)(p & m) << (2 * lg)) + col[s]; };
    auto load_u = [&](int p, int s) -> double { return uin[offset(p, s)]; };
    auto buf = [&](int p) { return (p - i0 + 3) % 3; };

    // registers of plane p-2, p-1, p, p+1 for each column slot, and the raw loads of planes
    // p+2 and p+3 in flight
    double um2[NS], um1[NS], u0[NS], up1[NS];
    double bm2[NS], bm1[NS], b0[NS], bp1[NS];
    double fm1[NS], f0[NS], fp1[NS];
    double un2[NS], fn2[NS];
#pragma unroll
    for (int s = 0; s < NS; ++s) {
        um2[s] = bm2[s] = 0.0;
        um1[s] = bm1[s] = u0[s] = b0[s] = up1[s] = bp1[s] = 0.0;
        fm1[s] = f0[s] = fp1[s] = 0.0;
        un2[s] = fn2[s] = 0.0;
        if (fl[s]) {
            um1[s] = load_u(i0 - 2, s);
            u0[s] = load_u(i0 - 1, s);
            up1[s] = load_u(i0, s);
            un2[s] = load_u(i0 + 1, s);
            fm1[s] = dev::rhs_value(g, src[offset(i0 - 2, s)]);
            f0[s] = dev::rhs_value(g, src[offset(i0 - 1, s)]);
            fp1[s] = dev::rhs_value(g, src[offset(i0, s)]);
            fn2[s] = src[offset(i0 + 1, s)];  // raw: transformed when it becomes plane p+1
            bm1[s] = exp(um1[s]);
            b0[s] = exp(u0[s]);
            bp1[s] = exp(up1[s]);
            const int c = threadIdx.x + s * NT;
            lu[buf(i0 - 1)][c] = u0[s];
            lb[buf(i0 - 1)][c] = b0[s];
        }
    }
    __syncthreads();

    const double ms = g.max_step;
    for (int p = i0 - 1; p <= i0 + a.ti; ++p) {
        // issue the loads of plane p+3 two steps ahead of their use
        const bool more3 = p + 3 <= last;
        double un3[NS], fn3[NS];
#pragma unroll
        for (int s = 0; s < NS; ++s) {
            un3[s] = 0.0;
            fn3[s] = 0.0;
            if (more3 && fl[s]) {
                un3[s] = load_u(p + 3, s);
                fn3[s] = src[offset(p + 3, s)];
            }
        }
        double* LA = lu[buf(p)];
        double* BA = lb[buf(p)];
        // red cells of plane p (tile + ring); their black neighbours are all old
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
        // black cells of plane p-1 (tile); their red neighbours are all new, then plane p-1
        // is final
        if (p - 1 >= i0) {
            const double* LB = lu[buf(p - 1)];
            const double* BB = lb[buf(p - 1)];
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
        // stage plane p+1 for the next step, then shift the register planes
        double* LC = lu[buf(p + 1)];
        double* BC = lb[buf(p + 1)];
        const bool more2 = p + 2 <= last;
#pragma unroll
        for (int s = 0; s < NS; ++s) {
            const int c = threadIdx.x + s * NT;
            if (fl[s]) {
                LC[c] = up1[s];
                BC[c] = bp1[s];
            }
            um2[s] = um1[s];
            bm2[s] = bm1[s];
            um1[s] = u0[s];
            bm1[s] = b0[s];
            fm1[s] = f0[s];
            u0[s] = up1[s];
            b0[s] = bp1[s];
            f0[s] = fp1[s];
            if (more2 && fl[s]) {
                up1[s] = un2[s];
                bp1[s] = exp(un2[s]);
                fp1[s] = dev::rhs_value(g, fn2[s]);
            }
            un2[s] = un3[s];
            fn2[s] = fn3[s];
        }
        __syncthreads();
    }
}

template <int TJ, int NT>
hipError_t launch(const Grid& g, const double* uin, double* uout, const double* src, FusedSweep a,
                  hipStream_t s)
{
    a.ntj = g.n / TJ;
    a.ntk = g.n / kTK;
    const int nti = g.n / a.ti;
    const unsigned nb = (unsigned)(nti * a.ntj * a.ntk);
    hipLaunchKernelGGL((k_ngs_fused<TJ, NT>), dim3(nb), dim3(NT), 0, s, g, uin, uout, src, a);
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

hipError_t ngs_sweep_fused(const Grid& g, const double* uin, double* uout, const double* src, int ti,
                           hipStream_t s)
{
    if (g.n < kTK || g.n > 1024 || uin == uout || ti < 1 || ti > g.n || (g.n % ti) != 0) return hipErrorInvalidValue;
    FusedSweep a{};
    a.ti = ti;
    return launch<16, 1024>(g, uin, uout, src, a, s);
}

}  // namespace mgfr
