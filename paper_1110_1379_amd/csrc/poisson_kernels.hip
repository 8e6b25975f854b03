// Kernels of the modified Poisson solve (eq. discrete_poisson): the potential phi of the
// density and of delta R of the scalaron,
//   (1/h^2) [sum of the 6 neighbours of phi - 6 phi] = S - mean(S),
//   S = 2 Om a (rho~ - 1) - (1/2) (A exp(-u/(n+1)) - Sbar)
// with A = (1/3) Om a^4 (n a^2 xi)^(1/(n+1)) and Sbar = Om a^4 (a^-3 + 4 OL/Om), so that the
// bracket of the paper's delta R term, times Om a^4 / 6, is (A exp(-u/(n+1)) - Sbar) / 2.
// Linear multigrid (Sec. V.A.3, correction scheme): red-black Gauss-Seidel, x_i =
// (sum_nb x_nb - h^2 b_i) / 6, the residual restricted by 8-child means, the coarse
// correction prolongated 27/9/3/1 (prolong.hip).  Every level is periodic.
#include "mgfr_impl.h"

namespace mgfr {
namespace {

constexpr int kB = 256;
constexpr int kTK = 64;

__device__ __forceinline__ unsigned at3(int lg, int i, int j, int k)
{
    return ((((unsigned)i << lg) + (unsigned)j) << lg) + (unsigned)k;
}

// ---- source and its mean -----------------------------------------------------------------
__global__ void __launch_bounds__(kB) kp_source(PoissonSource c, long long n3, const double* __restrict__ rho,
                                                const double* __restrict__ u, double* __restrict__ S,
                                                double* __restrict__ partial)
{
    __shared__ double rs[kB], rm[kB];
    double s = 0.0, mx = 0.0;
    for (long long q = (long long)blockIdx.x * kB + threadIdx.x; q < n3; q += (long long)gridDim.x * kB) {
        const double v = 2.0 * c.D * (rho[q] - 1.0) - 0.5 * (c.A * exp(-u[q] * c.inv_np1) - c.Sbar);
        S[q] = v;
        s += v;
        const double av = fabs(v);
        if (!(mx >= av)) mx = av;  // NaN propagates
    }
    rs[threadIdx.x] = s;
    rm[threadIdx.x] = mx;
    __syncthreads();
    for (int w = kB / 2; w > 0; w >>= 1) {
        if (threadIdx.x < w) {
            rs[threadIdx.x] += rs[threadIdx.x + w];
            const double o = rm[threadIdx.x + w];
            if (!(rm[threadIdx.x] >= o)) rm[threadIdx.x] = o;
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        partial[2 * blockIdx.x] = rs[0];
        partial[2 * blockIdx.x + 1] = rm[0];
    }
}

// ---- residual norm: r = b - bmean - lap x (x null: r = b - bmean) --------------------------
__global__ void __launch_bounds__(kB) kp_resid_norm(PGrid g, const double* __restrict__ x, const double* __restrict__ b,
                                                    double bmean, double* __restrict__ partial)
{
    __shared__ double rs[kB], rm[kB];
    const int m = g.n - 1;
    const long long n3 = 1LL << (3 * g.lg);
    double s = 0.0, mx = 0.0;
    for (long long q = (long long)blockIdx.x * kB + threadIdx.x; q < n3; q += (long long)gridDim.x * kB) {
        double r = b[q] - bmean;
        if (x) {
            const int i = (int)(q >> (2 * g.lg)), j = (int)((q >> g.lg) & m), k = (int)(q & m);
            const double lap = (x[at3(g.lg, (i + 1) & m, j, k)] + x[at3(g.lg, (i - 1) & m, j, k)] +
                                x[at3(g.lg, i, (j + 1) & m, k)] + x[at3(g.lg, i, (j - 1) & m, k)] +
                                x[at3(g.lg, i, j, (k + 1) & m)] + x[at3(g.lg, i, j, (k - 1) & m)] - 6.0 * x[q]) *
                               g.inv_hh;
            r -= lap;
        }
        s += r * r;
        const double ar = fabs(r);
        if (!(mx >= ar)) mx = ar;
    }
    rs[threadIdx.x] = s;
    rm[threadIdx.x] = mx;
    __syncthreads();
    for (int w = kB / 2; w > 0; w >>= 1) {
        if (threadIdx.x < w) {
            rs[threadIdx.x] += rs[threadIdx.x + w];
            const double o = rm[threadIdx.x + w];
            if (!(rm[threadIdx.x] >= o)) rm[threadIdx.x] = o;
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        partial[2 * blockIdx.x] = rs[0];
        partial[2 * blockIdx.x + 1] = rm[0];
    }
}

// ---- one colour of a Gauss-Seidel sweep, in place (levels below 64) ----------------------
__global__ void __launch_bounds__(kB) kp_ngs_colour(PGrid g, double* __restrict__ x, const double* __restrict__ b,
                                                    double bmean, int colour)
{
    const long long half = 1LL << (3 * g.lg - 1);
    const long long t = (long long)blockIdx.x * kB + threadIdx.x;
    if (t >= half) return;
    const int m = g.n - 1, hk = g.n >> 1;
    const int s = (int)(t & (hk - 1));
    const long long row = t >> (g.lg - 1);
    const int i = (int)(row >> g.lg), j = (int)(row & m);
    const int k = 2 * s + ((i + j + colour) & 1);
    const double sum = x[at3(g.lg, (i + 1) & m, j, k)] + x[at3(g.lg, (i - 1) & m, j, k)] + x[at3(g.lg, i, (j + 1) & m, k)] +
                       x[at3(g.lg, i, (j - 1) & m, k)] + x[at3(g.lg, i, j, (k + 1) & m)] + x[at3(g.lg, i, j, (k - 1) & m)];
    const unsigned q = at3(g.lg, i, j, k);
    x[q] = (sum - g.hh * (b[q] - bmean)) * (1.0 / 6.0);
}

// ---- fused red-black sweep (n >= 64), out of place ----------------------------------------
// Same scheme as the nonlinear fused sweep: a workgroup streams the planes of a TJ x 64
// tile; per plane the tile plus a 2-cell in-plane halo is staged in LDS (three buffers, one
// barrier per plane), the i-neighbours stay in registers; at step p the red cells of plane
// p (tile + ring) and then the black cells of plane p-1 (tile) are updated; the ring is
// recomputed from the same old values by every tile that sees it, so the sweep equals the
// two-pass red-then-black sweep.
template <int TJ, int NT>
__global__ void __launch_bounds__(NT) kp_fused(PGrid g, const double* __restrict__ xin, double* __restrict__ xout,
                                               const double* __restrict__ b, double bmean, int ti, int ntj, int ntk)
{
    constexpr int LJ = TJ + 4, LK = kTK + 4, NL = LJ * LK;
    constexpr int NS = (NL + NT - 1) / NT;
    __shared__ double lx[3][NL];
    const int nb = gridDim.x;
    int lid = blockIdx.x;
    if ((nb & 7) == 0) lid = (lid & 7) * (nb >> 3) + (lid >> 3);
    const int tk = lid % ntk;
    lid /= ntk;
    const int tj = lid % ntj;
    const int ci = lid / ntj;
    const int i0 = ci * ti, j0 = tj * TJ, k0 = tk * kTK;
    const int lg = g.lg, m = g.n - 1;
    const int last = i0 + ti + 1;  // last plane read
    const double hh = g.hh;

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
            if (jj >= 1 && jj <= LJ - 2 && kk >= 1 && kk <= LK - 2) fl[s] |= 2;
            if (jj >= 2 && jj <= LJ - 3 && kk >= 2 && kk <= LK - 3) fl[s] |= 4;
        }
    }
    // element offsets fit in 32 bits (n <= 1024)
    auto offset = [&](int p, int s) -> unsigned { return ((unsigned)(p & m) << (2 * lg)) + col[s]; };
    auto buf = [&](int p) { return (p - i0 + 3) % 3; };

    // x of planes p-2 .. p+1, the right-hand side (minus its mean, times h^2) of planes
    // p-1 .. p+1, and the raw loads of plane p+2
    double xm2[NS], xm1[NS], x0[NS], xp1[NS], bm1[NS], b0[NS], bp1[NS], xn2[NS], bn2[NS];
#pragma unroll
    for (int s = 0; s < NS; ++s) {
        xm2[s] = xm1[s] = x0[s] = xp1[s] = bm1[s] = b0[s] = bp1[s] = xn2[s] = bn2[s] = 0.0;
        if (fl[s]) {
            xm1[s] = xin[offset(i0 - 2, s)];
            x0[s] = xin[offset(i0 - 1, s)];
            xp1[s] = xin[offset(i0, s)];
            xn2[s] = xin[offset(i0 + 1, s)];
            bm1[s] = hh * (b[offset(i0 - 2, s)] - bmean);
            b0[s] = hh * (b[offset(i0 - 1, s)] - bmean);
            bp1[s] = hh * (b[offset(i0, s)] - bmean);
            bn2[s] = b[offset(i0 + 1, s)];
            lx[buf(i0 - 1)][threadIdx.x + s * NT] = x0[s];
        }
    }
    __syncthreads();
    for (int p = i0 - 1; p <= i0 + ti; ++p) {
        const bool more3 = p + 3 <= last;
        double xn3[NS], bn3[NS];
#pragma unroll
        for (int s = 0; s < NS; ++s) {
            xn3[s] = bn3[s] = 0.0;
            if (more3 && fl[s]) {
                xn3[s] = xin[offset(p + 3, s)];
                bn3[s] = b[offset(p + 3, s)];
            }
        }
        double* LA = lx[buf(p)];
#pragma unroll
        for (int s = 0; s < NS; ++s) {
            const int c = threadIdx.x + s * NT;
            if ((fl[s] & 2) && ((p + par[s]) & 1) == 0) {
                const double v = (xm1[s] + xp1[s] + LA[c - LK] + LA[c + LK] + LA[c - 1] + LA[c + 1] - b0[s]) * (1.0 / 6.0);
                x0[s] = v;
                LA[c] = v;
            }
        }
        if (p - 1 >= i0) {
            const double* LB = lx[buf(p - 1)];
#pragma unroll
            for (int s = 0; s < NS; ++s) {
                const int c = threadIdx.x + s * NT;
                if (fl[s] & 4) {
                    if (((p - 1 + par[s]) & 1) == 1)
                        xm1[s] = (xm2[s] + x0[s] + LB[c - LK] + LB[c + LK] + LB[c - 1] + LB[c + 1] - bm1[s]) * (1.0 / 6.0);
                    xout[offset(p - 1, s)] = xm1[s];
                }
            }
        }
        double* LC = lx[buf(p + 1)];
        const bool more2 = p + 2 <= last;
#pragma unroll
        for (int s = 0; s < NS; ++s) {
            if (fl[s]) LC[threadIdx.x + s * NT] = xp1[s];
            xm2[s] = xm1[s];
            xm1[s] = x0[s];
            bm1[s] = b0[s];
            x0[s] = xp1[s];
            b0[s] = bp1[s];
            if (more2 && fl[s]) {
                xp1[s] = xn2[s];
                bp1[s] = hh * (bn2[s] - bmean);
            }
            xn2[s] = xn3[s];
            bn2[s] = bn3[s];
        }
        __syncthreads();
    }
}

// ---- two fused red-black sweeps per pass (n >= 256), out of place --------------------------
// Temporal blocking of the sweep above: one pass over the planes applies two complete
// red-black sweeps, A then B, so x and b come from HBM once for both.  At plane step p:
//   A red on plane p (tile + 3-cell ring), A black on plane p-1 (tile + 2-cell ring),
//   B red on plane p-2 (tile + 1-cell ring), B black on plane p-3 (tile),
// each reading exactly the values that the one-sweep kernel would have at that point (the
// rings are recomputed from identical values by every tile that sees them), with the same
// arithmetic, so the pass equals two one-sweep launches bit for bit.  The tile carries a
// 4-cell in-plane halo; a plane's LDS buffer serves, in turn, as the staged plane, A's red
// and black planes, then B's red and black planes (five buffers, one barrier per plane).
// The planes i0-4 .. i0+ti+3 are read and i0 .. i0+ti-1 written.
template <int TJ, int NT>
__global__ void __launch_bounds__(NT) kp_fused2(PGrid g, const double* __restrict__ xin, double* __restrict__ xout,
                                                const double* __restrict__ b, double bmean, int ti, int ntj, int ntk)
{
    constexpr int H = 4, LJ = TJ + 2 * H, LK = kTK + 2 * H, NL = LJ * LK;
    constexpr int NS = (NL + NT - 1) / NT;
    __shared__ double lx[5][NL];
    const int nb = gridDim.x;
    int lid = blockIdx.x;
    if ((nb & 7) == 0) lid = (lid & 7) * (nb >> 3) + (lid >> 3);
    const int tk = lid % ntk;
    lid /= ntk;
    const int tj = lid % ntj;
    const int ci = lid / ntj;
    const int i0 = ci * ti, j0 = tj * TJ, k0 = tk * kTK;
    const int lg = g.lg, m = g.n - 1;
    const int last = i0 + ti + H - 1;  // last plane read
    const double hh = g.hh;

    // per slot: column offset, parity of (j + k), and the rings it is updated on:
    // 1 loaded, 2 A red (ring <= 3), 4 A black (ring <= 2), 8 B red (ring <= 1), 16 tile
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
            const int gj = (j0 - H + jj) & m, gk = (k0 - H + kk) & m;
            col[s] = (unsigned)((gj << lg) | gk);
            par[s] = (gj + gk) & 1;
            fl[s] = 1;
#pragma unroll
            for (int r = 1; r <= 4; ++r)
                if (jj >= r && jj <= LJ - 1 - r && kk >= r && kk <= LK - 1 - r) fl[s] |= 1 << r;
        }
    }
    // element offsets fit in 32 bits (n <= 1024)
    auto offset = [&](int p, int s) -> unsigned { return ((unsigned)(p & m) << (2 * lg)) + col[s]; };
    auto buf = [&](int p) { return (p - i0 + 2 * H) % 5; };

    // x of planes p-4 .. p+1 in xr[0..5] (plane p+d in xr[d+4]) and the raw load of plane
    // p+2; the right-hand side (minus its mean, times h^2) of planes p-3 .. p+1 in br[0..4]
    // (plane p+d in br[d+3]) and the raw load of plane p+2
    double xr[NS][6], br[NS][5], xn2[NS], bn2[NS];
    const int p0 = i0 - H + 1;  // first step
#pragma unroll
    for (int s = 0; s < NS; ++s) {
#pragma unroll
        for (int d = 0; d < 6; ++d) xr[s][d] = 0.0;
#pragma unroll
        for (int d = 0; d < 5; ++d) br[s][d] = 0.0;
        xn2[s] = bn2[s] = 0.0;
        if (fl[s]) {
            // step p0 needs planes p0-1 (= i0-4) .. p0+1 and loads p0+2 raw
            xr[s][3] = xin[offset(p0 - 1, s)];
            xr[s][4] = xin[offset(p0, s)];
            xr[s][5] = xin[offset(p0 + 1, s)];
            br[s][3] = hh * (b[offset(p0, s)] - bmean);
            br[s][4] = hh * (b[offset(p0 + 1, s)] - bmean);
            xn2[s] = xin[offset(p0 + 2, s)];
            bn2[s] = b[offset(p0 + 2, s)];
            lx[buf(p0)][threadIdx.x + s * NT] = xr[s][4];
        }
    }
    __syncthreads();
    for (int p = p0; p <= i0 + ti + H - 2; ++p) {
        const bool more3 = p + 3 <= last;
        double xn3[NS], bn3[NS];
#pragma unroll
        for (int s = 0; s < NS; ++s) {
            xn3[s] = bn3[s] = 0.0;
            if (more3 && fl[s]) {
                xn3[s] = xin[offset(p + 3, s)];
                bn3[s] = b[offset(p + 3, s)];
            }
        }
        // A red, plane p
        {
            double* L = lx[buf(p)];
#pragma unroll
            for (int s = 0; s < NS; ++s) {
                const int c = threadIdx.x + s * NT;
                if ((fl[s] & 2) && ((p + par[s]) & 1) == 0) {
                    const double v =
                        (xr[s][3] + xr[s][5] + L[c - LK] + L[c + LK] + L[c - 1] + L[c + 1] - br[s][3]) * (1.0 / 6.0);
                    xr[s][4] = v;
                    L[c] = v;
                }
            }
        }
        // A black, plane p-1
        if (p - 1 >= i0 - H + 2) {
            double* L = lx[buf(p - 1)];
#pragma unroll
            for (int s = 0; s < NS; ++s) {
                const int c = threadIdx.x + s * NT;
                if ((fl[s] & 4) && ((p - 1 + par[s]) & 1) == 1) {
                    const double v =
                        (xr[s][2] + xr[s][4] + L[c - LK] + L[c + LK] + L[c - 1] + L[c + 1] - br[s][2]) * (1.0 / 6.0);
                    xr[s][3] = v;
                    L[c] = v;
                }
            }
        }
        // B red, plane p-2
        if (p - 2 >= i0 - 1) {
            double* L = lx[buf(p - 2)];
#pragma unroll
            for (int s = 0; s < NS; ++s) {
                const int c = threadIdx.x + s * NT;
                if ((fl[s] & 8) && ((p - 2 + par[s]) & 1) == 0) {
                    const double v =
                        (xr[s][1] + xr[s][3] + L[c - LK] + L[c + LK] + L[c - 1] + L[c + 1] - br[s][1]) * (1.0 / 6.0);
                    xr[s][2] = v;
                    L[c] = v;
                }
            }
        }
        // B black, plane p-3, and the tile of that plane is final
        if (p - 3 >= i0) {
            const double* L = lx[buf(p - 3)];
#pragma unroll
            for (int s = 0; s < NS; ++s) {
                const int c = threadIdx.x + s * NT;
                if (fl[s] & 16) {
                    if (((p - 3 + par[s]) & 1) == 1)
                        xr[s][1] =
                            (xr[s][0] + xr[s][2] + L[c - LK] + L[c + LK] + L[c - 1] + L[c + 1] - br[s][0]) * (1.0 / 6.0);
                    xout[offset(p - 3, s)] = xr[s][1];
                }
            }
        }
        // stage plane p+1; shift the register planes
        double* LC = lx[buf(p + 1)];
        const bool more2 = p + 2 <= last;
#pragma unroll
        for (int s = 0; s < NS; ++s) {
            if (fl[s]) LC[threadIdx.x + s * NT] = xr[s][5];
#pragma unroll
            for (int d = 0; d < 5; ++d) xr[s][d] = xr[s][d + 1];
#pragma unroll
            for (int d = 0; d < 4; ++d) br[s][d] = br[s][d + 1];
            if (more2 && fl[s]) {
                xr[s][5] = xn2[s];
                br[s][4] = hh * (bn2[s] - bmean);
            }
            xn2[s] = xn3[s];
            bn2[s] = bn3[s];
        }
        __syncthreads();
    }
}

// ---- residual restricted to the coarse level: bc = R (b - bmean - lap x) ---------------------
__global__ void __launch_bounds__(kB) kp_resid_restrict(PGrid g, const double* __restrict__ x,
                                                        const double* __restrict__ b, double bmean,
                                                        double* __restrict__ bc)
{
    const int lgc = g.lg - 1, nc = g.n >> 1, m = g.n - 1;
    const long long tc = (long long)blockIdx.x * kB + threadIdx.x;
    if (tc >= (1LL << (3 * lgc))) return;
    const int I = (int)(tc >> (2 * lgc)), J = (int)((tc >> lgc) & (nc - 1)), K = (int)(tc & (nc - 1));
    double s = 0.0;
    for (int a = 0; a < 2; ++a)
        for (int bb = 0; bb < 2; ++bb)
            for (int z = 0; z < 2; ++z) {
                const int i = 2 * I + a, j = 2 * J + bb, k = 2 * K + z;
                const unsigned q = at3(g.lg, i, j, k);
                const double lap = (x[at3(g.lg, (i + 1) & m, j, k)] + x[at3(g.lg, (i - 1) & m, j, k)] +
                                    x[at3(g.lg, i, (j + 1) & m, k)] + x[at3(g.lg, i, (j - 1) & m, k)] +
                                    x[at3(g.lg, i, j, (k + 1) & m)] + x[at3(g.lg, i, j, (k - 1) & m)] - 6.0 * x[q]) *
                                   g.inv_hh;
                s += b[q] - bmean - lap;
            }
    bc[tc] = 0.125 * s;
}

// ---- streaming residual (n >= 64): norm partials or restriction ----------------------------
// r = b - bmean - lap x.  A workgroup owns a TJ x 64 tile of columns and a chunk of ti planes
// (ti even): x of the tile plus a one-cell in-plane halo is staged in LDS per plane (two
// buffers, one barrier per plane), the i-neighbours stay in registers, and the loads run two
// planes ahead.  NORM: per-workgroup (sum r^2, max |r|); RESTRICT: 8-child means into bc.
template <int TJ, int NT, bool RESTRICT>
__global__ void __launch_bounds__(NT) kp_resid_stream(PGrid g, const double* __restrict__ x,
                                                      const double* __restrict__ b, double bmean, int ti, int ntj,
                                                      int ntk, double* __restrict__ out)
{
    constexpr int LJ = TJ + 2, LK = kTK + 2, NL = LJ * LK;
    constexpr int NS = (NL + NT - 1) / NT;
    __shared__ double lx[2][NL];
    __shared__ double rr[RESTRICT ? TJ * kTK : 1];
    __shared__ double red_s[NT], red_m[NT];
    const int nb = gridDim.x;
    int lid = blockIdx.x;
    if ((nb & 7) == 0) lid = (lid & 7) * (nb >> 3) + (lid >> 3);
    const int tk = lid % ntk;
    lid /= ntk;
    const int tj = lid % ntj;
    const int ci = lid / ntj;
    const int i0 = ci * ti, j0 = tj * TJ, k0 = tk * kTK;
    const int lg = g.lg, m = g.n - 1;
    const int last = i0 + ti;  // last plane read
    unsigned col[NS];
    int fl[NS], li[NS];
#pragma unroll
    for (int s = 0; s < NS; ++s) {
        const int c = threadIdx.x + s * NT;
        col[s] = 0;
        fl[s] = li[s] = 0;
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
    auto offset = [&](int p, int s) -> unsigned { return ((unsigned)(p & m) << (2 * lg)) + col[s]; };
    // x of planes p-1, p, p+1 and b of plane p in registers; x of p+2 (and b of p+1) in flight
    double xm1[NS], x0[NS], xp1[NS], xn2[NS], b0[NS], prev[NS];
#pragma unroll
    for (int s = 0; s < NS; ++s) {
        xm1[s] = x0[s] = xp1[s] = xn2[s] = b0[s] = prev[s] = 0.0;
        if (fl[s] & 2) b0[s] = b[offset(i0, s)];
        if (fl[s]) {
            xm1[s] = x[offset(i0 - 1, s)];
            x0[s] = x[offset(i0, s)];
            xp1[s] = x[offset(i0 + 1, s)];
            xn2[s] = x[offset(i0 + 2, s)];
            lx[0][threadIdx.x + s * NT] = x0[s];
        }
    }
    __syncthreads();
    double acc = 0.0, mx = 0.0;
    for (int p = i0; p < i0 + ti; ++p) {
        const bool more3 = p + 3 <= last, moreb = p + 1 < last;
        double xn3[NS], b1[NS];
#pragma unroll
        for (int s = 0; s < NS; ++s) {
            xn3[s] = b1[s] = 0.0;
            if (fl[s] && more3) xn3[s] = x[offset(p + 3, s)];
            if ((fl[s] & 2) && moreb) b1[s] = b[offset(p + 1, s)];
        }
        const double* LX = lx[(p - i0) & 1];
        const bool second = RESTRICT && ((p - i0) & 1);
#pragma unroll
        for (int s = 0; s < NS; ++s) {
            const int c = threadIdx.x + s * NT;
            if (fl[s] & 2) {
                const double lap =
                    (xm1[s] + xp1[s] + LX[c - LK] + LX[c + LK] + LX[c - 1] + LX[c + 1] - 6.0 * x0[s]) * g.inv_hh;
                const double r = b0[s] - bmean - lap;
                if (!RESTRICT) {
                    acc += r * r;
                    const double ar = fabs(r);
                    if (!(mx >= ar)) mx = ar;
                } else if (second) {
                    rr[li[s]] = prev[s] + r;
                } else {
                    prev[s] = r;
                }
            }
        }
        if (second) {
            __syncthreads();
            const int lgc = lg - 1;
            for (int t = threadIdx.x; t < (TJ / 2) * (kTK / 2); t += NT) {
                const int cj = t / (kTK / 2), ck = t - cj * (kTK / 2);
                const int q = (2 * cj) * kTK + 2 * ck;
                const double sr = rr[q] + rr[q + 1] + rr[q + kTK] + rr[q + kTK + 1];
                out[at3(lgc, (p & m) >> 1, (j0 >> 1) + cj, (k0 >> 1) + ck)] = 0.125 * sr;
            }
        }
        double* NX = lx[(p + 1 - i0) & 1];
        const bool more2 = p + 2 <= last;
#pragma unroll
        for (int s = 0; s < NS; ++s) {
            if (fl[s]) NX[threadIdx.x + s * NT] = xp1[s];
            xm1[s] = x0[s];
            x0[s] = xp1[s];
            if (more2) xp1[s] = xn2[s];
            xn2[s] = xn3[s];
            b0[s] = b1[s];
        }
        __syncthreads();
    }
    if (!RESTRICT) {
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
            out[2 * blockIdx.x] = red_s[0];
            out[2 * blockIdx.x + 1] = red_m[0];
        }
    }
}

// ---- coarsest level in one workgroup (n <= 8) --------------------------------------------
// Gauss-Seidel until rms(residual) <= rtol x initial, or down to its rounding floor, or cap
// sweeps.  The periodic Laplacian has the constant null mode; the restricted residual has
// zero mean, and the constant part of x is irrelevant (the potential's mean is fixed last).
__global__ void __launch_bounds__(kB) kp_coarsest(PGrid g, double* __restrict__ x, const double* __restrict__ b,
                                                  double bmean, int cap, double rtol)
{
    __shared__ double sx[512], sb[512];
    __shared__ double ra[kB], rb[kB];
    const int nc = 1 << (3 * g.lg), m = g.n - 1;
    for (int q = threadIdx.x; q < nc; q += kB) {
        sx[q] = x[q];
        sb[q] = b[q] - bmean;
    }
    __syncthreads();
    auto nsum = [&](int q) {
        const int i = q >> (2 * g.lg), j = (q >> g.lg) & m, k = q & m;
        return sx[at3(g.lg, (i + 1) & m, j, k)] + sx[at3(g.lg, (i - 1) & m, j, k)] + sx[at3(g.lg, i, (j + 1) & m, k)] +
               sx[at3(g.lg, i, (j - 1) & m, k)] + sx[at3(g.lg, i, j, (k + 1) & m)] + sx[at3(g.lg, i, j, (k - 1) & m)];
    };
    auto rms = [&](double& floor) {
        double s = 0.0, fl = 0.0;
        for (int q = threadIdx.x; q < nc; q += kB) {
            const double ns = nsum(q);
            const double r = sb[q] - (ns - 6.0 * sx[q]) * g.inv_hh;
            s += r * r;
            const double f1 = 2.220446049250313e-16 * ((fabs(ns) + 6.0 * fabs(sx[q])) * g.inv_hh + fabs(sb[q]));
            fl += f1 * f1;
        }
        ra[threadIdx.x] = s;
        rb[threadIdx.x] = fl;
        __syncthreads();
        for (int w = kB / 2; w > 0; w >>= 1) {
            if (threadIdx.x < w) {
                ra[threadIdx.x] += ra[threadIdx.x + w];
                rb[threadIdx.x] += rb[threadIdx.x + w];
            }
            __syncthreads();
        }
        const double ts = ra[0], tf = rb[0];
        __syncthreads();
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
            for (int q = threadIdx.x; q < nc; q += kB) {
                const int i = q >> (2 * g.lg), j = (q >> g.lg) & m, k = q & m;
                if (((i + j + k) & 1) != colour) continue;
                sx[q] = (nsum(q) - g.hh * sb[q]) * (1.0 / 6.0);
            }
            __syncthreads();
        }
    }
    for (int q = threadIdx.x; q < nc; q += kB) x[q] = sx[q];
}

__global__ void __launch_bounds__(kB) kp_add(double* __restrict__ x, double v, long long n)
{
    for (long long q = (long long)blockIdx.x * kB + threadIdx.x; q < n; q += (long long)gridDim.x * kB) x[q] += v;
}

unsigned grid_for(long long n)
{
    long long b = (n + kB - 1) / kB;
    if (b > 8192) b = 8192;
    return (unsigned)(b < 1 ? 1 : b);
}

}  // namespace

int poisson_partials(long long n) { return (int)grid_for(n); }

hipError_t poisson_source(const PoissonSource& c, long long n3, const double* rho, const double* u, double* S,
                          double* partial, hipStream_t s)
{
    hipLaunchKernelGGL(kp_source, dim3(grid_for(n3)), dim3(kB), 0, s, c, n3, rho, u, S, partial);
    return hipGetLastError();
}

// Streaming residual launch geometry: TJ x 64 tiles, ti planes per workgroup (even, dividing
// n), few enough workgroups for the partial-sum scratch.
constexpr int kRTJ = 8, kRNT = 256;

int resid_planes(int n)
{
    const long long tiles = (long long)(n / kRTJ) * (n / kTK);
    int ti = 8;
    while (ti < n && tiles * (n / ti) > 8192) ti *= 2;
    return ti;
}

hipError_t poisson_resid_norm(const PGrid& g, const double* x, const double* b, double bmean, double* partial,
                              int* nparts, hipStream_t s)
{
    if (x && g.n >= kTK && g.n <= 1024) {
        const int ti = resid_planes(g.n), ntj = g.n / kRTJ, ntk = g.n / kTK;
        const unsigned nb = (unsigned)((g.n / ti) * ntj * ntk);
        *nparts = (int)nb;
        hipLaunchKernelGGL((kp_resid_stream<kRTJ, kRNT, false>), dim3(nb), dim3(kRNT), 0, s, g, x, b, bmean, ti, ntj,
                           ntk, partial);
        return hipGetLastError();
    }
    const unsigned nb = grid_for(1LL << (3 * g.lg));
    *nparts = (int)nb;
    hipLaunchKernelGGL(kp_resid_norm, dim3(nb), dim3(kB), 0, s, g, x, b, bmean, partial);
    return hipGetLastError();
}

hipError_t poisson_ngs(const PGrid& g, double* x, const double* b, double bmean, hipStream_t s)
{
    const long long half = 1LL << (3 * g.lg - 1);
    for (int colour = 0; colour < 2; ++colour)
        hipLaunchKernelGGL(kp_ngs_colour, dim3((unsigned)((half + kB - 1) / kB)), dim3(kB), 0, s, g, x, b, bmean,
                           colour);
    return hipGetLastError();
}

// below 256 a level has too few tiles to fill the chip; the per-colour sweep is used there
int poisson_fused_min_n() { return 4 * kTK; }

hipError_t poisson_ngs_fused(const PGrid& g, const double* xin, double* xout, const double* b, double bmean, int ti,
                             hipStream_t s)
{
    constexpr int TJ = 16, NT = 512;
    if (g.n < kTK || g.n > 1024 || xin == xout || ti < 1 || ti > g.n || (g.n % ti) != 0) return hipErrorInvalidValue;
    const int ntj = g.n / TJ, ntk = g.n / kTK;
    const unsigned nb = (unsigned)((g.n / ti) * ntj * ntk);
    hipLaunchKernelGGL((kp_fused<TJ, NT>), dim3(nb), dim3(NT), 0, s, g, xin, xout, b, bmean, ti, ntj, ntk);
    return hipGetLastError();
}

int poisson_fused2_planes(int n) { return n / 4 < 128 ? n / 4 : 128; }

hipError_t poisson_ngs_fused2(const PGrid& g, const double* xin, double* xout, const double* b, double bmean, int ti,
                              hipStream_t s)
{
    // 24 x 72 cells with the halo, 4 slots per thread; 8 x 64 tiles (3 slots of 384 threads)
    // re-read more halo per pass and ran slower (1.39 against 1.21 ms at 512^3)
    constexpr int TJ = 16, NT = 512;
    if (g.n < kTK || g.n > 1024 || xin == xout || ti < 1 || ti > g.n || (g.n % ti) != 0) return hipErrorInvalidValue;
    const int ntj = g.n / TJ, ntk = g.n / kTK;
    const unsigned nb = (unsigned)((g.n / ti) * ntj * ntk);
    hipLaunchKernelGGL((kp_fused2<TJ, NT>), dim3(nb), dim3(NT), 0, s, g, xin, xout, b, bmean, ti, ntj, ntk);
    return hipGetLastError();
}

hipError_t poisson_resid_restrict(const PGrid& g, const double* x, const double* b, double bmean, double* bc,
                                  hipStream_t s)
{
    if (g.n >= kTK && g.n <= 1024) {
        const int ti = resid_planes(g.n), ntj = g.n / kRTJ, ntk = g.n / kTK;
        const unsigned nb = (unsigned)((g.n / ti) * ntj * ntk);
        hipLaunchKernelGGL((kp_resid_stream<kRTJ, kRNT, true>), dim3(nb), dim3(kRNT), 0, s, g, x, b, bmean, ti, ntj,
                           ntk, bc);
        return hipGetLastError();
    }
    const long long ncell = 1LL << (3 * (g.lg - 1));
    hipLaunchKernelGGL(kp_resid_restrict, dim3((unsigned)((ncell + kB - 1) / kB)), dim3(kB), 0, s, g, x, b, bmean, bc);
    return hipGetLastError();
}

hipError_t poisson_coarsest(const PGrid& g, double* x, const double* b, double bmean, int cap, double rtol,
                            hipStream_t s)
{
    if (g.n > 8) return hipErrorInvalidValue;
    hipLaunchKernelGGL(kp_coarsest, dim3(1), dim3(kB), 0, s, g, x, b, bmean, cap, rtol);
    return hipGetLastError();
}

hipError_t poisson_add(double* x, double v, long long n, hipStream_t s)
{
    hipLaunchKernelGGL(kp_add, dim3(grid_for(n)), dim3(kB), 0, s, x, v, n);
    return hipGetLastError();
}

}  // namespace mgfr
