// Single-precision kernels of the defect-correction (mixed precision) domain solver.
//
// The outer double-precision loop holds u and its residual d = L(u) - f.  In between, a
// single-precision FAS multigrid solves N(e) = r for the correction e of u, in the
// correction form of device_fp32.h (r = -d, base ub = u rounded to single precision).
// The coarse levels of this inner multigrid use the restricted base R ub.  Smoother:
// red-black Newton-Gauss-Seidel on N (Sec. V.B.1 applied to the correction equation).
#include "device_fp32.h"
#include "fused_fp32.h"

#include <type_traits>

namespace mgfr {
namespace {

using dev32::em1f;
using dev32::make_v;
using dev32::newton32;
using dev32::Op32;
using dev32::op32;
using dev32::Res32;
using dev32::V32;

constexpr int kBlock = 256;
constexpr int kTK = 64;

__device__ __forceinline__ long long at(int lg, int i, int j, int k)
{
    return ((((long long)i << lg) + j) << lg) + k;
}

__device__ __forceinline__ void nbr_index(int lg, int i, int j, int k, long long (&q)[6])
{
    const int m = (1 << lg) - 1;
    q[0] = at(lg, (i - 1) & m, j, k);
    q[1] = at(lg, (i + 1) & m, j, k);
    q[2] = at(lg, i, (j - 1) & m, k);
    q[3] = at(lg, i, (j + 1) & m, k);
    q[4] = at(lg, i, j, (k - 1) & m);
    q[5] = at(lg, i, j, (k + 1) & m);
}

// ---- per-colour sweep, in place (small levels) ------------------------------------------
__global__ void __launch_bounds__(kBlock) k32_ngs_colour(Grid g, const float* __restrict__ ub, float* __restrict__ e,
                                                         const float* __restrict__ f, int colour)
{
    if (g.halt && *g.halt) return;
    const Op32 o = op32(g);
    const long long half = 1LL << (3 * g.lg - 1);
    const long long t = (long long)blockIdx.x * kBlock + threadIdx.x;
    if (t >= half) return;
    const int hk = g.n >> 1;
    const int s = (int)(t & (hk - 1));
    const long long row = t >> (g.lg - 1);
    const int i = (int)(row >> g.lg), j = (int)(row & (g.n - 1));
    const int k = 2 * s + ((i + j + colour) & 1);
    const long long q = at(g.lg, i, j, k);
    long long qn[6];
    nbr_index(g.lg, i, j, k, qn);
    V32 nb[6];
#pragma unroll
    for (int v = 0; v < 6; ++v) nb[v] = make_v(ub[qn[v]], e[qn[v]]);
    const V32 c = make_v(ub[q], e[q]);
    const Res32 r = dev32::corr_op(o, c, nb, f[q]);
    e[q] = c.e + newton32(r, o.max_step);
}

// ---- fused red-black sweep (n >= 64), same scheme as the double-precision one ----------
// Three LDS plane buffers, one barrier per plane, the red ring recomputed per tile.  A thread
// owns a pair of k-adjacent columns: at every plane step exactly one column of each pair
// holds the cells to update (red on plane p, black on plane p-1), and the two swap at the
// next step, so with the step loop unrolled by two every lane updates a cell at every step.
using fused32::Col32;

template <int TJ, int TK, int NT>
__global__ void __launch_bounds__(NT) k32_fused(Grid g, const float* __restrict__ ub, const float* __restrict__ ein,
                                                float* __restrict__ eout, const float* __restrict__ f,
                                                FusedSweep32 a)
{
    if (g.halt && *g.halt) return;
    constexpr int LJ = TJ + 4, LK = TK + 4, NL = LJ * LK, NP = NL / 2;
    static_assert(NP <= NT, "one column pair per thread");
    __shared__ V32 lv[3][NL];
    const Op32 o = op32(g);
    const int nb = gridDim.x;
    int lid = blockIdx.x;
    if ((nb & 7) == 0) lid = (lid & 7) * (nb >> 3) + (lid >> 3);
    const int tk = lid % a.ntk;
    lid /= a.ntk;
    const int tj = lid % a.ntj;
    const int ci = lid / a.ntj;
    const int i0 = ci * a.ti, j0 = tj * TJ, k0 = tk * TK;
    const int lg = g.lg, m = g.n - 1;
    const int last = i0 + a.ti + 1;  // last plane read

    // X: the column of the pair whose cell on plane i0-1 is red; Y: the other one
    Col32 X{}, Y{};
    const int pc = threadIdx.x;
    if (pc < NP) {
        const int jj = pc / (LK / 2), kk0 = 2 * (pc - jj * (LK / 2));
        const int gj = (j0 - 2 + jj) & m, gk0 = (k0 - 2 + kk0) & m;
        const int sx = (i0 - 1 + gj + gk0) & 1;
        auto setup = [&](Col32& q, int d) {
            const int kk = kk0 + d;
            q.col = (unsigned)((gj << lg) | (gk0 + d));
            q.c = jj * LK + kk;
            q.fl = 1;
            if (jj >= 1 && jj <= LJ - 2 && kk >= 1 && kk <= LK - 2) q.fl |= 2;
            if (jj >= 2 && jj <= LJ - 3 && kk >= 2 && kk <= LK - 3) q.fl |= 4;
        };
        setup(X, sx);
        setup(Y, 1 - sx);
    }
    // element offsets fit in 32 bits (n <= 1024)
    auto offset = [&](int p, const Col32& q) -> unsigned { return ((unsigned)(p & m) << (2 * lg)) + q.col; };
    auto buf = [&](int p) { return (p - i0 + 3) % 3; };
    auto prologue = [&](Col32& q) {
        if (!q.fl) return;
        // planes i0-2, i0-1, i0 in slots 1, 2, 3; plane i0+1 raw in slot 1
        q.v[1] = make_v(ub[offset(i0 - 2, q)], ein[offset(i0 - 2, q)]);
        q.v[2] = make_v(ub[offset(i0 - 1, q)], ein[offset(i0 - 1, q)]);
        q.v[3] = make_v(ub[offset(i0, q)], ein[offset(i0, q)]);
        q.f[1] = f[offset(i0 - 2, q)];
        q.f[2] = f[offset(i0 - 1, q)];
        q.f[3] = f[offset(i0, q)];
        q.rub[1] = ub[offset(i0 + 1, q)];
        q.re[1] = ein[offset(i0 + 1, q)];
        q.rf[1] = f[offset(i0 + 1, q)];
        lv[buf(i0 - 1)][q.c] = q.v[2];
    };
    prologue(X);
    prologue(Y);
    __syncthreads();

    // One plane step, R = (p - i0 + 1) mod 4 fixed at compile time so that the register
    // planes rotate by renaming.  A holds the red cell of plane p and the black cell of
    // plane p-1.
    auto step = [&](auto Rc, int p, Col32& A, Col32& B) {
        constexpr int R = decltype(Rc)::value;
        constexpr int M2 = R, M1 = (R + 1) & 3, P0 = (R + 2) & 3, P1 = (R + 3) & 3;
        constexpr int N2 = (R + 1) & 1, N3 = R & 1;  // raw slots of planes p+2, p+3
        if (p + 3 <= last) {
            if (A.fl) {
                A.rub[N3] = ub[offset(p + 3, A)];
                A.re[N3] = ein[offset(p + 3, A)];
                A.rf[N3] = f[offset(p + 3, A)];
            }
            if (B.fl) {
                B.rub[N3] = ub[offset(p + 3, B)];
                B.re[N3] = ein[offset(p + 3, B)];
                B.rf[N3] = f[offset(p + 3, B)];
            }
        }
        V32* LA = lv[buf(p)];
        if (A.fl & 2) {
            const int c = A.c;
            const V32 nbv[6] = {A.v[M1], A.v[P1], LA[c - LK], LA[c + LK], LA[c - 1], LA[c + 1]};
            const Res32 r = dev32::corr_op(o, A.v[P0], nbv, A.f[P0]);
            A.v[P0] = dev32::remake_v(A.v[P0], A.v[P0].e + newton32(r, o.max_step));
            LA[c] = A.v[P0];
        }
        if (p - 1 >= i0) {
            if (A.fl & 4) {
                const V32* LB = lv[buf(p - 1)];
                const int c = A.c;
                const V32 nbv[6] = {A.v[M2], A.v[P0], LB[c - LK], LB[c + LK], LB[c - 1], LB[c + 1]};
                const Res32 r = dev32::corr_op(o, A.v[M1], nbv, A.f[M1]);
                A.v[M1].e = A.v[M1].e + newton32(r, o.max_step);
                eout[offset(p - 1, A)] = A.v[M1].e;
            }
            if (B.fl & 4) eout[offset(p - 1, B)] = B.v[M1].e;
        }
        V32* LC = lv[buf(p + 1)];
        const bool more2 = p + 2 <= last;
        auto advance = [&](Col32& q) {
            if (q.fl) {
                LC[q.c] = q.v[P1];
                if (more2) {  // plane p+2 takes the slot of plane p-2
                    q.v[M2] = make_v(q.rub[N2], q.re[N2]);
                    q.f[M2] = q.rf[N2];
                }
            }
        };
        advance(A);
        advance(B);
        __syncthreads();
    };
    using I0 = std::integral_constant<int, 0>;
    using I1 = std::integral_constant<int, 1>;
    using I2 = std::integral_constant<int, 2>;
    using I3 = std::integral_constant<int, 3>;
    // a.ti + 2 steps (a.ti a multiple of 4): two, then groups of four so that the register
    // planes and the column roles are back in place at the end of every iteration.  X holds
    // the red cells of planes i0-1, i0+1, ...
    step(I0{}, i0 - 1, X, Y);
    step(I1{}, i0, Y, X);
    for (int p = i0 + 1; p <= i0 + a.ti; p += 4) {
        step(I2{}, p, X, Y);
        step(I3{}, p + 1, Y, X);
        step(I0{}, p + 2, X, Y);
        step(I1{}, p + 3, Y, X);
    }
}

// ---- fused red-black sweep, one tile column pair per thread -------------------------------
// The tile sweep itself is in fused_fp32.h (shared with the batched solves).
template <int TJ, int TK>
__global__ void __launch_bounds__(TJ * TK / 2) k32_fused2(Grid g, const float* __restrict__ ub,
                                                         const float* __restrict__ ein, float* __restrict__ eout,
                                                         const float* __restrict__ f, FusedSweep32 a)
{
    if (g.halt && *g.halt) return;
    __shared__ V32 lv[3][(TJ + 4) * (TK + 4)];
    const int nb = gridDim.x;
    int lid = blockIdx.x;
    if ((nb & 7) == 0) lid = (lid & 7) * (nb >> 3) + (lid >> 3);
    const int tk = lid % a.ntk;
    lid /= a.ntk;
    const int tj = lid % a.ntj;
    const int ci = lid / a.ntj;
    fused32::sweep_tile<TJ, TK>(op32(g), g.n, g.lg, ci * a.ti, tj * TJ, tk * TK, a.ti, ub, ein, eout, f, lv);
}

// ---- streaming residual + restriction (n >= 64) ----------------------------------------
// Per plane the tile's cell values (ub, e, B, M) plus a one-cell in-plane halo sit in LDS and
// the i-neighbours in registers, so every cell's exponentials are evaluated once; the
// residual N(e) - f of plane pairs is summed over 2x2x2 children into the coarse level.
template <int TJ, int NT>
__global__ void __launch_bounds__(NT) k32_resid_stream(Grid g, const float* __restrict__ ub, const float* __restrict__ e,
                                                       const float* __restrict__ f, float* __restrict__ ec,
                                                       float* __restrict__ ehat, float* __restrict__ fc, int ti,
                                                       int ntj, int ntk)
{
    if (g.halt && *g.halt) return;
    constexpr int LJ = TJ + 2, LK = kTK + 2, NL = LJ * LK;
    constexpr int NS = (NL + NT - 1) / NT;
    __shared__ V32 lv[2][NL];
    __shared__ float re[TJ * kTK], rd[TJ * kTK];
    const Op32 o = op32(g);
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
    // element offsets fit in 32 bits (n <= 1024)
    auto offset = [&](int p, int s) -> unsigned { return ((unsigned)(p & m) << (2 * lg)) + col[s]; };
    // planes p-1, p, p+1 expanded in registers; raw (ub, e) of plane p+2 and f of plane p+1 in flight
    V32 vm1[NS], v0[NS], vp1[NS];
    float u2[NS], e2[NS], f0[NS], eprev[NS], dprev[NS];
#pragma unroll
    for (int s = 0; s < NS; ++s) {
        vm1[s] = v0[s] = vp1[s] = V32{0.f, 0.f, 0.f, 0.f};
        u2[s] = e2[s] = f0[s] = eprev[s] = dprev[s] = 0.0f;
        if (fl[s] & 2) f0[s] = f[offset(i0, s)];
        if (fl[s]) {
            vm1[s] = make_v(ub[offset(i0 - 1, s)], e[offset(i0 - 1, s)]);
            v0[s] = make_v(ub[offset(i0, s)], e[offset(i0, s)]);
            vp1[s] = make_v(ub[offset(i0 + 1, s)], e[offset(i0 + 1, s)]);
            u2[s] = ub[offset(i0 + 2, s)];
            e2[s] = e[offset(i0 + 2, s)];
            lv[0][threadIdx.x + s * NT] = v0[s];
        }
    }
    __syncthreads();
    for (int p = i0; p < i0 + ti; ++p) {
        const bool more3 = p + 3 <= last, moref = p + 1 < last;
        float u3[NS], e3[NS], f1[NS];
#pragma unroll
        for (int s = 0; s < NS; ++s) {
            u3[s] = e3[s] = f1[s] = 0.0f;
            if (fl[s] && more3) {
                u3[s] = ub[offset(p + 3, s)];
                e3[s] = e[offset(p + 3, s)];
            }
            if ((fl[s] & 2) && moref) f1[s] = f[offset(p + 1, s)];
        }
        const V32* LV = lv[(p - i0) & 1];
        const bool second = (p - i0) & 1;
#pragma unroll
        for (int s = 0; s < NS; ++s) {
            const int c = threadIdx.x + s * NT;
            if (fl[s] & 2) {
                const V32 nbv[6] = {vm1[s], vp1[s], LV[c - LK], LV[c + LK], LV[c - 1], LV[c + 1]};
                const float d = dev32::corr_op(o, v0[s], nbv, f0[s]).N;
                if (second) {
                    re[li[s]] = eprev[s] + v0[s].e;
                    rd[li[s]] = dprev[s] + d;
                } else {
                    eprev[s] = v0[s].e;
                    dprev[s] = d;
                }
            }
        }
        if (second) {
            __syncthreads();
            const int lgc = lg - 1;
            for (int t = threadIdx.x; t < (TJ / 2) * (kTK / 2); t += NT) {
                const int cj = t / (kTK / 2), ck = t - cj * (kTK / 2);
                const int q = (2 * cj) * kTK + 2 * ck;
                const float se = re[q] + re[q + 1] + re[q + kTK] + re[q + kTK + 1];
                const float sd = rd[q] + rd[q + 1] + rd[q + kTK] + rd[q + kTK + 1];
                const long long qc = at(lgc, (p & m) >> 1, (j0 >> 1) + cj, (k0 >> 1) + ck);
                ec[qc] = 0.125f * se;
                ehat[qc] = 0.125f * se;
                fc[qc] = 0.125f * sd;
            }
        }
        // stage plane p+1 into the other buffer and shift the registers
        V32* NV = lv[(p + 1 - i0) & 1];
        const bool more2 = p + 2 <= last;
#pragma unroll
        for (int s = 0; s < NS; ++s) {
            if (fl[s]) NV[threadIdx.x + s * NT] = vp1[s];
            vm1[s] = v0[s];
            v0[s] = vp1[s];
            if (more2 && fl[s]) vp1[s] = make_v(u2[s], e2[s]);
            u2[s] = u3[s];
            e2[s] = e3[s];
            f0[s] = f1[s];
        }
        __syncthreads();
    }
}

// ---- residual + restriction, FAS right-hand side, transfers ----------------------------
__global__ void __launch_bounds__(kBlock) k32_resid_restrict(Grid g, const float* __restrict__ ub,
                                                             const float* __restrict__ e,
                                                             const float* __restrict__ f,
                                                             float* __restrict__ ec, float* __restrict__ ehat,
                                                             float* __restrict__ fc)
{
    if (g.halt && *g.halt) return;
    const Op32 o = op32(g);
    const int lgc = g.lg - 1, nc = g.n >> 1;
    const long long tc = (long long)blockIdx.x * kBlock + threadIdx.x;
    if (tc >= (1LL << (3 * lgc))) return;
    const int I = (int)(tc >> (2 * lgc)), J = (int)((tc >> lgc) & (nc - 1)), K = (int)(tc & (nc - 1));
    float se = 0.0f, sd = 0.0f;
#pragma unroll
    for (int x = 0; x < 2; ++x)
#pragma unroll
        for (int y = 0; y < 2; ++y)
#pragma unroll
            for (int z = 0; z < 2; ++z) {
                const int i = 2 * I + x, j = 2 * J + y, k = 2 * K + z;
                const long long q = at(g.lg, i, j, k);
                long long qn[6];
                nbr_index(g.lg, i, j, k, qn);
                V32 nb[6];
#pragma unroll
                for (int v = 0; v < 6; ++v) nb[v] = make_v(ub[qn[v]], e[qn[v]]);
                const V32 c = make_v(ub[q], e[q]);
                se += c.e;
                sd += dev32::corr_op(o, c, nb, f[q]).N;
            }
    ec[tc] = 0.125f * se;
    ehat[tc] = 0.125f * se;
    fc[tc] = 0.125f * sd;
}

__global__ void __launch_bounds__(kBlock) k32_fas_rhs(Grid g, const float* __restrict__ ub,
                                                      const float* __restrict__ ehat, float* __restrict__ f)
{
    if (g.halt && *g.halt) return;
    const Op32 o = op32(g);
    const long long q = (long long)blockIdx.x * kBlock + threadIdx.x;
    if (q >= (1LL << (3 * g.lg))) return;
    const int i = (int)(q >> (2 * g.lg)), j = (int)((q >> g.lg) & (g.n - 1)), k = (int)(q & (g.n - 1));
    long long qn[6];
    nbr_index(g.lg, i, j, k, qn);
    V32 nb[6];
#pragma unroll
    for (int v = 0; v < 6; ++v) nb[v] = make_v(ub[qn[v]], ehat[qn[v]]);
    f[q] = dev32::corr_op(o, make_v(ub[q], ehat[q]), nb, 0.0f).N - f[q];
}

__global__ void __launch_bounds__(kBlock) k32_restrict_mean(int lgc, const float* __restrict__ fine,
                                                            float* __restrict__ coarse)
{
    const long long tc = (long long)blockIdx.x * kBlock + threadIdx.x;
    if (tc >= (1LL << (3 * lgc))) return;
    const int nc = 1 << lgc, lg = lgc + 1;
    const int I = (int)(tc >> (2 * lgc)), J = (int)((tc >> lgc) & (nc - 1)), K = (int)(tc & (nc - 1));
    float s = 0.0f;
#pragma unroll
    for (int x = 0; x < 2; ++x)
#pragma unroll
        for (int y = 0; y < 2; ++y)
#pragma unroll
            for (int z = 0; z < 2; ++z) s += fine[at(lg, 2 * I + x, 2 * J + y, 2 * K + z)];
    coarse[tc] = 0.125f * s;
}

__global__ void __launch_bounds__(kBlock) k32_fill(float* __restrict__ x, float v, long long n)
{
    for (long long q = (long long)blockIdx.x * kBlock + threadIdx.x; q < n; q += (long long)gridDim.x * kBlock) x[q] = v;
}

// ---- coarsest level in one workgroup (n <= 8) ------------------------------------------
__global__ void __launch_bounds__(kBlock) k32_coarsest(Grid g, const float* __restrict__ ub, float* __restrict__ e,
                                                       const float* __restrict__ f, int cap, float rtol)
{
    if (g.halt && *g.halt) return;
    __shared__ float sub[512], se[512], sf[512];
    __shared__ float rs[kBlock], rf[kBlock];
    const Op32 o = op32(g);
    const int nc = 1 << (3 * g.lg);
    for (int q = threadIdx.x; q < nc; q += kBlock) {
        sub[q] = ub[q];
        se[q] = e[q];
        sf[q] = f[q];
    }
    __syncthreads();
    auto cell = [&](int q, V32& c, V32 (&nb)[6]) {
        const int i = q >> (2 * g.lg), j = (q >> g.lg) & (g.n - 1), k = q & (g.n - 1);
        long long qn[6];
        nbr_index(g.lg, i, j, k, qn);
#pragma unroll
        for (int v = 0; v < 6; ++v) nb[v] = make_v(sub[qn[v]], se[qn[v]]);
        c = make_v(sub[q], se[q]);
        return (i + j + k) & 1;
    };
    // rms of N - f and its rounding floor (single precision: one unit in the last place of
    // |dN||e| plus the summed magnitudes)
    auto rms = [&](float& floor) {
        float s = 0.0f, fl = 0.0f;
        for (int q = threadIdx.x; q < nc; q += kBlock) {
            V32 c, nb[6];
            cell(q, c, nb);
            const Res32 r = dev32::corr_op(o, c, nb, sf[q]);
            s += r.N * r.N;
            const float f1 = 1.1920929e-7f * (fabsf(r.dN) * fabsf(c.e) + fabsf(sf[q]));
            fl += f1 * f1;
        }
        rs[threadIdx.x] = s;
        rf[threadIdx.x] = fl;
        __syncthreads();
        for (int w = kBlock / 2; w > 0; w >>= 1) {
            if (threadIdx.x < w) {
                rs[threadIdx.x] += rs[threadIdx.x + w];
                rf[threadIdx.x] += rf[threadIdx.x + w];
            }
            __syncthreads();
        }
        const float tot = rs[0], tf = rf[0];
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
            for (int q = threadIdx.x; q < nc; q += kBlock) {
                V32 c, nb[6];
                if (cell(q, c, nb) != colour) continue;
                const Res32 r = dev32::corr_op(o, c, nb, sf[q]);
                se[q] = c.e + newton32(r, o.max_step);
            }
            __syncthreads();
        }
    }
    for (int q = threadIdx.x; q < nc; q += kBlock) e[q] = se[q];
}

inline unsigned blocks_for(long long work) { return (unsigned)((work + kBlock - 1) / kBlock); }

}  // namespace

hipError_t ngs_sweep32(const Grid& g, const float* ub, float* e, const float* f, hipStream_t s)
{
    const long long half = cells(g) / 2;
    for (int colour = 0; colour < 2; ++colour)
        hipLaunchKernelGGL(k32_ngs_colour, dim3(blocks_for(half)), dim3(kBlock), 0, s, g, ub, e, f, colour);
    return hipGetLastError();
}

hipError_t ngs_sweep32_fused(const Grid& g, const float* ub, const float* ein, float* eout, const float* f,
                             int ti, int tile, hipStream_t s)
{
    if (g.n < kTK || g.n > 1024 || ein == eout || ti < 4 || (ti & 3) || ti > g.n || (g.n % ti) != 0)
        return hipErrorInvalidValue;
    if (tile != kTile32Paired) {
        // one tile column pair per thread
        FusedSweep32 a{};
        a.ti = ti;
        auto launch = [&](auto kern, int TJ, int TK) {
            if (g.n % TJ || g.n % TK) return hipErrorInvalidValue;
            a.ntj = g.n / TJ;
            a.ntk = g.n / TK;
            const unsigned nb = (unsigned)((g.n / ti) * a.ntj * a.ntk);
            hipLaunchKernelGGL(kern, dim3(nb), dim3(TJ * TK / 2), 0, s, g, ub, ein, eout, f, a);
            return hipGetLastError();
        };
        if (tile == kTile32x32) return launch(k32_fused2<32, 32>, 32, 32);
        if (tile == kTile16x64) return launch(k32_fused2<16, 64>, 16, 64);
        if (tile == kTile32x64) return launch(k32_fused2<32, 64>, 32, 64);
        return launch(k32_fused2<16, 32>, 16, 32);
    }
    // 216 column pairs per 12 x 36 tile.  With 90 VGPRs a SIMD holds 5 wavefronts, so five
    // 4-wavefront workgroups share a CU: narrower tiles re-read more halo than 8 x 64 tiles
    // of 7 wavefronts, but the extra resident waves hide more of the per-plane barrier and
    // load latency (0.90 against 0.95 ms per 512^3 sweep).
    constexpr int TJ = 8, TK = 32, NT = 256;
    FusedSweep32 a{};
    a.ti = ti;
    a.ntj = g.n / TJ;
    a.ntk = g.n / TK;
    const unsigned nb = (unsigned)((g.n / ti) * a.ntj * a.ntk);
    hipLaunchKernelGGL((k32_fused<TJ, TK, NT>), dim3(nb), dim3(NT), 0, s, g, ub, ein, eout, f, a);
    return hipGetLastError();
}

hipError_t resid_restrict32(const Grid& g, const float* ub, const float* e, const float* f, float* ec,
                            float* ehat, float* fc, hipStream_t s)
{
    if (g.n >= kTK) {
        constexpr int TJ = 8, NT = 256;
        const int ntj = g.n / TJ, ntk = g.n / kTK;
        int ti = 8;
        while (ti < g.n && (long long)ntj * ntk * (g.n / ti) > 8192) ti *= 2;
        const unsigned nb = (unsigned)((g.n / ti) * ntj * ntk);
        hipLaunchKernelGGL((k32_resid_stream<TJ, NT>), dim3(nb), dim3(NT), 0, s, g, ub, e, f, ec, ehat, fc, ti, ntj,
                           ntk);
        return hipGetLastError();
    }
    hipLaunchKernelGGL(k32_resid_restrict, dim3(blocks_for(cells(g) / 8)), dim3(kBlock), 0, s, g, ub, e, f, ec,
                       ehat, fc);
    return hipGetLastError();
}

hipError_t fas_rhs32(const Grid& gc, const float* ubc, const float* ehat, float* f, hipStream_t s)
{
    hipLaunchKernelGGL(k32_fas_rhs, dim3(blocks_for(cells(gc))), dim3(kBlock), 0, s, gc, ubc, ehat, f);
    return hipGetLastError();
}

hipError_t restrict_mean32(const Grid& gc, const float* fine, float* coarse, hipStream_t s)
{
    hipLaunchKernelGGL(k32_restrict_mean, dim3(blocks_for(cells(gc))), dim3(kBlock), 0, s, gc.lg, fine, coarse);
    return hipGetLastError();
}

hipError_t coarsest_solve32(const Grid& g, const float* ub, float* e, const float* f, int cap, double rtol,
                            hipStream_t s)
{
    if (g.n > 8) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k32_coarsest, dim3(1), dim3(kBlock), 0, s, g, ub, e, f, cap, (float)rtol);
    return hipGetLastError();
}

hipError_t fill32(float* x, float v, long long n, hipStream_t s)
{
    long long b = (n + kBlock - 1) / kBlock;
    if (b > 4096) b = 4096;
    if (b < 1) b = 1;
    hipLaunchKernelGGL(k32_fill, dim3((unsigned)b), dim3(kBlock), 0, s, x, v, n);
    return hipGetLastError();
}

}  // namespace mgfr
