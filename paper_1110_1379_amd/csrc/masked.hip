// Kernels of a refinement level solved with the mask scheme (Sec. V), double precision.
//
// The level is the periodic N^3 grid of its resolution.  A cell with mask > 0 is active and
// relaxed; a cell with mask <= 0 keeps a fixed value w (the coarser level's solution
// interpolated there).  A masked neighbour nb of an active cell i enters the operator as
// the ghost value u_g = (1 - r) u_b + r u_i, r = m_nb / m_i (eq. u_i-1jk), with the boundary
// value u_b = (m_i w_nb - m_nb w_i) / (m_i - m_nb) fixed where the linearly interpolated mask
// vanishes (eq. phi_b), and b_g = exp(u_g) (b is not interpolated): eq. bc_modified_fR_op
// and eq. bc_modified_fR_dop.  Coarse levels carry the 8-child means of the masks and of w.
// The residual is restricted from active children (masked ones count zero) into active coarse
// cells, R u from all 8 children; the coarse correction is zero in masked coarse cells and
// is prolongated into active fine cells only (Sec. V.A.2, V.A.3, V.B.2).
//
// On the finest level a mask that only holds +1 and -1 is read as one byte per cell (1:
// active), which gives the same values as the float mask.
#include "device_fp64.h"

#include <type_traits>

namespace mgfr {
namespace {

constexpr int kB = 256;
constexpr int kMaxParts = 8192;

using dev::OpVal;
using dev::at;
using dev::bounded;
using u8 = unsigned char;

// mask value of cell q: the float mask, or a byte flag standing for +1 / -1
__device__ __forceinline__ double mval(const float* __restrict__ m, long long q) { return m[q]; }
__device__ __forceinline__ double mval(const u8* __restrict__ m, long long q) { return m[q] ? 1.0 : -1.0; }

// The term of a masked neighbour (mask mn <= 0, fixed value wn) in L_i and dL_i/du_i of an
// active cell of mask mi, value ui, b_i = bi and fixed value wi: the boundary value
// u_b = (mi wn - mn wi) / (mi - mn), the ghost u_g = (1 - r) u_b + r ui with r = mn / mi, and
// b_g = exp(u_g) (eq. phi_b, eq. u_i-1jk, eq. bc_modified_fR_op, eq. bc_modified_fR_dop).
__device__ __forceinline__ void masked_face(double mi, double mn, double wn, double wi, double ui, double bi,
                                            double& L, double& dL)
{
    const double r = mn / mi;
    const double ubv = (mi * wn - mn * wi) / (mi - mn);
    const double ug = (1.0 - r) * ubv + r * ui;
    const double bg = exp(ug), du = ug - ui;
    L = fma(bg + bi, du, L);
    // chain rule: du_g/du_i = r, db_g/du_i = r b_g
    dL += (r * bg + bi) * du + (bg + bi) * (r - 1.0);
}

// L_i - f and dL_i/du_i at active cell (i,j,k) of value ui, mask mi.
template <class M>
__device__ __forceinline__ OpVal masked_op(const Grid& g, const M* __restrict__ mask,
                                           const double* __restrict__ w, const double* __restrict__ u,
                                           int i, int j, int k, double ui, double mi, double f)
{
    const int m = g.n - 1;
    const long long qn[6] = {at(g, (i - 1) & m, j, k), at(g, (i + 1) & m, j, k), at(g, i, (j - 1) & m, k),
                             at(g, i, (j + 1) & m, k), at(g, i, j, (k - 1) & m), at(g, i, j, (k + 1) & m)};
    const double bi = exp(ui);
    double L = 0.0, dL = 0.0, wi = 0.0;
    bool have_wi = false;
#pragma unroll
    for (int v = 0; v < 6; ++v) {
        const double mn = mval(mask, qn[v]);
        if (mn > 0.0) {
            const double un = u[qn[v]], bn = exp(un), du = un - ui;
            L = fma(bn + bi, du, L);
            dL += bi * du - bn - bi;
        } else {
            if (!have_wi) {
                wi = w[at(g, i, j, k)];
                have_wi = true;
            }
            masked_face(mi, mn, w[qn[v]], wi, ui, bi, L, dL);
        }
    }
    const double S = dev::curvature(g, ui, bi);
    OpVal o;
    o.L = fma(g.C, L, S) - f;
    o.dL = fma(g.C, dL, -S * g.inv_np1);
    return o;
}

// Summed magnitudes of the terms of L_i - f at an active cell: C (b_nb + b_i)|u_nb - u_i| per
// face (the ghost's for a masked neighbour), the curvature term and |f|.
__device__ double masked_mag(const Grid& g, const float* mask, const double* w, const double* u, int i, int j, int k,
                             double ui, double mi, double f)
{
    const int m = g.n - 1;
    const long long qn[6] = {at(g, (i - 1) & m, j, k), at(g, (i + 1) & m, j, k), at(g, i, (j - 1) & m, k),
                             at(g, i, (j + 1) & m, k), at(g, i, j, (k - 1) & m), at(g, i, j, (k + 1) & m)};
    const double bi = exp(ui), wi = w[at(g, i, j, k)];
    double t = 0.0;
    for (int v = 0; v < 6; ++v) {
        const double mn = mask[qn[v]];
        double un;
        if (mn > 0.0) {
            un = u[qn[v]];
        } else {
            const double r = mn / mi;
            un = (1.0 - r) * ((mi * w[qn[v]] - mn * wi) / (mi - mn)) + r * ui;
        }
        t += g.C * (exp(un) + bi) * fabs(un - ui);
    }
    return t + g.A * exp(-ui * g.inv_np1) + fabs(f);
}

__device__ __forceinline__ void cell_of(const Grid& g, long long q, int& i, int& j, int& k)
{
    i = (int)(q >> (2 * g.lg));
    j = (int)((q >> g.lg) & (g.n - 1));
    k = (int)(q & (g.n - 1));
}

// Block reduction over kB threads in a fixed order: a summed, b maxed (NaN propagates).
__device__ __forceinline__ void block_sum_max(double& a, double& b, double* sa, double* sb)
{
    sa[threadIdx.x] = a;
    sb[threadIdx.x] = b;
    __syncthreads();
    for (int s = kB / 2; s > 0; s >>= 1) {
        if (threadIdx.x < s) {
            sa[threadIdx.x] += sa[threadIdx.x + s];
            const double o = sb[threadIdx.x + s];
            if (!(sb[threadIdx.x] >= o)) sb[threadIdx.x] = o;
        }
        __syncthreads();
    }
    a = sa[0];
    b = sb[0];
    __syncthreads();
}

// Block reduction over kB threads in a fixed order: a and b both summed.
__device__ __forceinline__ void block_sum2(double& a, double& b, double* sa, double* sb)
{
    sa[threadIdx.x] = a;
    sb[threadIdx.x] = b;
    __syncthreads();
    for (int s = kB / 2; s > 0; s >>= 1) {
        if (threadIdx.x < s) {
            sa[threadIdx.x] += sa[threadIdx.x + s];
            sb[threadIdx.x] += sb[threadIdx.x + s];
        }
        __syncthreads();
    }
    a = sa[0];
    b = sb[0];
    __syncthreads();
}

// One colour of a red-black Newton-Gauss-Seidel sweep; one thread per cell of the colour,
// masked cells untouched.
template <class M>
__global__ void __launch_bounds__(kB) km_ngs_colour(Grid g, const M* __restrict__ mask,
                                                    const double* __restrict__ w, double* __restrict__ u,
                                                    const double* __restrict__ src, int colour)
{
    const long long half = 1LL << (3 * g.lg - 1);
    const long long t = (long long)blockIdx.x * kB + threadIdx.x;
    if (t >= half) return;
    const int hk = g.n >> 1;
    const int s = (int)(t & (hk - 1));
    const long long row = t >> (g.lg - 1);
    const int i = (int)(row >> g.lg), j = (int)(row & (g.n - 1));
    const int k = 2 * s + ((i + j + colour) & 1);
    const long long q = at(g, i, j, k);
    const double mi = mval(mask, q);
    if (!(mi > 0.0)) return;
    const double ui = u[q];
    const OpVal r = masked_op(g, mask, w, u, i, j, k, ui, mi, dev::rhs_value(g, src[q]));
    u[q] = ui + bounded(-r.L / r.dL, g.max_step);
}

// ---- fused red-black sweep of a level read as byte flags (n >= 64) ------------------------
// The domain's fused sweep (red cells of plane p, then black cells of plane p-1, in one pass
// over HBM; tiles of TJ x 64 columns and a chunk of planes per workgroup, u and b = exp(u)
// of each plane staged once in LDS, out of place from uin to uout) with the mask scheme of
// km_ngs_colour: a staged masked cell carries b = -1 (b of an active cell is positive), is
// never updated and is copied to uout unchanged; its value, which a masked cell keeps for
// the whole solve, is the w its active neighbours need.  Every update sees the operands of
// the two-colour sweep in the same order (masked_op with mask +1 / -1).  The fixed values w
// are loaded with u, three planes ahead (a load at the update would stall the wavefront).
constexpr int kMK = 64;  // tile width along k

struct ColM {
    double u[4], b[4], f[4], w[4];
    double ru[2], rf[2], rw[2];
    int rm[2];     // raw flags of planes p+2, p+3
    unsigned col;  // (j,k) offset within a plane
    int c, fl;     // LDS cell; 1 loaded, 2 red range (tile + ring), 4 tile
};

// L_i - f and dL_i/du_i of an active cell (mask +1, fixed value wi) with staged neighbours:
// b_nb > 0 active, else masked (mask -1, value = its fixed value w).
__device__ __forceinline__ OpVal masked_op_staged(const Grid& g, double ui, double bi, const double (&un)[6],
                                                  const double (&bn)[6], double f, double wi)
{
    double L = 0.0, dL = 0.0;
#pragma unroll
    for (int v = 0; v < 6; ++v) {
        if (bn[v] > 0.0) {
            const double du = un[v] - ui;
            L = fma(bn[v] + bi, du, L);
            dL += bi * du - bn[v] - bi;
        } else {
            masked_face(1.0, -1.0, un[v], wi, ui, bi, L, dL);
        }
    }
    const double S = dev::curvature(g, ui, bi);
    OpVal o;
    o.L = fma(g.C, L, S) - f;
    o.dL = fma(g.C, dL, -S * g.inv_np1);
    return o;
}

template <int TJ, int NT>
__global__ void __launch_bounds__(NT) km_ngs_fused(Grid g, const u8* __restrict__ flags, const double* __restrict__ w,
                                                   const double* __restrict__ uin, double* __restrict__ uout,
                                                   const double* __restrict__ src, FusedSweep a)
{
    constexpr int LJ = TJ + 4, LK = kMK + 4, NL = LJ * LK, NP = NL / 2;
    static_assert(NP <= NT, "one column pair per thread");
    __shared__ double lu[3][NL];
    __shared__ double lb[3][NL];
    const int nb = gridDim.x;
    int lid = blockIdx.x;
    if ((nb & 7) == 0) lid = (lid & 7) * (nb >> 3) + (lid >> 3);
    const int tk = lid % a.ntk;
    lid /= a.ntk;
    const int tj = lid % a.ntj;
    const int ci = lid / a.ntj;
    const int i0 = ci * a.ti, j0 = tj * TJ, k0 = tk * kMK;
    const int lg = g.lg, m = g.n - 1;
    const int last = i0 + a.ti + 1;  // last plane read

    // X: the column of the thread's pair whose cell on plane i0-1 is red; Y the other
    ColM X{}, Y{};
    const int pc = threadIdx.x;
    if (pc < NP) {
        const int jj = pc / (LK / 2), kk0 = 2 * (pc - jj * (LK / 2));
        const int gj = (j0 - 2 + jj) & m, gk0 = (k0 - 2 + kk0) & m;
        const int sx = (i0 - 1 + gj + gk0) & 1;
        auto setup = [&](ColM& q, int d) {
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
    auto offset = [&](int p, const ColM& q) -> unsigned { return ((unsigned)(p & m) << (2 * lg)) + q.col; };
    auto buf = [&](int p) { return (p - i0 + 3) % 3; };
    auto bval = [](double u, int active) { return active ? exp(u) : -1.0; };
    auto prologue = [&](ColM& q) {
        if (!q.fl) return;
        for (int t = 1; t < 4; ++t) {
            q.u[t] = uin[offset(i0 - 3 + t, q)];
            q.b[t] = bval(q.u[t], flags[offset(i0 - 3 + t, q)]);
            q.f[t] = dev::rhs_value(g, src[offset(i0 - 3 + t, q)]);
            q.w[t] = w[offset(i0 - 3 + t, q)];
        }
        q.ru[1] = uin[offset(i0 + 1, q)];
        q.rm[1] = flags[offset(i0 + 1, q)];
        q.rf[1] = src[offset(i0 + 1, q)];
        q.rw[1] = w[offset(i0 + 1, q)];
        lu[buf(i0 - 1)][q.c] = q.u[2];
        lb[buf(i0 - 1)][q.c] = q.b[2];
    };
    prologue(X);
    prologue(Y);
    __syncthreads();

    const double ms = g.max_step;
    auto step = [&](auto Rc, int p, ColM& A, ColM& B) {
        constexpr int R = decltype(Rc)::value;
        constexpr int M2 = R, M1 = (R + 1) & 3, P0 = (R + 2) & 3, P1 = (R + 3) & 3;
        constexpr int N2 = (R + 1) & 1, N3 = R & 1;
        if (p + 3 <= last) {
            if (A.fl) {
                A.ru[N3] = uin[offset(p + 3, A)];
                A.rm[N3] = flags[offset(p + 3, A)];
                A.rf[N3] = src[offset(p + 3, A)];
                A.rw[N3] = w[offset(p + 3, A)];
            }
            if (B.fl) {
                B.ru[N3] = uin[offset(p + 3, B)];
                B.rm[N3] = flags[offset(p + 3, B)];
                B.rf[N3] = src[offset(p + 3, B)];
                B.rw[N3] = w[offset(p + 3, B)];
            }
        }
        // red cell of plane p (tile + ring), if active
        double* LA = lu[buf(p)];
        double* BA = lb[buf(p)];
        if ((A.fl & 2) && A.b[P0] > 0.0) {
            const int c = A.c;
            const double un[6] = {A.u[M1], A.u[P1], LA[c - LK], LA[c + LK], LA[c - 1], LA[c + 1]};
            const double bn[6] = {A.b[M1], A.b[P1], BA[c - LK], BA[c + LK], BA[c - 1], BA[c + 1]};
            const OpVal r = masked_op_staged(g, A.u[P0], A.b[P0], un, bn, A.f[P0], A.w[P0]);
            const double v = A.u[P0] + bounded(-r.L / r.dL, ms);
            const double bv = exp(v);
            A.u[P0] = v;
            A.b[P0] = bv;
            LA[c] = v;
            BA[c] = bv;
        }
        // black cell of plane p-1 (tile), if active; plane p-1 is then final in both columns
        if (p - 1 >= i0) {
            if (A.fl & 4) {
                if (A.b[M1] > 0.0) {
                    const double* LB = lu[buf(p - 1)];
                    const double* BB = lb[buf(p - 1)];
                    const int c = A.c;
                    const double un[6] = {A.u[M2], A.u[P0], LB[c - LK], LB[c + LK], LB[c - 1], LB[c + 1]};
                    const double bn[6] = {A.b[M2], A.b[P0], BB[c - LK], BB[c + LK], BB[c - 1], BB[c + 1]};
                    const OpVal r = masked_op_staged(g, A.u[M1], A.b[M1], un, bn, A.f[M1], A.w[M1]);
                    A.u[M1] = A.u[M1] + bounded(-r.L / r.dL, ms);
                }
                uout[offset(p - 1, A)] = A.u[M1];
            }
            if (B.fl & 4) uout[offset(p - 1, B)] = B.u[M1];
        }
        double* LC = lu[buf(p + 1)];
        double* BC = lb[buf(p + 1)];
        const bool more2 = p + 2 <= last;
        auto advance = [&](ColM& q) {
            if (q.fl) {
                LC[q.c] = q.u[P1];
                BC[q.c] = q.b[P1];
                if (more2) {
                    q.u[M2] = q.ru[N2];
                    q.b[M2] = bval(q.ru[N2], q.rm[N2]);
                    q.f[M2] = dev::rhs_value(g, q.rf[N2]);
                    q.w[M2] = q.rw[N2];
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
    step(I0{}, i0 - 1, X, Y);
    step(I1{}, i0, Y, X);
    for (int p = i0 + 1; p <= i0 + a.ti; p += 4) {
        step(I2{}, p, X, Y);
        step(I3{}, p + 1, Y, X);
        step(I0{}, p + 2, X, Y);
        step(I1{}, p + 3, Y, X);
    }
}

// One thread per coarse cell: R u of all 8 children and R d of the active ones into active
// coarse cells; masked coarse cells take their fixed value and a zero right-hand side.
template <class M>
__global__ void __launch_bounds__(kB) km_resid_restrict(Grid g, const M* __restrict__ mask,
                                                        const double* __restrict__ w, const double* __restrict__ u,
                                                        const double* __restrict__ src,
                                                        const float* __restrict__ maskc,
                                                        const double* __restrict__ wc, double* __restrict__ uc,
                                                        double* __restrict__ uhat, double* __restrict__ fc)
{
    const int lgc = g.lg - 1, nc = g.n >> 1;
    const long long tc = (long long)blockIdx.x * kB + threadIdx.x;
    if (tc >= (1LL << (3 * lgc))) return;
    if (!(maskc[tc] > 0.0f)) {
        uc[tc] = wc[tc];
        uhat[tc] = wc[tc];
        fc[tc] = 0.0;
        return;
    }
    const int I = (int)(tc >> (2 * lgc)), J = (int)((tc >> lgc) & (nc - 1)), K = (int)(tc & (nc - 1));
    double su = 0.0, sd = 0.0;
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b)
#pragma unroll
            for (int c = 0; c < 2; ++c) {
                const int i = 2 * I + a, j = 2 * J + b, k = 2 * K + c;
                const long long q = at(g, i, j, k);
                const double ui = u[q], mi = mval(mask, q);
                su += ui;
                if (mi > 0.0) sd += masked_op(g, mask, w, u, i, j, k, ui, mi, dev::rhs_value(g, src[q])).L;
            }
    uc[tc] = 0.125 * su;
    uhat[tc] = 0.125 * su;
    fc[tc] = 0.125 * sd;
}

// FAS right-hand side at active coarse cells: f = L^H(R u) - R d.
__global__ void __launch_bounds__(kB) km_fas_rhs(Grid g, const float* __restrict__ mask,
                                                 const double* __restrict__ w, const double* __restrict__ uhat,
                                                 double* __restrict__ f)
{
    const long long q = (long long)blockIdx.x * kB + threadIdx.x;
    if (q >= (1LL << (3 * g.lg))) return;
    const double mi = mask[q];
    if (!(mi > 0.0)) return;
    int i, j, k;
    cell_of(g, q, i, j, k);
    f[q] = masked_op(g, mask, w, uhat, i, j, k, uhat[q], mi, 0.0).L - f[q];
}

// Coarse correction u^H - R u^h at active coarse cells, zero at masked ones (no correction
// comes from a cell that is not a valid multigrid cell), written over uhat.
__global__ void __launch_bounds__(kB) km_coarse_diff(long long n, const float* __restrict__ maskc,
                                                     const double* __restrict__ uc, double* __restrict__ uhat)
{
    const long long q = (long long)blockIdx.x * kB + threadIdx.x;
    if (q >= n) return;
    uhat[q] = maskc[q] > 0.0f ? uc[q] - uhat[q] : 0.0;
}

// Block partials (sum d^2, max |d|) over the active cells.  A thread takes one 2x2x2 block of
// cells, the eight cells unrolled so that their loads overlap; one partial pair per workgroup.
template <class M>
__global__ void __launch_bounds__(kB) km_norm(Grid g, const M* __restrict__ mask,
                                              const double* __restrict__ w, const double* __restrict__ u,
                                              const double* __restrict__ src, double* __restrict__ partial)
{
    __shared__ double sa[kB], sb[kB];
    const int lgc = g.lg - 1, nc = g.n >> 1;
    const long long nblk = 1LL << (3 * lgc);
    double s = 0.0, mx = 0.0;
    const long long t = (long long)blockIdx.x * kB + threadIdx.x;
    if (t < nblk) {
        const int I = (int)(t >> (2 * lgc)), J = (int)((t >> lgc) & (nc - 1)), K = (int)(t & (nc - 1));
#pragma unroll
        for (int x = 0; x < 2; ++x)
#pragma unroll
            for (int y = 0; y < 2; ++y)
#pragma unroll
                for (int z = 0; z < 2; ++z) {
                    const int i = 2 * I + x, j = 2 * J + y, k = 2 * K + z;
                    const long long q = at(g, i, j, k);
                    const double mi = mval(mask, q);
                    if (mi > 0.0) {
                        const double d = masked_op(g, mask, w, u, i, j, k, u[q], mi, dev::rhs_value(g, src[q])).L;
                        s += d * d;
                        const double a = fabs(d);
                        if (!(mx >= a)) mx = a;
                    }
                }
    }
    block_sum_max(s, mx, sa, sb);
    if (threadIdx.x == 0) {
        partial[2 * blockIdx.x] = s;
        partial[2 * blockIdx.x + 1] = mx;
    }
}

// The same partials for a level read as byte flags (n >= 64), streamed: a workgroup owns a
// tile of TJ x 64 columns and a chunk of ti planes; per plane it stages u and b = exp(u) of
// the tile and a one-cell ring in LDS (b = -1 at masked cells, as in km_ngs_fused), keeps the
// i-neighbours in registers and loads the next planes while it evaluates this one, so each
// value and exponential is fetched and formed once.  Sums in a fixed order (a thread's cells
// plane by plane, then a tree over the workgroup); one partial pair per workgroup.
template <int TJ, int NT>
__global__ void __launch_bounds__(NT) km_norm_fused(Grid g, const u8* __restrict__ flags, const double* __restrict__ w,
                                                    const double* __restrict__ u, const double* __restrict__ src,
                                                    double* __restrict__ partial, int ti)
{
    constexpr int LJ = TJ + 2, LK = kMK + 2, NL = LJ * LK;
    static_assert(NL <= NT, "one column per thread");
    __shared__ double lu[NL], lb[NL];
    __shared__ double ra[NT], rb[NT];
    const int ntk = g.n / kMK, ntj = g.n / TJ;
    int lid = blockIdx.x;
    const int tk = lid % ntk;
    lid /= ntk;
    const int tj = lid % ntj;
    const int i0 = (lid / ntj) * ti, j0 = tj * TJ, k0 = tk * kMK;
    const int lg = g.lg, m = g.n - 1;
    const int t = threadIdx.x;
    const bool on = t < NL;
    const int jj = on ? t / LK : 0, kk = on ? t - jj * LK : 0;
    const bool in = on && jj >= 1 && jj <= TJ && kk >= 1 && kk <= kMK;
    const unsigned col = (unsigned)((((j0 - 1 + jj) & m) << lg) | ((k0 - 1 + kk) & m));
    auto off = [&](int p) -> unsigned { return ((unsigned)(p & m) << (2 * lg)) + col; };
    auto bval = [](double v, int a) { return a ? exp(v) : -1.0; };
    double um = 0.0, uc = 0.0, up = 0.0, bm = 0.0, bc = 0.0, bp = 0.0, fc = 0.0, wc = 0.0;
    double ru = 0.0, rf = 0.0, rw = 0.0;
    int rm = 0;
    if (on) {
        um = u[off(i0 - 1)];
        bm = bval(um, flags[off(i0 - 1)]);
        uc = u[off(i0)];
        bc = bval(uc, flags[off(i0)]);
        up = u[off(i0 + 1)];
        bp = bval(up, flags[off(i0 + 1)]);
        if (in) {
            fc = src[off(i0)];
            wc = w[off(i0)];
        }
    }
    double s = 0.0, mx = 0.0;
    for (int p = i0; p < i0 + ti; ++p) {
        // the loads of the next steps: u and flag of plane p+2, rho and w of plane p+1
        if (on && p + 2 <= i0 + ti) {
            ru = u[off(p + 2)];
            rm = flags[off(p + 2)];
        }
        if (in && p + 1 < i0 + ti) {
            rf = src[off(p + 1)];
            rw = w[off(p + 1)];
        }
        if (on) {
            lu[t] = uc;
            lb[t] = bc;
        }
        __syncthreads();
        if (in && bc > 0.0) {
            const double un[6] = {um, up, lu[t - LK], lu[t + LK], lu[t - 1], lu[t + 1]};
            const double bn[6] = {bm, bp, lb[t - LK], lb[t + LK], lb[t - 1], lb[t + 1]};
            const double d = masked_op_staged(g, uc, bc, un, bn, dev::rhs_value(g, fc), wc).L;
            s += d * d;
            const double a = fabs(d);
            if (!(mx >= a)) mx = a;
        }
        __syncthreads();
        um = uc;
        bm = bc;
        uc = up;
        bc = bp;
        up = ru;
        bp = bval(ru, rm);
        fc = rf;
        wc = rw;
    }
    ra[t] = s;
    rb[t] = mx;
    __syncthreads();
    for (int h = 512; h > 0; h >>= 1) {
        if (t < h && t + h < NT) {
            ra[t] += ra[t + h];
            const double o = rb[t + h];
            if (!(rb[t] >= o)) rb[t] = o;
        }
        __syncthreads();
    }
    if (t == 0) {
        partial[2 * blockIdx.x] = ra[0];
        partial[2 * blockIdx.x + 1] = rb[0];
    }
}

// Block partials (number of active cells, max |mask|; NaN propagates).
__global__ void __launch_bounds__(kB) km_count(const float* __restrict__ mask, long long n,
                                               double* __restrict__ partial)
{
    __shared__ double sa[kB], sb[kB];
    double s = 0.0, mx = 0.0;
    for (long long q = (long long)blockIdx.x * kB + threadIdx.x; q < n; q += (long long)gridDim.x * kB) {
        const float m = mask[q];
        if (m > 0.0f) s += 1.0;
        const double a = fabs((double)m);
        if (!(mx >= a)) mx = a;
    }
    block_sum_max(s, mx, sa, sb);
    if (threadIdx.x == 0) {
        partial[2 * blockIdx.x] = s;
        partial[2 * blockIdx.x + 1] = mx;
    }
}

// Byte flags of a mask (1 where > 0) and block partials of the number of cells whose mask is
// neither +1 nor -1 (the flags stand for the mask only when there is none).
__global__ void __launch_bounds__(kB) km_flags(const float* __restrict__ mask, long long n, u8* __restrict__ flags,
                                               double* __restrict__ partial)
{
    __shared__ double sa[kB], sb[kB];
    double s = 0.0, mx = 0.0;
    for (long long q = (long long)blockIdx.x * kB + threadIdx.x; q < n; q += (long long)gridDim.x * kB) {
        const float m = mask[q];
        flags[q] = m > 0.0f ? 1 : 0;
        if (m != 1.0f && m != -1.0f) s += 1.0;
    }
    block_sum_max(s, mx, sa, sb);
    if (threadIdx.x == 0) {
        partial[2 * blockIdx.x] = s;
        partial[2 * blockIdx.x + 1] = mx;
    }
}

// Coarse mask and fixed values: 8-child means.
__global__ void __launch_bounds__(kB) km_restrict_setup(int lgc, const float* __restrict__ maskf,
                                                        const double* __restrict__ wf, float* __restrict__ maskc,
                                                        double* __restrict__ wc)
{
    const int lg = lgc + 1, nc = 1 << lgc;
    const long long tc = (long long)blockIdx.x * kB + threadIdx.x;
    if (tc >= (1LL << (3 * lgc))) return;
    const int I = (int)(tc >> (2 * lgc)), J = (int)((tc >> lgc) & (nc - 1)), K = (int)(tc & (nc - 1));
    double sm = 0.0, sw = 0.0;
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b)
#pragma unroll
            for (int c = 0; c < 2; ++c) {
                const long long q = ((((long long)(2 * I + a) << lg) + 2 * J + b) << lg) + 2 * K + c;
                sm += maskf[q];
                sw += wf[q];
            }
    maskc[tc] = (float)(0.125 * sm);
    wc[tc] = 0.125 * sw;
}

// Coarsest level (n <= 8) in one workgroup, through LDS: relax the active cells until the rms
// residual over them is <= rtol x its initial value or its rounding floor, or cap sweeps.
__global__ void __launch_bounds__(kB) km_coarsest(Grid g, const float* __restrict__ mask,
                                                  const double* __restrict__ w, double* __restrict__ u,
                                                  const double* __restrict__ f, int cap, double rtol,
                                                  long long* __restrict__ sweeps_done)
{
    __shared__ double su[512], sw[512], sf[512];
    __shared__ float sm[512];
    __shared__ double sa[kB], sb[kB];
    const int nc = 1 << (3 * g.lg);
    for (int q = threadIdx.x; q < nc; q += kB) {
        su[q] = u[q];
        sw[q] = w[q];
        sf[q] = dev::rhs_value(g, f[q]);
        sm[q] = mask[q];
    }
    __syncthreads();
    // rms residual over the active cells, and its rounding floor: per cell one unit in the
    // last place of u times |dL/du| plus one of the summed magnitudes of the terms
    __shared__ double sc[kB];
    auto rms = [&](double& floor) {
        double s = 0.0, fl = 0.0, cnt = 0.0;
        for (int q = threadIdx.x; q < nc; q += kB) {
            const double mi = sm[q];
            if (!(mi > 0.0)) continue;
            int i, j, k;
            cell_of(g, q, i, j, k);
            const OpVal r = masked_op(g, sm, sw, su, i, j, k, su[q], mi, sf[q]);
            s += r.L * r.L;
            const double f1 = 2.220446049250313e-16 *
                              (fabs(r.dL) * fabs(su[q]) + masked_mag(g, sm, sw, su, i, j, k, su[q], mi, sf[q]));
            fl += f1 * f1;
            cnt += 1.0;
        }
        block_sum2(s, fl, sa, sb);
        sc[threadIdx.x] = cnt;
        __syncthreads();
        for (int w2 = kB / 2; w2 > 0; w2 >>= 1) {
            if (threadIdx.x < w2) sc[threadIdx.x] += sc[threadIdx.x + w2];
            __syncthreads();
        }
        cnt = sc[0];
        __syncthreads();
        floor = cnt > 0.0 ? sqrt(fl / cnt) : 0.0;
        return cnt > 0.0 ? sqrt(s / cnt) : 0.0;
    };
    double floor0 = 0.0;
    const double r0 = rtol > 0.0 ? rms(floor0) : 0.0;
    int sweep = 0;
    for (; sweep < cap; ++sweep) {
        if (rtol > 0.0) {
            // stop once reduced by rtol or down to the rounding floor
            double floor;
            const double r = rms(floor);
            if (r <= rtol * r0 || r <= floor) break;
        }
        for (int colour = 0; colour < 2; ++colour) {
            for (int q = threadIdx.x; q < nc; q += kB) {
                const double mi = sm[q];
                int i, j, k;
                cell_of(g, q, i, j, k);
                if (((i + j + k) & 1) != colour || !(mi > 0.0)) continue;
                const double ui = su[q];
                const OpVal r = masked_op(g, sm, sw, su, i, j, k, ui, mi, sf[q]);
                su[q] = ui + bounded(-r.L / r.dL, g.max_step);
            }
            __syncthreads();
        }
    }
    for (int q = threadIdx.x; q < nc; q += kB) u[q] = su[q];
    if (threadIdx.x == 0 && sweeps_done) sweeps_done[0] += sweep;
}

inline unsigned blocks(long long work) { return (unsigned)((work + kB - 1) / kB); }

inline unsigned rblocks(long long work)
{
    const long long b = (work + kB - 1) / kB;
    return (unsigned)(b < kMaxParts ? (b < 1 ? 1 : b) : kMaxParts);
}

}  // namespace

hipError_t masked_count(const float* mask, long long n, double* partial, int* nparts, hipStream_t s)
{
    const unsigned nb = rblocks(n);
    hipLaunchKernelGGL(km_count, dim3(nb), dim3(kB), 0, s, mask, n, partial);
    *nparts = (int)nb;
    return hipGetLastError();
}

hipError_t masked_restrict_setup(const Grid& gc, const float* maskf, const double* wf, float* maskc, double* wc,
                                 hipStream_t s)
{
    hipLaunchKernelGGL(km_restrict_setup, dim3(blocks(cells(gc))), dim3(kB), 0, s, gc.lg, maskf, wf, maskc, wc);
    return hipGetLastError();
}

hipError_t masked_flags(const float* mask, long long n, unsigned char* flags, double* partial, int* nparts,
                        hipStream_t s)
{
    const unsigned nb = rblocks(n);
    hipLaunchKernelGGL(km_flags, dim3(nb), dim3(kB), 0, s, mask, n, flags, partial);
    *nparts = (int)nb;
    return hipGetLastError();
}

template <class M>
hipError_t ngs_t(const Grid& g, const M* mask, const double* w, double* u, const double* src, hipStream_t s)
{
    if (g.n < 2) return hipErrorInvalidValue;
    const long long half = cells(g) / 2;
    for (int colour = 0; colour < 2; ++colour) {
        hipLaunchKernelGGL(km_ngs_colour<M>, dim3(blocks(half)), dim3(kB), 0, s, g, mask, w, u, src, colour);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

hipError_t masked_ngs(const Grid& g, const float* mask, const double* w, double* u, const double* src, hipStream_t s)
{
    return ngs_t(g, mask, w, u, src, s);
}

hipError_t masked_ngs(const Grid& g, const unsigned char* flags, const double* w, double* u, const double* src,
                      hipStream_t s)
{
    return ngs_t(g, flags, w, u, src, s);
}

hipError_t masked_ngs_fused(const Grid& g, const unsigned char* flags, const double* w, const double* uin,
                            double* uout, const double* src, int ti, hipStream_t s)
{
    if (g.n < kMK || g.n > 1024 || uin == uout || ti < 4 || (ti & 3) || ti > g.n || (g.n % ti) != 0)
        return hipErrorInvalidValue;
    constexpr int TJ = 16, NT = 704;  // 680 column pairs per 20 x 68 tile
    FusedSweep a{};
    a.ti = ti;
    a.ntj = g.n / TJ;
    a.ntk = g.n / kMK;
    const unsigned nb = (unsigned)((g.n / ti) * a.ntj * a.ntk);
    hipLaunchKernelGGL((km_ngs_fused<TJ, NT>), dim3(nb), dim3(NT), 0, s, g, flags, w, uin, uout, src, a);
    return hipGetLastError();
}

template <class M>
hipError_t resid_restrict_t(const Grid& g, const M* mask, const double* w, const double* u, const double* src,
                            const float* maskc, const double* wc, double* uc, double* uhat, double* fc, hipStream_t s)
{
    if (g.n < 2) return hipErrorInvalidValue;
    hipLaunchKernelGGL(km_resid_restrict<M>, dim3(blocks(cells(g) / 8)), dim3(kB), 0, s, g, mask, w, u, src, maskc,
                       wc, uc, uhat, fc);
    return hipGetLastError();
}

hipError_t masked_resid_restrict(const Grid& g, const float* mask, const double* w, const double* u,
                                 const double* src, const float* maskc, const double* wc, double* uc, double* uhat,
                                 double* fc, hipStream_t s)
{
    return resid_restrict_t(g, mask, w, u, src, maskc, wc, uc, uhat, fc, s);
}

hipError_t masked_resid_restrict(const Grid& g, const unsigned char* flags, const double* w, const double* u,
                                 const double* src, const float* maskc, const double* wc, double* uc, double* uhat,
                                 double* fc, hipStream_t s)
{
    return resid_restrict_t(g, flags, w, u, src, maskc, wc, uc, uhat, fc, s);
}

hipError_t masked_fas_rhs(const Grid& gc, const float* maskc, const double* wc, const double* uhat, double* f,
                          hipStream_t s)
{
    hipLaunchKernelGGL(km_fas_rhs, dim3(blocks(cells(gc))), dim3(kB), 0, s, gc, maskc, wc, uhat, f);
    return hipGetLastError();
}

hipError_t masked_prolong(const Grid& gc, const float* maskc, const double* uc, double* uhat, const float* maskf,
                          double* uf, hipStream_t s)
{
    // the correction, then the streaming 27/9/3/1 prolongation into the active fine cells
    hipLaunchKernelGGL(km_coarse_diff, dim3(blocks(cells(gc))), dim3(kB), 0, s, cells(gc), maskc, uc, uhat);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    return prolong_add_masked(gc, uf, uhat, maskf, s);
}

long long masked_norm_partials(const Grid& g) { return (long long)blocks(cells(g) / 8); }

template <class M>
hipError_t norm_t(const Grid& g, const M* mask, const double* w, const double* u, const double* src, double* partial,
                  int* nparts, hipStream_t s)
{
    if (g.n < 2) return hipErrorInvalidValue;
    const unsigned nb = blocks(cells(g) / 8);
    hipLaunchKernelGGL(km_norm<M>, dim3(nb), dim3(kB), 0, s, g, mask, w, u, src, partial);
    *nparts = (int)nb;
    return hipGetLastError();
}

hipError_t masked_norm(const Grid& g, const float* mask, const double* w, const double* u, const double* src,
                       double* partial, int* nparts, hipStream_t s)
{
    return norm_t(g, mask, w, u, src, partial, nparts, s);
}

hipError_t masked_norm(const Grid& g, const unsigned char* flags, const double* w, const double* u,
                       const double* src, double* partial, int* nparts, hipStream_t s)
{
    if (g.n < kMK) return norm_t(g, flags, w, u, src, partial, nparts, s);
    // streamed: 8 x 64 column tiles, chunks of 64 planes (at most n)
    constexpr int TJ = 8, NT = 704;
    const int ti = g.n < 64 ? g.n : 64;
    const unsigned nb = (unsigned)((g.n / ti) * (g.n / TJ) * (g.n / kMK));
    if ((long long)nb > masked_norm_partials(g)) return hipErrorInvalidValue;
    hipLaunchKernelGGL((km_norm_fused<TJ, NT>), dim3(nb), dim3(NT), 0, s, g, flags, w, u, src, partial, ti);
    *nparts = (int)nb;
    return hipGetLastError();
}

hipError_t masked_coarsest(const Grid& g, const float* mask, const double* w, double* u, const double* f, int cap,
                           double rtol, long long* sweeps, hipStream_t s)
{
    if (cells(g) > 512) return hipErrorInvalidValue;
    hipLaunchKernelGGL(km_coarsest, dim3(1), dim3(kB), 0, s, g, mask, w, u, f, cap, rtol, sweeps);
    return hipGetLastError();
}

}  // namespace mgfr
