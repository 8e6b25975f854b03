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

#include <type_traits>

namespace mgfr {
namespace {

using dev::OpVal;

constexpr int kTK = 64;  // tile width along k (contiguous)

// State of one column of a thread's pair.  Plane q of u and b = exp(u) sits in slot
// (q - i0 + 3) & 3 (planes p-2 .. p+1 at step p), its right-hand side in the same slot
// (planes p-1 .. p+1 used), and the raw loads of planes p+2 and p+3 in slot (q - i0) & 1.
struct Col64 {
    double u[4], b[4], f[4];
    double ru[2], rf[2];
    unsigned col;  // (j,k) offset within a plane
    int c, fl;     // LDS cell; 1 loaded, 2 red range (tile + ring), 4 tile
};

template <int TJ, int NT>
__global__ void __launch_bounds__(NT) k_ngs_fused(Grid g, const double* __restrict__ uin,
                                                  double* __restrict__ uout,
                                                  const double* __restrict__ src, FusedSweep a)
{
    if (g.halt && *g.halt) return;
    constexpr int LJ = TJ + 4, LK = kTK + 4, NL = LJ * LK, NP = NL / 2;
    static_assert(NP <= NT, "one column pair per thread");
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

    // A thread owns the k-adjacent columns (kk0, kk0+1) of one tile row.  At step p the
    // column whose cell on plane p is red does both updates of the step (red on plane p,
    // black on plane p-1, the same column); the other column's cells there are black on p
    // and red on p-1, so it has nothing to do until the next step.  X is the column with
    // the red cell on plane i0-1, Y the other; as the roles alternate, every lane updates
    // at every step.
    Col64 X{}, Y{};
    const int pc = threadIdx.x;
    if (pc < NP) {
        const int jj = pc / (LK / 2), kk0 = 2 * (pc - jj * (LK / 2));
        const int gj = (j0 - 2 + jj) & m, gk0 = (k0 - 2 + kk0) & m;
        const int sx = (i0 - 1 + gj + gk0) & 1;
        auto setup = [&](Col64& q, int d) {
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
    auto offset = [&](int p, const Col64& q) -> unsigned { return ((unsigned)(p & m) << (2 * lg)) + q.col; };
    auto buf = [&](int p) { return (p - i0 + 3) % 3; };
    auto prologue = [&](Col64& q) {
        if (!q.fl) return;
        // planes i0-2, i0-1, i0 in slots 1, 2, 3; plane i0+1 raw in slot 1
        for (int t = 1; t < 4; ++t) {
            q.u[t] = uin[offset(i0 - 3 + t, q)];
            q.f[t] = dev::rhs_value(g, src[offset(i0 - 3 + t, q)]);
        }
        q.ru[1] = uin[offset(i0 + 1, q)];
        q.rf[1] = src[offset(i0 + 1, q)];  // raw: transformed when it becomes plane p+1
        for (int t = 1; t < 4; ++t) q.b[t] = exp(q.u[t]);
        lu[buf(i0 - 1)][q.c] = q.u[2];
        lb[buf(i0 - 1)][q.c] = q.b[2];
    };
    prologue(X);
    prologue(Y);
    __syncthreads();

    const double ms = g.max_step;
    // One plane step, R = (p - i0 + 1) mod 4 fixed at compile time so that the register
    // planes rotate by renaming.  A holds the red cell of plane p and the black cell of
    // plane p-1.
    auto step = [&](auto Rc, int p, Col64& A, Col64& B) {
        constexpr int R = decltype(Rc)::value;
        constexpr int M2 = R, M1 = (R + 1) & 3, P0 = (R + 2) & 3, P1 = (R + 3) & 3;
        constexpr int N2 = (R + 1) & 1, N3 = R & 1;  // raw slots of planes p+2, p+3
        // issue the loads of plane p+3 two steps ahead of their use
        if (p + 3 <= last) {
            if (A.fl) {
                A.ru[N3] = uin[offset(p + 3, A)];
                A.rf[N3] = src[offset(p + 3, A)];
            }
            if (B.fl) {
                B.ru[N3] = uin[offset(p + 3, B)];
                B.rf[N3] = src[offset(p + 3, B)];
            }
        }
        // red cell of plane p (tile + ring); its black neighbours are all old
        double* LA = lu[buf(p)];
        double* BA = lb[buf(p)];
        if (A.fl & 2) {
            const int c = A.c;
            const double un[6] = {A.u[M1], A.u[P1], LA[c - LK], LA[c + LK], LA[c - 1], LA[c + 1]};
            const double bn[6] = {A.b[M1], A.b[P1], BA[c - LK], BA[c + LK], BA[c - 1], BA[c + 1]};
            const OpVal r = dev::cell_op_b(g, A.u[P0], A.b[P0], un, bn, A.f[P0]);
            const double v = A.u[P0] + dev::bounded(-r.L / r.dL, ms);
            const double bv = exp(v);
            A.u[P0] = v;
            A.b[P0] = bv;
            LA[c] = v;
            BA[c] = bv;
        }
        // black cell of plane p-1 (tile); its red neighbours are all new.  Plane p-1 is then
        // final in both columns.
        if (p - 1 >= i0) {
            if (A.fl & 4) {
                const double* LB = lu[buf(p - 1)];
                const double* BB = lb[buf(p - 1)];
                const int c = A.c;
                const double un[6] = {A.u[M2], A.u[P0], LB[c - LK], LB[c + LK], LB[c - 1], LB[c + 1]};
                const double bn[6] = {A.b[M2], A.b[P0], BB[c - LK], BB[c + LK], BB[c - 1], BB[c + 1]};
                const OpVal r = dev::cell_op_b(g, A.u[M1], A.b[M1], un, bn, A.f[M1]);
                A.u[M1] = A.u[M1] + dev::bounded(-r.L / r.dL, ms);
                uout[offset(p - 1, A)] = A.u[M1];
            }
            if (B.fl & 4) uout[offset(p - 1, B)] = B.u[M1];
        }
        // stage plane p+1 for the next step; plane p+2 takes the slot of plane p-2
        double* LC = lu[buf(p + 1)];
        double* BC = lb[buf(p + 1)];
        const bool more2 = p + 2 <= last;
        auto advance = [&](Col64& q) {
            if (q.fl) {
                LC[q.c] = q.u[P1];
                BC[q.c] = q.b[P1];
                if (more2) {
                    q.u[M2] = q.ru[N2];
                    q.b[M2] = exp(q.ru[N2]);
                    q.f[M2] = dev::rhs_value(g, q.rf[N2]);
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
    // planes and the column roles are back in place at the end of every iteration
    step(I0{}, i0 - 1, X, Y);
    step(I1{}, i0, Y, X);
    for (int p = i0 + 1; p <= i0 + a.ti; p += 4) {
        step(I2{}, p, X, Y);
        step(I3{}, p + 1, Y, X);
        step(I0{}, p + 2, X, Y);
        step(I1{}, p + 3, Y, X);
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

hipError_t ngs_sweep_fused(const Grid& g, const double* uin, double* uout, const double* src, int ti, int tile,
                           hipStream_t s)
{
    if (g.n < kTK || g.n > 1024 || uin == uout || ti < 4 || (ti & 3) || ti > g.n || (g.n % ti) != 0)
        return hipErrorInvalidValue;
    FusedSweep a{};
    a.ti = ti;
    if (tile == kTile64x8x64) return launch<8, 448>(g, uin, uout, src, a, s);  // 408 column pairs per 12 x 68
    return launch<16, 704>(g, uin, uout, src, a, s);  // 680 column pairs per 20 x 68 tile
}

}  // namespace mgfr
