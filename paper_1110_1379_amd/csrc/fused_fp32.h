// The fused red-black sweep of the single-precision correction equation N(e) = r over one
// tile column of a unit grid: the periodic domain grid, a periodic box of a batched solve, or
// a refinement patch of one (cube with ghost faces outside, batch_dev.h).  Planes are
// streamed through three LDS plane buffers, one barrier per plane, and the red ring around
// the tile is recomputed by every tile that sees it.
//
// The work is laid out so that lanes hold only cells that need updating.  Thread t owns the
// pair of k-adjacent tile columns t (TJ x TK tile, TJ TK / 2 threads): at every step it
// updates one red cell on plane p and one black cell on plane p-1, every one of them part of
// the result.  The ring of red cells around the tile (recomputed from the same old values by
// every tile that sees them) and the outer halo (only read) are extra columns E of the first
// threads: thread t < NR holds ring cell t, which it updates on the planes where that cell is
// red; the next NH threads hold one halo cell each, which they only stage.  Every updated
// cell's (B, M) are formed again from (ub, e) as the per-colour kernel forms them, so both
// sweeps give the same bits.
//
// On a patch, a position outside the patch next to a cell inside it (across one face) holds
// that face's boundary value u_b in the ub field of its V32, for the ghost term of the
// inside cell (batch_dev.h); positions outside are never relaxed, and other positions
// outside (the patch's edges and corners) are never read.
#pragma once

#include "device_fp32.h"

#include <type_traits>

namespace mgfr {
namespace fused32 {

using dev32::em1f;
using dev32::make_v;
using dev32::newton32;
using dev32::Res32;
using dev32::Op32;
using dev32::V32;

// Mask ratio m_ghost / m_i of a ghost cell next to a cell of a cube patch (every cell of the
// patch is active), as in the per-cell kernels.
constexpr float kGhostR = -1.0f;

// One column of a thread: the values of planes p-2 .. p+1 and the loads in flight.
struct Col32 {
    V32 v[4];                 // plane q in v[(q - i0 + 3) & 3]: planes p-2 .. p+1 at step p
    float f[4];               // right-hand side, same slots (planes p-1 .. p+1 used)
    float rub[2], re[2], rf[2];  // raw loads of planes p+2 and p+3, plane q in [(q - i0) & 1]
    unsigned col;             // (j,k) offset within a plane
    int c, fl;                // LDS cell; 1 loaded, 2 red range (tile + ring), 4 tile
};

// A column of a patch tile: also its position, whether it lies inside the patch, and for a
// column outside it across one face, that face's boundary values at plane 0 (index of the
// [6][n][n] array; plane p adds p n).
struct ColP : Col32 {
    int j, k, fq;
    bool in;
};

// N_i - f_i and dN_i/de_i of a patch cell with the ghost faces of the neighbours flagged out
// (their ub field holds u_b): the arithmetic of the per-cell kernel (bcell32), in the same
// order.
__device__ __forceinline__ Res32 corr_op_patch(const Op32& o, const V32& c, const V32 (&nb)[6], const bool (&out)[6],
                                               float f)
{
    float t1 = 0.0f, t2 = 0.0f, su = 0.0f, se = 0.0f, sB = 0.0f, nreg = 0.0f, lgh = 0.0f, dgh = 0.0f;
#pragma unroll
    for (int x = 0; x < 6; ++x) {
        if (out[x]) {
            const float ubg = (1.0f - kGhostR) * nb[x].ub + kGhostR * c.ub;
            const float eg = kGhostR * c.e;
            const float bg = __expf(ubg);
            const float Mg = bg * em1f(eg), Bg = bg + Mg;
            const float du = ubg - c.ub, de = eg - c.e;
            lgh += (Mg + c.M) * du + (Bg + c.B) * de;
            dgh += (kGhostR * Bg + c.B) * (du + de) + (Bg + c.B) * (kGhostR - 1.0f);
        } else {
            const float du = nb[x].ub - c.ub, de = nb[x].e - c.e;
            t1 = fmaf(nb[x].M, du, t1);
            t2 = fmaf(nb[x].B, de, t2);
            su += du;
            se += de;
            sB += nb[x].B;
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

// Sweeps the TJ x TK tile at (j0, k0) for planes i0 .. i0 + ti - 1 of a grid of side n = 2^lg
// (ti a multiple of 4), reading ein and writing eout (never the same array): every thread of
// the TJ TK / 2 of the workgroup calls it, with lv its workgroup's LDS.  PATCH: the grid is a
// patch whose boundary values are faces ([6][n][n], batch_dev.h); otherwise it is periodic.
// ADDU: the sweep is the last of a correction solve; instead of writing e it adds it to the
// double-precision field, uadd += e (each cell of the tile once, after its black update).
template <int TJ, int TK, bool PATCH = false, bool ADDU = false>
__device__ __forceinline__ void sweep_tile(const Op32& o, int n, int lg, int i0, int j0, int k0, int ti,
                                           const float* __restrict__ ub, const float* __restrict__ ein,
                                           float* __restrict__ eout, const float* __restrict__ f,
                                           V32 (*lv)[(TJ + 4) * (TK + 4)], const double* __restrict__ faces = nullptr,
                                           double* __restrict__ uadd = nullptr)
{
    constexpr int NT = TJ * TK / 2;
    constexpr int LK = TK + 4;
    constexpr int NR = 2 * (TK + 2) + 2 * TJ;        // ring around the tile
    constexpr int NH = 2 * (TK + 4) + 2 * (TJ + 2);  // outer halo
    static_assert(NR + NH <= NT, "one extra column per thread");
    using Col = typename std::conditional<PATCH, ColP, Col32>::type;
    const int m = n - 1;
    const int last = i0 + ti + 1;  // last plane read
    const int t = threadIdx.x;

    // X: the tile column of the pair whose cell on plane i0-1 is red; Y: the other one
    Col X{}, Y{}, E{};
    {
        const int jj = t / (TK / 2), kk0 = 2 * (t - jj * (TK / 2));
        const int gj = (j0 + jj) & m, gk0 = (k0 + kk0) & m;
        const int sx = (i0 - 1 + gj + gk0) & 1;
        auto setup = [&](Col& q, int d) {
            q.col = (unsigned)((gj << lg) | (gk0 + d));
            q.c = (jj + 2) * LK + kk0 + 2 + d;
            q.fl = 7;
            if constexpr (PATCH) {
                q.j = gj;
                q.k = gk0 + d;
                q.in = true;
                q.fq = 0;
            }
        };
        setup(X, sx);
        setup(Y, 1 - sx);
    }
    // E: ring cell t or halo cell t - NR, walked around its rectangle (rows first, then the
    // two side columns)
    int epar = 0;  // parity of (j + k) of E's column
    if (t < NR + NH) {
        const bool ring = t < NR;
        const int r = ring ? t : t - NR;
        const int ra = ring ? TJ + 2 : TJ + 4, rb = ring ? TK + 2 : TK + 4, off = ring ? 1 : 0;
        int ej, ek;
        if (r < rb) { ej = 0; ek = r; }
        else if (r < 2 * rb) { ej = ra - 1; ek = r - rb; }
        else if (r < 2 * rb + ra - 2) { ej = 1 + (r - 2 * rb); ek = 0; }
        else { ej = 1 + (r - 2 * rb - (ra - 2)); ek = rb - 1; }
        ej += off;
        ek += off;
        const int gj = (j0 - 2 + ej) & m, gk = (k0 - 2 + ek) & m;
        E.col = (unsigned)((gj << lg) | gk);
        E.c = ej * LK + ek;
        E.fl = ring ? 3 : 1;
        epar = (gj + gk) & 1;
        if constexpr (PATCH) {
            E.j = j0 - 2 + ej;
            E.k = k0 - 2 + ek;
            const bool jo = E.j < 0 || E.j > m, ko = E.k < 0 || E.k > m;
            E.in = !jo && !ko;
            // outside across one face: face 2 / 3 (index (i, k)) or 4 / 5 (index (i, j))
            const int fc = jo ? (E.j < 0 ? 2 : 3) : (E.k < 0 ? 4 : 5);
            E.fq = (jo != ko) ? (fc << (2 * lg)) + (jo ? E.k : E.j) : -1;
        }
    }
    // element offsets fit in 32 bits (n <= 1024)
    auto offset = [&](int p, const Col& q) -> unsigned { return ((unsigned)(p & m) << (2 * lg)) + q.col; };
    auto buf = [&](int p) { return (p - i0 + 3) % 3; };
    // On a patch, whether column q holds a boundary value on plane p: outside the patch across
    // a j or k face on planes inside it, or inside it in (j, k) on the planes -1 and n.
    auto holds_face = [&](int p, const Col& q) -> bool {
        if constexpr (PATCH) return (p >= 0 && p <= m) ? (!q.in && q.fq >= 0) : q.in;
        else return false;
    };
    // Raw values of column q on plane p.  A boundary value is loaded as the two halves of its
    // double through the same pair of loads, so that no branch waits on a load; cells outside
    // the patch that hold nothing load a wrapped cell in vain.
    auto load_raw = [&](int p, const Col& q, float& rub, float& re) {
        if constexpr (PATCH) {
            const bool fc = holds_face(p, q);
            const int fi = (p >= 0 && p <= m) ? q.fq + (p << lg) : ((p < 0 ? 0 : 1) << (2 * lg)) + (int)q.col;
            const float* px = fc ? (const float*)(faces + (fc ? fi : 0)) : ub + offset(p, q);
            const float* py = fc ? px + 1 : ein + offset(p, q);
            rub = *px;
            re = *py;
        } else {
            rub = ub[offset(p, q)];
            re = ein[offset(p, q)];
        }
    };
    auto make = [&](int p, const Col& q, float rub, float re) -> V32 {
        if constexpr (PATCH) {
            const unsigned long long bits = ((unsigned long long)__builtin_bit_cast(unsigned, re) << 32) |
                                            __builtin_bit_cast(unsigned, rub);
            const float fv = (float)__builtin_bit_cast(double, bits);
            if (holds_face(p, q)) return V32{fv, 0.0f, 0.0f, 0.0f};
        }
        return make_v(rub, re);
    };
    auto prologue = [&](Col& q) {
        if (!q.fl) return;
        // planes i0-2, i0-1, i0 in slots 1, 2, 3; plane i0+1 raw in slot 1
        float a, b;
        load_raw(i0 - 2, q, a, b);
        q.v[1] = make(i0 - 2, q, a, b);
        load_raw(i0 - 1, q, a, b);
        q.v[2] = make(i0 - 1, q, a, b);
        load_raw(i0, q, a, b);
        q.v[3] = make(i0, q, a, b);
        load_raw(i0 + 1, q, q.rub[1], q.re[1]);
        if (q.fl & 2) {
            q.f[1] = f[offset(i0 - 2, q)];
            q.f[2] = f[offset(i0 - 1, q)];
            q.f[3] = f[offset(i0, q)];
            q.rf[1] = f[offset(i0 + 1, q)];
        }
        lv[buf(i0 - 1)][q.c] = q.v[2];
    };
    prologue(X);
    prologue(Y);
    prologue(E);
    __syncthreads();

    // the faces of cell (p, q) that lie on the patch boundary
    auto outs = [&](int p, const Col& q, bool (&out)[6]) {
        if constexpr (PATCH) {
            out[0] = p == 0;
            out[1] = p == m;
            out[2] = q.j == 0;
            out[3] = q.j == m;
            out[4] = q.k == 0;
            out[5] = q.k == m;
        }
    };
    auto op = [&](int p, const Col& q, const V32& c, const V32 (&nbv)[6], float fr) -> Res32 {
        if constexpr (PATCH) {
            bool out[6];
            outs(p, q, out);
            return corr_op_patch(o, c, nbv, out, fr);
        } else {
            return dev32::corr_op(o, c, nbv, fr);
        }
    };

    // One plane step, R = (p - i0 + 1) mod 4 fixed at compile time so that the register planes
    // rotate by renaming.  A holds the red cell of plane p and the black cell of plane p-1.
    auto step = [&](auto Rc, int p, Col& A, Col& B) {
        constexpr int R = decltype(Rc)::value;
        constexpr int M2 = R, M1 = (R + 1) & 3, P0 = (R + 2) & 3, P1 = (R + 3) & 3;
        constexpr int N2 = (R + 1) & 1, N3 = R & 1;  // raw slots of planes p+2, p+3
        auto fetch = [&](Col& q) {
            if (!q.fl) return;
            load_raw(p + 3, q, q.rub[N3], q.re[N3]);
            if (q.fl & 2) q.rf[N3] = f[offset(p + 3, q)];
        };
        if (p + 3 <= last) {
            fetch(A);
            fetch(B);
            fetch(E);
        }
        // ADDU: the field of this step's two output cells, loaded before the updates
        double ua = 0.0, ubv = 0.0;
        if constexpr (ADDU) {
            if (p - 1 >= i0) {
                ua = uadd[offset(p - 1, A)];
                ubv = uadd[offset(p - 1, B)];
            }
        }
        V32* LA = lv[buf(p)];
        const bool pin = !PATCH || (p >= 0 && p <= m);  // a patch's planes -1 and n are not relaxed
        auto red = [&](Col& q) {
            const int c = q.c;
            const V32 nbv[6] = {q.v[M1], q.v[P1], LA[c - LK], LA[c + LK], LA[c - 1], LA[c + 1]};
            const Res32 r = op(p, q, q.v[P0], nbv, q.f[P0]);
            q.v[P0] = make_v(q.v[P0].ub, q.v[P0].e + newton32(r, o.max_step));
            LA[c] = q.v[P0];
        };
        if (pin) red(A);
        bool ered = (E.fl & 2) && ((p + epar) & 1) == 0;
        if constexpr (PATCH) ered = ered && pin && E.in;
        if (ered) red(E);
        if (p - 1 >= i0) {
            const V32* LB = lv[buf(p - 1)];
            const int c = A.c;
            const V32 nbv[6] = {A.v[M2], A.v[P0], LB[c - LK], LB[c + LK], LB[c - 1], LB[c + 1]};
            const Res32 r = op(p - 1, A, A.v[M1], nbv, A.f[M1]);
            A.v[M1].e = A.v[M1].e + newton32(r, o.max_step);
            if constexpr (ADDU) {
                uadd[offset(p - 1, A)] = ua + (double)A.v[M1].e;
                uadd[offset(p - 1, B)] = ubv + (double)B.v[M1].e;
            } else {
                eout[offset(p - 1, A)] = A.v[M1].e;
                eout[offset(p - 1, B)] = B.v[M1].e;
            }
        }
        V32* LC = lv[buf(p + 1)];
        const bool more2 = p + 2 <= last;
        auto advance = [&](Col& q) {
            if (!q.fl) return;
            LC[q.c] = q.v[P1];
            if (more2) {  // plane p+2 takes the slot of plane p-2
                q.v[M2] = make(p + 2, q, q.rub[N2], q.re[N2]);
                q.f[M2] = q.rf[N2];
            }
        };
        advance(A);
        advance(B);
        advance(E);
        __syncthreads();
    };
    using I0 = std::integral_constant<int, 0>;
    using I1 = std::integral_constant<int, 1>;
    using I2 = std::integral_constant<int, 2>;
    using I3 = std::integral_constant<int, 3>;
    // ti + 2 steps (ti a multiple of 4): two, then groups of four so that the register
    // planes and the column roles are back in place at the end of every iteration.  X holds
    // the red cells of planes i0-1, i0+1, ...
    step(I0{}, i0 - 1, X, Y);
    step(I1{}, i0, Y, X);
    for (int p = i0 + 1; p <= i0 + ti; p += 4) {
        step(I2{}, p, X, Y);
        step(I3{}, p + 1, Y, X);
        step(I0{}, p + 2, X, Y);
        step(I1{}, p + 3, Y, X);
    }
}

}  // namespace fused32
}  // namespace mgfr
