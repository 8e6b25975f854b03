// Batched red-black sweeps of units of side >= 32, one colour per launch, column-walking:
// a workgroup owns a 16 x 32 column tile of one unit and a chunk of 16 planes i, which it
// walks in order.  Each plane of the tile and its one-cell in-plane halo is staged in LDS
// once, with everything a neighbour contributes (double precision: u and b = exp(u); single
// precision: ub, e, B and M), so a cell's exponentials are evaluated once per launch instead
// of at every visit from each of its six neighbours.  Outside a patch the staged value is the
// boundary value u_b of the face there (the face term needs only u_b and the cell's own
// value), so no visit waits on a load.  Loads run kAhead planes ahead of the plane being
// updated: the raw values of the next planes are in flight while the current one is relaxed.
//
// The update of a cell of the colour is that of kb_ngs / kb32_ngs (batch_dev.h: bcell,
// bcell32), with the same operands in the same order, so the results are the same bits.
// Each thread updates one cell of the colour per plane, in place: within one colour launch a
// cell's neighbours are all of the other colour and are not written.
#include "batch_dev.h"
#include "fused_fp32.h"

namespace mgfr {
namespace {

using namespace bdev;

constexpr int kTJ = 16, kTK = 32, kTI = 16;     // tile and plane chunk
constexpr int kPatchTI = 8;                     // plane chunk of the fused sweep of a patch
constexpr int kAhead = 4;                       // planes whose loads are in flight
constexpr int kNT = kTJ * kTK / 2;              // one cell of the colour per thread per plane
constexpr int kLK = kTK + 2, kNL = (kTJ + 2) * kLK;
constexpr int kSlots = (kNL + kNT - 1) / kNT;   // staged entries per thread and plane
constexpr int kRing = 4;                        // staged planes p - 1 .. p + 2

// Global-memory accesses through the pointers of a grid descriptor.  Read from a table, they
// would otherwise be accessed as flat addresses, which the LDS wait before every barrier of
// the walk also waits for: the loads issued for the planes ahead would have to land first.
template <class T>
__device__ __forceinline__ T gload(const T* p)
{
    return *(const __attribute__((address_space(1))) T*)p;
}
template <class T>
__device__ __forceinline__ void gstore(T* p, T v)
{
    *(__attribute__((address_space(1))) T*)p = v;
}

// ---- the two precisions ------------------------------------------------------------------
// Raw: what is loaded for a staged entry, from offset off of the cell values or (face) of
// the boundary values; Lds: what is staged; Rhs: the right-hand side of a cell.  A staged
// entry outside a patch holds the face's u_b in its first field.  The loads take no branch
// on the kind of entry (a branch whose result is converted or copied at its join would wait
// there for every load in flight).
struct P64 {
    using Raw = double;
    using Lds = double2;
    using Rhs = double;
    __device__ __forceinline__ static Raw load(const BGrid& g, bool face, long long off)
    {
        const double* base = face ? g.ub : g.u;
        return gload(base + off);
    }
    __device__ __forceinline__ static Raw cell(const BGrid& g, unsigned off) { return gload(g.u + off); }
    __device__ __forceinline__ static Lds make(Raw v, bool) { return make_double2(v, exp(v)); }
    __device__ __forceinline__ static Rhs rhs(const BGrid& g, unsigned q) { return gload(g.src + q); }

    // bcell's L - f and dL with the neighbours (i-1, i+1, j-1, j+1, k-1, k+1) and the cell
    // from LDS
    __device__ __forceinline__ static void op(const BGrid& g, const bool (&out)[6], const Lds (&nb)[6], Lds c, Rhs src,
                                              double& L, double& dL)
    {
        const double ui = c.x, bi = c.y;
        double su = 0.0, sb = 0.0, sbu = 0.0, lg_ = 0.0, dlg = 0.0;
        int nreg = 0;
#pragma unroll
        for (int x = 0; x < 6; ++x) {
            if (__builtin_expect(out[x], 0)) {
                const double ug = (1.0 - kR) * nb[x].x + kR * ui;
                const double bg = exp(ug);
                lg_ += (bg + bi) * (ug - ui);
                dlg += (kR * bg + bi) * (ug - ui) + (bg + bi) * (kR - 1.0);
            } else {
                const double un = nb[x].x, bn = nb[x].y, du = un - ui;
                su += du;
                sb += bn;
                sbu = fma(bn, du, sbu);
                ++nreg;
            }
        }
        const double S = g.A * exp(-ui * g.inv_np1);
        L = g.C * (fma(bi, su, sbu) + lg_) + S - fma(g.fscale, src - g.sref, g.fshift);
        dL = g.C * (fma(bi, su, -sb) - nreg * bi + dlg) - S * g.inv_np1;
    }
    // bcell's update
    __device__ __forceinline__ static void update(const BGrid& g, unsigned q, const bool (&out)[6], const Lds (&nb)[6], Lds c, Rhs src)
    {
        double L, dL;
        op(g, out, nb, c, src, L, dL);
        gstore(g.u + q, c.x + dev::bounded(-L / dL, g.max_step));
    }
    // the value restricted, the residual, and the coarse cell they set
    __device__ __forceinline__ static double value(Lds c) { return c.x; }
    __device__ __forceinline__ static double residual(const BGrid& g, const bool (&out)[6], const Lds (&nb)[6], Lds c,
                                                      Rhs src)
    {
        double L, dL;
        op(g, out, nb, c, src, L, dL);
        return L;
    }
    __device__ __forceinline__ static void restrict_to(const BGrid& c, unsigned qc, double su, double sd)
    {
        gstore(c.u + qc, 0.125 * su);
        gstore(c.uhat + qc, 0.125 * su);
        gstore(c.f + qc, 0.125 * sd);
    }
};

struct F2 {
    float x, y;
};

struct P32 {
    using Raw = F2;
    using Lds = V32;
    using Rhs = float;
    // a cell: (ub, e); a face: the two halves of the double u_b
    __device__ __forceinline__ static Raw load(const BGrid& g, bool face, long long off)
    {
        const float* px = face ? (const float*)(g.ub + off) : g.ub32 + off;
        const float* py = face ? px + 1 : g.e32 + off;
        return F2{gload(px), gload(py)};
    }
    __device__ __forceinline__ static Raw cell(const BGrid& g, unsigned off)
    {
        return F2{gload(g.ub32 + off), gload(g.e32 + off)};
    }
    __device__ __forceinline__ static Lds make(Raw v, bool face)
    {
        const unsigned long long bits = ((unsigned long long)__builtin_bit_cast(unsigned, v.y) << 32) |
                                        __builtin_bit_cast(unsigned, v.x);
        const float ubf = (float)__builtin_bit_cast(double, bits);
        return make_v(face ? ubf : v.x, face ? 0.0f : v.y);
    }
    __device__ __forceinline__ static Rhs rhs(const BGrid& g, unsigned q) { return gload(g.f32 + q); }

    // bcell32's N - f and dN with the neighbours and the cell from LDS
    __device__ __forceinline__ static Res32 op(const BGrid& g, const bool (&out)[6], const Lds (&nb)[6], Lds c, Rhs f)
    {
        const Op32 o = op32(g);
        float t1 = 0.0f, t2 = 0.0f, su = 0.0f, se = 0.0f, sB = 0.0f, nreg = 0.0f, lgh = 0.0f, dgh = 0.0f;
#pragma unroll
        for (int x = 0; x < 6; ++x) {
            if (__builtin_expect(out[x], 0)) {
                const float ubg = (1.0f - kR32) * nb[x].ub + kR32 * c.ub;
                const float eg = kR32 * c.e;
                const float bg = __expf(ubg);
                const float Mg = bg * em1f(eg), Bg = bg + Mg;
                const float du = ubg - c.ub, de = eg - c.e;
                lgh += (Mg + c.M) * du + (Bg + c.B) * de;
                dgh += (kR32 * Bg + c.B) * (du + de) + (Bg + c.B) * (kR32 - 1.0f);
            } else {
                const V32 n = nb[x];
                const float du = n.ub - c.ub, de = n.e - c.e;
                t1 = fmaf(n.M, du, t1);
                t2 = fmaf(n.B, de, t2);
                su += du;
                se += de;
                sB += n.B;
                nreg += 1.0f;
            }
        }
        const float S = o.A * __expf(-c.ub * o.inv_np1);
        const float xx = em1f(-c.e * o.inv_np1);
        Res32 r;
        r.N = o.C * (fmaf(c.M, su, t1) + fmaf(c.B, se, t2) + lgh) + S * xx - f;
        r.dN = o.C * (c.B * (su + se) - sB - nreg * c.B + dgh) - S * o.inv_np1 * (1.0f + xx);
        return r;
    }
    // bcell32's update
    __device__ __forceinline__ static void update(const BGrid& g, unsigned q, const bool (&out)[6], const Lds (&nb)[6], Lds c, Rhs f)
    {
        const Res32 r = op(g, out, nb, c, f);
        gstore(g.e32 + q, c.e + newton32(r, (float)g.max_step));
    }
    __device__ __forceinline__ static float value(Lds c) { return c.e; }
    __device__ __forceinline__ static float residual(const BGrid& g, const bool (&out)[6], const Lds (&nb)[6], Lds c, Rhs f)
    {
        return op(g, out, nb, c, f).N;
    }
    __device__ __forceinline__ static void restrict_to(const BGrid& c, unsigned qc, float se, float sd)
    {
        gstore(c.e32 + qc, 0.125f * se);
        gstore(c.eh32 + qc, 0.125f * se);
        gstore(c.f32 + qc, 0.125f * sd);
    }
};

// ---- the walk ------------------------------------------------------------------------------
// Staged entry e = (row jj, column kk) of the tile and its halo: what a plane p holds there.
//   kind 0: a cell of the unit (periodic: wrapped), at plane offset a = (j << lg) + k; on a
//           patch's planes -1 and n it is the i-face's u_b at (f << 2 lg) + a, f = 0 / 1;
//   kind 1: outside a patch in j or k only: the face's u_b at fq + (p << lg);
//   kind 2: nothing (a corner of the halo, or past the halo).
// Entries that hold nothing on a plane load cell (p, 0, 0) of the unit, or cell 0, in vain.
struct Entry {
    int kind, a, fq;
};

__device__ __forceinline__ Entry entry(const BGrid& g, int j0, int k0, int e)
{
    Entry s{2, 0, 0};
    if (e >= kNL) return s;
    const int m = g.n - 1;
    int j = j0 - 1 + e / kLK, k = k0 - 1 + e % kLK;
    if (g.periodic) {
        j &= m;
        k &= m;
    }
    const bool jo = j < 0 || j > m, ko = k < 0 || k > m;
    if (!jo && !ko) {
        s.kind = 0;
        s.a = (j << g.lg) + k;
    } else if (jo != ko) {
        // face 2 / 3 (index (i, k)) or 4 / 5 (index (i, j))
        const int f = jo ? (j < 0 ? 2 : 3) : (k < 0 ? 4 : 5);
        s.kind = 1;
        s.fq = (f << (2 * g.lg)) + (jo ? k : j);
    }
    return s;
}

// What a walk does at each plane (A): A::kCells cells per thread, in its tile column pair
// (row jj, columns kb and kb + 1), column kb + A::column(parity of the plane, j, c) for cell
// c; act(g, q, c, out, nb, centre, rhs) on each, then act.plane_end(p) (every thread).
//
// A colour sweep: one cell per thread and plane, the one of the colour.
template <class P>
struct ColourSweep {
    static constexpr int kCells = 1;
    int colour;
    __device__ __forceinline__ int column(int par, int j, int) const { return (par + j + colour) & 1; }
    __device__ __forceinline__ void operator()(const BGrid& g, unsigned q, int, const bool (&out)[6],
                                               const typename P::Lds (&nb)[6], typename P::Lds c, typename P::Rhs f)
    {
        P::update(g, q, out, nb, c, f);
    }
    __device__ __forceinline__ void plane_end(int) {}
};

// The walk of one tile, PER: the unit is a periodic box (no faces, indices wrap).
template <class P, bool PER, class A>
__device__ __forceinline__ void walk(const BGrid g, int tile, typename P::Lds (*lv)[kNL], A& act)
{
    using Raw = typename P::Raw;
    const int m = g.n - 1, lg = g.lg;
    int i0, j0, k0;
    {
        const int ntk = g.n / kTK, ntj = g.n / kTJ;
        k0 = (tile % ntk) * kTK;
        tile /= ntk;
        j0 = (tile % ntj) * kTJ;
        i0 = (tile / ntj) * kTI;
    }
    const int t = threadIdx.x;
    Entry en[kSlots];
#pragma unroll
    for (int s = 0; s < kSlots; ++s) en[s] = entry(g, j0, k0, t + s * kNT);

    // raw values of plane p; a plane outside a patch holds its i-face
    auto outside = [&](int p) { return !PER && (p < 0 || p > m); };
    auto fetch = [&](int p, Raw (&r)[kSlots]) __attribute__((always_inline)) {
        if (PER) {
            const unsigned pl = (unsigned)(p & m) << (2 * lg);
#pragma unroll
            for (int s = 0; s < kSlots; ++s) r[s] = P::cell(g, pl + (unsigned)en[s].a);
        } else if (!outside(p)) {
            const long long pl = (long long)p << (2 * lg);
#pragma unroll
            for (int s = 0; s < kSlots; ++s) {
                const bool face = en[s].kind == 1;
                r[s] = P::load(g, face, face ? en[s].fq + (p << lg) : pl + en[s].a);
            }
        } else {
            const int fb = (p < 0 ? 0 : 1) << (2 * lg);
#pragma unroll
            for (int s = 0; s < kSlots; ++s) {
                const bool face = en[s].kind == 0;
                r[s] = P::load(g, face, face ? fb + en[s].a : 0);
            }
        }
    };
    auto put = [&](int p, const Raw (&r)[kSlots]) __attribute__((always_inline)) {
        typename P::Lds* L = lv[(p - i0 + 1) % kRing];
        const int fk = outside(p) ? 0 : 1;  // the kind that holds a face on this plane
#pragma unroll
        for (int s = 0; s < kSlots; ++s)
            if (en[s].kind != 2) L[t + s * kNT] = P::make(r[s], !PER && en[s].kind == fk);
    };
    // The cells this thread handles on plane p: row jj of the tile, columns chosen by the
    // action from kb, kb + 1 by the parity of p (i0 is even, so that of the step).  Their
    // offsets in the plane and LDS entries for even and odd steps.
    constexpr int NC = A::kCells;
    const int jj = t / (kTK / 2);
    const int kb = 2 * (t - jj * (kTK / 2));
    const int j = j0 + jj;
    int kc[2][NC];
    unsigned jk[2][NC];
    int ec[2][NC];
#pragma unroll
    for (int par = 0; par < 2; ++par) {
#pragma unroll
        for (int c = 0; c < NC; ++c) {
            kc[par][c] = k0 + kb + act.column(par, j, c);
            jk[par][c] = ((unsigned)j << lg) + (unsigned)kc[par][c];
            ec[par][c] = (jj + 1) * kLK + (kc[par][c] - k0) + 1;
        }
    }
    auto cell_q = [&](int p, int par, int c) { return ((unsigned)p << (2 * lg)) + jk[par][c]; };

    Raw ahead[kAhead][kSlots];
    typename P::Rhs rh[kAhead][NC];
    {
        Raw r0[kSlots], r1[kSlots], r2[kSlots];
        fetch(i0 - 1, r0);
        fetch(i0, r1);
        fetch(i0 + 1, r2);
#pragma unroll
        for (int d = 0; d < kAhead; ++d) fetch(i0 + 2 + d, ahead[d]);
#pragma unroll
        for (int d = 0; d < kAhead; ++d)
#pragma unroll
            for (int c = 0; c < NC; ++c) rh[d][c] = P::rhs(g, cell_q(i0 + d, d & 1, c));
        put(i0 - 1, r0);
        put(i0, r1);
        put(i0 + 1, r2);
    }
    __syncthreads();
#pragma unroll
    for (int s = 0; s < kTI; ++s) {
        const int p = i0 + s, d = s % kAhead, par = s & 1;
#pragma unroll
        for (int c = 0; c < NC; ++c) {
            const typename P::Lds* Lm = lv[(s + 0) % kRing];
            const typename P::Lds* L0 = lv[(s + 1) % kRing];
            const typename P::Lds* Lp = lv[(s + 2) % kRing];
            const int e = ec[par][c], k = kc[par][c];
            const bool out[6] = {!PER && p == 0, !PER && p == m, !PER && j == 0,
                                 !PER && j == m, !PER && k == 0, !PER && k == m};
            const typename P::Lds nb[6] = {Lm[e], Lp[e], L0[e - kLK], L0[e + kLK], L0[e - 1], L0[e + 1]};
            act(g, cell_q(p, par, c), c, out, nb, L0[e], rh[d][c]);
        }
        act.plane_end(p);
        if (s + kAhead < kTI)
#pragma unroll
            for (int c = 0; c < NC; ++c) rh[d][c] = P::rhs(g, cell_q(p + kAhead, par, c));
        if (s + 2 <= kTI) put(p + 2, ahead[d]);
        if (s + 2 + kAhead <= kTI) fetch(p + 2 + kAhead, ahead[d]);
        __syncthreads();
    }
}

template <class P>
__global__ void __launch_bounds__(kNT) kc_ngs(BTable t, int colour)
{
    __shared__ typename P::Lds lv[kRing][kNL];
    const int2 blk = t.blk[blockIdx.x];
    const BGrid g = t.grids[blk.x];
    if (!live(t, g)) return;
    ColourSweep<P> act{colour};
    if (g.periodic)
        walk<P, true>(g, blk.y, lv, act);
    else
        walk<P, false>(g, blk.y, lv, act);
}

// ---- double-precision residual over the same tiles ------------------------------------------
// d = L(u) - f at both cells of the thread's column pair on every plane (bcell's arithmetic,
// the exponentials of each staged cell formed once); the thread keeps sum d^2 and max |d|,
// the workgroup folds them into one (sum, max) pair per tile.  CAST (the outer loop of a
// mixed solve): also r = -d, ub = u in single precision and e = 0, as kb_resid_cast.
// The running sums are also written to the thread's LDS slots at every cell: kept only in
// registers, their updates would be sunk to the end of the walk, every d held live until
// then (over 256 VGPRs).
template <bool CAST>
struct Resid64 {
    static constexpr int kCells = 2;
    double s = 0.0, mx = 0.0;
    double *ls, *lm;
    __device__ __forceinline__ int column(int, int, int c) const { return c; }
    __device__ __forceinline__ void operator()(const BGrid& g, unsigned q, int, const bool (&out)[6],
                                               const double2 (&nb)[6], double2 c, double src)
    {
        double d, dL;
        P64::op(g, out, nb, c, src, d, dL);
        if (CAST) {
            gstore(g.f32 + q, (float)(-d));
            gstore(g.ub32 + q, (float)c.x);
            gstore(g.e32 + q, 0.0f);
        }
        s += d * d;
        const double a = fabs(d);
        if (!(mx >= a)) mx = a;
        *ls = s;
        *lm = mx;
    }
    __device__ __forceinline__ void plane_end(int) {}
};

// ---- residual and restriction over the same tiles --------------------------------------------
// The residual of both cells of the thread's column pair on every plane (P64: L(u) - f; P32:
// N(e) - r), and with them the sums over each 2 x 2 x 2 block that the coarse level takes:
// coarse value = mean of the fine values, coarse right-hand side = mean of the residuals
// (kb_resid_restrict / kb32_resid_restrict, summed in their order: i, then j, then k).  The
// rows jj and jj + 1 of a block lie on lanes t and t + 16 of one wavefront.
template <class P>
struct ResidRestrict {
    using T = decltype(P::value(typename P::Lds{}));
    static constexpr int kCells = 2;
    BGrid c;       // the coarse grid
    T v[2], r[2];  // this plane's values and residuals
    T sv = 0, sr = 0;
    unsigned q0 = 0;
    __device__ __forceinline__ int column(int, int, int cc) const { return cc; }
    __device__ __forceinline__ void operator()(const BGrid& g, unsigned q, int cc, const bool (&out)[6],
                                               const typename P::Lds (&nb)[6], typename P::Lds ctr,
                                               typename P::Rhs rhs)
    {
        v[cc] = P::value(ctr);
        r[cc] = P::residual(g, out, nb, ctr, rhs);
        if (cc == 0) q0 = q;
    }
    __device__ __forceinline__ void plane_end(int p)
    {
        const T pv0 = __shfl_down(v[0], 16), pv1 = __shfl_down(v[1], 16);
        const T pr0 = __shfl_down(r[0], 16), pr1 = __shfl_down(r[1], 16);
        if (!(p & 1)) {
            sv = 0;
            sr = 0;
        }
        sv += v[0];
        sr += r[0];
        sv += v[1];
        sr += r[1];
        sv += pv0;
        sr += pr0;
        sv += pv1;
        sr += pr1;
        const int lg = c.lg + 1, m = (1 << lg) - 1;
        const int j = (int)(q0 >> lg) & m;
        if ((p & 1) && !(j & 1)) {
            const int k = (int)(q0 & m) & ~1;
            const unsigned qc = ((((unsigned)(p >> 1) << c.lg) + (unsigned)(j >> 1)) << c.lg) + (unsigned)(k >> 1);
            P::restrict_to(c, qc, sv, sr);
        }
    }
};

template <bool CAST>
__global__ void __launch_bounds__(kNT) kc_resid(BTable t, double* __restrict__ partial)
{
    __shared__ double2 lv[kRing][kNL];
    __shared__ double ra[kNT], rb[kNT];
    const int2 blk = t.blk[blockIdx.x];
    const BGrid g = t.grids[blk.x];
    Resid64<CAST> act;
    act.ls = ra + threadIdx.x;
    act.lm = rb + threadIdx.x;
    ra[threadIdx.x] = 0.0;
    rb[threadIdx.x] = 0.0;
    if (live(t, g)) {
        if (g.periodic)
            walk<P64, true>(g, blk.y, lv, act);
        else
            walk<P64, false>(g, blk.y, lv, act);
    }
    __syncthreads();
    for (int w = kNT / 2; w > 0; w >>= 1) {
        if (threadIdx.x < w) {
            ra[threadIdx.x] += ra[threadIdx.x + w];
            const double o = rb[threadIdx.x + w];
            if (!(rb[threadIdx.x] >= o)) rb[threadIdx.x] = o;
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        partial[2 * blockIdx.x] = ra[0];
        partial[2 * blockIdx.x + 1] = rb[0];
    }
}

template <class P>
__global__ void __launch_bounds__(kNT) kc_resid_restrict(BTable t, const BGrid* __restrict__ tc)
{
    __shared__ typename P::Lds lv[kRing][kNL];
    const int2 blk = t.blk[blockIdx.x];
    const BGrid g = t.grids[blk.x];
    if (!live(t, g)) return;
    ResidRestrict<P> act;
    act.c = tc[blk.x];
    if (g.periodic)
        walk<P, true>(g, blk.y, lv, act);
    else
        walk<P, false>(g, blk.y, lv, act);
}

// ---- both colours in one pass (single precision) --------------------------------------------
// The tile sweep of the domain solve over the same 16 x 32 x 16 tiles (on a patch with its
// boundary values in the halo, fused_fp32.h), out of place: a tile's
// halo is read from the old values while neighbouring tiles write theirs, so each sweep reads
// one buffer of e and writes the other (dir 0: e32 to e32b, dir 1: back).  Consecutive table
// entries go to the same XCD (workgroups are dealt to the 8 XCDs in turn).
// PER: periodic boxes, else patches (kernels of their own: the patch form's registers would
// push the box form into spills).  ADDU (dir 1, boxes only): the last sweep of a correction
// solve, which adds its e to u instead of writing it back.
template <bool PER, bool ADDU = false>
__global__ void __launch_bounds__(kNT, 4) kf32_ngs(BTable t, int dir)
{
    __shared__ V32 lv[3][(kTJ + 4) * (kTK + 4)];
    const int nb = gridDim.x;
    int b = blockIdx.x;
    if ((nb & 7) == 0) b = (b & 7) * (nb >> 3) + (b >> 3);
    const int2 blk = t.blk[b];
    const BGrid g = t.grids[blk.x];
    if (!live(t, g)) return;
    const int ntk = g.n / kTK, ntj = g.n / kTJ;
    int tile = blk.y;
    const int k0 = (tile % ntk) * kTK;
    tile /= ntk;
    const int j0 = (tile % ntj) * kTJ;
    const int ti = PER ? kTI : kPatchTI;
    const int i0 = (tile / ntj) * ti;
    const float* ein = dir ? g.e32b : g.e32;
    float* eout = dir ? g.e32 : g.e32b;
    if (PER)
        fused32::sweep_tile<kTJ, kTK, false, ADDU>(op32(g), g.n, g.lg, i0, j0, k0, ti, g.ub32, ein, eout, g.f32, lv,
                                                   nullptr, g.u);
    else
        fused32::sweep_tile<kTJ, kTK, true, ADDU>(op32(g), g.n, g.lg, i0, j0, k0, ti, g.ub32, ein, eout, g.f32, lv,
                                                  g.ub, g.u);
}

}  // namespace

long long batch_col_tiles(int n)
{
    if (n < kTK || n % kTK || n % kTI) return 0;
    return (long long)(n / kTI) * (n / kTJ) * (n / kTK);
}

long long batch_pair_tiles(int n, int periodic)
{
    const int ti = periodic ? kTI : kPatchTI;
    if (n < kTK || n % kTK || n % ti) return 0;
    return (long long)(n / ti) * (n / kTJ) * (n / kTK);
}

hipError_t batch_ngs_col(const BTable& t, int nblk, hipStream_t s)
{
    for (int colour = 0; colour < 2; ++colour)
        hipLaunchKernelGGL(kc_ngs<P64>, dim3(nblk), dim3(kNT), 0, s, t, colour);
    return hipGetLastError();
}

hipError_t batch_ngs32_col(const BTable& t, int nblk, hipStream_t s)
{
    for (int colour = 0; colour < 2; ++colour)
        hipLaunchKernelGGL(kc_ngs<P32>, dim3(nblk), dim3(kNT), 0, s, t, colour);
    return hipGetLastError();
}

hipError_t batch_ngs32_pair(const BTable& t, int nblk, bool periodic, bool add_u, hipStream_t s)
{
    if (add_u && !periodic) return hipErrorInvalidValue;  // boxes only (the patch form would spill)
    for (int dir = 0; dir < 2; ++dir) {
        if (dir == 1 && add_u) {
            hipLaunchKernelGGL((kf32_ngs<true, true>), dim3(nblk), dim3(kNT), 0, s, t, dir);
        } else if (periodic) {
            hipLaunchKernelGGL(kf32_ngs<true>, dim3(nblk), dim3(kNT), 0, s, t, dir);
        } else {
            hipLaunchKernelGGL(kf32_ngs<false>, dim3(nblk), dim3(kNT), 0, s, t, dir);
        }
    }
    return hipGetLastError();
}

hipError_t batch_resid_col(const BTable& t, int nblk, double* partial, bool cast, hipStream_t s)
{
    if (cast)
        hipLaunchKernelGGL(kc_resid<true>, dim3(nblk), dim3(kNT), 0, s, t, partial);
    else
        hipLaunchKernelGGL(kc_resid<false>, dim3(nblk), dim3(kNT), 0, s, t, partial);
    return hipGetLastError();
}

hipError_t batch_resid_restrict_col(const BTable& t, int nblk, const BGrid* coarse, bool single, hipStream_t s)
{
    if (single)
        hipLaunchKernelGGL(kc_resid_restrict<P32>, dim3(nblk), dim3(kNT), 0, s, t, coarse);
    else
        hipLaunchKernelGGL(kc_resid_restrict<P64>, dim3(nblk), dim3(kNT), 0, s, t, coarse);
    return hipGetLastError();
}

}  // namespace mgfr
