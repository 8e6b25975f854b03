// Workgroup-per-unit kernels of the batched solves (refinement patches of one level, or
// independent boxes).
//
// A unit small enough for one workgroup is solved there completely: every V-cycle (Sec. V.B.2;
// in the mixed solver every single-precision correction V-cycle and the double-precision
// defect correction around it), the stop test rms(L) <= tol and its residual history.  One
// persistent launch per batch takes units from a device counter, largest first, until the
// list is empty; no phase needs another workgroup, so no step of a unit's solve waits on
// anything outside its workgroup.  (On this GPU a barrier between workgroups, with the
// device-scope release and acquire it needs for the data to be seen, costs about four kernel
// launches; phases that span workgroups are therefore ordered by launches instead.)
//
// A larger unit runs its fine levels as batched launches over all large units of the batch;
// when its V-cycle reaches a level small enough, one workgroup per unit runs the rest of the
// V-cycle from there (the tail kernels).  After every cycle the judge kernel turns the
// per-unit residual sums into rms values, histories, cycle counts and active flags on the
// device, so the host reads only one "any unit active" word per chunk of cycles.
//
// Units and tail levels of side <= 16 run with every level in LDS (the resident kernels):
// the workgroup reads the unit's data once, runs its cycles there and writes the result
// back, so the many short phases of a small V-cycle wait on LDS rather than on device memory.
// Larger ones (unit_n > 16) use the same steps on device memory.
//
// The per-cell arithmetic is that of the batched kernels (batch_dev.h), in the same order.
#include <algorithm>

#include "batch_dev.h"

namespace mgfr {
namespace {

using namespace bdev;

constexpr int kU = 256;  // threads per workgroup

__device__ __forceinline__ void cell_of(const BGrid& g, long long q, int& i, int& j, int& k)
{
    i = (int)(q >> (2 * g.lg));
    j = (int)((q >> g.lg) & (g.n - 1));
    k = (int)(q & (g.n - 1));
}

// cell t of colour c (red: i + j + k even), t < n^3 / 2
__device__ __forceinline__ long long colour_cell(const BGrid& g, long long t, int colour, int& i, int& j, int& k)
{
    const int hk = g.n >> 1;
    const int s = (int)(t & (hk - 1));
    const long long row = t >> (g.lg - 1);
    i = (int)(row >> g.lg);
    j = (int)(row & (g.n - 1));
    k = 2 * s + ((i + j + colour) & 1);
    return idx3(g.lg, i, j, k);
}

// Sum over the workgroup of one value per thread (fixed tree order); every thread gets it.
__device__ double wg_sum(double v, double* red)
{
    red[threadIdx.x] = v;
    __syncthreads();
    for (int w = kU / 2; w > 0; w >>= 1) {
        if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    const double s = red[0];
    __syncthreads();
    return s;
}

// ---- double precision -------------------------------------------------------------------
__device__ void sweep64(const BGrid& g, int colour)
{
    const long long half = 1LL << (3 * g.lg - 1);
    for (long long t = threadIdx.x; t < half; t += kU) {
        int i, j, k;
        const long long q = colour_cell(g, t, colour, i, j, k);
        const OpVal r = bcell(g, g.u, i, j, k, brhs(g, q));
        g.u[q] = g.u[q] + dev::bounded(-r.L / r.dL, g.max_step);
    }
    __syncthreads();
}

// uc = uhat = R u and fc = R d on the level below
__device__ void resid_restrict64(const BGrid& g, const BGrid& c)
{
    const long long ncc = 1LL << (3 * c.lg);
    for (long long qc = threadIdx.x; qc < ncc; qc += kU) {
        int I, J, K;
        cell_of(c, qc, I, J, K);
        double su = 0.0, sd = 0.0;
        for (int a = 0; a < 2; ++a)
            for (int b = 0; b < 2; ++b)
                for (int z = 0; z < 2; ++z) {
                    const int i = 2 * I + a, j = 2 * J + b, k = 2 * K + z;
                    const long long q = idx3(g.lg, i, j, k);
                    su += g.u[q];
                    sd += bcell(g, g.u, i, j, k, brhs(g, q)).L;
                }
        c.u[qc] = 0.125 * su;
        c.uhat[qc] = 0.125 * su;
        c.f[qc] = 0.125 * sd;
    }
    __syncthreads();
}

// f = L^H(uhat) - f
__device__ void fas_rhs64(const BGrid& c)
{
    const long long nc = 1LL << (3 * c.lg);
    for (long long q = threadIdx.x; q < nc; q += kU) {
        int i, j, k;
        cell_of(c, q, i, j, k);
        c.f[q] = bcell(c, c.uhat, i, j, k, 0.0).L - c.f[q];
    }
    __syncthreads();
}

// uhat = u - uhat (the coarse correction), then u^h += P(uhat) (27/9/3/1; outside a patch a
// coarse cell contributes zero, Sec. V.A.3)
__device__ void correct64(const BGrid& g, const BGrid& c)
{
    const long long nc = 1LL << (3 * c.lg);
    for (long long q = threadIdx.x; q < nc; q += kU) c.uhat[q] = c.u[q] - c.uhat[q];
    __syncthreads();
    const long long nf = 1LL << (3 * g.lg);
    const int mc = c.n - 1;
    for (long long q = threadIdx.x; q < nf; q += kU) {
        int i, j, k;
        cell_of(g, q, i, j, k);
        const int I = i >> 1, J = j >> 1, K = k >> 1;
        const int si = (i & 1) ? 1 : -1, sj = (j & 1) ? 1 : -1, sk = (k & 1) ? 1 : -1;
        auto E = [&](int a, int b, int z) -> double {
            if (c.periodic) return c.uhat[idx3(c.lg, a & mc, b & mc, z & mc)];
            if (a < 0 || a > mc || b < 0 || b > mc || z < 0 || z > mc) return 0.0;
            return c.uhat[idx3(c.lg, a, b, z)];
        };
        const double p = (27.0 / 64.0) * E(I, J, K) +
                         (9.0 / 64.0) * (E(I + si, J, K) + E(I, J + sj, K) + E(I, J, K + sk)) +
                         (3.0 / 64.0) * (E(I + si, J + sj, K) + E(I + si, J, K + sk) + E(I, J + sj, K + sk)) +
                         (1.0 / 64.0) * E(I + si, J + sj, K + sk);
        g.u[q] += p;
    }
    __syncthreads();
}

// rms of the finest residual L(u) - f
__device__ double rms64(const BGrid& g, double* red)
{
    const long long nf = 1LL << (3 * g.lg);
    double s = 0.0;
    for (long long q = threadIdx.x; q < nf; q += kU) {
        int i, j, k;
        cell_of(g, q, i, j, k);
        const double d = bcell(g, g.u, i, j, k, brhs(g, q)).L;
        s += d * d;
    }
    return sqrt(wg_sum(s, red) / (double)nf);
}

// V-cycle from level m0 of a unit whose levels are G[0 .. nlev-1]
__device__ void vcycle64(const BGrid* G, int m0, int nlev, const UnitCfg& cfg, Coarse64<kU>& co)
{
    for (int m = m0; m < nlev - 1; ++m) {
        for (int s = 0; s < cfg.pre; ++s) {
            sweep64(G[m], 0);
            sweep64(G[m], 1);
        }
        resid_restrict64(G[m], G[m + 1]);
        fas_rhs64(G[m + 1]);
    }
    coarsest64<kU>(G[nlev - 1], cfg.cap, cfg.rtol, co);
    for (int m = nlev - 2; m >= m0; --m) {
        correct64(G[m], G[m + 1]);
        for (int s = 0; s < cfg.post; ++s) {
            sweep64(G[m], 0);
            sweep64(G[m], 1);
        }
    }
}

// ---- single precision (correction V-cycles of the mixed solver) --------------------------
__device__ void sweep32(const BGrid& g, int colour)
{
    const Op32 o = op32(g);
    const long long half = 1LL << (3 * g.lg - 1);
    for (long long t = threadIdx.x; t < half; t += kU) {
        int i, j, k;
        const long long q = colour_cell(g, t, colour, i, j, k);
        const Res32 r = bcell32(g, o, g.ub32, g.e32, i, j, k, g.f32[q]);
        g.e32[q] = g.e32[q] + newton32(r, o.max_step);
    }
    __syncthreads();
}

__device__ void resid_restrict32(const BGrid& g, const BGrid& c)
{
    const Op32 o = op32(g);
    const long long ncc = 1LL << (3 * c.lg);
    for (long long qc = threadIdx.x; qc < ncc; qc += kU) {
        int I, J, K;
        cell_of(c, qc, I, J, K);
        float se = 0.0f, sd = 0.0f;
        for (int a = 0; a < 2; ++a)
            for (int b = 0; b < 2; ++b)
                for (int z = 0; z < 2; ++z) {
                    const int i = 2 * I + a, j = 2 * J + b, k = 2 * K + z;
                    const long long q = idx3(g.lg, i, j, k);
                    se += g.e32[q];
                    sd += bcell32(g, o, g.ub32, g.e32, i, j, k, g.f32[q]).N;
                }
        c.e32[qc] = 0.125f * se;
        c.eh32[qc] = 0.125f * se;
        c.f32[qc] = 0.125f * sd;
    }
    __syncthreads();
}

__device__ void fas_rhs32(const BGrid& c)
{
    const Op32 o = op32(c);
    const long long nc = 1LL << (3 * c.lg);
    for (long long q = threadIdx.x; q < nc; q += kU) {
        int i, j, k;
        cell_of(c, q, i, j, k);
        c.f32[q] = bcell32(c, o, c.ub32, c.eh32, i, j, k, 0.0f).N - c.f32[q];
    }
    __syncthreads();
}

__device__ void correct32(const BGrid& g, const BGrid& c)
{
    const long long nc = 1LL << (3 * c.lg);
    for (long long q = threadIdx.x; q < nc; q += kU) c.eh32[q] = c.e32[q] - c.eh32[q];
    __syncthreads();
    const long long nf = 1LL << (3 * g.lg);
    const int mc = c.n - 1;
    for (long long q = threadIdx.x; q < nf; q += kU) {
        int i, j, k;
        cell_of(g, q, i, j, k);
        const int I = i >> 1, J = j >> 1, K = k >> 1;
        const int si = (i & 1) ? 1 : -1, sj = (j & 1) ? 1 : -1, sk = (k & 1) ? 1 : -1;
        auto E = [&](int a, int b, int z) -> float {
            if (c.periodic) return c.eh32[idx3(c.lg, a & mc, b & mc, z & mc)];
            if (a < 0 || a > mc || b < 0 || b > mc || z < 0 || z > mc) return 0.0f;
            return c.eh32[idx3(c.lg, a, b, z)];
        };
        const float p = (27.0f / 64.0f) * E(I, J, K) +
                        (9.0f / 64.0f) * (E(I + si, J, K) + E(I, J + sj, K) + E(I, J, K + sk)) +
                        (3.0f / 64.0f) * (E(I + si, J + sj, K) + E(I + si, J, K + sk) + E(I, J + sj, K + sk)) +
                        (1.0f / 64.0f) * E(I + si, J + sj, K + sk);
        g.e32[q] += p;
    }
    __syncthreads();
}

// coarse bases R ub from level m0 down
__device__ void restrict_base32(const BGrid* G, int m0, int nlev)
{
    for (int m = m0; m + 1 < nlev; ++m) {
        const BGrid& g = G[m];
        const BGrid& c = G[m + 1];
        const long long ncc = 1LL << (3 * c.lg);
        for (long long qc = threadIdx.x; qc < ncc; qc += kU) {
            int I, J, K;
            cell_of(c, qc, I, J, K);
            float s = 0.0f;
            for (int a = 0; a < 2; ++a)
                for (int b = 0; b < 2; ++b)
                    for (int z = 0; z < 2; ++z) s += g.ub32[idx3(g.lg, 2 * I + a, 2 * J + b, 2 * K + z)];
            c.ub32[qc] = 0.125f * s;
        }
        __syncthreads();
    }
}

__device__ void vcycle32(const BGrid* G, int m0, int nlev, const UnitCfg& cfg, Coarse32<kU>& co)
{
    for (int m = m0; m < nlev - 1; ++m) {
        for (int s = 0; s < cfg.pre; ++s) {
            sweep32(G[m], 0);
            sweep32(G[m], 1);
        }
        resid_restrict32(G[m], G[m + 1]);
        fas_rhs32(G[m + 1]);
    }
    coarsest32<kU>(G[nlev - 1], cfg.cap, (float)cfg.rtol, co);
    for (int m = nlev - 2; m >= m0; --m) {
        correct32(G[m], G[m + 1]);
        for (int s = 0; s < cfg.post; ++s) {
            sweep32(G[m], 0);
            sweep32(G[m], 1);
        }
    }
}

// Finest level, double precision: d = L(u) - f; r = -d and ub = u in single precision and
// e = 0 for the next inner solve; returns rms(d).
__device__ double resid_cast(const BGrid& g, double* red)
{
    const long long nf = 1LL << (3 * g.lg);
    double s = 0.0;
    for (long long q = threadIdx.x; q < nf; q += kU) {
        int i, j, k;
        cell_of(g, q, i, j, k);
        const double d = bcell(g, g.u, i, j, k, brhs(g, q)).L;
        g.f32[q] = (float)(-d);
        g.ub32[q] = (float)g.u[q];
        g.e32[q] = 0.0f;
        s += d * d;
    }
    return sqrt(wg_sum(s, red) / (double)nf);
}

__device__ void add_correction(const BGrid& g)
{
    const long long nf = 1LL << (3 * g.lg);
    for (long long q = threadIdx.x; q < nf; q += kU) g.u[q] += (double)g.e32[q];
    __syncthreads();
}

// ---- kernels ----------------------------------------------------------------------------
// The next unit of the queue, the same value in every lane (read through LDS, then made
// wave-uniform so that its descriptors load through the scalar unit).  The first barrier
// ends the previous unit (its last reads of the slot and its lane-0 stores) before lane 0
// takes the next one.  It must stay: without a barrier between the lane-0 stores that end a
// unit and the lane-0 atomic that starts the next, the compiler may join the two lane-0
// branches across the loop's back edge, and in the wave code that results the other lanes
// pass the barrier below and read the slot again before lane 0 has refilled it, so the
// workgroup repeats its last unit forever.
__device__ int next_unit(int* queue, int* slot)
{
    __syncthreads();
    if (threadIdx.x == 0) *slot = atomicAdd(queue, 1);
    __syncthreads();
    return __builtin_amdgcn_readfirstlane(*slot);
}

__device__ void finish(const UnitOut& out, int u, int k, double rms, double tol)
{
    if (threadIdx.x == 0) {
        out.ncyc[u] = k;
        out.status[u] = !isfinite(rms) ? 2 : rms <= tol ? 0 : 1;
    }
}

__global__ void __launch_bounds__(kU) ku_whole64(UnitSet us, int begin, int end, int* queue, UnitOut out, UnitCfg cfg)
{
    __shared__ Coarse64<kU> co;
    __shared__ int slot;
    for (;;) {
        const int it = begin + next_unit(queue, &slot);
        if (it >= end) break;
        const int u = __builtin_amdgcn_readfirstlane(us.order[it]);
        const BGrid* G = us.grids + us.first[u];
        const int nlev = us.nlev[u];
        double* hist = out.hist + (long long)u * out.H;
        double rms = rms64(G[0], co.ra);
        if (threadIdx.x == 0) hist[0] = rms;
        int k = 0;
        while (isfinite(rms) && rms > cfg.tol && k < cfg.max_cycles) {
            vcycle64(G, 0, nlev, cfg, co);
            rms = rms64(G[0], co.ra);
            ++k;
            if (threadIdx.x == 0) hist[k] = rms;
        }
        finish(out, u, k, rms, cfg.tol);
    }
}

__global__ void __launch_bounds__(kU) ku_whole_mixed(UnitSet us, int begin, int end, int* queue, UnitOut out,
                                                    UnitCfg cfg)
{
    __shared__ Coarse32<kU> co;
    __shared__ double red[kU];
    __shared__ int slot;
    for (;;) {
        const int it = begin + next_unit(queue, &slot);
        if (it >= end) break;
        const int u = __builtin_amdgcn_readfirstlane(us.order[it]);
        const BGrid* G = us.grids + us.first[u];
        const int nlev = us.nlev[u];
        double* hist = out.hist + (long long)u * out.H;
        double rms = resid_cast(G[0], red);
        if (threadIdx.x == 0) hist[0] = rms;
        int k = 0;
        while (isfinite(rms) && rms > cfg.tol && k < cfg.max_cycles) {
            restrict_base32(G, 0, nlev);
            for (int ic = 0; ic < cfg.inner; ++ic) vcycle32(G, 0, nlev, cfg, co);
            add_correction(G[0]);
            rms = resid_cast(G[0], red);
            ++k;
            if (threadIdx.x == 0) hist[k] = rms;
        }
        finish(out, u, k, rms, cfg.tol);
    }
}

// One workgroup per large unit: the rest of its V-cycle from its tail level down.
__global__ void __launch_bounds__(kU) ku_tail64(UnitSet us, const int2* __restrict__ tails, const int* __restrict__ active,
                                               UnitCfg cfg)
{
    __shared__ Coarse64<kU> co;
    const int2 t = tails[blockIdx.x];
    const BGrid* G = us.grids + t.x;
    if (!active[G[0].unit]) return;
    vcycle64(G, 0, t.y, cfg, co);
}

__global__ void __launch_bounds__(kU) ku_tail32(UnitSet us, const int2* __restrict__ tails, const int* __restrict__ active,
                                               UnitCfg cfg)
{
    __shared__ Coarse32<kU> co;
    const int2 t = tails[blockIdx.x];
    const BGrid* G = us.grids + t.x;
    if (!active[G[0].unit]) return;
    vcycle32(G, 0, t.y, cfg, co);
}

// Coarse bases R ub of the tail levels of every large unit (from its tail level down).
__global__ void __launch_bounds__(kU) ku_tail_base32(UnitSet us, const int2* __restrict__ tails,
                                                    const int* __restrict__ active)
{
    const int2 t = tails[blockIdx.x];
    const BGrid* G = us.grids + t.x;
    if (!active[G[0].unit]) return;
    restrict_base32(G, 0, t.y);
}

// After a cycle of the large units: sums[2 i] = sum of d^2 over the finest cells of large unit
// i (ids[i] its unit, ncell[i] its finest cells).  first != 0: the residual before the first
// cycle.  Writes the rms into the unit's history, counts the cycle, switches off units that
// reached tol, became non-finite or used max_cycles, and stores the number still active in
// *any.  One workgroup; units in a fixed order.
__global__ void __launch_bounds__(kU) ku_judge(const double* __restrict__ sums, const int* __restrict__ ids,
                                              const double* __restrict__ ncell, int nl, int* __restrict__ active,
                                              UnitOut out, double tol, int max_cycles, int first, int* any)
{
    __shared__ double red[kU];
    double cnt = 0.0;
    for (int i = threadIdx.x; i < nl; i += kU) {
        const int u = ids[i];
        if (!first && !active[u]) continue;
        const double rms = sqrt(sums[2 * i] / ncell[i]);
        const int k = first ? 0 : out.ncyc[u] + 1;
        out.ncyc[u] = k;
        out.hist[(long long)u * out.H + k] = rms;
        const bool stop = !isfinite(rms) || rms <= tol || k >= max_cycles;
        active[u] = stop ? 0 : 1;
        out.status[u] = !isfinite(rms) ? 2 : rms <= tol ? 0 : 1;
        if (!stop) cnt += 1.0;
    }
    const double tot = wg_sum(cnt, red);
    if (threadIdx.x == 0) *any = (int)tot;
}

// ---- LDS-resident solves -------------------------------------------------------------------
// A unit of side W, or a large unit's levels from its tail level (side W) down, with level d
// (side W >> d) held in LDS:
//   double precision: u, b = exp(u) (rewritten with every update of u) and f, and below the
//     top uh;
//   single precision: ub, e, f, b = exp(ub) and S = A exp(-ub/(n+1)) (both fixed while the
//     base is), and below the top eh.
// b and S are exactly the values the device-memory kernels evaluate at every visit, so every
// result is theirs bit for bit; only where the operands wait changes.
constexpr int cube(int s) { return s * s * s; }

// workgroup size of the resident kernels of side W
constexpr int res_threads(int W) { return W >= 16 ? 512 : 256; }
// The tails relax one unit's lower levels per launch (no persistent loop): twice the threads,
// for more waves to hide the LDS and arithmetic latency of their sweeps.
constexpr int tail_threads(int W) { return W >= 16 ? 1024 : res_threads(W); }

// element offsets of level d in the LDS array (double precision: top u, b, f; below + uh;
// every level its boundary values fc [6][s][s])
struct Off64 {
    int u, b, f, uh, fc;
};
constexpr int sq6(int s) { return 6 * s * s; }
template <int W>
__device__ __forceinline__ Off64 off64(int d)
{
    int at = 3 * cube(W) + sq6(W);
    Off64 o{0, cube(W), 2 * cube(W), -1, 3 * cube(W)};
    for (int e = 1, s = W / 2; e <= d; ++e, s /= 2) {
        o = Off64{at, at + cube(s), at + 2 * cube(s), at + 3 * cube(s), at + 4 * cube(s)};
        at += 4 * cube(s) + sq6(s);
    }
    return o;
}
template <int W>
constexpr int res64_size()
{
    int t = 3 * cube(W) + sq6(W);
    for (int s = W / 2; s >= 2; s /= 2) t += 4 * cube(s) + sq6(s);
    return t;
}

// single precision: top ub, e, f, b, S; below + eh; every level its boundary values fc
struct Off32 {
    int ub, e, f, b, S, eh, fc;
};
template <int W>
__device__ __forceinline__ Off32 off32(int d)
{
    int at = 5 * cube(W) + sq6(W);
    Off32 o{0, cube(W), 2 * cube(W), 3 * cube(W), 4 * cube(W), -1, 5 * cube(W)};
    for (int e = 1, s = W / 2; e <= d; ++e, s /= 2) {
        o = Off32{at, at + cube(s), at + 2 * cube(s), at + 3 * cube(s), at + 4 * cube(s), at + 5 * cube(s),
                  at + 6 * cube(s)};
        at += 6 * cube(s) + sq6(s);
    }
    return o;
}
template <int W>
constexpr int res32_size()
{
    int t = 5 * cube(W) + sq6(W);
    for (int s = W / 2; s >= 2; s /= 2) t += 6 * cube(s) + sq6(s);
    return t;
}

template <int NT>
__device__ double wg_sum_t(double v, double* red)
{
    red[threadIdx.x] = v;
    __syncthreads();
    for (int w = NT / 2; w > 0; w >>= 1) {
        if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    const double s = red[0];
    __syncthreads();
    return s;
}

// bcell with b and the boundary values read from the level instead of evaluated / loaded
__device__ __forceinline__ OpVal rcell64(const BGrid& g, const double* u, const double* b, const double* fc, int i,
                                         int j, int k, double f)
{
    const int m = g.n - 1;
    const int q = (((i << g.lg) + j) << g.lg) + k;
    const double ui = u[q], bi = b[q];
    double su = 0.0, sb = 0.0, sbu = 0.0, lg_ = 0.0, dlg = 0.0;
    int nreg = 0;
    const int di[6] = {-1, 1, 0, 0, 0, 0}, dj[6] = {0, 0, -1, 1, 0, 0}, dk[6] = {0, 0, 0, 0, -1, 1};
#pragma unroll
    for (int x = 0; x < 6; ++x) {
        const int ii = i + di[x], jj = j + dj[x], kk = k + dk[x];
        const bool out = ii < 0 || ii > m || jj < 0 || jj > m || kk < 0 || kk > m;
        if (out && !g.periodic) {
            const double ug = (1.0 - kR) * fc[face_index(g.lg, x, i, j, k)] + kR * ui;
            const double bg = exp(ug);
            lg_ += (bg + bi) * (ug - ui);
            dlg += (kR * bg + bi) * (ug - ui) + (bg + bi) * (kR - 1.0);
        } else {
            const int qn = ((((ii & m) << g.lg) + (jj & m)) << g.lg) + (kk & m);
            const double bn = b[qn], du = u[qn] - ui;
            su += du;
            sb += bn;
            sbu = fma(bn, du, sbu);
            ++nreg;
        }
    }
    const double S = g.A * exp(-ui * g.inv_np1);
    OpVal r;
    r.L = g.C * (fma(bi, su, sbu) + lg_) + S - f;
    r.dL = g.C * (fma(bi, su, -sb) - nreg * bi + dlg) - S * g.inv_np1;
    return r;
}

template <int NT>
__device__ void rsweep64(const BGrid& g, double* u, double* b, const double* f, const double* fc, int colour)
{
    const int half = 1 << (3 * g.lg - 1);
    for (int t = threadIdx.x; t < half; t += NT) {
        int i, j, k;
        const int q = (int)colour_cell(g, t, colour, i, j, k);
        const OpVal r = rcell64(g, u, b, fc, i, j, k, f[q]);
        const double v = u[q] + dev::bounded(-r.L / r.dL, g.max_step);
        u[q] = v;
        b[q] = exp(v);
    }
    __syncthreads();
}


// coarse u = uh = R u, b = exp(u), f = R d; then f = L^H(uh) - f.  Rounds of NT fine cells
// (whole slabs of coarse cells: NT is a multiple of 2 n^2, or the level fits one round):
// every thread evaluates one fine residual into red (NT entries), then each coarse cell of
// the round sums its eight children in (i, j, k) order.
template <int NT>
__device__ void rcoarsen64(const BGrid& g, const BGrid& c, double* lds, const Off64& a, const Off64& z, double* red)
{
    const int ncc = 1 << (3 * c.lg);
    const int nf = 1 << (3 * g.lg);
    for (int r0 = 0; r0 < nf; r0 += NT) {
        const int q = r0 + (int)threadIdx.x;
        if (q < nf) {
            int i, j, k;
            cell_of(g, q, i, j, k);
            red[threadIdx.x] = rcell64(g, lds + a.u, lds + a.b, lds + a.fc, i, j, k, lds[a.f + q]).L;
        }
        __syncthreads();
        const int nct = min(NT, nf - r0) / 8;
        for (int t = threadIdx.x; t < nct; t += NT) {
            const int qc = r0 / 8 + t;
            int I, J, K;
            cell_of(c, qc, I, J, K);
            double su = 0.0, sd = 0.0;
            for (int x = 0; x < 2; ++x)
                for (int y = 0; y < 2; ++y)
                    for (int w = 0; w < 2; ++w) {
                        const int qf = (int)idx3(g.lg, 2 * I + x, 2 * J + y, 2 * K + w);
                        su += lds[a.u + qf];
                        sd += red[qf - r0];
                    }
            lds[z.u + qc] = 0.125 * su;
            lds[z.uh + qc] = 0.125 * su;
            lds[z.b + qc] = exp(0.125 * su);
            lds[z.f + qc] = 0.125 * sd;
        }
        __syncthreads();
    }
    for (int q = threadIdx.x; q < ncc; q += NT) {
        int i, j, k;
        cell_of(c, q, i, j, k);
        lds[z.f + q] = rcell64(c, lds + z.uh, lds + z.b, lds + z.fc, i, j, k, 0.0).L - lds[z.f + q];
    }
    __syncthreads();
}

// uh = u - uh on the coarse level, then u += P(uh) on the fine one (with its b)
template <int NT>
__device__ void rcorrect64(const BGrid& g, const BGrid& c, double* lds, const Off64& a, const Off64& z)
{
    const int nc = 1 << (3 * c.lg);
    for (int q = threadIdx.x; q < nc; q += NT) lds[z.uh + q] = lds[z.u + q] - lds[z.uh + q];
    __syncthreads();
    const int nf = 1 << (3 * g.lg);
    const int mc = c.n - 1;
    const double* eh = lds + z.uh;
    for (int q = threadIdx.x; q < nf; q += NT) {
        int i, j, k;
        cell_of(g, q, i, j, k);
        const int I = i >> 1, J = j >> 1, K = k >> 1;
        const int si = (i & 1) ? 1 : -1, sj = (j & 1) ? 1 : -1, sk = (k & 1) ? 1 : -1;
        auto E = [&](int x, int y, int w) -> double {
            if (c.periodic) return eh[idx3(c.lg, x & mc, y & mc, w & mc)];
            if (x < 0 || x > mc || y < 0 || y > mc || w < 0 || w > mc) return 0.0;
            return eh[idx3(c.lg, x, y, w)];
        };
        const double p = (27.0 / 64.0) * E(I, J, K) +
                         (9.0 / 64.0) * (E(I + si, J, K) + E(I, J + sj, K) + E(I, J, K + sk)) +
                         (3.0 / 64.0) * (E(I + si, J + sj, K) + E(I + si, J, K + sk) + E(I, J + sj, K + sk)) +
                         (1.0 / 64.0) * E(I + si, J + sj, K + sk);
        const double v = lds[a.u + q] + p;
        lds[a.u + q] = v;
        lds[a.b + q] = exp(v);
    }
    __syncthreads();
}

template <int NT>
__device__ double rrms64(const BGrid& g, double* lds, const Off64& a, double* red)
{
    const int nf = 1 << (3 * g.lg);
    double s = 0.0;
    for (int q = threadIdx.x; q < nf; q += NT) {
        int i, j, k;
        cell_of(g, q, i, j, k);
        const double d = rcell64(g, lds + a.u, lds + a.b, lds + a.fc, i, j, k, lds[a.f + q]).L;
        s += d * d;
    }
    return sqrt(wg_sum_t<NT>(s, red) / (double)nf);
}

// V-cycle of the resident levels 0 .. nl - 1 (G[d] the descriptor of level d)
template <int W, int NT>
__device__ void rvcycle64(const BGrid* G, int nl, const UnitCfg& cfg, double* lds, double* cS, double* ra, double* rb)
{
    // the restriction rounds: whole slabs of coarse cells per NT fine cells on every level
    static_assert(NT >= 2 * W * W && NT % (2 * W * W) == 0, "NT threads per resident workgroup");
    for (int d = 0; d + 1 < nl; ++d) {
        const Off64 a = off64<W>(d), z = off64<W>(d + 1);
        for (int s = 0; s < cfg.pre; ++s) {
            rsweep64<NT>(G[d], lds + a.u, lds + a.b, lds + a.f, lds + a.fc, 0);
            rsweep64<NT>(G[d], lds + a.u, lds + a.b, lds + a.f, lds + a.fc, 1);
        }
        rcoarsen64<NT>(G[d], G[d + 1], lds, a, z, ra);
    }
    {
        const BGrid& g = G[nl - 1];
        const Off64 a = off64<W>(nl - 1);
        const int nc = 1 << (3 * g.lg);
        for (int q = threadIdx.x; q < nc; q += NT) cS[q] = g.A * exp(-lds[a.u + q] * g.inv_np1);
        __syncthreads();
        const double* fc = lds + a.fc;
        coarsest64_core<NT>(g, cfg.cap, cfg.rtol, C64{lds + a.u, lds + a.b, cS, lds + a.f, ra, rb},
                            [&](int f, int i, int j, int k) { return fc[face_index(g.lg, f, i, j, k)]; });
        __syncthreads();
    }
    for (int d = nl - 2; d >= 0; --d) {
        const Off64 a = off64<W>(d), z = off64<W>(d + 1);
        rcorrect64<NT>(G[d], G[d + 1], lds, a, z);
        for (int s = 0; s < cfg.post; ++s) {
            rsweep64<NT>(G[d], lds + a.u, lds + a.b, lds + a.f, lds + a.fc, 0);
            rsweep64<NT>(G[d], lds + a.u, lds + a.b, lds + a.f, lds + a.fc, 1);
        }
    }
}

// level 0 from device memory: u, b = exp(u), f = the level's right-hand side; and the
// boundary values of levels 0 .. nl - 1 (patches)
template <int W, int NT>
__device__ void rload64(const BGrid* G, int nl, double* lds)
{
    const BGrid& g = G[0];
    const Off64 a = off64<W>(0);
    for (int q = threadIdx.x; q < cube(W); q += NT) {
        const double v = g.u[q];
        lds[a.u + q] = v;
        lds[a.b + q] = exp(v);
        lds[a.f + q] = brhs(g, q);
    }
    if (!g.periodic)
        for (int d = 0; d < nl; ++d) {
            const int n6 = 6 << (2 * G[d].lg), fc = off64<W>(d).fc;
            for (int q = threadIdx.x; q < n6; q += NT) lds[fc + q] = G[d].ub[q];
        }
    __syncthreads();
}

template <int W, int NT>
__device__ void rstore64(const BGrid& g, const double* lds)
{
    const Off64 a = off64<W>(0);
    for (int q = threadIdx.x; q < cube(W); q += NT) g.u[q] = lds[a.u + q];
}

template <int W>
__global__ void __launch_bounds__(res_threads(W)) kr_whole64(UnitSet us, int begin, int end, int* queue, UnitOut out,
                                                            UnitCfg cfg)
{
    constexpr int NT = res_threads(W);
    __shared__ double lds[res64_size<W>()];
    __shared__ double cS[cube(W < 8 ? W : 8)];
    __shared__ double ra[NT], rb[NT];
    __shared__ int slot;
    for (;;) {
        const int it = begin + next_unit(queue, &slot);
        if (it >= end) break;
        const int u = __builtin_amdgcn_readfirstlane(us.order[it]);
        const BGrid* G = us.grids + us.first[u];
        const int nl = us.nlev[u];
        double* hist = out.hist + (long long)u * out.H;
        rload64<W, NT>(G, nl, lds);
        double rms = rrms64<NT>(G[0], lds, off64<W>(0), ra);
        if (threadIdx.x == 0) hist[0] = rms;
        int k = 0;
        while (isfinite(rms) && rms > cfg.tol && k < cfg.max_cycles) {
            rvcycle64<W, NT>(G, nl, cfg, lds, cS, ra, rb);
            rms = rrms64<NT>(G[0], lds, off64<W>(0), ra);
            ++k;
            if (threadIdx.x == 0) hist[k] = rms;
        }
        rstore64<W, NT>(G[0], lds);
        finish(out, u, k, rms, cfg.tol);
    }
}

template <int W>
__global__ void __launch_bounds__(tail_threads(W)) kr_tail64(UnitSet us, const int2* __restrict__ tails,
                                                            const int* __restrict__ active, UnitCfg cfg)
{
    constexpr int NT = tail_threads(W);
    __shared__ double lds[res64_size<W>()];
    __shared__ double cS[cube(W < 8 ? W : 8)];
    __shared__ double ra[NT], rb[NT];
    const int2 t = tails[blockIdx.x];
    const BGrid* G = us.grids + t.x;
    if (!active[G[0].unit]) return;
    rload64<W, NT>(G, t.y, lds);
    rvcycle64<W, NT>(G, t.y, cfg, lds, cS, ra, rb);
    rstore64<W, NT>(G[0], lds);
}

// ---- single precision, resident ---------------------------------------------------------
// bcell32 with b, S and the boundary values read from the level instead of evaluated / loaded
__device__ __forceinline__ Res32 rcell32(const BGrid& g, const Op32& o, const float* ub, const float* e,
                                         const float* b, const float* S, const float* fc, int i, int j, int k,
                                         float f)
{
    const int m = g.n - 1;
    const int q = (((i << g.lg) + j) << g.lg) + k;
    V32 c;
    c.ub = ub[q];
    c.e = e[q];
    c.M = b[q] * em1f(c.e);
    c.B = b[q] + c.M;
    float t1 = 0.0f, t2 = 0.0f, su = 0.0f, se = 0.0f, sB = 0.0f, nreg = 0.0f, lgh = 0.0f, dgh = 0.0f;
    const int di[6] = {-1, 1, 0, 0, 0, 0}, dj[6] = {0, 0, -1, 1, 0, 0}, dk[6] = {0, 0, 0, 0, -1, 1};
#pragma unroll
    for (int x = 0; x < 6; ++x) {
        const int ii = i + di[x], jj = j + dj[x], kk = k + dk[x];
        const bool out = ii < 0 || ii > m || jj < 0 || jj > m || kk < 0 || kk > m;
        if (out && !g.periodic) {
            const float ubg = (1.0f - kR32) * fc[face_index(g.lg, x, i, j, k)] + kR32 * c.ub;
            const float eg = kR32 * c.e;
            const float bg = __expf(ubg);
            const float Mg = bg * em1f(eg), Bg = bg + Mg;
            const float du = ubg - c.ub, de = eg - c.e;
            lgh += (Mg + c.M) * du + (Bg + c.B) * de;
            dgh += (kR32 * Bg + c.B) * (du + de) + (Bg + c.B) * (kR32 - 1.0f);
        } else {
            const int qn = ((((ii & m) << g.lg) + (jj & m)) << g.lg) + (kk & m);
            const float nM = b[qn] * em1f(e[qn]);
            const float nB = b[qn] + nM;
            const float du = ub[qn] - c.ub, de = e[qn] - c.e;
            t1 = fmaf(nM, du, t1);
            t2 = fmaf(nB, de, t2);
            su += du;
            se += de;
            sB += nB;
            nreg += 1.0f;
        }
    }
    const float Si = S[q];
    const float x = em1f(-c.e * o.inv_np1);
    Res32 r;
    r.N = o.C * (fmaf(c.M, su, t1) + fmaf(c.B, se, t2) + lgh) + Si * x - f;
    r.dN = o.C * (c.B * (su + se) - sB - nreg * c.B + dgh) - Si * o.inv_np1 * (1.0f + x);
    return r;
}

template <int NT>
__device__ void rsweep32(const BGrid& g, float* lds, const Off32& a, int colour)
{
    const Op32 o = op32(g);
    const int half = 1 << (3 * g.lg - 1);
    for (int t = threadIdx.x; t < half; t += NT) {
        int i, j, k;
        const int q = (int)colour_cell(g, t, colour, i, j, k);
        const Res32 r = rcell32(g, o, lds + a.ub, lds + a.e, lds + a.b, lds + a.S, lds + a.fc, i, j, k, lds[a.f + q]);
        lds[a.e + q] = lds[a.e + q] + newton32(r, o.max_step);
    }
    __syncthreads();
}


// coarse e = eh = R e, f = R N; then f = N^H(eh) - f (red: NT entries, as in rcoarsen64)
template <int NT>
__device__ void rcoarsen32(const BGrid& g, const BGrid& c, float* lds, const Off32& a, const Off32& z, float* red)
{
    const Op32 o = op32(g), oc = op32(c);
    const int ncc = 1 << (3 * c.lg);
    const int nf = 1 << (3 * g.lg);
    // as rcoarsen64: the fine residuals of a round of whole coarse slabs, one per thread
    for (int r0 = 0; r0 < nf; r0 += NT) {
        const int q = r0 + (int)threadIdx.x;
        if (q < nf) {
            int i, j, k;
            cell_of(g, q, i, j, k);
            red[threadIdx.x] =
                rcell32(g, o, lds + a.ub, lds + a.e, lds + a.b, lds + a.S, lds + a.fc, i, j, k, lds[a.f + q]).N;
        }
        __syncthreads();
        const int nct = min(NT, nf - r0) / 8;
        for (int t = threadIdx.x; t < nct; t += NT) {
            const int qc = r0 / 8 + t;
            int I, J, K;
            cell_of(c, qc, I, J, K);
            float se = 0.0f, sd = 0.0f;
            for (int x = 0; x < 2; ++x)
                for (int y = 0; y < 2; ++y)
                    for (int w = 0; w < 2; ++w) {
                        const int qf = (int)idx3(g.lg, 2 * I + x, 2 * J + y, 2 * K + w);
                        se += lds[a.e + qf];
                        sd += red[qf - r0];
                    }
            lds[z.e + qc] = 0.125f * se;
            lds[z.eh + qc] = 0.125f * se;
            lds[z.f + qc] = 0.125f * sd;
        }
        __syncthreads();
    }
    for (int q = threadIdx.x; q < ncc; q += NT) {
        int i, j, k;
        cell_of(c, q, i, j, k);
        lds[z.f + q] =
            rcell32(c, oc, lds + z.ub, lds + z.eh, lds + z.b, lds + z.S, lds + z.fc, i, j, k, 0.0f).N - lds[z.f + q];
    }
    __syncthreads();
}

template <int NT>
__device__ void rcorrect32(const BGrid& g, const BGrid& c, float* lds, const Off32& a, const Off32& z)
{
    const int nc = 1 << (3 * c.lg);
    for (int q = threadIdx.x; q < nc; q += NT) lds[z.eh + q] = lds[z.e + q] - lds[z.eh + q];
    __syncthreads();
    const int nf = 1 << (3 * g.lg);
    const int mc = c.n - 1;
    const float* eh = lds + z.eh;
    for (int q = threadIdx.x; q < nf; q += NT) {
        int i, j, k;
        cell_of(g, q, i, j, k);
        const int I = i >> 1, J = j >> 1, K = k >> 1;
        const int si = (i & 1) ? 1 : -1, sj = (j & 1) ? 1 : -1, sk = (k & 1) ? 1 : -1;
        auto E = [&](int x, int y, int w) -> float {
            if (c.periodic) return eh[idx3(c.lg, x & mc, y & mc, w & mc)];
            if (x < 0 || x > mc || y < 0 || y > mc || w < 0 || w > mc) return 0.0f;
            return eh[idx3(c.lg, x, y, w)];
        };
        const float p = (27.0f / 64.0f) * E(I, J, K) +
                        (9.0f / 64.0f) * (E(I + si, J, K) + E(I, J + sj, K) + E(I, J, K + sk)) +
                        (3.0f / 64.0f) * (E(I + si, J + sj, K) + E(I + si, J, K + sk) + E(I, J + sj, K + sk)) +
                        (1.0f / 64.0f) * E(I + si, J + sj, K + sk);
        lds[a.e + q] += p;
    }
    __syncthreads();
}

// b = exp(ub) and S of level d, from its base
template <int NT>
__device__ void rbase_terms32(const BGrid& g, float* lds, const Off32& a)
{
    const Op32 o = op32(g);
    const int n3 = 1 << (3 * g.lg);
    for (int q = threadIdx.x; q < n3; q += NT) {
        const float ub = lds[a.ub + q];
        lds[a.b + q] = __expf(ub);
        lds[a.S + q] = o.A * __expf(-ub * o.inv_np1);
    }
}

// coarse bases R ub of levels 1 .. nl - 1 with their b and S
template <int W, int NT>
__device__ void rbases32(const BGrid* G, int nl, float* lds)
{
    for (int d = 1; d < nl; ++d) {
        const BGrid& g = G[d - 1];
        const BGrid& c = G[d];
        const Off32 a = off32<W>(d - 1), z = off32<W>(d);
        const int ncc = 1 << (3 * c.lg);
        for (int qc = threadIdx.x; qc < ncc; qc += NT) {
            int I, J, K;
            cell_of(c, qc, I, J, K);
            float s = 0.0f;
            for (int x = 0; x < 2; ++x)
                for (int y = 0; y < 2; ++y)
                    for (int w = 0; w < 2; ++w) s += lds[a.ub + idx3(g.lg, 2 * I + x, 2 * J + y, 2 * K + w)];
            lds[z.ub + qc] = 0.125f * s;
        }
        __syncthreads();
        rbase_terms32<NT>(c, lds, z);
    }
    __syncthreads();
}

// the coarsest solve's own LDS: (B, M) per cell and the ghost-face terms
struct R32Co {
    float* cB;
    float* cM;
    float* gdu;
    float* gbb;
    float* ra;
    float* rb;
};

template <int W, int NT>
__device__ void rvcycle32(const BGrid* G, int nl, const UnitCfg& cfg, float* lds, const R32Co& co)
{
    // the restriction rounds: whole slabs of coarse cells per NT fine cells on every level
    static_assert(NT >= 2 * W * W && NT % (2 * W * W) == 0, "NT threads per resident workgroup");
    for (int d = 0; d + 1 < nl; ++d) {
        const Off32 a = off32<W>(d), z = off32<W>(d + 1);
        for (int s = 0; s < cfg.pre; ++s) {
            rsweep32<NT>(G[d], lds, a, 0);
            rsweep32<NT>(G[d], lds, a, 1);
        }
        rcoarsen32<NT>(G[d], G[d + 1], lds, a, z, co.ra);
    }
    {
        const BGrid& g = G[nl - 1];
        const Off32 a = off32<W>(nl - 1);
        const int nc = 1 << (3 * g.lg);
        for (int q = threadIdx.x; q < nc; q += NT) {
            const float bq = lds[a.b + q];
            const float M = bq * em1f(lds[a.e + q]);
            co.cM[q] = M;
            co.cB[q] = bq + M;
            const float* fc = lds + a.fc;
            coarse_ghosts32(g, q, lds[a.ub + q], co.gdu, co.gbb,
                            [&](int f, int i, int j, int k) { return fc[face_index(g.lg, f, i, j, k)]; });
        }
        __syncthreads();
        coarsest32_core<NT>(g, cfg.cap, (float)cfg.rtol,
                            C32{lds + a.ub, lds + a.b, lds + a.e, co.cB, co.cM, lds + a.S, lds + a.f, co.gdu, co.gbb,
                                co.ra, co.rb});
        __syncthreads();
    }
    for (int d = nl - 2; d >= 0; --d) {
        const Off32 a = off32<W>(d), z = off32<W>(d + 1);
        rcorrect32<NT>(G[d], G[d + 1], lds, a, z);
        for (int s = 0; s < cfg.post; ++s) {
            rsweep32<NT>(G[d], lds, a, 0);
            rsweep32<NT>(G[d], lds, a, 1);
        }
    }
}

// boundary values of levels 0 .. nl - 1 (patches), in single precision
template <int W, int NT>
__device__ void rfaces32(const BGrid* G, int nl, float* lds)
{
    if (G[0].periodic) return;
    for (int d = 0; d < nl; ++d) {
        const int n6 = 6 << (2 * G[d].lg), fc = off32<W>(d).fc;
        for (int q = threadIdx.x; q < n6; q += NT) lds[fc + q] = (float)G[d].ub[q];
    }
}

// Finest level in double precision from device memory: d = L(u) - f; r = -d, ub = u (with its
// b and S) and e = 0 into level 0; returns rms(d).
template <int W, int NT>
__device__ double rresid_cast(const BGrid& g, float* lds, double* red)
{
    const Off32 a = off32<W>(0);
    const long long nf = 1LL << (3 * g.lg);
    double s = 0.0;
    for (long long q = threadIdx.x; q < nf; q += NT) {
        int i, j, k;
        cell_of(g, q, i, j, k);
        const double d = bcell(g, g.u, i, j, k, brhs(g, q)).L;
        lds[a.f + q] = (float)(-d);
        lds[a.ub + q] = (float)g.u[q];
        lds[a.e + q] = 0.0f;
        s += d * d;
    }
    __syncthreads();
    rbase_terms32<NT>(g, lds, a);
    return sqrt(wg_sum_t<NT>(s, red) / (double)nf);
}

#define MGFR_R32_LDS(W, NTV)                           \
    constexpr int NT = NTV;                            \
    __shared__ float lds[res32_size<W>()];             \
    constexpr int NC = cube(W < 8 ? W : 8);            \
    __shared__ float cB[NC], cM[NC], gdu[6 * 512], gbb[6 * 512]; \
    __shared__ float ra[NT], rb[NT];                   \
    const R32Co co{cB, cM, gdu, gbb, ra, rb};

template <int W>
__global__ void __launch_bounds__(res_threads(W)) kr_whole_mixed(UnitSet us, int begin, int end, int* queue,
                                                                UnitOut out, UnitCfg cfg)
{
    MGFR_R32_LDS(W, res_threads(W))
    __shared__ double red[NT];
    __shared__ int slot;
    for (;;) {
        const int it = begin + next_unit(queue, &slot);
        if (it >= end) break;
        const int u = __builtin_amdgcn_readfirstlane(us.order[it]);
        const BGrid* G = us.grids + us.first[u];
        const int nl = us.nlev[u];
        double* hist = out.hist + (long long)u * out.H;
        rfaces32<W, NT>(G, nl, lds);
        double rms = rresid_cast<W, NT>(G[0], lds, red);
        if (threadIdx.x == 0) hist[0] = rms;
        int k = 0;
        while (isfinite(rms) && rms > cfg.tol && k < cfg.max_cycles) {
            rbases32<W, NT>(G, nl, lds);
            for (int ic = 0; ic < cfg.inner; ++ic) rvcycle32<W, NT>(G, nl, cfg, lds, co);
            {
                const Off32 a = off32<W>(0);
                for (int q = threadIdx.x; q < cube(W); q += NT) G[0].u[q] += (double)lds[a.e + q];
                __syncthreads();
            }
            rms = rresid_cast<W, NT>(G[0], lds, red);
            ++k;
            if (threadIdx.x == 0) hist[k] = rms;
        }
        finish(out, u, k, rms, cfg.tol);
    }
}

template <int W>
__global__ void __launch_bounds__(tail_threads(W)) kr_tail32(UnitSet us, const int2* __restrict__ tails,
                                                            const int* __restrict__ active, UnitCfg cfg)
{
    MGFR_R32_LDS(W, tail_threads(W))
    const int2 t = tails[blockIdx.x];
    const BGrid* G = us.grids + t.x;
    if (!active[G[0].unit]) return;
    const BGrid& g = G[0];
    const Off32 a = off32<W>(0);
    for (int q = threadIdx.x; q < cube(W); q += NT) {
        lds[a.ub + q] = g.ub32[q];
        lds[a.e + q] = g.e32[q];
        lds[a.f + q] = g.f32[q];
    }
    rfaces32<W, NT>(G, t.y, lds);
    __syncthreads();
    rbase_terms32<NT>(g, lds, a);
    __syncthreads();
    rbases32<W, NT>(G, t.y, lds);
    rvcycle32<W, NT>(G, t.y, cfg, lds, co);
    for (int q = threadIdx.x; q < cube(W); q += NT) g.e32[q] = lds[a.e + q];
}
#undef MGFR_R32_LDS

__global__ void __launch_bounds__(kU) ku_fill_int(int* __restrict__ p, int v, int n)
{
    for (int q = blockIdx.x * kU + threadIdx.x; q < n; q += gridDim.x * kU) p[q] = v;
}

}  // namespace

int unit_block() { return kU; }

template <int W>
hipError_t whole_resident(const UnitSet& us, int begin, int end, int* queue, const UnitOut& out, const UnitCfg& cfg,
                          bool mixed, int nwg, hipStream_t s)
{
    if (mixed)
        hipLaunchKernelGGL(kr_whole_mixed<W>, dim3(nwg), dim3(res_threads(W)), 0, s, us, begin, end, queue, out, cfg);
    else
        hipLaunchKernelGGL(kr_whole64<W>, dim3(nwg), dim3(res_threads(W)), 0, s, us, begin, end, queue, out, cfg);
    return hipGetLastError();
}

template <int W>
hipError_t tail_resident(const UnitSet& us, const int2* tails, int ntail, const int* active, const UnitCfg& cfg,
                         bool mixed, hipStream_t s)
{
    if (mixed)
        hipLaunchKernelGGL(kr_tail32<W>, dim3(ntail), dim3(tail_threads(W)), 0, s, us, tails, active, cfg);
    else
        hipLaunchKernelGGL(kr_tail64<W>, dim3(ntail), dim3(tail_threads(W)), 0, s, us, tails, active, cfg);
    return hipGetLastError();
}

hipError_t unit_whole(const UnitSet& us, int begin, int end, int side, int* queue, const UnitOut& out,
                      const UnitCfg& cfg, bool mixed, int max_wg, hipStream_t s)
{
    if (end <= begin) return hipSuccess;
    const int nwg = std::max(1, std::min({end - begin, 1024, max_wg}));
    hipLaunchKernelGGL(ku_fill_int, dim3(1), dim3(kU), 0, s, queue, 0, 1);
    switch (side) {
    case 2: return whole_resident<2>(us, begin, end, queue, out, cfg, mixed, nwg, s);
    case 4: return whole_resident<4>(us, begin, end, queue, out, cfg, mixed, nwg, s);
    case 8: return whole_resident<8>(us, begin, end, queue, out, cfg, mixed, nwg, s);
    case 16: return whole_resident<16>(us, begin, end, queue, out, cfg, mixed, nwg, s);
    default: break;
    }
    if (mixed)
        hipLaunchKernelGGL(ku_whole_mixed, dim3(nwg), dim3(kU), 0, s, us, begin, end, queue, out, cfg);
    else
        hipLaunchKernelGGL(ku_whole64, dim3(nwg), dim3(kU), 0, s, us, begin, end, queue, out, cfg);
    return hipGetLastError();
}

hipError_t unit_tail(const UnitSet& us, const int2* tails, int ntail, int side, const int* active, const UnitCfg& cfg,
                     bool mixed, hipStream_t s)
{
    if (ntail <= 0) return hipSuccess;
    switch (side) {
    case 2: return tail_resident<2>(us, tails, ntail, active, cfg, mixed, s);
    case 4: return tail_resident<4>(us, tails, ntail, active, cfg, mixed, s);
    case 8: return tail_resident<8>(us, tails, ntail, active, cfg, mixed, s);
    case 16: return tail_resident<16>(us, tails, ntail, active, cfg, mixed, s);
    default: break;
    }
    if (mixed)
        hipLaunchKernelGGL(ku_tail32, dim3(ntail), dim3(kU), 0, s, us, tails, active, cfg);
    else
        hipLaunchKernelGGL(ku_tail64, dim3(ntail), dim3(kU), 0, s, us, tails, active, cfg);
    return hipGetLastError();
}

hipError_t unit_tail_base32(const UnitSet& us, const int2* tails, int ntail, const int* active, hipStream_t s)
{
    hipLaunchKernelGGL(ku_tail_base32, dim3(ntail), dim3(kU), 0, s, us, tails, active);
    return hipGetLastError();
}

hipError_t unit_judge(const double* sums, const int* ids, const double* ncell, int nl, int* active, const UnitOut& out,
                      double tol, int max_cycles, bool first, int* any, hipStream_t s)
{
    hipLaunchKernelGGL(ku_judge, dim3(1), dim3(kU), 0, s, sums, ids, ncell, nl, active, out, tol, max_cycles,
                       first ? 1 : 0, any);
    return hipGetLastError();
}

hipError_t unit_fill_int(int* p, int v, int n, hipStream_t s)
{
    hipLaunchKernelGGL(ku_fill_int, dim3((unsigned)std::max(1, std::min(1024, (n + kU - 1) / kU))), dim3(kU), 0, s, p,
                       v, n);
    return hipGetLastError();
}

}  // namespace mgfr
