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

__global__ void __launch_bounds__(kU) ku_whole64(UnitSet us, int* queue, UnitOut out, UnitCfg cfg)
{
    __shared__ Coarse64<kU> co;
    __shared__ int slot;
    for (;;) {
        const int it = next_unit(queue, &slot);
        if (it >= us.nwhole) break;
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

__global__ void __launch_bounds__(kU) ku_whole_mixed(UnitSet us, int* queue, UnitOut out, UnitCfg cfg)
{
    __shared__ Coarse32<kU> co;
    __shared__ double red[kU];
    __shared__ int slot;
    for (;;) {
        const int it = next_unit(queue, &slot);
        if (it >= us.nwhole) break;
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

__global__ void __launch_bounds__(kU) ku_fill_int(int* __restrict__ p, int v, int n)
{
    for (int q = blockIdx.x * kU + threadIdx.x; q < n; q += gridDim.x * kU) p[q] = v;
}

}  // namespace

int unit_block() { return kU; }

hipError_t unit_whole(const UnitSet& us, int* queue, const UnitOut& out, const UnitCfg& cfg, bool mixed, int nwg,
                      hipStream_t s)
{
    hipLaunchKernelGGL(ku_fill_int, dim3(1), dim3(kU), 0, s, queue, 0, 1);
    if (mixed)
        hipLaunchKernelGGL(ku_whole_mixed, dim3(nwg), dim3(kU), 0, s, us, queue, out, cfg);
    else
        hipLaunchKernelGGL(ku_whole64, dim3(nwg), dim3(kU), 0, s, us, queue, out, cfg);
    return hipGetLastError();
}

hipError_t unit_tail(const UnitSet& us, const int2* tails, int ntail, const int* active, const UnitCfg& cfg,
                     bool mixed, hipStream_t s)
{
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
