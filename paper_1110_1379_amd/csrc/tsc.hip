// Triangle-shaped-cloud (TSC) density assignment and force interpolation (Sec. VI.C),
// double precision, and their C entry points.
//
// Box units, periodic: cell i of the N^3 grid covers [i/N, (i+1)/N).  A particle at x has
// s = x N (modulo N), nearest cell floor(s) and offset d = s - floor(s) - 1/2; the cells
// floor(s) - 1, floor(s), floor(s) + 1 get the weights (1/2 - d)^2 / 2, 3/4 - d^2,
// (1/2 + d)^2 / 2 per axis, their product in 3-D.  Interpolation applies the same weights to
// the cell accelerations -grad phi, taken by central differences, so the pair conserves
// momentum.  Contraction into fused multiply-adds is switched off in the weight, product and
// sum arithmetic, so every operation rounds as written.
//
// Assignment is a gather, not a scatter: the particles are sorted by the key of their nearest
// cell (radix sort), a table gives each cell's range in that order, and every cell sums the
// contributions of the particles whose nearest cell is one of its 27 neighbours, through
// per-cell moments of each neighbour row (k_tsc_density), in a fixed order, so the density
// is the same bits on every call.  No atomics: in the clumps a scatter would put many lanes
// of a wavefront on the same few addresses.
#include <cstring>

#include <rocprim/rocprim.hpp>

#include "host_internal.h"

using namespace mgfr_host;

namespace mgfr {
namespace {

constexpr int kB = 256;

#pragma clang fp contract(off)

// Workgroup index remapped so that each of the 8 XCDs (which take workgroups round robin)
// runs one contiguous eighth of the grid: neighbouring cells and particles then share an L2.
__device__ __forceinline__ long long xcd_block()
{
    const unsigned nb = gridDim.x, b = blockIdx.x;
    if (nb & 7) return b;
    return (long long)(b & 7) * (nb >> 3) + (b >> 3);
}

// Nearest cell index and the three weights per axis of the particle at p[0..2].
__device__ __forceinline__ void tsc_weights(const double* __restrict__ p, int N, int (&c)[3], double (&w)[3][3])
{
    const double Nd = (double)N, inv = 1.0 / Nd;  // N is a power of two: s * inv is s / N exactly
#pragma unroll
    for (int ax = 0; ax < 3; ++ax) {
        double s = p[ax] * Nd;
        s = s - Nd * floor(s * inv);
        if (s >= Nd) s -= Nd;
        const double fl = floor(s);
        const double d = s - fl - 0.5;
        c[ax] = (int)fl & (N - 1);
        const double tl = 0.5 - d, tr = 0.5 + d;
        w[ax][0] = 0.5 * (tl * tl);
        w[ax][1] = 0.75 - d * d;
        w[ax][2] = 0.5 * (tr * tr);
    }
}

// Key (flat index of the nearest cell) and identity index of every particle.
__global__ void __launch_bounds__(kB) k_tsc_keys(const double* __restrict__ pos, long long np, int N, int lg,
                                                 unsigned* __restrict__ key, unsigned* __restrict__ idx)
{
    const long long p = (long long)blockIdx.x * kB + threadIdx.x;
    if (p >= np) return;
    int c[3];
    double w[3][3];
    tsc_weights(pos + 3 * p, N, c, w);
    key[p] = ((unsigned)c[0] << (2 * lg)) | ((unsigned)c[1] << lg) | (unsigned)c[2];
    idx[p] = (unsigned)p;
}

// Offsets d (x, y, z) of the particles from their nearest cell centre, in key order: the
// weights of a particle follow from d alone, and its nearest cell from its key.
__global__ void __launch_bounds__(kB) k_tsc_gather(const double* __restrict__ pos, const unsigned* __restrict__ idx,
                                                   long long np, int N, double* __restrict__ dsorted)
{
    const long long t = (long long)blockIdx.x * kB + threadIdx.x;
    if (t >= np) return;
    const long long p = idx[t];
    const double Nd = (double)N, inv = 1.0 / Nd;
#pragma unroll
    for (int ax = 0; ax < 3; ++ax) {
        double s = pos[3 * p + ax] * Nd;
        s = s - Nd * floor(s * inv);
        if (s >= Nd) s -= Nd;
        dsorted[3 * t + ax] = s - floor(s) - 0.5;
    }
}

// The TSC weight of offset o in {0, 1, 2} (cells -1, 0, +1 from the nearest) at offset d.
__device__ __forceinline__ double tsc_w(double d, int o)
{
    if (o == 1) return 0.75 - d * d;
    const double t = o == 0 ? 0.5 - d : 0.5 + d;
    return 0.5 * (t * t);
}

// start[c] = first position in key order of a particle with key >= c, for c = 0 .. ncell
// (start[ncell] = np): the particles of cell c are start[c] .. start[c+1] - 1.
__global__ void __launch_bounds__(kB) k_tsc_cell_start(const unsigned* __restrict__ key, long long np,
                                                       long long ncell, unsigned* __restrict__ start)
{
    const long long t = (long long)blockIdx.x * kB + threadIdx.x;
    if (t >= np) return;
    const long long k = key[t];
    const long long prev = t > 0 ? (long long)key[t - 1] : -1;
    for (long long c = prev + 1; c <= k; ++c) start[c] = (unsigned)t;
    if (t == np - 1)
        for (long long c = k + 1; c <= ncell; ++c) start[c] = (unsigned)np;
}

__global__ void __launch_bounds__(kB) k_tsc_fill_start(unsigned* __restrict__ start, long long n)
{
    const long long t = (long long)blockIdx.x * kB + threadIdx.x;
    if (t < n) start[t] = 0u;
}

// Density of cell (i,j,k): the sum over the particles whose nearest cell is (i+a, j+b, k+c),
// a, b, c in {-1, 0, 1}, of mass x their weight for offset (-a, -b, -c).  A workgroup owns a
// segment of S = min(N, kB) cells of one row.  For each of the 9 neighbour rows (a, b) in
// turn:
//  - the particles of the source cells k0-1 .. k0+S of that row are taken kCH at a time, in
//    up to three key ranges: the wrapped cell N-1 (when k0 = 0), the cells
//    max(k0-1, 0) .. min(k0+S, N-1), the wrapped cell 0 (when k0 + S = N); every thread
//    evaluates mass x w_x(-a) x w_y(-b) x w_z(o) for the three z offsets o of its particles
//    of the chunk into LDS, so that the weights cost the same in every lane;
//  - one thread per source cell sums those terms over the cell's particles in key order
//    (three moments, kept in LDS);
//  - every cell adds the moments of its source cells k-1, k, k+1 for the offsets that reach
//    it.
// Each particle's weights are evaluated once per neighbour row rather than once per target
// cell, and the serial walk over a dense cell's particles is one lane's three additions per
// particle.  The order of
// every sum is fixed, so the density is the same bits on every call.
constexpr int kCH = 512;

__global__ void __launch_bounds__(kB) k_tsc_density(const double* __restrict__ dsorted,
                                                    const unsigned* __restrict__ start, int N, int lg, double mass,
                                                    double* __restrict__ rho)
{
    __shared__ double cw[3][kCH];                // per particle of the chunk: its three terms
    __shared__ double mom[3][kB + 2];            // moments of source cell k0-1+sc for z offsets 0, 1, 2
    const int m = N - 1;
    const int S = N < kB ? N : kB;               // cells per segment
    const int nseg = N / S;                      // segments per row
    const long long wg = xcd_block();
    const long long rowid = wg / nseg;           // (i, j)
    const int k0 = (int)(wg % nseg) * S;
    const int i = (int)(rowid >> lg), j = (int)(rowid & m);
    const int tid = threadIdx.x;
    const bool live = tid < S;
    double sum = 0.0;
    for (int ab = 0; ab < 9; ++ab) {
        const int a = ab / 3 - 1, b = ab % 3 - 1;
        const unsigned row = ((unsigned)((i + a) & m) << (2 * lg)) | ((unsigned)((j + b) & m) << lg);
        // the source cells of this thread (slots tid and tid + kB): particle range and the
        // key range (0, 1, 2 as above; -1 none) that holds it
        unsigned lo[2], hi[2];
        int rg[2];
        double mm[2][3];
#pragma unroll
        for (int q = 0; q < 2; ++q) {
            const int sc = tid + q * kB;
            lo[q] = hi[q] = 0;
            rg[q] = -1;
            if (sc < S + 2) {
                const unsigned key = row | (unsigned)((k0 - 1 + sc) & m);
                lo[q] = start[key];
                hi[q] = start[key + 1];
                rg[q] = (sc == 0 && k0 == 0) ? 0 : (sc == S + 1 && k0 + S == N) ? 2 : 1;
            }
            mm[q][0] = mm[q][1] = mm[q][2] = 0.0;
        }
        for (int sg = 0; sg < 3; ++sg) {
            unsigned g0, g1;
            if (sg == 0) {
                if (k0 != 0) continue;
                g0 = start[row + N - 1];
                g1 = start[row + N];
            } else if (sg == 1) {
                g0 = start[row + (k0 > 0 ? k0 - 1 : 0)];
                g1 = start[row + (k0 + S < N ? k0 + S + 1 : N)];
            } else {
                if (k0 + S != N) continue;
                g0 = start[row];
                g1 = start[row + 1];
            }
            for (unsigned c0 = g0; c0 < g1; c0 += kCH) {
                const unsigned c1 = c0 + kCH < g1 ? c0 + kCH : g1;
                __syncthreads();
                for (unsigned t = c0 + tid; t < c1; t += kB) {
                    const double* d = dsorted + 3 * (long long)t;
                    const double wxy = mass * tsc_w(d[0], 1 - a) * tsc_w(d[1], 1 - b);
                    const double dz = d[2];
                    cw[0][t - c0] = wxy * tsc_w(dz, 0);
                    cw[1][t - c0] = wxy * tsc_w(dz, 1);
                    cw[2][t - c0] = wxy * tsc_w(dz, 2);
                }
                __syncthreads();
#pragma unroll
                for (int q = 0; q < 2; ++q) {
                    if (rg[q] != sg) continue;
                    const unsigned t0 = lo[q] > c0 ? lo[q] : c0, t1 = hi[q] < c1 ? hi[q] : c1;
                    for (unsigned t = t0; t < t1; ++t) {
                        const unsigned l = t - c0;
                        mm[q][0] = mm[q][0] + cw[0][l];
                        mm[q][1] = mm[q][1] + cw[1][l];
                        mm[q][2] = mm[q][2] + cw[2][l];
                    }
                }
            }
        }
#pragma unroll
        for (int q = 0; q < 2; ++q) {
            const int sc = tid + q * kB;
            if (sc < S + 2) {
                mom[0][sc] = mm[q][0];
                mom[1][sc] = mm[q][1];
                mom[2][sc] = mm[q][2];
            }
        }
        __syncthreads();
        // source cells k-1, k, k+1 are slots tid, tid+1, tid+2; they reach cell k with the
        // z weights of offsets +1, 0, -1 (o = 2, 1, 0)
        if (live) {
            sum = sum + mom[2][tid];
            sum = sum + mom[1][tid + 1];
            sum = sum + mom[0][tid + 2];
        }
        __syncthreads();  // the next row rewrites mom (it may stage nothing before that)
    }
    if (live) rho[((long long)rowid << lg) + k0 + tid] = sum;
}

// acc = sum over the 27 cells of weight x (-grad phi), -grad phi by central differences.
__global__ void __launch_bounds__(kB) k_tsc_force(const double* __restrict__ phi, int N, int lg,
                                                  const double* __restrict__ pos, long long np,
                                                  double* __restrict__ acc)
{
    const long long p = xcd_block() * kB + threadIdx.x;
    if (p >= np) return;
    int c[3];
    double w[3][3];
    tsc_weights(pos + 3 * p, N, c, w);
    const int m = N - 1;
    const double half = (double)N / 2.0;
    // offsets of the planes c0-2 .. c0+2, rows c1-2 .. c1+2 and columns c2-2 .. c2+2
    unsigned pi[5], rj[5], ck[5];
#pragma unroll
    for (int t = 0; t < 5; ++t) {
        pi[t] = (unsigned)((c[0] + t - 2) & m) << (2 * lg);
        rj[t] = (unsigned)((c[1] + t - 2) & m) << lg;
        ck[t] = (unsigned)((c[2] + t - 2) & m);
    }
    double fx = 0.0, fy = 0.0, fz = 0.0;
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int b = 0; b < 3; ++b)
#pragma unroll
            for (int z = 0; z < 3; ++z) {
                // cell (c0 + a - 1, c1 + b - 1, c2 + z - 1) is index a+1, b+1, z+1 of the 5-wide ranges
                const double wt = w[0][a] * w[1][b] * w[2][z];
                const double gx = -(phi[pi[a + 2] + rj[b + 1] + ck[z + 1]] - phi[pi[a] + rj[b + 1] + ck[z + 1]]) * half;
                const double gy = -(phi[pi[a + 1] + rj[b + 2] + ck[z + 1]] - phi[pi[a + 1] + rj[b] + ck[z + 1]]) * half;
                const double gz = -(phi[pi[a + 1] + rj[b + 1] + ck[z + 2]] - phi[pi[a + 1] + rj[b + 1] + ck[z]]) * half;
                fx = fx + wt * gx;
                fy = fy + wt * gy;
                fz = fz + wt * gz;
            }
    acc[3 * p] = fx;
    acc[3 * p + 1] = fy;
    acc[3 * p + 2] = fz;
}

#pragma clang fp contract(fast)

inline unsigned blocks(long long n) { return (unsigned)((n + kB - 1) / kB); }

int check_args(mgfr_ctx* c, const double* pos, long long np, int N)
{
    if (!is_pow2(N) || N < 4 || N > 1024) return c->fail(MGFR_EINVAL, "N=%d must be a power of two in [4, 1024]", N);
    if (np < 0 || np > (1LL << 36)) return c->fail(MGFR_EINVAL, "particle count %lld out of range", np);
    if (np > 0 && !pos) return c->fail(MGFR_EINVAL, "pos is NULL");
    return MGFR_OK;
}

// Non-finite positions would give arbitrary cells: refuse them (synchronises).
int check_positions(mgfr_ctx* c, const double* pos, long long np, hipStream_t s)
{
    if (np == 0) return MGFR_OK;
    MGFR_TRY(ensure_scratch(c));
    MGFR_TRY(hip_check(c, sum_and_count_nonfinite(pos, 3 * np, c->partial, c->red, s), "position check"));
    double r[2];
    MGFR_TRY(read_reduction(c, s, r));
    if (r[1] != 0.0) return c->fail(MGFR_ENONFINITE, "%.0f non-finite particle coordinates", r[1]);
    return MGFR_OK;
}

}  // namespace
}  // namespace mgfr

extern "C" {

int mgfr_tsc_density(mgfr_ctx* c, const double* pos, long long np, int N, double mass, double* rho, void* stream)
{
    if (!c) return MGFR_EINVAL;
    c->err.clear();
    MGFR_TRY(mgfr::check_args(c, pos, np, N));
    if (np >= (1LL << 31)) return c->fail(MGFR_EINVAL, "assignment takes at most 2^31 - 1 particles (%lld)", np);
    if (!rho) return c->fail(MGFR_EINVAL, "rho is NULL");
    if (!std::isfinite(mass)) return c->fail(MGFR_EINVAL, "mass must be finite");
    MGFR_TRY(hip_check(c, hipSetDevice(c->device), "hipSetDevice"));
    hipStream_t s = (hipStream_t)stream;
    MGFR_TRY(mgfr::check_positions(c, pos, np, s));
    const int lg = ilog2(N);
    const long long ncell = (long long)N * N * N;
    // scratch: keys and indices (twice, for the sort), positions in key order, cell starts,
    // sort temporary storage -- one block kept in the context
    auto al = [](size_t b) { return (b + 255) & ~(size_t)255; };
    size_t tmp_bytes = 0;
    if (np > 0)
        MGFR_TRY(hip_check(c, rocprim::radix_sort_pairs(nullptr, tmp_bytes, (unsigned*)nullptr, (unsigned*)nullptr,
                                                        (unsigned*)nullptr, (unsigned*)nullptr, (size_t)np, 0, 3 * lg, s),
                           "radix_sort_pairs (size query)"));
    const size_t ub = al(sizeof(unsigned) * (size_t)np);
    const size_t need = 4 * ub + al(sizeof(double) * 3 * (size_t)np) + al(sizeof(unsigned) * (size_t)(ncell + 1)) +
                        al(tmp_bytes);
    if (c->tsc_bytes < need) {
        (void)hipStreamSynchronize(s);
        (void)hipFree(c->tsc);
        c->tsc = nullptr;
        c->tsc_bytes = 0;
        if (hipMalloc(&c->tsc, need) != hipSuccess) return c->fail(MGFR_ENOMEM, "hipMalloc of %zu bytes failed", need);
        c->tsc_bytes = need;
    }
    char* b = (char*)c->tsc;
    unsigned* key = (unsigned*)b;
    unsigned* key2 = (unsigned*)(b + ub);
    unsigned* idx = (unsigned*)(b + 2 * ub);
    unsigned* idx2 = (unsigned*)(b + 3 * ub);
    double* sorted = (double*)(b + 4 * ub);
    unsigned* start = (unsigned*)(b + 4 * ub + al(sizeof(double) * 3 * (size_t)np));
    void* tmp = b + 4 * ub + al(sizeof(double) * 3 * (size_t)np) + al(sizeof(unsigned) * (size_t)(ncell + 1));
    if (np > 0) {
        hipLaunchKernelGGL(mgfr::k_tsc_keys, dim3(mgfr::blocks(np)), dim3(mgfr::kB), 0, s, pos, np, N, lg, key, idx);
        MGFR_TRY(hip_check(c, hipGetLastError(), "k_tsc_keys"));
        MGFR_TRY(hip_check(c, rocprim::radix_sort_pairs(tmp, tmp_bytes, key, key2, idx, idx2, (size_t)np, 0, 3 * lg, s),
                           "radix_sort_pairs"));
        hipLaunchKernelGGL(mgfr::k_tsc_gather, dim3(mgfr::blocks(np)), dim3(mgfr::kB), 0, s, pos, idx2, np, N, sorted);
        MGFR_TRY(hip_check(c, hipGetLastError(), "k_tsc_gather"));
        hipLaunchKernelGGL(mgfr::k_tsc_cell_start, dim3(mgfr::blocks(np)), dim3(mgfr::kB), 0, s, key2, np, ncell, start);
        MGFR_TRY(hip_check(c, hipGetLastError(), "k_tsc_cell_start"));
    } else {
        hipLaunchKernelGGL(mgfr::k_tsc_fill_start, dim3(mgfr::blocks(ncell + 1)), dim3(mgfr::kB), 0, s, start, ncell + 1);
        MGFR_TRY(hip_check(c, hipGetLastError(), "k_tsc_fill_start"));
    }
    const long long segs = (long long)N * N * (N < mgfr::kB ? 1 : N / mgfr::kB);
    hipLaunchKernelGGL(mgfr::k_tsc_density, dim3((unsigned)segs), dim3(mgfr::kB), 0, s, sorted, start, N, lg, mass, rho);
    MGFR_TRY(hip_check(c, hipGetLastError(), "k_tsc_density"));
    return MGFR_OK;
}

int mgfr_tsc_force(mgfr_ctx* c, const double* phi, int N, const double* pos, long long np, double* acc, void* stream)
{
    if (!c) return MGFR_EINVAL;
    c->err.clear();
    MGFR_TRY(mgfr::check_args(c, pos, np, N));
    if (!phi || (np > 0 && !acc)) return c->fail(MGFR_EINVAL, "phi or acc is NULL");
    MGFR_TRY(hip_check(c, hipSetDevice(c->device), "hipSetDevice"));
    hipStream_t s = (hipStream_t)stream;
    MGFR_TRY(mgfr::check_positions(c, pos, np, s));
    if (np > 0) {
        hipLaunchKernelGGL(mgfr::k_tsc_force, dim3(mgfr::blocks(np)), dim3(mgfr::kB), 0, s, phi, N, ilog2(N), pos, np,
                           acc);
        MGFR_TRY(hip_check(c, hipGetLastError(), "k_tsc_force"));
    }
    return MGFR_OK;
}

}  // extern "C"
