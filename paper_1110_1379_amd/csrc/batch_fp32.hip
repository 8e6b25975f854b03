// Batched single-precision correction kernels of the mixed-precision patch and box solves.
//
// Same batching as batch_fp64.hip (one launch per multigrid depth over every unit, a block
// table of (unit grid, block) pairs, per-unit active flags), applied to the correction
// equation N(e) = r of device_fp32.h; the correction form of a patch's ghost faces is in
// batch_dev.h.
#include "batch_dev.h"

namespace mgfr {
namespace {

using namespace bdev;

constexpr int kB = 256;

// ---- smoother: one colour per launch, one thread per cell of that colour ------------------
__global__ void __launch_bounds__(kB) kb32_ngs(BTable t, int colour)
{
    const int2 b = t.blk[blockIdx.x];
    const BGrid g = t.grids[b.x];
    if (!live(t, g)) return;
    const long long half = 1LL << (3 * g.lg - 1);
    const long long tt = (long long)b.y * kB + threadIdx.x;
    if (tt >= half) return;
    const int hk = g.n >> 1;
    const int s = (int)(tt & (hk - 1));
    const long long row = tt >> (g.lg - 1);
    const int i = (int)(row >> g.lg), j = (int)(row & (g.n - 1));
    const int k = 2 * s + ((i + j + colour) & 1);
    const long long q = idx3(g.lg, i, j, k);
    const Op32 o = op32(g);
    const Res32 r = bcell32(g, o, g.ub32, g.e32, i, j, k, g.f32[q]);
    g.e32[q] = g.e32[q] + newton32(r, o.max_step);
}

// ---- residual + restriction (table over the coarse cells; tc = coarse grids) -------------
__global__ void __launch_bounds__(kB) kb32_resid_restrict(BTable t, const BGrid* __restrict__ tc)
{
    const int2 b = t.blk[blockIdx.x];
    const BGrid g = t.grids[b.x];
    if (!live(t, g)) return;
    const BGrid c = tc[b.x];
    const long long qc = (long long)b.y * kB + threadIdx.x;
    if (qc >= (1LL << (3 * c.lg))) return;
    const int I = (int)(qc >> (2 * c.lg)), J = (int)((qc >> c.lg) & (c.n - 1)), K = (int)(qc & (c.n - 1));
    const Op32 o = op32(g);
    float se = 0.0f, sd = 0.0f;
    for (int a = 0; a < 2; ++a)
        for (int bb = 0; bb < 2; ++bb)
            for (int z = 0; z < 2; ++z) {
                const int i = 2 * I + a, j = 2 * J + bb, k = 2 * K + z;
                const long long q = idx3(g.lg, i, j, k);
                se += g.e32[q];
                sd += bcell32(g, o, g.ub32, g.e32, i, j, k, g.f32[q]).N;
            }
    c.e32[qc] = 0.125f * se;
    c.eh32[qc] = 0.125f * se;
    c.f32[qc] = 0.125f * sd;
}

// coarse base R ub (table over the coarse cells; tc = coarse grids)
__global__ void __launch_bounds__(kB) kb32_restrict_base(BTable t, const BGrid* __restrict__ tc)
{
    const int2 b = t.blk[blockIdx.x];
    const BGrid g = t.grids[b.x];
    if (!live(t, g)) return;
    const BGrid c = tc[b.x];
    const long long qc = (long long)b.y * kB + threadIdx.x;
    if (qc >= (1LL << (3 * c.lg))) return;
    const int I = (int)(qc >> (2 * c.lg)), J = (int)((qc >> c.lg) & (c.n - 1)), K = (int)(qc & (c.n - 1));
    float s = 0.0f;
    for (int a = 0; a < 2; ++a)
        for (int bb = 0; bb < 2; ++bb)
            for (int z = 0; z < 2; ++z) s += g.ub32[idx3(g.lg, 2 * I + a, 2 * J + bb, 2 * K + z)];
    c.ub32[qc] = 0.125f * s;
}

// f = N^H(eh) - f on coarse grids (f holds R d on entry)
__global__ void __launch_bounds__(kB) kb32_fas_rhs(BTable t)
{
    const int2 b = t.blk[blockIdx.x];
    const BGrid c = t.grids[b.x];
    if (!live(t, c)) return;
    const long long q = (long long)b.y * kB + threadIdx.x;
    if (q >= (1LL << (3 * c.lg))) return;
    const int i = (int)(q >> (2 * c.lg)), j = (int)((q >> c.lg) & (c.n - 1)), k = (int)(q & (c.n - 1));
    c.f32[q] = bcell32(c, op32(c), c.ub32, c.eh32, i, j, k, 0.0f).N - c.f32[q];
}

__global__ void __launch_bounds__(kB) kb32_coarse_diff(BTable t)
{
    const int2 b = t.blk[blockIdx.x];
    const BGrid c = t.grids[b.x];
    if (!live(t, c)) return;
    const long long q = (long long)b.y * kB + threadIdx.x;
    if (q >= (1LL << (3 * c.lg))) return;
    c.eh32[q] = c.e32[q] - c.eh32[q];
}

// e += P(coarse difference) on fine grids, as kb_prolong_add8 (outside a patch a coarse cell
// contributes zero, Sec. V.A.3): one thread per coarse cell and its eight fine cells.
__global__ void __launch_bounds__(kB) kb32_prolong_add8(BTable t, const BGrid* __restrict__ tc)
{
    const int2 b = t.blk[blockIdx.x];
    const BGrid g = t.grids[b.x];
    if (!live(t, g)) return;
    const BGrid c = tc[b.x];
    const long long qc = (long long)b.y * kB + threadIdx.x;
    if (qc >= (1LL << (3 * c.lg))) return;
    const int mc = c.n - 1;
    const int I = (int)(qc >> (2 * c.lg)), J = (int)((qc >> c.lg) & mc), K = (int)(qc & mc);
    auto E = [&](int a, int bb, int z) -> float {
        if (c.periodic) return c.eh32[idx3(c.lg, a & mc, bb & mc, z & mc)];
        if (a < 0 || a > mc || bb < 0 || bb > mc || z < 0 || z > mc) return 0.0f;
        return c.eh32[idx3(c.lg, a, bb, z)];
    };
    float v[3][3][3];
#pragma unroll
    for (int x = 0; x < 3; ++x)
#pragma unroll
        for (int y = 0; y < 3; ++y)
#pragma unroll
            for (int z = 0; z < 3; ++z) v[x][y][z] = E(I + x - 1, J + y - 1, K + z - 1);
#pragma unroll
    for (int x = 0; x < 2; ++x)
#pragma unroll
        for (int y = 0; y < 2; ++y)
#pragma unroll
            for (int z = 0; z < 2; ++z) {
                const int si = x ? 2 : 0, sj = y ? 2 : 0, sk = z ? 2 : 0;  // index of I + s
                const float p = (27.0f / 64.0f) * v[1][1][1] +
                                (9.0f / 64.0f) * (v[si][1][1] + v[1][sj][1] + v[1][1][sk]) +
                                (3.0f / 64.0f) * (v[si][sj][1] + v[si][1][sk] + v[1][sj][sk]) +
                                (1.0f / 64.0f) * v[si][sj][sk];
                const long long q = idx3(g.lg, 2 * I + x, 2 * J + y, 2 * K + z);
                g.e32[q] += p;
            }
}

// ---- coarsest level: one workgroup per grid (n <= 8) --------------------------------------
template <int NT>
__global__ void __launch_bounds__(NT) kb32_coarsest(const BGrid* __restrict__ grids, const int* __restrict__ active,
                                                   int cap, float rtol)
{
    __shared__ Coarse32<NT> sm;
    const BGrid g = grids[blockIdx.x];
    if (active && !active[g.unit]) return;
    coarsest32<NT>(g, cap, rtol, sm);
}

}  // namespace

hipError_t batch_restrict_base32(const BTable& t, int nblk, const BGrid* coarse, hipStream_t s)
{
    hipLaunchKernelGGL(kb32_restrict_base, dim3(nblk), dim3(kB), 0, s, t, coarse);
    return hipGetLastError();
}
hipError_t batch_ngs32(const BTable& t, int nblk, hipStream_t s)
{
    for (int colour = 0; colour < 2; ++colour) hipLaunchKernelGGL(kb32_ngs, dim3(nblk), dim3(kB), 0, s, t, colour);
    return hipGetLastError();
}
hipError_t batch_resid_restrict32(const BTable& t, int nblk, const BGrid* coarse, hipStream_t s)
{
    hipLaunchKernelGGL(kb32_resid_restrict, dim3(nblk), dim3(kB), 0, s, t, coarse);
    return hipGetLastError();
}
hipError_t batch_fas_rhs32(const BTable& t, int nblk, hipStream_t s)
{
    hipLaunchKernelGGL(kb32_fas_rhs, dim3(nblk), dim3(kB), 0, s, t);
    return hipGetLastError();
}
hipError_t batch_coarse_diff32(const BTable& t, int nblk, hipStream_t s)
{
    hipLaunchKernelGGL(kb32_coarse_diff, dim3(nblk), dim3(kB), 0, s, t);
    return hipGetLastError();
}
hipError_t batch_prolong_add8_32(const BTable& t, int nblk, const BGrid* coarse, hipStream_t s)
{
    hipLaunchKernelGGL(kb32_prolong_add8, dim3(nblk), dim3(kB), 0, s, t, coarse);
    return hipGetLastError();
}
hipError_t batch_coarsest32(const BGrid* grids, int ngrid, int n, const int* active, int cap, double rtol,
                            hipStream_t s)
{
    // one wavefront per grid when it fits (barriers and reductions stay within the wave)
    if (n <= 4)
        hipLaunchKernelGGL((kb32_coarsest<64>), dim3(ngrid), dim3(64), 0, s, grids, active, cap, (float)rtol);
    else
        hipLaunchKernelGGL((kb32_coarsest<kB>), dim3(ngrid), dim3(kB), 0, s, grids, active, cap, (float)rtol);
    return hipGetLastError();
}

}  // namespace mgfr
