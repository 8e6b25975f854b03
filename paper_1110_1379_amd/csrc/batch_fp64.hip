// Batched double-precision multigrid kernels: many independent units (refinement patches
// or periodic boxes) of uneven sizes, each launch covering every unit of one multigrid
// depth.  A block table maps each workgroup to (unit grid, block within that grid); units
// whose solve has converged are switched off through a per-unit flag and their workgroups
// return at once.
// The cell operator of a unit grid (cube patch with ghost faces, or periodic box) is in
// batch_dev.h.
#include "batch_dev.h"

namespace mgfr {
namespace {

constexpr int kB = 256;

using namespace bdev;

// ---- smoother ---------------------------------------------------------------------------
__global__ void __launch_bounds__(kB) kb_ngs(BTable t, int colour)
{
    const int2 e = t.blk[blockIdx.x];
    const BGrid g = t.grids[e.x];
    if (!live(t, g)) return;
    const long long half = 1LL << (3 * g.lg - 1);
    const long long tt = (long long)e.y * kB + threadIdx.x;
    if (tt >= half) return;
    const int hk = g.n >> 1;
    const int s = (int)(tt & (hk - 1));
    const long long row = tt >> (g.lg - 1);
    const int i = (int)(row >> g.lg), j = (int)(row & (g.n - 1));
    const int k = 2 * s + ((i + j + colour) & 1);
    const long long q = idx3(g.lg, i, j, k);
    const OpVal r = bcell(g, g.u, i, j, k, brhs(g, q));
    g.u[q] = g.u[q] + dev::bounded(-r.L / r.dL, g.max_step);
}

// ---- residual + restriction (table over the coarse cells; tc = coarse grids) -------------
__global__ void __launch_bounds__(kB) kb_resid_restrict(BTable t, const BGrid* __restrict__ tc)
{
    const int2 e = t.blk[blockIdx.x];
    const BGrid g = t.grids[e.x];
    if (!live(t, g)) return;
    const BGrid c = tc[e.x];
    const long long qc = (long long)e.y * kB + threadIdx.x;
    if (qc >= (1LL << (3 * c.lg))) return;
    const int I = (int)(qc >> (2 * c.lg)), J = (int)((qc >> c.lg) & (c.n - 1)), K = (int)(qc & (c.n - 1));
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

// f = L^H(uhat) - f on coarse grids (table over their cells)
__global__ void __launch_bounds__(kB) kb_fas_rhs(BTable t)
{
    const int2 e = t.blk[blockIdx.x];
    const BGrid c = t.grids[e.x];
    if (!live(t, c)) return;
    const long long q = (long long)e.y * kB + threadIdx.x;
    if (q >= (1LL << (3 * c.lg))) return;
    const int i = (int)(q >> (2 * c.lg)), j = (int)((q >> c.lg) & (c.n - 1)), k = (int)(q & (c.n - 1));
    c.f[q] = bcell(c, c.uhat, i, j, k, 0.0).L - c.f[q];
}

__global__ void __launch_bounds__(kB) kb_coarse_diff(BTable t)
{
    const int2 e = t.blk[blockIdx.x];
    const BGrid c = t.grids[e.x];
    if (!live(t, c)) return;
    const long long q = (long long)e.y * kB + threadIdx.x;
    if (q >= (1LL << (3 * c.lg))) return;
    c.uhat[q] = c.u[q] - c.uhat[q];
}

// u += P(e) on fine grids, trilinear (27/9/3/1 over the eight nearest coarse centres; tc =
// coarse grids holding e in uhat).  Outside a patch a coarse cell is not a multigrid cell and
// contributes zero (Sec. V.A.3).  A table of coarse cells (blocks of the fine grids' cells /
// 8): one thread per coarse cell adds the correction to its eight fine cells, from the
// 3 x 3 x 3 coarse values around it loaded once (a fine cell's interpolation reads 8 of
// them); consecutive threads write consecutive pairs of fine cells along k.
__global__ void __launch_bounds__(kB) kb_prolong_add8(BTable t, const BGrid* __restrict__ tc)
{
    const int2 e = t.blk[blockIdx.x];
    const BGrid g = t.grids[e.x];
    if (!live(t, g)) return;
    const BGrid c = tc[e.x];
    const long long qc = (long long)e.y * kB + threadIdx.x;
    if (qc >= (1LL << (3 * c.lg))) return;
    const int mc = c.n - 1;
    const int I = (int)(qc >> (2 * c.lg)), J = (int)((qc >> c.lg) & mc), K = (int)(qc & mc);
    auto E = [&](int a, int b, int z) -> double {
        if (c.periodic) return c.uhat[idx3(c.lg, a & mc, b & mc, z & mc)];
        if (a < 0 || a > mc || b < 0 || b > mc || z < 0 || z > mc) return 0.0;
        return c.uhat[idx3(c.lg, a, b, z)];
    };
    double v[3][3][3];
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
                const double p = (27.0 / 64.0) * v[1][1][1] +
                                 (9.0 / 64.0) * (v[si][1][1] + v[1][sj][1] + v[1][1][sk]) +
                                 (3.0 / 64.0) * (v[si][sj][1] + v[si][1][sk] + v[1][sj][sk]) +
                                 (1.0 / 64.0) * v[si][sj][sk];
                const long long q = idx3(g.lg, 2 * I + x, 2 * J + y, 2 * K + z);
                g.u[q] += p;
            }
}

// ---- coarsest level: one workgroup per grid (n <= 8) --------------------------------------
template <int NT>
__global__ void __launch_bounds__(NT) kb_coarsest(const BGrid* __restrict__ grids, const int* __restrict__ active,
                                                 int cap, double rtol)
{
    __shared__ Coarse64<NT> sm;
    const BGrid g = grids[blockIdx.x];
    if (active && !active[g.unit]) return;
    coarsest64<NT>(g, cap, rtol, sm);
}

// ---- per-grid residual norms -------------------------------------------------------------
__global__ void __launch_bounds__(kB) kb_norm(BTable t, double* __restrict__ partial)
{
    __shared__ double ra[kB], rb[kB];
    const int2 e = t.blk[blockIdx.x];
    const BGrid g = t.grids[e.x];
    double s = 0.0, mx = 0.0;
    const long long q = (long long)e.y * kB + threadIdx.x;
    if (live(t, g) && q < (1LL << (3 * g.lg))) {
        const int i = (int)(q >> (2 * g.lg)), j = (int)((q >> g.lg) & (g.n - 1)), k = (int)(q & (g.n - 1));
        const double d = bcell(g, g.u, i, j, k, brhs(g, q)).L;
        s = d * d;
        mx = fabs(d);
    }
    ra[threadIdx.x] = s;
    rb[threadIdx.x] = mx;
    __syncthreads();
    for (int w = kB / 2; w > 0; w >>= 1) {
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

// one workgroup per grid: fold its contiguous block partials [first[g], first[g] + count[g])
__global__ void __launch_bounds__(kB) kb_fold(const double* __restrict__ partial, const int* __restrict__ first,
                                             const int* __restrict__ count, double* __restrict__ out)
{
    __shared__ double ra[kB], rb[kB];
    const int g = blockIdx.x;
    double s = 0.0, mx = 0.0;
    for (int b = threadIdx.x; b < count[g]; b += kB) {
        s += partial[2 * (first[g] + b)];
        const double o = partial[2 * (first[g] + b) + 1];
        if (!(mx >= o)) mx = o;
    }
    ra[threadIdx.x] = s;
    rb[threadIdx.x] = mx;
    __syncthreads();
    for (int w = kB / 2; w > 0; w >>= 1) {
        if (threadIdx.x < w) {
            ra[threadIdx.x] += ra[threadIdx.x + w];
            const double o = rb[threadIdx.x + w];
            if (!(rb[threadIdx.x] >= o)) rb[threadIdx.x] = o;
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        out[2 * g] = ra[0];
        out[2 * g + 1] = rb[0];
    }
}

// ---- patch set-up from the parent level ----------------------------------------------------
__device__ double parent_at(const PatchParent& p, int I, int J, int K)
{
    if (p.periodic) {
        const int m = p.n - 1;
        return p.u[idx3(p.lg, I & m, J & m, K & m)];
    }
    return p.u[idx3(p.lg, I, J, K)];
}

// trilinear 27/9/3/1 interpolation of the parent u at child-level global cell (x, y, z)
__device__ double parent_interp(const PatchParent& p, int x, int y, int z)
{
    const int I = (x >> 1) - p.origin[0], J = (y >> 1) - p.origin[1], K = (z >> 1) - p.origin[2];
    const int si = (x & 1) ? 1 : -1, sj = (y & 1) ? 1 : -1, sk = (z & 1) ? 1 : -1;
    return (27.0 / 64.0) * parent_at(p, I, J, K) +
           (9.0 / 64.0) * (parent_at(p, I + si, J, K) + parent_at(p, I, J + sj, K) + parent_at(p, I, J, K + sk)) +
           (3.0 / 64.0) * (parent_at(p, I + si, J + sj, K) + parent_at(p, I + si, J, K + sk) +
                           parent_at(p, I, J + sj, K + sk)) +
           (1.0 / 64.0) * parent_at(p, I + si, J + sj, K + sk);
}

// table over (6 + 1) n^2 columns per patch: item w < n^2 fills a column of the interior
// initial guess (n cells along i); items n^2 .. 7 n^2 fill the face boundary values.
__global__ void __launch_bounds__(kB) kb_setup(BTable t, const PatchParent* __restrict__ parents)
{
    const int2 e = t.blk[blockIdx.x];
    const BGrid g = t.grids[e.x];
    const PatchParent p = parents[e.x];
    const long long w = (long long)e.y * kB + threadIdx.x;
    const int n = g.n, n2 = n * n;
    if (w >= 7LL * n2) return;
    if (w < n2) {
        const int j = (int)(w / n), k = (int)(w % n);
        for (int i = 0; i < n; ++i)
            g.u[idx3(g.lg, i, j, k)] = parent_interp(p, p.child[0] + i, p.child[1] + j, p.child[2] + k);
        return;
    }
    const int f = (int)((w - n2) / n2), r = (int)((w - n2) % n2), a = r / n, b = r % n;
    int ci, cj, ck;
    if (f < 2) { ci = f == 0 ? 0 : n - 1; cj = a; ck = b; }
    else if (f < 4) { ci = a; cj = f == 2 ? 0 : n - 1; ck = b; }
    else { ci = a; cj = b; ck = f == 4 ? 0 : n - 1; }
    const int gi = ci + (f == 0 ? -1 : f == 1 ? 1 : 0), gj = cj + (f == 2 ? -1 : f == 3 ? 1 : 0),
              gk = ck + (f == 4 ? -1 : f == 5 ? 1 : 0);
    const double ug = parent_interp(p, p.child[0] + gi, p.child[1] + gj, p.child[2] + gk);
    const double ui = parent_interp(p, p.child[0] + ci, p.child[1] + cj, p.child[2] + ck);
    // eq. u_i-1jk solved for u_b
    g.ub[((long long)f * n + a) * n + b] = (ug - kR * ui) / (1.0 - kR);
}

// coarse boundary values: mean of the 4 fine ones on the same face (table over 6 nc^2 items
// of the coarse grids; tf = the fine grids)
__global__ void __launch_bounds__(kB) kb_restrict_faces(BTable t, const BGrid* __restrict__ tf)
{
    const int2 e = t.blk[blockIdx.x];
    const BGrid c = t.grids[e.x];
    const BGrid g = tf[e.x];
    const long long w = (long long)e.y * kB + threadIdx.x;
    const int nc = c.n, n = g.n;
    if (w >= 6LL * nc * nc) return;
    const int f = (int)(w / (nc * nc)), r = (int)(w % (nc * nc)), P = r / nc, Q = r % nc;
    double s = 0.0;
    for (int a = 0; a < 2; ++a)
        for (int b = 0; b < 2; ++b) s += g.ub[((long long)f * n + 2 * P + a) * n + 2 * Q + b];
    c.ub[((long long)f * nc + P) * nc + Q] = 0.25 * s;
}

__global__ void __launch_bounds__(kB) kb_fill(BTable t)
{
    const int2 e = t.blk[blockIdx.x];
    const BGrid g = t.grids[e.x];
    const long long q = (long long)e.y * kB + threadIdx.x;
    if (q < (1LL << (3 * g.lg))) g.u[q] = g.u0;
}

// density check over every unit: sum of non-finite counts
__global__ void __launch_bounds__(kB) kb_nonfinite(BTable t, double* __restrict__ partial)
{
    __shared__ double ra[kB];
    const int2 e = t.blk[blockIdx.x];
    const BGrid g = t.grids[e.x];
    const long long q = (long long)e.y * kB + threadIdx.x;
    double c = 0.0;
    if (q < (1LL << (3 * g.lg))) {
        if (!isfinite(g.src[q]) || !isfinite(g.u[q])) c = 1.0;
    }
    ra[threadIdx.x] = c;
    __syncthreads();
    for (int w = kB / 2; w > 0; w >>= 1) {
        if (threadIdx.x < w) ra[threadIdx.x] += ra[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        partial[2 * blockIdx.x] = ra[0];
        partial[2 * blockIdx.x + 1] = 0.0;
    }
}

// ---- outer double-precision loop of the mixed solves --------------------------------------
// d = L(u) - f on finest grids: r = -d and ub = u in single precision, e = 0, and block
// partials of (sum d^2, max |d|) as kb_norm.
__global__ void __launch_bounds__(kB) kb_resid_cast(BTable t, double* __restrict__ partial)
{
    __shared__ double ra[kB], rb[kB];
    const int2 e = t.blk[blockIdx.x];
    const BGrid g = t.grids[e.x];
    double s = 0.0, mx = 0.0;
    const long long q = (long long)e.y * kB + threadIdx.x;
    if (live(t, g) && q < (1LL << (3 * g.lg))) {
        const int i = (int)(q >> (2 * g.lg)), j = (int)((q >> g.lg) & (g.n - 1)), k = (int)(q & (g.n - 1));
        const double d = bcell(g, g.u, i, j, k, brhs(g, q)).L;
        g.f32[q] = (float)(-d);
        g.ub32[q] = (float)g.u[q];
        g.e32[q] = 0.0f;
        s = d * d;
        mx = fabs(d);
    }
    ra[threadIdx.x] = s;
    rb[threadIdx.x] = mx;
    __syncthreads();
    for (int w = kB / 2; w > 0; w >>= 1) {
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

// u += e on finest grids
__global__ void __launch_bounds__(kB) kb_add_correction(BTable t)
{
    const int2 e = t.blk[blockIdx.x];
    const BGrid g = t.grids[e.x];
    if (!live(t, g)) return;
    const long long q = (long long)e.y * kB + threadIdx.x;
    if (q < (1LL << (3 * g.lg))) g.u[q] += (double)g.e32[q];
}

}  // namespace

int batch_block() { return kB; }

hipError_t batch_ngs(const BTable& t, int nblk, hipStream_t s)
{
    for (int colour = 0; colour < 2; ++colour) hipLaunchKernelGGL(kb_ngs, dim3(nblk), dim3(kB), 0, s, t, colour);
    return hipGetLastError();
}
hipError_t batch_resid_restrict(const BTable& t, int nblk, const BGrid* coarse, hipStream_t s)
{
    hipLaunchKernelGGL(kb_resid_restrict, dim3(nblk), dim3(kB), 0, s, t, coarse);
    return hipGetLastError();
}
hipError_t batch_fas_rhs(const BTable& t, int nblk, hipStream_t s)
{
    hipLaunchKernelGGL(kb_fas_rhs, dim3(nblk), dim3(kB), 0, s, t);
    return hipGetLastError();
}
hipError_t batch_coarse_diff(const BTable& t, int nblk, hipStream_t s)
{
    hipLaunchKernelGGL(kb_coarse_diff, dim3(nblk), dim3(kB), 0, s, t);
    return hipGetLastError();
}
hipError_t batch_prolong_add8(const BTable& t, int nblk, const BGrid* coarse, hipStream_t s)
{
    hipLaunchKernelGGL(kb_prolong_add8, dim3(nblk), dim3(kB), 0, s, t, coarse);
    return hipGetLastError();
}
hipError_t batch_coarsest(const BGrid* grids, int ngrid, int n, const int* active, int cap, double rtol,
                          hipStream_t s)
{
    // one wavefront per grid when it fits (barriers and reductions stay within the wave)
    if (n <= 4)
        hipLaunchKernelGGL((kb_coarsest<64>), dim3(ngrid), dim3(64), 0, s, grids, active, cap, rtol);
    else
        hipLaunchKernelGGL((kb_coarsest<kB>), dim3(ngrid), dim3(kB), 0, s, grids, active, cap, rtol);
    return hipGetLastError();
}
hipError_t batch_norm(const BTable& t, int nblk, double* partial, const int* first, const int* count, int ngrid,
                      double* out, hipStream_t s)
{
    hipLaunchKernelGGL(kb_norm, dim3(nblk), dim3(kB), 0, s, t, partial);
    hipLaunchKernelGGL(kb_fold, dim3(ngrid), dim3(kB), 0, s, partial, first, count, out);
    return hipGetLastError();
}
hipError_t batch_fold(const double* partial, const int* first, const int* count, int ngrid, double* out,
                      hipStream_t s)
{
    hipLaunchKernelGGL(kb_fold, dim3(ngrid), dim3(kB), 0, s, partial, first, count, out);
    return hipGetLastError();
}
hipError_t batch_setup(const BTable& t, int nblk, const PatchParent* parents, hipStream_t s)
{
    hipLaunchKernelGGL(kb_setup, dim3(nblk), dim3(kB), 0, s, t, parents);
    return hipGetLastError();
}
hipError_t batch_restrict_faces(const BTable& t, int nblk, const BGrid* fine, hipStream_t s)
{
    hipLaunchKernelGGL(kb_restrict_faces, dim3(nblk), dim3(kB), 0, s, t, fine);
    return hipGetLastError();
}
hipError_t batch_fill(const BTable& t, int nblk, hipStream_t s)
{
    hipLaunchKernelGGL(kb_fill, dim3(nblk), dim3(kB), 0, s, t);
    return hipGetLastError();
}
hipError_t batch_nonfinite(const BTable& t, int nblk, double* partial, hipStream_t s)
{
    hipLaunchKernelGGL(kb_nonfinite, dim3(nblk), dim3(kB), 0, s, t, partial);
    return hipGetLastError();
}

hipError_t batch_norm_blocks(const BTable& t, int nblk, double* partial, hipStream_t s)
{
    hipLaunchKernelGGL(kb_norm, dim3(nblk), dim3(kB), 0, s, t, partial);
    return hipGetLastError();
}
hipError_t batch_resid_cast(const BTable& t, int nblk, double* partial, hipStream_t s)
{
    hipLaunchKernelGGL(kb_resid_cast, dim3(nblk), dim3(kB), 0, s, t, partial);
    return hipGetLastError();
}
hipError_t batch_add_correction(const BTable& t, int nblk, hipStream_t s)
{
    hipLaunchKernelGGL(kb_add_correction, dim3(nblk), dim3(kB), 0, s, t);
    return hipGetLastError();
}

}  // namespace mgfr
