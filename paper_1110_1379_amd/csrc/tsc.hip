// Triangle-shaped-cloud (TSC) density assignment and force interpolation (Sec. VI.C),
// double precision, and their C entry points.
//
// Box units, periodic: cell i of the N^3 grid covers [i/N, (i+1)/N).  A particle at x has
// s = x N (modulo N), nearest cell floor(s) and offset d = s - floor(s) - 1/2; the cells
// floor(s) - 1, floor(s), floor(s) + 1 get the weights (1/2 - d)^2 / 2, 3/4 - d^2,
// (1/2 + d)^2 / 2 per axis, their product in 3-D.  Assignment adds mass x weight to the 27
// cells (hardware double-precision atomics in L2; the order of the additions is not fixed,
// so the density is exact up to the rounding of a sum in some order).  Interpolation applies
// the same weights to the cell accelerations -grad phi, taken by central differences, so the
// pair conserves momentum.  Contraction into fused multiply-adds is switched off in the
// weight and interpolation arithmetic, so every product and sum rounds as written.
#include "host_internal.h"

using namespace mgfr_host;

namespace mgfr {
namespace {

constexpr int kB = 256;

#pragma clang fp contract(off)

// Nearest cell index and the three weights per axis of the particle at p[0..2].
__device__ __forceinline__ void tsc_weights(const double* __restrict__ p, int N, int (&c)[3], double (&w)[3][3])
{
    const double Nd = (double)N;
#pragma unroll
    for (int ax = 0; ax < 3; ++ax) {
        double s = p[ax] * Nd;
        s = s - Nd * floor(s / Nd);
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

__global__ void __launch_bounds__(kB) k_tsc_deposit(const double* __restrict__ pos, long long np, int N, int lg,
                                                    double mass, double* __restrict__ rho)
{
    const long long p = (long long)blockIdx.x * kB + threadIdx.x;
    if (p >= np) return;
    int c[3];
    double w[3][3];
    tsc_weights(pos + 3 * p, N, c, w);
    const int m = N - 1;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const long long ia = (long long)((c[0] + a - 1) & m) << (2 * lg);
        const double ma = mass * w[0][a];
#pragma unroll
        for (int b = 0; b < 3; ++b) {
            const long long jb = ia + ((long long)((c[1] + b - 1) & m) << lg);
            const double mab = ma * w[1][b];
#pragma unroll
            for (int z = 0; z < 3; ++z) unsafeAtomicAdd(rho + jb + ((c[2] + z - 1) & m), mab * w[2][z]);
        }
    }
}

// acc = sum over the 27 cells of weight x (-grad phi), -grad phi by central differences.
__global__ void __launch_bounds__(kB) k_tsc_force(const double* __restrict__ phi, int N, int lg,
                                                  const double* __restrict__ pos, long long np,
                                                  double* __restrict__ acc)
{
    const long long p = (long long)blockIdx.x * kB + threadIdx.x;
    if (p >= np) return;
    int c[3];
    double w[3][3];
    tsc_weights(pos + 3 * p, N, c, w);
    const int m = N - 1;
    const double half = (double)N / 2.0;
    auto at = [&](int i, int j, int k) { return phi[((((long long)(i & m) << lg) + (j & m)) << lg) + (k & m)]; };
    double fx = 0.0, fy = 0.0, fz = 0.0;
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int b = 0; b < 3; ++b)
#pragma unroll
            for (int z = 0; z < 3; ++z) {
                const int i = c[0] + a - 1, j = c[1] + b - 1, k = c[2] + z - 1;
                const double wt = w[0][a] * w[1][b] * w[2][z];
                const double gx = -(at(i + 1, j, k) - at(i - 1, j, k)) * half;
                const double gy = -(at(i, j + 1, k) - at(i, j - 1, k)) * half;
                const double gz = -(at(i, j, k + 1) - at(i, j, k - 1)) * half;
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
    if (!rho) return c->fail(MGFR_EINVAL, "rho is NULL");
    if (!std::isfinite(mass)) return c->fail(MGFR_EINVAL, "mass must be finite");
    MGFR_TRY(hip_check(c, hipSetDevice(c->device), "hipSetDevice"));
    hipStream_t s = (hipStream_t)stream;
    MGFR_TRY(mgfr::check_positions(c, pos, np, s));
    MGFR_TRY(hip_check(c, mgfr::fill(rho, 0.0, (long long)N * N * N, s), "fill"));
    if (np > 0) {
        hipLaunchKernelGGL(mgfr::k_tsc_deposit, dim3(mgfr::blocks(np)), dim3(mgfr::kB), 0, s, pos, np, N, ilog2(N), mass,
                           rho);
        MGFR_TRY(hip_check(c, hipGetLastError(), "k_tsc_deposit"));
    }
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
