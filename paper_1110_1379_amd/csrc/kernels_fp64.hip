// Double-precision multigrid kernels for gfx950 (wave64).
//
// The equation is the f(R) field equation in the variable u, f~_R = -exp(u) (Sec. III.C),
// discretised with the conservative 7-point flux of eq. discrete_fR (face b = arithmetic
// mean of the two cell values), multiplied by c~^2 as in eq. bc_modified_fR_op.  Each
// Newton-Gauss-Seidel visit of a cell replaces u_i by u_i - (L_i - f_i) / (dL_i/du_i)
// (Sec. V.B.1, with the derivative of eq. bc_modified_fR_dop for a cell with no ghost).
#include "device_fp64.h"

namespace mgfr {
namespace {

constexpr int kBlock = 256;
constexpr int kMaxPartials = 8192;

using dev::OpVal;
using dev::at;
using dev::bounded;
using dev::cell_op;

__device__ __forceinline__ double rhs(const Grid& g, const double* src, long long q)
{
    return dev::rhs_value(g, src[q]);
}

__device__ __forceinline__ void load_nbrs(const Grid& g, const double* u, int i, int j, int k,
                                          double (&un)[6])
{
    const int m = g.n - 1;
    un[0] = u[at(g, (i - 1) & m, j, k)];
    un[1] = u[at(g, (i + 1) & m, j, k)];
    un[2] = u[at(g, i, (j - 1) & m, k)];
    un[3] = u[at(g, i, (j + 1) & m, k)];
    un[4] = u[at(g, i, j, (k - 1) & m)];
    un[5] = u[at(g, i, j, (k + 1) & m)];
}

// One colour of a sweep; one thread per cell of that colour.
__global__ void __launch_bounds__(kBlock) k_ngs_colour(Grid g, double* __restrict__ u,
                                                       const double* __restrict__ src, int colour)
{
    if (g.halt && *g.halt) return;
    const long long half = 1LL << (3 * g.lg - 1);
    const long long t = (long long)blockIdx.x * kBlock + threadIdx.x;
    if (t >= half) return;
    const int hk = g.n >> 1;
    const int s = (int)(t & (hk - 1));
    const long long row = t >> (g.lg - 1);
    const int i = (int)(row >> g.lg), j = (int)(row & (g.n - 1));
    const int k = 2 * s + ((i + j + colour) & 1);
    const long long q = at(g, i, j, k);
    double un[6];
    load_nbrs(g, u, i, j, k, un);
    const double ui = u[q];
    const OpVal r = cell_op(g, ui, un, rhs(g, src, q));
    u[q] = ui + bounded(-r.L / r.dL, g.max_step);
}

// One thread per coarse cell: residuals of its 8 children, restricted by the mean.
__global__ void __launch_bounds__(kBlock) k_resid_restrict(Grid g, const double* __restrict__ u,
                                                           const double* __restrict__ src,
                                                           double* __restrict__ uc,
                                                           double* __restrict__ uhat,
                                                           double* __restrict__ fc)
{
    if (g.halt && *g.halt) return;
    const int lgc = g.lg - 1, nc = g.n >> 1;
    const long long tc = (long long)blockIdx.x * kBlock + threadIdx.x;
    if (tc >= (1LL << (3 * lgc))) return;
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
                double un[6];
                load_nbrs(g, u, i, j, k, un);
                const double ui = u[q];
                su += ui;
                sd += cell_op(g, ui, un, rhs(g, src, q)).L;
            }
    uc[tc] = 0.125 * su;
    uhat[tc] = 0.125 * su;
    fc[tc] = 0.125 * sd;
}

__global__ void __launch_bounds__(kBlock) k_fas_rhs(Grid g, const double* __restrict__ uhat,
                                                    double* __restrict__ f)
{
    if (g.halt && *g.halt) return;
    const long long q = (long long)blockIdx.x * kBlock + threadIdx.x;
    if (q >= (1LL << (3 * g.lg))) return;
    const int i = (int)(q >> (2 * g.lg)), j = (int)((q >> g.lg) & (g.n - 1)), k = (int)(q & (g.n - 1));
    double un[6];
    load_nbrs(g, uhat, i, j, k, un);
    f[q] = cell_op(g, uhat[q], un, 0.0).L - f[q];
}

// tau = fH - R f_src on the coarse level (fH = L^H(R u) - R d, the FAS right-hand side), with
// f_src = fscale (rho - sref) + fshift of the fine grid g; block partials (sum tau^2, max |tau|).
__global__ void __launch_bounds__(kBlock) k_tau_finish(Grid g, const double* __restrict__ rho,
                                                       const double* __restrict__ fH, double* __restrict__ tau,
                                                       double* __restrict__ partial)
{
    __shared__ double rs[kBlock], rm[kBlock];
    const int lgc = g.lg - 1, nc = g.n >> 1;
    const long long ncell = 1LL << (3 * lgc);
    double s = 0.0, mx = 0.0;
    for (long long q = (long long)blockIdx.x * kBlock + threadIdx.x; q < ncell; q += (long long)gridDim.x * kBlock) {
        const int I = (int)(q >> (2 * lgc)), J = (int)((q >> lgc) & (nc - 1)), K = (int)(q & (nc - 1));
        double sf = 0.0;
        for (int a = 0; a < 2; ++a)
            for (int b = 0; b < 2; ++b)
                for (int z = 0; z < 2; ++z) sf += dev::rhs_value(g, rho[at(g, 2 * I + a, 2 * J + b, 2 * K + z)]);
        const double t = fH[q] - 0.125 * sf;
        if (tau) tau[q] = t;
        s += t * t;
        const double at_ = fabs(t);
        if (!(mx >= at_)) mx = at_;
    }
    rs[threadIdx.x] = s;
    rm[threadIdx.x] = mx;
    __syncthreads();
    for (int w = kBlock / 2; w > 0; w >>= 1) {
        if (threadIdx.x < w) {
            rs[threadIdx.x] += rs[threadIdx.x + w];
            const double o = rm[threadIdx.x + w];
            if (!(rm[threadIdx.x] >= o)) rm[threadIdx.x] = o;
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        partial[2 * blockIdx.x] = rs[0];
        partial[2 * blockIdx.x + 1] = rm[0];
    }
}

// Deterministic block reductions over kBlock threads (fixed tree order).
// block_sum_max: a <- sum of a, b <- max of b (NaN propagates).  block_sum2: both summed.
template <bool SecondIsMax>
__device__ void block_reduce2(double& a, double& b, double* sh_a, double* sh_b)
{
    const int t = threadIdx.x;
    sh_a[t] = a;
    sh_b[t] = b;
    __syncthreads();
    for (int w = kBlock / 2; w > 0; w >>= 1) {
        if (t < w) {
            sh_a[t] += sh_a[t + w];
            const double o = sh_b[t + w];
            if (SecondIsMax) {
                if (!(sh_b[t] >= o)) sh_b[t] = o;
            } else {
                sh_b[t] += o;
            }
        }
        __syncthreads();
    }
    a = sh_a[0];
    b = sh_b[0];
    __syncthreads();
}

__global__ void __launch_bounds__(kBlock) k_coarsest(Grid g, double* __restrict__ u,
                                                     const double* __restrict__ src, int cap,
                                                     double rtol, long long* __restrict__ sweeps_done)
{
    if (g.halt && *g.halt) return;
    __shared__ double su[512];
    __shared__ double sf[512];
    __shared__ double rs[kBlock], rm[kBlock];
    const int nc = 1 << (3 * g.lg);
    for (int q = threadIdx.x; q < nc; q += kBlock) {
        su[q] = u[q];
        sf[q] = rhs(g, src, q);
    }
    __syncthreads();
    const int m = g.n - 1;
    auto nbrs = [&](int q, double (&un)[6]) {
        const int i = q >> (2 * g.lg), j = (q >> g.lg) & m, k = q & m;
        un[0] = su[(((i - 1) & m) << (2 * g.lg)) + (j << g.lg) + k];
        un[1] = su[(((i + 1) & m) << (2 * g.lg)) + (j << g.lg) + k];
        un[2] = su[(i << (2 * g.lg)) + (((j - 1) & m) << g.lg) + k];
        un[3] = su[(i << (2 * g.lg)) + (((j + 1) & m) << g.lg) + k];
        un[4] = su[(i << (2 * g.lg)) + (j << g.lg) + ((k - 1) & m)];
        un[5] = su[(i << (2 * g.lg)) + (j << g.lg) + ((k + 1) & m)];
        return (i + j + k) & 1;
    };
    // rms of L - f, and the rounding floor of that rms: per cell one unit in the last place
    // of u times |dL/du| plus one of the summed magnitudes (C (b_nb + b_i)|u_nb - u_i| per
    // face, the curvature term and |f|)
    auto rms = [&](double& floor) {
        double s = 0.0, fl = 0.0;
        for (int q = threadIdx.x; q < nc; q += kBlock) {
            double un[6];
            nbrs(q, un);
            const double ui = su[q];
            const OpVal r = cell_op(g, ui, un, sf[q]);
            s += r.L * r.L;
            const double bi = exp(ui);
            double t = 0.0;
#pragma unroll
            for (int v = 0; v < 6; ++v) t += g.C * (exp(un[v]) + bi) * fabs(un[v] - ui);
            t += g.A * exp(-ui * g.inv_np1) + fabs(sf[q]);
            const double f1 = 2.220446049250313e-16 * (fabs(r.dL) * fabs(ui) + t);
            fl += f1 * f1;
        }
        block_reduce2<false>(s, fl, rs, rm);
        floor = sqrt(fl / nc);
        return sqrt(s / nc);
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
            for (int q = threadIdx.x; q < nc; q += kBlock) {
                double un[6];
                if (nbrs(q, un) != colour) continue;
                const double ui = su[q];
                const OpVal r = cell_op(g, ui, un, sf[q]);
                su[q] = ui + bounded(-r.L / r.dL, g.max_step);
            }
            __syncthreads();
        }
    }
    for (int q = threadIdx.x; q < nc; q += kBlock) u[q] = su[q];
    if (threadIdx.x == 0 && sweeps_done) sweeps_done[0] += sweep;
}

__global__ void __launch_bounds__(kBlock) k_residual_field(Grid g, const double* __restrict__ u,
                                                           const double* __restrict__ src,
                                                           double* __restrict__ d)
{
    const long long q = (long long)blockIdx.x * kBlock + threadIdx.x;
    if (q >= (1LL << (3 * g.lg))) return;
    const int i = (int)(q >> (2 * g.lg)), j = (int)((q >> g.lg) & (g.n - 1)), k = (int)(q & (g.n - 1));
    double un[6];
    load_nbrs(g, u, i, j, k, un);
    d[q] = cell_op(g, u[q], un, rhs(g, src, q)).L;
}

__global__ void __launch_bounds__(kBlock) k_residual_partial(Grid g, const double* __restrict__ u,
                                                             const double* __restrict__ src,
                                                             double* __restrict__ partial)
{
    if (g.halt && *g.halt) return;
    __shared__ double rs[kBlock], rm[kBlock];
    const long long ncell = 1LL << (3 * g.lg);
    double s = 0.0, mx = 0.0;
    for (long long q = (long long)blockIdx.x * kBlock + threadIdx.x; q < ncell;
         q += (long long)gridDim.x * kBlock) {
        const int i = (int)(q >> (2 * g.lg)), j = (int)((q >> g.lg) & (g.n - 1)), k = (int)(q & (g.n - 1));
        double un[6];
        load_nbrs(g, u, i, j, k, un);
        const double d = cell_op(g, u[q], un, rhs(g, src, q)).L;
        s += d * d;
        const double ad = fabs(d);
        if (!(mx >= ad)) mx = ad;
    }
    block_reduce2<true>(s, mx, rs, rm);
    if (threadIdx.x == 0) {
        partial[2 * blockIdx.x] = s;
        partial[2 * blockIdx.x + 1] = mx;
    }
}

__global__ void __launch_bounds__(kBlock) k_sum_count_partial(const double* __restrict__ x,
                                                              long long n,
                                                              double* __restrict__ partial)
{
    __shared__ double rs[kBlock], rm[kBlock];
    double s = 0.0, c = 0.0;
    for (long long q = (long long)blockIdx.x * kBlock + threadIdx.x; q < n; q += (long long)gridDim.x * kBlock) {
        const double v = x[q];
        if (isfinite(v)) s += v;
        else c += 1.0;
    }
    block_reduce2<false>(s, c, rs, rm);
    if (threadIdx.x == 0) {
        partial[2 * blockIdx.x] = s;
        partial[2 * blockIdx.x + 1] = c;
    }
}

// One workgroup folds `nb` (sum, max-or-sum) pairs in a fixed order.
__global__ void __launch_bounds__(kBlock) k_fold(const double* __restrict__ partial, int nb,
                                                 int second_is_sum, double* __restrict__ out)
{
    __shared__ double rs[kBlock], rm[kBlock];
    double s = 0.0, m = 0.0;
    for (int b = threadIdx.x; b < nb; b += kBlock) {
        s += partial[2 * b];
        const double o = partial[2 * b + 1];
        if (second_is_sum) m += o;
        else if (!(m >= o)) m = o;
    }
    if (second_is_sum) block_reduce2<false>(s, m, rs, rm);
    else block_reduce2<true>(s, m, rs, rm);
    if (threadIdx.x == 0) {
        out[0] = s;
        out[1] = m;
    }
}

__global__ void __launch_bounds__(kBlock) k_add_correction(double* __restrict__ u, const float* __restrict__ e,
                                                           long long n, const int* __restrict__ halt)
{
    if (halt && *halt) return;
    for (long long q = (long long)blockIdx.x * kBlock + threadIdx.x; q < n; q += (long long)gridDim.x * kBlock)
        u[q] += (double)e[q];
}

__global__ void __launch_bounds__(kBlock) k_residual_cast(Grid g, const double* __restrict__ u,
                                                          const double* __restrict__ src, float* __restrict__ r32,
                                                          float* __restrict__ ub32, double* __restrict__ partial)
{
    if (g.halt && *g.halt) return;
    __shared__ double rs[kBlock], rm[kBlock];
    const long long ncell = 1LL << (3 * g.lg);
    double s = 0.0, mx = 0.0;
    for (long long q = (long long)blockIdx.x * kBlock + threadIdx.x; q < ncell; q += (long long)gridDim.x * kBlock) {
        const int i = (int)(q >> (2 * g.lg)), j = (int)((q >> g.lg) & (g.n - 1)), k = (int)(q & (g.n - 1));
        double un[6];
        load_nbrs(g, u, i, j, k, un);
        const double d = cell_op(g, u[q], un, rhs(g, src, q)).L;
        r32[q] = (float)(-d);
        ub32[q] = (float)u[q];
        s += d * d;
        const double ad = fabs(d);
        if (!(mx >= ad)) mx = ad;
    }
    block_reduce2<true>(s, mx, rs, rm);
    if (threadIdx.x == 0) {
        partial[2 * blockIdx.x] = s;
        partial[2 * blockIdx.x + 1] = mx;
    }
}

__global__ void __launch_bounds__(kBlock) k_fill(double* __restrict__ x, double v, long long n)
{
    for (long long q = (long long)blockIdx.x * kBlock + threadIdx.x; q < n; q += (long long)gridDim.x * kBlock)
        x[q] = v;
}

// Stop test of a domain solve captured in a graph: red[0] holds the sum of d^2 over the
// finest cells after a cycle.  Unless the solve has stopped (state[1] set), count the cycle
// (state[0]), store rms(d) in hist, and stop when rms is not above tol, non-finite, or the
// cycle cap is reached.  One thread.
__global__ void k_domain_stop(const double* __restrict__ red, long long ncell, double tol, int max_cycles,
                              double* __restrict__ hist, int* __restrict__ state)
{
    if (threadIdx.x != 0 || state[1]) return;
    const double rms = sqrt(red[0] / (double)ncell);
    const int k = state[0] + 1;
    state[0] = k;
    hist[k] = rms;
    if (!isfinite(rms) || !(rms > tol) || k >= max_cycles) state[1] = 1;
}

__global__ void k_fill_int(int* __restrict__ p, int v, int n)
{
    if ((int)threadIdx.x < n) p[threadIdx.x] = v;
}

inline unsigned blocks_for(long long work)
{
    return (unsigned)((work + kBlock - 1) / kBlock);
}

inline unsigned reduction_blocks(long long work)
{
    long long b = (work + kBlock - 1) / kBlock;
    return (unsigned)(b < kMaxPartials ? (b < 1 ? 1 : b) : kMaxPartials);
}

}  // namespace

long long reduction_scratch() { return 2LL * kMaxPartials; }

hipError_t ngs_sweep(const Grid& g, double* u, const double* src, hipStream_t s)
{
    const long long half = cells(g) / 2;
    for (int colour = 0; colour < 2; ++colour) {
        hipLaunchKernelGGL(k_ngs_colour, dim3(blocks_for(half)), dim3(kBlock), 0, s, g, u, src, colour);
    }
    return hipGetLastError();
}

hipError_t resid_restrict(const Grid& g, const double* u, const double* src, double* uc,
                          double* uhat, double* fc, hipStream_t s)
{
    hipLaunchKernelGGL(k_resid_restrict, dim3(blocks_for(cells(g) / 8)), dim3(kBlock), 0, s, g, u, src,
                       uc, uhat, fc);
    return hipGetLastError();
}

hipError_t fas_rhs(const Grid& gc, const double* uhat, double* f, hipStream_t s)
{
    hipLaunchKernelGGL(k_fas_rhs, dim3(blocks_for(cells(gc))), dim3(kBlock), 0, s, gc, uhat, f);
    return hipGetLastError();
}

hipError_t coarsest_solve(const Grid& g, double* u, const double* src, int cap, double rtol,
                          long long* sweeps_done, hipStream_t s)
{
    if (g.n > 8) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_coarsest, dim3(1), dim3(kBlock), 0, s, g, u, src, cap, rtol, sweeps_done);
    return hipGetLastError();
}

hipError_t residual_field(const Grid& g, const double* u, const double* src, double* d, hipStream_t s)
{
    hipLaunchKernelGGL(k_residual_field, dim3(blocks_for(cells(g))), dim3(kBlock), 0, s, g, u, src, d);
    return hipGetLastError();
}

hipError_t residual_norm(const Grid& g, const double* u, const double* src, double* partial,
                         double* out, hipStream_t s)
{
    const unsigned nb = reduction_blocks(cells(g));
    hipLaunchKernelGGL(k_residual_partial, dim3(nb), dim3(kBlock), 0, s, g, u, src, partial);
    hipLaunchKernelGGL(k_fold, dim3(1), dim3(kBlock), 0, s, partial, (int)nb, 0, out);
    return hipGetLastError();
}

hipError_t sum_and_count_nonfinite(const double* x, long long n, double* partial, double* out,
                                   hipStream_t s)
{
    const unsigned nb = reduction_blocks(n);
    hipLaunchKernelGGL(k_sum_count_partial, dim3(nb), dim3(kBlock), 0, s, x, n, partial);
    hipLaunchKernelGGL(k_fold, dim3(1), dim3(kBlock), 0, s, partial, (int)nb, 1, out);
    return hipGetLastError();
}

hipError_t add_correction(double* u, const float* e, long long n, hipStream_t s, const int* halt)
{
    hipLaunchKernelGGL(k_add_correction, dim3(reduction_blocks(n)), dim3(kBlock), 0, s, u, e, n, halt);
    return hipGetLastError();
}

hipError_t residual_cast(const Grid& g, const double* u, const double* src, float* r32, float* ub32,
                         double* partial, double* out, hipStream_t s)
{
    const unsigned nb = reduction_blocks(cells(g));
    hipLaunchKernelGGL(k_residual_cast, dim3(nb), dim3(kBlock), 0, s, g, u, src, r32, ub32, partial);
    hipLaunchKernelGGL(k_fold, dim3(1), dim3(kBlock), 0, s, partial, (int)nb, 0, out);
    return hipGetLastError();
}

hipError_t fold_partials(const double* partial, int nb, double* out, hipStream_t s)
{
    hipLaunchKernelGGL(k_fold, dim3(1), dim3(kBlock), 0, s, partial, nb, 0, out);
    return hipGetLastError();
}

hipError_t fill(double* x, double v, long long n, hipStream_t s)
{
    hipLaunchKernelGGL(k_fill, dim3(reduction_blocks(n)), dim3(kBlock), 0, s, x, v, n);
    return hipGetLastError();
}

hipError_t domain_stop(const double* red, long long ncell, double tol, int max_cycles, double* hist, int* state,
                       hipStream_t s)
{
    hipLaunchKernelGGL(k_domain_stop, dim3(1), dim3(64), 0, s, red, ncell, tol, max_cycles, hist, state);
    return hipGetLastError();
}

hipError_t fill_int(int* p, int v, int n, hipStream_t s)
{
    if (n > 64) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_fill_int, dim3(1), dim3(64), 0, s, p, v, n);
    return hipGetLastError();
}

int tau_finish(const Grid& g, const double* rho, const double* fH, double* tau, double* partial, hipStream_t s)
{
    const long long ncell = 1LL << (3 * (g.lg - 1));
    const unsigned nb = reduction_blocks(ncell);
    hipLaunchKernelGGL(k_tau_finish, dim3(nb), dim3(kBlock), 0, s, g, rho, fH, tau, partial);
    return hipGetLastError() == hipSuccess ? (int)nb : -1;
}

}  // namespace mgfr
