// Coarse-grid correction u^h += P(u^H - R u^h) (Sec. V.B.3), double and single precision.
//
// P is the cell-centred trilinear interpolation with weights 27/9/3/1 over 64 (Sec. V.A.3),
// periodic.  It factors into an in-plane bilinear part (9/16, 3/16, 3/16, 1/16) on each
// coarse plane and a 3/4, 1/4 blend of the two coarse planes nearest the fine plane.  A
// thread owns one fine column (j,k) and a chunk of fine planes: it forms the in-plane
// interpolant once per coarse plane and reuses it for the two fine planes that need it, so
// a fine cell costs one load and one store of u plus a share of the coarse reads.  The
// difference e = u^H - R u^h is formed on the fly from the two coarse arrays (FAS); the
// linear correction scheme passes the correction itself (no second array).
#include "mgfr_impl.h"

namespace mgfr {
namespace {

constexpr int kPT = 256;  // threads (fine columns) per workgroup

// DIFF: the correction is uc - uhat (else uc itself).  maskf (may be null): add only where
// the fine mask is positive (the active cells of a masked level).
template <typename T, int PI, bool DIFF>
__global__ void __launch_bounds__(kPT) k_prolong_stream(int lgc, T* __restrict__ uf, const T* __restrict__ uc,
                                                        const T* __restrict__ uhat, const float* __restrict__ maskf,
                                                        int ncolblk, const int* __restrict__ halt)
{
    if (halt && *halt) return;
    const int lg = lgc + 1, n = 1 << lg, mc = (1 << lgc) - 1;
    const int nb = gridDim.x;
    int lid = blockIdx.x;
    if ((nb & 7) == 0) lid = (lid & 7) * (nb >> 3) + (lid >> 3);
    const int cb = lid % ncolblk, chunk = lid / ncolblk;
    const unsigned col = (unsigned)cb * kPT + threadIdx.x;
    if (col >= (1u << (2 * lg))) return;
    const int j = (int)(col >> lg), k = (int)(col & (unsigned)(n - 1));
    const int J = j >> 1, K = k >> 1;
    const int Jn = (J + ((j & 1) ? 1 : -1)) & mc, Kn = (K + ((k & 1) ? 1 : -1)) & mc;
    const unsigned c00 = ((unsigned)J << lgc) + K, c10 = ((unsigned)Jn << lgc) + K;
    const unsigned c01 = ((unsigned)J << lgc) + Kn, c11 = ((unsigned)Jn << lgc) + Kn;
    const int i0 = chunk * PI;

    // element offsets fit in 32 bits (n <= 1024)
    T v[PI];
#pragma unroll
    for (int t = 0; t < PI; ++t) v[t] = uf[((unsigned)(i0 + t) << (2 * lg)) + col];

    // fine plane i lies between coarse planes (i-1)>>1 and (i+1)>>1; for the chunk these are
    // coarse planes ib .. ib + PI/2 + 1 (periodic)
    const int ib = (i0 - 1) >> 1;
    T ep[PI / 2 + 2];
#pragma unroll
    for (int t = 0; t < PI / 2 + 2; ++t) {
        const unsigned base = (unsigned)((ib + t) & mc) << (2 * lgc);
        auto E = [&](unsigned c) -> T { return DIFF ? uc[base + c] - uhat[base + c] : uc[base + c]; };
        ep[t] = T(9.0 / 16.0) * E(c00) + T(3.0 / 16.0) * (E(c10) + E(c01)) + T(1.0 / 16.0) * E(c11);
    }
#pragma unroll
    for (int t = 0; t < PI; ++t) {
        const int i = i0 + t;
        const int lo = ((i - 1) >> 1) - ib;
        // odd i: the nearer coarse plane is the lower one
        const T wlo = (i & 1) ? T(0.75) : T(0.25);
        const unsigned q = ((unsigned)i << (2 * lg)) + col;
        if (maskf && !(maskf[q] > 0.0f)) continue;
        uf[q] = v[t] + (wlo * ep[lo] + (T(1) - wlo) * ep[lo + 1]);
    }
}

template <typename T, bool DIFF>
hipError_t launch(const Grid& gc, T* uf, const T* uc, const T* uhat, hipStream_t s, const float* maskf = nullptr)
{
    const int n = gc.n * 2;
    if (gc.n < 2 || n > 1024) return hipErrorInvalidValue;
    const int ncolblk = (n * n + kPT - 1) / kPT;
    if (n >= 8) {
        const unsigned nb = (unsigned)(ncolblk * (n / 8));
        hipLaunchKernelGGL((k_prolong_stream<T, 8, DIFF>), dim3(nb), dim3(kPT), 0, s, gc.lg, uf, uc, uhat, maskf,
                           ncolblk, gc.halt);
    } else {
        hipLaunchKernelGGL((k_prolong_stream<T, 4, DIFF>), dim3((unsigned)ncolblk), dim3(kPT), 0, s, gc.lg, uf, uc, uhat,
                           maskf, ncolblk, gc.halt);
    }
    return hipGetLastError();
}

}  // namespace

hipError_t prolong_correct(const Grid& gc, double* uf, const double* uc, const double* uhat, hipStream_t s)
{
    return launch<double, true>(gc, uf, uc, uhat, s);
}

hipError_t prolong_correct32(const Grid& gc, float* ef, const float* ec, const float* ehat, hipStream_t s)
{
    return launch<float, true>(gc, ef, ec, ehat, s);
}

hipError_t prolong_add_direct(const Grid& gc, double* uf, const double* ec, hipStream_t s)
{
    return launch<double, false>(gc, uf, ec, nullptr, s);
}

hipError_t prolong_add_masked(const Grid& gc, double* uf, const double* ec, const float* maskf, hipStream_t s)
{
    return launch<double, false>(gc, uf, ec, nullptr, s, maskf);
}

}  // namespace mgfr
