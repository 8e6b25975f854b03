// Host side of libmgfr.so: model constants, the multigrid hierarchy, the V-cycle driver
// and the C ABI declared in include/mgfr.h.
#include <hip/hip_runtime.h>

#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <algorithm>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "host_internal.h"

namespace {

using namespace mgfr_host;

// Planes per workgroup of a fused sweep: the option on the finest level, else automatic.
int planes_for(const mgfr_opts* o, size_t m, int n)
{
    if (m == 0 && o->planes > 0 && o->planes <= n) return o->planes;
    return mgfr::fused_sweep_planes(n);
}

// The same for the single-precision sweep, whose 8 x 32 tiles give more workgroups per plane
// chunk: measured best at 8 planes up to 128^3, 32 at 256^3 and 64 from 512^3.
int planes_for32(const mgfr_opts* o, size_t m, int n)
{
    if (m == 0 && o->planes > 0 && o->planes <= n) return o->planes;
    return n <= 128 ? 8 : n == 256 ? 32 : 64;
}

// The storage one domain solve works on: the multigrid levels (double precision, and single
// precision for the mixed solver) and the reduction buffers.  The context's own (allocated on
// demand) or carved from the library's fixed device array by mg_fr_solve_noalloc.
struct Hier {
    Level* lv = nullptr;
    size_t nlev = 0;
    Level32* lv32 = nullptr;
    size_t nlev32 = 0;
    double* partial = nullptr;   // block partials of the reductions
    double* red = nullptr;       // device result of a reduction (2 doubles)
    double* host = nullptr;      // host copy of it
    long long* counter = nullptr;  // coarsest-level sweeps of the current solve
};

Hier ctx_hier(mgfr_ctx* c)
{
    Hier h;
    h.lv = c->lv.data();
    h.nlev = c->lv.size();
    h.lv32 = c->lv32.data();
    h.nlev32 = c->lv32.size();
    h.partial = c->partial;
    h.red = c->red;
    h.host = c->host_red;
    h.counter = c->counter;
    return h;
}

// Copies the 2-double reduction result to the host (synchronises the stream).
int read_red(mgfr_ctx* c, const Hier& h, hipStream_t s, double* out2)
{
    MGFR_TRY(hip_check(c, hipMemcpyAsync(h.host, h.red, 2 * sizeof(double), hipMemcpyDeviceToHost, s),
                       "hipMemcpyAsync"));
    MGFR_TRY(hip_check(c, hipStreamSynchronize(s), "hipStreamSynchronize"));
    out2[0] = h.host[0];
    out2[1] = h.host[1];
    return MGFR_OK;
}

// Tile of the single-precision fused sweep: the option on the finest level, else automatic.
int tile_for32(const mgfr_opts* o, size_t m)
{
    return m == 0 && o->tile > 0 ? o->tile : mgfr::kTile16x32;
}

struct Cycle {
    mgfr_ctx* c;
    const Hier& h;
    const mgfr_opts* o;
    hipStream_t s;
    const double* finest_src = nullptr;

    // One smoother sweep on level m, from *cur into the other buffer for the fused kernel
    // (cur is updated) or in place.  Finest-level sweeps are timed under MGFR_PROFILE.
    int sweep(size_t m, const double* src, double*& cur)
    {
        Level& L = h.lv[m];
        const bool fused = L.alt != nullptr && !o_simple;
        const bool timed = m == 0 && (o->flags & MGFR_PROFILE);
        if (timed) {
            if ((size_t)c->ev_used + 2 > c->ev.size()) {
                for (int k = 0; k < 64; ++k) {
                    hipEvent_t ev;
                    MGFR_TRY(hip_check(c, hipEventCreate(&ev), "hipEventCreate"));
                    c->ev.push_back(ev);
                }
            }
            MGFR_TRY(hip_check(c, hipEventRecord(c->ev[c->ev_used], s), "hipEventRecord"));
        }
        if (fused) {
            double* out = cur == L.u ? L.alt : L.u;
            MGFR_TRY(hip_check(c, mgfr::ngs_sweep_fused(L.g, cur, out, src, planes_for(o, m, L.g.n),
                                                          m == 0 && o->tile > 0 ? o->tile : mgfr::kTile64x16x64, s),
                               "ngs_sweep_fused"));
            cur = out;
        } else {
            MGFR_TRY(hip_check(c, mgfr::ngs_sweep(L.g, cur, src, s), "ngs_sweep"));
        }
        if (timed) {
            MGFR_TRY(hip_check(c, hipEventRecord(c->ev[c->ev_used + 1], s), "hipEventRecord"));
            c->ev_used += 2;
            c->stats.sweep_launches += fused ? 1 : 2;
            c->stats.sweep_bytes += 24.0 * (double)mgfr::cells(L.g);
        }
        c->stats.cell_updates += mgfr::cells(L.g);
        if (m == 0) c->stats.finest_updates += mgfr::cells(L.g);
        return MGFR_OK;
    }

    // Sums the timed intervals recorded so far (synchronises) and releases the events.
    int harvest()
    {
        if (c->ev_used == 0) return MGFR_OK;
        MGFR_TRY(hip_check(c, hipStreamSynchronize(s), "hipStreamSynchronize"));
        for (int k = 0; k < c->ev_used; k += 2) {
            float ms = 0.0f;
            MGFR_TRY(hip_check(c, hipEventElapsedTime(&ms, c->ev[k], c->ev[k + 1]), "hipEventElapsedTime"));
            c->stats.sweep_ms += ms;
        }
        c->ev_used = 0;
        return MGFR_OK;
    }

    int vcycle(size_t m)
    {
        Level& L = h.lv[m];
        const double* src = m == 0 ? finest_src : L.f;
        if (m + 1 == h.nlev) {
            return hip_check(c, mgfr::coarsest_solve(L.g, L.u, src, o->coarsest_sweeps, o->coarsest_rtol,
                                                     h.counter, s),
                             "coarsest_solve");
        }
        double* cur = L.u;
        for (int k = 0; k < o->pre; ++k) MGFR_TRY(sweep(m, src, cur));
        Level& H = h.lv[m + 1];
        if (L.alt && !o_simple) {
            mgfr::ResidStream a{};
            a.ti = mgfr::resid_stream_planes(L.g.n);
            a.uc = H.u;
            a.uhat = H.uhat;
            a.fc = H.f;
            MGFR_TRY(hip_check(c, mgfr::resid_stream(L.g, cur, src, a, s), "resid_stream"));
        } else {
            MGFR_TRY(hip_check(c, mgfr::resid_restrict(L.g, cur, src, H.u, H.uhat, H.f, s), "resid_restrict"));
        }
        MGFR_TRY(hip_check(c, mgfr::fas_rhs(H.g, H.uhat, H.f, s), "fas_rhs"));
        MGFR_TRY(vcycle(m + 1));
        // u^h += P(u^H - R u^h)
        MGFR_TRY(hip_check(c, mgfr::prolong_correct(H.g, cur, H.u, H.uhat, s), "prolong_correct"));
        for (int k = 0; k < o->post; ++k) MGFR_TRY(sweep(m, src, cur));
        if (cur != L.u)
            MGFR_TRY(hip_check(c, hipMemcpyAsync(L.u, cur, sizeof(double) * mgfr::cells(L.g), hipMemcpyDeviceToDevice, s),
                               "hipMemcpyAsync"));
        return MGFR_OK;
    }

    bool o_simple = false;
};

// V-cycle of the single-precision correction multigrid.
struct Cycle32 {
    mgfr_ctx* c;
    const Hier& h;
    const mgfr_opts* o;
    hipStream_t s;

    int sweep(size_t m, float*& cur)
    {
        Level32& L = h.lv32[m];
        const bool timed = m == 0 && (o->flags & MGFR_PROFILE);
        if (timed) {
            if ((size_t)c->ev_used + 2 > c->ev.size()) {
                for (int k = 0; k < 64; ++k) {
                    hipEvent_t ev;
                    MGFR_TRY(hip_check(c, hipEventCreate(&ev), "hipEventCreate"));
                    c->ev.push_back(ev);
                }
            }
            MGFR_TRY(hip_check(c, hipEventRecord(c->ev[c->ev_used], s), "hipEventRecord"));
        }
        if (L.ealt) {
            float* out = cur == L.e ? L.ealt : L.e;
            MGFR_TRY(hip_check(c, mgfr::ngs_sweep32_fused(L.g, L.ub, cur, out, L.f, planes_for32(o, m, L.g.n), tile_for32(o, m), s),
                               "ngs_sweep32_fused"));
            cur = out;
        } else {
            MGFR_TRY(hip_check(c, mgfr::ngs_sweep32(L.g, L.ub, cur, L.f, s), "ngs_sweep32"));
        }
        if (timed) {
            MGFR_TRY(hip_check(c, hipEventRecord(c->ev[c->ev_used + 1], s), "hipEventRecord"));
            c->ev_used += 2;
            c->stats.sweep_launches += L.ealt ? 1 : 2;
            c->stats.sweep_bytes += 12.0 * (double)mgfr::cells(L.g);
        }
        c->stats.cell_updates += mgfr::cells(L.g);
        if (m == 0) c->stats.finest_updates += mgfr::cells(L.g);
        return MGFR_OK;
    }

    int vcycle(size_t m)
    {
        Level32& L = h.lv32[m];
        if (m + 1 == h.nlev32)
            return hip_check(c, mgfr::coarsest_solve32(L.g, L.ub, L.e, L.f, o->coarsest_sweeps, o->coarsest_rtol, s),
                             "coarsest_solve32");
        float* cur = L.e;
        for (int k = 0; k < o->pre; ++k) MGFR_TRY(sweep(m, cur));
        Level32& H = h.lv32[m + 1];
        MGFR_TRY(hip_check(c, mgfr::resid_restrict32(L.g, L.ub, cur, L.f, H.e, H.ehat, H.f, s), "resid_restrict32"));
        MGFR_TRY(hip_check(c, mgfr::fas_rhs32(H.g, H.ub, H.ehat, H.f, s), "fas_rhs32"));
        MGFR_TRY(vcycle(m + 1));
        // e^h += P(e^H - R e^h)
        MGFR_TRY(hip_check(c, mgfr::prolong_correct32(H.g, cur, H.e, H.ehat, s), "prolong_correct32"));
        for (int k = 0; k < o->post; ++k) MGFR_TRY(sweep(m, cur));
        if (cur != L.e)
            MGFR_TRY(hip_check(c, hipMemcpyAsync(L.e, cur, sizeof(float) * mgfr::cells(L.g), hipMemcpyDeviceToDevice, s),
                               "hipMemcpyAsync"));
        return MGFR_OK;
    }
};

// ---- fixed device scratch of mg_fr_solve_noalloc ------------------------------------------
// A file-scope device array that every GPU the library runs on holds until the process ends.
// Host code never uses its name as an address: each device's copy sits at its own address,
// which hipGetSymbolAddress gives once per device (with that device current) and which is kept
// in fixed_ptr[] and handed to the kernels from there.
constexpr int kNoAllocMaxN = 128;                         // largest grid side it takes
constexpr size_t kFixedScratchBytes = size_t(72) << 20;   // 72 MiB: a mixed 128^3 solve needs ~63
constexpr int kMaxLevels = 12;
constexpr int kMaxDevices = 64;

static __device__ __align__(256) char scratch[kFixedScratchBytes];

std::mutex fixed_mutex;
void* fixed_ptr[kMaxDevices] = {};
bool fixed_tried[kMaxDevices] = {};

// This device's address of the scratch array (resolved on the first call for the device, with
// the device current; the caller's current device is restored).  Null if it cannot be had.
void* fixed_scratch_address(int device)
{
    if (device < 0 || device >= kMaxDevices) return nullptr;
    std::lock_guard<std::mutex> lock(fixed_mutex);
    if (!fixed_tried[device]) {
        fixed_tried[device] = true;
        int prev = -1;
        const bool had = hipGetDevice(&prev) == hipSuccess;
        void* p = nullptr;
        if (hipSetDevice(device) == hipSuccess && hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) == hipSuccess)
            fixed_ptr[device] = p;
        else
            (void)hipGetLastError();
        if (had) (void)hipSetDevice(prev);
    }
    return fixed_ptr[device];
}

// Lays out the storage of a domain solve of side N (levels N ... coarsest; single-precision
// levels too when mixed) on the device block at base, each array 256-byte aligned, and
// returns the bytes it needs (base null: sizes only, nothing written but the byte count).
size_t carve(char* base, int N, int coarsest, bool mixed, Hier* h, Level* lv, Level32* lv32)
{
    size_t at = 0;
    auto take = [&](size_t bytes) -> char* {
        char* p = base ? base + at : nullptr;
        at += (bytes + 255) & ~size_t(255);
        return p;
    };
    h->partial = (double*)take(sizeof(double) * (size_t)mgfr::reduction_scratch());
    h->red = (double*)take(2 * sizeof(double));
    h->counter = (long long*)take(sizeof(long long));
    size_t m = 0;
    for (int n = N; n >= coarsest && m < (size_t)kMaxLevels; n /= 2, ++m) {
        const size_t n3 = (size_t)n * n * n;
        Level L{};
        if (n < N) {
            L.u = (double*)take(sizeof(double) * n3);
            L.uhat = (double*)take(sizeof(double) * n3);
            L.f = (double*)take(sizeof(double) * n3);
        }
        if (n >= mgfr::fused_sweep_min_n()) L.alt = (double*)take(sizeof(double) * n3);
        lv[m] = L;
        if (mixed) {
            Level32 E{};
            E.ub = (float*)take(sizeof(float) * n3);
            E.e = (float*)take(sizeof(float) * n3);
            E.f = (float*)take(sizeof(float) * n3);
            if (n < N) E.ehat = (float*)take(sizeof(float) * n3);
            if (n >= mgfr::fused_sweep_min_n()) E.ealt = (float*)take(sizeof(float) * n3);
            lv32[m] = E;
        }
    }
    h->lv = lv;
    h->nlev = m;
    h->lv32 = lv32;
    h->nlev32 = mixed ? m : 0;
    return at;
}

// rms and max of the finest residual L(u) - f (synchronises).
int finest_norm(mgfr_ctx* c, const Hier& h, const mgfr::Grid& g, const double* u, const double* rho,
                hipStream_t s, double* rms, double* mx)
{
    if (g.n >= mgfr::fused_sweep_min_n()) {
        mgfr::ResidStream a{};
        a.ti = mgfr::resid_stream_planes(g.n);
        a.partial = h.partial;
        MGFR_TRY(hip_check(c, mgfr::resid_stream(g, u, rho, a, s), "resid_stream"));
        MGFR_TRY(hip_check(c, mgfr::fold_partials(h.partial, (int)mgfr::resid_stream_blocks(g.n), h.red, s),
                           "fold_partials"));
    } else {
        MGFR_TRY(hip_check(c, mgfr::residual_norm(g, u, rho, h.partial, h.red, s), "residual_norm"));
    }
    double r[2];
    MGFR_TRY(read_red(c, h, s, r));
    *rms = std::sqrt(r[0] / (double)mgfr::cells(g));
    if (mx) *mx = r[1];
    return MGFR_OK;
}

}  // namespace

extern "C" {

int mgfr_create(mgfr_ctx** ctx, int device)
{
    if (!ctx) return MGFR_EINVAL;
    *ctx = nullptr;
    int count = 0;
    if (hipGetDeviceCount(&count) != hipSuccess || device < 0 || device >= count) return MGFR_EDEVICE;
    mgfr_ctx* c = new (std::nothrow) mgfr_ctx();
    if (!c) return MGFR_ENOMEM;
    c->device = device;
    // error messages are at most 511 characters: later failures never allocate
    c->err.reserve(512);
    c->fixed_scratch = fixed_scratch_address(device);
    *ctx = c;
    return MGFR_OK;
}

void mgfr_destroy(mgfr_ctx* c)
{
    if (!c) return;
    (void)hipSetDevice(c->device);
    (void)hipDeviceSynchronize();
    c->free_levels();
    c->free_levels32();
    (void)hipFree(c->partial);
    (void)hipFree(c->red);
    (void)hipFree(c->counter);
    for (hipEvent_t e : c->ev) (void)hipEventDestroy(e);
    if (c->ev_fork) (void)hipEventDestroy(c->ev_fork);
    if (c->ev_join) (void)hipEventDestroy(c->ev_join);
    if (c->side) (void)hipStreamDestroy(c->side);
    for (int d = 0; d < mgfr_ctx::kTailForks; ++d) {
        if (c->ev_tf[d]) (void)hipEventDestroy(c->ev_tf[d]);
        if (c->ev_tj[d]) (void)hipEventDestroy(c->ev_tj[d]);
    }
    if (c->tail) (void)hipStreamDestroy(c->tail);
    c->drop_graph();
    if (c->dcap) (void)hipStreamDestroy(c->dcap);
    (void)hipFree(c->gstate);
    (void)hipFree(c->ghist);
    if (c->host_red) (void)hipHostFree(c->host_red);
    if (c->pin) (void)hipHostFree(c->pin);
    c->free_spare();
    c->free_poisson();
    c->free_masked();
    (void)hipFree(c->tsc);
    delete c;
}

const char* mgfr_last_error(const mgfr_ctx* c) { return c ? c->err.c_str() : "no context"; }

int mgfr_get_stats(const mgfr_ctx* c, mgfr_stats* out)
{
    if (!c || !out) return MGFR_EINVAL;
    *out = c->stats;
    return MGFR_OK;
}

void mgfr_default_opts(mgfr_opts* o)
{
    if (!o) return;
    o->tol = 1e-8;
    o->pre = 2;
    o->post = 2;
    o->coarsest_n = 4;
    o->coarsest_sweeps = 400;
    o->max_cycles = 60;
    o->precision = MGFR_FP64;
    o->flags = 0;
    o->inner_cycles = 1;
    o->max_step = 1.0;
    o->coarsest_rtol = 1e-3;
    o->planes = 0;
    o->tau_alpha = 0.0;
    o->unit_n = 0;
    o->tile = 0;
}

int mgfr_constants(const mgfr_params* params, int N, double* out8)
{
    Model md;
    if (!out8 || N < 1 || derive_model(params, &md) != MGFR_OK) return MGFR_EINVAL;
    const double h = 1.0 / N;
    out8[0] = md.xi;
    out8[1] = md.ct;
    out8[2] = md.K;
    out8[3] = md.A;
    out8[4] = md.Sbar;
    out8[5] = md.D;
    out8[6] = md.ubar;
    out8[7] = md.ct * md.ct / (2.0 * h * h);
    return MGFR_OK;
}

}  // extern "C"

namespace {

// Finest-level grid with the density source; rho_ref = 1 or mean(rho).
int finest_grid(mgfr_ctx* c, const Hier& h, const Model& md, const double* rho, int N, int flags,
                double max_step, hipStream_t s, mgfr::Grid* g)
{
    *g = make_grid(md, N, 1.0 / N, max_step);
    const long long ncell = (long long)N * N * N;
    MGFR_TRY(hip_check(c, mgfr::sum_and_count_nonfinite(rho, ncell, h.partial, h.red, s), "density check"));
    double r[2];
    MGFR_TRY(read_red(c, h, s, r));
    if (r[1] != 0.0) return c->fail(MGFR_ENONFINITE, "density has %.0f non-finite cells", r[1]);
    g->fscale = md.D;
    g->sref = (flags & MGFR_SUBTRACT_MEAN) ? r[0] / (double)ncell : 1.0;
    g->fshift = md.Sbar;
    return MGFR_OK;
}

// rms of the truncation-error estimate tau = L^H(R u) - R L^h(u) (Sec. V.B) of the finest
// field u, through the coarse level's scratch: R u and R d by the restriction pass, the FAS
// right-hand side fH = L^H(R u) - R d, then tau = fH - R f_src (synchronises).  tau_out: the
// tau field (may be null).
int tau_rms(mgfr_ctx* c, const Hier& h, const mgfr::Grid& g0, const double* u, const double* rho, hipStream_t s,
            double* rms, double* tau_out)
{
    if (h.nlev < 2) {
        *rms = 0.0;
        return MGFR_OK;
    }
    Level& H = h.lv[1];
    if (g0.n >= mgfr::fused_sweep_min_n()) {
        mgfr::ResidStream a{};
        a.ti = mgfr::resid_stream_planes(g0.n);
        a.uc = H.u;
        a.uhat = H.uhat;
        a.fc = H.f;
        MGFR_TRY(hip_check(c, mgfr::resid_stream(g0, u, rho, a, s), "resid_stream"));
    } else {
        MGFR_TRY(hip_check(c, mgfr::resid_restrict(g0, u, rho, H.u, H.uhat, H.f, s), "resid_restrict"));
    }
    MGFR_TRY(hip_check(c, mgfr::fas_rhs(H.g, H.uhat, H.f, s), "fas_rhs"));
    const int nb = mgfr::tau_finish(g0, rho, H.f, tau_out, h.partial, s);
    if (nb < 0) return hip_check(c, hipGetLastError(), "tau_finish");
    MGFR_TRY(hip_check(c, mgfr::fold_partials(h.partial, nb, h.red, s), "fold_partials"));
    double r[2];
    MGFR_TRY(read_red(c, h, s, r));
    *rms = std::sqrt(r[0] / (double)mgfr::cells(H.g));
    return MGFR_OK;
}

// Stop test of the domain solves: rms(L) <= tol, or <= tau_alpha x rms(tau) when tau_alpha > 0.
int converged(mgfr_ctx* c, const Hier& h, const mgfr_opts* o, const mgfr::Grid& g0, const double* u,
              const double* rho, hipStream_t s, double rms, bool* done)
{
    *done = !(rms > o->tol);
    if (*done || !(o->tau_alpha > 0.0) || !std::isfinite(rms)) return MGFR_OK;
    double t;
    MGFR_TRY(tau_rms(c, h, g0, u, rho, s, &t, nullptr));
    c->stats.tau_rms = t;
    *done = rms <= o->tau_alpha * t;
    return MGFR_OK;
}

}  // namespace

extern "C" {

int mgfr_tau(mgfr_ctx* c, const double* rho, const double* u, int N, const mgfr_params* params, int flags,
             double* tau, double* rms, void* stream)
{
    if (!c) return MGFR_EINVAL;
    c->err.clear();
    Model md;
    if (!rho || !u || !is_pow2(N) || N < 4 || N > 1024) return c->fail(MGFR_EINVAL, "invalid arguments");
    if (derive_model(params, &md) != MGFR_OK) return c->fail(MGFR_EINVAL, "invalid model parameters");
    MGFR_TRY(hip_check(c, hipSetDevice(c->device), "hipSetDevice"));
    MGFR_TRY(ensure_scratch(c));
    hipStream_t s = (hipStream_t)stream;
    const int coarsest = c->coarsest >= 2 && c->coarsest <= N / 2 ? c->coarsest : 2;
    MGFR_TRY(ensure_levels(c, N, coarsest));
    const Hier h = ctx_hier(c);
    Level& L0 = h.lv[0];
    MGFR_TRY(finest_grid(c, h, md, rho, N, flags, 0.0, s, &L0.g));
    for (size_t m = 1; m < h.nlev; ++m) {
        const int n = N >> m;
        h.lv[m].g = make_grid(md, n, 1.0 / n, 0.0);
    }
    double r;
    MGFR_TRY(tau_rms(c, h, L0.g, u, rho, s, &r, tau));
    if (rms) *rms = r;
    return MGFR_OK;
}

int mgfr_residual(mgfr_ctx* c, const double* rho, const double* u, int N, const mgfr_params* params,
                  int flags, double* d, void* stream)
{
    if (!c) return MGFR_EINVAL;
    Model md;
    if (!rho || !u || !d || !is_pow2(N) || N < 2) return c->fail(MGFR_EINVAL, "invalid arguments");
    if (derive_model(params, &md) != MGFR_OK) return c->fail(MGFR_EINVAL, "invalid model parameters");
    MGFR_TRY(hip_check(c, hipSetDevice(c->device), "hipSetDevice"));
    MGFR_TRY(ensure_scratch(c));
    hipStream_t s = (hipStream_t)stream;
    mgfr::Grid g;
    MGFR_TRY(finest_grid(c, ctx_hier(c), md, rho, N, flags, 0.0, s, &g));
    return hip_check(c, mgfr::residual_field(g, u, rho, d, s), "residual_field");
}

int mgfr_smooth(mgfr_ctx* c, const double* rho, double* u, int N, const mgfr_params* params,
                const mgfr_opts* o, int nsweeps, int variant, void* stream)
{
    if (!c) return MGFR_EINVAL;
    c->err.clear();
    c->stats = mgfr_stats{};
    MGFR_TRY(check_opts(c, o));
    Model md;
    if (derive_model(params, &md) != MGFR_OK) return c->fail(MGFR_EINVAL, "invalid model parameters");
    if (!rho || !u || !is_pow2(N) || N < 2 || N > 1024 || nsweeps < 0 || variant < 0 || variant > 2)
        return c->fail(MGFR_EINVAL, "invalid arguments");
    if (variant == 2 && N < mgfr::fused_sweep_min_n())
        return c->fail(MGFR_EINVAL, "the fused sweep needs N >= %d", mgfr::fused_sweep_min_n());
    MGFR_TRY(hip_check(c, hipSetDevice(c->device), "hipSetDevice"));
    hipStream_t s = (hipStream_t)stream;
    MGFR_TRY(ensure_scratch(c));
    MGFR_TRY(ensure_levels(c, N, std::min(N, o->coarsest_n)));
    const Hier h = ctx_hier(c);
    Level& L0 = h.lv[0];
    MGFR_TRY(finest_grid(c, h, md, rho, N, o->flags, o->max_step, s, &L0.g));
    L0.u = u;
    Cycle cyc{c, h, o, s};
    cyc.finest_src = rho;
    cyc.o_simple = variant == 1;
    c->ev_used = 0;
    double* cur = u;
    for (int k = 0; k < nsweeps; ++k) MGFR_TRY(cyc.sweep(0, rho, cur));
    if (cur != u)
        MGFR_TRY(hip_check(c, hipMemcpyAsync(u, cur, sizeof(double) * mgfr::cells(L0.g), hipMemcpyDeviceToDevice, s),
                           "hipMemcpyAsync"));
    return cyc.harvest();
}

int mgfr_smooth32(mgfr_ctx* c, const float* ub, float* e, const float* f, int N, const mgfr_params* params,
                  const mgfr_opts* o, int nsweeps, int variant, void* stream)
{
    if (!c) return MGFR_EINVAL;
    c->err.clear();
    c->stats = mgfr_stats{};
    MGFR_TRY(check_opts(c, o));
    Model md;
    if (derive_model(params, &md) != MGFR_OK) return c->fail(MGFR_EINVAL, "invalid model parameters");
    if (!ub || !e || !f || !is_pow2(N) || N < 2 || N > 1024 || nsweeps < 0 || variant < 0 || variant > 2)
        return c->fail(MGFR_EINVAL, "invalid arguments");
    const bool fused = variant == 2 || (variant == 0 && N >= mgfr::fused_sweep_min_n());
    if (fused && N < mgfr::fused_sweep_min_n())
        return c->fail(MGFR_EINVAL, "the fused sweep needs N >= %d", mgfr::fused_sweep_min_n());
    if (fused && o->planes > 0 && (o->planes > N || (o->planes & 3)))
        return c->fail(MGFR_EINVAL, "planes=%d must be a multiple of 4 and <= N", o->planes);
    MGFR_TRY(hip_check(c, hipSetDevice(c->device), "hipSetDevice"));
    hipStream_t s = (hipStream_t)stream;
    MGFR_TRY(ensure_scratch(c));
    if (fused) MGFR_TRY(ensure_levels32(c, N, std::min(N, o->coarsest_n)));
    const mgfr::Grid g = make_grid(md, N, 1.0 / N, o->max_step);
    const bool timed = (o->flags & MGFR_PROFILE) != 0;
    c->ev_used = 0;
    float* cur = e;
    for (int k = 0; k < nsweeps; ++k) {
        if (timed) {
            if ((size_t)c->ev_used + 2 > c->ev.size()) {
                for (int q = 0; q < 64; ++q) {
                    hipEvent_t ev;
                    MGFR_TRY(hip_check(c, hipEventCreate(&ev), "hipEventCreate"));
                    c->ev.push_back(ev);
                }
            }
            MGFR_TRY(hip_check(c, hipEventRecord(c->ev[c->ev_used], s), "hipEventRecord"));
        }
        if (fused) {
            float* out = cur == e ? c->lv32[0].ealt : e;
            MGFR_TRY(hip_check(c, mgfr::ngs_sweep32_fused(g, ub, cur, out, f, planes_for32(o, 0, N), tile_for32(o, 0), s),
                               "ngs_sweep32_fused"));
            cur = out;
        } else {
            MGFR_TRY(hip_check(c, mgfr::ngs_sweep32(g, ub, cur, f, s), "ngs_sweep32"));
        }
        if (timed) {
            MGFR_TRY(hip_check(c, hipEventRecord(c->ev[c->ev_used + 1], s), "hipEventRecord"));
            c->ev_used += 2;
            c->stats.sweep_launches += fused ? 1 : 2;
            c->stats.sweep_bytes += 12.0 * (double)mgfr::cells(g);
        }
        c->stats.cell_updates += mgfr::cells(g);
        c->stats.finest_updates += mgfr::cells(g);
    }
    if (cur != e)
        MGFR_TRY(hip_check(c, hipMemcpyAsync(e, cur, sizeof(float) * mgfr::cells(g), hipMemcpyDeviceToDevice, s),
                           "hipMemcpyAsync"));
    const Hier h = ctx_hier(c);
    Cycle cyc{c, h, o, s};
    return cyc.harvest();
}

}  // extern "C"

namespace {

// FP64 stop test inside a captured graph: the finest residual's block sums, their fold into
// h.red and the device stop test.
int norm_and_stop(mgfr_ctx* c, const Hier& h, const mgfr::Grid& g, const double* u, const double* rho,
                  const mgfr_opts* o, hipStream_t s)
{
    if (g.n >= mgfr::fused_sweep_min_n()) {
        mgfr::ResidStream a{};
        a.ti = mgfr::resid_stream_planes(g.n);
        a.partial = h.partial;
        MGFR_TRY(hip_check(c, mgfr::resid_stream(g, u, rho, a, s), "resid_stream"));
        MGFR_TRY(hip_check(c, mgfr::fold_partials(h.partial, (int)mgfr::resid_stream_blocks(g.n), h.red, s),
                           "fold_partials"));
    } else {
        MGFR_TRY(hip_check(c, mgfr::residual_norm(g, u, rho, h.partial, h.red, s), "residual_norm"));
    }
    return hip_check(c, mgfr::domain_stop(h.red, mgfr::cells(g), o->tol, o->max_cycles, c->ghist, c->gstate, s),
                     "domain_stop");
}

// What a captured domain solve depends on besides the data: replayed only while all of it
// is unchanged.
struct GraphKey {
    const void *rho, *u, *lv, *lv32, *partial, *red, *counter, *alt;
    int N, precision, pre, post, inner, cap, planes, tile, max_cycles, nlev, nlev32;
    double tol, rtol;
    mgfr::Grid g0;
};

// Replays body (two cycles, each ending in the device stop test) from a graph until the
// stop test has stopped the solve; *k gets the cycles run, *rms the last residual and
// res_hist[1 .. k] the history.  Every level's kernels return at once after the stop.
template <class Body>
int run_graph(mgfr_ctx* c, const Hier& h, const mgfr_opts* o, const double* rho, double* u, int N, hipStream_t s,
              Body body, double* res_hist, int* k, double* rms)
{
    const int H = o->max_cycles + 1;
    if (c->ghist_n < H) {
        (void)hipFree(c->ghist);
        c->ghist = nullptr;
        c->ghist_n = 0;
        if (hipMalloc(&c->ghist, sizeof(double) * H) != hipSuccess) return c->fail(MGFR_ENOMEM, "hipMalloc failed");
        c->ghist_n = H;
    }
    if (!c->gstate && hipMalloc(&c->gstate, 2 * sizeof(int)) != hipSuccess) {
        c->gstate = nullptr;
        return c->fail(MGFR_ENOMEM, "hipMalloc failed");
    }
    int* halt = c->gstate + 1;
    for (size_t m = 0; m < h.nlev; ++m) h.lv[m].g.halt = halt;
    for (size_t m = 0; m < h.nlev32; ++m) h.lv32[m].g.halt = halt;
    GraphKey key;
    std::memset(&key, 0, sizeof key);
    key.rho = rho;
    key.u = u;
    key.lv = h.lv;
    key.lv32 = h.lv32;
    key.partial = h.partial;
    key.red = h.red;
    key.counter = h.counter;
    key.alt = h.lv[0].alt;
    key.N = N;
    key.precision = o->precision;
    key.pre = o->pre;
    key.post = o->post;
    key.inner = o->inner_cycles;
    key.cap = o->coarsest_sweeps;
    key.planes = o->planes;
    key.tile = o->tile;
    key.max_cycles = o->max_cycles;
    key.nlev = (int)h.nlev;
    key.nlev32 = (int)h.nlev32;
    key.tol = o->tol;
    key.rtol = o->coarsest_rtol;
    key.g0 = h.lv[0].g;
    auto restore = [&]() {
        for (size_t m = 0; m < h.nlev; ++m) h.lv[m].g.halt = nullptr;
        for (size_t m = 0; m < h.nlev32; ++m) h.lv32[m].g.halt = nullptr;
    };
    int st = MGFR_OK;
    if (!c->dgexec || c->dkey.size() != sizeof key || std::memcmp(c->dkey.data(), &key, sizeof key) != 0) {
        if (c->dgexec) (void)hipGraphExecDestroy(c->dgexec);
        if (c->dgraph) (void)hipGraphDestroy(c->dgraph);
        c->dgexec = nullptr;
        c->dgraph = nullptr;
        c->dkey.clear();
        if (!c->dcap && hipStreamCreateWithFlags(&c->dcap, hipStreamNonBlocking) != hipSuccess) {
            c->dcap = nullptr;
            restore();
            return c->fail(MGFR_EDEVICE, "hipStreamCreate failed");
        }
        const mgfr_stats base = c->stats;
        st = hip_check(c, hipStreamBeginCapture(c->dcap, hipStreamCaptureModeThreadLocal), "hipStreamBeginCapture");
        if (st == MGFR_OK) {
            st = body(c->dcap);
            hipGraph_t g = nullptr;
            const hipError_t e = hipStreamEndCapture(c->dcap, &g);
            c->dgraph = g;
            if (st == MGFR_OK) st = hip_check(c, e, "hipStreamEndCapture");
            if (st == MGFR_OK)
                st = hip_check(c, hipGraphInstantiate(&c->dgexec, c->dgraph, nullptr, nullptr, 0), "hipGraphInstantiate");
        }
        // what one cycle of the graph adds to the counters (the capture ran two)
        c->dper_updates = (c->stats.cell_updates - base.cell_updates) / 2;
        c->dper_finest = (c->stats.finest_updates - base.finest_updates) / 2;
        c->dper_inner = (c->stats.inner_cycles - base.inner_cycles) / 2;
        c->stats = base;
        if (st != MGFR_OK) {
            restore();
            return st;
        }
        c->dkey.assign((const char*)&key, (const char*)&key + sizeof key);
    }
    MGFR_TRY(hip_check(c, mgfr::fill_int(c->gstate, 0, 2, s), "fill_int"));
    int* hs = (int*)c->host_red;
    hs[0] = hs[1] = 0;
    // two cycles per launch; the stop test ends the solve by max_cycles at the latest
    for (int launch = 0; launch <= o->max_cycles / 2 && !hs[1]; ++launch) {
        MGFR_TRY(hip_check(c, hipGraphLaunch(c->dgexec, s), "hipGraphLaunch"));
        MGFR_TRY(hip_check(c, hipMemcpyAsync(hs, c->gstate, 2 * sizeof(int), hipMemcpyDeviceToHost, s),
                           "hipMemcpyAsync"));
        MGFR_TRY(hip_check(c, hipStreamSynchronize(s), "hipStreamSynchronize"));
    }
    restore();
    *k = hs[0];
    if (*k > 0) {
        MGFR_TRY(hip_check(c, hipMemcpyAsync(c->host_red, c->ghist + *k, sizeof(double), hipMemcpyDeviceToHost, s),
                           "hipMemcpyAsync"));
        if (res_hist)
            MGFR_TRY(hip_check(c, hipMemcpyAsync(res_hist + 1, c->ghist + 1, sizeof(double) * *k, hipMemcpyDeviceToHost, s),
                               "hipMemcpyAsync"));
        MGFR_TRY(hip_check(c, hipStreamSynchronize(s), "hipStreamSynchronize"));
        *rms = c->host_red[0];
    }
    c->stats.cell_updates += c->dper_updates * *k;
    c->stats.finest_updates += c->dper_finest * *k;
    c->stats.inner_cycles += c->dper_inner * *k;
    return MGFR_OK;
}

// The domain solve on the storage h, whose levels (and single-precision levels for the
// mixed solver) are sized for N; level 0's u is the caller's.  Allocates nothing (unless
// MGFR_GRAPH, whose graph and device stop state are kept in the context).
int solve_body(mgfr_ctx* c, const Hier& h, const Model& md, const double* rho, int N, const mgfr_opts* o,
               double* u, double* res_hist, int* n_hist, hipStream_t s,
               std::chrono::steady_clock::time_point t0, bool graphs)
{
    const long long ncell = (long long)N * N * N;
    Level& L0 = h.lv[0];
    MGFR_TRY(finest_grid(c, h, md, rho, N, o->flags, o->max_step, s, &L0.g));
    L0.u = u;
    for (size_t m = 1; m < h.nlev; ++m) {
        const int n = N >> m;
        h.lv[m].g = make_grid(md, n, 1.0 / n, o->max_step);
    }

    double r[2];
    if (o->flags & MGFR_WARM_START) {
        MGFR_TRY(hip_check(c, mgfr::sum_and_count_nonfinite(u, ncell, h.partial, h.red, s), "start check"));
        MGFR_TRY(read_red(c, h, s, r));
        if (r[1] != 0.0) return c->fail(MGFR_ENONFINITE, "start field has %.0f non-finite cells", r[1]);
    } else {
        MGFR_TRY(hip_check(c, mgfr::fill(u, md.ubar, ncell, s), "fill"));
    }

    Cycle cyc{c, h, o, s};
    cyc.finest_src = rho;
    c->ev_used = 0;
    MGFR_TRY(hip_check(c, hipMemsetAsync(h.counter, 0, sizeof(long long), s), "hipMemsetAsync"));
    double rms;
    int k = 0;
    bool stop = false;  // the stop test passed
    // MGFR_GRAPH: the cycles are captured once, with the stop test on the device, and replayed
    // until it stops them (the rms test only: the truncation-error rule and event timing stay
    // eager, as does an odd sweep count, whose finest level ends in the second buffer)
    const bool graph = (o->flags & MGFR_GRAPH) && !(o->flags & MGFR_PROFILE) && !(o->tau_alpha > 0.0) &&
                       (o->pre + o->post) % 2 == 0 && graphs;
    if (o->precision == MGFR_FP64) {
        MGFR_TRY(finest_norm(c, h, L0.g, u, rho, s, &rms, nullptr));
        if (res_hist) res_hist[0] = rms;
        MGFR_TRY(converged(c, h, o, L0.g, u, rho, s, rms, &stop));
        if (graph && std::isfinite(rms) && !stop && k < o->max_cycles) {
            auto body = [&](hipStream_t st) -> int {
                const hipStream_t keep = s;
                s = st;
                cyc.s = st;
                int r = MGFR_OK;
                for (int it = 0; it < 2 && r == MGFR_OK; ++it) {
                    r = cyc.vcycle(0);
                    if (r == MGFR_OK) r = norm_and_stop(c, h, L0.g, u, rho, o, st);
                }
                s = keep;
                cyc.s = keep;
                return r;
            };
            MGFR_TRY(run_graph(c, h, o, rho, u, N, s, body, res_hist, &k, &rms));
            stop = !(rms > o->tol);
        }
        while (std::isfinite(rms) && !stop && k < o->max_cycles) {
            MGFR_TRY(cyc.vcycle(0));
            MGFR_TRY(finest_norm(c, h, L0.g, u, rho, s, &rms, nullptr));
            MGFR_TRY(cyc.harvest());
            ++k;
            if (res_hist) res_hist[k] = rms;
            MGFR_TRY(converged(c, h, o, L0.g, u, rho, s, rms, &stop));
        }
    } else {
        // Defect correction: d = L(u) - f in double precision; a single-precision FAS
        // multigrid solves N(e) = -d for the correction; u += e; repeat.
        for (size_t m = 0; m < h.nlev32; ++m) h.lv32[m].g = h.lv[m].g;
        Level32& I0 = h.lv32[0];
        Cycle32 cyc32{c, h, o, s};
        const bool stream = N >= mgfr::fused_sweep_min_n();
        double* ucur = u;
        // residual of ucur (+ e when `update`), cast to the single-precision right-hand side
        auto outer_residual = [&](bool update) -> int {
            if (stream) {
                mgfr::ResidStream a{};
                a.ti = mgfr::resid_stream_planes(N);
                a.partial = h.partial;
                a.r32 = I0.f;
                a.ub32 = I0.ub;
                double* next = ucur;
                if (update) {
                    next = ucur == u ? L0.alt : u;
                    a.e32 = I0.e;
                    a.uout = next;
                }
                MGFR_TRY(hip_check(c, mgfr::resid_stream(L0.g, ucur, rho, a, s), "resid_stream"));
                MGFR_TRY(hip_check(c, mgfr::fold_partials(h.partial, (int)mgfr::resid_stream_blocks(N), h.red, s),
                                   "fold_partials"));
                ucur = next;
            } else {
                if (update) MGFR_TRY(hip_check(c, mgfr::add_correction(ucur, I0.e, ncell, s), "add_correction"));
                MGFR_TRY(hip_check(c, mgfr::residual_cast(L0.g, ucur, rho, I0.f, I0.ub, h.partial, h.red, s),
                                   "residual_cast"));
            }
            double r2[2];
            MGFR_TRY(read_red(c, h, s, r2));
            rms = std::sqrt(r2[0] / (double)ncell);
            return MGFR_OK;
        };
        MGFR_TRY(outer_residual(false));
        if (res_hist) res_hist[0] = rms;
        MGFR_TRY(converged(c, h, o, L0.g, ucur, rho, s, rms, &stop));
        if (graph && std::isfinite(rms) && !stop && k < o->max_cycles) {
            // one outer iteration: coarse bases, e = 0, the inner V-cycles, then u += e with
            // the double-precision residual; u and the second finest buffer alternate, so
            // the graph holds two iterations and the solve starts from u
            auto iteration = [&]() -> int {
                for (size_t m = 1; m < h.nlev32; ++m)
                    MGFR_TRY(hip_check(c, mgfr::restrict_mean32(h.lv32[m].g, h.lv32[m - 1].ub, h.lv32[m].ub, s),
                                       "restrict_mean32"));
                MGFR_TRY(hip_check(c, mgfr::fill32(I0.e, 0.0f, ncell, s), "fill32"));
                for (int ic = 0; ic < o->inner_cycles; ++ic) {
                    MGFR_TRY(cyc32.vcycle(0));
                    ++c->stats.inner_cycles;
                }
                if (stream) {
                    mgfr::ResidStream a{};
                    a.ti = mgfr::resid_stream_planes(N);
                    a.partial = h.partial;
                    a.r32 = I0.f;
                    a.ub32 = I0.ub;
                    double* next = ucur == u ? L0.alt : u;
                    a.e32 = I0.e;
                    a.uout = next;
                    MGFR_TRY(hip_check(c, mgfr::resid_stream(L0.g, ucur, rho, a, s), "resid_stream"));
                    MGFR_TRY(hip_check(c, mgfr::fold_partials(h.partial, (int)mgfr::resid_stream_blocks(N), h.red, s),
                                       "fold_partials"));
                    ucur = next;
                } else {
                    MGFR_TRY(hip_check(c, mgfr::add_correction(ucur, I0.e, ncell, s, L0.g.halt), "add_correction"));
                    MGFR_TRY(hip_check(c, mgfr::residual_cast(L0.g, ucur, rho, I0.f, I0.ub, h.partial, h.red, s),
                                       "residual_cast"));
                }
                return hip_check(c, mgfr::domain_stop(h.red, ncell, o->tol, o->max_cycles, c->ghist, c->gstate, s),
                                 "domain_stop");
            };
            auto body = [&](hipStream_t st) -> int {
                const hipStream_t keep = s;
                s = st;
                cyc.s = st;
                cyc32.s = st;
                int r = iteration();
                if (r == MGFR_OK) r = iteration();
                s = keep;
                cyc.s = keep;
                cyc32.s = keep;
                return r;
            };
            MGFR_TRY(run_graph(c, h, o, rho, u, N, s, body, res_hist, &k, &rms));
            stop = !(rms > o->tol);
            if (stream && (k & 1)) ucur = L0.alt;  // an odd count ends in the second buffer
        }
        while (std::isfinite(rms) && !stop && k < o->max_cycles) {
            for (size_t m = 1; m < h.nlev32; ++m)
                MGFR_TRY(hip_check(c, mgfr::restrict_mean32(h.lv32[m].g, h.lv32[m - 1].ub, h.lv32[m].ub, s),
                                   "restrict_mean32"));
            MGFR_TRY(hip_check(c, mgfr::fill32(I0.e, 0.0f, ncell, s), "fill32"));
            for (int ic = 0; ic < o->inner_cycles; ++ic) {
                MGFR_TRY(cyc32.vcycle(0));
                ++c->stats.inner_cycles;
            }
            MGFR_TRY(outer_residual(true));
            MGFR_TRY(cyc.harvest());
            ++k;
            if (res_hist) res_hist[k] = rms;
            MGFR_TRY(converged(c, h, o, L0.g, ucur, rho, s, rms, &stop));
        }
        if (ucur != u)
            MGFR_TRY(hip_check(c, hipMemcpyAsync(u, ucur, sizeof(double) * ncell, hipMemcpyDeviceToDevice, s),
                               "hipMemcpyAsync"));
    }
    if (n_hist) *n_hist = k + 1;
    {
        long long coarse_sweeps = 0;
        MGFR_TRY(hip_check(c, hipMemcpyAsync(&coarse_sweeps, h.counter, sizeof coarse_sweeps, hipMemcpyDeviceToHost, s),
                           "hipMemcpyAsync"));
        MGFR_TRY(hip_check(c, hipStreamSynchronize(s), "hipStreamSynchronize"));
        const long long nc = mgfr::cells(h.lv[h.nlev - 1].g);
        c->stats.cell_updates += coarse_sweeps * nc;
        if (h.nlev == 1) c->stats.finest_updates += coarse_sweeps * nc;
        c->stats.cycles = k;
        c->stats.solve_ms =
            std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    }
    if (!std::isfinite(rms)) return c->fail(MGFR_ENONFINITE, "residual became non-finite after %d cycles", k);
    if (!stop) return c->fail(MGFR_ENOTCONV, "rms residual %.3e > tol %.3e after %d cycles", rms, o->tol, k);
    return MGFR_OK;
}

}  // namespace

extern "C" {

int mg_fr_solve(mgfr_ctx* c, const double* rho, int N, const mgfr_params* params, const mgfr_opts* o,
                double* u, double* res_hist, int* n_hist, void* stream)
{
    if (!c) return MGFR_EINVAL;
    c->err.clear();
    c->stats = mgfr_stats{};
    const auto t0 = std::chrono::steady_clock::now();
    if (n_hist) *n_hist = 0;
    MGFR_TRY(check_opts(c, o));
    Model md;
    if (derive_model(params, &md) != MGFR_OK) return c->fail(MGFR_EINVAL, "invalid model parameters");
    if (!rho || !u) return c->fail(MGFR_EINVAL, "rho or u is NULL");
    if (!is_pow2(N) || N < o->coarsest_n || N > 1024)
        return c->fail(MGFR_EINVAL, "N=%d must be a power of two in [coarsest_n, 1024]", N);
    MGFR_TRY(hip_check(c, hipSetDevice(c->device), "hipSetDevice"));
    MGFR_TRY(ensure_scratch(c));
    MGFR_TRY(ensure_levels(c, N, o->coarsest_n));
    if (o->precision == MGFR_MIXED) MGFR_TRY(ensure_levels32(c, N, o->coarsest_n));
    Hier h = ctx_hier(c);
    if (o->precision != MGFR_MIXED) h.nlev32 = 0;
    return solve_body(c, h, md, rho, N, o, u, res_hist, n_hist, (hipStream_t)stream, t0, true);
}

int mg_fr_solve_noalloc(mgfr_ctx* c, const double* rho, int N, const mgfr_params* params, const mgfr_opts* o,
                        double* u, double* res_hist, int* n_hist, void* stream)
{
    if (!c) return MGFR_EINVAL;
    c->err.clear();
    c->stats = mgfr_stats{};
    const auto t0 = std::chrono::steady_clock::now();
    if (n_hist) *n_hist = 0;
    MGFR_TRY(check_opts(c, o));
    if (o->flags & MGFR_PROFILE) return c->fail(MGFR_EINVAL, "MGFR_PROFILE needs HIP events: not available here");
    if (o->flags & MGFR_GRAPH)
        return c->fail(MGFR_EINVAL, "MGFR_GRAPH keeps a graph and device state in the context: not available here");
    Model md;
    if (derive_model(params, &md) != MGFR_OK) return c->fail(MGFR_EINVAL, "invalid model parameters");
    if (!rho || !u) return c->fail(MGFR_EINVAL, "rho or u is NULL");
    if (!is_pow2(N) || N < o->coarsest_n || N > kNoAllocMaxN)
        return c->fail(MGFR_EINVAL, "N=%d: this entry point takes powers of two in [coarsest_n, %d]", N, kNoAllocMaxN);
    Level lv[kMaxLevels];
    Level32 lv32[kMaxLevels];
    Hier h;
    const bool mixed = o->precision == MGFR_MIXED;
    const size_t need = carve(nullptr, N, o->coarsest_n, mixed, &h, lv, lv32);
    if (need > kFixedScratchBytes)
        return c->fail(MGFR_EINVAL, "N=%d needs %zu bytes of scratch, more than the %zu held", N, need,
                       kFixedScratchBytes);
    if (!c->fixed_scratch)
        return c->fail(MGFR_EDEVICE, "the fixed scratch array of device %d could not be resolved", c->device);
    MGFR_TRY(hip_check(c, hipSetDevice(c->device), "hipSetDevice"));
    carve((char*)c->fixed_scratch, N, o->coarsest_n, mixed, &h, lv, lv32);
    h.host = c->fixed_host;
    return solve_body(c, h, md, rho, N, o, u, res_hist, n_hist, (hipStream_t)stream, t0, false);
}

}  // extern "C"

extern "C" {

int mgfr_autotune(mgfr_ctx* c, const double* rho, int N, const mgfr_params* params, const mgfr_opts* base,
                  double* u_scratch, mgfr_opts* best, double* best_ms, void* stream)
{
    if (!c) return MGFR_EINVAL;
    if (!base || !best || !u_scratch) return c->fail(MGFR_EINVAL, "invalid autotune arguments");
    MGFR_TRY(check_opts(c, base));
    const int H = base->max_cycles + 1;
    std::vector<double> hist(H);
    double best_t = -1.0;
    mgfr_opts cur_best = *base;
    auto trial = [&](const mgfr_opts& o, double* t) -> int {
        double tmin = -1.0;
        for (int rep = 0; rep < 2; ++rep) {
            int nh = 0;
            mgfr_opts oo = o;
            oo.flags &= ~(MGFR_WARM_START | MGFR_PROFILE);
            const int st = mg_fr_solve(c, rho, N, params, &oo, u_scratch, hist.data(), &nh, stream);
            if (st == MGFR_ENOTCONV || st == MGFR_ENONFINITE) {
                *t = -1.0;
                return MGFR_OK;
            }
            if (st != MGFR_OK) return st;
            if (tmin < 0.0 || c->stats.solve_ms < tmin) tmin = c->stats.solve_ms;
        }
        *t = tmin;
        return MGFR_OK;
    };
    auto consider = [&](const mgfr_opts& o) -> int {
        double t;
        MGFR_TRY(trial(o, &t));
        if (t > 0.0 && (best_t < 0.0 || t < best_t)) {
            best_t = t;
            cur_best = o;
        }
        return MGFR_OK;
    };
    // stage 1: sweeps before / after the coarse step (and inner cycles for mixed)
    const int sweeps[][2] = {{1, 1}, {2, 1}, {1, 2}, {2, 2}, {3, 3}};
    const int inners[] = {1, 2, 3};
    for (const auto& pp : sweeps)
        for (int ic : inners) {
            if (ic > 1 && base->precision != MGFR_MIXED) continue;
            mgfr_opts o = *base;
            o.pre = pp[0];
            o.post = pp[1];
            o.inner_cycles = ic;
            MGFR_TRY(consider(o));
        }
    // stage 2: planes per workgroup of the finest-level fused sweep
    if (N >= mgfr::fused_sweep_min_n()) {
        const mgfr_opts stage1 = cur_best;
        for (int planes = 8; planes <= 128 && planes <= N; planes *= 2) {
            mgfr_opts o = stage1;
            o.planes = planes;
            MGFR_TRY(consider(o));
        }
        // stage 3: its tile (double precision: 16 x 64 or 8 x 64; single precision: 16 x 32,
        // 32 x 32, 16 x 64 or 32 x 64 with one column pair per thread, or 8 x 32 with pairs
        // over the halo)
        const mgfr_opts stage2 = cur_best;
        const int ntile = base->precision == MGFR_MIXED ? 5 : 2;
        for (int tile = 1; tile <= ntile; ++tile) {
            mgfr_opts o = stage2;
            o.tile = tile;
            if (o.planes == 0) o.planes = base->precision == MGFR_MIXED ? planes_for32(&o, 0, N) : planes_for(&o, 0, N);
            MGFR_TRY(consider(o));
        }
    }
    if (best_t < 0.0) return c->fail(MGFR_ENOTCONV, "no candidate setting converged");
    *best = cur_best;
    if (best_ms) *best_ms = best_t;
    c->err.clear();
    return MGFR_OK;
}

}  // extern "C"
