// Host side of libmgfr.so: model constants, the multigrid hierarchy, the V-cycle driver
// and the C ABI declared in include/mgfr.h.
#include <hip/hip_runtime.h>

#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "../../include/mgfr.h"
#include "mgfr_impl.h"

namespace {

// Derived model constants (Sec. II, Sec. III.A, Sec. VI.A.1).
struct Model {
    double xi, ct, K, A, Sbar, D, ubar, inv_np1;
};

int derive_model(const mgfr_params* p, Model* m)
{
    if (!p) return MGFR_EINVAL;
    const double om = p->omega_m, a = p->a, n = p->n;
    const double ol = p->omega_l < 0.0 ? 1.0 - om : p->omega_l;
    if (!(om > 0.0) || !(a > 0.0) || !(n > 0.0) || !(p->fr0_abs > 0.0) || !(p->box_mpc_h > 0.0) ||
        !(ol >= 0.0) || !std::isfinite(om + a + n + p->fr0_abs + p->box_mpc_h + ol))
        return MGFR_EINVAL;
    // present background: f_R0 = -n xi / [3 (1 + 4 OL/Om)]^(n+1)
    m->xi = p->fr0_abs * std::pow(3.0 * (1.0 + 4.0 * ol / om), n + 1.0) / n;
    // c~ = c / (B H0), c = 299792.458 km/s, H0 = 100 h km/s/Mpc
    m->ct = 299792.458 / (100.0 * p->box_mpc_h);
    const double q = std::pow(a, -3.0) + 4.0 * ol / om;
    m->K = std::pow(n * a * a * m->xi, 1.0 / (n + 1.0));
    m->A = om * std::pow(a, 4.0) * m->K / 3.0;
    m->Sbar = om * std::pow(a, 4.0) * q;
    m->D = om * a;
    m->ubar = std::log(n * a * a * m->xi / std::pow(3.0 * q, n + 1.0));
    m->inv_np1 = 1.0 / (n + 1.0);
    return MGFR_OK;
}

int ilog2(int x)
{
    int l = 0;
    while ((1 << l) < x) ++l;
    return l;
}

bool is_pow2(int x) { return x > 0 && (x & (x - 1)) == 0; }

struct Level {
    mgfr::Grid g;
    double* u = nullptr;     // level 0: the caller's u
    double* uhat = nullptr;  // R u of the finer level (m >= 1)
    double* f = nullptr;     // FAS right-hand side (m >= 1)
};

}  // namespace

struct mgfr_ctx {
    int device = 0;
    std::string err;
    // hierarchy for one finest size, kept between calls
    int N = 0, coarsest = 0;
    std::vector<Level> lv;
    double* partial = nullptr;  // reduction scratch
    double* red = nullptr;      // device result of a reduction (2 doubles)
    double* host_red = nullptr; // pinned copy of it
    long long* counter = nullptr;  // device: coarsest-level sweeps of the current solve
    mgfr_stats stats{};
    // MGFR_PROFILE: event pairs around finest-level smoother launches
    std::vector<hipEvent_t> ev;
    int ev_used = 0;

    int fail(int code, const char* fmt, ...)
    {
        char buf[512];
        va_list ap;
        va_start(ap, fmt);
        vsnprintf(buf, sizeof buf, fmt, ap);
        va_end(ap);
        err = buf;
        return code;
    }

    void free_levels()
    {
        for (size_t m = 1; m < lv.size(); ++m) {
            (void)hipFree(lv[m].u);
            (void)hipFree(lv[m].uhat);
            (void)hipFree(lv[m].f);
        }
        lv.clear();
        N = 0;
    }
};

namespace {

int hip_check(mgfr_ctx* c, hipError_t e, const char* what)
{
    if (e == hipSuccess) return MGFR_OK;
    return c->fail(MGFR_EDEVICE, "%s: %s", what, hipGetErrorString(e));
}

#define MGFR_TRY(expr)                       \
    do {                                     \
        int rc_ = (expr);                    \
        if (rc_ != MGFR_OK) return rc_;      \
    } while (0)

int check_opts(mgfr_ctx* c, const mgfr_opts* o)
{
    if (!o) return c->fail(MGFR_EINVAL, "opts is NULL");
    if (!(o->tol >= 0.0) || o->pre < 0 || o->post < 0 || o->max_cycles < 0 || o->coarsest_sweeps < 0 ||
        !is_pow2(o->coarsest_n) || o->coarsest_n < 2 || o->coarsest_n > 8 || !(o->max_step >= 0.0) ||
        !(o->coarsest_rtol >= 0.0) || (o->precision != MGFR_FP64 && o->precision != MGFR_MIXED) ||
        o->inner_cycles < 1)
        return c->fail(MGFR_EINVAL, "invalid options (tol=%g pre=%d post=%d coarsest_n=%d precision=%d)",
                       o->tol, o->pre, o->post, o->coarsest_n, o->precision);
    return MGFR_OK;
}

mgfr::Grid make_grid(const Model& md, int n, double h, double max_step)
{
    mgfr::Grid g;
    g.n = n;
    g.lg = ilog2(n);
    g.C = md.ct * md.ct / (2.0 * h * h);
    g.A = md.A;
    g.inv_np1 = md.inv_np1;
    g.max_step = max_step;
    g.fscale = 1.0;
    g.sref = 0.0;
    g.fshift = 0.0;
    return g;
}

int ensure_scratch(mgfr_ctx* c)
{
    if (!c->partial) {
        if (hipMalloc(&c->partial, sizeof(double) * mgfr::reduction_scratch()) != hipSuccess)
            return c->fail(MGFR_ENOMEM, "hipMalloc of reduction scratch failed");
        if (hipMalloc(&c->red, sizeof(double) * 2) != hipSuccess)
            return c->fail(MGFR_ENOMEM, "hipMalloc of reduction result failed");
        if (hipHostMalloc(&c->host_red, sizeof(double) * 2, hipHostMallocDefault) != hipSuccess)
            return c->fail(MGFR_ENOMEM, "hipHostMalloc failed");
        if (hipMalloc(&c->counter, sizeof(long long)) != hipSuccess)
            return c->fail(MGFR_ENOMEM, "hipMalloc of the sweep counter failed");
    }
    return MGFR_OK;
}

// Allocates levels N/2 ... coarsest (level 0 uses the caller's arrays).
int ensure_levels(mgfr_ctx* c, int N, int coarsest)
{
    if (c->N == N && c->coarsest == coarsest) return MGFR_OK;
    c->free_levels();
    c->lv.emplace_back();
    for (int n = N / 2; n >= coarsest; n /= 2) {
        Level L;
        const size_t bytes = sizeof(double) * (size_t)n * n * n;
        if (hipMalloc(&L.u, bytes) != hipSuccess || hipMalloc(&L.uhat, bytes) != hipSuccess ||
            hipMalloc(&L.f, bytes) != hipSuccess) {
            (void)hipFree(L.u);
            (void)hipFree(L.uhat);
            (void)hipFree(L.f);
            c->free_levels();
            return c->fail(MGFR_ENOMEM, "hipMalloc of the %d^3 level failed", n);
        }
        c->lv.push_back(L);
    }
    c->N = N;
    c->coarsest = coarsest;
    return MGFR_OK;
}

// Copies a 2-double device reduction result to the host (synchronises the stream).
int read_reduction(mgfr_ctx* c, hipStream_t s, double* out2)
{
    MGFR_TRY(hip_check(c, hipMemcpyAsync(c->host_red, c->red, 2 * sizeof(double), hipMemcpyDeviceToHost, s),
                       "hipMemcpyAsync"));
    MGFR_TRY(hip_check(c, hipStreamSynchronize(s), "hipStreamSynchronize"));
    out2[0] = c->host_red[0];
    out2[1] = c->host_red[1];
    return MGFR_OK;
}

struct Cycle {
    mgfr_ctx* c;
    const mgfr_opts* o;
    hipStream_t s;
    const double* finest_src = nullptr;

    // One smoother sweep on level m; finest-level sweeps are timed under MGFR_PROFILE.
    int sweep(size_t m, const double* src)
    {
        Level& L = c->lv[m];
        const bool timed = m == 0 && (o->flags & MGFR_PROFILE);
        if (timed) {
            if ((size_t)c->ev_used + 2 > c->ev.size()) {
                for (int k = 0; k < 64; ++k) {
                    hipEvent_t e;
                    MGFR_TRY(hip_check(c, hipEventCreate(&e), "hipEventCreate"));
                    c->ev.push_back(e);
                }
            }
            MGFR_TRY(hip_check(c, hipEventRecord(c->ev[c->ev_used], s), "hipEventRecord"));
        }
        MGFR_TRY(hip_check(c, mgfr::ngs_sweep(L.g, L.u, src, s), "ngs_sweep"));
        if (timed) {
            MGFR_TRY(hip_check(c, hipEventRecord(c->ev[c->ev_used + 1], s), "hipEventRecord"));
            c->ev_used += 2;
            c->stats.sweep_launches += 2;
            c->stats.sweep_bytes += 2.0 * 12.0 * (double)mgfr::cells(L.g);
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
        Level& L = c->lv[m];
        const double* src = m == 0 ? finest_src : L.f;
        if (m + 1 == c->lv.size()) {
            return hip_check(c, mgfr::coarsest_solve(L.g, L.u, src, o->coarsest_sweeps, o->coarsest_rtol,
                                                     c->counter, s),
                             "coarsest_solve");
        }
        for (int k = 0; k < o->pre; ++k) MGFR_TRY(sweep(m, src));
        Level& H = c->lv[m + 1];
        MGFR_TRY(hip_check(c, mgfr::resid_restrict(L.g, L.u, src, H.u, H.uhat, H.f, s), "resid_restrict"));
        MGFR_TRY(hip_check(c, mgfr::fas_rhs(H.g, H.uhat, H.f, s), "fas_rhs"));
        MGFR_TRY(vcycle(m + 1));
        MGFR_TRY(hip_check(c, mgfr::prolong_correct(H.g, L.u, H.u, H.uhat, s), "prolong_correct"));
        for (int k = 0; k < o->post; ++k) MGFR_TRY(sweep(m, src));
        return MGFR_OK;
    }
};

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
    *ctx = c;
    return MGFR_OK;
}

void mgfr_destroy(mgfr_ctx* c)
{
    if (!c) return;
    (void)hipSetDevice(c->device);
    (void)hipDeviceSynchronize();
    c->free_levels();
    (void)hipFree(c->partial);
    (void)hipFree(c->red);
    (void)hipFree(c->counter);
    for (hipEvent_t e : c->ev) (void)hipEventDestroy(e);
    if (c->host_red) (void)hipHostFree(c->host_red);
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
int finest_grid(mgfr_ctx* c, const Model& md, const double* rho, int N, int flags, double max_step,
                hipStream_t s, mgfr::Grid* g)
{
    *g = make_grid(md, N, 1.0 / N, max_step);
    const long long ncell = (long long)N * N * N;
    MGFR_TRY(hip_check(c, mgfr::sum_and_count_nonfinite(rho, ncell, c->partial, c->red, s), "density check"));
    double r[2];
    MGFR_TRY(read_reduction(c, s, r));
    if (r[1] != 0.0) return c->fail(MGFR_ENONFINITE, "density has %.0f non-finite cells", r[1]);
    g->fscale = md.D;
    g->sref = (flags & MGFR_SUBTRACT_MEAN) ? r[0] / (double)ncell : 1.0;
    g->fshift = md.Sbar;
    return MGFR_OK;
}

}  // namespace

extern "C" {

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
    MGFR_TRY(finest_grid(c, md, rho, N, flags, 0.0, s, &g));
    return hip_check(c, mgfr::residual_field(g, u, rho, d, s), "residual_field");
}

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
    if (!is_pow2(N) || N < o->coarsest_n || N > 2048)
        return c->fail(MGFR_EINVAL, "N=%d must be a power of two in [coarsest_n, 2048]", N);
    if (o->precision != MGFR_FP64) return c->fail(MGFR_EINVAL, "precision %d not available", o->precision);
    MGFR_TRY(hip_check(c, hipSetDevice(c->device), "hipSetDevice"));
    hipStream_t s = (hipStream_t)stream;
    MGFR_TRY(ensure_scratch(c));
    MGFR_TRY(ensure_levels(c, N, o->coarsest_n));
    const long long ncell = (long long)N * N * N;

    Level& L0 = c->lv[0];
    MGFR_TRY(finest_grid(c, md, rho, N, o->flags, o->max_step, s, &L0.g));
    L0.u = u;
    for (size_t m = 1; m < c->lv.size(); ++m) {
        const int n = N >> m;
        c->lv[m].g = make_grid(md, n, 1.0 / n, o->max_step);
    }

    double r[2];
    if (o->flags & MGFR_WARM_START) {
        MGFR_TRY(hip_check(c, mgfr::sum_and_count_nonfinite(u, ncell, c->partial, c->red, s), "start check"));
        MGFR_TRY(read_reduction(c, s, r));
        if (r[1] != 0.0) return c->fail(MGFR_ENONFINITE, "start field has %.0f non-finite cells", r[1]);
    } else {
        MGFR_TRY(hip_check(c, mgfr::fill(u, md.ubar, ncell, s), "fill"));
    }

    Cycle cyc{c, o, s};
    cyc.finest_src = rho;
    c->ev_used = 0;
    MGFR_TRY(hip_check(c, hipMemsetAsync(c->counter, 0, sizeof(long long), s), "hipMemsetAsync"));
    auto norm = [&](double* rms) -> int {
        MGFR_TRY(hip_check(c, mgfr::residual_norm(L0.g, u, rho, c->partial, c->red, s), "residual_norm"));
        MGFR_TRY(read_reduction(c, s, r));
        *rms = std::sqrt(r[0] / (double)ncell);
        return MGFR_OK;
    };
    double rms;
    MGFR_TRY(norm(&rms));
    int k = 0;
    if (res_hist) res_hist[0] = rms;
    while (std::isfinite(rms) && rms > o->tol && k < o->max_cycles) {
        MGFR_TRY(cyc.vcycle(0));
        MGFR_TRY(norm(&rms));
        MGFR_TRY(cyc.harvest());
        ++k;
        if (res_hist) res_hist[k] = rms;
    }
    if (n_hist) *n_hist = k + 1;
    {
        long long coarse_sweeps = 0;
        MGFR_TRY(hip_check(c, hipMemcpy(&coarse_sweeps, c->counter, sizeof coarse_sweeps, hipMemcpyDeviceToHost),
                           "hipMemcpy"));
        const long long nc = mgfr::cells(c->lv.back().g);
        c->stats.cell_updates += coarse_sweeps * nc;
        if (c->lv.size() == 1) c->stats.finest_updates += coarse_sweeps * nc;
        c->stats.cycles = k;
        c->stats.solve_ms =
            std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    }
    if (!std::isfinite(rms)) return c->fail(MGFR_ENONFINITE, "residual became non-finite after %d cycles", k);
    if (rms > o->tol) return c->fail(MGFR_ENOTCONV, "rms residual %.3e > tol %.3e after %d cycles", rms, o->tol, k);
    return MGFR_OK;
}

}  // extern "C"
