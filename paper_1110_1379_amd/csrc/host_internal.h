// Host-side internals shared by the drivers of libmgfr.so: model constants, the context,
// level storage and error handling.  Not installed.
#pragma once

#include <hip/hip_runtime.h>

#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <string>
#include <utility>
#include <vector>

#include "../../include/mgfr.h"
#include "mgfr_impl.h"

namespace mgfr_host {

// Derived model constants (Sec. II, Sec. III.A, Sec. VI.A.1).
struct Model {
    double xi, ct, K, A, Sbar, D, ubar, inv_np1;
};

inline int derive_model(const mgfr_params* p, Model* m)
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

inline int ilog2(int x)
{
    int l = 0;
    while ((1 << l) < x) ++l;
    return l;
}

inline bool is_pow2(int x) { return x > 0 && (x & (x - 1)) == 0; }

struct Level {
    mgfr::Grid g;
    double* u = nullptr;     // level 0: the caller's u
    double* alt = nullptr;   // second copy for out-of-place (fused) sweeps, n >= 64
    double* uhat = nullptr;  // R u of the finer level (m >= 1); turned into u^H - R u^h
    double* f = nullptr;     // FAS right-hand side (m >= 1)
};

// One level of the single-precision correction multigrid (mixed precision).
struct Level32 {
    mgfr::Grid g;
    float* ub = nullptr;    // base u (level 0: u rounded; coarse: restricted)
    float* e = nullptr;     // correction
    float* ealt = nullptr;  // second copy for the fused sweep (n >= 64)
    float* ehat = nullptr;  // R e of the finer level (m >= 1); turned into e^H - R e^h
    float* f = nullptr;     // right-hand side (level 0: r = -d)
};

}  // namespace mgfr_host

struct mgfr_ctx {
    int device = 0;
    std::string err;
    // hierarchy for one finest size, kept between calls
    int N = 0, coarsest = 0;
    std::vector<mgfr_host::Level> lv;
    int N32 = 0, coarsest32 = 0;
    std::vector<mgfr_host::Level32> lv32;
    double* partial = nullptr;  // reduction scratch
    double* red = nullptr;      // device result of a reduction (2 doubles)
    double* host_red = nullptr; // pinned copy of it
    void* pin = nullptr;        // pinned host staging of the batched solves' per-cycle copies
    size_t pin_bytes = 0;
    // modified Poisson solve: levels (finest x is the caller's phi), source and scratch
    struct PLevel {
        mgfr::PGrid g{};
        double* x = nullptr;    // coarse levels: the correction
        double* b = nullptr;    // finest: the source S; coarse: the restricted residual
        double* alt = nullptr;  // n >= 64: second buffer of the out-of-place fused sweep
    };
    int PN = 0, Pcoarsest = 0;
    std::vector<PLevel> plv;
    void free_poisson()
    {
        for (size_t m = 0; m < plv.size(); ++m) {
            if (m > 0) (void)hipFree(plv[m].x);
            (void)hipFree(plv[m].b);
            (void)hipFree(plv[m].alt);
        }
        plv.clear();
        PN = 0;
    }
    // refinement level with the mask scheme: levels (level 0 u and mask are the caller's)
    struct MLevel {
        mgfr::Grid g{};
        const float* mask = nullptr;  // level 0: the caller's; coarse: owned (mbuf)
        float* mbuf = nullptr;
        double* w = nullptr;          // fixed values (level 0: u on entry)
        double* u = nullptr;          // coarse levels
        double* uhat = nullptr;       // coarse: R u of the finer level
        double* f = nullptr;          // coarse: FAS right-hand side
        long long active = 0;         // number of active cells
        const unsigned char* flags = nullptr;  // level 0 with a +1 / -1 mask: its byte flags
    };
    int MN = 0, Mcoarsest = 0;
    std::vector<MLevel> mlv;
    double* mpart = nullptr;  // block partials of the finest-level norm
    unsigned char* mflags = nullptr;  // byte flags of the finest mask
    double* malt = nullptr;           // N >= 64: second buffer of the finest level's fused sweeps
    void free_masked()
    {
        (void)hipFree(mpart);
        mpart = nullptr;
        (void)hipFree(mflags);
        mflags = nullptr;
        (void)hipFree(malt);
        malt = nullptr;
        for (size_t m = 0; m < mlv.size(); ++m) {
            (void)hipFree(mlv[m].mbuf);
            (void)hipFree(mlv[m].w);
            if (m > 0) {
                (void)hipFree(mlv[m].u);
                (void)hipFree(mlv[m].uhat);
                (void)hipFree(mlv[m].f);
            }
        }
        mlv.clear();
        MN = 0;
    }
    // TSC assignment scratch (keys, indices, sorted positions, cell table, sort storage)
    void* tsc = nullptr;
    size_t tsc_bytes = 0;
    // device blocks of finished batched solves, reused by later ones (smallest that fits)
    std::vector<std::pair<void*, size_t>> spare;

    // the smallest kept block of at least `bytes`, or null; *size gets its full size
    void* take_spare(size_t bytes, size_t* size)
    {
        size_t best = spare.size();
        for (size_t i = 0; i < spare.size(); ++i)
            if (spare[i].second >= bytes && (best == spare.size() || spare[i].second < spare[best].second)) best = i;
        if (best == spare.size()) return nullptr;
        void* p = spare[best].first;
        *size = spare[best].second;
        spare.erase(spare.begin() + (long)best);
        return p;
    }
    void free_spare()
    {
        for (auto& b : spare) (void)hipFree(b.first);
        spare.clear();
    }
    long long* counter = nullptr;  // device: coarsest-level sweeps of the current solve
    // batched solves: a second stream (default priority) for the workgroup-per-unit kernel
    // beside the launches of the large units, and the events that fork and join it
    hipStream_t side = nullptr;
    hipEvent_t ev_fork = nullptr, ev_join = nullptr;
    // and a third (default priority) for the one-workgroup tails of the large units that end
    // at a depth while others go deeper: per depth, the events that fork and join it
    static constexpr int kTailForks = 16;
    hipStream_t tail = nullptr;
    hipEvent_t ev_tf[kTailForks] = {}, ev_tj[kTailForks] = {};
    // mg_fr_solve_noalloc: this device's address of the library's fixed scratch array (null if
    // it could not be resolved) and the host side of its reductions
    void* fixed_scratch = nullptr;
    double fixed_host[2] = {0.0, 0.0};
    // mg_fr_solve with MGFR_GRAPH: the captured cycles (graph, instance and what they were
    // captured for), the stream they were captured on, the device stop state (cycles done,
    // stopped) and residual history, and what one captured cycle adds to the counters
    hipGraph_t dgraph = nullptr;
    hipGraphExec_t dgexec = nullptr;
    std::vector<char> dkey;
    hipStream_t dcap = nullptr;
    int* gstate = nullptr;
    double* ghist = nullptr;
    int ghist_n = 0;
    long long dper_updates = 0, dper_finest = 0;
    int dper_inner = 0;
    void drop_graph()
    {
        if (dgexec) (void)hipGraphExecDestroy(dgexec);
        if (dgraph) (void)hipGraphDestroy(dgraph);
        dgexec = nullptr;
        dgraph = nullptr;
        dkey.clear();
    }
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

    // (the level buffers are in a captured graph's kernel arguments: it goes with them)
    void free_levels()
    {
        drop_graph();
        for (size_t m = 0; m < lv.size(); ++m) {
            if (m > 0) {
                (void)hipFree(lv[m].u);
                (void)hipFree(lv[m].uhat);
                (void)hipFree(lv[m].f);
            }
            (void)hipFree(lv[m].alt);
        }
        lv.clear();
        N = 0;
    }

    void free_levels32()
    {
        drop_graph();
        for (mgfr_host::Level32& L : lv32) {
            (void)hipFree(L.ub);
            (void)hipFree(L.e);
            (void)hipFree(L.ealt);
            (void)hipFree(L.ehat);
            (void)hipFree(L.f);
        }
        lv32.clear();
        N32 = 0;
    }
};

namespace mgfr_host {

inline int hip_check(mgfr_ctx* c, hipError_t e, const char* what)
{
    if (e == hipSuccess) return MGFR_OK;
    return c->fail(MGFR_EDEVICE, "%s: %s", what, hipGetErrorString(e));
}

#define MGFR_TRY(expr)                       \
    do {                                     \
        int rc_ = (expr);                    \
        if (rc_ != MGFR_OK) return rc_;      \
    } while (0)

inline int check_opts(mgfr_ctx* c, const mgfr_opts* o)
{
    if (!o) return c->fail(MGFR_EINVAL, "opts is NULL");
    if (!(o->tol >= 0.0) || o->pre < 0 || o->post < 0 || o->max_cycles < 0 || o->coarsest_sweeps < 0 ||
        !is_pow2(o->coarsest_n) || o->coarsest_n < 2 || o->coarsest_n > 8 || !(o->max_step >= 0.0) ||
        !(o->coarsest_rtol >= 0.0) || (o->precision != MGFR_FP64 && o->precision != MGFR_MIXED) ||
        o->inner_cycles < 1 || o->planes < 0 || (o->planes > 0 && (!is_pow2(o->planes) || o->planes < 4)) ||
        !(o->tau_alpha >= 0.0) || o->unit_n < 0 || o->unit_n > 1024 || o->tile < 0 || o->tile > 5)
        return c->fail(MGFR_EINVAL, "invalid options (tol=%g pre=%d post=%d coarsest_n=%d precision=%d)",
                       o->tol, o->pre, o->post, o->coarsest_n, o->precision);
    return MGFR_OK;
}

inline mgfr::Grid make_grid(const Model& md, int n, double h, double max_step)
{
    mgfr::Grid g;
    g.n = n;
    g.lg = ilog2(n);
    g.C = md.ct * md.ct / (2.0 * h * h);
    g.A = md.A;
    g.inv_np1 = md.inv_np1;
    g.half_power = md.inv_np1 == 0.5 ? 1 : 0;
    g.max_step = max_step;
    g.fscale = 1.0;
    g.sref = 0.0;
    g.fshift = 0.0;
    g.halt = nullptr;
    return g;
}

inline int ensure_scratch(mgfr_ctx* c)
{
    // each buffer on its own, so that a call after a failed one completes the set
    if (!c->partial && hipMalloc(&c->partial, sizeof(double) * mgfr::reduction_scratch()) != hipSuccess) {
        c->partial = nullptr;
        return c->fail(MGFR_ENOMEM, "hipMalloc of reduction scratch failed");
    }
    if (!c->red && hipMalloc(&c->red, sizeof(double) * 2) != hipSuccess) {
        c->red = nullptr;
        return c->fail(MGFR_ENOMEM, "hipMalloc of reduction result failed");
    }
    if (!c->host_red && hipHostMalloc(&c->host_red, sizeof(double) * 2, hipHostMallocDefault) != hipSuccess) {
        c->host_red = nullptr;
        return c->fail(MGFR_ENOMEM, "hipHostMalloc failed");
    }
    if (!c->counter && hipMalloc(&c->counter, sizeof(long long)) != hipSuccess) {
        c->counter = nullptr;
        return c->fail(MGFR_ENOMEM, "hipMalloc of the sweep counter failed");
    }
    return MGFR_OK;
}

// The side stream and its fork/join events (created once per context).
inline int ensure_side(mgfr_ctx* c)
{
    if (!c->side && hipStreamCreateWithFlags(&c->side, hipStreamNonBlocking) != hipSuccess) {
        c->side = nullptr;
        return c->fail(MGFR_EDEVICE, "hipStreamCreate failed");
    }
    if (!c->ev_fork && hipEventCreateWithFlags(&c->ev_fork, hipEventDisableTiming) != hipSuccess) {
        c->ev_fork = nullptr;
        return c->fail(MGFR_EDEVICE, "hipEventCreate failed");
    }
    if (!c->ev_join && hipEventCreateWithFlags(&c->ev_join, hipEventDisableTiming) != hipSuccess) {
        c->ev_join = nullptr;
        return c->fail(MGFR_EDEVICE, "hipEventCreate failed");
    }
    return MGFR_OK;
}

// The tail stream and its per-depth fork/join events (created once per context).
inline int ensure_tail(mgfr_ctx* c)
{
    if (!c->tail && hipStreamCreateWithFlags(&c->tail, hipStreamNonBlocking) != hipSuccess) {
        c->tail = nullptr;
        return c->fail(MGFR_EDEVICE, "hipStreamCreate failed");
    }
    for (int d = 0; d < mgfr_ctx::kTailForks; ++d) {
        if (!c->ev_tf[d] && hipEventCreateWithFlags(&c->ev_tf[d], hipEventDisableTiming) != hipSuccess) {
            c->ev_tf[d] = nullptr;
            return c->fail(MGFR_EDEVICE, "hipEventCreate failed");
        }
        if (!c->ev_tj[d] && hipEventCreateWithFlags(&c->ev_tj[d], hipEventDisableTiming) != hipSuccess) {
            c->ev_tj[d] = nullptr;
            return c->fail(MGFR_EDEVICE, "hipEventCreate failed");
        }
    }
    return MGFR_OK;
}

// Pinned host buffer of at least `bytes` (kept in the context; contents not preserved).
inline int ensure_pinned(mgfr_ctx* c, size_t bytes)
{
    if (c->pin_bytes >= bytes) return MGFR_OK;
    if (c->pin) {
        (void)hipDeviceSynchronize();
        (void)hipHostFree(c->pin);
        c->pin = nullptr;
        c->pin_bytes = 0;
    }
    if (hipHostMalloc(&c->pin, bytes, hipHostMallocDefault) != hipSuccess)
        return c->fail(MGFR_ENOMEM, "hipHostMalloc of %zu bytes failed", bytes);
    c->pin_bytes = bytes;
    return MGFR_OK;
}

// Allocates levels N/2 ... coarsest (level 0 uses the caller's arrays).
inline int ensure_levels(mgfr_ctx* c, int N, int coarsest)
{
    if (c->N == N && c->coarsest == coarsest) return MGFR_OK;
    c->free_levels();
    for (int n = N; n >= coarsest; n /= 2) {
        Level L;
        const size_t bytes = sizeof(double) * (size_t)n * n * n;
        bool ok = true;
        if (n < N)
            ok = hipMalloc(&L.u, bytes) == hipSuccess && hipMalloc(&L.uhat, bytes) == hipSuccess &&
                 hipMalloc(&L.f, bytes) == hipSuccess;
        if (ok && n >= mgfr::fused_sweep_min_n()) ok = hipMalloc(&L.alt, bytes) == hipSuccess;
        if (!ok) {
            if (n < N) {
                (void)hipFree(L.u);
                (void)hipFree(L.uhat);
                (void)hipFree(L.f);
            }
            (void)hipFree(L.alt);
            c->free_levels();
            return c->fail(MGFR_ENOMEM, "hipMalloc of the %d^3 level failed", n);
        }
        c->lv.push_back(L);
    }
    c->N = N;
    c->coarsest = coarsest;
    return MGFR_OK;
}

// Single-precision hierarchy N ... coarsest for the mixed solver.
inline int ensure_levels32(mgfr_ctx* c, int N, int coarsest)
{
    if (c->N32 == N && c->coarsest32 == coarsest) return MGFR_OK;
    c->free_levels32();
    for (int n = N; n >= coarsest; n /= 2) {
        Level32 L;
        const size_t bytes = sizeof(float) * (size_t)n * n * n;
        bool ok = hipMalloc(&L.ub, bytes) == hipSuccess && hipMalloc(&L.e, bytes) == hipSuccess &&
                  hipMalloc(&L.f, bytes) == hipSuccess;
        if (ok && n < N) ok = hipMalloc(&L.ehat, bytes) == hipSuccess;
        if (ok && n >= mgfr::fused_sweep_min_n()) ok = hipMalloc(&L.ealt, bytes) == hipSuccess;
        c->lv32.push_back(L);
        if (!ok) {
            c->free_levels32();
            return c->fail(MGFR_ENOMEM, "hipMalloc of the single-precision %d^3 level failed", n);
        }
    }
    c->N32 = N;
    c->coarsest32 = coarsest;
    return MGFR_OK;
}

// Copies a 2-double device reduction result to the host (synchronises the stream).
inline int read_reduction(mgfr_ctx* c, hipStream_t s, double* out2)
{
    MGFR_TRY(hip_check(c, hipMemcpyAsync(c->host_red, c->red, 2 * sizeof(double), hipMemcpyDeviceToHost, s),
                       "hipMemcpyAsync"));
    MGFR_TRY(hip_check(c, hipStreamSynchronize(s), "hipStreamSynchronize"));
    out2[0] = c->host_red[0];
    out2[1] = c->host_red[1];
    return MGFR_OK;
}

}  // namespace mgfr_host
