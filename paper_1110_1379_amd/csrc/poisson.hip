// Host driver of the modified Poisson solve (eq. discrete_poisson; Sec. V.A.3 for the linear
// multigrid): the source from the density and the scalaron u, its mean removed, linear
// V-cycles until the residual has fallen by opts->tol relative to the source, and the
// potential shifted to zero mean.
#include <algorithm>

#include "host_internal.h"

using namespace mgfr_host;

namespace {

mgfr::PGrid pgrid(int n)
{
    mgfr::PGrid g;
    g.n = n;
    g.lg = ilog2(n);
    g.hh = 1.0 / ((double)n * (double)n);
    g.inv_hh = (double)n * (double)n;
    return g;
}

mgfr::Grid coarse_grid(const mgfr::PGrid& p)
{
    mgfr::Grid g{};
    g.n = p.n;
    g.lg = p.lg;
    return g;
}

int ensure_poisson(mgfr_ctx* c, int N, int coarsest)
{
    if (c->PN == N && c->Pcoarsest == coarsest) return MGFR_OK;
    (void)hipDeviceSynchronize();
    c->free_poisson();
    const int fused = mgfr::poisson_fused_min_n();
    for (int n = N; n >= coarsest; n /= 2) {
        mgfr_ctx::PLevel L;
        L.g = pgrid(n);
        const size_t bytes = sizeof(double) * (size_t)n * n * n;
        bool ok = hipMalloc(&L.b, bytes) == hipSuccess;
        if (ok && n < N) ok = hipMalloc(&L.x, bytes) == hipSuccess;
        if (ok && n >= fused) ok = hipMalloc(&L.alt, bytes) == hipSuccess;
        c->plv.push_back(L);
        if (!ok) {
            c->free_poisson();
            return c->fail(MGFR_ENOMEM, "hipMalloc of Poisson level n=%d failed", n);
        }
    }
    c->PN = N;
    c->Pcoarsest = coarsest;
    return MGFR_OK;
}

struct PCycle {
    mgfr_ctx* c;
    const mgfr_opts* o;
    hipStream_t s;
    double mean0;  // mean of the finest source

    // `count` sweeps: one launch, or on levels with the fused kernels as many two-sweep
    // passes as fit and one single sweep for an odd remainder
    int sweeps(size_t m, double*& cur, double bm, int count)
    {
        int k = 0;
        if (c->plv[m].alt)
            for (; k + 2 <= count; k += 2) MGFR_TRY(sweep(m, cur, bm, 2));
        for (; k < count; ++k) MGFR_TRY(sweep(m, cur, bm, 1));
        return MGFR_OK;
    }

    int sweep(size_t m, double*& cur, double bm, int passes)
    {
        mgfr_ctx::PLevel& L = c->plv[m];
        // MGFR_PROFILE: HIP events around every finest-level sweep, on the solve's stream
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
        if (L.alt) {
            double* out = cur == L.alt ? (m == 0 ? finest_x : L.x) : L.alt;
            const bool opt = m == 0 && o->planes > 0 && o->planes <= L.g.n;
            if (passes == 2) {
                const int ti = opt ? o->planes : mgfr::poisson_fused2_planes(L.g.n);
                MGFR_TRY(hip_check(c, mgfr::poisson_ngs_fused2(L.g, cur, out, L.b, bm, ti, s), "poisson_ngs_fused2"));
            } else {
                const int ti = opt ? o->planes : mgfr::fused_sweep_planes(L.g.n);
                MGFR_TRY(hip_check(c, mgfr::poisson_ngs_fused(L.g, cur, out, L.b, bm, ti, s), "poisson_ngs_fused"));
            }
            cur = out;
        } else {
            MGFR_TRY(hip_check(c, mgfr::poisson_ngs(L.g, cur, L.b, bm, s), "poisson_ngs"));
        }
        if (timed) {
            MGFR_TRY(hip_check(c, hipEventRecord(c->ev[c->ev_used + 1], s), "hipEventRecord"));
            c->ev_used += 2;
            c->stats.sweep_launches += L.alt ? 1 : 2;
            // read x, b; write x: once per launch, also for a two-sweep pass
            c->stats.sweep_bytes += 24.0 * (double)(1LL << (3 * L.g.lg));
        }
        c->stats.cell_updates += passes * (1LL << (3 * L.g.lg));
        if (m == 0) c->stats.finest_updates += passes * (1LL << (3 * L.g.lg));
        return MGFR_OK;
    }

    double* finest_x = nullptr;

    int vcycle(size_t m)
    {
        mgfr_ctx::PLevel& L = c->plv[m];
        double* x = m == 0 ? finest_x : L.x;
        const double bm = m == 0 ? mean0 : 0.0;
        if (m + 1 == c->plv.size())
            return hip_check(c, mgfr::poisson_coarsest(L.g, x, L.b, bm, o->coarsest_sweeps, o->coarsest_rtol, s),
                             "poisson_coarsest");
        mgfr_ctx::PLevel& H = c->plv[m + 1];
        double* cur = x;
        MGFR_TRY(sweeps(m, cur, bm, o->pre));
        MGFR_TRY(hip_check(c, mgfr::poisson_resid_restrict(L.g, cur, L.b, bm, H.b, s), "poisson_resid_restrict"));
        MGFR_TRY(hip_check(c, mgfr::fill(H.x, 0.0, 1LL << (3 * H.g.lg), s), "fill"));
        MGFR_TRY(vcycle(m + 1));
        MGFR_TRY(hip_check(c, mgfr::prolong_add_direct(coarse_grid(H.g), cur, H.x, s), "prolong_add_direct"));
        MGFR_TRY(sweeps(m, cur, bm, o->post));
        if (cur != x)
            MGFR_TRY(hip_check(c, hipMemcpyAsync(x, cur, sizeof(double) * ((size_t)1 << (3 * L.g.lg)),
                                                 hipMemcpyDeviceToDevice, s),
                               "hipMemcpyAsync"));
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

    // rms and max of b - bmean - lap x on the finest level (x null: of b - bmean); synchronises
    int norm(const double* x, double* rms, double* mx)
    {
        mgfr_ctx::PLevel& L = c->plv[0];
        const long long n3 = 1LL << (3 * L.g.lg);
        int nparts = 0;
        MGFR_TRY(hip_check(c, mgfr::poisson_resid_norm(L.g, x, L.b, mean0, c->partial, &nparts, s),
                           "poisson_resid_norm"));
        MGFR_TRY(hip_check(c, mgfr::fold_partials(c->partial, nparts, c->red, s), "fold_partials"));
        double out[2];
        MGFR_TRY(read_reduction(c, s, out));
        *rms = std::sqrt(out[0] / (double)n3);
        *mx = out[1];
        return MGFR_OK;
    }
};

}  // namespace

extern "C" {

int mg_poisson_solve(mgfr_ctx* c, const double* rho, const double* u, int N, const mgfr_params* params,
                     const mgfr_opts* o, double* phi, double* res_hist, int* n_hist, void* stream)
{
    if (!c) return MGFR_EINVAL;
    c->err.clear();
    c->stats = mgfr_stats{};
    const auto t0 = std::chrono::steady_clock::now();
    MGFR_TRY(check_opts(c, o));
    if (o->precision != MGFR_FP64) return c->fail(MGFR_EINVAL, "the Poisson solve runs in double precision");
    if (!rho || !u || !phi) return c->fail(MGFR_EINVAL, "null rho, u or phi");
    if (!is_pow2(N) || N < 2 * o->coarsest_n || N > 1024)
        return c->fail(MGFR_EINVAL, "N=%d must be a power of two in [2 coarsest_n, 1024]", N);
    Model md;
    if (derive_model(params, &md) != MGFR_OK) return c->fail(MGFR_EINVAL, "invalid model parameters");
    MGFR_TRY(hip_check(c, hipSetDevice(c->device), "hipSetDevice"));
    hipStream_t s = (hipStream_t)stream;
    MGFR_TRY(ensure_scratch(c));
    MGFR_TRY(ensure_poisson(c, N, o->coarsest_n));
    c->ev_used = 0;
    const long long n3 = (long long)N * N * N;
    mgfr_ctx::PLevel& L0 = c->plv[0];

    // source and its mean
    mgfr::PoissonSource src{md.D, md.A, md.inv_np1, md.Sbar};
    MGFR_TRY(hip_check(c, mgfr::poisson_source(src, n3, rho, u, L0.b, c->partial, s), "poisson_source"));
    MGFR_TRY(hip_check(c, mgfr::fold_partials(c->partial, mgfr::poisson_partials(n3), c->red, s), "fold_partials"));
    double sm[2];
    MGFR_TRY(read_reduction(c, s, sm));
    if (!std::isfinite(sm[0]) || !std::isfinite(sm[1]))
        return c->fail(MGFR_ENONFINITE, "the source is not finite (non-finite rho or u)");
    PCycle cyc{c, o, s, sm[0] / (double)n3};
    cyc.finest_x = phi;
    if (!(o->flags & MGFR_WARM_START)) MGFR_TRY(hip_check(c, mgfr::fill(phi, 0.0, n3, s), "fill"));

    double ref, mx;
    MGFR_TRY(cyc.norm(nullptr, &ref, &mx));  // rms of the source about its mean
    const double target = o->tol * ref;
    int k = 0, status = MGFR_OK;
    double rms;
    MGFR_TRY(cyc.norm(phi, &rms, &mx));
    if (res_hist) res_hist[0] = rms;
    while (rms > target) {
        if (!std::isfinite(rms)) {
            status = MGFR_ENONFINITE;
            break;
        }
        if (k >= o->max_cycles) {
            status = MGFR_ENOTCONV;
            break;
        }
        MGFR_TRY(cyc.vcycle(0));
        MGFR_TRY(cyc.harvest());
        ++k;
        MGFR_TRY(cyc.norm(phi, &rms, &mx));
        if (res_hist) res_hist[k] = rms;
    }
    if (n_hist) *n_hist = k + 1;
    c->stats.cycles = k;
    // zero-mean potential
    double ps[2];
    MGFR_TRY(hip_check(c, mgfr::sum_and_count_nonfinite(phi, n3, c->partial, c->red, s), "sum_and_count_nonfinite"));
    MGFR_TRY(read_reduction(c, s, ps));
    MGFR_TRY(hip_check(c, mgfr::poisson_add(phi, -ps[0] / (double)n3, n3, s), "poisson_add"));
    MGFR_TRY(hip_check(c, hipStreamSynchronize(s), "hipStreamSynchronize"));
    c->stats.solve_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    if (status == MGFR_ENONFINITE) return c->fail(status, "the Poisson residual became non-finite");
    if (status == MGFR_ENOTCONV) return c->fail(status, "rms residual %.3e above tol x source rms after %d cycles", rms, k);
    return MGFR_OK;
}

int mg_poisson_smooth(mgfr_ctx* c, const double* rho, const double* u, int N, const mgfr_params* params,
                      int nsweeps, int variant, double* phi, void* stream)
{
    if (!c) return MGFR_EINVAL;
    c->err.clear();
    if (!rho || !u || !phi) return c->fail(MGFR_EINVAL, "null rho, u or phi");
    if (!is_pow2(N) || N < 4 || N > 1024) return c->fail(MGFR_EINVAL, "N=%d must be a power of two in [4, 1024]", N);
    if (nsweeps < 0 || variant < 0 || variant > 2 || (variant == 2 && (nsweeps & 1)))
        return c->fail(MGFR_EINVAL, "invalid sweep count or variant");
    if (variant > 0 && N < mgfr::poisson_fused_min_n())
        return c->fail(MGFR_EINVAL, "the fused sweeps need N >= %d", mgfr::poisson_fused_min_n());
    Model md;
    if (derive_model(params, &md) != MGFR_OK) return c->fail(MGFR_EINVAL, "invalid model parameters");
    MGFR_TRY(hip_check(c, hipSetDevice(c->device), "hipSetDevice"));
    hipStream_t s = (hipStream_t)stream;
    MGFR_TRY(ensure_scratch(c));
    MGFR_TRY(ensure_poisson(c, N, N));  // the finest level alone: its source and second buffer
    const long long n3 = (long long)N * N * N;
    mgfr_ctx::PLevel& L0 = c->plv[0];
    mgfr::PoissonSource src{md.D, md.A, md.inv_np1, md.Sbar};
    MGFR_TRY(hip_check(c, mgfr::poisson_source(src, n3, rho, u, L0.b, c->partial, s), "poisson_source"));
    MGFR_TRY(hip_check(c, mgfr::fold_partials(c->partial, mgfr::poisson_partials(n3), c->red, s), "fold_partials"));
    double sm[2];
    MGFR_TRY(read_reduction(c, s, sm));
    if (!std::isfinite(sm[0]) || !std::isfinite(sm[1]))
        return c->fail(MGFR_ENONFINITE, "the source is not finite (non-finite rho or u)");
    const double mean = sm[0] / (double)n3;
    double* cur = phi;
    for (int k = 0; k < nsweeps; k += variant == 2 ? 2 : 1) {
        double* out = cur == phi ? L0.alt : phi;
        if (variant == 0)
            MGFR_TRY(hip_check(c, mgfr::poisson_ngs(L0.g, cur, L0.b, mean, s), "poisson_ngs"));
        else if (variant == 1)
            MGFR_TRY(hip_check(c, mgfr::poisson_ngs_fused(L0.g, cur, out, L0.b, mean, mgfr::fused_sweep_planes(N), s),
                               "poisson_ngs_fused"));
        else
            MGFR_TRY(hip_check(c, mgfr::poisson_ngs_fused2(L0.g, cur, out, L0.b, mean, mgfr::poisson_fused2_planes(N), s),
                               "poisson_ngs_fused2"));
        if (variant > 0) cur = out;
    }
    if (cur != phi)
        MGFR_TRY(hip_check(c, hipMemcpyAsync(phi, cur, sizeof(double) * (size_t)n3, hipMemcpyDeviceToDevice, s),
                           "hipMemcpyAsync"));
    return hip_check(c, hipStreamSynchronize(s), "hipStreamSynchronize");
}

}  // extern "C"
