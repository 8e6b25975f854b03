// Host driver of a refinement level solved with the mask scheme (Sec. V): the periodic N^3
// grid of the level's resolution, active cells where the mask is positive, the other cells
// fixed at the values the caller interpolated from the coarser level.  FAS V-cycles (Sec.
// V.B.2) over coarse levels whose masks and fixed values are 8-child means, until the rms
// residual over the active cells is <= opts->tol.
#include "host_internal.h"

using namespace mgfr_host;

namespace {

int ensure_masked(mgfr_ctx* c, int N, int coarsest)
{
    if (c->MN == N && c->Mcoarsest == coarsest) return MGFR_OK;
    (void)hipDeviceSynchronize();
    c->free_masked();
    for (int n = N; n >= coarsest; n /= 2) {
        mgfr_ctx::MLevel L;
        const size_t nc = (size_t)n * n * n;
        bool ok = hipMalloc(&L.w, sizeof(double) * nc) == hipSuccess;
        if (ok && n < N)
            ok = hipMalloc(&L.mbuf, sizeof(float) * nc) == hipSuccess && hipMalloc(&L.u, sizeof(double) * nc) == hipSuccess &&
                 hipMalloc(&L.uhat, sizeof(double) * nc) == hipSuccess &&
                 hipMalloc(&L.f, sizeof(double) * nc) == hipSuccess;
        L.mask = L.mbuf;
        c->mlv.push_back(L);
        if (!ok) {
            c->free_masked();
            return c->fail(MGFR_ENOMEM, "hipMalloc of the masked %d^3 level failed", n);
        }
    }
    mgfr::Grid gN{};
    gN.n = N;
    gN.lg = ilog2(N);
    if (hipMalloc(&c->mpart, sizeof(double) * 2 * (size_t)mgfr::masked_norm_partials(gN)) != hipSuccess ||
        hipMalloc(&c->mflags, (size_t)N * N * N) != hipSuccess ||
        (N >= mgfr::fused_sweep_min_n() && hipMalloc(&c->malt, sizeof(double) * N * N * N) != hipSuccess)) {
        c->free_masked();
        return c->fail(MGFR_ENOMEM, "hipMalloc of the norm partials, flags or sweep buffer failed");
    }
    c->MN = N;
    c->Mcoarsest = coarsest;
    return MGFR_OK;
}

struct MCycle {
    mgfr_ctx* c;
    const mgfr_opts* o;
    hipStream_t s;
    const double* rho;
    double* user_u;  // the caller's finest u (the finest level's u alternates with c->malt)

    const double* src(size_t m) const { return m == 0 ? rho : c->mlv[m].f; }

    int sweep(size_t m)
    {
        mgfr_ctx::MLevel& L = c->mlv[m];
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
        // a finest level of byte flags (n >= 64): both colours in one pass, out of place
        // between the caller's u and the context's second buffer (opts->tile = 1: per colour)
        const bool fused = m == 0 && L.flags && c->malt && o->tile != 1;
        if (fused) {
            double* out = L.u == c->malt ? user_u : c->malt;
            const int ti = o->planes > 0 && o->planes <= L.g.n ? o->planes : mgfr::fused_sweep_planes(L.g.n);
            MGFR_TRY(hip_check(c, mgfr::masked_ngs_fused(L.g, L.flags, L.w, L.u, out, src(m), ti, s),
                               "masked_ngs_fused"));
            L.u = out;
        } else if (L.flags) {
            MGFR_TRY(hip_check(c, mgfr::masked_ngs(L.g, L.flags, L.w, L.u, src(m), s), "masked_ngs"));
        } else {
            MGFR_TRY(hip_check(c, mgfr::masked_ngs(L.g, L.mask, L.w, L.u, src(m), s), "masked_ngs"));
        }
        if (timed) {
            MGFR_TRY(hip_check(c, hipEventRecord(c->ev[c->ev_used + 1], s), "hipEventRecord"));
            c->ev_used += 2;
            c->stats.sweep_launches += fused ? 1 : 2;
            // every mask read (one byte per cell with flags); per active cell u read and written
            // and the density read
            c->stats.sweep_bytes += (L.flags ? 1.0 : 4.0) * (double)mgfr::cells(L.g) + 24.0 * (double)L.active;
        }
        c->stats.cell_updates += L.active;
        if (m == 0) c->stats.finest_updates += L.active;
        return MGFR_OK;
    }

    int vcycle(size_t m)
    {
        mgfr_ctx::MLevel& L = c->mlv[m];
        if (m + 1 == c->mlv.size())
            return hip_check(c, mgfr::masked_coarsest(L.g, L.mask, L.w, L.u, src(m), o->coarsest_sweeps,
                                                      o->coarsest_rtol, c->counter, s),
                             "masked_coarsest");
        mgfr_ctx::MLevel& H = c->mlv[m + 1];
        for (int k = 0; k < o->pre; ++k) MGFR_TRY(sweep(m));
        if (L.flags)
            MGFR_TRY(hip_check(c, mgfr::masked_resid_restrict(L.g, L.flags, L.w, L.u, src(m), H.mask, H.w, H.u,
                                                              H.uhat, H.f, s),
                               "masked_resid_restrict"));
        else
            MGFR_TRY(hip_check(c, mgfr::masked_resid_restrict(L.g, L.mask, L.w, L.u, src(m), H.mask, H.w, H.u,
                                                              H.uhat, H.f, s),
                               "masked_resid_restrict"));
        MGFR_TRY(hip_check(c, mgfr::masked_fas_rhs(H.g, H.mask, H.w, H.uhat, H.f, s), "masked_fas_rhs"));
        MGFR_TRY(vcycle(m + 1));
        MGFR_TRY(hip_check(c, mgfr::masked_prolong(H.g, H.mask, H.u, H.uhat, L.mask, L.u, s), "masked_prolong"));
        for (int k = 0; k < o->post; ++k) MGFR_TRY(sweep(m));
        return MGFR_OK;
    }

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

    // rms of the residual over the finest active cells (synchronises)
    int norm(double* rms)
    {
        mgfr_ctx::MLevel& L = c->mlv[0];
        int nparts = 0;
        if (L.flags)
            MGFR_TRY(hip_check(c, mgfr::masked_norm(L.g, L.flags, L.w, L.u, rho, c->mpart, &nparts, s), "masked_norm"));
        else
            MGFR_TRY(hip_check(c, mgfr::masked_norm(L.g, L.mask, L.w, L.u, rho, c->mpart, &nparts, s), "masked_norm"));
        MGFR_TRY(hip_check(c, mgfr::fold_partials(c->mpart, nparts, c->red, s), "fold_partials"));
        double r[2];
        MGFR_TRY(read_reduction(c, s, r));
        *rms = L.active > 0 ? std::sqrt(r[0] / (double)L.active) : 0.0;
        return MGFR_OK;
    }
};

// Number of active cells and max |mask| of one level (synchronises).
int count_active(mgfr_ctx* c, const float* mask, long long n, hipStream_t s, long long* active, double* maxabs)
{
    int nparts = 0;
    MGFR_TRY(hip_check(c, mgfr::masked_count(mask, n, c->partial, &nparts, s), "masked_count"));
    MGFR_TRY(hip_check(c, mgfr::fold_partials(c->partial, nparts, c->red, s), "fold_partials"));
    double r[2];
    MGFR_TRY(read_reduction(c, s, r));
    *active = (long long)r[0];
    *maxabs = r[1];
    return MGFR_OK;
}

}  // namespace

extern "C" {

int mg_fr_solve_masked(mgfr_ctx* c, const double* rho, const float* mask, int N, const mgfr_params* params,
                       const mgfr_opts* o, double* u, double* res_hist, int* n_hist, void* stream)
{
    if (!c) return MGFR_EINVAL;
    c->err.clear();
    c->stats = mgfr_stats{};
    const auto t0 = std::chrono::steady_clock::now();
    if (n_hist) *n_hist = 0;
    MGFR_TRY(check_opts(c, o));
    if (o->precision != MGFR_FP64) return c->fail(MGFR_EINVAL, "the masked level solve runs in double precision");
    if (o->tau_alpha > 0.0) return c->fail(MGFR_EINVAL, "tau_alpha is not supported by the masked level solve");
    if (!rho || !mask || !u) return c->fail(MGFR_EINVAL, "rho, mask or u is NULL");
    if (!is_pow2(N) || N < o->coarsest_n || N > 1024)
        return c->fail(MGFR_EINVAL, "N=%d must be a power of two in [coarsest_n, 1024]", N);
    Model md;
    if (derive_model(params, &md) != MGFR_OK) return c->fail(MGFR_EINVAL, "invalid model parameters");
    MGFR_TRY(hip_check(c, hipSetDevice(c->device), "hipSetDevice"));
    hipStream_t s = (hipStream_t)stream;
    MGFR_TRY(ensure_scratch(c));
    MGFR_TRY(ensure_masked(c, N, o->coarsest_n));
    const long long ncell = (long long)N * N * N;

    // finest level: density (finite; its mean for MGFR_SUBTRACT_MEAN), mask in [-1, 1], u finite
    mgfr_ctx::MLevel& L0 = c->mlv[0];
    L0.g = make_grid(md, N, 1.0 / N, o->max_step);
    double r[2];
    MGFR_TRY(hip_check(c, mgfr::sum_and_count_nonfinite(rho, ncell, c->partial, c->red, s), "density check"));
    MGFR_TRY(read_reduction(c, s, r));
    if (r[1] != 0.0) return c->fail(MGFR_ENONFINITE, "density has %.0f non-finite cells", r[1]);
    L0.g.fscale = md.D;
    L0.g.sref = (o->flags & MGFR_SUBTRACT_MEAN) ? r[0] / (double)ncell : 1.0;
    L0.g.fshift = md.Sbar;
    MGFR_TRY(hip_check(c, mgfr::sum_and_count_nonfinite(u, ncell, c->partial, c->red, s), "field check"));
    MGFR_TRY(read_reduction(c, s, r));
    if (r[1] != 0.0) return c->fail(MGFR_ENONFINITE, "u has %.0f non-finite cells", r[1]);
    L0.mask = mask;
    L0.u = u;
    double mx;
    MGFR_TRY(count_active(c, mask, ncell, s, &L0.active, &mx));
    if (!(mx <= 1.0)) return c->fail(MGFR_EINVAL, "mask values must lie in [-1, 1] (max |mask| = %g)", mx);
    // a mask of +1 and -1 only is read as byte flags on this level (the same values)
    {
        int nparts = 0;
        MGFR_TRY(hip_check(c, mgfr::masked_flags(mask, ncell, c->mflags, c->partial, &nparts, s), "masked_flags"));
        MGFR_TRY(hip_check(c, mgfr::fold_partials(c->partial, nparts, c->red, s), "fold_partials"));
        MGFR_TRY(read_reduction(c, s, r));
        L0.flags = r[0] == 0.0 ? c->mflags : nullptr;
    }
    // fixed values: u on entry; coarse masks and fixed values by 8-child means
    MGFR_TRY(hip_check(c, hipMemcpyAsync(L0.w, u, sizeof(double) * ncell, hipMemcpyDeviceToDevice, s),
                       "hipMemcpyAsync"));
    for (size_t m = 1; m < c->mlv.size(); ++m) {
        mgfr_ctx::MLevel& H = c->mlv[m];
        const mgfr_ctx::MLevel& F = c->mlv[m - 1];
        const int n = N >> m;
        H.g = make_grid(md, n, 1.0 / n, o->max_step);
        MGFR_TRY(hip_check(c, mgfr::masked_restrict_setup(H.g, F.mask, F.w, H.mbuf, H.w, s), "masked_restrict_setup"));
        MGFR_TRY(count_active(c, H.mask, mgfr::cells(H.g), s, &H.active, &mx));
    }

    MCycle cyc{c, o, s, rho, u};
    c->ev_used = 0;
    MGFR_TRY(hip_check(c, hipMemsetAsync(c->counter, 0, sizeof(long long), s), "hipMemsetAsync"));
    double rms;
    int k = 0;
    MGFR_TRY(cyc.norm(&rms));
    if (res_hist) res_hist[0] = rms;
    while (std::isfinite(rms) && rms > o->tol && k < o->max_cycles) {
        MGFR_TRY(cyc.vcycle(0));
        MGFR_TRY(cyc.norm(&rms));
        MGFR_TRY(cyc.harvest());
        ++k;
        if (res_hist) res_hist[k] = rms;
    }
    if (n_hist) *n_hist = k + 1;
    if (L0.u != u)  // an odd number of fused sweeps left the field in the second buffer
        MGFR_TRY(hip_check(c, hipMemcpyAsync(u, L0.u, sizeof(double) * ncell, hipMemcpyDeviceToDevice, s),
                           "hipMemcpyAsync"));
    L0.u = u;
    long long coarse_sweeps = 0;
    MGFR_TRY(hip_check(c, hipMemcpy(&coarse_sweeps, c->counter, sizeof coarse_sweeps, hipMemcpyDeviceToHost),
                       "hipMemcpy"));
    c->stats.cell_updates += coarse_sweeps * c->mlv.back().active;
    if (c->mlv.size() == 1) c->stats.finest_updates += coarse_sweeps * c->mlv.back().active;
    c->stats.cycles = k;
    c->stats.solve_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    if (!std::isfinite(rms)) return c->fail(MGFR_ENONFINITE, "residual became non-finite after %d cycles", k);
    if (rms > o->tol) return c->fail(MGFR_ENOTCONV, "rms residual %.3e > tol %.3e after %d cycles", rms, o->tol, k);
    return MGFR_OK;
}

}  // extern "C"
