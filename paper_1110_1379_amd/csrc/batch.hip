// Host driver of the batched solves: refinement patches level by level (Sec. V, Sec. VI.B)
// and many independent periodic boxes.  Every unit of a batch runs the same FAS V-cycle
// (Sec. V.B.2) with its own size, constants and hierarchy.
//
// Default engine (workgroup per unit, unit.hip): units of side <= opts.unit_n are solved
// whole, every cycle and stop test, by one workgroup each, in one persistent launch that
// takes them from a device queue (largest first).  Larger units run their fine levels as one
// launch per phase over all of them, through a table of (unit grid, block) pairs, and the
// rest of each V-cycle (levels of side <= unit_n) in one workgroup per unit; their stop tests
// run on the device, and the host reads one word per chunk of cycles.  The two kinds run
// concurrently on two streams.
//
// MGFR_PER_PHASE selects the earlier engine, kept as the baseline: every phase of every level
// is one launch over all units, and after every cycle the per-unit residual norms come back
// to the host, which switches converged units off for the remaining cycles.
#include <algorithm>
#include <cstring>

#include "host_internal.h"

using namespace mgfr_host;

namespace {

constexpr int kMinTiles = 256;  // automatic sweep form: column tiles from this many per depth
constexpr int kQueues = 12;  // whole-unit launches per batch, at most one per unit side (2 ... 1024)

struct Unit {
    int n = 0, nlev = 0;
    bool periodic = false;
    Model md{};
    double h = 0.0;              // finest spacing
    double* u = nullptr;         // caller's solution (finest)
    const double* rho = nullptr; // caller's density (finest)
    std::vector<mgfr::BGrid> g;  // descriptor of each multigrid level
};

// Host image of everything the kernels of one batch read from device memory: descriptor
// arrays and workgroup tables, concatenated into one buffer.
struct Meta {
    std::vector<char> bytes;
    template <class T>
    size_t add(const std::vector<T>& v)
    {
        size_t off = (bytes.size() + 255) & ~size_t(255);
        bytes.resize(off + v.size() * sizeof(T));
        if (!v.empty()) std::memcpy(bytes.data() + off, v.data(), v.size() * sizeof(T));
        return off;
    }
};

struct Launch {
    size_t grids = 0, blk = 0, other = 0;  // offsets into the device meta buffer
    int nblk = 0, ngrid = 0;
};

// Red-black sweep of one depth: the grids swept one thread per cell of the colour, those swept
// by column tiles (side >= 32), and the periodic boxes of a mixed solve swept in fused pairs
// (column tiles, e32b set).
struct Sweep {
    Launch cell, col;
    Launch pair[2], pair1[2];  // [periodic] fused pairs; pair1: their grids as column tiles (an odd sweep)
    std::vector<const double*> box_pairs;  // u of the periodic grids swept in fused pairs
};

// The finest grids whose correction a separate u += e must add: all of them, unless the
// last post-smoothing sweep adds it (an even number of post sweeps >= 2 of a mixed solve;
// then all but the boxes that depth 0 sweeps in fused pairs).
std::vector<mgfr::BGrid> add_rest(const std::vector<mgfr::BGrid>& g0, const Sweep* S0, bool fuse)
{
    std::vector<mgfr::BGrid> rest;
    for (const mgfr::BGrid& g : g0)
        if (!fuse || !S0 || std::find(S0->box_pairs.begin(), S0->box_pairs.end(), g.u) == S0->box_pairs.end())
            rest.push_back(g);
    return rest;
}

// Residual and restriction of one depth: column tiles over the fine grids that take them,
// one thread per coarse cell for the rest; each with its coarse grids (other, same order).
struct RR {
    Launch tile, cell;
};

struct Depth {
    Sweep half;
    RR rr;
    Launch coarse_f, coarse_c, faces_c, crs;
    bool deep = false, coarsest = false;
};

// The finest residual of a list of units: column tiles for the grids that take them (side
// >= 32), one thread per cell for the others; the (sum, max) partials of the tiles first,
// then those of the cell blocks, and each unit's range of them for the fold.
struct NormPlan {
    Launch tile, cell;
    size_t first = 0, count = 0;
    int ngrid = 0;
    long long nparts = 0;
};

struct Plan {
    std::vector<Depth> depth;
    Launch cells0, setup;
    Launch add0;                  // finest grids of the separate u += e (add_rest)
    bool fuse_add = false;        // the last post sweep of a correction solve adds it for the others
    size_t first = 0, count = 0;  // per-unit block ranges of cells0 (for the non-finite fold)
    NormPlan norm;
    int nunit = 0;
    long long nblk_cells0 = 0;
};

// Launch-based depth of the large units (workgroup-per-unit engine): their grids at depth m
// whose level m is larger than unit_n, and the units whose V-cycle continues in one
// workgroup from level m + 1 (tails: (index of that level in the all-levels array, levels
// from there)).
struct UDepth {
    Sweep half;
    RR rr;
    Launch coarse_f, coarse_c;
    size_t tails = 0;
    int ntail = 0;
    bool deep = false;
};

struct UPlan {
    std::vector<UDepth> depth;
    size_t grids = 0, first = 0, nlev = 0, order = 0;  // all levels of all units; whole units in queue order
    int nwhole = 0, nlarge = 0;
    std::vector<int3> ranges;          // whole units: (begin, end, side) in queue order, one launch each
    size_t ids = 0, ncell = 0;        // large units: unit index, finest cells
    Launch cells0;                     // finest cells of the large units
    Launch add0;                       // of those, the grids of the separate u += e (add_rest)
    NormPlan norm;                     // their residual
    size_t all_tails = 0;              // every large unit's tail (for the tail bases)
    int nall_tails = 0;
};

// Blocks of `work(g)` items for each grid; grids listed in order, so each grid's blocks are
// contiguous.
template <class W>
Launch table(Meta& meta, const std::vector<mgfr::BGrid>& grids, W work, std::vector<int>* first = nullptr,
             std::vector<int>* count = nullptr)
{
    const int B = mgfr::batch_block();
    std::vector<int2> blk;
    for (size_t i = 0; i < grids.size(); ++i) {
        const long long w = work(grids[i]);
        const int nb = (int)((w + B - 1) / B);
        if (first) first->push_back((int)blk.size());
        if (count) count->push_back(nb);
        for (int b = 0; b < nb; ++b) blk.push_back(make_int2((int)i, b));
    }
    Launch L;
    L.grids = meta.add(grids);
    L.blk = meta.add(blk);
    L.nblk = (int)blk.size();
    L.ngrid = (int)grids.size();
    return L;
}

long long cells3(const mgfr::BGrid& g) { return 1LL << (3 * g.lg); }

RR rr_tables(Meta& meta, const std::vector<mgfr::BGrid>& f, const std::vector<mgfr::BGrid>& cg)
{
    std::vector<mgfr::BGrid> tf, tc, cf, cc;
    std::vector<int2> tb;
    for (size_t i = 0; i < f.size(); ++i) {
        const long long nt = mgfr::batch_col_tiles(f[i].n);
        if (nt > 0) {
            for (long long b = 0; b < nt; ++b) tb.push_back(make_int2((int)tf.size(), (int)b));
            tf.push_back(f[i]);
            tc.push_back(cg[i]);
        } else {
            cf.push_back(f[i]);
            cc.push_back(cg[i]);
        }
    }
    RR R;
    R.tile.grids = meta.add(tf);
    R.tile.blk = meta.add(tb);
    R.tile.nblk = (int)tb.size();
    R.tile.ngrid = (int)tf.size();
    R.tile.other = meta.add(tc);
    R.cell = table(meta, cf, [](const mgfr::BGrid& g) { return cells3(g) / 8; });
    R.cell.other = meta.add(cc);
    return R;
}

NormPlan norm_tables(Meta& meta, const std::vector<mgfr::BGrid>& g0)
{
    std::vector<mgfr::BGrid> tg, cg;
    std::vector<int2> tb, cb;
    std::vector<int> first(g0.size()), count(g0.size());
    const int B = mgfr::batch_block();
    for (size_t u = 0; u < g0.size(); ++u) {
        const long long nt = mgfr::batch_col_tiles(g0[u].n);
        if (nt > 0) {
            first[u] = (int)tb.size();
            count[u] = (int)nt;
            for (long long b = 0; b < nt; ++b) tb.push_back(make_int2((int)tg.size(), (int)b));
            tg.push_back(g0[u]);
        }
    }
    for (size_t u = 0; u < g0.size(); ++u) {
        if (mgfr::batch_col_tiles(g0[u].n) > 0) continue;
        const long long nb = (cells3(g0[u]) + B - 1) / B;
        first[u] = (int)(tb.size() + cb.size());
        count[u] = (int)nb;
        for (long long b = 0; b < nb; ++b) cb.push_back(make_int2((int)cg.size(), (int)b));
        cg.push_back(g0[u]);
    }
    NormPlan N;
    N.tile.grids = meta.add(tg);
    N.tile.blk = meta.add(tb);
    N.tile.nblk = (int)tb.size();
    N.tile.ngrid = (int)tg.size();
    N.cell.grids = meta.add(cg);
    N.cell.blk = meta.add(cb);
    N.cell.nblk = (int)cb.size();
    N.cell.ngrid = (int)cg.size();
    N.first = meta.add(first);
    N.count = meta.add(count);
    N.ngrid = (int)g0.size();
    N.nparts = (long long)tb.size() + (long long)cb.size();
    return N;
}

// Sweep tables of the grids f: fused pairs for the grids with a second correction buffer;
// column tiles for the others that take them (side >= 32; tile = 2: all, 1: none, otherwise
// periodic boxes); one thread per cell of the colour for the rest.
Sweep sweep_tables(Meta& meta, const std::vector<mgfr::BGrid>& f, int tile)
{
    std::vector<mgfr::BGrid> cell, col, pair[2];
    std::vector<int2> bcol, bpair[2], bpair1[2];
    std::vector<const double*> box_u;
    // Automatic choice: tiles only for a depth that has at least one per compute unit.  A
    // tile's walk is a chain of barrier-separated plane steps; with fewer tiles than CUs the
    // one-thread-per-cell launches finish sooner (16 boxes of 32^3: 64 tiles take 22 us per
    // fused sweep, the two per-cell colour launches 12 us).
    bool few = false;
    if (tile != 1 && tile != 2 && tile != 3) {
        long long total = 0;
        for (const mgfr::BGrid& g : f)
            if (g.periodic || g.e32b) total += mgfr::batch_col_tiles(g.n);
        few = total < kMinTiles;
    }
    for (const mgfr::BGrid& g : f) {
        const long long nt = mgfr::batch_col_tiles(g.n), np = mgfr::batch_pair_tiles(g.n, g.periodic);
        if (few) {
            cell.push_back(g);
            continue;
        }
        if (g.e32b && nt > 0 && np > 0) {
            const int w = g.periodic ? 1 : 0;
            for (long long b = 0; b < np; ++b) bpair[w].push_back(make_int2((int)pair[w].size(), (int)b));
            for (long long b = 0; b < nt; ++b) bpair1[w].push_back(make_int2((int)pair[w].size(), (int)b));
            pair[w].push_back(g);
            if (g.periodic) box_u.push_back(g.u);
            continue;
        }
        const bool want = tile == 2 || (tile != 1 && g.periodic);
        if (!want || nt == 0) {
            cell.push_back(g);
            continue;
        }
        for (long long b = 0; b < nt; ++b) bcol.push_back(make_int2((int)col.size(), (int)b));
        col.push_back(g);
    }
    Sweep S;
    S.cell = table(meta, cell, [](const mgfr::BGrid& g) { return cells3(g) / 2; });
    auto tiles = [&](Launch& L, const std::vector<mgfr::BGrid>& gs, const std::vector<int2>& blk) {
        L.grids = meta.add(gs);
        L.blk = meta.add(blk);
        L.nblk = (int)blk.size();
        L.ngrid = (int)gs.size();
    };
    tiles(S.col, col, bcol);
    for (int w = 0; w < 2; ++w) {
        tiles(S.pair[w], pair[w], bpair[w]);
        tiles(S.pair1[w], pair[w], bpair1[w]);
    }
    S.box_pairs = std::move(box_u);
    return S;
}

struct Batch {
    mgfr_ctx* c;
    const mgfr_opts* o;
    hipStream_t s;
    std::vector<Unit>& units;
    bool phases = false;  // MGFR_PER_PHASE: the per-phase engine with host stop tests
    int W = 16;           // workgroup-per-unit engine: units and levels of side <= W in one workgroup
    Plan plan;
    UPlan up;
    char* dmeta = nullptr;
    int* dactive = nullptr;
    std::vector<int> active;
    double* dpartial = nullptr;
    double* dout = nullptr;
    double* dhist = nullptr;  // workgroup-per-unit engine: per-unit histories on the device
    int* dints = nullptr;     // ... per-unit cycles and status, the active count and the queue
    double* hout = nullptr;  // pinned: per-unit (sum d^2, max |d|) read back every cycle
    int* hact = nullptr;     // pinned: per-unit active flags uploaded every cycle
    std::vector<std::pair<void*, size_t>> owned;

    // Device blocks go back to the context for the next batched solve once this one's work
    // has finished.
    ~Batch()
    {
        (void)hipStreamSynchronize(s);
        if (gexec) (void)hipGraphExecDestroy(gexec);
        if (graph) (void)hipGraphDestroy(graph);
        if (cap_stream) (void)hipStreamDestroy(cap_stream);
        for (auto& b : owned) c->spare.push_back(b);
    }

    template <class T>
    int alloc(T** p, size_t count)
    {
        if (count == 0) count = 1;
        const size_t bytes = count * sizeof(T);
        size_t size = bytes;  // a reused block keeps its full size for later reuse
        void* q = c->take_spare(bytes, &size);
        if (!q && hipMalloc(&q, bytes) != hipSuccess) {
            (void)hipGetLastError();
            c->free_spare();  // give cached blocks back and try once more
            if (hipMalloc(&q, bytes) != hipSuccess)
                return c->fail(MGFR_ENOMEM, "hipMalloc of %zu bytes for a batch failed", bytes);
        }
        *p = (T*)q;
        owned.emplace_back(q, size);
        return MGFR_OK;
    }

    mgfr::BTable tab(const Launch& L) const
    {
        mgfr::BTable t;
        t.grids = (const mgfr::BGrid*)(dmeta + L.grids);
        t.blk = (const int2*)(dmeta + L.blk);
        t.active = dactive;
        return t;
    }
    const mgfr::BGrid* grids(const Launch& L) const { return (const mgfr::BGrid*)(dmeta + L.grids); }

    // A level of side n swept in fused pairs: a level of a mixed solve, side >= 32, swept by
    // launches (not inside a one-workgroup solve); periodic boxes by default (tile 0, 4, 5),
    // patches too with tile 3.  (On patches of the sizes of a refinement level the fused pairs
    // gain nothing over one thread per cell: their launches are few workgroups deep.)
    bool pair_level(const Unit& U, int n) const
    {
        const bool want = o->tile == 3 || (o->tile != 1 && o->tile != 2 && U.periodic);
        return o->precision == MGFR_MIXED && want && mgfr::batch_col_tiles(n) > 0 &&
               mgfr::batch_pair_tiles(n, U.periodic) > 0 && (phases || n > W);
    }

    // Allocates each unit's coarse levels (and patch boundary faces), fills the descriptors
    // and uploads the plan.
    int prepare()
    {
        const int cn = o->coarsest_n;
        // storage
        size_t need = 0;
        for (Unit& U : units) {
            U.nlev = 0;
            for (int n = U.n; n >= cn; n /= 2) ++U.nlev;
            for (int m = 0; m < U.nlev; ++m) {
                const size_t n = (size_t)(U.n >> m);
                if (m > 0) need += 3 * n * n * n;
                if (!U.periodic) need += 6 * n * n;
            }
        }
        double* pool = nullptr;
        MGFR_TRY(alloc(&pool, need));
        size_t at = 0;
        // mixed precision: single-precision base, correction, right-hand side (every level),
        // coarse difference (coarse levels) and the second correction buffer of fused pairs
        const bool mixed = o->precision == MGFR_MIXED;
        float* pool32 = nullptr;
        size_t at32 = 0;
        if (mixed) {
            size_t need32 = 0;
            for (Unit& U : units)
                for (int m = 0; m < U.nlev; ++m) {
                    const size_t n = (size_t)(U.n >> m);
                    need32 += (m > 0 ? 4 : 3) * n * n * n + (pair_level(U, (int)n) ? n * n * n : 0);
                }
            MGFR_TRY(alloc(&pool32, need32));
        }
        for (size_t ui = 0; ui < units.size(); ++ui) {
            Unit& U = units[ui];
            U.g.assign(U.nlev, mgfr::BGrid{});
            for (int m = 0; m < U.nlev; ++m) {
                mgfr::BGrid& G = U.g[m];
                const int n = U.n >> m;
                const double hm = U.h * (double)(1 << m);
                G.n = n;
                G.lg = ilog2(n);
                G.periodic = U.periodic ? 1 : 0;
                G.unit = (int)ui;
                G.C = U.md.ct * U.md.ct / (2.0 * hm * hm);
                G.A = U.md.A;
                G.inv_np1 = U.md.inv_np1;
                G.max_step = o->max_step;
                G.u0 = U.md.ubar;
                const size_t n3 = (size_t)n * n * n;
                if (m == 0) {
                    G.u = U.u;
                    G.src = U.rho;
                    G.fscale = U.md.D;
                    G.sref = 1.0;
                    G.fshift = U.md.Sbar;
                } else {
                    G.u = pool + at;
                    G.uhat = pool + at + n3;
                    G.f = pool + at + 2 * n3;
                    G.src = G.f;
                    G.fscale = 1.0;
                    G.sref = 0.0;
                    G.fshift = 0.0;
                    at += 3 * n3;
                }
                if (!U.periodic) {
                    G.ub = pool + at;
                    at += 6 * (size_t)n * n;
                }
                if (mixed) {
                    G.ub32 = pool32 + at32;
                    G.e32 = pool32 + at32 + n3;
                    G.f32 = pool32 + at32 + 2 * n3;
                    at32 += 3 * n3;
                    if (m > 0) {
                        G.eh32 = pool32 + at32;
                        at32 += n3;
                    }
                    if (pair_level(U, n)) {
                        G.e32b = pool32 + at32;
                        at32 += n3;
                    }
                }
            }
        }
        // tables
        Meta meta;
        int maxlev = 0;
        for (Unit& U : units) maxlev = std::max(maxlev, U.nlev);
        plan.depth.assign(maxlev, Depth{});
        for (int m = 0; m < maxlev; ++m) {
            std::vector<mgfr::BGrid> f, cgr, crs;
            for (Unit& U : units) {
                if (U.nlev > m + 1) {
                    f.push_back(U.g[m]);
                    cgr.push_back(U.g[m + 1]);
                } else if (U.nlev == m + 1) {
                    crs.push_back(U.g[m]);
                }
            }
            Depth& D = plan.depth[m];
            D.deep = !f.empty();
            D.coarsest = !crs.empty();
            if (D.deep) {
                D.half = sweep_tables(meta, f, o->tile);
                D.coarse_c = table(meta, cgr, [](const mgfr::BGrid& g) { return cells3(g); });
                // resid_restrict: table over the coarse cells, indexed by the fine grids
                D.coarse_f = table(meta, f, [](const mgfr::BGrid& g) { return cells3(g) / 8; });
                D.coarse_f.other = D.coarse_c.grids;  // coarse grids, same order
                D.rr = rr_tables(meta, f, cgr);
                std::vector<mgfr::BGrid> pf, pc;
                for (size_t i = 0; i < f.size(); ++i)
                    if (!f[i].periodic) {
                        pf.push_back(f[i]);
                        pc.push_back(cgr[i]);
                    }
                D.faces_c = table(meta, pc, [](const mgfr::BGrid& g) { return 6LL * g.n * g.n; });
                D.faces_c.other = meta.add(pf);
            }
            if (D.coarsest) {
                D.crs.grids = meta.add(crs);
                D.crs.ngrid = (int)crs.size();
            }
        }
        std::vector<mgfr::BGrid> g0;
        for (Unit& U : units) g0.push_back(U.g[0]);
        std::vector<int> first, count;
        plan.cells0 = table(meta, g0, [](const mgfr::BGrid& g) { return cells3(g); }, &first, &count);
        plan.fuse_add = o->precision == MGFR_MIXED && o->post >= 2 && o->post % 2 == 0;
        plan.add0 = table(meta, add_rest(g0, plan.depth.empty() || !plan.depth[0].deep ? nullptr : &plan.depth[0].half,
                                         plan.fuse_add),
                          [](const mgfr::BGrid& g) { return cells3(g); });
        plan.first = meta.add(first);
        plan.count = meta.add(count);
        plan.norm = norm_tables(meta, g0);
        plan.nunit = (int)units.size();
        plan.nblk_cells0 = plan.cells0.nblk;
        if (!phases) build_units(meta);
        setup_offset = meta.bytes.size();
        meta_image = std::move(meta.bytes);
        return MGFR_OK;
    }

    // Tables of the workgroup-per-unit engine: every level of every unit in one array, the
    // whole units in queue order (largest first), and the launch-based depths of the large
    // units with the tails that start below each.
    void build_units(Meta& meta)
    {
        std::vector<mgfr::BGrid> allg;
        std::vector<int> first, nlev, order, ids;
        std::vector<double> ncell;
        for (size_t ui = 0; ui < units.size(); ++ui) {
            first.push_back((int)allg.size());
            nlev.push_back(units[ui].nlev);
            for (const mgfr::BGrid& G : units[ui].g) allg.push_back(G);
            if (units[ui].n <= W) {
                order.push_back((int)ui);
            } else {
                ids.push_back((int)ui);
                ncell.push_back((double)cells3(units[ui].g[0]));
            }
        }
        std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return units[a].n > units[b].n; });
        up.grids = meta.add(allg);
        up.first = meta.add(first);
        up.nlev = meta.add(nlev);
        up.order = meta.add(order);
        up.nwhole = (int)order.size();
        up.ranges.clear();
        for (int b = 0; b < up.nwhole;) {
            const int side = units[order[b]].n;
            int e = b;
            while (e < up.nwhole && units[order[e]].n == side) ++e;
            up.ranges.push_back(make_int3(b, e, side));
            b = e;
        }
        up.nlarge = (int)ids.size();
        up.ids = meta.add(ids);
        up.ncell = meta.add(ncell);
        std::vector<mgfr::BGrid> g0;
        for (int u : ids) g0.push_back(units[u].g[0]);
        up.cells0 = table(meta, g0, [](const mgfr::BGrid& g) { return cells3(g); });
        up.norm = norm_tables(meta, g0);
        std::vector<int2> all_tails;
        up.depth.clear();
        for (int m = 0;; ++m) {
            std::vector<mgfr::BGrid> f, cg;
            std::vector<int2> tails;
            for (int u : ids) {
                const Unit& U = units[u];
                if (m + 1 >= U.nlev || U.g[m].n <= W) continue;  // not launch-based at depth m
                f.push_back(U.g[m]);
                cg.push_back(U.g[m + 1]);
                if (U.g[m + 1].n <= W) tails.push_back(make_int2(first[u] + m + 1, U.nlev - m - 1));
            }
            if (f.empty()) break;
            UDepth D;
            D.deep = true;
            D.half = sweep_tables(meta, f, o->tile);
            D.coarse_c = table(meta, cg, [](const mgfr::BGrid& g) { return cells3(g); });
            D.coarse_f = table(meta, f, [](const mgfr::BGrid& g) { return cells3(g) / 8; });
            D.coarse_f.other = D.coarse_c.grids;
            D.rr = rr_tables(meta, f, cg);
            D.tails = meta.add(tails);
            D.ntail = (int)tails.size();
            all_tails.insert(all_tails.end(), tails.begin(), tails.end());
            up.depth.push_back(D);
        }
        up.all_tails = meta.add(all_tails);
        up.nall_tails = (int)all_tails.size();
        up.add0 = table(meta, add_rest(g0, up.depth.empty() ? nullptr : &up.depth[0].half, plan.fuse_add),
                        [](const mgfr::BGrid& g) { return cells3(g); });
    }

    std::vector<char> meta_image;
    size_t setup_offset = 0;

    // Appends extra tables (patch set-up) before the upload.
    template <class T>
    size_t add_extra(const std::vector<T>& v)
    {
        Meta m;
        m.bytes = std::move(meta_image);
        const size_t off = m.add(v);
        meta_image = std::move(m.bytes);
        return off;
    }

    int upload()
    {
        // pinned staging: [per-unit (sum, max) | per-unit flags | descriptor image]
        const size_t nu = units.size();
        const size_t meta_at = (sizeof(double) * 2 * nu + sizeof(int) * nu + 255) & ~size_t(255);
        MGFR_TRY(ensure_pinned(c, meta_at + meta_image.size()));
        hout = (double*)c->pin;
        hact = (int*)(hout + 2 * nu);
        char* hmeta = (char*)c->pin + meta_at;
        std::memcpy(hmeta, meta_image.data(), meta_image.size());
        MGFR_TRY(alloc(&dmeta, meta_image.size()));
        MGFR_TRY(hip_check(c, hipMemcpyAsync(dmeta, hmeta, meta_image.size(), hipMemcpyHostToDevice, s),
                           "hipMemcpyAsync"));
        MGFR_TRY(alloc(&dactive, nu));
        active.assign(nu, 1);
        MGFR_TRY(upload_active());
        const long long nparts = std::max({plan.nblk_cells0, plan.norm.nparts, up.norm.nparts, 1LL});
        MGFR_TRY(alloc(&dpartial, 2 * (size_t)nparts));
        MGFR_TRY(alloc(&dout, 2 * nu));
        if (!phases) {
            MGFR_TRY(alloc(&dhist, nu * (size_t)(o->max_cycles + 1)));
            MGFR_TRY(alloc(&dints, 2 * nu + 1 + kQueues));  // cycles, status per unit; any; queues
        }
        // the staging area must stay unchanged until the copies have run
        return hip_check(c, hipStreamSynchronize(s), "hipStreamSynchronize");
    }

    // Copies the host active flags to the device (through pinned memory, so the copy is a
    // direct transfer; the staging area is next rewritten after a later synchronisation).
    int upload_active()
    {
        std::copy(active.begin(), active.end(), hact);
        return hip_check(c, hipMemcpyAsync(dactive, hact, sizeof(int) * active.size(), hipMemcpyHostToDevice, s),
                         "hipMemcpyAsync");
    }

    // Cell updates of one V-cycle of the active units (pre + post sweeps on every level
    // above the coarsest), added to the statistics per cycle run.
    void count_vcycle(int times)
    {
        for (size_t i = 0; i < units.size(); ++i) {
            if (!active[i]) continue;
            for (int m = 0; m + 1 < units[i].nlev; ++m) {
                const long long n3 = cells3(units[i].g[m]) * (o->pre + o->post) * times;
                c->stats.cell_updates += n3;
                if (m == 0) c->stats.finest_updates += n3;
            }
        }
    }

    // MGFR_PROFILE, eager cycles only: HIP events around every sweep of the finest depth (the
    // finest level of every unit), with the algorithmic bytes of its active units.
    long long act0 = 0;  // cells of the finest levels of the active units, this cycle
    bool profiled(int m) const { return m == 0 && (o->flags & MGFR_PROFILE) && !(o->flags & MGFR_GRAPH); }
    int ev_begin(int m)
    {
        if (!profiled(m)) return MGFR_OK;
        if ((size_t)c->ev_used + 2 > c->ev.size()) {
            for (int k = 0; k < 64; ++k) {
                hipEvent_t ev;
                MGFR_TRY(hip_check(c, hipEventCreate(&ev), "hipEventCreate"));
                c->ev.push_back(ev);
            }
        }
        return hip_check(c, hipEventRecord(c->ev[c->ev_used], s), "hipEventRecord");
    }
    int ev_end(int m, double bytes_per_cell, int count, int launches)
    {
        if (!profiled(m)) return MGFR_OK;
        MGFR_TRY(hip_check(c, hipEventRecord(c->ev[c->ev_used + 1], s), "hipEventRecord"));
        c->ev_used += 2;
        c->stats.sweep_launches += launches;
        c->stats.sweep_bytes += bytes_per_cell * (double)act0 * count;
        return MGFR_OK;
    }
    // Sums the timed intervals (the stream has been synchronised) and releases the events.
    int harvest()
    {
        for (int k = 0; k < c->ev_used; k += 2) {
            float ms = 0.0f;
            MGFR_TRY(hip_check(c, hipEventElapsedTime(&ms, c->ev[k], c->ev[k + 1]), "hipEventElapsedTime"));
            c->stats.sweep_ms += ms;
        }
        c->ev_used = 0;
        return MGFR_OK;
    }

    // `count` red-black sweeps of a depth's grids (grids are independent: the tables in turn);
    // the number of kernel launches in *launches.  add_u (an even count): the last sweep of
    // the boxes swept in fused pairs also adds their correction, u += e.
    int ngs(const Sweep& S, bool mixed, int count, int* launches, bool add_u = false)
    {
        int nl = 0;
        for (int k = 0; k < count; ++k) {
            if (S.cell.nblk > 0) {
                if (mixed)
                    MGFR_TRY(hip_check(c, mgfr::batch_ngs32(tab(S.cell), S.cell.nblk, s), "batch_ngs32"));
                else
                    MGFR_TRY(hip_check(c, mgfr::batch_ngs(tab(S.cell), S.cell.nblk, s), "batch_ngs"));
                nl += 2;
            }
            if (S.col.nblk > 0) {
                if (mixed)
                    MGFR_TRY(hip_check(c, mgfr::batch_ngs32_col(tab(S.col), S.col.nblk, s), "batch_ngs32_col"));
                else
                    MGFR_TRY(hip_check(c, mgfr::batch_ngs_col(tab(S.col), S.col.nblk, s), "batch_ngs_col"));
                nl += 2;
            }
        }
        for (int w = 0; w < 2; ++w) {
            if (S.pair[w].nblk == 0) continue;
            // pairs of fused sweeps end where they began (e32); an odd one out runs in place
            for (int k = 0; k + 2 <= count; k += 2) {
                const bool add = add_u && w == 1 && k + 2 == count && !(count & 1);
                MGFR_TRY(hip_check(c, mgfr::batch_ngs32_pair(tab(S.pair[w]), S.pair[w].nblk, w == 1, add, s),
                                   "batch_ngs32_pair"));
                nl += 2;
            }
            if (count & 1) {
                MGFR_TRY(hip_check(c, mgfr::batch_ngs32_col(tab(S.pair1[w]), S.pair1[w].nblk, s), "batch_ngs32_col"));
                nl += 2;
            }
        }
        if (launches) *launches = nl;
        return MGFR_OK;
    }

    // Residual and restriction of a depth into its coarse level (FP64, or single: the
    // correction equation)
    int resid_restrict(const RR& R, bool single)
    {
        if (R.tile.nblk > 0)
            MGFR_TRY(hip_check(c, mgfr::batch_resid_restrict_col(tab(R.tile), R.tile.nblk,
                                                                 (const mgfr::BGrid*)(dmeta + R.tile.other), single, s),
                               "batch_resid_restrict_col"));
        if (R.cell.nblk > 0) {
            const mgfr::BGrid* coarse = (const mgfr::BGrid*)(dmeta + R.cell.other);
            if (single)
                MGFR_TRY(hip_check(c, mgfr::batch_resid_restrict32(tab(R.cell), R.cell.nblk, coarse, s),
                                   "batch_resid_restrict32"));
            else
                MGFR_TRY(hip_check(c, mgfr::batch_resid_restrict(tab(R.cell), R.cell.nblk, coarse, s),
                                   "batch_resid_restrict"));
        }
        return MGFR_OK;
    }

    // read u and rho, write u
    int sweep(int m, int count)
    {
        if (count == 0) return MGFR_OK;
        const Depth& D = plan.depth[m];
        int nl = 0;
        MGFR_TRY(ev_begin(m));
        MGFR_TRY(ngs(D.half, false, count, &nl));
        return ev_end(m, 24.0, count, nl);
    }

    int vcycle(int m)
    {
        const Depth& D = plan.depth[m];
        if (D.coarsest)
            MGFR_TRY(hip_check(c, mgfr::batch_coarsest(grids(D.crs), D.crs.ngrid, o->coarsest_n, dactive, o->coarsest_sweeps,
                                                       o->coarsest_rtol, s),
                               "batch_coarsest"));
        if (!D.deep) return MGFR_OK;
        MGFR_TRY(sweep(m, o->pre));
        MGFR_TRY(resid_restrict(D.rr, false));
        MGFR_TRY(hip_check(c, mgfr::batch_fas_rhs(tab(D.coarse_c), D.coarse_c.nblk, s), "batch_fas_rhs"));
        MGFR_TRY(vcycle(m + 1));
        MGFR_TRY(hip_check(c, mgfr::batch_coarse_diff(tab(D.coarse_c), D.coarse_c.nblk, s), "batch_coarse_diff"));
        MGFR_TRY(hip_check(c, mgfr::batch_prolong_add8(tab(D.coarse_f), D.coarse_f.nblk,
                                                       (const mgfr::BGrid*)(dmeta + D.coarse_f.other), s),
                           "batch_prolong_add8"));
        MGFR_TRY(sweep(m, o->post));
        return MGFR_OK;
    }

    // ---- mixed precision: single-precision correction V-cycle, double-precision outer loop
    // credited 12 B per cell: e and the right-hand side read, e written (the fixed base ub,
    // also read, is not counted)
    int sweep32(int m, int count, bool add_u = false)
    {
        if (count == 0) return MGFR_OK;
        const Depth& D = plan.depth[m];
        int nl = 0;
        MGFR_TRY(ev_begin(m));
        MGFR_TRY(ngs(D.half, true, count, &nl, add_u));
        return ev_end(m, 12.0, count, nl);
    }

    // add_u: the last correction cycle of an outer iteration (its last finest sweep adds u += e
    // for the boxes swept in fused pairs)
    int vcycle32(int m, bool add_u = false)
    {
        const Depth& D = plan.depth[m];
        if (D.coarsest)
            MGFR_TRY(hip_check(c, mgfr::batch_coarsest32(grids(D.crs), D.crs.ngrid, o->coarsest_n, dactive, o->coarsest_sweeps,
                                                         o->coarsest_rtol, s),
                               "batch_coarsest32"));
        if (!D.deep) return MGFR_OK;
        MGFR_TRY(sweep32(m, o->pre));
        MGFR_TRY(resid_restrict(D.rr, true));
        MGFR_TRY(hip_check(c, mgfr::batch_fas_rhs32(tab(D.coarse_c), D.coarse_c.nblk, s), "batch_fas_rhs32"));
        MGFR_TRY(vcycle32(m + 1));
        MGFR_TRY(hip_check(c, mgfr::batch_coarse_diff32(tab(D.coarse_c), D.coarse_c.nblk, s), "batch_coarse_diff32"));
        MGFR_TRY(hip_check(c, mgfr::batch_prolong_add8_32(tab(D.coarse_f), D.coarse_f.nblk,
                                                          (const mgfr::BGrid*)(dmeta + D.coarse_f.other), s),
                           "batch_prolong_add8_32"));
        MGFR_TRY(sweep32(m, o->post, add_u && m == 0 && plan.fuse_add));
        return MGFR_OK;
    }

    // Base of every coarse level: R ub, from the finest down.
    int restrict_base32()
    {
        for (size_t m = 0; m < plan.depth.size(); ++m) {
            const Depth& D = plan.depth[m];
            if (!D.deep) continue;
            MGFR_TRY(hip_check(c, mgfr::batch_restrict_base32(tab(D.coarse_f), D.coarse_f.nblk,
                                                              (const mgfr::BGrid*)(dmeta + D.coarse_f.other), s),
                               "batch_restrict_base32"));
        }
        return MGFR_OK;
    }

    // Per-unit (sum d^2, max |d|) of the finest double-precision residual of N's units into
    // dout; cast: also the single-precision r = -d, ub = u and e = 0 of the next inner solve.
    int resid_norm(const NormPlan& N, bool cast)
    {
        if (N.tile.nblk > 0)
            MGFR_TRY(hip_check(c, mgfr::batch_resid_col(tab(N.tile), N.tile.nblk, dpartial, cast, s), "batch_resid_col"));
        if (N.cell.nblk > 0) {
            double* part = dpartial + 2 * (size_t)N.tile.nblk;
            if (cast)
                MGFR_TRY(hip_check(c, mgfr::batch_resid_cast(tab(N.cell), N.cell.nblk, part, s), "batch_resid_cast"));
            else
                MGFR_TRY(hip_check(c, mgfr::batch_norm_blocks(tab(N.cell), N.cell.nblk, part, s), "batch_norm_blocks"));
        }
        return hip_check(c, mgfr::batch_fold(dpartial, (const int*)(dmeta + N.first), (const int*)(dmeta + N.count),
                                             N.ngrid, dout, s),
                         "batch_fold");
    }

    // Per-unit rms of the finest double-precision residual (synchronises); also writes the
    // single-precision right-hand side r = -d, base ub = u and e = 0 of the next inner solve.
    int norms_cast(std::vector<double>& rms, std::vector<double>& mx)
    {
        MGFR_TRY(resid_norm(plan.norm, true));
        MGFR_TRY(hip_check(c, hipMemcpyAsync(hout, dout, sizeof(double) * 2 * units.size(), hipMemcpyDeviceToHost, s),
                           "hipMemcpyAsync"));
        MGFR_TRY(hip_check(c, hipStreamSynchronize(s), "hipStreamSynchronize"));
        for (size_t i = 0; i < units.size(); ++i) {
            if (!active[i]) continue;
            rms[i] = std::sqrt(hout[2 * i] / (double)cells3(units[i].g[0]));
            mx[i] = hout[2 * i + 1];
        }
        return MGFR_OK;
    }

    // Coarse-level patch boundary values, from the finest ones down.
    int restrict_faces()
    {
        for (size_t m = 0; m < plan.depth.size(); ++m) {
            const Depth& D = plan.depth[m];
            if (!D.deep || D.faces_c.nblk == 0) continue;
            MGFR_TRY(hip_check(c, mgfr::batch_restrict_faces(tab(D.faces_c), D.faces_c.nblk,
                                                             (const mgfr::BGrid*)(dmeta + D.faces_c.other), s),
                               "batch_restrict_faces"));
        }
        return MGFR_OK;
    }

    // Per-unit rms of the finest residual into rms[] (synchronises).
    int norms(std::vector<double>& rms, std::vector<double>& mx)
    {
        MGFR_TRY(resid_norm(plan.norm, false));
        MGFR_TRY(hip_check(c, hipMemcpyAsync(hout, dout, sizeof(double) * 2 * units.size(), hipMemcpyDeviceToHost, s),
                           "hipMemcpyAsync"));
        MGFR_TRY(hip_check(c, hipStreamSynchronize(s), "hipStreamSynchronize"));
        for (size_t i = 0; i < units.size(); ++i) {
            if (!active[i]) continue;
            rms[i] = std::sqrt(hout[2 * i] / (double)cells3(units[i].g[0]));
            mx[i] = hout[2 * i + 1];
        }
        return MGFR_OK;
    }

    int check_finite()
    {
        MGFR_TRY(hip_check(c, mgfr::batch_nonfinite(tab(plan.cells0), plan.cells0.nblk, dpartial, s), "batch_nonfinite"));
        MGFR_TRY(hip_check(c, mgfr::batch_fold(dpartial, (const int*)(dmeta + plan.first),
                                               (const int*)(dmeta + plan.count), plan.nunit, dout, s),
                           "batch_fold"));
        MGFR_TRY(hip_check(c, hipMemcpyAsync(hout, dout, sizeof(double) * 2 * units.size(), hipMemcpyDeviceToHost, s),
                           "hipMemcpyAsync"));
        MGFR_TRY(hip_check(c, hipStreamSynchronize(s), "hipStreamSynchronize"));
        for (size_t i = 0; i < units.size(); ++i)
            if (hout[2 * i] != 0.0)
                return c->fail(MGFR_ENONFINITE, "unit %zu: %.0f non-finite density or start values", i, hout[2 * i]);
        return MGFR_OK;
    }

    // The launches of one cycle: a double-precision V-cycle, or (mixed) the coarse bases,
    // inner_cycles single-precision V-cycles on the correction and u += e.  Every launch
    // reads the active flags from device memory, so the same sequence serves every cycle.
    int cycle_body()
    {
        if (o->precision != MGFR_MIXED) return vcycle(0);
        MGFR_TRY(restrict_base32());
        for (int it = 0; it < o->inner_cycles; ++it) MGFR_TRY(vcycle32(0, it + 1 == o->inner_cycles));
        if (plan.add0.nblk == 0) return MGFR_OK;
        return hip_check(c, mgfr::batch_add_correction(tab(plan.add0), plan.add0.nblk, s), "batch_add_correction");
    }

    // With MGFR_GRAPH, the body is captured once on a private stream and the graph is
    // launched on the caller's stream for every cycle.
    hipStream_t cap_stream = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t gexec = nullptr;

    int cycle()
    {
        if (!(o->flags & MGFR_GRAPH)) return cycle_body();
        if (!gexec) {
            MGFR_TRY(hip_check(c, hipStreamCreateWithFlags(&cap_stream, hipStreamNonBlocking), "hipStreamCreate"));
            hipStream_t caller = s;
            s = cap_stream;
            MGFR_TRY(hip_check(c, hipStreamBeginCapture(cap_stream, hipStreamCaptureModeThreadLocal),
                               "hipStreamBeginCapture"));
            const int st = cycle_body();
            hipGraph_t g = nullptr;
            const hipError_t e = hipStreamEndCapture(cap_stream, &g);
            s = caller;
            graph = g;
            MGFR_TRY(st);
            MGFR_TRY(hip_check(c, e, "hipStreamEndCapture"));
            MGFR_TRY(hip_check(c, hipGraphInstantiate(&gexec, graph, nullptr, nullptr, 0), "hipGraphInstantiate"));
        }
        return hip_check(c, hipGraphLaunch(gexec, s), "hipGraphLaunch");
    }

    // Cycles until every unit has rms <= tol or max_cycles; histories per unit.  Double
    // precision: one V-cycle per cycle.  Mixed: one outer iteration per cycle (inner_cycles
    // single-precision V-cycles on the correction, then u += e and the double-precision
    // residual).
    int run(double* res_hist, int* n_hist, int* worst_status)
    {
        const bool mixed = o->precision == MGFR_MIXED;
        const int H = o->max_cycles + 1;
        std::vector<double> rms(units.size(), 0.0), mx(units.size(), 0.0);
        std::vector<int> k(units.size(), 0);
        MGFR_TRY(mixed ? norms_cast(rms, mx) : norms(rms, mx));
        for (size_t i = 0; i < units.size(); ++i) {
            if (res_hist) res_hist[i * H] = rms[i];
            if (!(std::isfinite(rms[i])) || rms[i] <= o->tol) active[i] = 0;
        }
        int cycles = 0;
        for (;;) {
            bool any = false;
            for (size_t i = 0; i < units.size(); ++i) any = any || active[i];
            if (!any || cycles >= o->max_cycles) break;
            MGFR_TRY(upload_active());
            act0 = 0;
            for (size_t i = 0; i < units.size(); ++i)
                if (active[i] && units[i].nlev > 1) act0 += cells3(units[i].g[0]);  // swept at depth 0
            MGFR_TRY(cycle());
            count_vcycle(mixed ? o->inner_cycles : 1);
            if (mixed) {
                MGFR_TRY(norms_cast(rms, mx));
                c->stats.inner_cycles += o->inner_cycles;
            } else {
                MGFR_TRY(norms(rms, mx));
            }
            MGFR_TRY(harvest());  // the norms synchronised the stream
            ++cycles;
            for (size_t i = 0; i < units.size(); ++i) {
                if (!active[i]) continue;
                ++k[i];
                if (res_hist) res_hist[i * H + k[i]] = rms[i];
                if (!std::isfinite(rms[i]) || rms[i] <= o->tol) active[i] = 0;
            }
        }
        c->stats.cycles += cycles;
        *worst_status = MGFR_OK;
        for (size_t i = 0; i < units.size(); ++i) {
            if (n_hist) n_hist[i] = k[i] + 1;
            if (!std::isfinite(rms[i])) *worst_status = MGFR_ENONFINITE;
            else if (rms[i] > o->tol && *worst_status == MGFR_OK) *worst_status = MGFR_ENOTCONV;
        }
        return MGFR_OK;
    }

    // ---- workgroup-per-unit engine ------------------------------------------------------------
    mgfr::UnitSet uset() const
    {
        mgfr::UnitSet u;
        u.grids = (const mgfr::BGrid*)(dmeta + up.grids);
        u.first = (const int*)(dmeta + up.first);
        u.nlev = (const int*)(dmeta + up.nlev);
        u.order = (const int*)(dmeta + up.order);
        return u;
    }
    mgfr::UnitOut uout() const
    {
        const size_t nu = units.size();
        return mgfr::UnitOut{dhist, dints, dints + nu, o->max_cycles + 1};
    }
    mgfr::UnitCfg ucfg() const
    {
        mgfr::UnitCfg f;
        f.tol = o->tol;
        f.rtol = o->coarsest_rtol;
        f.pre = o->pre;
        f.post = o->post;
        f.max_cycles = o->max_cycles;
        f.inner = o->inner_cycles;
        f.cap = o->coarsest_sweeps;
        return f;
    }
    int* dany() const { return dints + 2 * units.size(); }
    // the device counter of whole-unit launch r (one per side, at most kQueues)
    int* dqueue(size_t r) const { return dints + 2 * units.size() + 1 + r; }
    mgfr::BTable utab(const Launch& L) const
    {
        mgfr::BTable t;
        t.grids = (const mgfr::BGrid*)(dmeta + L.grids);
        t.blk = (const int2*)(dmeta + L.blk);
        t.active = dactive;
        return t;
    }

    // one V-cycle of the large units from depth m (double precision, or the single-precision
    // correction cycle when mixed): launch-based phases while their level is larger than W,
    // then one workgroup per unit for the rest
    int uvcycle(int m, bool mixed, bool add_u = false)
    {
        const UDepth& D = up.depth[m];
        const mgfr::BGrid* coarse = (const mgfr::BGrid*)(dmeta + D.coarse_f.other);
        MGFR_TRY(usweep(m, mixed, o->pre));
        if (mixed) {
            MGFR_TRY(resid_restrict(D.rr, true));
            MGFR_TRY(hip_check(c, mgfr::batch_fas_rhs32(utab(D.coarse_c), D.coarse_c.nblk, s), "batch_fas_rhs32"));
        } else {
            MGFR_TRY(resid_restrict(D.rr, false));
            MGFR_TRY(hip_check(c, mgfr::batch_fas_rhs(utab(D.coarse_c), D.coarse_c.nblk, s), "batch_fas_rhs"));
        }
        // The tails (every tail level has side W) touch only their own units: while other
        // units go deeper they run on the tail stream, joined before the prolongation.
        const bool deeper = (size_t)m + 1 < up.depth.size();
        const bool fork = D.ntail > 0 && deeper && m < mgfr_ctx::kTailForks;
        if (D.ntail > 0) {
            hipStream_t ts = s;
            if (fork) {
                MGFR_TRY(ensure_tail(c));
                MGFR_TRY(hip_check(c, hipEventRecord(c->ev_tf[m], s), "hipEventRecord"));
                MGFR_TRY(hip_check(c, hipStreamWaitEvent(c->tail, c->ev_tf[m], 0), "hipStreamWaitEvent"));
                ts = c->tail;
            }
            MGFR_TRY(hip_check(c, mgfr::unit_tail(uset(), (const int2*)(dmeta + D.tails), D.ntail, W, dactive, ucfg(),
                                                  mixed, ts),
                               "unit_tail"));
            if (fork) MGFR_TRY(hip_check(c, hipEventRecord(c->ev_tj[m], c->tail), "hipEventRecord"));
        }
        if (deeper) MGFR_TRY(uvcycle(m + 1, mixed));
        if (fork) MGFR_TRY(hip_check(c, hipStreamWaitEvent(s, c->ev_tj[m], 0), "hipStreamWaitEvent"));
        if (mixed) {
            MGFR_TRY(hip_check(c, mgfr::batch_coarse_diff32(utab(D.coarse_c), D.coarse_c.nblk, s),
                               "batch_coarse_diff32"));
            MGFR_TRY(hip_check(c, mgfr::batch_prolong_add8_32(utab(D.coarse_f), D.coarse_f.nblk, coarse, s),
                               "batch_prolong_add8_32"));
        } else {
            MGFR_TRY(hip_check(c, mgfr::batch_coarse_diff(utab(D.coarse_c), D.coarse_c.nblk, s), "batch_coarse_diff"));
            MGFR_TRY(hip_check(c, mgfr::batch_prolong_add8(utab(D.coarse_f), D.coarse_f.nblk, coarse, s),
                               "batch_prolong_add8"));
        }
        MGFR_TRY(usweep(m, mixed, o->post, mixed && add_u && m == 0 && plan.fuse_add));
        return MGFR_OK;
    }

    int usweep(int m, bool mixed, int count, bool add_u = false)
    {
        if (count == 0) return MGFR_OK;
        const UDepth& D = up.depth[m];
        const bool timed = m == 0 && (o->flags & MGFR_PROFILE) && !(o->flags & MGFR_GRAPH);
        if (timed) MGFR_TRY(ev_begin(0));
        int nl = 0;
        MGFR_TRY(ngs(D.half, mixed, count, &nl, add_u));
        if (timed) {
            MGFR_TRY(hip_check(c, hipEventRecord(c->ev[c->ev_used + 1], s), "hipEventRecord"));
            c->ev_used += 2;
            c->stats.sweep_launches += nl;
        }
        return MGFR_OK;
    }

    // Stop test of the large units on the device: the residual (mixed: with the cast of the
    // next right-hand side and base), its per-unit sums and the judge.
    int ujudge(bool mixed, bool first)
    {
        MGFR_TRY(resid_norm(up.norm, mixed));
        return hip_check(c, mgfr::unit_judge(dout, (const int*)(dmeta + up.ids), (const double*)(dmeta + up.ncell),
                                             up.nlarge, dactive, uout(), o->tol, o->max_cycles, first, dany(), s),
                         "unit_judge");
    }

    // One cycle of the large units: a double-precision V-cycle, or (mixed) the coarse bases,
    // inner_cycles single-precision V-cycles and u += e; then the device stop test.
    int ucycle_body()
    {
        const bool mixed = o->precision == MGFR_MIXED;
        if (mixed) {
            for (size_t m = 0; m < up.depth.size(); ++m) {
                const UDepth& D = up.depth[m];
                MGFR_TRY(hip_check(c, mgfr::batch_restrict_base32(utab(D.coarse_f), D.coarse_f.nblk,
                                                                  (const mgfr::BGrid*)(dmeta + D.coarse_f.other), s),
                                   "batch_restrict_base32"));
            }
            if (!mgfr::unit_resident(W))  // the resident tail kernels form these themselves
                MGFR_TRY(hip_check(c, mgfr::unit_tail_base32(uset(), (const int2*)(dmeta + up.all_tails),
                                                             up.nall_tails, dactive, s),
                                   "unit_tail_base32"));
            for (int it = 0; it < o->inner_cycles; ++it) MGFR_TRY(uvcycle(0, true, it + 1 == o->inner_cycles));
            if (up.add0.nblk > 0)
                MGFR_TRY(hip_check(c, mgfr::batch_add_correction(utab(up.add0), up.add0.nblk, s),
                                   "batch_add_correction"));
        } else {
            MGFR_TRY(uvcycle(0, false));
        }
        return ujudge(mixed, false);
    }

    int ucycle()
    {
        if (!(o->flags & MGFR_GRAPH)) return ucycle_body();
        if (!gexec) {
            MGFR_TRY(hip_check(c, hipStreamCreateWithFlags(&cap_stream, hipStreamNonBlocking), "hipStreamCreate"));
            hipStream_t caller = s;
            s = cap_stream;
            MGFR_TRY(hip_check(c, hipStreamBeginCapture(cap_stream, hipStreamCaptureModeThreadLocal),
                               "hipStreamBeginCapture"));
            const int st = ucycle_body();
            hipGraph_t g = nullptr;
            const hipError_t e = hipStreamEndCapture(cap_stream, &g);
            s = caller;
            graph = g;
            MGFR_TRY(st);
            MGFR_TRY(hip_check(c, e, "hipStreamEndCapture"));
            MGFR_TRY(hip_check(c, hipGraphInstantiate(&gexec, graph, nullptr, nullptr, 0), "hipGraphInstantiate"));
        }
        return hip_check(c, hipGraphLaunch(gexec, s), "hipGraphLaunch");
    }

    // Number of large units still active (synchronises).
    int read_any(int* any)
    {
        int* h = hact;
        MGFR_TRY(hip_check(c, hipMemcpyAsync(h, dany(), sizeof(int), hipMemcpyDeviceToHost, s), "hipMemcpyAsync"));
        MGFR_TRY(hip_check(c, hipStreamSynchronize(s), "hipStreamSynchronize"));
        *any = *h;
        return MGFR_OK;
    }

    // Solves every unit; histories, cycle counts and statuses come back once at the end.
    int run_units(double* res_hist, int* n_hist, int* worst_status)
    {
        const bool mixed = o->precision == MGFR_MIXED;
        const size_t nu = units.size();
        const int H = o->max_cycles + 1;
        c->ev_used = 0;
        // whole units: one persistent launch on the side stream, beside the large units; while
        // those run, the whole-unit workgroups (one per CU at side 16) keep a quarter of the
        // compute units free for the large units' launches (amr workload: 31.1 -> 29.9 ms mixed)
        if (up.nwhole > 0) {
            MGFR_TRY(ensure_side(c));
            int max_wg = 1 << 30;
            if (up.nlarge > 0) {
                int cus = 0;
                MGFR_TRY(hip_check(c, hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, c->device),
                                   "hipDeviceGetAttribute"));
                max_wg = std::max(1, 3 * cus / 4);
            }
            MGFR_TRY(hip_check(c, hipEventRecord(c->ev_fork, s), "hipEventRecord"));
            MGFR_TRY(hip_check(c, hipStreamWaitEvent(c->side, c->ev_fork, 0), "hipStreamWaitEvent"));
            for (size_t r = 0; r < up.ranges.size(); ++r) {
                const int3 g = up.ranges[r];
                MGFR_TRY(hip_check(c, mgfr::unit_whole(uset(), g.x, g.y, g.z, dqueue(r), uout(), ucfg(), mixed, max_wg,
                                                       c->side),
                                   "unit_whole"));
            }
            MGFR_TRY(hip_check(c, hipEventRecord(c->ev_join, c->side), "hipEventRecord"));
        }
        int cycles = 0;
        if (up.nlarge > 0) {
            MGFR_TRY(hip_check(c, mgfr::unit_fill_int(dactive, 1, (int)nu, s), "unit_fill_int"));
            MGFR_TRY(ujudge(mixed, true));
            int any = 0;
            MGFR_TRY(read_any(&any));
            while (any > 0 && cycles < o->max_cycles) {
                // a chunk of cycles between host checks: units converge after several cycles,
                // and the ones that have are switched off on the device
                const int chunk = std::min(cycles == 0 ? 4 : 2, o->max_cycles - cycles);
                for (int k = 0; k < chunk; ++k) MGFR_TRY(ucycle());
                cycles += chunk;
                MGFR_TRY(read_any(&any));
            }
        }
        if (up.nwhole > 0) MGFR_TRY(hip_check(c, hipStreamWaitEvent(s, c->ev_join, 0), "hipStreamWaitEvent"));
        // results: histories, then cycles and statuses, through the pinned staging buffer
        const size_t hb = sizeof(double) * nu * H, ib = sizeof(int) * 2 * nu;
        MGFR_TRY(ensure_pinned(c, hb + ib));
        double* hh = (double*)c->pin;
        int* hi = (int*)((char*)c->pin + hb);
        MGFR_TRY(hip_check(c, hipMemcpyAsync(hh, dhist, hb, hipMemcpyDeviceToHost, s), "hipMemcpyAsync"));
        MGFR_TRY(hip_check(c, hipMemcpyAsync(hi, dints, ib, hipMemcpyDeviceToHost, s), "hipMemcpyAsync"));
        MGFR_TRY(hip_check(c, hipStreamSynchronize(s), "hipStreamSynchronize"));
        MGFR_TRY(harvest());
        *worst_status = MGFR_OK;
        const int per = mixed ? o->inner_cycles : 1;
        int maxk = 0;
        for (size_t i = 0; i < nu; ++i) {
            const int k = hi[i], st = hi[nu + i];
            maxk = std::max(maxk, k);
            if (res_hist) std::memcpy(res_hist + i * H, hh + i * H, sizeof(double) * (k + 1));
            if (n_hist) n_hist[i] = k + 1;
            if (st == 2) *worst_status = MGFR_ENONFINITE;
            else if (st == 1 && *worst_status == MGFR_OK) *worst_status = MGFR_ENOTCONV;
            const Unit& U = units[i];
            for (int m = 0; m + 1 < U.nlev; ++m) {
                const long long n3 = cells3(U.g[m]) * (o->pre + o->post) * (long long)k * per;
                c->stats.cell_updates += n3;
                if (m == 0) c->stats.finest_updates += n3;
            }
            if (U.n > W && (o->flags & MGFR_PROFILE) && !(o->flags & MGFR_GRAPH))
                c->stats.sweep_bytes += (mixed ? 12.0 : 24.0) * (double)cells3(U.g[0]) * (o->pre + o->post) *
                                        (double)k * per;
        }
        c->stats.cycles += maxk;
        if (mixed) c->stats.inner_cycles += maxk * o->inner_cycles;
        return MGFR_OK;
    }
};

// Which engine a batch runs, and the side up to which the default one relaxes a unit in
// one workgroup.
void engine(Batch& b)
{
    b.phases = (b.o->flags & MGFR_PER_PHASE) != 0;
    // a power of two, so that every tail level has side W
    const int w = std::max(b.o->unit_n > 0 ? b.o->unit_n : 16, b.o->coarsest_n);
    b.W = 1;
    while (2 * b.W <= w) b.W *= 2;
}

int check_batch_opts(mgfr_ctx* c, const mgfr_opts* o)
{
    MGFR_TRY(check_opts(c, o));
    if (o->flags & MGFR_SUBTRACT_MEAN) return c->fail(MGFR_EINVAL, "MGFR_SUBTRACT_MEAN is not available for batches");
    if (o->tau_alpha > 0.0) return c->fail(MGFR_EINVAL, "tau_alpha is not available for batches");
    return MGFR_OK;
}

}  // namespace

extern "C" {

int mg_fr_solve_patches(mgfr_ctx* c, const double* u_domain, int N0, const mgfr_patch* patches, int npatch,
                        const double* rho_packed, double* u_packed, long long packed_cells,
                        const mgfr_params* params, const mgfr_opts* o, double* res_hist, int* n_hist,
                        void* stream)
{
    if (!c) return MGFR_EINVAL;
    c->err.clear();
    c->stats = mgfr_stats{};
    const auto t0 = std::chrono::steady_clock::now();
    MGFR_TRY(check_batch_opts(c, o));
    Model md;
    if (derive_model(params, &md) != MGFR_OK) return c->fail(MGFR_EINVAL, "invalid model parameters");
    if (npatch < 0 || (npatch > 0 && (!patches || !u_domain || !rho_packed || !u_packed)))
        return c->fail(MGFR_EINVAL, "invalid patch arguments");
    if (!is_pow2(N0) || N0 < 2 || N0 > 2048) return c->fail(MGFR_EINVAL, "N0=%d must be a power of two", N0);
    if (npatch == 0) return MGFR_OK;
    // layout rules
    int maxlevel = 0;
    std::vector<std::pair<long long, long long>> ranges;
    for (int p = 0; p < npatch; ++p) {
        const mgfr_patch& P = patches[p];
        if (P.level < 1 || P.level > 10 || !is_pow2(P.n) || P.n < o->coarsest_n || P.n > 128)
            return c->fail(MGFR_EINVAL, "patch %d: level %d / n %d out of range", p, P.level, P.n);
        const long long side = (long long)N0 << P.level;
        for (int d = 0; d < 3; ++d) {
            if (P.origin[d] & 1) return c->fail(MGFR_EINVAL, "patch %d: origin not aligned to parent cells", p);
            if (P.origin[d] < 0 || P.origin[d] + P.n > side)
                return c->fail(MGFR_EINVAL, "patch %d: outside the level-%d domain", p, P.level);
        }
        if (P.level == 1) {
            if (P.parent != -1) return c->fail(MGFR_EINVAL, "patch %d: level-1 patches have parent -1", p);
        } else {
            if (P.parent < 0 || P.parent >= npatch || patches[P.parent].level != P.level - 1)
                return c->fail(MGFR_EINVAL, "patch %d: parent must be a level-%d patch", p, P.level - 1);
            const mgfr_patch& Q = patches[P.parent];
            for (int d = 0; d < 3; ++d)
                if (P.origin[d] / 2 - 1 < Q.origin[d] || (P.origin[d] + P.n) / 2 > Q.origin[d] + Q.n - 1)
                    return c->fail(MGFR_EINVAL, "patch %d: needs a one-cell margin inside patch %d", p, P.parent);
        }
        const long long n3 = (long long)P.n * P.n * P.n;
        if (P.offset < 0 || P.offset + n3 > packed_cells)
            return c->fail(MGFR_EINVAL, "patch %d: offset outside the packed arrays", p);
        ranges.emplace_back(P.offset, P.offset + n3);
        maxlevel = std::max(maxlevel, P.level);
    }
    std::sort(ranges.begin(), ranges.end());
    for (size_t i = 1; i < ranges.size(); ++i)
        if (ranges[i].first < ranges[i - 1].second) return c->fail(MGFR_EINVAL, "patch blocks overlap in the packed arrays");
    for (int p = 0; p < npatch; ++p)
        for (int q = p + 1; q < npatch; ++q) {
            const mgfr_patch &A = patches[p], &B = patches[q];
            if (A.level != B.level) continue;
            bool sep = false;
            for (int d = 0; d < 3; ++d)
                sep = sep || A.origin[d] + A.n <= B.origin[d] || B.origin[d] + B.n <= A.origin[d];
            if (!sep) return c->fail(MGFR_EINVAL, "patches %d and %d overlap", p, q);
        }
    MGFR_TRY(hip_check(c, hipSetDevice(c->device), "hipSetDevice"));
    hipStream_t s = (hipStream_t)stream;
    int worst = MGFR_OK;
    const int H = o->max_cycles + 1;
    for (int lev = 1; lev <= maxlevel; ++lev) {
        std::vector<int> ids;
        for (int p = 0; p < npatch; ++p)
            if (patches[p].level == lev) ids.push_back(p);
        if (ids.empty()) continue;
        std::vector<Unit> units(ids.size());
        for (size_t i = 0; i < ids.size(); ++i) {
            const mgfr_patch& P = patches[ids[i]];
            Unit& U = units[i];
            U.n = P.n;
            U.periodic = false;
            U.md = md;
            U.h = 1.0 / ((double)N0 * (double)(1 << lev));
            U.u = u_packed + P.offset;
            U.rho = rho_packed + P.offset;
        }
        Batch b{c, o, s, units};
        engine(b);
        MGFR_TRY(b.prepare());
        // boundary set-up: interior initial guess and boundary faces from the parent level
        std::vector<mgfr::PatchParent> parents;
        std::vector<mgfr::BGrid> g0;
        for (size_t i = 0; i < ids.size(); ++i) {
            const mgfr_patch& P = patches[ids[i]];
            mgfr::PatchParent pp{};
            if (P.parent < 0) {
                pp.u = u_domain;
                pp.n = N0;
                pp.periodic = 1;
            } else {
                const mgfr_patch& Q = patches[P.parent];
                pp.u = u_packed + Q.offset;
                pp.n = Q.n;
                pp.periodic = 0;
                for (int d = 0; d < 3; ++d) pp.origin[d] = Q.origin[d];
            }
            pp.lg = ilog2(pp.n);
            for (int d = 0; d < 3; ++d) pp.child[d] = P.origin[d];
            parents.push_back(pp);
            g0.push_back(units[i].g[0]);
        }
        Meta extra;
        extra.bytes = std::move(b.meta_image);
        Launch setup = table(extra, g0, [](const mgfr::BGrid& g) { return 7LL * g.n * g.n; });
        const size_t parents_off = extra.add(parents);
        b.meta_image = std::move(extra.bytes);
        MGFR_TRY(b.upload());
        MGFR_TRY(hip_check(c, mgfr::batch_setup(b.tab(setup), setup.nblk, (const mgfr::PatchParent*)(b.dmeta + parents_off), s),
                           "batch_setup"));
        MGFR_TRY(b.restrict_faces());
        MGFR_TRY(b.check_finite());
        std::vector<double> hist_level(ids.size() * H, 0.0);
        std::vector<int> nh_level(ids.size(), 0);
        int st = MGFR_OK;
        MGFR_TRY(b.phases ? b.run(hist_level.data(), nh_level.data(), &st)
                          : b.run_units(hist_level.data(), nh_level.data(), &st));
        if (st == MGFR_ENONFINITE) worst = st;
        else if (st == MGFR_ENOTCONV && worst == MGFR_OK) worst = st;
        for (size_t i = 0; i < ids.size(); ++i) {
            if (res_hist) std::memcpy(res_hist + (size_t)ids[i] * H, hist_level.data() + i * H, sizeof(double) * H);
            if (n_hist) n_hist[ids[i]] = nh_level[i];
        }
    }
    c->stats.solve_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    if (worst == MGFR_ENONFINITE) return c->fail(worst, "a patch residual became non-finite");
    if (worst == MGFR_ENOTCONV) return c->fail(worst, "some patches did not reach tol in max_cycles");
    return MGFR_OK;
}

int mg_fr_solve_batch(mgfr_ctx* c, int nbox, const int* N, const double* const* rho, const mgfr_params* per_box,
                      const mgfr_opts* o, double* const* u, double* res_hist, int* n_hist, void* stream)
{
    if (!c) return MGFR_EINVAL;
    c->err.clear();
    c->stats = mgfr_stats{};
    const auto t0 = std::chrono::steady_clock::now();
    MGFR_TRY(check_batch_opts(c, o));
    if (nbox < 0 || (nbox > 0 && (!N || !rho || !per_box || !u))) return c->fail(MGFR_EINVAL, "invalid batch arguments");
    if (nbox == 0) return MGFR_OK;
    std::vector<Unit> units(nbox);
    for (int b = 0; b < nbox; ++b) {
        if (!is_pow2(N[b]) || N[b] < o->coarsest_n || N[b] > 1024 || !rho[b] || !u[b])
            return c->fail(MGFR_EINVAL, "box %d: N=%d must be a power of two in [coarsest_n, 1024]", b, N[b]);
        if (derive_model(&per_box[b], &units[b].md) != MGFR_OK)
            return c->fail(MGFR_EINVAL, "box %d: invalid model parameters", b);
        units[b].n = N[b];
        units[b].periodic = true;
        units[b].h = 1.0 / N[b];
        units[b].u = u[b];
        units[b].rho = rho[b];
    }
    MGFR_TRY(hip_check(c, hipSetDevice(c->device), "hipSetDevice"));
    hipStream_t s = (hipStream_t)stream;
    Batch bt{c, o, s, units};
    engine(bt);
    MGFR_TRY(bt.prepare());
    MGFR_TRY(bt.upload());
    if (!(o->flags & MGFR_WARM_START))
        MGFR_TRY(hip_check(c, mgfr::batch_fill(bt.tab(bt.plan.cells0), bt.plan.cells0.nblk, s), "batch_fill"));
    MGFR_TRY(bt.check_finite());
    int st = MGFR_OK;
    MGFR_TRY(bt.phases ? bt.run(res_hist, n_hist, &st) : bt.run_units(res_hist, n_hist, &st));
    c->stats.solve_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    if (st == MGFR_ENONFINITE) return c->fail(st, "a box residual became non-finite");
    if (st == MGFR_ENOTCONV) return c->fail(st, "some boxes did not reach tol in max_cycles");
    return MGFR_OK;
}

}  // extern "C"
