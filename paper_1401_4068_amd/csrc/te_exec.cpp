// te_exec.cpp -- execution paths of libte: the batched surrogate path (one
// persistent search launch per batch, optional hipGraph replay), the plain
// per-window path, and the pre-embedded neighbour-count export.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdlib>
#include <mutex>
#include <cstring>
#include <numeric>
#include <vector>

#include "te.h"
#include "te_internal.h"
#include "te_runtime.h"

namespace te {

int search_occupancy(int d_y, int d_x, int k, int slots, int waves_per_wg);

static int env_int(const char *name, int dflt)
{
    const char *v = std::getenv(name);
    return (v && *v) ? std::atoi(v) : dflt;
}

bool tuned_config(int d_y, int d_x, int k, int64_t n, SearchConfig *out);

// Launch shape of the search kernel for chunks of about n points: the autotuner's
// table entry when there is one (TE_TUNE_FILE names a table loaded on first use),
// else 4 slots, 4 waves per workgroup and full occupancy (the fastest shape measured
// on the nonlinear-ensemble and MEG-like workloads).  TE_SLOTS,
// TE_WAVES_PER_WG and TE_WG_PER_CU override single fields (measurements).
SearchConfig default_config(const DeviceInfo &dev, int d_y, int d_x, int k, int64_t n)
{
    (void)dev;
    static std::once_flag once;
    std::call_once(once, [] {
        const char *f = std::getenv("TE_TUNE_FILE");
        if (f && *f)
            te_tune_load(f);
    });
    SearchConfig c{4, 4, 0};
    SearchConfig t;
    if (tuned_config(d_y, d_x, k, n, &t))
        c = t;
    c.slots = env_int("TE_SLOTS", c.slots);
    if (c.slots != 4 && c.slots != 8 && c.slots != 16)
        c.slots = 4;
    c.waves_per_wg = std::min(kMaxWavesPerWG, std::max(1, env_int("TE_WAVES_PER_WG", c.waves_per_wg)));
    const int occ = search_occupancy(d_y, d_x, k, c.slots, c.waves_per_wg);
    if (c.wg_per_cu <= 0 || c.wg_per_cu > std::max(1, occ))
        c.wg_per_cu = std::max(1, occ);
    c.wg_per_cu = std::max(1, env_int("TE_WG_PER_CU", c.wg_per_cu));
    return c;
}

// Split the full batch into batches whose layout fits ws_bytes; groups (all S+1
// chunks of one (pair, point)) are never split.  Results do not depend on the split.
te_status Plan::split_batches(size_t ws_bytes, std::vector<Batch> *out) const
{
    TraceRange trace_range("te.split_batches");
    const int G = p.n_pairs * p.n_points;
    std::vector<int> cur;
    for (int g = 0; g < G; ++g) {
        std::vector<int> trial = cur;
        trial.push_back(g);
        Batch b;
        build_group_batch(trial, p.n_surrogates, &b);
        if (b.total_bytes <= ws_bytes) {
            cur.swap(trial);
            continue;
        }
        if (cur.empty())
            return fail(TE_ERR_NOMEM, "workspace of %zu bytes cannot hold window group %d (%zu bytes)", ws_bytes, g,
                        b.total_bytes);
        out->emplace_back();
        build_group_batch(cur, p.n_surrogates, &out->back());
        cur.assign(1, g);
    }
    if (!cur.empty()) {
        out->emplace_back();
        build_group_batch(cur, p.n_surrogates, &out->back());
    }
    return TE_OK;
}

te_status Plan::run_surrogates(const float *x, const float *y, const int32_t *perms, char *ws, size_t ws_bytes,
                               hipStream_t st, bool use_graph, double *te_orig, double *te_surr,
                               double *p_value) const
{
    TraceRange trace_range("te.surrogates");
    if (ws_bytes < min_bytes)
        return fail(TE_ERR_NOMEM, "workspace %zu bytes < minimum %zu", ws_bytes, min_bytes);
    hipError_t e;

    if (use_graph) {
        std::lock_guard<std::mutex> lk(graph_mu);
        GraphEntry *ge = nullptr;
        for (auto &g : graphs)
            if (g.x == x && g.y == y && g.perms == perms && g.ws == ws && g.stream == st && g.ws_bytes == ws_bytes)
                ge = &g;
        if (!ge) {
            TraceRange capture_range("te.graph_capture");
            GraphEntry ne;
            ne.x = x;
            ne.y = y;
            ne.perms = perms;
            ne.ws = ws;
            ne.stream = st;
            ne.ws_bytes = ws_bytes;
            if (ws_bytes >= full.total_bytes) {
                ne.batches.push_back(full);
            } else {
                te_status s2 = split_batches(ws_bytes, &ne.batches);
                if (s2 != TE_OK)
                    return s2;
            }
            for (auto &b : ne.batches) {
                void *stg = pool.take(b.stage_bytes());
                if (!stg)
                    return fail(TE_ERR_NOMEM, "pinned staging allocation failed");
                ne.stages.push_back(stg);
            }
            if (st == nullptr)
                return fail(TE_ERR_INVALID, "graph capture needs a non-default stream");
            e = hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal);
            if (e != hipSuccess)
                return hip_fail(e, "hipStreamBeginCapture");
            te_status s2 = TE_OK;
            for (size_t i = 0; i < ne.batches.size() && s2 == TE_OK; ++i)
                s2 = enqueue_batch(ne.batches[i], x, y, perms, ws, ne.stages[i], st);
            hipGraph_t graph = nullptr;
            e = hipStreamEndCapture(st, &graph);
            if (s2 != TE_OK) {
                if (graph)
                    hipGraphDestroy(graph);
                return s2;
            }
            if (e != hipSuccess)
                return hip_fail(e, "hipStreamEndCapture");
            hipGraphExec_t exec = nullptr;
            e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
            if (e != hipSuccess) {
                hipGraphDestroy(graph);
                return hip_fail(e, "hipGraphInstantiate");
            }
            ne.graph = graph;
            ne.exec = exec;
            graphs.push_back(std::move(ne));
            ge = &graphs.back();
        }
        if ((e = hipGraphLaunch(ge->exec, st)) != hipSuccess)
            return hip_fail(e, "hipGraphLaunch");
        {
            TraceRange wait_range("te.wait");
            if ((e = hipStreamSynchronize(st)) != hipSuccess)
                return hip_fail(e, "hipStreamSynchronize");
        }
        bool bad = false;
        for (size_t i = 0; i < ge->batches.size(); ++i)
            unpack_batch(ge->batches[i], ge->stages[i], te_orig, te_surr, p_value, &bad);
        if (bad)
            return fail(TE_ERR_INVALID, "non-finite input value or invalid surrogate permutation");
        return TE_OK;
    }

    std::vector<Batch> local;
    const std::vector<Batch> *batches = &local;
    std::vector<Batch> one;
    if (ws_bytes >= full.total_bytes) {
        one.push_back(full);
        batches = &one;
    } else {
        te_status s2 = split_batches(ws_bytes, &local);
        if (s2 != TE_OK)
            return s2;
    }
    std::vector<void *> stages;
    te_status s = TE_OK;
    for (const Batch &b : *batches) {
        void *stg = pool.take(b.stage_bytes());
        if (!stg) {
            s = fail(TE_ERR_NOMEM, "pinned staging allocation failed");
            break;
        }
        stages.push_back(stg);
        s = enqueue_batch(b, x, y, perms, ws, stg, st);
        if (s != TE_OK)
            break;
    }
    if (s == TE_OK && (e = hipStreamSynchronize(st)) != hipSuccess)
        s = hip_fail(e, "hipStreamSynchronize");
    if (s != TE_OK)
        hipStreamSynchronize(st);           // queued copies may still read the staging buffers
    bool bad = false;
    if (s == TE_OK)
        for (size_t i = 0; i < batches->size(); ++i)
            unpack_batch((*batches)[i], stages[i], te_orig, te_surr, p_value, &bad);
    for (void *stg : stages)
        pool.give(stg);
    if (s == TE_OK && bad)
        s = fail(TE_ERR_INVALID, "non-finite input value or invalid surrogate permutation");
    return s;
}

// The full batch enqueued on the stream with no host round trip: tables from a
// pinned copy that never changes after it is made, results copied to `out`.
te_status Plan::run_surrogates_async(const float *x, const float *y, const int32_t *perms, char *ws,
                                     size_t ws_bytes, hipStream_t st, double *out) const
{
    TraceRange trace_range("te.surrogates_async");
    if (ws_bytes < full.total_bytes)
        return fail(TE_ERR_NOMEM, "te_surrogates_async needs the full workspace (%zu bytes), got %zu",
                    full.total_bytes, ws_bytes);
    const void *tables = nullptr;
    {
        std::lock_guard<std::mutex> lk(async_mu);
        if (!async_tables) {
            void *h = nullptr;
            hipError_t e = hipHostMalloc(&h, std::max<size_t>(full.tables_bytes, 64), hipHostMallocDefault);
            if (e != hipSuccess)
                return hip_fail(e, "hipHostMalloc (tables)");
            std::memcpy(h, full.host_tables.data(), full.tables_bytes);
            async_tables = h;
        }
        tables = async_tables;
    }
    return enqueue_batch(full, x, y, perms, ws, nullptr, st, nullptr, nullptr, tables, out);
}

// Local TE: the originals of every window in one batch, per-point terms written
// through the sort maps to window order.
te_status Plan::run_local(const float *x, const float *y, char *ws, size_t ws_bytes, hipStream_t st, double *lte,
                          double *te_out) const
{
    TraceRange trace_range("te.local");
    const int G = p.n_pairs * p.n_points;
    std::vector<int> all(G);
    std::iota(all.begin(), all.end(), 0);
    Batch b;
    BatchOptions opt;
    opt.local_outputs = true;
    build_group_batch(all, 0, &b, opt);
    if (ws_bytes < b.total_bytes)
        return fail(TE_ERR_NOMEM, "local TE needs a workspace of %zu bytes", b.total_bytes);
    void *stg = pool.take(b.stage_bytes());
    if (!stg)
        return fail(TE_ERR_NOMEM, "pinned staging allocation failed");
    te_status s = enqueue_batch(b, x, y, nullptr, ws, stg, st, lte);
    hipError_t e = hipSuccess;
    if (s == TE_OK && (e = hipStreamSynchronize(st)) != hipSuccess)
        s = hip_fail(e, "hipStreamSynchronize");
    bool bad = false;
    std::vector<double> tmp(G);
    if (s == TE_OK)
        unpack_batch(b, stg, tmp.data(), nullptr, nullptr, &bad);
    pool.give(stg);
    if (s != TE_OK)
        return s;
    if (te_out)
        std::copy(tmp.begin(), tmp.end(), te_out);
    if (bad)
        return fail(TE_ERR_INVALID, "non-finite input value");
    return TE_OK;
}

// Layout of the plain per-chunk path's workspace for n_surr surrogates per window:
// one chunk's coordinates (the target block, then one source block), partial sums,
// results [group][original, surrogates] and p-values, per-launch counters, the
// tables, the window's sort map, its surrogates' permutation rows, sort scratch.
PlainLayout Plan::plain_layout(int n_surr) const
{
    PlainLayout L;
    const int64_t G = (int64_t)p.n_pairs * p.n_points;
    const int D = 1 + p.d_y + p.d_x + p.cond_source;
    const int64_t maxn = *std::max_element(npts.begin(), npts.end());
    const int64_t maxr = *std::max_element(trials.begin(), trials.end());
    const int64_t C = G * (n_surr + 1);
    size_t o = 0;
    L.coords = o;
    o = align_up(o + sizeof(float) * (size_t)maxn * D, 256);
    L.partial = o;
    o = align_up(o + sizeof(double) * (size_t)((maxn + kWave - 1) / kWave), 256);
    L.results = o;
    o = o + sizeof(double) * (size_t)C;
    L.pv = o;
    o = align_up(o + sizeof(double) * (size_t)G, 256);
    L.ctr = o;
    o = align_up(o + sizeof(int32_t) * 4 * (size_t)C + 16, 256);
    L.tables = o;
    L.t_chunks = 0;
    L.t_items = align_up(sizeof(ChunkDesc) * C, 16);
    L.t_tasks = L.t_items + align_up(sizeof(int32_t) * C, 16);
    L.t_sorts = L.t_tasks + align_up(sizeof(EmbedTask) * C, 16);
    L.t_perms = L.t_sorts + align_up(sizeof(SortTask) * G, 16);
    L.tables_bytes = L.t_perms + sizeof(PermTask) * (size_t)G * n_surr;
    o = align_up(o + L.tables_bytes, 256);
    L.sigma = o;
    o = align_up(o + sizeof(int32_t) * (size_t)maxn, 256);
    L.perm = o;
    o = align_up(o + sizeof(int32_t) * (size_t)maxr * n_surr, 256);
    L.scratch = o;
    o = align_up(o + sizeof(uint64_t) * (size_t)sort_npad((int)maxn), 256);
    L.total = o + 4096;
    return L;
}

// Plain path: each (pair, window) on its own and each of its chunks on its own --
// the window sorted once, then per chunk embed, search and reduce (three launches)
// -- in window order on one stream; the estimates, p-values and error words are
// copied back at the end.  n_surr = 0: originals only (te_estimate).
te_status Plan::estimate_each(const float *x, const float *y, const int32_t *perms, int n_surr, char *ws,
                              size_t ws_bytes, hipStream_t st, double *te_orig, double *te_surr,
                              double *p_value) const
{
    TraceRange trace_range("te.estimate_each");
    const PlainLayout L = plain_layout(n_surr);
    if (ws_bytes < L.total)
        return fail(TE_ERR_NOMEM, "workspace %zu bytes < plain-path size %zu", ws_bytes, L.total);
    const int G = p.n_pairs * p.n_points;
    const int S1 = n_surr + 1;
    const int64_t C = (int64_t)G * S1;
    const size_t out_off = align_up(L.tables_bytes, 256);
    const size_t out_bytes = sizeof(double) * (size_t)(C + G) + sizeof(int32_t) * 4 * (size_t)C;
    char *stg = static_cast<char *>(pool.take(out_off + out_bytes));
    if (!stg)
        return fail(TE_ERR_NOMEM, "pinned staging allocation failed");
    ChunkDesc *hc = reinterpret_cast<ChunkDesc *>(stg + L.t_chunks);
    int32_t *hi = reinterpret_cast<int32_t *>(stg + L.t_items);
    EmbedTask *ht = reinterpret_cast<EmbedTask *>(stg + L.t_tasks);
    SortTask *hs = reinterpret_cast<SortTask *>(stg + L.t_sorts);
    PermTask *hp = reinterpret_cast<PermTask *>(stg + L.t_perms);
    const int dT = 1 + p.d_y + p.cond_source;     // x_t, when conditioned on, is the last target-past row
    const bool cond = p.cond_source != 0;
    for (int g = 0; g < G; ++g) {
        const int pair = g / p.n_points, c = g % p.n_points;
        const int N = (int)npts[c];
        SortTask so{};
        so.sig = 0;
        so.npad = sort_npad(N);
        so.scratch = so.npad > kSortLds ? 0 : -1;
        so.key_off = -1;
        so.mode = 0;
        so.pair = pair;
        so.w = wstart[c];
        so.W = wlen[c];
        so.Rc = trials[c];
        so.n = N;
        hs[g] = so;
        for (int s = 0; s < S1; ++s) {
            const int64_t ci = (int64_t)g * S1 + s;
            ChunkDesc d{};
            d.tp = 0;
            d.s = (int64_t)dT * N;
            d.ld = N;
            d.out = -1;
            d.perm = -1;
            d.n = N;
            d.result = (int32_t)ci;
            hc[ci] = d;
            hi[ci] = 0;
            EmbedTask t{};
            // the target block is written with the original and kept for its surrogates
            // (with x_t conditioned on, every chunk writes its own: x_t follows the shuffle)
            t.tp = (s == 0 || cond) ? 0 : -1;
            t.s = (int64_t)dT * N;
            t.perm = -1;
            t.sig = sorted ? 0 : -1;
            t.pair = pair;
            t.w = wstart[c];
            t.W = wlen[c];
            t.Rc = trials[c];
            t.n = N;
            if (s > 0) {
                PermTask pt{};
                pt.src = (((int64_t)pair * p.n_points + c) * n_surr + (s - 1)) * p.n_trials;
                pt.dst = (int64_t)(s - 1) * trials[c];
                pt.rc = trials[c];
                pt.len = trials[c];
                pt.pair = pair;
                pt.point = c;
                pt.surr = s - 1;
                hp[(int64_t)g * n_surr + (s - 1)] = pt;
                t.perm = pt.dst;
            }
            ht[ci] = t;
        }
    }
    hipError_t e = hipMemcpyAsync(ws + L.tables, stg, L.tables_bytes, hipMemcpyHostToDevice, st);
    int32_t *ctr = reinterpret_cast<int32_t *>(ws + L.ctr);
    if (e == hipSuccess)
        e = launch_fill_i32(ctr, 0, 4 * C, st);
    float *base = reinterpret_cast<float *>(ws + L.coords);
    double *partial = reinterpret_cast<double *>(ws + L.partial);
    double *res = reinterpret_cast<double *>(ws + L.results);
    double *pv = reinterpret_cast<double *>(ws + L.pv);
    const ChunkDesc *dc = reinterpret_cast<const ChunkDesc *>(ws + L.tables + L.t_chunks);
    const int32_t *di = reinterpret_cast<const int32_t *>(ws + L.tables + L.t_items);
    const EmbedTask *dt = reinterpret_cast<const EmbedTask *>(ws + L.tables + L.t_tasks);
    const SortTask *ds = reinterpret_cast<const SortTask *>(ws + L.tables + L.t_sorts);
    const PermTask *dp = reinterpret_cast<const PermTask *>(ws + L.tables + L.t_perms);
    int32_t *sigma = reinterpret_cast<int32_t *>(ws + L.sigma);
    int32_t *parea = reinterpret_cast<int32_t *>(ws + L.perm);
    uint64_t *scratch = reinterpret_cast<uint64_t *>(ws + L.scratch);
    for (int g = 0; g < G && e == hipSuccess; ++g) {
        const int c = g % p.n_points;
        const int64_t items = (npts[c] + kWave - 1) / kWave;
        int32_t *gerr = ctr + 4 * (int64_t)g * S1 + 1;   // the window's error word: its original's
        if (sorted && (e = launch_sort(y, nullptr, ds + g, 1, sigma, scratch, p.n_trials, p.n_samples, st)) !=
                          hipSuccess)
            break;
        if (n_surr > 0 &&
            (e = launch_perms(perms, dp + (int64_t)g * n_surr, n_surr, parea, p.seed, gerr, st)) != hipSuccess)
            break;
        for (int s = 0; s < S1 && e == hipSuccess; ++s) {
            const int64_t ci = (int64_t)g * S1 + s;
            e = launch_embed(x, y, parea, sigma, nullptr, dt + ci, 1, (int)npts[c], base, p.n_trials, p.n_samples,
                             p.d_y, p.d_x, p.tau, p.u, p.cond_source, gerr, st);
            if (e != hipSuccess)
                break;
            SearchArgs a{};
            a.base = base;
            a.chunks = dc + ci;
            a.item_start = di + ci;
            a.n_chunks = 1;
            a.n_items = (int32_t)items;
            a.k = p.k;
            a.counter = ctr + 4 * ci;
            a.partial = partial;
            a.sorted = sorted ? 1 : 0;
            e = launch_search_timed(a, dy_eff(), p.d_x, cfg, grid_waves(items), st);
            if (e == hipSuccess)
                e = launch_reduce(dc + ci, 1, partial, p.k, gerr, res, st);
        }
    }
    if (e == hipSuccess && n_surr > 0)
        e = launch_pvalues(res, G, n_surr, pv, st);
    if (e == hipSuccess)
        e = hipMemcpyAsync(stg + out_off, res, sizeof(double) * (size_t)(C + G), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess)
        e = hipMemcpyAsync(stg + out_off + sizeof(double) * (C + G), ctr, sizeof(int32_t) * 4 * C,
                           hipMemcpyDeviceToHost, st);
    if (e == hipSuccess)
        e = hipStreamSynchronize(st);
    if (e != hipSuccess) {
        hipStreamSynchronize(st);
        pool.give(stg);
        return hip_fail(e, "plain path");
    }
    const double *hr = reinterpret_cast<const double *>(stg + out_off);
    const int32_t *errs = reinterpret_cast<const int32_t *>(stg + out_off + sizeof(double) * (C + G));
    bool bad = false;
    for (int g = 0; g < G; ++g) {
        bad |= errs[4 * (int64_t)g * S1 + 1] != 0;
        if (te_orig)
            te_orig[g] = hr[(int64_t)g * S1];
        if (te_surr)
            for (int s = 0; s < n_surr; ++s)
                te_surr[(int64_t)g * n_surr + s] = hr[(int64_t)g * S1 + 1 + s];
        if (p_value)
            p_value[g] = n_surr > 0 ? hr[C + g] : __builtin_nan("");
    }
    pool.give(stg);
    if (bad)
        return fail(TE_ERR_INVALID, "non-finite input value or invalid surrogate permutation");
    return TE_OK;
}

static PinnedPool g_knn_pool;

}  // namespace te

using namespace te;

extern "C" {

size_t te_knn_counts_workspace_bytes(int32_t n_chunks, int64_t n_points_total)
{
    if (n_chunks < 1 || n_points_total < 0)
        return 0;
    const size_t items = (size_t)(n_points_total / kWave + n_chunks + 1);
    // sorted copy of the points (up to 9 coordinates), maps, sort scratch (bounded by 2x points rounded up)
    const size_t copy = align_up(sizeof(float) * (size_t)n_points_total * (1 + kMaxDimY + kMaxDimX), 256);
    const size_t maps = align_up(sizeof(int32_t) * (size_t)n_points_total, 256);
    const size_t scratch = align_up(sizeof(uint64_t) * (2 * (size_t)n_points_total + (size_t)n_chunks), 256);
    const size_t tables = align_up((sizeof(ChunkDesc) + sizeof(int32_t) + sizeof(SortTask) + sizeof(GatherTask)) *
                                   (size_t)n_chunks + 64, 256);
    return tables + align_up(sizeof(double) * items, 256) + align_up(sizeof(double) * n_chunks, 256) + 256 + copy +
           maps + scratch + 256;
}

te_status te_knn_counts(const float *pts, int64_t dim_stride, const int64_t *offsets, int32_t n_chunks, int32_t d_y,
                        int32_t d_x, int32_t k, void *ws_, size_t ws_bytes, void *hip_stream, float *eps,
                        int32_t *counts, double *te_out)
{
    TraceRange trace_range("te.knn_counts");
    clear_error();
    if (!ws_)
        return fail(TE_ERR_INVALID, "null argument");
    return knn_counts_run(pts, dim_stride, offsets, n_chunks, d_y, d_x, k, static_cast<char *>(ws_), ws_bytes,
                          (hipStream_t)hip_stream, eps, counts, te_out, true, "workspace");
}

}  // extern "C"

namespace te {

// Body of te_knn_counts and te_knn_counts_noalloc.  ws: device scratch of ws_bytes
// (the caller's workspace, or the library's static scratch array).  pinned_staging:
// upload the tables and download the estimates through the pinned staging pool
// (which may allocate pinned host memory on first use); false: through ordinary
// host memory, so the call allocates no device or pinned memory.  ws_name names the
// scratch in the TE_ERR_NOMEM message.
te_status knn_counts_run(const float *pts, int64_t dim_stride, const int64_t *offsets, int32_t n_chunks, int32_t d_y,
                         int32_t d_x, int32_t k, char *ws, size_t ws_bytes, hipStream_t st, float *eps,
                         int32_t *counts, double *te_out, bool pinned_staging, const char *ws_name)
{
    if (!pts || !offsets || !ws || !eps || !counts)
        return fail(TE_ERR_INVALID, "null argument");
    if (n_chunks < 1)
        return fail(TE_ERR_INVALID, "n_chunks must be >= 1");
    if (d_y < 1 || d_y > kMaxDimY || d_x < 1 || d_x > kMaxDimX || k < 1 || k > kMaxK)
        return fail(TE_ERR_INVALID, "unsupported d_y=%d d_x=%d k=%d", d_y, d_x, k);
    const int64_t total = offsets[n_chunks];
    if (offsets[0] != 0 || total > dim_stride)
        return fail(TE_ERR_INVALID, "offsets must start at 0 and end at or below dim_stride");
    const int D = 1 + d_y + d_x;
    const bool sorted = sorting_enabled();
    int64_t items = 0, n_scratch = 0;
    std::vector<ChunkDesc> chunks(n_chunks);
    std::vector<SortTask> sorts(n_chunks);
    std::vector<GatherTask> gathers(n_chunks);
    for (int c = 0; c < n_chunks; ++c) {
        const int64_t n = offsets[c + 1] - offsets[c];
        if (n <= k || n > (1 << 30))
            return fail(TE_ERR_INVALID, "chunk %d has %lld points; need k < n <= 2^30", c, (long long)n);
        ChunkDesc d{};
        if (sorted) {
            // searched in a sorted copy: coordinate m of sorted point q at copy[offsets[c] * D + m * n + q]
            d.tp = offsets[c] * D;
            d.s = offsets[c] * D + (int64_t)(1 + d_y) * n;
            d.ld = n;
            d.perm = offsets[c];
        } else {
            d.tp = offsets[c];
            d.s = offsets[c] + (int64_t)(1 + d_y) * dim_stride;
            d.ld = dim_stride;
            d.perm = -1;
        }
        d.out = offsets[c];
        d.n = (int32_t)n;
        d.result = c;
        chunks[c] = d;
        SortTask so{};
        so.sig = offsets[c];
        so.npad = sort_npad((int)n);
        so.scratch = -1;
        if (so.npad > kSortLds) {
            so.scratch = n_scratch;
            n_scratch += so.npad;
        }
        so.key_off = offsets[c] + dim_stride;        // coordinate 1: first target-past coordinate
        so.mode = 1;
        so.n = (int32_t)n;
        sorts[c] = so;
        GatherTask gt{};
        gt.src = offsets[c];
        gt.ld = dim_stride;
        gt.dst = offsets[c] * D;
        gt.sig = offsets[c];
        gt.n = (int32_t)n;
        gathers[c] = gt;
    }
    // longest first
    std::vector<int> order(n_chunks);
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return chunks[a].n > chunks[b].n; });
    std::vector<ChunkDesc> sorted_chunks(n_chunks);
    std::vector<int32_t> starts(n_chunks);
    for (int i = 0; i < n_chunks; ++i) {
        sorted_chunks[i] = chunks[order[i]];
        sorted_chunks[i].item0 = (int32_t)items;
        sorted_chunks[i].block0 = 0;
        sorted_chunks[i].pbase = items;
        starts[i] = (int32_t)items;
        items += (sorted_chunks[i].n + kWave - 1) / kWave;
    }
    DeviceInfo dev;
    te_status s = current_device(&dev);
    if (s != TE_OK)
        return s;
    SearchConfig cfg = default_config(dev, d_y, d_x, k, total / n_chunks);
    size_t o = 0;
    const size_t off_chunks = o;
    o = align_up(o + sizeof(ChunkDesc) * n_chunks, 16);
    const size_t off_items = o;
    o = align_up(o + sizeof(int32_t) * n_chunks, 16);
    const size_t off_sorts = o;
    o = align_up(o + sizeof(SortTask) * n_chunks, 16);
    const size_t off_gathers = o;
    o = align_up(o + sizeof(GatherTask) * n_chunks, 256);
    const size_t tbytes = o;
    const size_t off_partial = o;
    o = align_up(o + sizeof(double) * (size_t)items, 256);
    const size_t off_results = o;
    o = align_up(o + sizeof(double) * n_chunks, 256);
    const size_t off_ctr = o;
    o += 256;
    const size_t off_copy = o;
    o = align_up(o + (sorted ? sizeof(float) * (size_t)total * D : 0), 256);
    const size_t off_sigma = o;
    o = align_up(o + (sorted ? sizeof(int32_t) * (size_t)total : 0), 256);
    const size_t off_scratch = o;
    o = align_up(o + (sorted ? sizeof(uint64_t) * (size_t)n_scratch : 0), 256);
    if (ws_bytes < o)
        return fail(TE_ERR_NOMEM, "%s too small (%zu < %zu bytes)", ws_name, ws_bytes, o);
    const size_t out_off = align_up(tbytes, 256);
    const size_t stg_bytes = out_off + sizeof(double) * n_chunks + 64;
    std::vector<char> host_stage;
    char *stg;
    if (pinned_staging) {
        stg = static_cast<char *>(g_knn_pool.take(stg_bytes));
        if (!stg)
            return fail(TE_ERR_NOMEM, "pinned staging allocation failed");
    } else {
        host_stage.resize(stg_bytes);
        stg = host_stage.data();
    }
    std::memcpy(stg + off_chunks, sorted_chunks.data(), sizeof(ChunkDesc) * n_chunks);
    std::memcpy(stg + off_items, starts.data(), sizeof(int32_t) * n_chunks);
    std::memcpy(stg + off_sorts, sorts.data(), sizeof(SortTask) * n_chunks);
    std::memcpy(stg + off_gathers, gathers.data(), sizeof(GatherTask) * n_chunks);
    hipError_t e = hipMemcpyAsync(ws, stg, tbytes, hipMemcpyHostToDevice, st);
    int32_t *ctr = reinterpret_cast<int32_t *>(ws + off_ctr);
    int32_t *sigma = reinterpret_cast<int32_t *>(ws + off_sigma);
    if (e == hipSuccess)
        e = launch_fill_i32(ctr, 0, 4, st);
    if (e == hipSuccess && sorted)
        e = launch_sort(nullptr, pts, reinterpret_cast<const SortTask *>(ws + off_sorts), n_chunks, sigma,
                        reinterpret_cast<uint64_t *>(ws + off_scratch), 0, 0, st);
    if (e == hipSuccess && sorted)
        e = launch_gather(pts, reinterpret_cast<const GatherTask *>(ws + off_gathers), n_chunks, sigma,
                          reinterpret_cast<float *>(ws + off_copy), D, st);
    SearchArgs a{};
    a.base = sorted ? reinterpret_cast<const float *>(ws + off_copy) : pts;
    a.chunks = reinterpret_cast<const ChunkDesc *>(ws + off_chunks);
    a.item_start = reinterpret_cast<const int32_t *>(ws + off_items);
    a.n_chunks = n_chunks;
    a.n_items = (int32_t)items;
    a.k = k;
    a.counter = ctr;
    a.partial = reinterpret_cast<double *>(ws + off_partial);
    a.eps_out = eps;
    a.cnt_out = counts;
    a.cnt_stride = total;
    a.perm_base = sigma;
    a.sorted = sorted ? 1 : 0;
    if (e == hipSuccess) {
        const int64_t full = (int64_t)dev.n_cu * cfg.wg_per_cu * cfg.waves_per_wg;
        e = launch_search_timed(a, d_y, d_x, cfg, (int)std::max<int64_t>(1, std::min<int64_t>(full, items)), st);
    }
    double *res = reinterpret_cast<double *>(ws + off_results);
    if (e == hipSuccess)
        e = launch_reduce(a.chunks, n_chunks, a.partial, k, ctr + 1, res, st);
    if (e == hipSuccess && te_out)
        e = hipMemcpyAsync(stg + out_off, res, sizeof(double) * n_chunks, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess)
        e = hipStreamSynchronize(st);
    if (e == hipSuccess && te_out)
        std::memcpy(te_out, stg + out_off, sizeof(double) * n_chunks);
    if (pinned_staging)
        g_knn_pool.give(stg);
    if (e != hipSuccess)
        return hip_fail(e, "te_knn_counts");
    return TE_OK;
}

}  // namespace te
