// te_tune.cpp -- autotuner for the search kernel's launch shape.
//
// A shape is (candidate slots per lane in the counting pass, waves per
// workgroup, resident workgroups per CU).  te_autotune times every shape on
// synthetic chunks of the requested (d_y, d_x, k, N) generated on the device,
// keeps the fastest in a process-wide table keyed by (d_y, d_x, k, N bucket),
// and default_config() consults that table.  te_tune_save / te_tune_load keep
// the table in a text file ("d_y d_x k n_bucket slots waves wg_per_cu ms" per line).

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <tuple>
#include <vector>

#include "te.h"
#include "te_internal.h"
#include "te_runtime.h"

namespace te {

int search_occupancy(int d_y, int d_x, int k, int slots, int waves_per_wg);
hipError_t launch_fill_uniform(float *p, int64_t n, uint64_t seed, hipStream_t st);

namespace {

struct TuneKey {
    int d_y, d_x, k, bucket;
    bool operator<(const TuneKey &o) const
    {
        return std::tie(d_y, d_x, k, bucket) < std::tie(o.d_y, o.d_x, o.k, o.bucket);
    }
};

struct TuneVal {
    SearchConfig cfg;
    double ms;
};

std::mutex g_mu;
std::map<TuneKey, TuneVal> g_table;

}  // namespace

// Chunk-size bucket: floor(log2(N)), so 1000..1023 -> 9, 5000 -> 12, 50000 -> 15.
int size_bucket(int64_t n)
{
    int b = 0;
    while (n > 1) {
        n >>= 1;
        ++b;
    }
    return b;
}

bool tuned_config(int d_y, int d_x, int k, int64_t n, SearchConfig *out)
{
    std::lock_guard<std::mutex> lk(g_mu);
    if (g_table.empty())
        return false;
    const int b = size_bucket(n);
    const TuneVal *best = nullptr;
    int bestd = 1 << 30;
    for (auto &kv : g_table) {
        const TuneKey &key = kv.first;
        if (key.d_y != d_y || key.d_x != d_x || key.k != k)
            continue;
        const int d = std::abs(key.bucket - b);
        if (d < bestd) {
            bestd = d;
            best = &kv.second;
        }
    }
    if (!best || bestd > 2)
        return false;
    *out = best->cfg;
    return true;
}

}  // namespace te

using namespace te;

extern "C" {

te_status te_autotune(int32_t d_y, int32_t d_x, int32_t k, int32_t n_points, int32_t n_chunks, void *ws_,
                      size_t ws_bytes, void *hip_stream, int32_t *slots, int32_t *waves_per_wg,
                      int32_t *wg_per_cu, double *best_ms)
{
    TraceRange trace_range("te.autotune");
    clear_error();
    if (d_y < 1 || d_y > kMaxDimY || d_x < 1 || d_x > kMaxDimX || k < 1 || k > kMaxK || n_points <= k ||
        n_chunks < 1 || !ws_)
        return fail(TE_ERR_INVALID, "bad tuning problem");
    const int D = 1 + d_y + d_x;
    const int64_t total = (int64_t)n_points * n_chunks;
    const int64_t items = (int64_t)n_chunks * ((n_points + kWave - 1) / kWave);
    const bool sorted = sorting_enabled();
    const int npad = sort_npad(n_points);
    const int64_t n_scratch = npad > kSortLds ? (int64_t)npad * n_chunks : 0;
    size_t o = 0;
    const size_t off_raw = o;                       // uniform random coordinates, [D][total]
    o = align_up(o + sizeof(float) * (size_t)total * D, 256);
    const size_t off_pts = o;                       // the same chunks sorted by coordinate 1, [chunk][D][n]
    o = align_up(o + sizeof(float) * (size_t)total * D, 256);
    const size_t off_chunks = o;
    o = align_up(o + sizeof(ChunkDesc) * n_chunks, 256);
    const size_t off_items = o;
    o = align_up(o + sizeof(int32_t) * n_chunks, 256);
    const size_t off_sorts = o;
    o = align_up(o + sizeof(SortTask) * n_chunks, 256);
    const size_t off_gathers = o;
    o = align_up(o + sizeof(GatherTask) * n_chunks, 256);
    const size_t off_sigma = o;
    o = align_up(o + sizeof(int32_t) * (size_t)total, 256);
    const size_t off_scratch = o;
    o = align_up(o + sizeof(uint64_t) * (size_t)n_scratch, 256);
    const size_t off_partial = o;
    o = align_up(o + sizeof(double) * (size_t)items, 256);
    const size_t off_ctr = o;
    o += 256;
    if (ws_bytes < o)
        return fail(TE_ERR_NOMEM, "tuning workspace needs %zu bytes", o);
    DeviceInfo dev;
    te_status s = current_device(&dev);
    if (s != TE_OK)
        return s;
    char *ws = static_cast<char *>(ws_);
    hipStream_t st = (hipStream_t)hip_stream;
    std::vector<ChunkDesc> cd(n_chunks);
    std::vector<int32_t> starts(n_chunks);
    std::vector<SortTask> sorts(n_chunks);
    std::vector<GatherTask> gathers(n_chunks);
    for (int c = 0; c < n_chunks; ++c) {
        ChunkDesc d{};
        if (sorted) {
            d.tp = (int64_t)c * n_points * D;
            d.s = d.tp + (int64_t)(1 + d_y) * n_points;
            d.ld = n_points;
        } else {
            d.tp = (int64_t)c * n_points;
            d.s = (int64_t)c * n_points + (int64_t)(1 + d_y) * total;
            d.ld = total;
        }
        d.out = -1;
        d.perm = -1;
        d.n = n_points;
        d.item0 = (int32_t)((int64_t)c * ((n_points + kWave - 1) / kWave));
        d.pbase = d.item0;
        d.block0 = 0;
        d.result = c;
        cd[c] = d;
        starts[c] = d.item0;
        SortTask so{};
        so.sig = (int64_t)c * n_points;
        so.npad = npad;
        so.scratch = npad > kSortLds ? (int64_t)c * npad : -1;
        so.key_off = (int64_t)c * n_points + total;  // coordinate 1
        so.mode = 1;
        so.n = n_points;
        sorts[c] = so;
        GatherTask g{};
        g.src = (int64_t)c * n_points;
        g.ld = total;
        g.dst = (int64_t)c * n_points * D;
        g.sig = (int64_t)c * n_points;
        g.n = n_points;
        gathers[c] = g;
    }
    hipError_t e = hipMemcpy(ws + off_chunks, cd.data(), sizeof(ChunkDesc) * n_chunks, hipMemcpyHostToDevice);
    if (e == hipSuccess)
        e = hipMemcpy(ws + off_items, starts.data(), sizeof(int32_t) * n_chunks, hipMemcpyHostToDevice);
    if (e == hipSuccess)
        e = hipMemcpy(ws + off_sorts, sorts.data(), sizeof(SortTask) * n_chunks, hipMemcpyHostToDevice);
    if (e == hipSuccess)
        e = hipMemcpy(ws + off_gathers, gathers.data(), sizeof(GatherTask) * n_chunks, hipMemcpyHostToDevice);
    float *raw = reinterpret_cast<float *>(ws + off_raw);
    if (e == hipSuccess)
        e = launch_fill_uniform(raw, total * D, 0x7e5eed, st);
    if (e == hipSuccess && sorted)
        e = launch_sort(nullptr, raw, reinterpret_cast<const SortTask *>(ws + off_sorts), n_chunks,
                        reinterpret_cast<int32_t *>(ws + off_sigma), reinterpret_cast<uint64_t *>(ws + off_scratch), 0,
                        0, st);
    if (e == hipSuccess && sorted)
        e = launch_gather(raw, reinterpret_cast<const GatherTask *>(ws + off_gathers), n_chunks,
                          reinterpret_cast<const int32_t *>(ws + off_sigma), reinterpret_cast<float *>(ws + off_pts), D,
                          st);
    if (e == hipSuccess)
        e = hipStreamSynchronize(st);
    if (e != hipSuccess)
        return hip_fail(e, "tuning setup");
    SearchArgs a{};
    a.base = reinterpret_cast<const float *>(ws + (sorted ? off_pts : off_raw));
    a.sorted = sorted ? 1 : 0;
    a.chunks = reinterpret_cast<const ChunkDesc *>(ws + off_chunks);
    a.item_start = reinterpret_cast<const int32_t *>(ws + off_items);
    a.n_chunks = n_chunks;
    a.n_items = (int32_t)items;
    a.k = k;
    a.counter = reinterpret_cast<int32_t *>(ws + off_ctr);
    a.partial = reinterpret_cast<double *>(ws + off_partial);
    hipEvent_t e0, e1;
    hipEventCreate(&e0);
    hipEventCreate(&e1);
    SearchConfig best{};
    double best_t = 1e30;
    const int slot_set[] = {4, 8, 16};
    const int wpg_set[] = {1, 2, 4};
    for (int sl : slot_set)
        for (int wpg : wpg_set) {
            const int occ = search_occupancy(d_y, d_x, k, sl, wpg);
            if (occ < 1)
                continue;
            // every occupancy from full down to half, in whole waves per SIMD: a
            // batch with few work items per wave ends sooner when its longest items
            // share their SIMD with fewer waves
            const int per_level = std::max(1, 4 / wpg);   // workgroups per wave per SIMD
            const int levels = occ / per_level;
            std::vector<int> wgs = {occ};
            for (int w = levels; w >= 1 && 2 * w >= levels; --w)
                if (std::find(wgs.begin(), wgs.end(), w * per_level) == wgs.end())
                    wgs.push_back(w * per_level);
            for (int wg : wgs) {
                SearchConfig c{sl, wpg, wg};
                double tmin = 1e30;
                for (int rep = 0; rep < 5 && e == hipSuccess; ++rep) {
                    e = launch_fill_i32(a.counter, 0, 1, st);
                    if (e == hipSuccess)
                        e = hipEventRecord(e0, st);
                    const int64_t full = (int64_t)dev.n_cu * wg * wpg;
                    if (e == hipSuccess)
                        e = launch_search(a, d_y, d_x, c, (int)std::max<int64_t>(1, std::min<int64_t>(full, items)), st);
                    if (e == hipSuccess)
                        e = hipEventRecord(e1, st);
                    if (e == hipSuccess)
                        e = hipEventSynchronize(e1);
                    float ms = 0;
                    if (e == hipSuccess)
                        hipEventElapsedTime(&ms, e0, e1);
                    tmin = std::min(tmin, (double)ms);
                }
                if (e != hipSuccess)
                    break;
                if (tmin < best_t) {
                    best_t = tmin;
                    best = c;
                }
            }
        }
    hipEventDestroy(e0);
    hipEventDestroy(e1);
    if (e != hipSuccess)
        return hip_fail(e, "tuning run");
    {
        std::lock_guard<std::mutex> lk(g_mu);
        g_table[TuneKey{d_y, d_x, k, size_bucket(n_points)}] = TuneVal{best, best_t};
    }
    if (slots)
        *slots = best.slots;
    if (waves_per_wg)
        *waves_per_wg = best.waves_per_wg;
    if (wg_per_cu)
        *wg_per_cu = best.wg_per_cu;
    if (best_ms)
        *best_ms = best_t;
    return TE_OK;
}

// Tuning on a plan's own data: the shapes of te_autotune, each timed on a batch
// of the plan's largest window groups (originals and surrogates, longest first)
// holding at least four items per resident wave of the widest shape, or as many
// groups as the workspace takes.  The fastest shape becomes the plan's and is
// recorded in the table under the plan's median chunk size.
te_status te_plan_autotune(te_plan plan, const float *x, const float *y, const int32_t *perms, void *ws_,
                           size_t ws_bytes, void *hip_stream, int32_t *slots, int32_t *waves_per_wg,
                           int32_t *wg_per_cu, double *best_ms)
{
    TraceRange trace_range("te.plan_autotune");
    clear_error();
    if (!plan || !x || !y || !ws_)
        return fail(TE_ERR_INVALID, "null argument");
    const Plan &P = plan->impl;
    te_status s = P.ensure_device();
    if (s != TE_OK)
        return s;
    char *ws = static_cast<char *>(ws_);
    hipStream_t st = (hipStream_t)hip_stream;
    const int G = P.p.n_pairs * P.p.n_points;
    std::vector<int> order(G);
    for (int g = 0; g < G; ++g)
        order[g] = g;
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
        return P.npts[a % P.p.n_points] > P.npts[b % P.p.n_points];
    });
    // at least 16 items per wave at full occupancy (or the whole batch): with fewer,
    // the subset's tail favours lower occupancies than the full batch wants
    const int64_t want_items = (int64_t)16 * P.dev.n_cu * 32;
    std::vector<int> groups;
    Batch b;
    for (int g : order) {
        std::vector<int> trial = groups;
        trial.push_back(g);
        Batch t;
        P.build_group_batch(trial, P.p.n_surrogates, &t);
        if (t.total_bytes > ws_bytes)
            break;
        groups.swap(trial);
        b = std::move(t);
        if (b.n_partials >= want_items)
            break;
    }
    if (groups.empty())
        return fail(TE_ERR_NOMEM, "workspace of %zu bytes cannot hold one window group", ws_bytes);
    void *stg = P.pool.take(b.stage_bytes());
    if (!stg)
        return fail(TE_ERR_NOMEM, "pinned staging allocation failed");
    hipEvent_t e0, e1;
    hipEventCreate(&e0);
    hipEventCreate(&e1);
    const SearchConfig saved = P.cfg;
    SearchConfig best = saved;
    double best_t = 1e30;
    hipError_t e = hipSuccess;
    const int slot_set[] = {4, 8, 16};
    const int wpg_set[] = {1, 2, 4};
    for (int sl : slot_set)
        for (int wpg : wpg_set) {
            if (b.use_sets && sl == 16)                  // the chunk-set search runs 16 slots as 8
                continue;
            const int occ = b.use_sets ? search_sets_occupancy(P.dy_eff(), P.p.d_x, sl, wpg)
                                       : search_occupancy(P.dy_eff(), P.p.d_x, P.p.k, sl, wpg);
            if (occ < 1)
                continue;
            // every occupancy from full down to half, in whole waves per SIMD: a
            // batch with few work items per wave ends sooner when its longest items
            // share their SIMD with fewer waves
            const int per_level = std::max(1, 4 / wpg);   // workgroups per wave per SIMD
            const int levels = occ / per_level;
            std::vector<int> wgs = {occ};
            for (int w = levels; w >= 1 && 2 * w >= levels; --w)
                if (std::find(wgs.begin(), wgs.end(), w * per_level) == wgs.end())
                    wgs.push_back(w * per_level);
            for (int wg : wgs) {
                P.cfg = SearchConfig{sl, wpg, wg};
                double tmin = 1e30;
                for (int rep = 0; rep < 5 && s == TE_OK && e == hipSuccess; ++rep) {
                    if (rep == 3 && tmin > 20.0)             // long runs: one warm-up and two timed
                        break;
                    e = hipEventRecord(e0, st);
                    if (e == hipSuccess)
                        s = P.enqueue_batch(b, x, y, perms, ws, stg, st);
                    if (s == TE_OK && e == hipSuccess)
                        e = hipEventRecord(e1, st);
                    if (s == TE_OK && e == hipSuccess)
                        e = hipEventSynchronize(e1);
                    float ms = 0;
                    if (s == TE_OK && e == hipSuccess)
                        hipEventElapsedTime(&ms, e0, e1);
                    if (rep > 0)                     // the first run of a shape warms it up
                        tmin = std::min(tmin, (double)ms);
                }
                if (s != TE_OK || e != hipSuccess)
                    break;
                if (tmin < best_t) {
                    best_t = tmin;
                    best = P.cfg;
                }
            }
        }
    hipEventDestroy(e0);
    hipEventDestroy(e1);
    P.pool.give(stg);
    P.cfg = (s == TE_OK && e == hipSuccess) ? best : saved;
    if (s != TE_OK)
        return s;
    if (e != hipSuccess)
        return hip_fail(e, "tuning run");
    {
        std::vector<int64_t> ns(P.npts);
        std::nth_element(ns.begin(), ns.begin() + ns.size() / 2, ns.end());
        std::lock_guard<std::mutex> lk(g_mu);
        g_table[TuneKey{P.dy_eff(), P.p.d_x, P.p.k, size_bucket(ns[ns.size() / 2])}] = TuneVal{best, best_t};
    }
    if (slots)
        *slots = best.slots;
    if (waves_per_wg)
        *waves_per_wg = best.waves_per_wg;
    if (wg_per_cu)
        *wg_per_cu = best.wg_per_cu;
    if (best_ms)
        *best_ms = best_t;
    return TE_OK;
}

te_status te_tune_save(const char *path)
{
    clear_error();
    FILE *f = path ? std::fopen(path, "w") : nullptr;
    if (!f)
        return fail(TE_ERR_INVALID, "cannot write %s", path ? path : "(null)");
    std::lock_guard<std::mutex> lk(g_mu);
    for (auto &kv : g_table)
        std::fprintf(f, "%d %d %d %d %d %d %d %.6f\n", kv.first.d_y, kv.first.d_x, kv.first.k, kv.first.bucket,
                     kv.second.cfg.slots, kv.second.cfg.waves_per_wg, kv.second.cfg.wg_per_cu, kv.second.ms);
    std::fclose(f);
    return TE_OK;
}

te_status te_tune_load(const char *path)
{
    clear_error();
    FILE *f = path ? std::fopen(path, "r") : nullptr;
    if (!f)
        return fail(TE_ERR_INVALID, "cannot read %s", path ? path : "(null)");
    int a, b, c, d, sl, w, g;
    double ms;
    int n = 0;
    std::lock_guard<std::mutex> lk(g_mu);
    while (std::fscanf(f, "%d %d %d %d %d %d %d %lf", &a, &b, &c, &d, &sl, &w, &g, &ms) == 8) {
        if (a < 1 || a > kMaxDimY || b < 1 || b > kMaxDimX || c < 1 || c > kMaxK || !search_supported(a, b, c, sl) ||
            w < 1 || w > kMaxWavesPerWG || g < 1)
            continue;
        g_table[TuneKey{a, b, c, d}] = TuneVal{SearchConfig{sl, w, g}, ms};
        ++n;
    }
    std::fclose(f);
    return n > 0 ? TE_OK : fail(TE_ERR_INVALID, "no tuning entries in %s", path);
}

te_status te_tune_clear(void)
{
    std::lock_guard<std::mutex> lk(g_mu);
    g_table.clear();
    return TE_OK;
}

}  // extern "C"
