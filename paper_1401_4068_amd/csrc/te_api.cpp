// te_api.cpp -- host runtime and C interface of libte.
//
// A plan fixes the geometry of one analysis job (Wollstadt et al. 2014:
// eq. 10 windows, embedding of eq. 6-7, S surrogates per window).  A batch is
// a set of chunks (search spaces) laid out in the caller's device workspace:
//   coordinates | chunk table | item starts | embed tasks | permutation rows |
//   per-item partial sums | per-chunk results | p-values | counters
// The tables are built on the host, uploaded with one copy, and consumed by
// the embed, search, reduce and p-value kernels on the caller's stream.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <memory>
#include <mutex>
#include <numeric>
#include <string>
#include <vector>

#include "te.h"
#include "te_internal.h"
#include "te_runtime.h"

namespace te {

// ------------------------------------------------------------------ errors

static thread_local std::string g_last_error;

te_status fail(te_status st, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return st;
}

te_status hip_fail(hipError_t e, const char *what)
{
    return fail(TE_ERR_DEVICE, "%s: %s", what, hipGetErrorString(e));
}

void clear_error() { g_last_error.clear(); }

// ------------------------------------------------------------------ device

static std::mutex g_dev_mu;
static std::vector<DeviceInfo> g_devs;

te_status current_device(DeviceInfo *out)
{
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess)
        return hip_fail(e, "hipGetDevice");
    std::lock_guard<std::mutex> lk(g_dev_mu);
    for (auto &d : g_devs)
        if (d.device == dev) {
            *out = d;
            return TE_OK;
        }
    hipDeviceProp_t prop;
    e = hipGetDeviceProperties(&prop, dev);
    if (e != hipSuccess)
        return hip_fail(e, "hipGetDeviceProperties");
    DeviceInfo d;
    d.device = dev;
    d.n_cu = prop.multiProcessorCount;
    std::snprintf(d.arch, sizeof d.arch, "%s", prop.gcnArchName);
    g_devs.push_back(d);
    *out = d;
    return TE_OK;
}

// ------------------------------------------------------------ batch layout

size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

// XCD work queues over a schedule of chunk pieces (ChunkDesc::item0 ascending,
// pieces of n points, items up to the next piece's item0 or n_items): contiguous
// item ranges of equal estimated work (an item of a chunk of n points costs
// about n).  A piece that is small next to a queue's share ends a queue whole, so
// the queue ends on the piece's cheapest blocks.
void queue_bounds(const std::vector<ChunkDesc> &pieces, int64_t n_items, std::vector<int32_t> *part_start)
{
    std::vector<int32_t> &ps = *part_start;
    ps.assign(kQueues + 1, 0);
    auto count = [&](size_t c) {
        return (c + 1 < pieces.size() ? (int64_t)pieces[c + 1].item0 : n_items) - pieces[c].item0;
    };
    double total = 0.0;
    for (size_t c = 0; c < pieces.size(); ++c)
        total += (double)pieces[c].n * count(c);
    double acc = 0.0;
    int p = 1;
    for (size_t c = 0; c < pieces.size(); ++c) {
        const ChunkDesc &d = pieces[c];
        const int64_t nb = count(c);
        const double w = (double)d.n * nb;
        if (w * 4 <= total / kQueues) {
            acc += w;
            while (p < kQueues && acc >= total * p / kQueues)
                ps[p++] = (int32_t)(d.item0 + nb);
            continue;
        }
        for (int64_t bk = 0; bk < nb; ++bk) {
            acc += d.n;
            while (p < kQueues && acc >= total * p / kQueues)
                ps[p++] = (int32_t)(d.item0 + bk + 1);
        }
    }
    while (p <= kQueues)
        ps[p++] = (int32_t)n_items;
    for (int q = 1; q <= kQueues; ++q)
        ps[q] = std::max(ps[q], ps[q - 1]);
}

void Batch::finish_layout()
{
    // LPT order: biggest chunks first so the persistent waves end together.
    order.resize(chunks.size());
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(),
                     [&](int a, int b) { return chunks[a].n > chunks[b].n; });
    std::vector<ChunkDesc> sorted;
    sorted.reserve(chunks.size());
    item_start.clear();
    set_first.clear();
    n_items = 0;
    n_partials = 0;
    std::vector<ChunkDesc> leaders;       // first chunk of each set, n scaled by the set's size (queue costs)
    for (int c : order) {
        ChunkDesc d = chunks[c];
        const int64_t nb = (d.n + kWave - 1) / kWave;
        // a new work unit: every chunk without sets; with sets, when the previous set is
        // full or belongs to another window (the stable LPT order keeps a window's chunks together)
        const bool start = !use_sets || set_first.empty() || (int)sorted.size() - set_first.back() >= set_v ||
                           sorted.back().tp != d.tp || sorted.back().n != d.n;
        if (start) {
            d.item0 = (int32_t)n_items;
            item_start.push_back(d.item0);
            if (use_sets) {
                set_first.push_back((int32_t)sorted.size());
                leaders.push_back(d);
            }
            n_items += nb;
        } else {
            d.item0 = sorted.back().item0;
            leaders.back().n += d.n;
        }
        d.block0 = 0;
        d.pbase = n_partials;
        n_partials += nb;
        sorted.push_back(d);
    }
    chunks.swap(sorted);
    if (use_sets)
        set_first.push_back((int32_t)chunks.size());

    queue_bounds(use_sets ? leaders : chunks, n_items, &part_start);

    size_t o = 0;
    off_coords = o;
    o = align_up(o + sizeof(float) * (size_t)n_floats, 256);
    off_tables = o;
    off_chunks = o;
    o = align_up(o + sizeof(ChunkDesc) * chunks.size(), 16);
    off_items = o;
    o = align_up(o + sizeof(int32_t) * item_start.size(), 16);
    off_tasks = o;
    o = align_up(o + sizeof(EmbedTask) * tasks.size(), 16);
    off_ptasks = o;
    o = align_up(o + sizeof(PermTask) * perm_tasks.size(), 16);
    off_sorts = o;
    o = align_up(o + sizeof(SortTask) * sorts.size(), 16);
    off_parts = o;
    o = align_up(o + sizeof(int32_t) * part_start.size(), 16);
    off_sets = o;
    o = align_up(o + sizeof(int32_t) * set_first.size(), 16);
    tables_bytes = o - off_tables;
    off_partial = align_up(o, 256);
    o = off_partial + sizeof(double) * (size_t)std::max<int64_t>(n_partials, 1);
    // results, p-values and a copy of the error word back to back: one download
    off_results = align_up(o, 256);
    o = off_results + sizeof(double) * (size_t)std::max(n_results, 1);
    off_pv = o;
    o = off_pv + sizeof(double) * (size_t)std::max(n_groups, 1);
    off_errout = o;
    o = off_errout + sizeof(double);
    // error word and reduce counter, then the XCD queue counters: one fill
    off_ctr = align_up(o, 256);
    o = off_ctr + sizeof(int32_t) * 4;
    off_qctr = o;
    o = off_qctr + sizeof(int32_t) * kQueues;
    off_sigma = align_up(o, 256);
    o = off_sigma + sizeof(int32_t) * (size_t)n_sigma;
    off_perm = align_up(o, 256);
    o = off_perm + sizeof(int32_t) * (size_t)n_perm;
    off_scratch = align_up(o, 256);
    o = off_scratch + sizeof(uint64_t) * (size_t)n_scratch;
    total_bytes = align_up(o, 256);

    host_tables.assign(tables_bytes, 0);
    std::memcpy(host_tables.data() + (off_chunks - off_tables), chunks.data(), sizeof(ChunkDesc) * chunks.size());
    std::memcpy(host_tables.data() + (off_items - off_tables), item_start.data(),
                sizeof(int32_t) * item_start.size());
    if (!tasks.empty())
        std::memcpy(host_tables.data() + (off_tasks - off_tables), tasks.data(), sizeof(EmbedTask) * tasks.size());
    if (!perm_tasks.empty())
        std::memcpy(host_tables.data() + (off_ptasks - off_tables), perm_tasks.data(),
                    sizeof(PermTask) * perm_tasks.size());
    if (!sorts.empty())
        std::memcpy(host_tables.data() + (off_sorts - off_tables), sorts.data(), sizeof(SortTask) * sorts.size());
    std::memcpy(host_tables.data() + (off_parts - off_tables), part_start.data(), sizeof(int32_t) * part_start.size());
    if (!set_first.empty())
        std::memcpy(host_tables.data() + (off_sets - off_tables), set_first.data(), sizeof(int32_t) * set_first.size());
}

bool sorting_enabled()
{
    const char *v = std::getenv("TE_NO_SORT");
    return !(v && *v && *v != '0');
}

// Padded sort length: the next power of two >= n.
int sort_npad(int n)
{
    int p = 1;
    while (p < n)
        p <<= 1;
    return p;
}

// ------------------------------------------------------------------- plan

static int history(const te_problem &p)
{
    return std::max(1 + (p.d_y - 1) * p.tau, p.u + (p.d_x - 1) * p.tau);
}

te_status Plan::build_group_batch(const std::vector<int> &groups, int n_surr, Batch *b, const BatchOptions &opt) const
{
    TraceRange trace_range("te.build_batch");
    if (opt.delays)
        n_surr = (int)opt.delays->size() - 1;
    // groups: indices g = pair * n_points + point; every group gets S+1 chunks
    // that share one (y_t', Y_past) block.
    b->n_groups = (int)groups.size();
    b->n_surr = n_surr;
    b->use_sets = opt.allow_sets && !opt.local_outputs && n_surr >= 1 && sets_eligible();
    b->set_v = set_variants(dy_eff(), p.d_x);
    b->n_results = b->n_groups * (n_surr + 1);
    b->groups = groups;
    int64_t fl = 0;
    // With x_t in the conditioning set the target block holds it as its last
    // target-past row; x_t follows the source shuffle, so every chunk then has a
    // target block of its own.
    const bool cond = p.cond_source != 0;
    const int dT = 1 + p.d_y + p.cond_source, dS = p.d_x;
    for (int gi = 0; gi < (int)groups.size(); ++gi) {
        const int g = groups[gi];
        const int pair = g / p.n_points, c = g % p.n_points;
        const int N = (int)npts[c];
        int64_t tp = fl;
        if (!cond)
            fl += (int64_t)dT * N;
        int64_t sig = -1;
        if (sorted) {
            SortTask st{};
            sig = b->n_sigma;
            st.sig = sig;
            st.npad = sort_npad(N);
            st.scratch = -1;
            if (st.npad > kSortLds) {
                st.scratch = b->n_scratch;
                b->n_scratch += st.npad;
            }
            st.key_off = -1;
            st.mode = 0;
            st.pair = pair;
            st.w = wstart[c];
            st.W = wlen[c];
            st.Rc = trials[c];
            st.n = N;
            b->sorts.push_back(st);
            b->n_sigma += N;
        }
        for (int s = 0; s <= n_surr; ++s) {
            if (cond) {
                tp = fl;
                fl += (int64_t)dT * N;
            }
            ChunkDesc d{};
            d.tp = tp;
            d.s = fl;
            d.ld = N;
            d.out = -1;
            d.perm = -1;
            if (opt.local_outputs && s == 0) {        // per-point outputs of the original, in window order
                d.out = local_off[g];
                d.perm = sig;
            }
            d.n = N;
            d.result = gi * (n_surr + 1) + s;
            b->chunks.push_back(d);
            EmbedTask t{};
            t.tp = (s == 0 || cond) ? tp : -1;
            t.s = fl;
            t.perm = -1;
            t.sig = sig;
            if (opt.delays)
                t.u = (*opt.delays)[s];
            if (opt.delay_from_device)
                t.u_slot = gi + 1;
            if (s > 0 && !opt.delays) {
                // the surrogate's trial permutation: row (pair, c, s-1) of the caller's
                // [pair][point][surrogate][trial] array, or drawn from the seed
                PermTask pt{};
                pt.src = (((int64_t)pair * p.n_points + c) * n_surr + (s - 1)) * p.n_trials;
                pt.dst = b->n_perm;
                pt.rc = trials[c];
                pt.len = trials[c];
                pt.pair = pair;
                pt.point = c;
                pt.surr = s - 1;
                b->perm_tasks.push_back(pt);
                b->n_perm += trials[c];
                t.perm = pt.dst;
            }
            t.pair = pair;
            t.w = wstart[c];
            t.W = wlen[c];
            t.Rc = trials[c];
            t.n = N;
            b->tasks.push_back(t);
            fl += (int64_t)dS * N;
        }
    }
    b->n_floats = fl;
    b->finish_layout();
    return TE_OK;
}

// Pinned host staging buffers, reused across calls.
void *PinnedPool::take(size_t bytes)
{
    std::lock_guard<std::mutex> lk(mu);
    for (auto &b : bufs)
        if (!b.busy && b.bytes >= bytes) {
            b.busy = true;
            return b.ptr;
        }
    Buf nb;
    nb.bytes = std::max<size_t>(bytes, 4096);
    if (hipHostMalloc(&nb.ptr, nb.bytes, hipHostMallocDefault) != hipSuccess)
        return nullptr;
    nb.busy = true;
    bufs.push_back(nb);
    return nb.ptr;
}

void PinnedPool::give(void *ptr)
{
    std::lock_guard<std::mutex> lk(mu);
    for (auto &b : bufs)
        if (b.ptr == ptr)
            b.busy = false;
}

PinnedPool::~PinnedPool()
{
    for (auto &b : bufs)
        if (b.ptr)
            hipHostFree(b.ptr);
}

Plan::~Plan()
{
    if (async_tables)
        hipHostFree(async_tables);
    for (auto &g : graphs) {
        if (g.exec)
            hipGraphExecDestroy(g.exec);
        if (g.graph)
            hipGraphDestroy(g.graph);
    }
}

// Device and launch configuration, resolved on first execution (plans can be
// created and sized without a GPU).
te_status Plan::ensure_device() const
{
    std::lock_guard<std::mutex> lk(dev_mu);
    if (dev_ready)
        return TE_OK;
    te_status st = current_device(&dev);
    if (st != TE_OK)
        return st;
    std::vector<int64_t> ns(npts);
    std::nth_element(ns.begin(), ns.begin() + ns.size() / 2, ns.end());
    cfg = default_config(dev, dy_eff(), p.d_x, p.k, ns[ns.size() / 2]);
    dev_ready = true;
    return TE_OK;
}

// Grid (in waves) for a persistent search over n_items items.
int Plan::grid_waves(int64_t n_items) const
{
    const int64_t full = (int64_t)dev.n_cu * cfg.wg_per_cu * cfg.waves_per_wg;
    return (int)std::max<int64_t>(1, std::min<int64_t>(full, n_items));
}

bool Plan::sets_eligible() const
{
    const char *v = std::getenv("TE_NO_SETS");
    if (v && *v && *v != '0')
        return false;
    return sorted && p.cond_source == 0 && search_sets_supported(dy_eff(), p.d_x, p.k);
}

SearchConfig Plan::batch_config(const Batch &b) const
{
    SearchConfig c = cfg;
    if (b.use_sets) {
        const int occ = search_sets_occupancy(dy_eff(), p.d_x, c.slots, c.waves_per_wg);
        c.wg_per_cu = std::max(1, std::min(c.wg_per_cu, occ));
    }
    return c;
}

// Enqueue one batch: upload tables, embed, search, reduce, p-values, copy results
// into the pinned staging block `stage` (results, p-values, error word).
te_status Plan::enqueue_batch(const Batch &b, const float *x, const float *y, const int32_t *perms, char *ws,
                              void *stage, hipStream_t st, double *lte_out, const int32_t *u_dev,
                              const void *tables_src, void *out_dst) const
{
    TraceRange trace_range("te.enqueue_batch");
    hipError_t e;
    char *tables_host = static_cast<char *>(stage);
    if (tables_src == nullptr) {
        std::memcpy(tables_host, b.host_tables.data(), b.tables_bytes);
        tables_src = tables_host;
    }
    e = hipMemcpyAsync(ws + b.off_tables, tables_src, b.tables_bytes, hipMemcpyHostToDevice, st);
    if (e != hipSuccess)
        return hip_fail(e, "upload tables");
    // ctr: [1] error word, [2] finished reduce workgroups; the queue counters follow
    int32_t *ctr = reinterpret_cast<int32_t *>(ws + b.off_ctr);
    int32_t *qctr = reinterpret_cast<int32_t *>(ws + b.off_qctr);
    if ((e = launch_fill_i32(ctr, 0, 4 + kQueues, st)) != hipSuccess)
        return hip_fail(e, "fill");
    float *base = reinterpret_cast<float *>(ws + b.off_coords);
    int32_t *parea = reinterpret_cast<int32_t *>(ws + b.off_perm);
    if (!b.perm_tasks.empty()) {
        // the caller's permutations (copied and checked) or ones drawn from the seed
        e = launch_perms(perms, reinterpret_cast<const PermTask *>(ws + b.off_ptasks), (int)b.perm_tasks.size(),
                         parea, p.seed, ctr + 1, st);
        if (e != hipSuccess)
            return hip_fail(e, "permutation launch");
    }
    int32_t *sigma = reinterpret_cast<int32_t *>(ws + b.off_sigma);
    e = launch_sort(y, nullptr, reinterpret_cast<const SortTask *>(ws + b.off_sorts), (int)b.sorts.size(), sigma,
                    reinterpret_cast<uint64_t *>(ws + b.off_scratch), p.n_trials, p.n_samples, st);
    if (e != hipSuccess)
        return hip_fail(e, "sort launch");
    int max_n = 0;
    for (const EmbedTask &t : b.tasks)
        max_n = std::max(max_n, t.n);
    e = launch_embed(x, y, parea, sigma, u_dev, reinterpret_cast<const EmbedTask *>(ws + b.off_tasks),
                     (int)b.tasks.size(), max_n, base, p.n_trials, p.n_samples, p.d_y, p.d_x, p.tau, p.u,
                     p.cond_source, ctr + 1, st);
    if (e != hipSuccess)
        return hip_fail(e, "embed launch");
    SearchArgs a{};
    a.base = base;
    a.chunks = reinterpret_cast<const ChunkDesc *>(ws + b.off_chunks);
    a.item_start = reinterpret_cast<const int32_t *>(ws + b.off_items);
    a.n_chunks = (int32_t)(b.use_sets ? b.set_first.size() - 1 : b.chunks.size());
    a.set_first = b.use_sets ? reinterpret_cast<const int32_t *>(ws + b.off_sets) : nullptr;
    a.n_items = (int32_t)b.n_items;
    a.k = p.k;
    a.counter = qctr;
    a.n_parts = kQueues;
    a.part_start = reinterpret_cast<const int32_t *>(ws + b.off_parts);
    a.partial = reinterpret_cast<double *>(ws + b.off_partial);
    a.eps_out = nullptr;
    a.cnt_out = nullptr;
    a.cnt_stride = 0;
    a.lte_out = lte_out;
    a.perm_base = sigma;
    a.sorted = sorted ? 1 : 0;
    const SearchConfig bc = batch_config(b);
    const int64_t full_grid = (int64_t)dev.n_cu * bc.wg_per_cu * bc.waves_per_wg;
    if ((e = launch_search_timed(a, dy_eff(), p.d_x, bc,
                                 (int)std::max<int64_t>(1, std::min<int64_t>(full_grid, b.n_items)), st)) != hipSuccess)
        return hip_fail(e, "search launch");
    double *res = reinterpret_cast<double *>(ws + b.off_results);
    double *pv = reinterpret_cast<double *>(ws + b.off_pv);
    int32_t *err_out = reinterpret_cast<int32_t *>(ws + b.off_errout);
    if ((e = launch_reduce(a.chunks, (int)b.chunks.size(), a.partial, p.k, ctr + 1, res, st, b.n_groups, b.n_surr, pv,
                           ctr + 2, err_out)) != hipSuccess)
        return hip_fail(e, "reduce launch");
    if (out_dst != nullptr)
        e = hipMemcpyAsync(out_dst, res, sizeof(double) * (b.n_results + b.n_groups), hipMemcpyDefault, st);
    else
        e = hipMemcpyAsync(tables_host + align_up(b.tables_bytes, 256), res,
                           sizeof(double) * (b.n_results + b.n_groups) + sizeof(int32_t), hipMemcpyDeviceToHost, st);
    if (e != hipSuccess)
        return hip_fail(e, "download results");
    return TE_OK;
}

size_t Batch::stage_bytes() const
{
    return align_up(tables_bytes, 256) + sizeof(double) * (n_results + n_groups) + 64;
}

te_status Plan::unpack_batch(const Batch &b, const void *stage, double *te_orig, double *te_surr, double *p_value,
                             bool *bad_input) const
{
    TraceRange trace_range("te.unpack_batch");
    const char *out = static_cast<const char *>(stage) + align_up(b.tables_bytes, 256);
    const double *res = reinterpret_cast<const double *>(out);
    const double *pv = res + b.n_results;
    int32_t err = 0;
    std::memcpy(&err, out + sizeof(double) * (b.n_results + b.n_groups), sizeof err);
    for (int gi = 0; gi < b.n_groups; ++gi) {
        const int g = b.groups[gi];
        const double *r = res + (size_t)gi * (b.n_surr + 1);
        if (te_orig)
            te_orig[g] = r[0];
        if (te_surr)
            for (int s = 0; s < b.n_surr; ++s)
                te_surr[(size_t)g * b.n_surr + s] = r[1 + s];
        if (p_value)
            p_value[g] = pv[gi];
    }
    if (err)
        *bad_input = true;
    return TE_OK;
}

}  // namespace te

using namespace te;

// =================================================================== C ABI

extern "C" {

const char *te_version(void) { return "libte 0.1 (gfx950)"; }

const char *te_last_error(void) { return g_last_error.c_str(); }

te_status te_plan_create(const te_problem *pr, te_plan *out)
{
    TraceRange trace_range("te.plan_create");
    clear_error();
    if (!pr || !out)
        return fail(TE_ERR_INVALID, "null argument");
    *out = nullptr;
    const te_problem &p = *pr;
    if (p.n_pairs < 1 || p.n_trials < 1 || p.n_samples < 1 || p.n_points < 1)
        return fail(TE_ERR_INVALID, "n_pairs, n_trials, n_samples and n_points must be >= 1");
    if (p.d_y < 1 || p.d_y > kMaxDimY || p.d_x < 1 || p.d_x > kMaxDimX)
        return fail(TE_ERR_INVALID, "d_y and d_x must be in 1..4 (got %d, %d)", p.d_y, p.d_x);
    if (p.tau < 1 || p.u < 1)
        return fail(TE_ERR_INVALID, "tau and u must be >= 1");
    if (p.k < 1 || p.k > kMaxK)
        return fail(TE_ERR_INVALID, "k must be in 1..%d", kMaxK);
    if (p.n_surrogates < 0)
        return fail(TE_ERR_INVALID, "n_surrogates must be >= 0");
    if (p.cond_source < 0 || p.cond_source > 1)
        return fail(TE_ERR_INVALID, "cond_source must be 0 or 1");
    if (p.d_y + p.cond_source > kMaxDimY)
        return fail(TE_ERR_INVALID, "conditioning on x_t needs d_y <= %d", kMaxDimY - 1);
    if (!p.window_start)
        return fail(TE_ERR_INVALID, "window_start is required");
    auto plan = std::make_unique<te_plan_s>();
    Plan &P = plan->impl;
    P.p = p;
    P.sorted = sorting_enabled();
    const int h = history(p);
    for (int c = 0; c < p.n_points; ++c) {
        const int w = p.window_start[c];
        const int W = p.window_len ? p.window_len[c] : p.window;
        const int Rc = p.trials ? p.trials[c] : p.n_trials;
        if (W < 1)
            return fail(TE_ERR_INVALID, "window %d: length %d < 1", c, W);
        if (w < h)
            return fail(TE_ERR_INVALID, "window %d starts at %d but the embedding needs %d samples of history", c,
                        w, h);
        if ((int64_t)w + W > p.n_samples)
            return fail(TE_ERR_INVALID, "window %d [%d, %d) runs past n_samples = %d", c, w, w + W, p.n_samples);
        if (Rc < 1 || Rc > p.n_trials)
            return fail(TE_ERR_INVALID, "window %d: trials %d outside 1..%d", c, Rc, p.n_trials);
        const int64_t N = (int64_t)Rc * W;
        if (N <= p.k)
            return fail(TE_ERR_INVALID, "window %d pools %lld points, need more than k = %d", c, (long long)N, p.k);
        // the search kernels address a coordinate of a block by a 32-bit byte offset from
        // the block's start (at most 5 rows of N floats before it): N <= 2^27 keeps it in range
        if (N > kMaxWindowPoints)
            return fail(TE_ERR_INVALID, "window %d pools %lld points, more than %d", c, (long long)N,
                        kMaxWindowPoints);
        P.wstart.push_back(w);
        P.wlen.push_back(W);
        P.trials.push_back(Rc);
        P.npts.push_back(N);
    }
    P.local_off.assign(1, 0);
    for (int pr = 0; pr < p.n_pairs; ++pr)
        for (int c = 0; c < p.n_points; ++c)
            P.local_off.push_back(P.local_off.back() + P.npts[c]);
    P.p.window_start = nullptr;
    P.p.window_len = nullptr;
    P.p.trials = nullptr;
    if (!search_supported(P.dy_eff(), p.d_x, p.k, 8))
        return fail(TE_ERR_INVALID, "no search kernel for d_y=%d d_x=%d k=%d", p.d_y, p.d_x, p.k);
    // full batch: every (pair, point) with all surrogates
    std::vector<int> all(p.n_pairs * p.n_points);
    std::iota(all.begin(), all.end(), 0);
    P.build_group_batch(all, p.n_surrogates, &P.full);
    // largest single group bounds the minimum workspace
    size_t mn = 0;
    for (int c = 0; c < p.n_points; ++c) {
        Batch one;
        P.build_group_batch({c}, p.n_surrogates, &one);
        mn = std::max(mn, one.total_bytes);
    }
    P.min_bytes = mn;
    // plain paths: one chunk at a time (te_estimate: originals; te_estimate_each: all chunks)
    P.plain_bytes = std::max(P.plain_layout(0).total, P.plain_layout(p.n_surrogates).total);
    *out = plan.release();
    return TE_OK;
}

te_status te_plan_destroy(te_plan plan)
{
    delete plan;
    return TE_OK;
}

te_status te_plan_workspace_bytes(te_plan plan, size_t *full, size_t *minimum, size_t *plain)
{
    clear_error();
    if (!plan)
        return fail(TE_ERR_INVALID, "null plan");
    if (full)
        *full = plan->impl.full.total_bytes;
    if (minimum)
        *minimum = plan->impl.min_bytes;
    if (plain)
        *plain = plan->impl.plain_bytes;
    return TE_OK;
}

te_status te_estimate(te_plan plan, const float *x, const float *y, void *ws, size_t ws_bytes, void *hip_stream,
                      double *te_out)
{
    clear_error();
    if (!plan || !x || !y || !ws || !te_out)
        return fail(TE_ERR_INVALID, "null argument");
    te_status s = plan->impl.ensure_device();
    if (s != TE_OK)
        return s;
    return plan->impl.estimate_each(x, y, nullptr, 0, static_cast<char *>(ws), ws_bytes, (hipStream_t)hip_stream,
                                    te_out, nullptr, nullptr);
}

te_status te_estimate_each(te_plan plan, const float *x, const float *y, const int32_t *perms, void *ws,
                           size_t ws_bytes, void *hip_stream, double *te_orig, double *te_surr, double *p_value)
{
    clear_error();
    if (!plan || !x || !y || !ws || !te_orig)
        return fail(TE_ERR_INVALID, "null argument");
    const Plan &P = plan->impl;
    if (P.p.n_surrogates > 0 && !te_surr)
        return fail(TE_ERR_INVALID, "n_surrogates > 0 needs te_surr");
    te_status s = P.ensure_device();
    if (s != TE_OK)
        return s;
    return P.estimate_each(x, y, perms, P.p.n_surrogates, static_cast<char *>(ws), ws_bytes, (hipStream_t)hip_stream,
                           te_orig, te_surr, p_value);
}

te_status te_surrogates(te_plan plan, const float *x, const float *y, const int32_t *perms, void *ws,
                        size_t ws_bytes, void *hip_stream, int32_t use_graph, double *te_orig, double *te_surr,
                        double *p_value)
{
    clear_error();
    if (!plan || !x || !y || !ws || !te_orig)
        return fail(TE_ERR_INVALID, "null argument");
    const Plan &P = plan->impl;
    if (P.p.n_surrogates > 0 && !te_surr)
        return fail(TE_ERR_INVALID, "n_surrogates > 0 needs te_surr");
    te_status s = plan->impl.ensure_device();
    if (s != TE_OK)
        return s;
    return plan->impl.run_surrogates(x, y, perms, static_cast<char *>(ws), ws_bytes, (hipStream_t)hip_stream,
                                     use_graph != 0, te_orig, te_surr, p_value);
}

te_status te_surrogates_async(te_plan plan, const float *x, const float *y, const int32_t *perms, void *ws,
                              size_t ws_bytes, void *hip_stream, double *out)
{
    clear_error();
    if (!plan || !x || !y || !ws || !out)
        return fail(TE_ERR_INVALID, "null argument");
    const Plan &P = plan->impl;
    te_status s = P.ensure_device();
    if (s != TE_OK)
        return s;
    return P.run_surrogates_async(x, y, perms, static_cast<char *>(ws), ws_bytes, (hipStream_t)hip_stream, out);
}

size_t te_plan_permutations_workspace_bytes(te_plan plan)
{
    if (!plan)
        return 0;
    return align_up(sizeof(PermTask) * plan->impl.full.perm_tasks.size(), 256) + 256;
}

te_status te_plan_permutations(te_plan plan, void *ws, size_t ws_bytes, void *hip_stream, int32_t *perms)
{
    clear_error();
    if (!plan || !ws || !perms)
        return fail(TE_ERR_INVALID, "null argument");
    const Plan &P = plan->impl;
    const std::vector<PermTask> &rows = P.full.perm_tasks;
    if (rows.empty())
        return TE_OK;
    const size_t need = te_plan_permutations_workspace_bytes(plan);
    if (ws_bytes < need)
        return fail(TE_ERR_NOMEM, "te_plan_permutations needs a workspace of %zu bytes", need);
    te_status s = P.ensure_device();
    if (s != TE_OK)
        return s;
    // every row at its place in the caller's [pair][point][surrogate][trial] array
    const size_t tbytes = sizeof(PermTask) * rows.size();
    char *stg = static_cast<char *>(P.pool.take(tbytes + 64));
    if (!stg)
        return fail(TE_ERR_NOMEM, "pinned staging allocation failed");
    PermTask *ht = reinterpret_cast<PermTask *>(stg);
    for (size_t i = 0; i < rows.size(); ++i) {
        ht[i] = rows[i];
        ht[i].dst = rows[i].src;
        ht[i].len = P.p.n_trials;
    }
    char *d = static_cast<char *>(ws);
    int32_t *err = reinterpret_cast<int32_t *>(d + need - 256);
    hipStream_t st = (hipStream_t)hip_stream;
    hipError_t e = hipMemcpyAsync(d, stg, tbytes, hipMemcpyHostToDevice, st);
    if (e == hipSuccess)
        e = launch_fill_i32(err, 0, 1, st);
    if (e == hipSuccess)
        e = launch_perms(nullptr, reinterpret_cast<const PermTask *>(d), (int)rows.size(), perms, P.p.seed, err, st);
    int32_t *herr = reinterpret_cast<int32_t *>(stg + tbytes);
    if (e == hipSuccess)
        e = hipMemcpyAsync(herr, err, sizeof(int32_t), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess)
        e = hipStreamSynchronize(st);
    const int32_t bad = e == hipSuccess ? *herr : 0;
    P.pool.give(stg);
    if (e != hipSuccess)
        return hip_fail(e, "te_plan_permutations");
    if (bad)
        return fail(TE_ERR_DEVICE, "permutation draw failed (more rejected draws than the kernel records)");
    return TE_OK;
}

te_status te_plan_local_offsets(te_plan plan, int64_t *offsets)
{
    clear_error();
    if (!plan || !offsets)
        return fail(TE_ERR_INVALID, "null argument");
    const auto &o = plan->impl.local_off;
    std::copy(o.begin(), o.end(), offsets);
    return TE_OK;
}

te_status te_local(te_plan plan, const float *x, const float *y, void *ws, size_t ws_bytes, void *hip_stream,
                   double *lte, double *te_out)
{
    clear_error();
    if (!plan || !x || !y || !ws || !lte)
        return fail(TE_ERR_INVALID, "null argument");
    te_status s = plan->impl.ensure_device();
    if (s != TE_OK)
        return s;
    return plan->impl.run_local(x, y, static_cast<char *>(ws), ws_bytes, (hipStream_t)hip_stream, lte, te_out);
}

}  // extern "C"
