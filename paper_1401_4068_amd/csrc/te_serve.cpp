// te_serve.cpp -- continuous-batching server for TE jobs.
//
// Jobs (a te_problem plus host series and permutations) are submitted from any
// thread.  A server thread admits them in FIFO order while a job slot is free
// and its footprint (series, permutations, embedded coordinates, tables,
// partial sums) fits in the caller's device arena; an admitted job's series is
// copied into the arena and embedded there once, then stays resident.  Work is
// issued in steps: each step is one persistent search launch per kernel class
// (d_y, d_x, k) over reference blocks taken from every ready job in admission
// order, up to a pair budget, so jobs that arrive while others are on the GPU
// join at the next step.  Two steps per class may be in flight.  When a job's
// last blocks are scheduled, its reduction, p-values and result copy are queued
// behind that step on the same stream.  Per-block partial sums are reduced in
// block order, so a job's estimates do not depend on what it was batched with.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <deque>
#include <list>
#include <map>
#include <memory>
#include <mutex>
#include <thread>
#include <vector>

#include "te.h"
#include "te_internal.h"
#include "te_runtime.h"

namespace te {

namespace {

double now_s()
{
    using namespace std::chrono;
    return duration<double>(steady_clock::now().time_since_epoch()).count();
}

// First-fit allocator over [0, size) in 256-byte units.
struct Arena {
    size_t size = 0;
    std::map<size_t, size_t> free_;   // offset -> length
    size_t used = 0, peak = 0;
    void init(size_t bytes)
    {
        size = bytes / 256 * 256;
        free_.clear();
        if (size)
            free_[0] = size;
    }
    bool alloc(size_t bytes, size_t *off)
    {
        bytes = align_up(std::max<size_t>(bytes, 1), 256);
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second >= bytes) {
                *off = it->first;
                const size_t rest = it->second - bytes;
                const size_t roff = it->first + bytes;
                free_.erase(it);
                if (rest)
                    free_[roff] = rest;
                used += bytes;
                peak = std::max(peak, used);
                return true;
            }
        }
        return false;
    }
    // the same from the top of the highest free block that fits: long-lived blocks (kernel
    // class step tables) stay apart from job regions, which are taken first-fit from below
    bool alloc_high(size_t bytes, size_t *off)
    {
        bytes = align_up(std::max<size_t>(bytes, 1), 256);
        for (auto it = free_.rbegin(); it != free_.rend(); ++it) {
            if (it->second >= bytes) {
                it->second -= bytes;
                *off = it->first + it->second;
                if (it->second == 0)
                    free_.erase(std::next(it).base());
                used += bytes;
                peak = std::max(peak, used);
                return true;
            }
        }
        return false;
    }
    void release(size_t off, size_t bytes)
    {
        bytes = align_up(std::max<size_t>(bytes, 1), 256);
        used -= bytes;
        auto it = free_.emplace(off, bytes).first;
        auto nx = std::next(it);
        if (nx != free_.end() && it->first + it->second == nx->first) {
            it->second += nx->second;
            free_.erase(nx);
        }
        if (it != free_.begin()) {
            auto pv = std::prev(it);
            if (pv->first + pv->second == it->first) {
                pv->second += it->second;
                free_.erase(it);
            }
        }
    }
};

enum JobState { QUEUED, SETUP, READY, DONE, FAILED, CANCELLED };

struct Job {
    uint64_t id = 0;
    std::unique_ptr<te_plan_s> plan;
    void *hin = nullptr;               // pinned copy of x | y | perms, taken at submit
    size_t hin_bytes = 0, hin_y = 0, hin_perm = 0, n_series = 0, n_perm = 0;
    Batch batch;                       // layout relative to the job's coordinate block
    size_t footprint = 0, region = 0;  // bytes, arena offset
    size_t off_x = 0, off_y = 0, off_perm = 0, off_batch = 0;
    int cls = 0;
    JobState state = QUEUED;
    std::vector<int32_t> next_block;   // per unit (chunk, or set of chunks; schedule order): next block
    size_t next_chunk = 0;             // first unit with unscheduled blocks
    bool all_scheduled = false;
    hipEvent_t ready_ev = nullptr, done_ev = nullptr;
    void *stage = nullptr;
    double t_submit = 0, t_done = 0;
    te_status status = TE_OK;
    std::string error;
    std::vector<double> te_orig, te_surr, pv;
};

struct StepRec {
    hipEvent_t ev = nullptr;
    int slot = 0;
    int cls = 0;
    std::vector<uint64_t> finishing;   // jobs whose reduction is queued behind this step
};

// Jobs with the same (d_y, d_x, k) share a search kernel and a stream; each class
// owns two step-table slots (arena + pinned staging) so two steps can be in flight.
struct KernelClass {
    int d_y = 0, d_x = 0, k = 0;
    int cond = 0;                       // conditioning on x_t (d_y above includes it)
    bool sorted = true;
    bool sets = false;                  // jobs searched as chunk sets (the chunk-set search kernel)
    int set_v = 1;                      // chunks per set
    hipStream_t stream[2] = {nullptr, nullptr};   // steps alternate, so one step's tail overlaps the next
    hipEvent_t last_ev[2] = {nullptr, nullptr};   // completion of the last step issued on each stream
    SearchConfig cfg{};
    int in_flight = 0;
    int64_t max_items = 0;
    size_t table_cap = 0;
    bool tables = false;                // table_off allocated in the arena (at the first admission of the class)
    size_t table_off[2] = {0, 0};
    void *stage[2] = {nullptr, nullptr};
    bool slot_busy[2] = {false, false};
};

}  // namespace

struct Server {
    char *arena = nullptr;
    size_t arena_bytes = 0;
    int max_slots = 0, max_queue = 0;
    int64_t step_pairs = 0;
    bool dry = false;
    bool held = false;   // admission paused (TE_SERVE_HOLD) until te_serve_resume
    DeviceInfo dev;

    std::mutex mu;
    std::condition_variable cv_done;
    // The server thread sleeps on cv_wake between state changes: a submission,
    // cancellation, resume or close, or the device finishing a job's setup or a
    // step (a host function queued behind that work on its stream).  wake_mu is
    // never held while a HIP call is made, so the runtime thread that runs those
    // host functions cannot block on a lock the server thread holds.
    std::mutex wake_mu;
    std::condition_variable cv_wake;
    bool wake = false;
    int64_t fault_staging = 0;                     // TE_SERVE_FAULT_STAGING: admission that fails its staging
    int64_t admissions = 0;
    bool stopping = false;
    std::thread thr;
    uint64_t next_id = 1;
    std::deque<Job *> queue;                       // submitted, not admitted (FIFO)
    std::list<Job *> resident;                     // admitted, in admission order
    std::map<uint64_t, std::unique_ptr<Job>> jobs; // all live tickets
    Arena alloc;
    std::vector<KernelClass> classes;
    std::deque<StepRec> steps;                     // in flight, issue order
    hipStream_t setup_stream = nullptr;
    PinnedPool pool;
    // stats
    std::vector<double> lat;
    double t_first = 0, t_last = 0;
    int64_t completed = 0, failed = 0, cancelled = 0, n_steps = 0, est_done = 0, peak_slots = 0;

    te_status start();
    void loop();
    void wake_up();
    void sleep_until_woken(std::unique_lock<std::mutex> &lk, int ms);
    void drain_streams(const KernelClass *kc);
    int class_of(const te_problem &p, bool sorted, bool sets, int set_v);
    bool ensure_tables(KernelClass &c);
    bool admit_one(Job *j);
    void poll_setup();
    bool issue_step(int ci);
    void poll_steps();
    void finish(Job *j);
    void fail_job(Job *j, te_status st, const char *msg);
    void release(Job *j);
};

// Kernel class of a problem, created on first use (-1 if its step tables do not fit).
int Server::class_of(const te_problem &p, bool sorted, bool sets, int set_v)
{
    for (size_t i = 0; i < classes.size(); ++i)
        if (classes[i].d_y == p.d_y + p.cond_source && classes[i].d_x == p.d_x && classes[i].k == p.k &&
            classes[i].sorted == sorted && classes[i].cond == p.cond_source && classes[i].sets == sets)
            return (int)i;
    KernelClass c;
    c.sorted = sorted;
    c.sets = sets;
    c.set_v = sets ? set_v : 1;
    c.d_y = p.d_y + p.cond_source;                   // as the search sees it
    c.cond = p.cond_source;
    c.d_x = p.d_x;
    c.k = p.k;
    if (!dry) {
        c.cfg = default_config(dev, c.d_y, p.d_x, p.k, 16384);
        if (sets)
            c.cfg.wg_per_cu = std::max(1, std::min(c.cfg.wg_per_cu,
                                                   search_sets_occupancy(c.d_y, c.d_x, c.cfg.slots, c.cfg.waves_per_wg)));
    }
    c.max_items = (int64_t)std::max(1, dev.n_cu) * std::max(1, c.cfg.wg_per_cu) * std::max(1, c.cfg.waves_per_wg) * 16;
    // step table: chunk descriptors (at most max_items), piece starts, set ranges, queue bounds, queue heads
    c.table_cap = align_up(sizeof(ChunkDesc) * (size_t)c.max_items, 16) +
                  align_up(sizeof(int32_t) * (size_t)c.max_items, 16) +
                  align_up(sizeof(int32_t) * ((size_t)c.max_items + 1), 16) + align_up(sizeof(int32_t) * (kQueues + 1), 16) +
                  sizeof(int32_t) * kQueues + 64;
    if (!dry) {
        for (int sl = 0; sl < 2; ++sl) {
            hipStreamCreateWithFlags(&c.stream[sl], hipStreamNonBlocking);
            hipEventCreateWithFlags(&c.last_ev[sl], hipEventDisableTiming);
            c.stage[sl] = pool.take(c.table_cap);
        }
    }
    classes.push_back(c);
    return (int)classes.size() - 1;
}

// The class's two step tables in the arena, taken when its first job is admitted
// (admission waits, like a job's footprint, while they do not fit).
bool Server::ensure_tables(KernelClass &c)
{
    if (c.tables)
        return true;
    for (int sl = 0; sl < 2; ++sl) {
        if (!alloc.alloc_high(c.table_cap, &c.table_off[sl])) {
            for (int u = 0; u < sl; ++u)
                alloc.release(c.table_off[u], c.table_cap);
            return false;
        }
    }
    c.tables = true;
    return true;
}

static int embed_max_n(const Batch &b)
{
    int m = 0;
    for (const EmbedTask &t : b.tasks)
        m = std::max(m, t.n);
    return m;
}

// Arena bytes of a job: its series, the caller's permutations (when given; drawn
// permutations live in the batch's own permutation area), then its batch layout.
static size_t job_footprint(const Plan &P, bool caller_perms, Batch *b, size_t *off_x, size_t *off_y,
                            size_t *off_perm, size_t *off_batch)
{
    const size_t ser = sizeof(float) * (size_t)P.p.n_pairs * P.p.n_trials * P.p.n_samples;
    const size_t perm = caller_perms ? sizeof(int32_t) * (size_t)P.p.n_pairs * P.p.n_points * P.p.n_surrogates *
                                           P.p.n_trials
                                     : 0;
    size_t o = 0;
    *off_x = o;
    o = align_up(o + ser, 256);
    *off_y = o;
    o = align_up(o + ser, 256);
    *off_perm = o;
    o = align_up(o + std::max<size_t>(perm, 4), 256);
    *off_batch = o;
    return o + b->total_bytes;
}

void Server::fail_job(Job *j, te_status st, const char *msg)
{
    j->status = st;
    j->error = msg;
    j->state = FAILED;
}

void Server::release(Job *j)
{
    if (j->footprint)
        alloc.release(j->region, j->footprint);
    j->footprint = 0;
    if (j->stage)
        pool.give(j->stage);
    j->stage = nullptr;
    if (j->hin) {
        if (!dry && j->ready_ev)
            hipEventSynchronize(j->ready_ev);   // uploads read the pinned inputs
        pool.give(j->hin);
    }
    j->hin = nullptr;
    if (j->ready_ev)
        hipEventDestroy(j->ready_ev);
    if (j->done_ev)
        hipEventDestroy(j->done_ev);
    j->ready_ev = j->done_ev = nullptr;
    resident.remove(j);
}

// Host function queued behind device work: wakes the server thread.
static void host_wake(void *srv) { static_cast<Server *>(srv)->wake_up(); }

void Server::wake_up()
{
    {
        std::lock_guard<std::mutex> lk(wake_mu);
        wake = true;
    }
    cv_wake.notify_one();
}

// Release mu and sleep until woken or ms pass, then take mu again.
void Server::sleep_until_woken(std::unique_lock<std::mutex> &lk, int ms)
{
    lk.unlock();
    {
        std::unique_lock<std::mutex> wl(wake_mu);
        cv_wake.wait_for(wl, std::chrono::milliseconds(ms), [&] { return wake; });
        wake = false;
    }
    lk.lock();
}

// Wait until the class's streams (every class when kc is null) and the setup
// stream have run everything queued on them.
void Server::drain_streams(const KernelClass *kc)
{
    if (dry)
        return;
    for (const KernelClass &c : classes)
        if (!kc || &c == kc)
            for (int sl = 0; sl < 2; ++sl)
                if (c.stream[sl])
                    hipStreamSynchronize(c.stream[sl]);
    if (setup_stream)
        hipStreamSynchronize(setup_stream);
}

// Copy the series in, upload the job's tables, embed every chunk once.
bool Server::admit_one(Job *j)
{
    TraceRange trace_range("te.serve.admit");
    size_t off = 0;
    if (!ensure_tables(classes[j->cls]))
        return false;
    if (!alloc.alloc(j->footprint, &off))
        return false;
    j->region = off;
    j->state = SETUP;
    resident.push_back(j);
    peak_slots = std::max<int64_t>(peak_slots, (int64_t)resident.size());
    Batch &b = j->batch;
    j->next_block.assign(b.use_sets ? b.set_first.size() - 1 : b.chunks.size(), 0);
    j->next_chunk = 0;
    const bool inject = fault_staging > 0 && ++admissions == fault_staging;
    if (dry) {
        if (inject)
            fail_job(j, TE_ERR_NOMEM, "pinned staging allocation failed (injected)");
        else
            j->state = READY;
        return true;
    }
    const Plan &P = j->plan->impl;
    char *reg = arena + off;
    char *bat = reg + j->off_batch;
    const size_t ser = sizeof(float) * j->n_series;
    const char *hin = static_cast<const char *>(j->hin);
    hipError_t e = hipMemcpyAsync(reg + j->off_x, hin, ser, hipMemcpyHostToDevice, setup_stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(reg + j->off_y, hin + j->hin_y, ser, hipMemcpyHostToDevice, setup_stream);
    if (e == hipSuccess && j->n_perm)
        e = hipMemcpyAsync(reg + j->off_perm, hin + j->hin_perm, sizeof(int32_t) * j->n_perm, hipMemcpyHostToDevice,
                           setup_stream);
    // the job's chunk table with arena-absolute coordinate and partial offsets
    const int64_t fbase = (int64_t)((off + j->off_batch + b.off_coords) / sizeof(float));
    const int64_t pbase = (int64_t)((off + j->off_batch + b.off_partial) / sizeof(double));
    std::vector<char> tables(b.host_tables);
    ChunkDesc *cd = reinterpret_cast<ChunkDesc *>(tables.data() + (b.off_chunks - b.off_tables));
    for (size_t c = 0; c < b.chunks.size(); ++c) {
        cd[c].tp += fbase;
        cd[c].s += fbase;
        cd[c].pbase += pbase;
    }
    j->stage = inject ? nullptr : pool.take(std::max(b.tables_bytes, sizeof(double) * (b.n_results + b.n_groups) + 64));
    if (!j->stage) {
        // the series uploads queued above read the pinned inputs and write the job's
        // region: let them finish before the caller releases either
        hipStreamSynchronize(setup_stream);
        fail_job(j, TE_ERR_NOMEM, inject ? "pinned staging allocation failed (injected)"
                                         : "pinned staging allocation failed");
        return true;
    }
    std::memcpy(j->stage, tables.data(), b.tables_bytes);
    if (e == hipSuccess)
        e = hipMemcpyAsync(bat + b.off_tables, j->stage, b.tables_bytes, hipMemcpyHostToDevice, setup_stream);
    int32_t *ctr = reinterpret_cast<int32_t *>(bat + b.off_ctr);
    if (e == hipSuccess)
        e = launch_fill_i32(ctr, 0, 4, setup_stream);
    // the job's permutations: copied (and checked) from the uploaded ones, or drawn from its seed
    int32_t *perm = reinterpret_cast<int32_t *>(bat + b.off_perm);
    if (e == hipSuccess && !b.perm_tasks.empty())
        e = launch_perms(j->n_perm ? reinterpret_cast<const int32_t *>(reg + j->off_perm) : nullptr,
                         reinterpret_cast<const PermTask *>(bat + b.off_ptasks), (int)b.perm_tasks.size(), perm,
                         P.p.seed, ctr + 1, setup_stream);
    int32_t *sigma = reinterpret_cast<int32_t *>(bat + b.off_sigma);
    if (e == hipSuccess)
        e = launch_sort(reinterpret_cast<const float *>(reg + j->off_y), nullptr,
                        reinterpret_cast<const SortTask *>(bat + b.off_sorts), (int)b.sorts.size(), sigma,
                        reinterpret_cast<uint64_t *>(bat + b.off_scratch), P.p.n_trials, P.p.n_samples, setup_stream);
    if (e == hipSuccess)
        e = launch_embed(reinterpret_cast<const float *>(reg + j->off_x), reinterpret_cast<const float *>(reg + j->off_y),
                         perm, sigma, nullptr, reinterpret_cast<const EmbedTask *>(bat + b.off_tasks), (int)b.tasks.size(),
                         embed_max_n(b), reinterpret_cast<float *>(bat + b.off_coords), P.p.n_trials, P.p.n_samples, P.p.d_y, P.p.d_x,
                         P.p.tau, P.p.u, P.p.cond_source, ctr + 1, setup_stream);
    if (e == hipSuccess)
        e = hipEventCreateWithFlags(&j->ready_ev, hipEventDisableTiming);
    if (e == hipSuccess)
        e = hipEventRecord(j->ready_ev, setup_stream);
    if (e == hipSuccess)
        e = hipEventCreateWithFlags(&j->done_ev, hipEventDisableTiming);
    if (e == hipSuccess)
        e = hipLaunchHostFunc(setup_stream, host_wake, this);
    if (e != hipSuccess) {
        // work queued before the failure may still be reading or writing the job's memory
        hipStreamSynchronize(setup_stream);
        fail_job(j, TE_ERR_DEVICE, hipGetErrorString(e));
    }
    return true;
}

void Server::poll_setup()
{
    for (Job *j : resident)
        if (j->state == SETUP && hipEventQuery(j->ready_ev) == hipSuccess) {
            j->state = READY;
            if (j->hin)
                pool.give(j->hin);      // inputs are on the device now
            j->hin = nullptr;
        }
}

// One search launch for class ci over blocks of ready jobs, FIFO, up to the pair budget.
bool Server::issue_step(int ci)
{
    TraceRange trace_range("te.serve.step");
    KernelClass &kc = classes[ci];
    std::vector<ChunkDesc> tab;          // chunk descriptors of the step's pieces
    std::vector<ChunkDesc> leaders;      // first descriptor of each piece, n scaled by its chunks (queue costs)
    std::vector<int32_t> starts, sfirst;
    std::vector<Job *> finishing, members;
    int64_t items = 0, pairs = 0;
    const int64_t max_items = kc.max_items;
    // a step always gives every resident wave several work items (the last items of a
    // step then end close together); the pair budget only bounds it beyond that
    const int64_t min_items = max_items / 4;
    const int slot = kc.slot_busy[0] ? 1 : 0;
    if (kc.slot_busy[slot])
        return false;
    for (Job *j : resident) {
        if (j->state != READY || j->cls != ci || j->all_scheduled)
            continue;
        Batch &b = j->batch;
        const int64_t fbase = dry ? 0 : (int64_t)((j->region + j->off_batch + b.off_coords) / sizeof(float));
        const int64_t pb = dry ? 0 : (int64_t)((j->region + j->off_batch + b.off_partial) / sizeof(double));
        // units of work: single chunks, or the job's chunk sets in a set class
        const size_t n_units = kc.sets ? b.set_first.size() - 1 : b.chunks.size();
        members.push_back(j);
        while (j->next_chunk < n_units && (pairs < step_pairs || items < min_items) && items < max_items) {
            const size_t u = j->next_chunk;
            const int c0 = kc.sets ? b.set_first[u] : (int)u;
            const int cnt = kc.sets ? b.set_first[u + 1] - c0 : 1;
            const ChunkDesc &src = b.chunks[c0];
            const int nb = (src.n + kWave - 1) / kWave;
            const int64_t per_block = (int64_t)kWave * src.n * cnt;
            int64_t want = std::max<int64_t>(1, (step_pairs - pairs) / std::max<int64_t>(per_block, 1));
            want = std::max<int64_t>(want, min_items - items);
            want = std::min<int64_t>(want, max_items - items);
            const int take = (int)std::min<int64_t>(want, nb - j->next_block[u]);
            if ((int64_t)tab.size() + cnt > max_items)       // the descriptor table is full
                break;
            if (kc.sets)
                sfirst.push_back((int32_t)tab.size());
            for (int v = 0; v < cnt; ++v) {
                ChunkDesc d = b.chunks[c0 + v];
                d.tp += fbase;
                d.s += fbase;
                d.pbase += pb;
                d.item0 = (int32_t)items;
                d.block0 = j->next_block[u];
                if (v == 0) {
                    ChunkDesc l = d;
                    l.n = src.n * cnt;
                    leaders.push_back(l);
                }
                tab.push_back(d);
            }
            starts.push_back((int32_t)items);
            items += take;
            pairs += (int64_t)take * per_block;
            j->next_block[u] += take;
            if (j->next_block[u] >= nb)
                j->next_chunk++;
        }
        if (j->next_chunk >= n_units) {
            j->all_scheduled = true;
            finishing.push_back(j);
        }
        if ((pairs >= step_pairs && items >= min_items) || items >= max_items ||
            (int64_t)tab.size() + kc.set_v > max_items)
            break;
    }
    if (tab.empty())
        return false;
    StepRec st;
    st.cls = ci;
    st.slot = slot;
    for (Job *j : finishing)
        st.finishing.push_back(j->id);
    n_steps++;
    kc.slot_busy[slot] = true;
    kc.in_flight++;
    if (dry) {
        steps.push_back(st);
        return true;
    }
    // step table into the class's slot: descriptors, the pieces' first items, their
    // descriptor ranges (set classes), XCD queue bounds, queue heads
    std::vector<int32_t> qb;
    queue_bounds(leaders, items, &qb);
    if (kc.sets)
        sfirst.push_back((int32_t)tab.size());
    const size_t o_starts = align_up(sizeof(ChunkDesc) * tab.size(), 16);
    const size_t o_sets = o_starts + align_up(sizeof(int32_t) * starts.size(), 16);
    const size_t o_qb = o_sets + align_up(sizeof(int32_t) * sfirst.size(), 16);
    const size_t tb = o_qb + sizeof(int32_t) * qb.size();
    char *h = static_cast<char *>(kc.stage[slot]);
    std::memcpy(h, tab.data(), sizeof(ChunkDesc) * tab.size());
    std::memcpy(h + o_starts, starts.data(), sizeof(int32_t) * starts.size());
    if (!sfirst.empty())
        std::memcpy(h + o_sets, sfirst.data(), sizeof(int32_t) * sfirst.size());
    std::memcpy(h + o_qb, qb.data(), sizeof(int32_t) * qb.size());
    char *dtab = arena + kc.table_off[slot];
    hipStream_t sm = kc.stream[slot];
    hipError_t e = hipMemcpyAsync(dtab, h, tb, hipMemcpyHostToDevice, sm);
    int32_t *ctr = reinterpret_cast<int32_t *>(dtab + align_up(tb, 16));
    if (e == hipSuccess)
        e = launch_fill_i32(ctr, 0, kQueues, sm);
    SearchArgs a{};
    a.base = reinterpret_cast<const float *>(arena);
    a.chunks = reinterpret_cast<const ChunkDesc *>(dtab);
    a.item_start = reinterpret_cast<const int32_t *>(dtab + o_starts);
    a.n_parts = kQueues;
    a.part_start = reinterpret_cast<const int32_t *>(dtab + o_qb);
    a.n_chunks = (int32_t)starts.size();
    a.set_first = kc.sets ? reinterpret_cast<const int32_t *>(dtab + o_sets) : nullptr;
    a.n_items = (int32_t)items;
    a.k = kc.k;
    a.counter = ctr;
    a.partial = reinterpret_cast<double *>(arena);
    a.sorted = kc.sorted ? 1 : 0;
    const int64_t full = (int64_t)dev.n_cu * kc.cfg.wg_per_cu * kc.cfg.waves_per_wg;
    if (e == hipSuccess)
        e = launch_search_timed(a, kc.d_y, kc.d_x, kc.cfg, (int)std::max<int64_t>(1, std::min<int64_t>(full, items)),
                                sm);
    // reductions of the jobs this step completes, behind it on the same stream; a job's
    // earlier blocks may sit in the previous step on the other stream, so wait for it first
    if (e == hipSuccess && !finishing.empty())
        e = hipStreamWaitEvent(sm, kc.last_ev[1 - slot], 0);
    for (Job *j : finishing) {
        if (e != hipSuccess)
            break;
        Batch &b = j->batch;
        char *bat = arena + j->region + j->off_batch;
        const ChunkDesc *jc = reinterpret_cast<const ChunkDesc *>(bat + b.off_chunks);
        const int32_t *jctr = reinterpret_cast<const int32_t *>(bat + b.off_ctr);
        double *res = reinterpret_cast<double *>(bat + b.off_results);
        double *pv = reinterpret_cast<double *>(bat + b.off_pv);
        e = launch_reduce(jc, (int)b.chunks.size(), reinterpret_cast<const double *>(arena), kc.k, jctr + 1, res,
                          sm);
        if (e == hipSuccess)
            e = launch_pvalues(res, b.n_groups, b.n_surr, pv, sm);
        char *out = static_cast<char *>(j->stage);
        if (e == hipSuccess)
            e = hipMemcpyAsync(out, res, sizeof(double) * b.n_results, hipMemcpyDeviceToHost, sm);
        if (e == hipSuccess)
            e = hipMemcpyAsync(out + sizeof(double) * b.n_results, pv, sizeof(double) * b.n_groups,
                               hipMemcpyDeviceToHost, sm);
        if (e == hipSuccess)
            e = hipMemcpyAsync(out + sizeof(double) * (b.n_results + b.n_groups), jctr + 1, sizeof(int32_t),
                               hipMemcpyDeviceToHost, sm);
        if (e == hipSuccess)
            e = hipEventRecord(j->done_ev, sm);
    }
    if (e == hipSuccess)
        e = hipEventCreateWithFlags(&st.ev, hipEventDisableTiming);
    if (e == hipSuccess)
        e = hipEventRecord(st.ev, sm);
    if (e == hipSuccess)
        e = hipEventRecord(kc.last_ev[slot], sm);
    if (e == hipSuccess)
        e = hipLaunchHostFunc(sm, host_wake, this);
    if (e != hipSuccess) {
        // every job with blocks in this step lacks some partial sums: it fails, and is
        // released once the class's streams (its earlier steps) have drained
        const char *msg = hipGetErrorString(e);
        drain_streams(&kc);
        st.finishing.clear();
        for (Job *j : members) {
            fail_job(j, TE_ERR_DEVICE, msg);
            j->all_scheduled = true;
            st.finishing.push_back(j->id);
        }
        if (st.ev)
            hipEventDestroy(st.ev);
        st.ev = nullptr;
    }
    steps.push_back(st);
    return true;
}

void Server::finish(Job *j)
{
    TraceRange trace_range("te.serve.finish");
    const Batch &b = j->batch;
    const te_problem &p = j->plan->impl.p;
    const int G = p.n_pairs * p.n_points;
    j->te_orig.assign(G, NAN);
    j->te_surr.assign((size_t)G * p.n_surrogates, NAN);
    j->pv.assign(G, NAN);
    if (!dry && j->state != FAILED) {
        const char *out = static_cast<const char *>(j->stage);
        const double *res = reinterpret_cast<const double *>(out);
        const double *pv = res + b.n_results;
        int32_t err = 0;
        std::memcpy(&err, out + sizeof(double) * (b.n_results + b.n_groups), sizeof err);
        for (int gi = 0; gi < b.n_groups; ++gi) {
            const int g = b.groups[gi];
            const double *r = res + (size_t)gi * (b.n_surr + 1);
            j->te_orig[g] = r[0];
            for (int s = 0; s < b.n_surr; ++s)
                j->te_surr[(size_t)g * b.n_surr + s] = r[1 + s];
            j->pv[g] = pv[gi];
        }
        if (err)
            fail_job(j, TE_ERR_INVALID, "non-finite input value or invalid surrogate permutation");
    }
    j->t_done = now_s();
    if (j->state != FAILED) {
        j->state = DONE;
        completed++;
        est_done += (int64_t)G * (p.n_surrogates + 1);
        lat.push_back(j->t_done - j->t_submit);
        t_last = j->t_done;
    } else {
        failed++;
    }
    release(j);
}

// Retire every finished step (steps of one class finish in issue order on its stream).
void Server::poll_steps()
{
    for (auto it = steps.begin(); it != steps.end();) {
        StepRec &st = *it;
        if (!dry && st.ev && hipEventQuery(st.ev) != hipSuccess) {
            ++it;
            continue;
        }
        for (uint64_t id : st.finishing) {
            auto jt = jobs.find(id);
            if (jt != jobs.end() && jt->second->state != CANCELLED && jt->second->state != DONE &&
                jt->second->footprint != 0) {
                Job *j = jt->second.get();
                // the result copy was recorded before the step's event on the same stream
                if (!dry && j->done_ev && j->state != FAILED)
                    hipEventSynchronize(j->done_ev);
                finish(j);
            }
        }
        if (!dry && st.ev)
            hipEventDestroy(st.ev);
        classes[st.cls].in_flight--;
        classes[st.cls].slot_busy[st.slot] = false;
        it = steps.erase(it);
        cv_done.notify_all();
    }
}

void Server::loop()
{
    std::unique_lock<std::mutex> lk(mu);
    while (true) {
        if (stopping && queue.empty() && resident.empty() && steps.empty())
            break;
        // admission: FIFO, no overtaking
        while (!held && !queue.empty() && (int)resident.size() < max_slots) {
            Job *j = queue.front();
            if (j->state == CANCELLED) {
                queue.pop_front();
                continue;
            }
            if (!admit_one(j))
                break;
            queue.pop_front();
            if (j->state == FAILED) {
                j->t_done = now_s();
                failed++;
                release(j);
                cv_done.notify_all();
            }
        }
        if (!dry)
            poll_setup();
        // At most two steps in flight over all classes (the second covers the tail of the
        // first); each new step goes to the class of the oldest resident job with blocks left
        // to schedule, so jobs progress in admission order across classes as within one and a
        // job is not slowed by younger jobs of other classes sharing the GPU.
        bool issued = false;
        for (;;) {
            int total = 0;
            for (const KernelClass &c : classes)
                total += c.in_flight;
            if (total >= 2)
                break;
            int ci = -1;
            for (Job *j : resident)
                if (j->state == READY && !j->all_scheduled && classes[j->cls].in_flight < 2) {
                    ci = j->cls;
                    break;
                }
            if (ci < 0 || !issue_step(ci))
                break;
            issued = true;
        }
        poll_steps();
        const bool busy = !steps.empty() || !queue.empty() ||
                          std::any_of(resident.begin(), resident.end(), [](Job *j) { return j->state == SETUP; });
        if (!busy && !issued) {
            if (stopping && resident.empty() && queue.empty())
                break;
            sleep_until_woken(lk, 50);
        } else if (!issued) {
            // device work in flight: its completion wakes the thread (the timeout is a backstop)
            sleep_until_woken(lk, dry ? 1 : 10);
        }
    }
}

te_status Server::start()
{
    if (!dry) {
        te_status st = current_device(&dev);
        if (st != TE_OK)
            return st;
        hipError_t e = hipStreamCreateWithFlags(&setup_stream, hipStreamNonBlocking);
        if (e != hipSuccess)
            return hip_fail(e, "hipStreamCreate");
    } else {
        dev.n_cu = 256;
    }
    alloc.init(arena_bytes);
    if (const char *f = std::getenv("TE_SERVE_FAULT_STAGING"))
        fault_staging = std::atoll(f);
    thr = std::thread([this] { loop(); });
    return TE_OK;
}

}  // namespace te

struct te_server_s {
    te::Server impl;
};

using namespace te;

extern "C" {

te_status te_serve_open(void *arena, size_t arena_bytes, int32_t max_slots, int32_t max_queue, int64_t step_pairs,
                        int32_t flags, te_server *out)
{
    clear_error();
    if (!out)
        return fail(TE_ERR_INVALID, "null argument");
    *out = nullptr;
    const bool dry = (flags & TE_SERVE_DRY_RUN) != 0;
    if ((!arena && !dry) || arena_bytes < 4096 || max_slots < 1 || max_queue < 1)
        return fail(TE_ERR_INVALID, "need an arena of >= 4096 bytes, max_slots >= 1 and max_queue >= 1");
    auto s = std::make_unique<te_server_s>();
    Server &S = s->impl;
    S.arena = static_cast<char *>(arena);
    S.arena_bytes = arena_bytes;
    S.max_slots = max_slots;
    S.max_queue = max_queue;
    S.step_pairs = step_pairs > 0 ? step_pairs : (int64_t)4000000000LL;
    S.dry = dry;
    S.held = (flags & TE_SERVE_HOLD) != 0;
    te_status st = S.start();
    if (st != TE_OK)
        return st;
    *out = s.release();
    return TE_OK;
}

te_status te_serve_submit(te_server srv, const te_problem *problem, const float *x, const float *y,
                          const int32_t *perms, uint64_t *ticket)
{
    clear_error();
    if (!srv || !problem || !x || !y || !ticket)
        return fail(TE_ERR_INVALID, "null argument");
    Server &S = srv->impl;
    auto j = std::make_unique<Job>();
    te_plan pl = nullptr;
    te_status st = te_plan_create(problem, &pl);
    if (st != TE_OK)
        return st;
    j->plan.reset(pl);
    const Plan &P = pl->impl;
    const bool caller_perms = P.p.n_surrogates > 0 && perms != nullptr;
    j->batch = P.full;
    j->footprint = job_footprint(P, caller_perms, &j->batch, &j->off_x, &j->off_y, &j->off_perm, &j->off_batch);
    if (j->footprint > S.alloc.size)
        return fail(TE_ERR_NOMEM, "job needs %zu bytes, the arena holds %zu", j->footprint, S.alloc.size);
    // stage the inputs in pinned memory now, on the submitting thread, so the
    // server's uploads are asynchronous copies
    j->n_series = (size_t)P.p.n_pairs * P.p.n_trials * P.p.n_samples;
    j->n_perm = caller_perms ? (size_t)P.p.n_pairs * P.p.n_points * P.p.n_surrogates * P.p.n_trials : 0;
    j->hin_y = align_up(sizeof(float) * j->n_series, 256);
    j->hin_perm = j->hin_y + align_up(sizeof(float) * j->n_series, 256);
    j->hin_bytes = j->hin_perm + sizeof(int32_t) * j->n_perm;
    if (!S.dry) {
        j->hin = S.pool.take(j->hin_bytes);
        if (!j->hin)
            return fail(TE_ERR_NOMEM, "pinned staging allocation failed");
        char *h = static_cast<char *>(j->hin);
        std::memcpy(h, x, sizeof(float) * j->n_series);
        std::memcpy(h + j->hin_y, y, sizeof(float) * j->n_series);
        if (j->n_perm)
            std::memcpy(h + j->hin_perm, perms, sizeof(int32_t) * j->n_perm);
    }
    std::lock_guard<std::mutex> lk(S.mu);
    auto reject = [&](te_status st2, const char *msg) {
        if (j->hin)
            S.pool.give(j->hin);
        j->hin = nullptr;
        return fail(st2, "%s", msg);
    };
    if (S.stopping)
        return reject(TE_ERR_CANCELLED, "server is closing");
    if ((int)S.queue.size() >= S.max_queue)
        return reject(TE_ERR_BUSY, "queue full");
    j->id = S.next_id++;
    j->t_submit = now_s();
    if (S.t_first == 0)
        S.t_first = j->t_submit;
    j->cls = S.class_of(P.p, P.sorted, P.full.use_sets, P.full.set_v);
    {
        // the job, with its class's step tables, must fit beside the tables of every other
        // class: they stay allocated once a job of theirs is admitted, and a class with jobs
        // queued ahead of this one will be before it is
        size_t others = 0;
        for (size_t c = 0; c < S.classes.size(); ++c)
            if ((int)c != j->cls)
                others += 2 * align_up(S.classes[c].table_cap, 256);
        const size_t own = 2 * align_up(S.classes[j->cls].table_cap, 256);
        if (align_up(j->footprint, 256) + own + others > S.alloc.size)
            return reject(TE_ERR_NOMEM, "the job and the step tables of its kernel class cannot fit the arena");
    }
    *ticket = j->id;
    S.queue.push_back(j.get());
    S.jobs[j->id] = std::move(j);
    S.wake_up();
    return TE_OK;
}

te_status te_serve_wait(te_server srv, uint64_t ticket, int64_t timeout_us, double *te_orig, double *te_surr,
                        double *p_value)
{
    clear_error();
    if (!srv)
        return fail(TE_ERR_INVALID, "null server");
    Server &S = srv->impl;
    std::unique_lock<std::mutex> lk(S.mu);
    auto it = S.jobs.find(ticket);
    if (it == S.jobs.end())
        return fail(TE_ERR_INVALID, "unknown ticket %llu", (unsigned long long)ticket);
    Job *j = it->second.get();
    auto terminal = [&] { return j->state == DONE || j->state == FAILED || j->state == CANCELLED; };
    if (timeout_us < 0)
        S.cv_done.wait(lk, terminal);
    else if (!S.cv_done.wait_for(lk, std::chrono::microseconds(timeout_us), terminal))
        return fail(TE_ERR_TIMEOUT, "ticket %llu not finished", (unsigned long long)ticket);
    te_status st = TE_OK;
    if (j->state == DONE) {
        if (te_orig)
            std::copy(j->te_orig.begin(), j->te_orig.end(), te_orig);
        if (te_surr)
            std::copy(j->te_surr.begin(), j->te_surr.end(), te_surr);
        if (p_value)
            std::copy(j->pv.begin(), j->pv.end(), p_value);
    } else if (j->state == CANCELLED) {
        st = fail(TE_ERR_CANCELLED, "ticket %llu was cancelled", (unsigned long long)ticket);
    } else {
        st = fail(j->status, "%s", j->error.c_str());
    }
    S.jobs.erase(it);
    return st;
}

te_status te_serve_cancel(te_server srv, uint64_t ticket)
{
    clear_error();
    if (!srv)
        return fail(TE_ERR_INVALID, "null server");
    Server &S = srv->impl;
    std::lock_guard<std::mutex> lk(S.mu);
    auto it = S.jobs.find(ticket);
    if (it == S.jobs.end())
        return fail(TE_ERR_INVALID, "unknown ticket");
    Job *j = it->second.get();
    if (j->state != QUEUED)
        return fail(TE_ERR_BUSY, "ticket %llu is already admitted", (unsigned long long)ticket);
    j->state = CANCELLED;
    S.queue.erase(std::remove(S.queue.begin(), S.queue.end(), j), S.queue.end());
    S.cancelled++;
    S.cv_done.notify_all();
    return TE_OK;
}

te_status te_serve_resume(te_server srv)
{
    clear_error();
    if (!srv)
        return fail(TE_ERR_INVALID, "null server");
    Server &S = srv->impl;
    std::lock_guard<std::mutex> lk(S.mu);
    S.held = false;
    S.wake_up();
    return TE_OK;
}

te_status te_serve_stats(te_server srv, te_serve_stats_t *out)
{
    clear_error();
    if (!srv || !out)
        return fail(TE_ERR_INVALID, "null argument");
    Server &S = srv->impl;
    std::lock_guard<std::mutex> lk(S.mu);
    std::vector<double> l = S.lat;
    std::sort(l.begin(), l.end());
    auto q = [&](double f) {
        if (l.empty())
            return (double)NAN;
        const size_t i = std::min(l.size() - 1, (size_t)std::ceil(f * l.size()) - (f * l.size() >= 1 ? 1 : 0));
        return l[i];
    };
    out->p50_s = q(0.50);
    out->p99_s = q(0.99);
    out->est_per_s = (S.t_last > S.t_first) ? (double)S.est_done / (S.t_last - S.t_first) : 0.0;
    out->completed = S.completed;
    out->failed = S.failed;
    out->cancelled = S.cancelled;
    out->steps = S.n_steps;
    out->queued = (int64_t)S.queue.size();
    out->resident = (int64_t)S.resident.size();
    out->peak_slots = S.peak_slots;
    out->peak_bytes = (int64_t)S.alloc.peak;
    return TE_OK;
}

te_status te_serve_close(te_server srv)
{
    if (!srv)
        return TE_OK;
    Server &S = srv->impl;
    {
        std::lock_guard<std::mutex> lk(S.mu);
        S.stopping = true;
        for (Job *j : S.queue) {
            j->state = CANCELLED;
            S.cancelled++;
        }
        S.queue.clear();
        S.wake_up();
        S.cv_done.notify_all();
    }
    if (S.thr.joinable())
        S.thr.join();
    for (auto &c : S.classes)
        for (int sl = 0; sl < 2; ++sl) {
            if (c.stream[sl])
                hipStreamDestroy(c.stream[sl]);
            if (c.last_ev[sl])
                hipEventDestroy(c.last_ev[sl]);
        }
    if (S.setup_stream)
        hipStreamDestroy(S.setup_stream);
    delete srv;
    return TE_OK;
}

}  // extern "C"
