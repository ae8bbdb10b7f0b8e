// te_runtime.h -- host-side plan, batch and execution state of libte.
#pragma once

#include <hip/hip_runtime.h>
#include <rocprofiler-sdk-roctx/roctx.h>

#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include "te.h"
#include "te_internal.h"

namespace te {

// A rocTX range over a host phase of the scheduler (planning, batch layout, enqueue,
// graph capture, serving admission and steps, tuning): shown by `rocprofv3
// --marker-trace`, a no-op without a profiler attached.  Ranges nest per thread.
struct TraceRange {
    explicit TraceRange(const char *name) { roctxRangePushA(name); }
    ~TraceRange() { roctxRangePop(); }
    TraceRange(const TraceRange &) = delete;
    TraceRange &operator=(const TraceRange &) = delete;
};

te_status fail(te_status st, const char *fmt, ...);
te_status hip_fail(hipError_t e, const char *what);
void clear_error();
te_status current_device(DeviceInfo *out);
SearchConfig default_config(const DeviceInfo &dev, int d_y, int d_x, int k, int64_t n);
size_t align_up(size_t v, size_t a);
int size_bucket(int64_t n);
bool sorting_enabled();
int sort_npad(int n);
void queue_bounds(const std::vector<ChunkDesc> &pieces, int64_t n_items, std::vector<int32_t> *part_start);
te_status knn_counts_run(const float *pts, int64_t dim_stride, const int64_t *offsets, int32_t n_chunks, int32_t d_y,
                         int32_t d_x, int32_t k, char *ws, size_t ws_bytes, hipStream_t st, float *eps,
                         int32_t *counts, double *te_out, bool pinned_staging, const char *ws_name);

// A set of chunks laid out in one device workspace, with the host copy of its
// tables.  Chunks are stored in schedule (longest-first) order.
struct Batch {
    std::vector<int> groups;              // (pair * n_points + point) of each group
    int n_groups = 0;
    int n_surr = 0;
    int n_results = 0;                    // n_groups * (n_surr + 1)
    int64_t n_floats = 0;                 // coordinate storage
    std::vector<ChunkDesc> chunks;
    std::vector<int> order;
    std::vector<int32_t> item_start;
    std::vector<EmbedTask> tasks;
    std::vector<PermTask> perm_tasks;     // one per surrogate chunk: its trial permutation
    int64_t n_perm = 0;                   // int32 entries of the batch's permutation area
    std::vector<SortTask> sorts;          // one per window group (empty when chunks are not sorted)
    int64_t n_sigma = 0;                  // int32 entries of the sorted-to-original maps
    int64_t n_scratch = 0;                // uint64 sort scratch entries
    int64_t n_items = 0;
    bool use_sets = false;                // chunk-set search: a window's chunks set_v at a time
    int set_v = 1;                        // chunks per set (set_variants of the plan's dimensions)
    std::vector<int32_t> set_first;       // [n_sets + 1] chunk range of each set (use_sets)
    int64_t n_partials = 0;               // per-item partial sums: one per 64-point block of every chunk
    std::vector<int32_t> part_start;      // [kQueues + 1] item ranges of the XCD work queues
    // byte offsets inside the workspace
    size_t off_coords = 0, off_tables = 0, off_chunks = 0, off_items = 0, off_tasks = 0, off_ptasks = 0,
           off_perm = 0, off_sorts = 0, off_partial = 0, off_results = 0, off_pv = 0, off_ctr = 0, off_sigma = 0,
           off_scratch = 0, off_parts = 0, off_qctr = 0, off_errout = 0, off_sets = 0;
    size_t tables_bytes = 0;
    size_t total_bytes = 0;
    std::vector<char> host_tables;

    void finish_layout();
    size_t stage_bytes() const;
};

// Pinned host staging buffers (table uploads, result downloads), reused across calls.
struct PinnedPool {
    struct Buf {
        void *ptr = nullptr;
        size_t bytes = 0;
        bool busy = false;
    };
    std::mutex mu;
    std::vector<Buf> bufs;
    void *take(size_t bytes);
    void give(void *ptr);
    ~PinnedPool();
};

struct GraphEntry {
    const void *x = nullptr, *y = nullptr, *perms = nullptr, *ws = nullptr;
    hipStream_t stream = nullptr;
    size_t ws_bytes = 0;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    std::vector<Batch> batches;
    std::vector<void *> stages;
};

// Variants of a window group in one batch: by default the original and the
// n_surr trial-shuffled surrogates.
struct BatchOptions {
    bool local_outputs = false;                   // per-point local TE of the originals
    const std::vector<int32_t> *delays = nullptr; // variants: the original at each of these source delays
    bool delay_from_device = false;               // source delay of group gi read from u_dev[gi]
    bool allow_sets = true;                       // chunk-set search where the plan allows it
};

// Byte offsets of the plain per-chunk path's workspace (Plan::plain_layout).
struct PlainLayout {
    size_t coords = 0, partial = 0, results = 0, pv = 0, ctr = 0, tables = 0, sigma = 0, perm = 0, scratch = 0;
    size_t t_chunks = 0, t_items = 0, t_tasks = 0, t_sorts = 0, t_perms = 0, tables_bytes = 0;
    size_t total = 0;
};

struct Plan {
    te_problem p{};
    bool sorted = true;                   // chunks sorted by the first target-past coordinate (TE_NO_SORT=1: off)
    std::vector<int32_t> wstart, wlen, trials;
    std::vector<int64_t> npts;
    std::vector<int64_t> local_off;       // [n_pairs * n_points + 1] offsets of the local-TE output
    mutable std::mutex dev_mu;
    mutable bool dev_ready = false;
    mutable DeviceInfo dev;
    mutable SearchConfig cfg{};
    Batch full;
    size_t min_bytes = 0;
    size_t plain_bytes = 0;

    mutable PinnedPool pool;
    mutable std::mutex async_mu;
    mutable void *async_tables = nullptr;  // pinned, immutable copy of full.host_tables (te_surrogates_async)
    mutable std::mutex graph_mu;
    mutable std::vector<GraphEntry> graphs;

    ~Plan();
    // target-past coordinates the search sees: d_y, plus x_t when conditioning on it
    int dy_eff() const { return p.d_y + p.cond_source; }
    te_status ensure_device() const;
    te_status build_group_batch(const std::vector<int> &groups, int n_surr, Batch *b,
                                const BatchOptions &opt = BatchOptions()) const;
    int grid_waves(int64_t n_items) const;
    // the window's chunks can be searched as sets (sorted, k = 4, no x_t in the target block)
    bool sets_eligible() const;
    // launch shape of a batch: the plan's, with the resident workgroups capped at the
    // chunk-set search's occupancy for batches that use it
    SearchConfig batch_config(const Batch &b) const;
    // tables_src: upload the tables from this pinned copy instead of through `stage`;
    // out_dst: copy the results block (estimates [group][original, surrogates], then
    // p-values) there (device or pinned host) instead of into `stage`.
    te_status enqueue_batch(const Batch &b, const float *x, const float *y, const int32_t *perms, char *ws,
                            void *stage, hipStream_t st, double *lte_out = nullptr,
                            const int32_t *u_dev = nullptr, const void *tables_src = nullptr,
                            void *out_dst = nullptr) const;
    te_status run_surrogates_async(const float *x, const float *y, const int32_t *perms, char *ws, size_t ws_bytes,
                                   hipStream_t st, double *out) const;
    size_t scan_bytes(const std::vector<int> &groups, const std::vector<int32_t> &delays) const;
    te_status run_scan(const float *x, const float *y, const int32_t *perms, const std::vector<int32_t> &delays,
                       char *ws, size_t ws_bytes, hipStream_t st, double *te_scan, int32_t *u_best,
                       double *te_surr, double *p_value) const;
    te_status run_local(const float *x, const float *y, char *ws, size_t ws_bytes, hipStream_t st, double *lte,
                        double *te_out) const;
    te_status unpack_batch(const Batch &b, const void *stage, double *te_orig, double *te_surr, double *p_value,
                           bool *bad_input) const;
    te_status split_batches(size_t ws_bytes, std::vector<Batch> *out) const;
    te_status run_surrogates(const float *x, const float *y, const int32_t *perms, char *ws, size_t ws_bytes,
                             hipStream_t st, bool use_graph, double *te_orig, double *te_surr,
                             double *p_value) const;
    PlainLayout plain_layout(int n_surr) const;
    te_status estimate_each(const float *x, const float *y, const int32_t *perms, int n_surr, char *ws,
                            size_t ws_bytes, hipStream_t st, double *te_orig, double *te_surr,
                            double *p_value) const;
};

}  // namespace te

struct te_plan_s {
    te::Plan impl;
};
