// te_internal.h -- structures shared by the host runtime and the HIP kernels of libte.
#pragma once

#include <hip/hip_runtime_api.h>
#include <stddef.h>
#include <stdint.h>

namespace te {

// Largest supported embedding dimensions and neighbour count.
constexpr int kMaxDimY = 4;
constexpr int kMaxDimX = 4;
constexpr int kMaxK = 15;
constexpr int kWave = 64;                 // wavefront width on gfx950
constexpr int kMaxWavesPerWG = 4;         // search kernel workgroup: up to 4 independent waves

// One search space ("chunk", eq. 10 pooled points) as the kernels see it.
// Coordinate m of point j lives at
//   base[tp + m * ld + j]                 for m <  1 + d_y  (y_t' and target past)
//   base[s + (m - 1 - d_y) * ld + j]      for m >= 1 + d_y  (source past)
// so the originals and surrogates of one window share the (y_t', Y_past) block.
struct ChunkDesc {
    int64_t tp;       // float offset of the target block
    int64_t s;        // float offset of the source block
    int64_t ld;       // stride between coordinates, in floats
    int64_t out;      // per-point output offset (eps / counts), or -1
    int64_t pbase;    // index in the partial-sum array of the chunk's block 0
    int64_t perm;     // offset in perm_base of the sorted-to-original point map, or -1
    int32_t n;        // points in the chunk
    int32_t item0;    // launch work-item index of the first scheduled block
    int32_t block0;   // first scheduled block (64 references) of the chunk
    int32_t result;   // slot of the chunk's estimate in the result array
};

// Work for the embedding kernel: writes one chunk's source block, and the
// target block when tp >= 0.
struct EmbedTask {
    int64_t tp;       // float offset of the target block, or -1
    int64_t s;        // float offset of the source block
    int64_t perm;     // int32 offset of the source permutation row in the batch's permutation area, or -1 (identity)
    int64_t sig;      // int32 offset of the window's sorted-to-original point map, or -1 (identity)
    int32_t pair, w, W, Rc;
    int32_t n;        // Rc * W
    int32_t u;        // source delay of this block; 0: the launch's delay
    int32_t u_slot;   // > 0: the delay is read on the device from u_dev[u_slot - 1] (overrides u)
    int32_t pad_;
};

// One surrogate's trial permutation in a batch's permutation area.  It is either
// copied from the caller's [pair][point][surrogate][trial] array (and checked to
// be a permutation of 0..rc-1) or drawn on the device from the problem's seed,
// keyed by (pair, point, surr).  Entries rc..len-1 of a written row are the
// identity.
struct PermTask {
    int64_t src;      // int32 offset of the row in the caller's array (copy mode)
    int64_t dst;      // int32 offset of the row in the destination
    int32_t rc;       // trials pooled by the window: the row permutes 0..rc-1
    int32_t len;      // entries written (>= rc)
    int32_t pair, point, surr, pad_;
};

// Sorting of one search space by its first target-past coordinate p0.  The
// result sigma[sig + q] is the original index of the point at sorted position q.
// Keys are (order-preserving bits of p0) << 32 | original index: a total order,
// so the permutation is unique.
struct SortTask {
    int64_t sig;      // int32 offset of the output map
    int64_t scratch;  // uint64 offset of global key scratch (npad > kSortLds), else -1
    int64_t key_off;  // mode 1: float offset of the key coordinate (point q at key_off + q)
    int32_t mode;     // 0: key = y[pair][r][t'-1] of window point q = r W + (t' - w); 1: stored coordinate
    int32_t pair, w, W, Rc, n, npad, pad_;
};
constexpr int kSortLds = 16384;   // keys sorted in LDS (128 KiB) up to this many (padded) points

// Copy of one pre-embedded chunk into sorted order: dst[dst + m n + q] = src[src + m ld + sigma[sig + q]].
struct GatherTask {
    int64_t src, ld, dst, sig;
    int32_t n, pad_;
};

// Arguments of the search kernel (passed by value; read from the kernarg segment).
struct SearchArgs {
    const float *base;          // coordinate storage
    const ChunkDesc *chunks;    // [n_chunks] in schedule order
    const int32_t *item_start;  // [n_chunks] chunks[c].item0, ascending
    int32_t n_chunks;
    int32_t n_items;
    int32_t k;
    int32_t pad_;
    int32_t *counter;           // work-queue head, zero before launch
    double *partial;            // [n_items] per-item sum of psi terms
    float *eps_out;             // optional per-point radius
    int32_t *cnt_out;           // optional per-point counts [3][cnt_stride]
    int64_t cnt_stride;
    const int32_t *perm_base;   // sorted-to-original point maps (per-point outputs only)
    unsigned long long *work;   // optional: [0] += pairs evaluated in pass 1, [1] += in pass 2 (a pair per chunk),
                                // [2], [3] += the same counted once per set of chunks
    double *lte_out;            // optional per-point local TE (at out + original index)
    int32_t sorted;             // chunks are sorted by the first target-past coordinate
    int32_t n_parts;            // > 1: items split into n_parts queues (counter[p] heads queue p), see kQueues
    const int32_t *part_start;  // [n_parts + 1] first item of each queue (n_parts > 1)
    const int32_t *set_first;   // non-null: chunk-set search; n_chunks counts sets, set c holds the chunks
                                // [set_first[c], set_first[c+1]) (at most set_variants(d_y, d_x)), item_start is per set
};

// Chunks of one window searched together by the chunk-set search (they share the
// (y_t', Y_past) block and its order and differ in the source block): as many as
// keep a group of four candidates' coordinates, 4 (1 + d_y + V d_x) values, within
// 64 scalar registers, two to four.
constexpr int set_variants(int d_y, int d_x)
{
    return (15 - d_y) / d_x >= 4 ? 4 : ((15 - d_y) / d_x <= 2 ? 2 : (15 - d_y) / d_x);
}
constexpr int kMaxSetVariants = 4;

// Points per window (pooled chunk) at most: the set search addresses coordinate m of a
// block as a 32-bit byte offset 4 (m ld + j) from the block's start, m <= 4 and ld = N.
constexpr int kMaxWindowPoints = 1 << 27;

// Work queues of a batched search: one per XCD of an MI355X.  Workgroups are
// dispatched to the XCDs round-robin, so the waves of workgroup g start on queue
// g % kQueues and a chunk's coordinates stay in one XCD's L2; a wave whose queue
// is empty moves on to the next one.
constexpr int kQueues = 8;

// Tunable launch shape of the search kernel.
struct SearchConfig {
    int slots;        // candidate slots per lane in the counting pass (4 or 8)
    int waves_per_wg; // independent wavefronts per workgroup
    int wg_per_cu;    // persistent workgroups per compute unit
};

struct DeviceInfo {
    int device = -1;
    int n_cu = 0;
    char arch[64] = {0};
};

// Kernel launchers (te_kernels.hip).  All return hipSuccess or the launch error.
hipError_t launch_fill_i32(int32_t *p, int32_t v, int64_t n, hipStream_t st);
hipError_t launch_embed(const float *x, const float *y, const int32_t *perms, const int32_t *sigma,
                        const int32_t *u_dev, const EmbedTask *tasks, int n_tasks, int max_n, float *base, int R,
                        int T, int d_y, int d_x, int tau, int u, int cond, int32_t *err, hipStream_t st);
hipError_t launch_sort(const float *y, const float *pts, const SortTask *tasks, int n_tasks, int32_t *sigma,
                       uint64_t *scratch, int R, int T, hipStream_t st);
hipError_t launch_gather(const float *src, const GatherTask *tasks, int n_tasks, const int32_t *sigma, float *dst,
                         int D, hipStream_t st);
// Fill a batch's permutation area: copy (and check) the caller's rows when src is
// given, else draw every row from `seed`.  Sets bit 2 of *err for an invalid row.
hipError_t launch_perms(const int32_t *src, const PermTask *tasks, int n_tasks, int32_t *dst,
                        uint64_t seed, int32_t *err, hipStream_t st);
hipError_t launch_search(const SearchArgs &a, int d_y, int d_x, const SearchConfig &cfg, int grid_waves,
                         hipStream_t st);
// With pv != nullptr the launch also computes the n_groups p-values (results laid
// out [group][original, surrogates...]; NaN when *err is set) and copies *err to
// *err_out when that is given: in its last-finishing workgroup, counted on `done`
// (zero before the launch), for small grids, else in a second kernel.
hipError_t launch_reduce(const ChunkDesc *chunks, int n_chunks, const double *partial, int k,
                         const int32_t *err, double *results, hipStream_t st, int n_groups = 0, int n_surr = 0,
                         double *pv = nullptr, int32_t *done = nullptr, int32_t *err_out = nullptr);
hipError_t launch_pvalues(const double *results, int n_groups, int n_surr, double *pv, hipStream_t st);
hipError_t launch_argmax_u(const double *results, int n_groups, int n_u, const int32_t *u_values, int32_t *u_sel,
                           hipStream_t st);
bool search_supported(int d_y, int d_x, int k, int slots);
bool search_sets_supported(int d_y, int d_x, int k);
// Resident workgroups per compute unit of the chunk-set search (0 if unknown).
int search_sets_occupancy(int d_y, int d_x, int slots, int waves_per_wg);
unsigned long long *work_counters();   // this device's evaluated-pair counters [4] (measurement)

// Search launch bracketed by profiling events when measurement is enabled (te_profile.cpp).
hipError_t launch_search_timed(const SearchArgs &a, int d_y, int d_x, const SearchConfig &cfg, int grid_waves,
                               hipStream_t st);

}  // namespace te
