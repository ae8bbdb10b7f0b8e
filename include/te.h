/*
 * te.h -- C interface of libte, ensemble transfer entropy (KSG estimator) on
 * AMD Instinct MI355X (gfx950).
 *
 * The library estimates TE_SPO(X -> Y, t, u) = I(Y_t ; X^{d_x}_{t-u} | Y^{d_y}_{t-1})
 * (Wollstadt et al. 2014, eq. 3) for every analysis time point of an ensemble
 * of repetitions (Background, eq. 1-2), with the ensemble KSG estimator of
 * eq. 9, pooled over a window of samples as in eq. 10, and tests it against
 * repetition-shuffled surrogates (Fig. 3; "TE calculation and statistical
 * testing against surrogate data").
 *
 * Conventions for every entry point
 *   - Return value: te_status.  TE_OK on success; otherwise te_last_error()
 *     returns a message for the calling thread.  No exception crosses the ABI.
 *   - "device" pointers are HIP device (HBM) addresses; "host" pointers are
 *     ordinary process memory.  The caller owns every buffer it passes in and
 *     keeps it alive until the call returns (or, for te_serve_submit, as stated
 *     there).  The library allocates no device memory on these paths: all
 *     device scratch space lives in the caller's workspace.
 *   - hip_stream is a hipStream_t (NULL = the default stream).  Calls enqueue
 *     their work on it; calls that write host outputs synchronise the stream
 *     before they return.
 *   - Series are float32, laid out [n_pairs][n_trials][n_samples] row-major:
 *     element (p, r, t) is the observation at sample t of repetition r of
 *     pair p.  Values must be finite: a NaN or Inf met while embedding makes
 *     the call return TE_ERR_INVALID (outputs are then NaN).
 *
 * Semantics fixed by the library (readings of points the paper leaves open)
 *   - embedding (eq. 6-7 and the remark that the source is embedded the same
 *     way at t-u): the point of repetition r at sample t' is
 *     ( y_t' | y_{t'-1}, y_{t'-1-tau}, ..., y_{t'-1-(d_y-1)tau}
 *            | x_{t'-u}, x_{t'-u-tau}, ..., x_{t'-u-(d_x-1)tau} );
 *   - a window pools repetitions r < R_c and samples t' in [w_c, w_c + W_c)
 *     (eq. 10), R_c * W_c points;
 *   - distances are max-norms of IEEE binary32 round-to-nearest-even
 *     coordinate differences; eps_i is the k-th smallest joint distance over
 *     j != i (self excluded by index); counts are strict (< eps_i) in the
 *     spaces (y_t', Y_past), (Y_past) and (Y_past, X_past) of eq. 8;
 *   - TE is in nats; surrogates permute the repetitions of the source block
 *     (the same point set as permuting the target with the inverse
 *     permutation); p = #{surrogates with TE >= original TE} / S.
 */
#ifndef TE_H
#define TE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    TE_OK = 0,
    TE_ERR_INVALID = 1,    /* bad argument, geometry or non-finite input        */
    TE_ERR_NOMEM = 2,      /* workspace / arena too small for the smallest unit  */
    TE_ERR_DEVICE = 3,     /* HIP runtime error (message in te_last_error)       */
    TE_ERR_BUSY = 4,       /* server queue full                                  */
    TE_ERR_TIMEOUT = 5,    /* te_serve_wait timed out                            */
    TE_ERR_CANCELLED = 6   /* ticket cancelled or server closed                  */
} te_status;

typedef struct te_plan_s *te_plan;       /* immutable after creation; caller destroys */
typedef struct te_server_s *te_server;   /* caller closes                             */

/* One analysis job: n_pairs source/target pairs, each an ensemble of
 * n_trials repetitions of n_samples samples, analysed at n_points windows
 * (eq. 10), with n_surrogates shuffled surrogates per (pair, point).
 * The arrays are copied by te_plan_create. */
typedef struct {
    int32_t n_pairs, n_trials, n_samples;
    int32_t d_y, d_x;          /* embedding dimensions, 1..4 each (eq. 6)          */
    int32_t tau;               /* embedding delay >= 1 (eq. 6)                      */
    int32_t u;                 /* assumed interaction delay >= 1 (eq. 3)            */
    int32_t k;                 /* neighbours in the joint space, 1..15 (eq. 9)     */
    int32_t n_points;          /* analysis windows                                  */
    int32_t window;            /* W for every window when window_len is NULL        */
    const int32_t *window_start;   /* host [n_points]: first sample w_c (0-based)  */
    const int32_t *window_len;     /* host [n_points] or NULL: W_c                  */
    const int32_t *trials;         /* host [n_points] or NULL: R_c (first R_c used) */
    int32_t n_surrogates;      /* S >= 0                                            */
    int32_t cond_source;       /* 1: condition on the current source sample x_t as well: the
                                  conditioning set is (Y_past, x_t) in all spaces of eq. 8-9, the
                                  control of instantaneous mixing noted with Fig. 2; needs
                                  d_y + 1 <= 4.  0: eq. 9 as written                        */
    uint64_t seed;             /* key of the surrogate permutations the library draws when a
                                  call is given no permutations (perms == NULL); see below   */
} te_problem;

/* Surrogate permutations drawn by the library (calls given perms == NULL, or
 * te_plan_permutations).  The surrogates test the estimate against trial
 * shuffles ("TE calculation and statistical testing against surrogate data";
 * Fig. 3): surrogate s of (pair p, point c) reads the source of repetition r
 * from repetition phi(r), phi a uniformly random permutation of 0..R_c-1,
 * independent across (p, c, s).  phi is Fisher-Yates from the top -- for
 * i = R_c-1 down to 1, swap positions i and j_i with j_i uniform on 0..i --
 * with integers from the counter-based SplitMix64 generator (Steele, Lea and
 * Flood, OOPSLA 2014): output q of the stream keyed K is
 * mix(K + (q+1) * 0x9E3779B97F4A7C15), where mix is SplitMix64's finaliser,
 * and K = f(f(f(f(f(0x5EED5EED5EED5EED, seed), 77), p), c), s) with
 * f(k, v) = mix(k + 0x9E3779B97F4A7C15 v + 1).  Draw t (t = R_c-1-i) uses
 * Lemire's multiply-and-reject rule on the high 32 bits w of an output:
 * m = w (i+1), j_i = m >> 32, rejected when (m mod 2^32) < 2^32 mod (i+1).
 * Draws are made in rounds: in round one draw t takes output t; each later
 * round gives the draws rejected so far, in draw order, the next unused
 * outputs.  The same seed gives the same permutations on every call, device
 * and batch split. */

/* Library version string. */
const char *te_version(void);

/* Message describing the last failure on the calling thread ("" if none). */
const char *te_last_error(void);

/* Validate a problem and precompute its geometry, chunk sizes and schedule.
 * TE_ERR_INVALID if a dimension is out of range, a window lacks history
 * (w_c < max(1+(d_y-1)tau, u+(d_x-1)tau)) or runs past n_samples, or a window
 * pools N_c = R_c W_c <= k points or more than 2^27 (134 217 728) points.  The plan is read-only afterwards and may be
 * used from several threads, each with its own workspace and stream. */
te_status te_plan_create(const te_problem *problem, te_plan *out);
te_status te_plan_destroy(te_plan plan);

/* Device workspace sizes in bytes.  full: te_surrogates in a single batch;
 * minimum: the smallest workspace te_surrogates accepts (it then splits the
 * batch into several launches, with identical results); plain: what
 * te_estimate and te_estimate_each need. */
te_status te_plan_workspace_bytes(te_plan plan, size_t *full, size_t *minimum, size_t *plain);

/* Plain per-time-point path: the original (unshuffled) estimate of every
 * (pair, point), one window at a time (embed, search, reduce per window).
 *   x, y     device float32 [n_pairs][n_trials][n_samples] source / target
 *   ws       device workspace of ws_bytes >= plain bytes
 *   te_out   host float64 [n_pairs][n_points], nats */
te_status te_estimate(te_plan plan, const float *x, const float *y,
                      void *ws, size_t ws_bytes, void *hip_stream, double *te_out);

/* Plain per-chunk path over originals and surrogates: every (pair, point) on
 * its own, its window sorted once, then each of its S+1 chunks on its own
 * (embed, search, reduce: three launches per chunk).  Same estimates and
 * p-values as te_surrogates bit for bit; the unbatched baseline the batched
 * and served forms are measured against.  perms, te_surr and p_value as for
 * te_surrogates (perms NULL: drawn from problem.seed); ws of ws_bytes >= the
 * plain bytes of te_plan_workspace_bytes. */
te_status te_estimate_each(te_plan plan, const float *x, const float *y, const int32_t *perms,
                           void *ws, size_t ws_bytes, void *hip_stream,
                           double *te_orig, double *te_surr, double *p_value);

/* Batched path: originals and all surrogates of every (pair, point) through
 * one persistent search launch per batch (eq. 9-10, surrogate test).
 *   perms    device int32 [n_pairs][n_points][n_surrogates][n_trials]: the
 *            source block of repetition r in surrogate s is read from
 *            repetition perms[p][c][s][r]; entries r < R_c must be a
 *            permutation of 0..R_c-1 (checked: TE_ERR_INVALID otherwise).
 *            NULL: the library draws them from problem.seed (see above), on
 *            the device, inside the call.
 *   ws       device workspace of ws_bytes >= minimum bytes
 *   te_orig  host float64 [n_pairs][n_points]
 *   te_surr  host float64 [n_pairs][n_points][n_surrogates] (NULL if S == 0)
 *   p_value  host float64 [n_pairs][n_points] (NaN if S == 0; may be NULL)
 *   use_graph  nonzero: capture the batch in a hipGraph on first use and
 *            replay it on later calls with the same pointers and stream. */
te_status te_surrogates(te_plan plan, const float *x, const float *y, const int32_t *perms,
                        void *ws, size_t ws_bytes, void *hip_stream, int32_t use_graph,
                        double *te_orig, double *te_surr, double *p_value);

/* The batched path of te_surrogates (same searches, same results bit for bit)
 * enqueued on hip_stream with no host synchronisation, for pipelines that keep
 * the GPU busy across calls.  Returns once the work is queued.
 *   x, y, perms  as for te_surrogates; they and ws must stay valid and unchanged
 *            until the stream has run the work (calls on one stream may reuse ws)
 *   ws       device workspace of ws_bytes >= the full bytes of
 *            te_plan_workspace_bytes (TE_ERR_NOMEM otherwise: no batch splitting)
 *   out      float64 [G (S + 1) + G], G = n_pairs * n_points, S = n_surrogates,
 *            device memory or pinned host memory (hipHostMalloc), filled in
 *            stream order: out[g (S + 1)] the original estimate of window group g,
 *            out[g (S + 1) + 1 + s] surrogate s, out[G (S + 1) + g] its p-value
 *            (NaN if S == 0).
 * Invalid input (a non-finite value, an invalid permutation) cannot be reported
 * through the status here: every estimate and p-value of the call is NaN then.
 * Destroy the plan only after the stream has finished its calls. */
te_status te_surrogates_async(te_plan plan, const float *x, const float *y, const int32_t *perms,
                              void *ws, size_t ws_bytes, void *hip_stream, double *out);

/* The permutations the library draws from the plan's seed, written to
 *   perms    device int32 [n_pairs][n_points][n_surrogates][n_trials] (entries
 *            r >= R_c are the identity), in stream order on hip_stream;
 *   ws       device workspace of ws_bytes >= te_plan_permutations_workspace_bytes.
 * Passing this array to te_surrogates gives the same results as passing NULL. */
size_t te_plan_permutations_workspace_bytes(te_plan plan);
te_status te_plan_permutations(te_plan plan, void *ws, size_t ws_bytes, void *hip_stream, int32_t *perms);

/* Local transfer entropy (the per-point quantity of eq. 17, whose average is
 * the estimate, eq. 18): for every pooled point i of every original window,
 *   lte_i = psi(k) + psi(n_P(i)+1) - psi(n_TP(i)+1) - psi(n_PS(i)+1),
 * the summand of eq. 9 with psi(k) included, so the mean over a window is its
 * estimate.  Same searches as te_estimate, all windows in one launch.
 *   lte      device float64 [off[n_pairs*n_points]] : window g = pair * n_points + point
 *            occupies [off[g], off[g+1]) with off from te_plan_local_offsets; points
 *            in window order q = r W_c + (t' - w_c)
 *   te_out   host float64 [n_pairs][n_points] (may be NULL)
 *   ws       device workspace of ws_bytes >= the plan's full size */
te_status te_plan_local_offsets(te_plan plan, int64_t *offsets /* host [n_pairs*n_points + 1] */);
te_status te_local(te_plan plan, const float *x, const float *y, void *ws, size_t ws_bytes,
                   void *hip_stream, double *lte, double *te_out);

/* Delay reconstruction (eq. 5 and the delay scan that goes with it): the
 * original estimate of every (pair, point) at each assumed source delay
 * u_values[j] (the source past is taken at t-u, eq. 6-7), the delay with the
 * largest estimate (the first in u_values order among equal maxima), and the
 * trial-shuffle surrogate test (eq. 10) at that delay.  The plan's own u plays
 * no part.  The maximizing delay is chosen on the device between the two
 * searches; nothing returns to the host before the end.
 *   u_values host int32 [n_u], 1 <= n_u <= 4096; each u >= 1 and every window
 *            start >= u + (d_x - 1) tau (TE_ERR_INVALID otherwise)
 *   perms    as te_surrogates (NULL: drawn from problem.seed)
 *   ws       device workspace of ws_bytes >= the minimum given by
 *            te_delay_scan_workspace_bytes (smaller workspaces are split into
 *            several launches over window groups, with identical results)
 *   te_scan  host float64 [n_pairs][n_points][n_u]
 *   u_best   host int32 [n_pairs][n_points] (may be NULL)
 *   te_surr  host float64 [n_pairs][n_points][n_surrogates] at u_best (NULL if S == 0)
 *   p_value  host float64 [n_pairs][n_points] at u_best (NaN if S == 0; may be NULL) */
te_status te_delay_scan_workspace_bytes(te_plan plan, const int32_t *u_values, int32_t n_u, size_t *full,
                                        size_t *minimum);
te_status te_delay_scan(te_plan plan, const float *x, const float *y, const int32_t *perms,
                        const int32_t *u_values, int32_t n_u, void *ws, size_t ws_bytes, void *hip_stream,
                        double *te_scan, int32_t *u_best, double *te_surr, double *p_value);

/* Kernel-level export in the shape of the paper's neighbour-search call
 * ("Input data"; "Implementation interface"): several pre-embedded chunks
 * searched in one launch.
 *   pts        device float32, coordinate-major: coordinate m of global point
 *              i is pts[m * dim_stride + i]; coordinates ordered
 *              (y_t | Y_past (d_y) | X_past (d_x))
 *   offsets    host int64 [n_chunks + 1]: chunk c holds points
 *              [offsets[c], offsets[c+1]); each chunk needs more than k points
 *   ws         device workspace of te_knn_counts_workspace_bytes(n_chunks) bytes
 *   eps        device float32 [offsets[n_chunks]]: radius of every point
 *   counts     device int32 [3][offsets[n_chunks]]: n_P, n_TP, n_PS of every
 *              point (counts[s * offsets[n_chunks] + i])
 *   te_out     host float64 [n_chunks] or NULL: eq. 9 from those counts */
size_t te_knn_counts_workspace_bytes(int32_t n_chunks, int64_t n_points_total);
te_status te_knn_counts(const float *pts, int64_t dim_stride, const int64_t *offsets,
                        int32_t n_chunks, int32_t d_y, int32_t d_x, int32_t k,
                        void *ws, size_t ws_bytes, void *hip_stream,
                        float *eps, int32_t *counts, double *te_out);

/* For callers that cannot allocate device memory -- code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc: te_knn_counts
 * with its device scratch (tables, sorted copy, sort keys, partial sums, queue
 * counters) in a static array of the library instead of a caller workspace.
 * The array holds TE_NOALLOC_SCRATCH_BYTES per device; each device that runs
 * the library's code holds its own copy until the process ends.
 *   Arguments, layouts and results as te_knn_counts (identical bit for bit).
 *   TE_ERR_NOMEM when te_knn_counts_workspace_bytes(n_chunks, offsets[n_chunks])
 *   exceeds TE_NOALLOC_SCRATCH_BYTES (up to about 590 000 points in all).
 * The call allocates no device memory and no pinned host memory: tables go up
 * and te_out comes down through ordinary host memory, and the stream is
 * synchronised before the call returns.  Every call on one device uses the same
 * array and leaves its contents behind (the queue counters are cleared at the
 * start of each call): calls that overlap on one device, from several threads or
 * streams, race and must be serialised by the caller. */
#define TE_NOALLOC_SCRATCH_BYTES (32u << 20)
te_status te_knn_counts_noalloc(const float *pts, int64_t dim_stride, const int64_t *offsets,
                                int32_t n_chunks, int32_t d_y, int32_t d_x, int32_t k, void *hip_stream,
                                float *eps, int32_t *counts, double *te_out);

/* ------------------------------------------------------ embedding choice
 * Local-predictor score of candidate embeddings (d_c, tau_c) of the target: the
 * embedding section chooses the target's embedding dimension and delay as the
 * pair whose past state best predicts the next sample with a local predictor
 * (Ragwitz and Kantz; the paper gives no formula).  For candidate c the points
 * are all trials r < n_trials and times t in [window_start, window_start +
 * window_len), pooled trial-major (point r * window_len + (t - window_start)),
 * with state (y_{t-1}, y_{t-1-tau_c}, ..., y_{t-1-(d_c-1)tau_c}) and target y_t.
 * Each point's prediction is the mean of the targets of its k nearest other
 * points (maximum norm of the binary32 coordinate differences; equal distances
 * ranked by point index; targets summed in fp64 in rank order), and
 *   score[c] = sum_i (y_i - pred_i)^2 / sum_i (y_i - mean y)^2   (NaN if the
 * targets are constant); the smallest score marks the chosen embedding.
 *   y        device float32 [n_trials][n_samples], the target series
 *   dims, taus  host int32 [n_cand]: 1 <= d_c <= TE_RAGWITZ_MAX_DIM, tau_c >= 1,
 *            and window_start >= 1 + (d_c - 1) tau_c (the state's history)
 *   k        1..TE_RAGWITZ_MAX_K, below the pooled point count N (N <= 2^27)
 *   ws       device workspace of te_ragwitz_workspace_bytes(...) bytes
 *   pred     device float64 [n_cand][N] per-point predictions, or NULL
 *   score    host float64 [n_cand], written before the call returns
 * The stream is synchronised before return.  TE_ERR_INVALID on bad geometry or
 * a non-finite value in a state or target (score untouched); TE_ERR_NOMEM if the
 * workspace is too small. */
#define TE_RAGWITZ_MAX_DIM 8
#define TE_RAGWITZ_MAX_K 16
#define TE_RAGWITZ_MAX_CANDIDATES 64
te_status te_ragwitz_workspace_bytes(int32_t n_trials, int32_t window_len, const int32_t *dims, int32_t n_cand,
                                     size_t *bytes);
te_status te_ragwitz(const float *y, int32_t n_trials, int32_t n_samples, int32_t window_start, int32_t window_len,
                     const int32_t *dims, const int32_t *taus, int32_t n_cand, int32_t k, void *ws, size_t ws_bytes,
                     void *hip_stream, double *pred, double *score);

/* ------------------------------------------------------------------ serving
 * A server keeps admitted jobs resident in a caller-provided device arena and
 * batches their searches continuously: a server thread admits queued jobs in
 * FIFO order while a job slot is free and the job's footprint (series,
 * permutations, embedded coordinates, tables, partial sums) fits in the arena,
 * embeds each admitted job once, and issues steps -- one persistent search
 * launch per kernel class (d_y, d_x, k) over reference blocks of all ready jobs,
 * oldest first, up to step_pairs directed pairs -- so jobs arriving while others
 * run join at the next step.  Estimates are reduced per job in a fixed order and
 * do not depend on which jobs shared a step.  Same semantics as te_surrogates. */

#define TE_SERVE_DRY_RUN 1   /* admission and scheduling only: no device work, results NaN */
#define TE_SERVE_HOLD 2      /* queue submissions without admitting them until te_serve_resume */

typedef struct {
    double p50_s, p99_s;      /* latency quantiles, submit -> result, completed jobs  */
    double est_per_s;         /* estimates (originals + surrogates) per second since
                                 the first submission                                 */
    int64_t completed, failed, cancelled;
    int64_t steps;            /* search launches issued                               */
    int64_t queued, resident; /* jobs waiting for admission / admitted, now           */
    int64_t peak_slots;       /* most jobs resident at once                           */
    int64_t peak_bytes;       /* most arena bytes in use at once                      */
} te_serve_stats_t;

/* Open a server on the current device.
 *   arena        device memory of arena_bytes owned by the caller, kept alive until
 *                te_serve_close returns (may be NULL with TE_SERVE_DRY_RUN)
 *   max_slots    jobs resident at once (>= 1); max_queue: jobs waiting (>= 1)
 *   step_pairs   directed pairs per search launch (0: 4e9, a few milliseconds)
 *   flags        0, TE_SERVE_DRY_RUN and/or TE_SERVE_HOLD */
te_status te_serve_open(void *arena, size_t arena_bytes, int32_t max_slots, int32_t max_queue,
                        int64_t step_pairs, int32_t flags, te_server *out);

/* Submit a job (non-blocking; any thread).  x, y: host float32
 * [n_pairs][n_trials][n_samples]; perms: host int32 [n_pairs][n_points][S][n_trials]
 * (NULL: drawn on the device from problem->seed).  Everything is copied before return.  TE_ERR_INVALID: bad
 * problem; TE_ERR_NOMEM: the job can never fit the arena; TE_ERR_BUSY: queue full. */
te_status te_serve_submit(te_server srv, const te_problem *problem, const float *x, const float *y,
                          const int32_t *perms, uint64_t *ticket);

/* Wait for a ticket: timeout_us < 0 waits forever, 0 polls.  On TE_OK writes the
 * host outputs (te_orig [n_pairs][n_points]; te_surr [..][S] and p_value may be
 * NULL) and releases the ticket; TE_ERR_TIMEOUT leaves it pending; a failed or
 * cancelled ticket returns its status and is released. */
te_status te_serve_wait(te_server srv, uint64_t ticket, int64_t timeout_us,
                        double *te_orig, double *te_surr, double *p_value);

/* Start admitting jobs on a server opened with TE_SERVE_HOLD. */
te_status te_serve_resume(te_server srv);

/* Cancel a ticket that has not been admitted yet (TE_ERR_BUSY once admitted). */
te_status te_serve_cancel(te_server srv, uint64_t ticket);

te_status te_serve_stats(te_server srv, te_serve_stats_t *out);

/* Stop accepting jobs, cancel queued ones, finish admitted ones, join the server
 * thread and free the server.  The arena may be freed afterwards. */
te_status te_serve_close(te_server srv);

/* ------------------------------------------------------------------ tuning
 * The search kernel's launch shape -- candidate slots per lane in the counting
 * pass (4, 8 or 16), waves per workgroup (1, 2 or 4) and resident workgroups per
 * compute unit (every whole number of waves per SIMD from full occupancy down to
 * half) -- is chosen per (d_y, d_x, k, chunk-size bucket floor(log2 N)).
 * te_autotune times every shape on n_chunks synthetic chunks of n_points points
 * (uniform random coordinates generated in ws) and records the fastest in a
 * process-wide table that plans and servers created afterwards use (the nearest
 * bucket within 2).  ws must hold n_chunks*n_points*(1+d_y+d_x) floats plus
 * small tables (TE_ERR_NOMEM names the size).  Outputs may be NULL.
 * te_tune_save / te_tune_load write / read the table as text; the environment
 * variable TE_TUNE_FILE names a table loaded on first use. */
te_status te_autotune(int32_t d_y, int32_t d_x, int32_t k, int32_t n_points, int32_t n_chunks,
                      void *ws, size_t ws_bytes, void *hip_stream,
                      int32_t *slots, int32_t *waves_per_wg, int32_t *wg_per_cu, double *best_ms);
/* Tuning on the plan's own data (x, y, perms as for te_surrogates, NULL drawn; ws of
 * ws_bytes >= the plan's minimum workspace): every shape te_autotune tries is
 * timed on a batch of the plan's largest window groups; the fastest becomes the
 * plan's launch shape and is recorded in the table.  Results of the plan do not
 * depend on the shape. */
te_status te_plan_autotune(te_plan plan, const float *x, const float *y, const int32_t *perms, void *ws,
                           size_t ws_bytes, void *hip_stream, int32_t *slots, int32_t *waves_per_wg,
                           int32_t *wg_per_cu, double *ms);
te_status te_tune_save(const char *path);
te_status te_tune_load(const char *path);
te_status te_tune_clear(void);

/* Measurement hook, process-wide, for search-kernel launches made outside
 * graph capture.  flags: TE_PROFILE_TIME brackets every launch with HIP events
 * recorded on the launch stream (te_profile_read waits for them and returns the
 * summed kernel time in milliseconds and the number of launches; reset != 0
 * clears the totals); TE_PROFILE_WORK makes each wave add the pairs it
 * evaluated to device counters once, after its last work item
 * (te_profile_work).  0 turns both off. */
#define TE_PROFILE_TIME 1
#define TE_PROFILE_WORK 2
te_status te_profile_enable(int32_t flags);
te_status te_profile_read(double *search_ms, int64_t *launches, int32_t reset);
/* Pairs the timed search launches actually evaluated: pass 1 (radius) and pass 2
 * (counts); with sorted search spaces these are below the method's N(N-1) per
 * pass.  Synchronises the device. */
te_status te_profile_work(int64_t *pass1_pairs, int64_t *pass2_pairs, int32_t reset);
/* All four counters: counts[0], counts[1] as te_profile_work (one pair per
 * chunk); counts[2], counts[3] the (reference, candidate) pairs of pass 1 and
 * pass 2 whose target coordinates (y_t', Y_past) were compared: the window
 * chunks searched together as one set (originals, surrogates or delays of one
 * window) share those comparisons, so these are below counts[0], counts[1]
 * when sets are used, and equal to them otherwise.  counts: host int64 [4]. */
te_status te_profile_work_all(int64_t *counts, int32_t reset);

#ifdef __cplusplus
}
#endif

#endif /* TE_H */
