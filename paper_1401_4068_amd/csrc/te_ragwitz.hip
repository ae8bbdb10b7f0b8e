// te_ragwitz.hip -- the local-predictor score of delay embeddings of the target
// (te_ragwitz): the embedding dimension d and delay tau are chosen as the pair whose
// past state best predicts the next sample with a local predictor (embedding section
// of Wollstadt et al. 2014, after Ragwitz and Kantz).  For each candidate (d, tau) the
// window's points of all trials are pooled; each point's k nearest other points in the
// maximum norm (equal distances ranked by point index) predict its next sample as the
// mean of theirs; the score is the normalised mean squared error.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <vector>

#include "te.h"
#include "te_internal.h"
#include "te_runtime.h"

namespace te {
namespace {

constexpr int kRagMaxDim = TE_RAGWITZ_MAX_DIM;
constexpr int kRagMaxK = TE_RAGWITZ_MAX_K;
constexpr int kScoreThreads = 256;

typedef float f8v __attribute__((ext_vector_type(8)));
typedef const __attribute__((address_space(4))) float rag_cfloat_t;
typedef const __attribute__((address_space(4))) f8v __attribute__((aligned(4))) rag_cf8_t;

// wave-uniform loads (scalar memory): one value, or eight consecutive values at a
// 32-bit byte offset from a uniform base
__device__ __forceinline__ float sload(const float *p) { return *(rag_cfloat_t *)p; }
__device__ __forceinline__ f8v sload8(const float *p, uint32_t byte_off)
{
    typedef const __attribute__((address_space(4))) char cchar_t;
    return *(rag_cf8_t *)((cchar_t *)p + byte_off);
}

// States of one candidate: rows[m N + i] = y[r][t - 1 - m tau] for point i = r W + (t - w),
// and with tgt non-null the targets tgt[i] = y[r][t].  A non-finite value sets *bad.
__global__ void rag_embed_kernel(const float *__restrict__ y, int T, int w, int W, int N, int d, int tau,
                                 float *__restrict__ rows, float *__restrict__ tgt, int *__restrict__ bad)
{
    const int i = (int)(blockIdx.x * blockDim.x + threadIdx.x);
    if (i >= N)
        return;
    const int r = i / W;
    const int t = w + (i - r * W);
    const float *yr = y + (int64_t)r * T;
    bool ok = true;
    for (int m = 0; m < d; ++m) {
        const float v = yr[t - 1 - m * tau];
        ok = ok && __builtin_isfinite(v);
        rows[(int64_t)m * N + i] = v;
    }
    if (tgt != nullptr) {
        const float v = yr[t];
        ok = ok && __builtin_isfinite(v);
        tgt[i] = v;
    }
    if (!ok)
        atomicOr(bad, 1);
}

// The k smallest (distance, index) pairs seen so far, ascending.  Entries arrive with
// an index above every listed entry of equal distance, so inserting only what is
// strictly closer than the k-th keeps equal distances in index order.
template <int KC>                                 // capacity: k <= KC
struct TopK {
    float bd[KC];
    int bi[KC];
    float thr;                                    // bd[k - 1]
    int k;
    __device__ void init(int k_)
    {
        thr = __builtin_inff();
        k = k_;
#pragma unroll
        for (int p = 0; p < KC; ++p) {
            bd[p] = __builtin_inff();
            bi[p] = 0;
        }
    }
    // (x, j) with x < thr: entries larger than x move down one place and x goes behind
    // the last entry <= x (from the last place up, each place reads the one above before
    // that one changes)
    __device__ __forceinline__ void insert(float x, int j)
    {
#pragma unroll
        for (int p = KC - 1; p >= 1; --p) {
            if (p < k) {
                const bool move = bd[p - 1] > x;
                const bool put = !move && bd[p] > x;
                bd[p] = move ? bd[p - 1] : (put ? x : bd[p]);
                bi[p] = move ? bi[p - 1] : (put ? j : bi[p]);
            }
        }
        if (bd[0] > x) {
            bd[0] = x;
            bi[0] = j;
        }
#pragma unroll
        for (int p = 0; p < KC; ++p)
            if (p == k - 1)
                thr = bd[p];
    }
};

// One wave per (64 RPL reference points, candidate segment): lane l holds references
// b + l + 64 r (r < RPL), the segment's candidates are uniform in index order, eight at
// a time on scalar loads, so each load feeds 8 RPL distances per lane.  The segment's
// list of each reference goes to lst_d / lst_i [segment][place][point] (places a
// segment cannot fill stay at distance +inf).  Four references per lane while their
// lists fit in registers (capacity up to 8), one for lists of 16.
constexpr int refs_per_lane(int kc) { return kc <= 8 ? 4 : 1; }

template <int D, int KC>
__global__ void __launch_bounds__(64) rag_knn_kernel(const float *__restrict__ rows, int N, int k, int seg_len,
                                                     float *__restrict__ lst_d, int *__restrict__ lst_i)
{
    constexpr int RPL = refs_per_lane(KC);
    const int lane = (int)threadIdx.x;
    const int seg = (int)blockIdx.y;
    const int j0 = seg * seg_len;
    const int j1 = min(N, j0 + seg_len);
    int ri[RPL];
    float ref[RPL][D];
#pragma unroll
    for (int r = 0; r < RPL; ++r) {
        ri[r] = (int)blockIdx.x * (kWave * RPL) + r * kWave + lane;
        const int ii = ri[r] < N ? ri[r] : N - 1;
#pragma unroll
        for (int m = 0; m < D; ++m)
            ref[r][m] = rows[(int64_t)m * N + ii];
    }
    TopK<KC> L[RPL];
#pragma unroll
    for (int r = 0; r < RPL; ++r)
        L[r].init(k);
    int j = j0;
    for (; j + 8 <= j1; j += 8) {
        float c[8][D];
#pragma unroll
        for (int m = 0; m < D; ++m) {
            const f8v v = sload8(rows + (int64_t)m * N, (uint32_t)j * 4u);
#pragma unroll
            for (int u = 0; u < 8; ++u)
                c[u][m] = v[u];
        }
#pragma unroll
        for (int r = 0; r < RPL; ++r) {
            float dist[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                float dm = __builtin_fabsf(c[u][0] - ref[r][0]);
#pragma unroll
                for (int m = 1; m < D; ++m)
                    dm = fmaxf(dm, __builtin_fabsf(c[u][m] - ref[r][m]));
                dist[u] = (j + u == ri[r]) ? __builtin_inff() : dm;
            }
            const float mn = fminf(fminf(fminf(dist[0], dist[1]), fminf(dist[2], dist[3])),
                                   fminf(fminf(dist[4], dist[5]), fminf(dist[6], dist[7])));
            if (__builtin_amdgcn_ballot_w64(mn < L[r].thr)) {
#pragma unroll
                for (int u = 0; u < 8; ++u)
                    if (dist[u] < L[r].thr)
                        L[r].insert(dist[u], j + u);
            }
        }
    }
    for (; j < j1; ++j) {
        float cj[D];
#pragma unroll
        for (int m = 0; m < D; ++m)
            cj[m] = sload(rows + (int64_t)m * N + j);
#pragma unroll
        for (int r = 0; r < RPL; ++r) {
            float dm = __builtin_fabsf(cj[0] - ref[r][0]);
#pragma unroll
            for (int m = 1; m < D; ++m)
                dm = fmaxf(dm, __builtin_fabsf(cj[m] - ref[r][m]));
            if (j != ri[r] && dm < L[r].thr)
                L[r].insert(dm, j);
        }
    }
#pragma unroll
    for (int r = 0; r < RPL; ++r)
        if (ri[r] < N) {
#pragma unroll
            for (int p = 0; p < KC; ++p)
                if (p < k) {
                    const int64_t o = ((int64_t)seg * k + p) * N + ri[r];
                    lst_d[o] = L[r].bd[p];
                    lst_i[o] = L[r].bi[p];
                }
        }
}

// Thread = point: the segments' lists merged in segment order (indices ascend across
// segments and within a list equal distances ascend in index, so the strict insertion
// keeps the rank order), then the prediction -- the neighbours' targets summed in rank
// order in fp64 -- and its squared error.
template <int KC>
__global__ void __launch_bounds__(256) rag_merge_kernel(const float *__restrict__ lst_d,
                                                        const int *__restrict__ lst_i,
                                                        const float *__restrict__ tgt, int N, int k, int n_seg,
                                                        double *__restrict__ pred, double *__restrict__ sq)
{
    const int i = (int)(blockIdx.x * blockDim.x + threadIdx.x);
    if (i >= N)
        return;
    TopK<KC> L;
    L.init(k);
#pragma unroll 4
    for (int seg = 0; seg < n_seg; ++seg) {
        float xd[KC];
        int xi[KC];
#pragma unroll
        for (int p = 0; p < KC; ++p) {            // the segment's list, all loads in flight
            const int64_t o = ((int64_t)seg * k + (p < k ? p : 0)) * N + i;
            xd[p] = p < k ? lst_d[o] : __builtin_inff();
            xi[p] = p < k ? lst_i[o] : 0;
        }
#pragma unroll
        for (int p = 0; p < KC; ++p)
            if (xd[p] < L.thr)
                L.insert(xd[p], xi[p]);
    }
    double s = 0.0;
#pragma unroll
    for (int p = 0; p < KC; ++p)
        if (p < k)
            s += (double)tgt[L.bi[p]];
    const double yhat = s / (double)k;
    if (pred != nullptr)
        pred[i] = yhat;
    const double e = (double)tgt[i] - yhat;
    sq[i] = e * e;
}

// Fixed-order sum over a workgroup of kScoreThreads threads.
__device__ double block_sum(double v, double *part)
{
    const int tid = (int)threadIdx.x;
    part[tid] = v;
    __syncthreads();
    for (int s = kScoreThreads / 2; s > 0; s >>= 1) {
        if (tid < s)
            part[tid] += part[tid + s];
        __syncthreads();
    }
    const double r = part[0];
    __syncthreads();
    return r;
}

// Score of candidate c = blockIdx.x: sum of squared errors / sum of squared deviations
// of the targets from their mean (NaN if the targets are constant).
__global__ void __launch_bounds__(kScoreThreads) rag_score_kernel(const float *__restrict__ tgt,
                                                                   const double *__restrict__ sq, int N,
                                                                   double *__restrict__ score)
{
    __shared__ double part[kScoreThreads];
    const int c = (int)blockIdx.x;
    double a = 0.0;
    for (int i = (int)threadIdx.x; i < N; i += kScoreThreads)
        a += (double)tgt[i];
    const double mean = block_sum(a, part) / (double)N;
    double v = 0.0, e = 0.0;
    for (int i = (int)threadIdx.x; i < N; i += kScoreThreads) {
        const double dlt = (double)tgt[i] - mean;
        v += dlt * dlt;
        e += sq[(int64_t)c * N + i];
    }
    const double V = block_sum(v, part);
    const double E = block_sum(e, part);
    if (threadIdx.x == 0)
        score[c] = V > 0.0 ? E / V : __builtin_nan("");
}

// Candidate segments per point: enough (wave, segment) pairs to give every SIMD of the
// chip several waves (a wave holds 64 rpl references), segments of at least 64 points
// (a multiple of 8), at most 64.
struct Segments {
    int len = 0, n = 0;
};

Segments segments(int64_t N, int rpl)
{
    const int64_t blocks = (N + kWave * rpl - 1) / (kWave * rpl);
    int64_t want = (16384 + blocks - 1) / blocks;
    want = want < 1 ? 1 : (want > 64 ? 64 : want);
    int64_t len = (N + want - 1) / want;
    len = len < 64 ? 64 : (len + 7) / 8 * 8;
    Segments s;
    s.len = (int)len;
    s.n = (int)((N + len - 1) / len);
    return s;
}

template <int KC>
hipError_t launch_knn_kc(int d, const float *rows, int N, int k, const Segments &sg, float *lst_d, int *lst_i,
                         hipStream_t st)
{
    constexpr int RPL = refs_per_lane(KC);
    const dim3 grid((unsigned)((N + kWave * RPL - 1) / (kWave * RPL)), (unsigned)sg.n);
    const dim3 block(kWave);
    switch (d) {
    case 1: rag_knn_kernel<1, KC><<<grid, block, 0, st>>>(rows, N, k, sg.len, lst_d, lst_i); break;
    case 2: rag_knn_kernel<2, KC><<<grid, block, 0, st>>>(rows, N, k, sg.len, lst_d, lst_i); break;
    case 3: rag_knn_kernel<3, KC><<<grid, block, 0, st>>>(rows, N, k, sg.len, lst_d, lst_i); break;
    case 4: rag_knn_kernel<4, KC><<<grid, block, 0, st>>>(rows, N, k, sg.len, lst_d, lst_i); break;
    case 5: rag_knn_kernel<5, KC><<<grid, block, 0, st>>>(rows, N, k, sg.len, lst_d, lst_i); break;
    case 6: rag_knn_kernel<6, KC><<<grid, block, 0, st>>>(rows, N, k, sg.len, lst_d, lst_i); break;
    case 7: rag_knn_kernel<7, KC><<<grid, block, 0, st>>>(rows, N, k, sg.len, lst_d, lst_i); break;
    case 8: rag_knn_kernel<8, KC><<<grid, block, 0, st>>>(rows, N, k, sg.len, lst_d, lst_i); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <int KC>
hipError_t launch_candidate(int d, const float *rows, const float *tgt, int N, int k, const Segments &sg,
                            float *lst_d, int *lst_i, double *pred, double *sq, hipStream_t st)
{
    hipError_t e = launch_knn_kc<KC>(d, rows, N, k, sg, lst_d, lst_i, st);
    if (e != hipSuccess)
        return e;
    rag_merge_kernel<KC><<<dim3((unsigned)((N + 255) / 256)), dim3(256), 0, st>>>(lst_d, lst_i, tgt, N, k, sg.n,
                                                                                 pred, sq);
    return hipGetLastError();
}

// the k nearest of each point for one candidate, merged, with its predictions: the list
// capacity is the smallest of 4, 8, 16 that holds k
hipError_t launch_knn(int d, const float *rows, const float *tgt, int N, int k, float *lst_d, int *lst_i,
                      double *pred, double *sq, hipStream_t st)
{
    if (k <= 4)
        return launch_candidate<4>(d, rows, tgt, N, k, segments(N, refs_per_lane(4)), lst_d, lst_i, pred, sq, st);
    if (k <= 8)
        return launch_candidate<8>(d, rows, tgt, N, k, segments(N, refs_per_lane(8)), lst_d, lst_i, pred, sq, st);
    return launch_candidate<16>(d, rows, tgt, N, k, segments(N, refs_per_lane(16)), lst_d, lst_i, pred, sq, st);
}

// Workspace layout: flag | targets [N] | states of each candidate [d_c][N] | squared errors
// [n_cand][N] | scores [n_cand] | segment lists (distances, indices) [segments][k][N] for
// k up to TE_RAGWITZ_MAX_K, reused by every candidate; each part 256-byte aligned.
struct RagLayout {
    size_t flag = 0, tgt = 0, sq = 0, score = 0, lst_d = 0, lst_i = 0, total = 0;
    std::vector<size_t> rows;
};

RagLayout rag_layout(int64_t N, const int32_t *dims, int n_cand)
{
    RagLayout L;
    size_t o = 256;
    L.tgt = o;
    o += align_up(sizeof(float) * (size_t)N, 256);
    for (int c = 0; c < n_cand; ++c) {
        L.rows.push_back(o);
        o += align_up(sizeof(float) * (size_t)N * (size_t)dims[c], 256);
    }
    L.sq = o;
    o += align_up(sizeof(double) * (size_t)N * (size_t)n_cand, 256);
    L.score = o;
    o += align_up(sizeof(double) * (size_t)n_cand, 256);
    const int n_seg = std::max(segments(N, refs_per_lane(8)).n, segments(N, refs_per_lane(16)).n);
    const size_t lst = (size_t)n_seg * (size_t)kRagMaxK * (size_t)N;
    L.lst_d = o;
    o += align_up(sizeof(float) * lst, 256);
    L.lst_i = o;
    o += align_up(sizeof(int) * lst, 256);
    L.total = o;
    return L;
}

te_status rag_check(int32_t n_trials, int32_t n_samples, int32_t window_start, int32_t window_len,
                    const int32_t *dims, const int32_t *taus, int32_t n_cand, int32_t k)
{
    if (!dims || !taus)
        return fail(TE_ERR_INVALID, "null argument");
    if (n_cand < 1 || n_cand > TE_RAGWITZ_MAX_CANDIDATES)
        return fail(TE_ERR_INVALID, "n_cand must be in 1..%d", TE_RAGWITZ_MAX_CANDIDATES);
    if (k < 1 || k > kRagMaxK)
        return fail(TE_ERR_INVALID, "k must be in 1..%d", kRagMaxK);
    if (n_trials < 1 || window_len < 1)
        return fail(TE_ERR_INVALID, "n_trials and window_len must be >= 1");
    if (window_start < 0 || (int64_t)window_start + window_len > n_samples)
        return fail(TE_ERR_INVALID, "window [%d, %d) runs past n_samples = %d", window_start,
                    window_start + window_len, n_samples);
    const int64_t N = (int64_t)n_trials * window_len;
    if (N <= k || N > kMaxWindowPoints)
        return fail(TE_ERR_INVALID, "the window pools %lld points; need k < N <= %d", (long long)N,
                    kMaxWindowPoints);
    for (int c = 0; c < n_cand; ++c) {
        if (dims[c] < 1 || dims[c] > kRagMaxDim || taus[c] < 1)
            return fail(TE_ERR_INVALID, "candidate %d: d = %d, tau = %d (need 1 <= d <= %d, tau >= 1)", c, dims[c],
                        taus[c], kRagMaxDim);
        if ((int64_t)window_start < 1 + (int64_t)(dims[c] - 1) * taus[c])
            return fail(TE_ERR_INVALID, "candidate %d: the window starts at %d but the state needs %lld samples of "
                        "history", c, window_start, (long long)(1 + (int64_t)(dims[c] - 1) * taus[c]));
    }
    return TE_OK;
}

}  // namespace
}  // namespace te

using namespace te;

extern "C" {

te_status te_ragwitz_workspace_bytes(int32_t n_trials, int32_t window_len, const int32_t *dims, int32_t n_cand,
                                     size_t *bytes)
{
    clear_error();
    if (!dims || !bytes)
        return fail(TE_ERR_INVALID, "null argument");
    if (n_trials < 1 || window_len < 1 || n_cand < 1 || n_cand > TE_RAGWITZ_MAX_CANDIDATES)
        return fail(TE_ERR_INVALID, "bad geometry");
    for (int c = 0; c < n_cand; ++c)
        if (dims[c] < 1 || dims[c] > kRagMaxDim)
            return fail(TE_ERR_INVALID, "candidate %d: d = %d outside 1..%d", c, dims[c], kRagMaxDim);
    *bytes = rag_layout((int64_t)n_trials * window_len, dims, n_cand).total;
    return TE_OK;
}

te_status te_ragwitz(const float *y, int32_t n_trials, int32_t n_samples, int32_t window_start, int32_t window_len,
                     const int32_t *dims, const int32_t *taus, int32_t n_cand, int32_t k, void *ws_, size_t ws_bytes,
                     void *hip_stream, double *pred, double *score)
{
    TraceRange trace_range("te.ragwitz");
    clear_error();
    if (!y || !ws_ || !score)
        return fail(TE_ERR_INVALID, "null argument");
    te_status s = rag_check(n_trials, n_samples, window_start, window_len, dims, taus, n_cand, k);
    if (s != TE_OK)
        return s;
    const int N = n_trials * window_len;
    const RagLayout L = rag_layout(N, dims, n_cand);
    if (ws_bytes < L.total)
        return fail(TE_ERR_NOMEM, "workspace %zu bytes < %zu", ws_bytes, L.total);
    char *ws = static_cast<char *>(ws_);
    hipStream_t st = (hipStream_t)hip_stream;
    int *bad = reinterpret_cast<int *>(ws + L.flag);
    float *tgt = reinterpret_cast<float *>(ws + L.tgt);
    double *sq = reinterpret_cast<double *>(ws + L.sq);
    double *dscore = reinterpret_cast<double *>(ws + L.score);
    hipError_t e = hipMemsetAsync(bad, 0, sizeof(int), st);
    if (e != hipSuccess)
        return hip_fail(e, "hipMemsetAsync");
    const dim3 eb(256), eg((unsigned)((N + 255) / 256));
    for (int c = 0; c < n_cand; ++c) {
        float *rows = reinterpret_cast<float *>(ws + L.rows[c]);
        rag_embed_kernel<<<eg, eb, 0, st>>>(y, n_samples, window_start, window_len, N, dims[c], taus[c], rows,
                                            c == 0 ? tgt : nullptr, bad);
        if ((e = hipGetLastError()) != hipSuccess)
            return hip_fail(e, "rag_embed_kernel");
    }
    float *lst_d = reinterpret_cast<float *>(ws + L.lst_d);
    int *lst_i = reinterpret_cast<int *>(ws + L.lst_i);
    for (int c = 0; c < n_cand; ++c) {
        const float *rows = reinterpret_cast<const float *>(ws + L.rows[c]);
        if ((e = launch_knn(dims[c], rows, tgt, N, k, lst_d, lst_i, pred ? pred + (int64_t)c * N : nullptr,
                            sq + (int64_t)c * N, st)) != hipSuccess)
            return hip_fail(e, "rag_knn_kernel / rag_merge_kernel");
    }
    rag_score_kernel<<<dim3((unsigned)n_cand), dim3(kScoreThreads), 0, st>>>(tgt, sq, N, dscore);
    if ((e = hipGetLastError()) != hipSuccess)
        return hip_fail(e, "rag_score_kernel");
    int bad_h = 0;
    std::vector<double> sc(n_cand);
    if ((e = hipMemcpyAsync(&bad_h, bad, sizeof(int), hipMemcpyDeviceToHost, st)) != hipSuccess ||
        (e = hipMemcpyAsync(sc.data(), dscore, sizeof(double) * n_cand, hipMemcpyDeviceToHost, st)) != hipSuccess)
        return hip_fail(e, "hipMemcpyAsync");
    {
        TraceRange wait_range("te.wait");
        if ((e = hipStreamSynchronize(st)) != hipSuccess)
            return hip_fail(e, "hipStreamSynchronize");
    }
    if (bad_h)
        return fail(TE_ERR_INVALID, "non-finite value in the window or its history");
    for (int c = 0; c < n_cand; ++c)
        score[c] = sc[c];
    return TE_OK;
}

}  // extern "C"
