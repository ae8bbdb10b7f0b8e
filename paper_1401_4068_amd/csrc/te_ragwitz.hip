// te_ragwitz.hip -- the local-predictor score of delay embeddings of the target
// (te_ragwitz): the embedding dimension d and delay tau are chosen as the pair whose
// past state best predicts the next sample with a local predictor (embedding section
// of Wollstadt et al. 2014, after Ragwitz and Kantz).  For each candidate (d, tau) the
// window's points of all trials are pooled; each point's k nearest other points in the
// maximum norm (equal distances ranked by point index) predict its next sample as the
// mean of theirs; the score is the normalised mean squared error.

#include <hip/hip_runtime.h>

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

// One wave per 64 reference points (lane = reference), candidates uniform in index
// order, eight at a time on scalar loads.  The list (bd, bi) holds the k smallest
// (distance, index) pairs seen so far, ascending; a candidate enters only if strictly
// closer than the k-th, so among equal distances the smaller index stays ahead.
template <int D>
__global__ void __launch_bounds__(64) rag_knn_kernel(const float *__restrict__ rows, const float *__restrict__ tgt,
                                                     int N, int k, double *__restrict__ pred,
                                                     double *__restrict__ sq)
{
    const int lane = (int)threadIdx.x;
    const int i = (int)blockIdx.x * kWave + lane;
    const bool valid = i < N;
    const int ii = valid ? i : N - 1;
    float ref[D];
#pragma unroll
    for (int m = 0; m < D; ++m)
        ref[m] = rows[(int64_t)m * N + ii];
    float bd[kRagMaxK];
    int bi[kRagMaxK];
#pragma unroll
    for (int p = 0; p < kRagMaxK; ++p) {
        bd[p] = __builtin_inff();
        bi[p] = 0;
    }
    float thr = __builtin_inff();                 // bd[k - 1]
    // (x, j) with x < bd[k - 1] and j above every listed index: entries larger than x
    // move down one place and x goes behind the last entry <= x, so equal distances
    // stay in index order (from the last place up, each place reads the one above
    // before that one changes)
    auto insert = [&](float x, int j) {
#pragma unroll
        for (int p = kRagMaxK - 1; p >= 1; --p) {
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
        for (int p = 0; p < kRagMaxK; ++p)
            if (p == k - 1)
                thr = bd[p];
    };
    int j = 0;
    for (; j + 8 <= N; j += 8) {
        float c[8][D];
#pragma unroll
        for (int m = 0; m < D; ++m) {
            const f8v v = sload8(rows + (int64_t)m * N, (uint32_t)j * 4u);
#pragma unroll
            for (int u = 0; u < 8; ++u)
                c[u][m] = v[u];
        }
        float dist[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            float dm = __builtin_fabsf(c[u][0] - ref[0]);
#pragma unroll
            for (int m = 1; m < D; ++m)
                dm = fmaxf(dm, __builtin_fabsf(c[u][m] - ref[m]));
            dist[u] = (j + u == i) ? __builtin_inff() : dm;
        }
        const float mn = fminf(fminf(fminf(dist[0], dist[1]), fminf(dist[2], dist[3])),
                               fminf(fminf(dist[4], dist[5]), fminf(dist[6], dist[7])));
        if (__builtin_amdgcn_ballot_w64(mn < thr)) {
#pragma unroll
            for (int u = 0; u < 8; ++u)
                if (dist[u] < thr)
                    insert(dist[u], j + u);
        }
    }
    for (; j < N; ++j) {
        float dm = __builtin_fabsf(sload(rows + j) - ref[0]);
#pragma unroll
        for (int m = 1; m < D; ++m)
            dm = fmaxf(dm, __builtin_fabsf(sload(rows + (int64_t)m * N + j) - ref[m]));
        if (j != i && dm < thr)
            insert(dm, j);
    }
    // the prediction: neighbour targets summed in rank order in fp64
    double s = 0.0;
#pragma unroll
    for (int p = 0; p < kRagMaxK; ++p)
        if (p < k)
            s += (double)tgt[bi[p]];
    const double yhat = s / (double)k;
    if (valid) {
        if (pred != nullptr)
            pred[i] = yhat;
        const double e = (double)tgt[i] - yhat;
        sq[i] = e * e;
    }
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

hipError_t launch_knn(int d, const float *rows, const float *tgt, int N, int k, double *pred, double *sq,
                      hipStream_t st)
{
    const dim3 grid((unsigned)((N + kWave - 1) / kWave)), block(kWave);
    switch (d) {
    case 1: rag_knn_kernel<1><<<grid, block, 0, st>>>(rows, tgt, N, k, pred, sq); break;
    case 2: rag_knn_kernel<2><<<grid, block, 0, st>>>(rows, tgt, N, k, pred, sq); break;
    case 3: rag_knn_kernel<3><<<grid, block, 0, st>>>(rows, tgt, N, k, pred, sq); break;
    case 4: rag_knn_kernel<4><<<grid, block, 0, st>>>(rows, tgt, N, k, pred, sq); break;
    case 5: rag_knn_kernel<5><<<grid, block, 0, st>>>(rows, tgt, N, k, pred, sq); break;
    case 6: rag_knn_kernel<6><<<grid, block, 0, st>>>(rows, tgt, N, k, pred, sq); break;
    case 7: rag_knn_kernel<7><<<grid, block, 0, st>>>(rows, tgt, N, k, pred, sq); break;
    case 8: rag_knn_kernel<8><<<grid, block, 0, st>>>(rows, tgt, N, k, pred, sq); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

// Workspace layout: flag | targets [N] | states of each candidate [d_c][N] | squared errors
// [n_cand][N] | scores [n_cand], each part 256-byte aligned.
struct RagLayout {
    size_t flag = 0, tgt = 0, sq = 0, score = 0, total = 0;
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
    for (int c = 0; c < n_cand; ++c) {
        const float *rows = reinterpret_cast<const float *>(ws + L.rows[c]);
        if ((e = launch_knn(dims[c], rows, tgt, N, k, pred ? pred + (int64_t)c * N : nullptr, sq + (int64_t)c * N,
                            st)) != hipSuccess)
            return hip_fail(e, "rag_knn_kernel");
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
