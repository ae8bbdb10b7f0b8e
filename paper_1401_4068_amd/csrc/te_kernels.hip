// te_kernels.hip -- HIP kernels of libte for gfx950 (CDNA4, wave64).
//
//   embed_kernel     eq. 6-7 / eq. 10: gathers the pooled points of a window
//                    from the raw [pair][trial][sample] series into
//                    coordinate-major blocks; bit copies only.
//   search_kernel    the KSG type-1 searches (text before eq. 9): per point
//                    the max-norm k-NN radius in the joint space, then strict
//                    range counts in the three marginal spaces of eq. 8, then
//                    the per-point digamma terms of eq. 9 summed per work item.
//   reduce_kernel    eq. 9/10 per chunk: psi(k) + mean of the terms.
//   pvalue_kernel    fraction of surrogate estimates >= the original.
//   argmax_u_kernel  eq. 5: the assumed delay with the largest estimate.
//
// The search kernel is persistent: every wavefront pulls work items (one
// chunk, 64 consecutive reference points) from a global counter until the
// queue is empty, so one launch covers any mix of chunk sizes.
//
// Pass 1 (radius): lane = reference point.  Candidates are wave-uniform and
// read with scalar loads straight into SGPRs, so each coordinate difference is
// one v_sub_f32 with an SGPR operand.  Each lane keeps the k+1 smallest joint
// distances in registers (self included, distance 0), inserted with a
// min / med3 network only when some lane of the wave improves its k+1-th
// distance; the radius is the k+1-th entry, i.e. the k-th neighbour without self.
//
// Pass 2 (counts): lane = candidate point.  Each wave holds a tile of 64 x
// SLOTS candidates in VGPRs and walks its 64 references uniformly (scalar
// loads), with the reference radius in an SGPR: the three strict comparisons
// become wave ballots and the counting is SALU popcounts.  The (y_t', Y_past)
// and (Y_past, X_past) conditions share the Y_past comparison:
// n_TP counts  [d_P < eps] & [d_T < eps],  n_PS counts [d_P < eps] & [d_S < eps].

#include <hip/hip_runtime.h>
#include <math.h>
#include <stddef.h>
#include <stdint.h>

#include "te_internal.h"

namespace te {

namespace {

typedef float f4v __attribute__((ext_vector_type(4)));
typedef const __attribute__((address_space(4))) float cfloat_t;
typedef const __attribute__((address_space(4))) int32_t cint_t;
typedef const __attribute__((address_space(4))) int64_t cint64_t;
typedef const __attribute__((address_space(4))) f4v __attribute__((aligned(4))) cf4_t;
typedef float f8v __attribute__((ext_vector_type(8)));
typedef const __attribute__((address_space(4))) f8v __attribute__((aligned(4))) cf8_t;

// Wave-uniform loads through the constant address space: the address is the
// same in every lane, so these become scalar (SMEM) loads into SGPRs.  Only
// scalar and vector-typed values are loaded this way (aggregate copies would
// be lowered to vector-memory loads).
__device__ __forceinline__ float uload(const float *p) { return *(cfloat_t *)p; }
__device__ __forceinline__ f4v uload4(const float *p) { return *(cf4_t *)p; }
__device__ __forceinline__ f8v uload8_at(const float *p, uint32_t byte_off)
{
    typedef const __attribute__((address_space(4))) char cchar_t;
    return *(cf8_t *)((cchar_t *)p + byte_off);
}
// the same at a 32-bit byte offset from a wave-uniform base: one SGPR offset shared
// by several bases, so the loads need no 64-bit address arithmetic
__device__ __forceinline__ f4v uload4_at(const float *p, uint32_t byte_off)
{
    typedef const __attribute__((address_space(4))) char cchar_t;
    return *(cf4_t *)((cchar_t *)p + byte_off);
}
// per-lane load at a 32-bit byte offset from a wave-uniform base: the base stays in
// SGPRs and the offset in one VGPR (no 64-bit address per lane)
__device__ __forceinline__ float vload_at(const float *p, uint32_t byte_off)
{
    return *reinterpret_cast<const float *>(reinterpret_cast<const char *>(p) + byte_off);
}
__device__ __forceinline__ int32_t uload_i(const int32_t *p) { return *(cint_t *)p; }
__device__ __forceinline__ int64_t uload_l(const int64_t *p) { return *(cint64_t *)p; }

// Compiler barrier that keeps a uniform branch a branch (a block containing it
// cannot be speculated and if-converted into selects).
__device__ __forceinline__ void keep_branch() { asm volatile("" ::: "memory"); }

constexpr float kInf = __builtin_inff();

// Sorted chunks of at least this many points walk pass 1 outward from the reference
// block in tiles (lane = candidate); smaller ones in groups (lane = reference).
constexpr int kTileScanMin = 8192;

__device__ __forceinline__ float absdiff(float a, float b) { return __builtin_fabsf(a - b); }

__device__ __forceinline__ uint64_t ballot(bool p) { return __builtin_amdgcn_ballot_w64(p); }

// psi(n + 1) = -gamma + H_n for integer n >= 0 in float64: upward recurrence
// psi(x) = psi(x + 1) - 1/x to x >= 16, then the asymptotic (Stirling-type)
// series psi(x) ~ ln x - 1/(2x) - sum_j B_2j / (2j x^2j) through B_10
// (Abramowitz & Stegun 6.3.18); truncation error < 1e-16 at x >= 16.
// Not inlined: its float64 constants (and those of log) would otherwise be
// hoisted out of the persistent work loop and held in VGPRs for the whole
// search, costing waves per SIMD.
__device__ __attribute__((noinline)) double psi_of_count(int n)
{
    double x = (double)n + 1.0;
    double shift = 0.0;
    while (x < 16.0) {
        shift -= 1.0 / x;
        x += 1.0;
    }
    const double r = 1.0 / x;
    const double r2 = r * r;
    const double series =
        r2 * (1.0 / 12 - r2 * (1.0 / 120 - r2 * (1.0 / 252 - r2 * (1.0 / 240 - r2 * (1.0 / 132)))));
    return log(x) - 0.5 * r - series + shift;
}

// Fixed-order butterfly sum over the 64 lanes (same order on every call).
__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1)
        v += __shfl_xor(v, o, 64);
    return v;
}

// Per-chunk coordinate base pointers (wave-uniform).
template <int DY, int DX>
struct Coords {
    static constexpr int D = 1 + DY + DX;
    const float *p[D];
    __device__ __forceinline__ Coords(const float *base, const ChunkDesc &c)
    {
#pragma unroll
        for (int m = 0; m < D; ++m)
            p[m] = (m < 1 + DY) ? base + c.tp + (int64_t)m * c.ld : base + c.s + (int64_t)(m - 1 - DY) * c.ld;
    }
};

// Joint, target-future, target-past and source-past distances of one pair.
template <int DY, int DX>
struct PairDist {
    float t, p, s;
};

template <int DY, int DX>
__device__ __forceinline__ PairDist<DY, DX> pair_dist(const float (&a)[1 + DY + DX], const float (&b)[1 + DY + DX])
{
    PairDist<DY, DX> d;
    d.t = absdiff(a[0], b[0]);
    float p = absdiff(a[1], b[1]);
#pragma unroll
    for (int m = 2; m < 1 + DY; ++m)
        p = fmaxf(p, absdiff(a[m], b[m]));
    float s = absdiff(a[1 + DY], b[1 + DY]);
#pragma unroll
    for (int m = 2 + DY; m < 1 + DY + DX; ++m)
        s = fmaxf(s, absdiff(a[m], b[m]));
    d.p = p;
    d.s = s;
    return d;
}

template <int DY, int DX, int RW>
__device__ __forceinline__ PairDist<DY, DX> pair_dist_row(const float (&a)[RW], const float (&b)[1 + DY + DX])
{
    float t[1 + DY + DX];
#pragma unroll
    for (int m = 0; m < 1 + DY + DX; ++m)
        t[m] = a[m];
    return pair_dist<DY, DX>(t, b);
}

// v_writelane_b32: returns old with lane `lane` replaced by the uniform value v.
__device__ __forceinline__ uint32_t writelane(uint32_t old, uint32_t v, int lane)
{
    // gfx9 allows one SGPR source per VALU op, so the lane select goes in M0.
    asm("v_writelane_b32 %0, %1, m0" : "+v"(old) : "s"(v), "{m0}"(lane));
    return old;
}

// Sorted-list insertion of x into the KP1 smallest values b[0] <= ... <= b[KP1-1]:
// from the top down, bi' = med3(b(i-1), bi, x), then b0' = min(b0, x).  Each
// step reads only entries not yet updated, so the list is rewritten in place
// (KP1 VALU ops, no copies).  Leaves the list unchanged when x >= b[KP1-1], so
// it can run on every lane of the wave.  All values are non-negative floats
// (+0 .. +inf), whose bit patterns order like unsigned integers; the minimum
// is taken on the bits (no NaN canonicalisation needed).
template <int KP1>
__device__ __forceinline__ void insert_sorted(float (&b)[KP1], float x)
{
#pragma unroll
    for (int i = KP1 - 1; i >= 1; --i)
        b[i] = __builtin_amdgcn_fmed3f(b[i - 1], b[i], x);
    const uint32_t lo = min(__builtin_bit_cast(uint32_t, b[0]), __builtin_bit_cast(uint32_t, x));
    b[0] = __builtin_bit_cast(float, lo);
}

template <int KP1, bool GENERIC>
__device__ __forceinline__ float kth(const float (&b)[KP1], int k)
{
    if (!GENERIC)
        return b[KP1 - 1];
    float r = b[0];
#pragma unroll
    for (int i = 1; i < KP1; ++i)
        r = (k == i) ? b[i] : r;
    return r;
}

// Work item -> chunk: the largest c with item_start[c] <= q (binary search on
// scalar loads).
__device__ __forceinline__ int find_chunk(const int32_t *item_start, int n_chunks, int q)
{
    int lo = 0, hi = n_chunks - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (uload_i(item_start + mid) <= q)
            lo = mid;
        else
            hi = mid - 1;
    }
    return lo;
}

// ---------------------------------------------------------------- the search

template <int DY, int DX, int KP1, bool GENERIC, int SLOTS, bool SORTED>
__global__ void __launch_bounds__(kMaxWavesPerWG * 64) search_kernel(SearchArgs a)
{
    constexpr int D = 1 + DY + DX;
    constexpr int RW = (D + 1 + 3) & ~3;       // LDS row: D coordinates + radius, 16-byte aligned
    constexpr bool kGroup8 = D <= 7;           // pass-1 groups of eight candidates (8 D SGPRs of data;
                                               // wider rows keep groups of four, within the SGPR budget)
    __shared__ __attribute__((aligned(16))) float rows[kMaxWavesPerWG * kWave * RW];
    const int lane = threadIdx.x & (kWave - 1);
    const int k = GENERIC ? a.k : KP1 - 1;

    const int nq = a.n_parts > 1 ? a.n_parts : 1;
    int qp = (int)(blockIdx.x % (unsigned)nq);   // this wave's queue
    int drained = 0;                              // queues found empty so far
    int last_ci = 0, last_lo = 0, last_hi = 0;    // the previous item's chunk and its item range
    unsigned long long work1 = 0, work2 = 0;      // pairs this wave evaluated in pass 1 / pass 2
    for (;;) {
        // ---- claim the next work item (wave-uniform)
        int q = 0;
        if (lane == 0)
            q = atomicAdd(a.counter + qp, 1);
        q = __builtin_amdgcn_readlane(q, 0);
        if (nq > 1) {
            q += uload_i(a.part_start + qp);
            if (q >= uload_i(a.part_start + qp + 1)) {
                if (++drained >= nq)
                    break;
                qp = qp + 1 == nq ? 0 : qp + 1;
                continue;
            }
        } else if (q >= a.n_items) {
            break;
        }
        // consecutive items of a queue are mostly blocks of one chunk
        if (q < last_lo || q >= last_hi) {
            last_ci = find_chunk(a.item_start, a.n_chunks, q);
            last_lo = uload_i(a.item_start + last_ci);
            last_hi = last_ci + 1 < a.n_chunks ? uload_i(a.item_start + last_ci + 1) : a.n_items;
        }
        const int ci = last_ci;
        ChunkDesc cd;
        {
            const char *w = reinterpret_cast<const char *>(a.chunks + ci);
            cd.tp = uload_l(reinterpret_cast<const int64_t *>(w + offsetof(ChunkDesc, tp)));
            cd.s = uload_l(reinterpret_cast<const int64_t *>(w + offsetof(ChunkDesc, s)));
            cd.ld = uload_l(reinterpret_cast<const int64_t *>(w + offsetof(ChunkDesc, ld)));
            cd.out = uload_l(reinterpret_cast<const int64_t *>(w + offsetof(ChunkDesc, out)));
            cd.pbase = uload_l(reinterpret_cast<const int64_t *>(w + offsetof(ChunkDesc, pbase)));
            cd.perm = uload_l(reinterpret_cast<const int64_t *>(w + offsetof(ChunkDesc, perm)));
            cd.n = uload_i(reinterpret_cast<const int32_t *>(w + offsetof(ChunkDesc, n)));
            cd.item0 = uload_i(reinterpret_cast<const int32_t *>(w + offsetof(ChunkDesc, item0)));
            cd.block0 = uload_i(reinterpret_cast<const int32_t *>(w + offsetof(ChunkDesc, block0)));
        }
        const int n = cd.n;
        int blk = q - cd.item0 + cd.block0;
        const int nb = (n + kWave - 1) / kWave;
        if (a.sorted && cd.block0 == 0 && last_hi - last_lo == nb) {
            // a whole sorted chunk: blocks are taken middle first (the middle of
            // the p0 order is densest, so those blocks scan most); the cheap outer
            // blocks come last and the waves of a queue end together
            const int mid = nb >> 1, kk = blk;
            const int pairs = min(mid, nb - mid);
            if (kk < 2 * pairs)
                blk = (kk & 1) ? mid - 1 - (kk >> 1) : mid + (kk >> 1);
            else
                blk = nb - mid > mid ? mid + pairs + (kk - 2 * pairs) : mid - 1 - pairs - (kk - 2 * pairs);
        }
        const int r0 = blk * kWave;
        const Coords<DY, DX> cp(a.base, cd);

        // ---- pass 1: lane = reference i, candidates uniform
        const int i = r0 + lane;
        const bool valid = i < n;
        const int ii = valid ? i : n - 1;
        float ref[D];
#pragma unroll
        for (int m = 0; m < D; ++m)
            ref[m] = cp.p[m][ii];
        float best[KP1];
#pragma unroll
        for (int s = 0; s < KP1; ++s)
            best[s] = kInf;
        float thr = kInf;

        // current k+1-th distance of this lane: a candidate can only enter the
        // list if its joint distance is strictly below it
        auto cur = [&]() { return GENERIC ? thr : best[KP1 - 1]; };
        auto visit = [&](const float (&c)[D]) {
            const PairDist<DY, DX> d = pair_dist<DY, DX>(ref, c);
            const float dj = fmaxf(d.t, fmaxf(d.p, d.s));
            if (ballot(dj < cur())) {
                keep_branch();
                insert_sorted<KP1>(best, dj);
                if (GENERIC)
                    thr = kth<KP1, GENERIC>(best, k);
            }
        };
        // four consecutive candidates j..j+3 (scalar loads, one per coordinate)
        auto load4 = [&](int j, float (&c)[4][D]) {
            const uint32_t off = (uint32_t)j * 4u;
#pragma unroll
            for (int m = 0; m < D; ++m) {
                const f4v v = uload4_at(cp.p[m], off);
                c[0][m] = v.x;
                c[1][m] = v.y;
                c[2][m] = v.z;
                c[3][m] = v.w;
            }
        };
        // Four candidates at once: their distances are independent, and a
        // candidate that is not below the current k+1-th distance leaves the list
        // unchanged when inserted (med3 / min network), so one wave-wide test of
        // the group's smallest distance decides whether any insertion is needed,
        // and a test per candidate skips the insertions no lane needs.
        auto visit_group = [&](const float (&c)[4][D]) {
            float dj[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const PairDist<DY, DX> d = pair_dist<DY, DX>(ref, c[u]);
                dj[u] = fmaxf(d.t, fmaxf(d.p, d.s));
            }
            const float m = fminf(fminf(dj[0], dj[1]), fminf(dj[2], dj[3]));
            if (ballot(m < cur())) {
                keep_branch();
#pragma unroll
                for (int u = 0; u < 4; ++u)
                    if (ballot(dj[u] < cur())) {
                        keep_branch();
                        insert_sorted<KP1>(best, dj[u]);
                        if (GENERIC)
                            thr = kth<KP1, GENERIC>(best, k);
                    }
            }
        };
        auto visit4 = [&](int j) {
            float c[4][D];
            load4(j, c);
            visit_group(c);
        };
        // eight consecutive candidates j..j+7, one scalar load per coordinate
        auto load8 = [&](int j, float (&c)[8][D]) {
            const uint32_t off = (uint32_t)j * 4u;
#pragma unroll
            for (int m = 0; m < D; ++m) {
                const f8v v = uload8_at(cp.p[m], off);
#pragma unroll
                for (int u = 0; u < 8; ++u)
                    c[u][m] = v[u];
            }
        };
        auto visit_group8 = [&](const float (&c)[8][D]) {
            float dj[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const PairDist<DY, DX> d = pair_dist<DY, DX>(ref, c[u]);
                dj[u] = fmaxf(d.t, fmaxf(d.p, d.s));
            }
            const float m = fminf(fminf(fminf(dj[0], dj[1]), fminf(dj[2], dj[3])),
                                  fminf(fminf(dj[4], dj[5]), fminf(dj[6], dj[7])));
            if (ballot(m < cur())) {
                keep_branch();
#pragma unroll
                for (int u = 0; u < 8; ++u)
                    if (ballot(dj[u] < cur())) {
                        keep_branch();
                        insert_sorted<KP1>(best, dj[u]);
                        if (GENERIC)
                            thr = kth<KP1, GENERIC>(best, k);
                    }
            }
        };
        auto visit1 = [&](int j) {
            float c[D];
#pragma unroll
            for (int m = 0; m < D; ++m)
                c[m] = uload(cp.p[m] + j);
            visit(c);
        };
        // In a chunk sorted by the first target-past coordinate p0, the joint
        // distance to candidate j is at least |fl32(p0_i - p0_j)|, which grows
        // monotonically away from the reference block (rounding is monotone).

        // (reference, candidate) pairs examined in pass 1
        unsigned long long pass1_pairs = (unsigned long long)n * (unsigned long long)min(kWave, n - r0);
        int scan_lo = 0, scan_hi = n;                     // pass 1 examined [scan_lo, scan_hi)
        if (!SORTED) {
            int j = 0;
            for (; j + 4 <= n; j += 4)
                visit4(j);
            for (; j < n; ++j)
                visit1(j);
        } else {
            const int e0 = min(n, r0 + kWave);
            int j = r0;                                   // the block's own points first
            if constexpr (kGroup8)
                for (; j + 8 <= e0; j += 8) {
                    float c[8][D];
                    load8(j, c);
                    visit_group8(c);
                }
            for (; j + 4 <= e0; j += 4)
                visit4(j);
            for (; j < e0; ++j)
                visit1(j);
            // Outward from the block: for chunks of at least kTileScanMin points in tiles of
            // 64 x TS candidates against the references whose windows reach them, below
            // that in groups of candidates against all 64 references (where a chunk is
            // small, the 64 windows nearly coincide and the groups' scalar loads cost less).
            int f, b;
            unsigned long long ev = (unsigned long long)(e0 - r0) * (unsigned long long)min(kWave, n - r0);
            if (n >= kTileScanMin) {
                // Then outward in tiles of 64 candidates, one per lane, alternating forward
                // (p0 increasing) and backward: a tile is compared only with the references
                // whose p0 window [p0 - r, p0 + r] (r their current (k+1)-th distance) reaches
                // the tile's p0 span, read back as LDS broadcasts; a candidate below a
                // reference's current (k+1)-th distance is moved to the reference's lane and
                // inserted there.  A direction ends at the first tile that no reference
                // reaches: every later candidate on that side is farther in p0.
                // LDS row of a reference: its coordinates, then its current (k+1)-th distance
                float *prow = rows + (threadIdx.x / kWave) * (kWave * RW);
                __builtin_amdgcn_wave_barrier();
#pragma unroll
                for (int m = 0; m < D; ++m)
                    prow[lane * RW + m] = ref[m];
                prow[lane * RW + D] = cur();
                __builtin_amdgcn_wave_barrier();
                constexpr int TS = 2;                        // a tile: 64 x TS candidates
                auto read_row = [&](int r, float (&rr)[RW]) {
                    const f4v *rowv = reinterpret_cast<const f4v *>(prow + r * RW);
#pragma unroll
                    for (int x = 0; x < RW / 4; ++x) {
                        const f4v q4 = rowv[x];
                        rr[4 * x + 0] = q4.x;
                        rr[4 * x + 1] = q4.y;
                        rr[4 * x + 2] = q4.z;
                        rr[4 * x + 3] = q4.w;
                    }
                };
                auto tile = [&](int t0, int t1) {
                    float cand[TS][D];
#pragma unroll
                    for (int sl = 0; sl < TS; ++sl) {
                        const int idx = t0 + sl * kWave + lane;
                        const bool ok = idx < t1;
                        const uint32_t ic4 = (uint32_t)(ok ? idx : t0) * 4u;
#pragma unroll
                        for (int m = 0; m < D; ++m) {
                            const float v = vload_at(cp.p[m], ic4);
                            cand[sl][m] = ok ? v : kInf;
                        }
                    }
                    const float tlo = uload(cp.p[1] + t0), thi = uload(cp.p[1] + t1 - 1);
                    const float c0 = cur();
                    uint64_t todo = ballot(valid && !(tlo - ref[1] >= c0 || ref[1] - thi >= c0));
                    ev += (unsigned long long)__builtin_popcountll(todo) * (unsigned long long)(t1 - t0);
                    // the candidates of the tile against reference r (row rr), in the reference's lane
                    auto against = [&](int r, const float (&rr)[RW]) {
                        float ut = rr[D];
#pragma unroll
                        for (int sl = 0; sl < TS; ++sl) {
                            const PairDist<DY, DX> d = pair_dist_row<DY, DX, RW>(rr, cand[sl]);
                            const float dj = fmaxf(d.t, fmaxf(d.p, d.s));
                            uint64_t hit = ballot(dj < ut);
                            while (hit != 0) {
                                keep_branch();
                                const int c = __builtin_ctzll(hit);
                                const float x =
                                    __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, dj), c));
                                if (lane == r) {
                                    insert_sorted<KP1>(best, x);
                                    if (GENERIC)
                                        thr = kth<KP1, GENERIC>(best, k);
                                    prow[r * RW + D] = cur();
                                }
                                ut = __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, cur()), r));
                                hit &= hit - 1;
                                hit &= ballot(dj < ut);
                            }
                        }
                    };
                    // two row buffers used in turn: the next reference's row is read while the
                    // current one is compared (rows of different references: an insertion
                    // rewrites only its own reference's row)
                    if (todo != 0) {
                        float ra[RW], rb[RW];
                        int ia = __builtin_ctzll(todo);
                        todo &= todo - 1;
                        read_row(ia, ra);
                        for (;;) {
                            const bool mb = todo != 0;
                            int ib = ia;
                            if (mb) {
                                ib = __builtin_ctzll(todo);
                                todo &= todo - 1;
                                read_row(ib, rb);
                            }
                            __builtin_amdgcn_sched_barrier(0);
                            against(ia, ra);
                            if (!mb)
                                break;
                            const bool mc = todo != 0;
                            int ic = ib;
                            if (mc) {
                                ic = __builtin_ctzll(todo);
                                todo &= todo - 1;
                                read_row(ic, ra);
                            }
                            __builtin_amdgcn_sched_barrier(0);
                            against(ib, rb);
                            if (!mc)
                                break;
                            ia = ic;
                        }
                    }
                };
                f = e0;
                b = r0;
                bool fgo = f < n && ballot(valid && absdiff(ref[1], uload(cp.p[1] + f)) < cur()) != 0;
                bool bgo = b > 0 && ballot(valid && absdiff(ref[1], uload(cp.p[1] + b - 1)) < cur()) != 0;
                while (fgo || bgo) {
                    if (fgo) {
                        const int t1 = min(n, f + kWave * TS);
                        tile(f, t1);
                        f = t1;
                        fgo = f < n && ballot(valid && absdiff(ref[1], uload(cp.p[1] + f)) < cur()) != 0;
                    }
                    if (bgo) {
                        const int t0 = max(0, b - kWave * TS);
                        tile(t0, b);
                        b = t0;
                        bgo = b > 0 && ballot(valid && absdiff(ref[1], uload(cp.p[1] + b - 1)) < cur()) != 0;
                    }
                }
            } else {
                // then outward: forward (p0 increasing), then backward, a group of eight
                // (four for wide rows, then four for the remainder) at a time.  After
                // each group, its candidate farthest from the block is tested: if no
                // lane could still use it, no later candidate of that direction could
                // either (so the next group is not loaded).  All loads of a group feed
                // its distances unconditionally: one wait per group.
                f = e0;
                bool go = f < n;
                while (kGroup8 && go && f + 8 <= n) {
                    float c[8][D];
                    load8(f, c);
                    visit_group8(c);
                    f += 8;
                    go = f < n && ballot(absdiff(ref[1], c[7][1]) < cur()) != 0;
                }
                while (go && f + 4 <= n) {
                    float c[4][D];
                    load4(f, c);
                    visit_group(c);
                    f += 4;
                    go = f < n && ballot(absdiff(ref[1], c[3][1]) < cur()) != 0;
                }
                while (go && f < n) {
                    const float p0 = uload(cp.p[1] + f);
                    visit1(f);
                    ++f;
                    go = f < n && ballot(absdiff(ref[1], p0) < cur()) != 0;
                }
                b = r0;
                go = b > 0;
                while (kGroup8 && go && b >= 8) {
                    float c[8][D];
                    load8(b - 8, c);
                    visit_group8(c);
                    b -= 8;
                    go = b > 0 && ballot(absdiff(ref[1], c[0][1]) < cur()) != 0;
                }
                while (go && b >= 4) {
                    float c[4][D];
                    load4(b - 4, c);
                    visit_group(c);
                    b -= 4;
                    go = b > 0 && ballot(absdiff(ref[1], c[0][1]) < cur()) != 0;
                }
                while (go && b > 0) {
                    const float p0 = uload(cp.p[1] + b - 1);
                    visit1(b - 1);
                    --b;
                    go = b > 0 && ballot(absdiff(ref[1], p0) < cur()) != 0;
                }
                ev = (unsigned long long)(f - b) * (unsigned long long)min(kWave, n - r0);
            }
            pass1_pairs = ev;
            scan_lo = b;
            scan_hi = f;
        }
        // k+1-th smallest including self (distance 0) = k-th neighbour without self
        const float eps = cur();

        // ---- pass 2: lane = candidate, references uniform
        // Each lane parks its reference row (coordinates, then the radius) in
        // this wave's LDS rows; the counting loop reads them back as
        // wave-wide broadcasts, so a reference costs no SALU address work.
        float *myrows = rows + (threadIdx.x / kWave) * (kWave * RW);
        __builtin_amdgcn_wave_barrier();
#pragma unroll
        for (int m = 0; m < D; ++m)
            myrows[lane * RW + m] = ref[m];
        myrows[lane * RW + D] = eps;
        __builtin_amdgcn_wave_barrier();

        // Candidate range [lo, hi): in a sorted chunk every point outside it is at
        // |fl32(p0_i - p0_j)| >= eps_i from every reference of the block, hence
        // outside all three marginal balls (each contains the target-past block).
        // Pass 1 stopped each direction at a candidate no lane could use with a
        // radius >= eps_i, so the range lies inside the one pass 1 examined; it is
        // narrowed from there in steps of 64 points that no reference reaches.
        int lo = 0, hi = n;
        if (SORTED) {
            const int e0 = min(n, r0 + kWave);
            hi = scan_hi;
            while (hi - kWave >= e0 && !ballot(valid && absdiff(ref[1], uload(cp.p[1] + hi - kWave)) < eps))
                hi -= kWave;
            lo = scan_lo;
            while (lo + kWave <= r0 && !ballot(valid && absdiff(ref[1], uload(cp.p[1] + lo + kWave - 1)) < eps))
                lo += kWave;
        }

        const int nref = min(kWave, n - r0);
        uint32_t accP = 0, accTP = 0, accPS = 0;
        unsigned long long evaluated2 = 0;                // candidate-reference pairs examined in pass 2
        for (int t0 = lo; t0 < hi; t0 += kWave * SLOTS) {
            float cand[SLOTS][D];
#pragma unroll
            for (int sl = 0; sl < SLOTS; ++sl) {
                const int idx = t0 + sl * kWave + lane;
                const bool ok = idx < hi;
                // in-bounds load, lanes past the range masked below
                const uint32_t ic4 = (uint32_t)(ok ? idx : n - 1) * 4u;
#pragma unroll
                for (int m = 0; m < D; ++m) {
                    const float v = vload_at(cp.p[m], ic4);
                    cand[sl][m] = ok ? v : kInf;
                }
            }
            uint32_t tP = 0, tTP = 0, tPS = 0;
            // p0 range of this tile's candidates (sorted chunks): first and last in range
            float tlo = 0.0f, thi = 0.0f;
            if (SORTED) {
                tlo = uload(cp.p[1] + t0);
                thi = uload(cp.p[1] + min(t0 + kWave * SLOTS, hi) - 1);
            }
            // references that can reach this tile: one lane-parallel test (each lane
            // holds its own reference); in a sorted chunk a reference whose window
            // [p0 - eps, p0 + eps] misses the tile's p0 range has nothing to count
            // here and keeps the zero its lane starts the tile with
            bool reach = valid;
            if (SORTED)
                reach = reach && !(tlo - ref[1] >= eps || ref[1] - thi >= eps);
            uint64_t todo = ballot(reach);
            evaluated2 += (unsigned long long)__builtin_popcountll(todo) *
                          (unsigned long long)min(kWave * SLOTS, hi - t0);
            auto read_row = [&](int r, f4v (&row)[RW / 4]) {
                const f4v *rowv = reinterpret_cast<const f4v *>(myrows + r * RW);
#pragma unroll
                for (int v = 0; v < RW / 4; ++v)
                    row[v] = rowv[v];
            };
            // orders a row's counting after the reads issued before it
            auto pin_row = [&](f4v (&row)[RW / 4]) {
#pragma unroll
                for (int v = 0; v < RW / 4; ++v)
                    asm volatile("" : "+v"(row[v]));
            };
            auto count_ref = [&](const f4v (&row)[RW / 4], int r) {
                float rr[RW];
#pragma unroll
                for (int v = 0; v < RW / 4; ++v) {
                    rr[4 * v + 0] = row[v].x;
                    rr[4 * v + 1] = row[v].y;
                    rr[4 * v + 2] = row[v].z;
                    rr[4 * v + 3] = row[v].w;
                }
                const float er = rr[D];
                uint32_t sP = 0, sTP = 0, sPS = 0;
#pragma unroll
                for (int sl = 0; sl < SLOTS; ++sl) {
                    const PairDist<DY, DX> d = pair_dist_row<DY, DX, RW>(rr, cand[sl]);
                    const uint64_t mT = ballot(d.t < er);
                    const uint64_t mP = ballot(d.p < er);
                    const uint64_t mS = ballot(d.s < er);
                    sP += (uint32_t)__builtin_popcountll(mP);
                    sTP += (uint32_t)__builtin_popcountll(mP & mT);
                    sPS += (uint32_t)__builtin_popcountll(mP & mS);
                }
                tP = writelane(tP, sP, r);
                tTP = writelane(tTP, sTP, r);
                tPS = writelane(tPS, sPS, r);
            };
            // rows of up to 8 floats (D <= 7): two row buffers used in turn, the
            // next reference's row read from LDS while the current one is counted.  Each round counts two
            // references; with an odd number the last one is counted twice, which
            // writes the same sums to the same lane.
            if constexpr (RW <= 8) {
            if (todo != 0) {
                f4v ra[RW / 4], rb[RW / 4];
                int ia = __builtin_ctzll(todo);
                todo &= todo - 1;
                read_row(ia, ra);
                for (;;) {
                    int ib = ia;
                    if (todo != 0) {
                        ib = __builtin_ctzll(todo);
                        todo &= todo - 1;
                    }
                    read_row(ib, rb);
                    __builtin_amdgcn_sched_barrier(0);
                    pin_row(ra);
                    count_ref(ra, ia);
                    const bool more = todo != 0;
                    int in = ib;
                    if (more) {
                        in = __builtin_ctzll(todo);
                        todo &= todo - 1;
                    }
                    read_row(in, ra);
                    __builtin_amdgcn_sched_barrier(0);
                    pin_row(rb);
                    count_ref(rb, ib);
                    if (!more)
                        break;
                    ia = in;
                }
            }
            } else {
            // wider rows (D > 7): one buffer, so that the occupancy is kept
            while (todo != 0) {
                const int r = __builtin_ctzll(todo);
                todo &= todo - 1;
                f4v ra[RW / 4];
                read_row(r, ra);
                count_ref(ra, r);
            }
            }
            accP += tP;
            accTP += tTP;
            accPS += tPS;
        }
        // self is at distance 0 in every space: counted iff eps > 0
        const uint32_t self = eps > 0.0f ? 1u : 0u;
        const int nP = (int)(accP - self), nTP = (int)(accTP - self), nPS = (int)(accPS - self);

        // ---- per-point digamma terms of eq. 9, summed over the item in fixed order
        double term = 0.0;
        if (valid)
            term = psi_of_count(nP) - psi_of_count(nTP) - psi_of_count(nPS);
        const double sum = wave_sum(term);
        if (lane == 0)
            a.partial[cd.pbase + blk] = sum;
        work1 += pass1_pairs;
        work2 += evaluated2;
        if (a.lte_out != nullptr && cd.out >= 0 && valid) {
            int o = (cd.perm >= 0) ? a.perm_base[cd.perm + i] : i;
            if (o < 0 || o >= n)
                o = i;
            a.lte_out[cd.out + o] = psi_of_count(k - 1) + term;
        }
        if (a.eps_out != nullptr && cd.out >= 0 && valid) {
            // per-point outputs go to the point's index before sorting
            int o = (cd.perm >= 0) ? a.perm_base[cd.perm + i] : i;
            if (o < 0 || o >= n)         // keep writes inside the chunk's output range regardless
                o = i;
            a.eps_out[cd.out + o] = eps;
            a.cnt_out[cd.out + o] = nP;
            a.cnt_out[a.cnt_stride + cd.out + o] = nTP;
            a.cnt_out[2 * a.cnt_stride + cd.out + o] = nPS;
        }
    }
    // measurement: one pair of counter updates per wave, after its last item
    if (a.work != nullptr && lane == 0) {
        atomicAdd(a.work, work1);
        atomicAdd(a.work + 1, work2);
        atomicAdd(a.work + 2, work1);
        atomicAdd(a.work + 3, work2);
    }
}

// ------------------------------------------------ the search over chunk sets
//
// The chunks of one window (its original and its surrogates, or its delays)
// share the (y_t', Y_past) block and its sorted order and differ only in the
// source block.  This variant searches a set of up to V such chunks per work
// item: for every (reference, candidate) pair the target-future and
// target-past differences are taken once, and only the source-past part is
// evaluated per chunk.  Radii, counts and per-item sums are those of the
// single-chunk search bit for bit (the same float operations decide every
// comparison; only the order in which independent pairs are visited and which
// lanes share a step differ).  Sorted chunks only.
//
//   d_J(v) = max(d_TP, d_S(v)),  d_TP = max(d_T, d_P)
//   n_TP  counts [d_TP < eps_v],  n_PS counts [max(d_P, d_S(v)) < eps_v]
//
// A set is a run of consecutive chunk descriptors [set_first[c], set_first[c+1]);
// its first descriptor supplies tp, ld, n, item0 and block0, each descriptor
// its own s and pbase.  Sets with fewer than V chunks repeat their last chunk
// in the unused variant slots and do not store those slots' sums.

// Wide sets (a candidate's coordinates, 1 + d_y + V d_x, at least 16) keep their per-tile counts packed three
// to a register (PACK) and are compiled for six waves per SIMD; see the kernels after this body.
template <int DY, int DX, int V, int SLOTS, bool PACK>
__device__ __forceinline__ void sets_search(const SearchArgs &a)
{
    constexpr int DT = 1 + DY;                 // shared coordinates: y_t' and the target past
    constexpr int KP1 = 5;                     // k = 4: the k+1 smallest distances, self included
    constexpr int NR = DT + V * DX + V;        // LDS row: shared coordinates, V source blocks, V radii
    constexpr int RW = (NR + 3) & ~3;
    constexpr int MO = DT > DX ? DT : DX;      // coordinate offsets shared by the target and source blocks
    extern __shared__ __attribute__((aligned(16))) float rows[];   // waves per workgroup x 64 x RW floats
    const int lane = threadIdx.x & (kWave - 1);

    const int nq = a.n_parts > 1 ? a.n_parts : 1;
    int qp = (int)(blockIdx.x % (unsigned)nq);
    int drained = 0;
    int last_ci = 0, last_lo = 0, last_hi = 0;
    unsigned long long work1 = 0, work2 = 0, shared1 = 0, shared2 = 0;
    for (;;) {
        int q = 0;
        if (lane == 0)
            q = atomicAdd(a.counter + qp, 1);
        q = __builtin_amdgcn_readlane(q, 0);
        if (nq > 1) {
            q += uload_i(a.part_start + qp);
            if (q >= uload_i(a.part_start + qp + 1)) {
                if (++drained >= nq)
                    break;
                qp = qp + 1 == nq ? 0 : qp + 1;
                continue;
            }
        } else if (q >= a.n_items) {
            break;
        }
        if (q < last_lo || q >= last_hi) {
            last_ci = find_chunk(a.item_start, a.n_chunks, q);
            last_lo = uload_i(a.item_start + last_ci);
            last_hi = last_ci + 1 < a.n_chunks ? uload_i(a.item_start + last_ci + 1) : a.n_items;
        }
        const int c0 = uload_i(a.set_first + last_ci);
        const int cnt = uload_i(a.set_first + last_ci + 1) - c0;   // chunks in the set, 1..V
        const char *w0 = reinterpret_cast<const char *>(a.chunks + c0);
        const int64_t tp = uload_l(reinterpret_cast<const int64_t *>(w0 + offsetof(ChunkDesc, tp)));
        const int64_t ld = uload_l(reinterpret_cast<const int64_t *>(w0 + offsetof(ChunkDesc, ld)));
        const int n = uload_i(reinterpret_cast<const int32_t *>(w0 + offsetof(ChunkDesc, n)));
        const int item0 = uload_i(reinterpret_cast<const int32_t *>(w0 + offsetof(ChunkDesc, item0)));
        const int block0 = uload_i(reinterpret_cast<const int32_t *>(w0 + offsetof(ChunkDesc, block0)));
        const float *tb = a.base + tp;                 // target block of the set
        const float *sb[V];                            // source block of each variant
        int64_t pb[V];
#pragma unroll
        for (int v = 0; v < V; ++v) {
            const char *wv = reinterpret_cast<const char *>(a.chunks + c0 + min(v, cnt - 1));
            sb[v] = a.base + uload_l(reinterpret_cast<const int64_t *>(wv + offsetof(ChunkDesc, s)));
            pb[v] = uload_l(reinterpret_cast<const int64_t *>(wv + offsetof(ChunkDesc, pbase)));
        }
        uint32_t moff[MO];                             // byte offset of coordinate m within a block
#pragma unroll
        for (int m = 0; m < MO; ++m)
            moff[m] = (uint32_t)((int64_t)m * ld * 4);

        int blk = q - item0 + block0;
        const int nb = (n + kWave - 1) / kWave;
        if (block0 == 0 && last_hi - last_lo == nb) {
            // middle blocks (densest in the p0 order) first, as in the single-chunk search
            const int mid = nb >> 1, kk = blk;
            const int pairs = min(mid, nb - mid);
            if (kk < 2 * pairs)
                blk = (kk & 1) ? mid - 1 - (kk >> 1) : mid + (kk >> 1);
            else
                blk = nb - mid > mid ? mid + pairs + (kk - 2 * pairs) : mid - 1 - pairs - (kk - 2 * pairs);
        }
        const int r0 = blk * kWave;

        // ---- pass 1: lane = reference i
        const int i = r0 + lane;
        const bool valid = i < n;
        const int ii = valid ? i : n - 1;
        float rt[DT];
        float rs[V][DX];
#pragma unroll
        for (int m = 0; m < DT; ++m)
            rt[m] = tb[(int64_t)m * ld + ii];
#pragma unroll
        for (int v = 0; v < V; ++v)
#pragma unroll
            for (int m = 0; m < DX; ++m)
                rs[v][m] = sb[v][(int64_t)m * ld + ii];
        float best[V][KP1];
#pragma unroll
        for (int v = 0; v < V; ++v)
#pragma unroll
            for (int s = 0; s < KP1; ++s)
                best[v][s] = kInf;
        // largest current k+1-th distance over the variants: a candidate farther
        // than it in p0 is of no use to any variant
        auto curmax = [&]() {
            float c = best[0][KP1 - 1];
#pragma unroll
            for (int v = 1; v < V; ++v)
                c = fmaxf(c, best[v][KP1 - 1]);
            return c;
        };
        // four consecutive candidates j..j+3: target coordinates ct, source coordinates cs
        auto load4 = [&](int j, float (&ct)[4][DT], float (&cs)[V][4][DX]) {
            const uint32_t off = (uint32_t)j * 4u;
#pragma unroll
            for (int m = 0; m < DT; ++m) {
                const f4v x = uload4_at(tb, moff[m] + off);
                ct[0][m] = x.x;
                ct[1][m] = x.y;
                ct[2][m] = x.z;
                ct[3][m] = x.w;
            }
#pragma unroll
            for (int v = 0; v < V; ++v)
#pragma unroll
                for (int m = 0; m < DX; ++m) {
                    const f4v x = uload4_at(sb[v], moff[m] + off);
                    cs[v][0][m] = x.x;
                    cs[v][1][m] = x.y;
                    cs[v][2][m] = x.z;
                    cs[v][3][m] = x.w;
                }
        };
        auto visit4 = [&](const float (&ct)[4][DT], const float (&cs)[V][4][DX]) {
            float dtp[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                float d = absdiff(rt[0], ct[u][0]);
#pragma unroll
                for (int m = 1; m < DT; ++m)
                    d = fmaxf(d, absdiff(rt[m], ct[u][m]));
                dtp[u] = d;
            }
#pragma unroll
            for (int v = 0; v < V; ++v) {
                float dj[4];
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    float d = absdiff(rs[v][0], cs[v][u][0]);
#pragma unroll
                    for (int m = 1; m < DX; ++m)
                        d = fmaxf(d, absdiff(rs[v][m], cs[v][u][m]));
                    dj[u] = fmaxf(dtp[u], d);
                }
                const float mn = fminf(fminf(dj[0], dj[1]), fminf(dj[2], dj[3]));
                if (ballot(mn < best[v][KP1 - 1])) {
                    keep_branch();
#pragma unroll
                    for (int u = 0; u < 4; ++u)
                        if (ballot(dj[u] < best[v][KP1 - 1])) {
                            keep_branch();
                            insert_sorted<KP1>(best[v], dj[u]);
                        }
                }
            }
        };
        auto visit1 = [&](int j) {
            float dtp = absdiff(rt[0], uload(tb + j));
#pragma unroll
            for (int m = 1; m < DT; ++m)
                dtp = fmaxf(dtp, absdiff(rt[m], uload(tb + (int64_t)m * ld + j)));
#pragma unroll
            for (int v = 0; v < V; ++v) {
                float d = absdiff(rs[v][0], uload(sb[v] + j));
#pragma unroll
                for (int m = 1; m < DX; ++m)
                    d = fmaxf(d, absdiff(rs[v][m], uload(sb[v] + (int64_t)m * ld + j)));
                const float dj = fmaxf(dtp, d);
                if (ballot(dj < best[v][KP1 - 1])) {
                    keep_branch();
                    insert_sorted<KP1>(best[v], dj);
                }
            }
        };

        // the block's own points, then outward in p0 order, forward then backward;
        // a direction stops at the first group whose farthest candidate no lane of
        // any variant could use (p0 is coordinate 1, a target-past coordinate)
        const int e0 = min(n, r0 + kWave);
        int j = r0;
        for (; j + 4 <= e0; j += 4) {
            float ct[4][DT], cs[V][4][DX];
            load4(j, ct, cs);
            visit4(ct, cs);
        }
        for (; j < e0; ++j)
            visit1(j);
        // Outward from the block: for chunks of at least kTileScanMin points in tiles of 64
        // candidates against the references whose windows reach them, below that in groups
        // of four candidates against all 64 references.
        int f, b;
        unsigned long long ev = (unsigned long long)(e0 - r0) * (unsigned long long)min(kWave, n - r0);
        if (n >= kTileScanMin) {
            // then outward in tiles of 64 candidates (lane = candidate), alternating forward and
            // backward, each compared only with the references whose p0 window at their largest
            // current radius reaches the tile; the LDS row of a reference holds its coordinates
            // and its current (k+1)-th distance per variant
            float *prow = rows + (threadIdx.x / kWave) * (kWave * RW);
            __builtin_amdgcn_wave_barrier();
#pragma unroll
            for (int m = 0; m < DT; ++m)
                prow[lane * RW + m] = rt[m];
#pragma unroll
            for (int v = 0; v < V; ++v) {
#pragma unroll
                for (int m = 0; m < DX; ++m)
                    prow[lane * RW + DT + v * DX + m] = rs[v][m];
                prow[lane * RW + DT + V * DX + v] = best[v][KP1 - 1];
            }
            __builtin_amdgcn_wave_barrier();
            auto read_row = [&](int r, float (&rr)[RW]) {
                const f4v *rowv = reinterpret_cast<const f4v *>(prow + r * RW);
#pragma unroll
                for (int x = 0; x < RW / 4; ++x) {
                    const f4v q4 = rowv[x];
                    rr[4 * x + 0] = q4.x;
                    rr[4 * x + 1] = q4.y;
                    rr[4 * x + 2] = q4.z;
                    rr[4 * x + 3] = q4.w;
                }
            };
            // a tile: 64 x TS candidates; two slots only where their coordinates stay few (the
            // candidate registers of a second slot would otherwise cost a wave per SIMD)
            constexpr int TS = (DT + V * DX <= 8) ? 2 : 1;
            auto tile = [&](int t0, int t1) {
                float ct[TS][DT], cs[TS][V][DX];
#pragma unroll
                for (int sl = 0; sl < TS; ++sl) {
                    const int idx = t0 + sl * kWave + lane;
                    const bool ok = idx < t1;
                    const uint32_t ic4 = (uint32_t)(ok ? idx : t0) * 4u;
#pragma unroll
                    for (int m = 0; m < DT; ++m) {
                        const float x = vload_at(tb, moff[m] + ic4);
                        ct[sl][m] = ok ? x : kInf;
                    }
#pragma unroll
                    for (int v = 0; v < V; ++v)
#pragma unroll
                        for (int m = 0; m < DX; ++m) {
                            const float x = vload_at(sb[v], moff[m] + ic4);
                            cs[sl][v][m] = ok ? x : kInf;
                        }
                }
                const float tlo = uload(tb + ld + t0), thi = uload(tb + ld + t1 - 1);
                const float c0 = curmax();
                uint64_t todo = ballot(valid && !(tlo - rt[1] >= c0 || rt[1] - thi >= c0));
                ev += (unsigned long long)__builtin_popcountll(todo) * (unsigned long long)(t1 - t0);
                // the tile against reference r (row rr): one branch per slot when no variant of the
                // reference improves, which is the common case once its lists have settled
                auto against = [&](int r, const float (&rr)[RW]) {
                    float ut[V];
#pragma unroll
                    for (int v = 0; v < V; ++v)
                        ut[v] = rr[DT + V * DX + v];
#pragma unroll
                    for (int sl = 0; sl < TS; ++sl) {
                        float dtp = absdiff(rr[0], ct[sl][0]);
#pragma unroll
                        for (int m = 1; m < DT; ++m)
                            dtp = fmaxf(dtp, absdiff(rr[m], ct[sl][m]));
                        float dj[V];
                        uint64_t hm[V], any = 0;
#pragma unroll
                        for (int v = 0; v < V; ++v) {
                            float d = absdiff(rr[DT + v * DX], cs[sl][v][0]);
#pragma unroll
                            for (int m = 1; m < DX; ++m)
                                d = fmaxf(d, absdiff(rr[DT + v * DX + m], cs[sl][v][m]));
                            dj[v] = fmaxf(dtp, d);
                            hm[v] = ballot(dj[v] < ut[v]);
                            any |= hm[v];
                        }
                        if (any == 0)
                            continue;
                        keep_branch();
#pragma unroll
                        for (int v = 0; v < V; ++v) {
                            uint64_t hit = hm[v];
                            while (hit != 0) {
                                keep_branch();
                                const int c = __builtin_ctzll(hit);
                                const float x = __builtin_bit_cast(
                                    float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, dj[v]), c));
                                if (lane == r) {
                                    insert_sorted<KP1>(best[v], x);
                                    prow[r * RW + DT + V * DX + v] = best[v][KP1 - 1];
                                }
                                ut[v] = __builtin_bit_cast(
                                    float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, best[v][KP1 - 1]), r));
                                hit &= hit - 1;
                                hit &= ballot(dj[v] < ut[v]);
                            }
                        }
                    }
                };
                while (todo != 0) {
                    const int r = __builtin_ctzll(todo);
                    todo &= todo - 1;
                    float rr[RW];
                    read_row(r, rr);
                    against(r, rr);
                }
            };
            f = e0;
            b = r0;
            bool fgo = f < n && ballot(valid && absdiff(rt[1], uload(tb + ld + f)) < curmax()) != 0;
            bool bgo = b > 0 && ballot(valid && absdiff(rt[1], uload(tb + ld + b - 1)) < curmax()) != 0;
            while (fgo || bgo) {
                if (fgo) {
                    const int t1 = min(n, f + kWave * TS);
                    tile(f, t1);
                    f = t1;
                    fgo = f < n && ballot(valid && absdiff(rt[1], uload(tb + ld + f)) < curmax()) != 0;
                }
                if (bgo) {
                    const int t0 = max(0, b - kWave * TS);
                    tile(t0, b);
                    b = t0;
                    bgo = b > 0 && ballot(valid && absdiff(rt[1], uload(tb + ld + b - 1)) < curmax()) != 0;
                }
            }
        } else {
            f = e0;
            bool go = f < n;
            while (go && f + 4 <= n) {
                float ct[4][DT], cs[V][4][DX];
                load4(f, ct, cs);
                visit4(ct, cs);
                f += 4;
                go = f < n && ballot(absdiff(rt[1], ct[3][1]) < curmax()) != 0;
            }
            while (go && f < n) {
                const float p0 = uload(tb + ld + f);
                visit1(f);
                ++f;
                go = f < n && ballot(absdiff(rt[1], p0) < curmax()) != 0;
            }
            b = r0;
            go = b > 0;
            while (go && b >= 4) {
                float ct[4][DT], cs[V][4][DX];
                load4(b - 4, ct, cs);
                visit4(ct, cs);
                b -= 4;
                go = b > 0 && ballot(absdiff(rt[1], ct[0][1]) < curmax()) != 0;
            }
            while (go && b > 0) {
                const float p0 = uload(tb + ld + b - 1);
                visit1(b - 1);
                --b;
                go = b > 0 && ballot(absdiff(rt[1], p0) < curmax()) != 0;
            }
            ev = (unsigned long long)(f - b) * (unsigned long long)min(kWave, n - r0);
        }
        float eps[V];
#pragma unroll
        for (int v = 0; v < V; ++v)
            eps[v] = best[v][KP1 - 1];
        const float emax = curmax();

        // ---- pass 2: lane = candidate, references uniform from this wave's LDS rows
        float *myrows = rows + (threadIdx.x / kWave) * (kWave * RW);
        __builtin_amdgcn_wave_barrier();
#pragma unroll
        for (int m = 0; m < DT; ++m)
            myrows[lane * RW + m] = rt[m];
#pragma unroll
        for (int v = 0; v < V; ++v) {
#pragma unroll
            for (int m = 0; m < DX; ++m)
                myrows[lane * RW + DT + v * DX + m] = rs[v][m];
            myrows[lane * RW + DT + V * DX + v] = eps[v];
        }
        __builtin_amdgcn_wave_barrier();

        // candidate range: outside it every point is at |fl32(p0_i - p0_j)| >= the
        // largest radius of every reference of the block
        int hi = f;
        while (hi - kWave >= e0 && !ballot(valid && absdiff(rt[1], uload(tb + ld + hi - kWave)) < emax))
            hi -= kWave;
        int lo = b;
        while (lo + kWave <= r0 && !ballot(valid && absdiff(rt[1], uload(tb + ld + lo + kWave - 1)) < emax))
            lo += kWave;

        const int nref = min(kWave, n - r0);
        uint32_t accP[V], accTP[V], accPS[V];
#pragma unroll
        for (int v = 0; v < V; ++v)
            accP[v] = accTP[v] = accPS[v] = 0;
        unsigned long long evaluated2 = 0;
        for (int t0 = lo; t0 < hi; t0 += kWave * SLOTS) {
            float ct[SLOTS][DT], cs[SLOTS][V][DX];
#pragma unroll
            for (int sl = 0; sl < SLOTS; ++sl) {
                const int idx = t0 + sl * kWave + lane;
                const bool ok = idx < hi;
                const uint32_t ic4 = (uint32_t)(ok ? idx : n - 1) * 4u;
#pragma unroll
                for (int m = 0; m < DT; ++m) {
                    const float x = vload_at(tb, moff[m] + ic4);
                    ct[sl][m] = ok ? x : kInf;
                }
#pragma unroll
                for (int v = 0; v < V; ++v)
#pragma unroll
                    for (int m = 0; m < DX; ++m) {
                        const float x = vload_at(sb[v], moff[m] + ic4);
                        cs[sl][v][m] = ok ? x : kInf;
                    }
            }
            const float tlo = uload(tb + ld + t0);
            const float thi = uload(tb + ld + min(t0 + kWave * SLOTS, hi) - 1);
            const bool reach = valid && !(tlo - rt[1] >= emax || rt[1] - thi >= emax);
            uint64_t todo = ballot(reach);
            evaluated2 += (unsigned long long)__builtin_popcountll(todo) *
                          (unsigned long long)min(kWave * SLOTS, hi - t0);
            // per-tile counts of every reference in its lane; with PACK as n_P | n_TP << 10 | n_PS << 20 (a
            // tile has at most 64 x SLOTS candidates), one register and one v_writelane per variant
            static_assert(!PACK || kWave * SLOTS < 1024, "packed per-tile counts take 10 bits each");
            uint32_t tP[V], tTP[V], tPS[V];
#pragma unroll
            for (int v = 0; v < V; ++v)
                tP[v] = tTP[v] = tPS[v] = 0;
            while (todo != 0) {
                const int r = __builtin_ctzll(todo);
                todo &= todo - 1;
                float rr[RW];
                {
                    const f4v *rowv = reinterpret_cast<const f4v *>(myrows + r * RW);
#pragma unroll
                    for (int x = 0; x < RW / 4; ++x) {
                        const f4v q4 = rowv[x];
                        rr[4 * x + 0] = q4.x;
                        rr[4 * x + 1] = q4.y;
                        rr[4 * x + 2] = q4.z;
                        rr[4 * x + 3] = q4.w;
                    }
                }
                uint32_t sP[V], sTP[V], sPS[V];
#pragma unroll
                for (int v = 0; v < V; ++v)
                    sP[v] = sTP[v] = sPS[v] = 0;
#pragma unroll
                for (int sl = 0; sl < SLOTS; ++sl) {
                    float dp = absdiff(rr[1], ct[sl][1]);
#pragma unroll
                    for (int m = 2; m < DT; ++m)
                        dp = fmaxf(dp, absdiff(rr[m], ct[sl][m]));
                    const float dtp = fmaxf(absdiff(rr[0], ct[sl][0]), dp);
#pragma unroll
                    for (int v = 0; v < V; ++v) {
                        float ds = absdiff(rr[DT + v * DX], cs[sl][v][0]);
#pragma unroll
                        for (int m = 1; m < DX; ++m)
                            ds = fmaxf(ds, absdiff(rr[DT + v * DX + m], cs[sl][v][m]));
                        const float er = rr[DT + V * DX + v];
                        sP[v] += (uint32_t)__builtin_popcountll(ballot(dp < er));
                        sTP[v] += (uint32_t)__builtin_popcountll(ballot(dtp < er));
                        sPS[v] += (uint32_t)__builtin_popcountll(ballot(fmaxf(dp, ds) < er));
                    }
                }
#pragma unroll
                for (int v = 0; v < V; ++v) {
                    if constexpr (PACK) {
                        tP[v] = writelane(tP[v], sP[v] | (sTP[v] << 10) | (sPS[v] << 20), r);
                    } else {
                        tP[v] = writelane(tP[v], sP[v], r);
                        tTP[v] = writelane(tTP[v], sTP[v], r);
                        tPS[v] = writelane(tPS[v], sPS[v], r);
                    }
                }
            }
#pragma unroll
            for (int v = 0; v < V; ++v) {
                if constexpr (PACK) {
                    accP[v] += tP[v] & 1023u;
                    accTP[v] += (tP[v] >> 10) & 1023u;
                    accPS[v] += tP[v] >> 20;
                } else {
                    accP[v] += tP[v];
                    accTP[v] += tTP[v];
                    accPS[v] += tPS[v];
                }
            }
        }

        // ---- digamma terms per variant, summed over the item in fixed order
#pragma unroll
        for (int v = 0; v < V; ++v) {
            const uint32_t self = eps[v] > 0.0f ? 1u : 0u;
            double term = 0.0;
            if (valid)
                term = psi_of_count((int)(accP[v] - self)) - psi_of_count((int)(accTP[v] - self)) -
                       psi_of_count((int)(accPS[v] - self));
            const double sum = wave_sum(term);
            if (lane == 0 && v < cnt)
                a.partial[pb[v] + blk] = sum;
        }
        work1 += ev * (unsigned long long)cnt;
        work2 += evaluated2 * (unsigned long long)cnt;
        shared1 += ev;
        shared2 += evaluated2;
    }
    if (a.work != nullptr && lane == 0) {
        atomicAdd(a.work, work1);
        atomicAdd(a.work + 1, work2);
        atomicAdd(a.work + 2, shared1);
        atomicAdd(a.work + 3, shared2);
    }
}

template <int DY, int DX, int V, int SLOTS>
__global__ void __launch_bounds__(kMaxWavesPerWG * 64) search_sets_kernel(SearchArgs a)
{
    sets_search<DY, DX, V, SLOTS, false>(a);
}

// Wide sets: at (3, 3, four chunks) the plain body needs 93 VGPRs (five waves per SIMD); packed counts and a
// six-wave bound bring it to 80 with a few spills to scratch, 2 % faster on the uneven-surrogate batch, while the
// narrower sets lost 2-4 % the same way.
template <int DY, int DX, int V, int SLOTS>
__global__ void __launch_bounds__(kMaxWavesPerWG * 64) __attribute__((amdgpu_waves_per_eu(6, 8)))
search_sets_wide_kernel(SearchArgs a)
{
    sets_search<DY, DX, V, SLOTS, true>(a);
}

constexpr bool wide_set(int d_y, int d_x) { return 1 + d_y + set_variants(d_y, d_x) * d_x >= 16; }

template <int DY, int DX, int SLOTS>
void (*sets_fn())(SearchArgs)
{
    if constexpr (wide_set(DY, DX))
        return search_sets_wide_kernel<DY, DX, set_variants(DY, DX), SLOTS>;
    else
        return search_sets_kernel<DY, DX, set_variants(DY, DX), SLOTS>;
}

// ------------------------------------------------------------ small kernels

// Uniform [0, 1) floats from a counter hash (SplitMix64 finaliser); synthetic
// data for launch-shape tuning only.
__global__ void fill_uniform_kernel(float *p, int64_t n, uint64_t seed)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n)
        return;
    uint64_t z = seed + (uint64_t)(i + 1) * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    z ^= z >> 31;
    p[i] = (float)(z >> 40) * (1.0f / 16777216.0f);
}

__global__ void fill_i32_kernel(int32_t *p, int32_t v, int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n)
        p[i] = v;
}

__global__ void embed_kernel(const float *__restrict__ x, const float *__restrict__ y,
                             const int32_t *__restrict__ perms, const int32_t *__restrict__ sigma,
                             const int32_t *__restrict__ u_dev, const EmbedTask *__restrict__ tasks,
                             float *__restrict__ base, int R, int T, int d_y, int d_x, int tau, int u, int cond,
                             int32_t *err)
{
    const EmbedTask tk = tasks[blockIdx.x];
    const int n = tk.n;
    // source delay of this block: the launch's, the task's own, or one chosen on the device
    if (tk.u > 0)
        u = tk.u;
    if (tk.u_slot > 0 && u_dev != nullptr)
        u = u_dev[tk.u_slot - 1];
    // the host checks every delay against the window starts; keep reads in bounds regardless
    const bool u_ok = u >= 1 && tk.w - u - (d_x - 1) * tau >= 0 && tk.w + tk.W - u <= T;
    const int64_t pr = (int64_t)tk.pair * R;
    bool bad = false;
    for (int q = blockIdx.y * blockDim.x + threadIdx.x; q < n; q += blockDim.x * gridDim.y) {
        // position q of the (sorted) chunk holds window point qo = r W + (t' - w)
        int qo = q;
        if (tk.sig >= 0) {
            qo = sigma[tk.sig + q];
            if (qo < 0 || qo >= n) {   // cannot happen for maps made by sort_kernel; keep reads in bounds
                bad = true;
                qo = q;
            }
        }
        const int r = qo / tk.W;
        const int t = tk.w + (qo - r * tk.W);
        int rs = r;
        if (tk.perm >= 0) {
            rs = perms[tk.perm + r];
            if (rs < 0 || rs >= tk.Rc) {   // caller error; keep reads in bounds
                bad = true;
                rs = r;
            }
        }
        const float *yr = y + (pr + r) * T;
        const float *xr = x + (pr + rs) * T;
        if (tk.tp >= 0) {
            const float v0 = yr[t];
            bad |= !isfinite(v0);
            base[tk.tp + q] = v0;
            for (int m = 0; m < d_y; ++m) {
                const float v = yr[t - 1 - m * tau];
                bad |= !isfinite(v);
                base[tk.tp + (int64_t)(1 + m) * n + q] = v;
            }
        }
        bad |= !u_ok;
        if (cond && tk.tp >= 0) {
            // the current source sample x_t joins the conditioning set: it is the last
            // target-past row of this chunk's own target block (it follows the shuffle)
            const float v = xr[t];
            bad |= !isfinite(v);
            base[tk.tp + (int64_t)(1 + d_y) * n + q] = v;
        }
        for (int m = 0; m < d_x; ++m) {
            const float v = u_ok ? xr[t - u - m * tau] : 0.0f;
            bad |= !isfinite(v);
            base[tk.s + (int64_t)m * n + q] = v;
        }
    }
    if (bad)
        atomicOr(err, 1);
}

// Order-preserving unsigned image of a float (negative values reversed), joined
// with the point index so that every key is distinct.
__device__ __forceinline__ uint64_t sort_key(float f, uint32_t q)
{
    uint32_t u = __builtin_bit_cast(uint32_t, f);
    u = (u & 0x80000000u) ? ~u : (u | 0x80000000u);
    return ((uint64_t)u << 32) | q;
}

// One bitonic compare-exchange pass with stride jj inside stage kk over the
// len elements of A (LDS tile or global array).  offset: global index of A[0],
// so the sort direction is that of the full network.  Workgroup-wide: every
// thread takes pairs across the whole range.
__device__ __forceinline__ void bitonic_pass(uint64_t *A, int len, int kk, int jj, int offset)
{
    for (int t = threadIdx.x; t < len; t += blockDim.x) {
        const int i = t;
        const int l = i ^ jj;
        if (l > i) {
            const uint64_t u0 = A[i], u1 = A[l];
            const bool up = ((offset + i) & kk) == 0;
            if ((u0 > u1) == up) {
                A[i] = u1;
                A[l] = u0;
            }
        }
    }
}

// All passes of stage kk with stride jj < seg, for an LDS array split into
// seg-sized segments of which each wave owns one (or several): partners of
// strides below seg lie in the same segment, so a wave runs these passes back
// to back without workgroup barriers (LDS accesses of one wave complete in order).
__device__ __forceinline__ void bitonic_wave_passes(uint64_t *A, int len, int kk, int jstart, int seg, int offset)
{
    const int lane = threadIdx.x & (kWave - 1);
    const int wave = threadIdx.x / kWave;
    const int nwaves = blockDim.x / kWave;
    for (int s0 = wave * seg; s0 < len; s0 += nwaves * seg) {
        for (int jj = jstart; jj > 0; jj >>= 1) {
            for (int t = lane; t < seg; t += kWave) {
                const int i = s0 + t;
                const int l = i ^ jj;
                if (l > i) {
                    const uint64_t u0 = A[i], u1 = A[l];
                    const bool up = ((offset + i) & kk) == 0;
                    if ((u0 > u1) == up) {
                        A[i] = u1;
                        A[l] = u0;
                    }
                }
            }
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        }
    }
}

// Full bitonic network over len (power of two) keys in LDS; offset as above.
// Strides of at least one wave segment run workgroup-wide with a barrier after
// each pass; the smaller strides of a stage run wave-locally.
__device__ void bitonic_lds(uint64_t *A, int len, int kk_first, int kk_last, int offset)
{
    const int nwaves = blockDim.x / kWave;
    const int seg = max(2, len / nwaves);        // keys per wave segment
    for (int kk = kk_first; kk <= kk_last; kk <<= 1) {
        int jj = kk >> 1;
        for (; jj >= seg; jj >>= 1) {
            bitonic_pass(A, len, kk, jj, offset);
            __syncthreads();
        }
        if (jj > 0) {
            bitonic_wave_passes(A, len, kk, jj, seg, offset);
            __syncthreads();
        }
    }
}

// One workgroup sorts one search space by its first target-past coordinate:
// a bitonic network over npad = 2^m keys (padding keys sort last).  Up to
// kSortLds keys the whole network runs in LDS.  Above that the keys live in
// global scratch; every stage's passes with stride below kSortLds only pair
// elements of the same kSortLds-aligned tile, so each tile is loaded into LDS
// once per stage for those passes and only the wider strides touch global memory.
// Stable LSD radix sort of up to kRadixMax packed keys (order key in the high 32
// bits, point index in the low 32) by their high 32 bits, 4 bits per pass, with
// kRadixThreads threads: thread t owns a contiguous run of keys, counts its
// digits into column t of L (digit-major), an exclusive scan over L gives every
// (digit, thread) its first output slot, and each thread scatters its run in
// order.  Keys enter in index order, so equal keys stay in index order: the
// result is the order of the full 64-bit keys.  Returns the buffer holding it.
constexpr int kRadixMax = 8192;
constexpr int kRadixThreads = 512;

__device__ uint64_t *radix_sort_lds(uint64_t *A, uint64_t *B, uint16_t *L, uint32_t *wsum, int n)
{
    const int t = threadIdx.x;
    const bool act = t < kRadixThreads;
    const int c = (n + kRadixThreads - 1) / kRadixThreads;
    const int i0 = min(n, t * c), i1 = min(n, i0 + c);
    const int lane = t & (kWave - 1), wave = t / kWave;
    for (int shift = 32; shift < 64; shift += 4) {
        if (act) {
#pragma unroll
            for (int d = 0; d < 16; ++d)
                L[d * kRadixThreads + t] = 0;
            for (int i = i0; i < i1; ++i) {
                const int d = (int)((A[i] >> shift) & 15u);
                L[d * kRadixThreads + t] = (uint16_t)(L[d * kRadixThreads + t] + 1);
            }
        }
        __syncthreads();
        // exclusive scan over the 16 x kRadixThreads counts, digit-major: thread s
        // owns the 16 consecutive entries [16 s, 16 s + 16)
        uint32_t own = 0;
        if (act)
#pragma unroll
            for (int e = 0; e < 16; ++e)
                own += L[16 * t + e];
        uint32_t inc = own;                       // inclusive scan over the wave
#pragma unroll
        for (int off = 1; off < kWave; off <<= 1) {
            const uint32_t v = __shfl_up(inc, off);
            if (lane >= off)
                inc += v;
        }
        if (act && lane == kWave - 1)
            wsum[wave] = inc;
        __syncthreads();
        if (act) {
            uint32_t base = inc - own;
            for (int w = 0; w < wave; ++w)
                base += wsum[w];
#pragma unroll
            for (int e = 0; e < 16; ++e) {
                const uint32_t v = L[16 * t + e];
                L[16 * t + e] = (uint16_t)base;
                base += v;
            }
        }
        __syncthreads();
        if (act)
            for (int i = i0; i < i1; ++i) {
                const uint64_t key = A[i];
                const int d = (int)((key >> shift) & 15u);
                const int slot = L[d * kRadixThreads + t];
                L[d * kRadixThreads + t] = (uint16_t)(slot + 1);
                B[slot] = key;
            }
        __syncthreads();
        uint64_t *tmp = A;
        A = B;
        B = tmp;
    }
    return A;
}

__global__ void __launch_bounds__(1024) sort_kernel(const float *__restrict__ y, const float *__restrict__ pts,
                                                    const SortTask *__restrict__ tasks, int32_t *__restrict__ sigma,
                                                    uint64_t *__restrict__ scratch, int R, int T)
{
    __shared__ uint64_t lds[kSortLds];
    __shared__ uint16_t radix_cnt[16 * kRadixThreads];
    __shared__ uint32_t radix_wsum[kRadixThreads / kWave];
    const SortTask tk = tasks[blockIdx.x];
    const int np = tk.npad;
    if (tk.n <= kRadixMax) {
        // small windows: radix sort in LDS (8 passes instead of a log^2 network)
        for (int i = threadIdx.x; i < tk.n; i += blockDim.x) {
            float f;
            if (tk.mode == 0) {
                const int r = i / tk.W;
                const int t = tk.w + (i - r * tk.W);
                f = y[((int64_t)tk.pair * R + r) * T + t - 1];
            } else {
                f = pts[tk.key_off + i];
            }
            lds[i] = sort_key(f, (uint32_t)i);
        }
        __syncthreads();
        const uint64_t *S = radix_sort_lds(lds, lds + kRadixMax, radix_cnt, radix_wsum, tk.n);
        for (int i = threadIdx.x; i < tk.n; i += blockDim.x)
            sigma[tk.sig + i] = (int32_t)(S[i] & 0xffffffffu);
        return;
    }
    uint64_t *A = (np <= kSortLds) ? lds : scratch + tk.scratch;
    for (int i = threadIdx.x; i < np; i += blockDim.x) {
        uint64_t key = ~0ull;
        if (i < tk.n) {
            float f;
            if (tk.mode == 0) {
                const int r = i / tk.W;
                const int t = tk.w + (i - r * tk.W);
                f = y[((int64_t)tk.pair * R + r) * T + t - 1];
            } else {
                f = pts[tk.key_off + i];
            }
            key = sort_key(f, (uint32_t)i);
        }
        A[i] = key;
    }
    __syncthreads();
    if (np <= kSortLds) {
        bitonic_lds(lds, np, 2, np, 0);
    } else {
        // stages that fit a tile: sort every tile in LDS
        for (int t0 = 0; t0 < np; t0 += kSortLds) {
            for (int i = threadIdx.x; i < kSortLds; i += blockDim.x)
                lds[i] = A[t0 + i];
            __syncthreads();
            bitonic_lds(lds, kSortLds, 2, kSortLds, t0);
            for (int i = threadIdx.x; i < kSortLds; i += blockDim.x)
                A[t0 + i] = lds[i];
            __syncthreads();
        }
        for (int kk = 2 * kSortLds; kk <= np; kk <<= 1) {
            for (int jj = kk >> 1; jj >= kSortLds; jj >>= 1) {
                bitonic_pass(A, np, kk, jj, 0);
                __syncthreads();
            }
            for (int t0 = 0; t0 < np; t0 += kSortLds) {
                for (int i = threadIdx.x; i < kSortLds; i += blockDim.x)
                    lds[i] = A[t0 + i];
                __syncthreads();
                // the remaining strides of stage kk, inside this tile
                const int nwaves = blockDim.x / kWave;
                const int seg = kSortLds / nwaves;
                for (int jj = kSortLds >> 1; jj >= seg; jj >>= 1) {
                    bitonic_pass(lds, kSortLds, kk, jj, t0);
                    __syncthreads();
                }
                bitonic_wave_passes(lds, kSortLds, kk, seg >> 1, seg, t0);
                __syncthreads();
                for (int i = threadIdx.x; i < kSortLds; i += blockDim.x)
                    A[t0 + i] = lds[i];
                __syncthreads();
            }
        }
    }
    for (int i = threadIdx.x; i < tk.n; i += blockDim.x)
        sigma[tk.sig + i] = (int32_t)(A[i] & 0xffffffffu);
}

__global__ void gather_kernel(const float *__restrict__ src, const GatherTask *__restrict__ tasks,
                              const int32_t *__restrict__ sigma, float *__restrict__ dst, int D)
{
    const GatherTask tk = tasks[blockIdx.x];
    for (int q = threadIdx.x; q < tk.n; q += blockDim.x) {
        int o = sigma[tk.sig + q];
        if (o < 0 || o >= tk.n)          // maps from sort_kernel are permutations; keep reads in bounds regardless
            o = q;
        for (int m = 0; m < D; ++m)
            dst[tk.dst + (int64_t)m * tk.n + q] = src[tk.src + (int64_t)m * tk.ld + o];
    }
}

// ------------------------------------------------------ surrogate permutations

constexpr int kMaxPermTrials = 1 << 16;

// Copy mode: row i of the caller's permutations into the batch's permutation
// area.  Entries < rc must be a permutation of 0..rc-1 (one workgroup per row,
// an LDS bitmap records the values seen); entries rc..len-1 are the identity.
__global__ void take_perms_kernel(const int32_t *__restrict__ src, const PermTask *__restrict__ tasks,
                                  int32_t *__restrict__ dst, int32_t *err)
{
    __shared__ uint32_t seen[kMaxPermTrials / 32];
    const PermTask tk = tasks[blockIdx.x];
    const int rc = tk.rc;
    const bool too_big = rc > kMaxPermTrials || rc < 1;
    const int words = too_big ? 0 : (rc + 31) / 32;
    for (int w = threadIdx.x; w < words; w += blockDim.x)
        seen[w] = 0;
    __syncthreads();
    bool bad = too_big;
    if (!bad) {
        for (int r = threadIdx.x; r < rc; r += blockDim.x) {
            const int v = src[tk.src + r];
            if (v < 0 || v >= rc) {
                bad = true;
                dst[tk.dst + r] = r;          // keep later reads in bounds; the call reports the error
            } else {
                const uint32_t bit = 1u << (v & 31);
                if (atomicOr(&seen[v >> 5], bit) & bit)
                    bad = true;
                dst[tk.dst + r] = v;
            }
        }
    }
    for (int r = max(rc, 0) + threadIdx.x; r < tk.len; r += blockDim.x)
        dst[tk.dst + r] = r;
    if (bad)
        atomicOr(err, 2);
}

// Seeded mode.  The permutation of (pair p, point c, surrogate s) is drawn from
// the counter-based SplitMix64 generator (Steele, Lea and Flood 2014): output q
// of the stream with key K is mix(K + (q + 1) G), and K folds the identifiers
// into the seed, K = f(f(f(f(f(0x5EED5EED5EED5EED, seed), 77), p), c), s) with
// f(k, v) = mix(k + G v + 1).  Fisher-Yates from the top: for i = rc-1 down to 1,
// swap positions i and j_i, j_i uniform on 0..i.  Draw number t = rc-1-i takes its
// bound i + 1 and Lemire's multiply-and-reject rule on the high 32 bits w of an
// output: m = w (i + 1), j_i = m >> 32, rejected when (m mod 2^32) < 2^32 mod (i+1).
// Draws are made in rounds: in round one draw t takes output t; each later round
// gives the draws rejected so far, in draw order, the next unused outputs.
// One wave per row: the rounds run across lanes, the swaps on one lane in LDS
// (rows of up to kDrawLds trials) or in the destination row itself (longer rows).
constexpr uint64_t kGolden = 0x9E3779B97F4A7C15ull;
constexpr int kDrawLds = 8192;
constexpr int kMaxRejects = 256;

__device__ __forceinline__ uint64_t mix64(uint64_t z)
{
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

__device__ __forceinline__ uint64_t fold_key(uint64_t k, uint64_t v) { return mix64(k + kGolden * v + 1ull); }

// Lemire's rule for bound s on output q of stream key: the draw, or -1 if rejected.
__device__ __forceinline__ int lemire_draw(uint64_t key, uint64_t q, uint32_t s)
{
    const uint32_t w = (uint32_t)(mix64(key + (q + 1ull) * kGolden) >> 32);
    const uint64_t m = (uint64_t)w * s;
    const uint32_t lo = (uint32_t)m;
    if (lo < s && lo < (0u - s) % s)
        return -1;
    return (int)(m >> 32);
}

__global__ void __launch_bounds__(64) draw_perms_kernel(const PermTask *__restrict__ tasks, int32_t *__restrict__ dst,
                                                        uint64_t seed, int32_t *err)
{
    __shared__ int32_t lds_perm[kDrawLds];
    __shared__ int32_t pend[2][kMaxRejects];
    __shared__ int32_t fix_t[kMaxRejects], fix_j[kMaxRejects];
    const PermTask tk = tasks[blockIdx.x];
    const int lane = threadIdx.x;
    const int n = tk.rc;
    int32_t *row = dst + tk.dst;
    if (n < 1 || n > kMaxPermTrials) {
        for (int r = lane; r < tk.len; r += kWave)
            row[r] = r;
        if (lane == 0)
            atomicOr(err, 2);
        return;
    }
    uint64_t key = 0x5EED5EED5EED5EEDull;
    key = fold_key(key, seed);
    key = fold_key(key, 77ull);
    key = fold_key(key, (uint64_t)(int64_t)tk.pair);
    key = fold_key(key, (uint64_t)(int64_t)tk.point);
    key = fold_key(key, (uint64_t)(int64_t)tk.surr);
    const int draws = n - 1;
    const uint64_t lanes_below = (lane == 0) ? 0ull : (~0ull >> (64 - lane));

    // round one: find the rejected draws (rare), in draw order
    int npend = 0;
    for (int t0 = 0; t0 < draws; t0 += kWave) {
        const int t = t0 + lane;
        const bool rej = t < draws && lemire_draw(key, (uint64_t)t, (uint32_t)(n - t)) < 0;
        const uint64_t mask = ballot(rej);
        if (rej) {
            const int idx = npend + __builtin_popcountll(mask & lanes_below);
            if (idx < kMaxRejects)
                pend[0][idx] = t;
        }
        npend += __builtin_popcountll(mask);
    }
    bool overflow = npend > kMaxRejects;
    // later rounds: pending draws take the next unused outputs, in draw order
    uint64_t pos = (uint64_t)max(draws, 0);
    int nfix = 0, cur = 0;
    while (npend > 0 && !overflow) {
        __builtin_amdgcn_wave_barrier();
        int nnext = 0;
        for (int b0 = 0; b0 < npend; b0 += kWave) {
            const int l = b0 + lane;
            int t = 0, j = -1;
            if (l < npend) {
                t = pend[cur][l];
                j = lemire_draw(key, pos + (uint64_t)l, (uint32_t)(n - t));
            }
            const bool acc = l < npend && j >= 0;
            const bool rej = l < npend && j < 0;
            const uint64_t ma = ballot(acc), mr = ballot(rej);
            if (acc) {
                const int idx = nfix + __builtin_popcountll(ma & lanes_below);
                if (idx < kMaxRejects) {
                    fix_t[idx] = t;
                    fix_j[idx] = j;
                }
            }
            if (rej) {
                const int idx = nnext + __builtin_popcountll(mr & lanes_below);
                if (idx < kMaxRejects)
                    pend[cur ^ 1][idx] = t;
            }
            nfix += __builtin_popcountll(ma);
            nnext += __builtin_popcountll(mr);
        }
        pos += (uint64_t)npend;
        npend = nnext;
        cur ^= 1;
        overflow = nfix > kMaxRejects || npend > kMaxRejects;
    }
    if (overflow) {
        for (int r = lane; r < tk.len; r += kWave)
            row[r] = r;
        if (lane == 0)
            atomicOr(err, 2);
        return;
    }
    __builtin_amdgcn_wave_barrier();
    // the swaps, in order, on one lane
    int32_t *a = n <= kDrawLds ? lds_perm : row;
    for (int r = lane; r < n; r += kWave)
        a[r] = r;
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    if (lane == 0) {
        for (int t = 0; t < draws; ++t) {
            const int i = n - 1 - t;
            int j = lemire_draw(key, (uint64_t)t, (uint32_t)(i + 1));
            if (j < 0)
                for (int f = 0; f < nfix; ++f)
                    if (fix_t[f] == t)
                        j = fix_j[f];
            if (j < 0 || j > i)              // cannot happen: every rejected draw has a fix
                j = i;
            const int32_t vi = a[i], vj = a[j];
            a[i] = vj;
            a[j] = vi;
        }
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    if (n <= kDrawLds)
        for (int r = lane; r < n; r += kWave)
            row[r] = lds_perm[r];
    for (int r = n + lane; r < tk.len; r += kWave)
        row[r] = r;
}

// p-value of window group g (eq. 10 test): the fraction of its n_surr surrogate
// estimates at or above the original (results [g][0] original, [g][1..] surrogates)
__device__ __forceinline__ double group_pvalue(const double *results, int g, int n_surr)
{
    const double *r = results + (int64_t)g * (n_surr + 1);
    int c = 0;
    for (int s = 1; s <= n_surr; ++s)
        c += r[s] >= r[0];
    return n_surr > 0 ? (double)c / (double)n_surr : __builtin_nan("");
}

__global__ void reduce_kernel(const ChunkDesc *__restrict__ chunks, int n_chunks,
                              const double *__restrict__ partial, int k, const int32_t *err,
                              double *results, int n_groups, int n_surr, double *__restrict__ pv,
                              int32_t *done, int32_t *err_out)
{
    // one wave per chunk: lane l sums items l, l + 64, ... in order, then a fixed
    // butterfly across the wave (the same order on every run and batch split)
    const int c = blockIdx.x * (blockDim.x / kWave) + threadIdx.x / kWave;
    const int lane = threadIdx.x & (kWave - 1);
    if (c < n_chunks) {
        const ChunkDesc cd = chunks[c];
        const int nb = (cd.n + kWave - 1) / kWave;
        double s = 0.0;
        for (int b = lane; b < nb; b += kWave)
            s += partial[cd.pbase + b];
        s = wave_sum(s);
        if (lane == 0) {
            double te = psi_of_count(k - 1) + s / (double)cd.n;
            if (*err != 0)
                te = __builtin_nan("");
            results[cd.result] = te;
        }
    }
    if (pv == nullptr)
        return;
    // the workgroup that finishes last (done counts finished workgroups, zero at
    // launch) computes every group's p-value and copies the error word behind them
    __shared__ int last;
    __threadfence();
    __syncthreads();
    if (threadIdx.x == 0)
        last = atomicAdd(done, 1) == (int)gridDim.x - 1;
    __syncthreads();
    if (!last)
        return;
    __threadfence();
    const bool bad = *err != 0;
    for (int g = threadIdx.x; g < n_groups; g += blockDim.x)
        pv[g] = bad ? __builtin_nan("") : group_pvalue(results, g, n_surr);
    if (threadIdx.x == 0 && err_out != nullptr)
        *err_out = *err;
}

__global__ void pvalue_kernel(const double *__restrict__ results, int n_groups, int n_surr,
                              double *__restrict__ pv, const int32_t *err, int32_t *err_out)
{
    const int g = blockIdx.x * blockDim.x + threadIdx.x;
    if (g == 0 && err_out != nullptr)
        *err_out = *err;
    if (g >= n_groups)
        return;
    pv[g] = (err != nullptr && *err != 0) ? __builtin_nan("") : group_pvalue(results, g, n_surr);
}

// Delay reconstruction (eq. 5): per window group, the delay whose original
// estimate is largest (the first one in table order among equal maxima).
__global__ void argmax_u_kernel(const double *__restrict__ results, int n_groups, int n_u,
                                const int32_t *__restrict__ u_values, int32_t *__restrict__ u_sel)
{
    const int g = blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= n_groups)
        return;
    const double *r = results + (int64_t)g * n_u;
    int best = 0;
    for (int j = 1; j < n_u; ++j)
        if (r[j] > r[best])
            best = j;
    u_sel[g] = u_values[best];
}

// ------------------------------------------------------------- dispatch

typedef void (*search_fn)(SearchArgs);

template <int DY, int DX, int SLOTS>
struct Table {
    static search_fn get(bool generic, bool sorted)
    {
        if (sorted)
            return generic ? search_kernel<DY, DX, kMaxK + 1, true, SLOTS, true>
                           : search_kernel<DY, DX, 5, false, SLOTS, true>;
        return generic ? search_kernel<DY, DX, kMaxK + 1, true, SLOTS, false>
                       : search_kernel<DY, DX, 5, false, SLOTS, false>;
    }
};

template <int SLOTS>
search_fn pick(int d_y, int d_x, bool generic, bool sorted)
{
#define TE_CASE(A, B) \
    if (d_y == A && d_x == B) return Table<A, B, SLOTS>::get(generic, sorted);
    TE_CASE(1, 1) TE_CASE(1, 2) TE_CASE(1, 3) TE_CASE(1, 4)
    TE_CASE(2, 1) TE_CASE(2, 2) TE_CASE(2, 3) TE_CASE(2, 4)
    TE_CASE(3, 1) TE_CASE(3, 2) TE_CASE(3, 3) TE_CASE(3, 4)
    TE_CASE(4, 1) TE_CASE(4, 2) TE_CASE(4, 3) TE_CASE(4, 4)
#undef TE_CASE
    return nullptr;
}

search_fn pick_any(int d_y, int d_x, int k, int slots, bool sorted)
{
    const bool generic = (k != 4);
    if (k < 1 || k > kMaxK)
        return nullptr;
    if (slots == 4)
        return pick<4>(d_y, d_x, generic, sorted);
    if (slots == 8)
        return pick<8>(d_y, d_x, generic, sorted);
    if (slots == 16)
        return pick<16>(d_y, d_x, generic, sorted);
    return nullptr;
}

// Chunk-set search: V = set_variants(d_y, d_x) chunks per item, k = 4, sorted chunks; two or
// four candidate slots per lane in the counting pass (the tuned slot count 4 -> 2,
// 8 or 16 -> 4).
template <int SLOTS>
search_fn pick_sets_slots(int d_y, int d_x)
{
#define TE_CASE(A, B) \
    if (d_y == A && d_x == B) return sets_fn<A, B, SLOTS>();
    TE_CASE(1, 1) TE_CASE(1, 2) TE_CASE(1, 3) TE_CASE(1, 4)
    TE_CASE(2, 1) TE_CASE(2, 2) TE_CASE(2, 3) TE_CASE(2, 4)
    TE_CASE(3, 1) TE_CASE(3, 2) TE_CASE(3, 3) TE_CASE(3, 4)
    TE_CASE(4, 1) TE_CASE(4, 2) TE_CASE(4, 3) TE_CASE(4, 4)
#undef TE_CASE
    return nullptr;
}

search_fn pick_sets(int d_y, int d_x, int slots)
{
    return slots <= 4 ? pick_sets_slots<2>(d_y, d_x) : pick_sets_slots<4>(d_y, d_x);
}

// LDS bytes of the chunk-set search per workgroup (its rows are dynamic shared memory).
size_t sets_lds_bytes(int d_y, int d_x, int waves_per_wg)
{
    const int v = set_variants(d_y, d_x);
    const int nr = 1 + d_y + v * d_x + v;
    return (size_t)waves_per_wg * kWave * (size_t)((nr + 3) & ~3) * sizeof(float);
}

}  // namespace

// Device counters of evaluated pairs for the measurement hook (one copy per device):
// [0] pass-1 and [1] pass-2 (reference, candidate, chunk) triples, [2] and [3] the
// (reference, candidate) pairs whose shared coordinates were evaluated once for them.
__device__ unsigned long long g_work_counters[4];

unsigned long long *work_counters()
{
    void *p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(g_work_counters)) != hipSuccess)
        return nullptr;
    return static_cast<unsigned long long *>(p);
}

bool search_supported(int d_y, int d_x, int k, int slots) { return pick_any(d_y, d_x, k, slots, false) != nullptr; }

// Resident workgroups per compute unit for the chosen search variant (0 if unknown).
int search_occupancy(int d_y, int d_x, int k, int slots, int waves_per_wg)
{
    search_fn f = pick_any(d_y, d_x, k, slots, true);
    if (!f)
        return 0;
    int blocks = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, f, kWave * waves_per_wg, 0) != hipSuccess)
        return 0;
    return blocks;
}

bool search_sets_supported(int d_y, int d_x, int k) { return k == 4 && pick_sets(d_y, d_x, 4) != nullptr; }

int search_sets_occupancy(int d_y, int d_x, int slots, int waves_per_wg)
{
    search_fn f = pick_sets(d_y, d_x, slots);
    if (!f)
        return 0;
    int blocks = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, f, kWave * waves_per_wg,
                                                     sets_lds_bytes(d_y, d_x, waves_per_wg)) != hipSuccess)
        return 0;
    return blocks;
}

hipError_t launch_search(const SearchArgs &a, int d_y, int d_x, const SearchConfig &cfg, int grid_waves,
                         hipStream_t st)
{
    const int wpg = cfg.waves_per_wg;
    const int blocks = (grid_waves + wpg - 1) / wpg;
    if (a.set_first != nullptr) {
        search_fn f = (a.k == 4 && a.sorted) ? pick_sets(d_y, d_x, cfg.slots) : nullptr;
        if (!f)
            return hipErrorInvalidValue;
        hipLaunchKernelGGL(f, dim3(blocks), dim3(kWave * wpg), sets_lds_bytes(d_y, d_x, wpg), st, a);
        return hipGetLastError();
    }
    search_fn f = pick_any(d_y, d_x, a.k, cfg.slots, a.sorted != 0);
    if (!f)
        return hipErrorInvalidValue;
    hipLaunchKernelGGL(f, dim3(blocks), dim3(kWave * wpg), 0, st, a);
    return hipGetLastError();
}

hipError_t launch_fill_uniform(float *p, int64_t n, uint64_t seed, hipStream_t st)
{
    if (n <= 0)
        return hipSuccess;
    hipLaunchKernelGGL(fill_uniform_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, p, n, seed);
    return hipGetLastError();
}

hipError_t launch_fill_i32(int32_t *p, int32_t v, int64_t n, hipStream_t st)
{
    if (n <= 0)
        return hipSuccess;
    hipLaunchKernelGGL(fill_i32_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, p, v, n);
    return hipGetLastError();
}

hipError_t launch_embed(const float *x, const float *y, const int32_t *perms, const int32_t *sigma,
                        const int32_t *u_dev, const EmbedTask *tasks, int n_tasks, int max_n, float *base, int R,
                        int T, int d_y, int d_x, int tau, int u, int cond, int32_t *err, hipStream_t st)
{
    if (n_tasks <= 0)
        return hipSuccess;
    // a few hundred to a few thousand points per workgroup, so small batches still fill the GPU
    const int parts = std::max(1, std::min(1024, (max_n + 1023) / 1024));
    hipLaunchKernelGGL(embed_kernel, dim3(n_tasks, parts), dim3(256), 0, st, x, y, perms, sigma, u_dev, tasks, base,
                       R, T, d_y, d_x, tau, u, cond, err);
    return hipGetLastError();
}

hipError_t launch_argmax_u(const double *results, int n_groups, int n_u, const int32_t *u_values, int32_t *u_sel,
                           hipStream_t st)
{
    if (n_groups <= 0 || n_u <= 0)
        return hipSuccess;
    hipLaunchKernelGGL(argmax_u_kernel, dim3((n_groups + 127) / 128), dim3(128), 0, st, results, n_groups, n_u,
                       u_values, u_sel);
    return hipGetLastError();
}

hipError_t launch_sort(const float *y, const float *pts, const SortTask *tasks, int n_tasks, int32_t *sigma,
                       uint64_t *scratch, int R, int T, hipStream_t st)
{
    if (n_tasks <= 0)
        return hipSuccess;
    hipLaunchKernelGGL(sort_kernel, dim3(n_tasks), dim3(1024), 0, st, y, pts, tasks, sigma, scratch, R, T);
    return hipGetLastError();
}

hipError_t launch_gather(const float *src, const GatherTask *tasks, int n_tasks, const int32_t *sigma, float *dst,
                         int D, hipStream_t st)
{
    if (n_tasks <= 0)
        return hipSuccess;
    hipLaunchKernelGGL(gather_kernel, dim3(n_tasks), dim3(256), 0, st, src, tasks, sigma, dst, D);
    return hipGetLastError();
}

hipError_t launch_perms(const int32_t *src, const PermTask *tasks, int n_tasks, int32_t *dst,
                        uint64_t seed, int32_t *err, hipStream_t st)
{
    if (n_tasks <= 0)
        return hipSuccess;
    if (src != nullptr)
        hipLaunchKernelGGL(take_perms_kernel, dim3(n_tasks), dim3(256), 0, st, src, tasks, dst, err);
    else
        hipLaunchKernelGGL(draw_perms_kernel, dim3(n_tasks), dim3(kWave), 0, st, tasks, dst, seed, err);
    return hipGetLastError();
}

hipError_t launch_reduce(const ChunkDesc *chunks, int n_chunks, const double *partial, int k,
                         const int32_t *err, double *results, hipStream_t st, int n_groups, int n_surr,
                         double *pv, int32_t *done, int32_t *err_out)
{
    if (n_chunks <= 0)
        return hipSuccess;
    if (pv != nullptr && done == nullptr)
        return hipErrorInvalidValue;
    // the p-values ride on the reduce's last workgroup while the grid is small; above
    // that, every workgroup's device-scope fence and counter atomic cost more than a
    // separate launch (about 1 ms for 16 000 workgroups)
    const int blocks = (n_chunks + 3) / 4;
    const bool fuse = pv != nullptr && blocks <= 256;
    hipLaunchKernelGGL(reduce_kernel, dim3(blocks), dim3(4 * kWave), 0, st, chunks, n_chunks, partial, k, err,
                       results, n_groups, n_surr, fuse ? pv : nullptr, done, err_out);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || pv == nullptr || fuse)
        return e;
    hipLaunchKernelGGL(pvalue_kernel, dim3((std::max(n_groups, 1) + 127) / 128), dim3(128), 0, st, results, n_groups,
                       n_surr, pv, err, err_out);
    return hipGetLastError();
}

hipError_t launch_pvalues(const double *results, int n_groups, int n_surr, double *pv, hipStream_t st)
{
    if (n_groups <= 0)
        return hipSuccess;
    hipLaunchKernelGGL(pvalue_kernel, dim3((n_groups + 127) / 128), dim3(128), 0, st, results, n_groups,
                       n_surr, pv, nullptr, nullptr);
    return hipGetLastError();
}

}  // namespace te
