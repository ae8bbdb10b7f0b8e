// te_scan.cpp -- delay reconstruction (eq. 5): the originals of every window
// at every assumed source delay u in one persistent search, the maximizing
// delay picked on the device, then the trial-shuffle surrogate test (eq. 10)
// at that delay, all on one stream with no host round trip in between.
//
// The delays of one window group share the target block (y_t', Y_past) and its
// sort map; only the source block X_past moves with u.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <numeric>
#include <vector>

#include "te.h"
#include "te_internal.h"
#include "te_runtime.h"

namespace te {

namespace {

struct ScanLayout {
    Batch delays;       // the originals at every delay
    Batch test;         // the original and surrogates at the chosen delay (n_surrogates > 0)
    size_t off_u = 0;   // int32 [n_u] delay table
    size_t off_sel = 0; // int32 [groups] chosen delay per group
    size_t total = 0;
};

}  // namespace

static void scan_layout(const Plan &P, const std::vector<int> &groups, const std::vector<int32_t> &delays,
                        ScanLayout *L)
{
    BatchOptions o1;
    o1.delays = &delays;
    P.build_group_batch(groups, 0, &L->delays, o1);
    size_t main = L->delays.total_bytes;
    if (P.p.n_surrogates > 0) {
        BatchOptions o2;
        o2.delay_from_device = true;
        P.build_group_batch(groups, P.p.n_surrogates, &L->test, o2);
        main = std::max(main, L->test.total_bytes);
    }
    L->off_u = align_up(main, 256);
    L->off_sel = align_up(L->off_u + sizeof(int32_t) * delays.size(), 256);
    L->total = align_up(L->off_sel + sizeof(int32_t) * groups.size(), 256);
}

size_t Plan::scan_bytes(const std::vector<int> &groups, const std::vector<int32_t> &delays) const
{
    ScanLayout L;
    scan_layout(*this, groups, delays, &L);
    return L.total;
}

te_status Plan::run_scan(const float *x, const float *y, const int32_t *perms, const std::vector<int32_t> &delays,
                         char *ws, size_t ws_bytes, hipStream_t st, double *te_scan, int32_t *u_best,
                         double *te_surr, double *p_value) const
{
    TraceRange trace_range("te.delay_scan");
    const int G = p.n_pairs * p.n_points;
    const int n_u = (int)delays.size();
    const int S = p.n_surrogates;
    bool bad = false;

    auto run = [&](const std::vector<int> &groups) -> te_status {
        ScanLayout L;
        scan_layout(*this, groups, delays, &L);
        const int Gs = (int)groups.size();
        void *stg1 = pool.take(L.delays.stage_bytes());
        void *stg2 = S > 0 ? pool.take(L.test.stage_bytes()) : nullptr;
        void *stgu = pool.take(sizeof(int32_t) * (n_u + Gs) + 64);
        auto release = [&] {
            if (stg1)
                pool.give(stg1);
            if (stg2)
                pool.give(stg2);
            if (stgu)
                pool.give(stgu);
        };
        if (!stg1 || (S > 0 && !stg2) || !stgu) {
            release();
            return fail(TE_ERR_NOMEM, "pinned staging allocation failed");
        }
        int32_t *hu = static_cast<int32_t *>(stgu);
        std::memcpy(hu, delays.data(), sizeof(int32_t) * n_u);
        int32_t *du = reinterpret_cast<int32_t *>(ws + L.off_u);
        int32_t *dsel = reinterpret_cast<int32_t *>(ws + L.off_sel);
        te_status s = TE_OK;
        hipError_t e = hipMemcpyAsync(du, hu, sizeof(int32_t) * n_u, hipMemcpyHostToDevice, st);
        if (e != hipSuccess)
            s = hip_fail(e, "upload delays");
        if (s == TE_OK)
            s = enqueue_batch(L.delays, x, y, nullptr, ws, stg1, st);
        if (s == TE_OK) {
            e = launch_argmax_u(reinterpret_cast<const double *>(ws + L.delays.off_results), Gs, n_u, du, dsel, st);
            if (e != hipSuccess)
                s = hip_fail(e, "argmax launch");
        }
        if (s == TE_OK && S > 0)
            s = enqueue_batch(L.test, x, y, perms, ws, stg2, st, nullptr, dsel);
        if (s == TE_OK) {
            e = hipMemcpyAsync(hu + n_u, dsel, sizeof(int32_t) * Gs, hipMemcpyDeviceToHost, st);
            if (e != hipSuccess)
                s = hip_fail(e, "download delays");
        }
        if (s == TE_OK && (e = hipStreamSynchronize(st)) != hipSuccess)
            s = hip_fail(e, "hipStreamSynchronize");
        if (s == TE_OK) {
            // originals at every delay: results [gi][j], then p-values, then the error word
            const char *out = static_cast<const char *>(stg1) + align_up(L.delays.tables_bytes, 256);
            const double *res = reinterpret_cast<const double *>(out);
            int32_t err = 0;
            std::memcpy(&err, out + sizeof(double) * (L.delays.n_results + L.delays.n_groups), sizeof err);
            bad |= err != 0;
            for (int gi = 0; gi < Gs; ++gi) {
                const int g = groups[gi];
                for (int j = 0; j < n_u; ++j)
                    te_scan[(size_t)g * n_u + j] = res[(size_t)gi * n_u + j];
                if (u_best)
                    u_best[g] = hu[n_u + gi];
            }
            if (S > 0)
                unpack_batch(L.test, stg2, nullptr, te_surr, p_value, &bad);
        }
        release();
        return s;
    };

    std::vector<int> cur;
    for (int g = 0; g < G; ++g) {
        std::vector<int> trial = cur;
        trial.push_back(g);
        if (scan_bytes(trial, delays) <= ws_bytes) {
            cur.swap(trial);
            continue;
        }
        if (cur.empty())
            return fail(TE_ERR_NOMEM, "workspace of %zu bytes cannot hold the delay scan of window group %d",
                        ws_bytes, g);
        te_status s = run(cur);
        if (s != TE_OK)
            return s;
        cur.assign(1, g);
    }
    if (!cur.empty()) {
        te_status s = run(cur);
        if (s != TE_OK)
            return s;
    }
    if (S == 0 && p_value)
        for (int g = 0; g < G; ++g)
            p_value[g] = __builtin_nan("");
    if (bad)
        return fail(TE_ERR_INVALID, "non-finite input value or invalid permutation");
    return TE_OK;
}

static te_status check_delays(const Plan &P, const int32_t *u_values, int n_u, std::vector<int32_t> *out)
{
    if (!u_values || n_u < 1 || n_u > 4096)
        return fail(TE_ERR_INVALID, "need 1 <= n_u <= 4096 delays");
    const int w_min = *std::min_element(P.wstart.begin(), P.wstart.end());
    out->assign(u_values, u_values + n_u);
    for (int32_t u : *out) {
        if (u < 1)
            return fail(TE_ERR_INVALID, "delay u = %d must be >= 1", u);
        const int need = u + (P.p.d_x - 1) * P.p.tau;
        if (w_min < need)
            return fail(TE_ERR_INVALID, "delay u = %d needs every window to start at sample >= %d (earliest is %d)",
                        u, need, w_min);
    }
    return TE_OK;
}

}  // namespace te

using namespace te;

extern "C" {

te_status te_delay_scan_workspace_bytes(te_plan plan, const int32_t *u_values, int32_t n_u, size_t *full,
                                        size_t *minimum)
{
    clear_error();
    if (!plan)
        return fail(TE_ERR_INVALID, "null argument");
    const Plan &P = plan->impl;
    std::vector<int32_t> d;
    te_status s = check_delays(P, u_values, n_u, &d);
    if (s != TE_OK)
        return s;
    const int G = P.p.n_pairs * P.p.n_points;
    std::vector<int> all(G);
    std::iota(all.begin(), all.end(), 0);
    if (full)
        *full = P.scan_bytes(all, d);
    if (minimum) {
        // the largest window group alone
        size_t m = 0;
        for (int c = 0; c < P.p.n_points; ++c)
            m = std::max(m, P.scan_bytes(std::vector<int>(1, c), d));
        *minimum = m;
    }
    return TE_OK;
}

te_status te_delay_scan(te_plan plan, const float *x, const float *y, const int32_t *perms, const int32_t *u_values,
                        int32_t n_u, void *ws, size_t ws_bytes, void *hip_stream, double *te_scan, int32_t *u_best,
                        double *te_surr, double *p_value)
{
    clear_error();
    if (!plan || !x || !y || !ws || !te_scan)
        return fail(TE_ERR_INVALID, "null argument");
    const Plan &P = plan->impl;
    if (P.p.n_surrogates > 0 && !te_surr)
        return fail(TE_ERR_INVALID, "n_surrogates > 0 needs te_surr");
    std::vector<int32_t> d;
    te_status s = check_delays(P, u_values, n_u, &d);
    if (s != TE_OK)
        return s;
    s = P.ensure_device();
    if (s != TE_OK)
        return s;
    return P.run_scan(x, y, perms, d, static_cast<char *>(ws), ws_bytes, (hipStream_t)hip_stream, te_scan, u_best,
                      te_surr, p_value);
}

}  // extern "C"
