// te_profile.cpp -- optional HIP-event timing of search-kernel launches.

#include <hip/hip_runtime.h>

#include <mutex>
#include <vector>

#include "te.h"
#include "te_internal.h"
#include "te_runtime.h"

namespace te {

namespace {
std::mutex g_mu;
bool g_on = false;        // HIP events around search launches
bool g_work_on = false;   // device counters of evaluated pairs
struct Pending {
    hipEvent_t a, b;
};
std::vector<Pending> g_pending;
std::vector<hipEvent_t> g_free;
double g_ms = 0.0;
int64_t g_launches = 0;
unsigned long long *g_work = nullptr;   // this device's counters of evaluated pairs (pass 1, pass 2)

hipEvent_t get_event()
{
    if (!g_free.empty()) {
        hipEvent_t e = g_free.back();
        g_free.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess)
        return nullptr;
    return e;
}
}  // namespace

hipError_t launch_search_timed(const SearchArgs &a, int d_y, int d_x, const SearchConfig &cfg, int grid_waves,
                               hipStream_t st)
{
    bool on, work_on;
    {
        std::lock_guard<std::mutex> lk(g_mu);
        on = g_on;
        work_on = g_work_on;
    }
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if ((on || work_on) && hipStreamIsCapturing(st, &cs) == hipSuccess && cs != hipStreamCaptureStatusNone)
        on = work_on = false;
    SearchArgs b = a;
    if (work_on) {
        std::lock_guard<std::mutex> lk(g_mu);
        if (!g_work)
            g_work = work_counters();
        b.work = g_work;
    }
    if (!on)
        return launch_search(b, d_y, d_x, cfg, grid_waves, st);
    hipEvent_t e0, e1;
    {
        std::lock_guard<std::mutex> lk(g_mu);
        e0 = get_event();
        e1 = get_event();
    }
    if (!e0 || !e1)
        return launch_search(b, d_y, d_x, cfg, grid_waves, st);
    hipEventRecord(e0, st);
    hipError_t e = launch_search(b, d_y, d_x, cfg, grid_waves, st);
    hipEventRecord(e1, st);
    std::lock_guard<std::mutex> lk(g_mu);
    g_pending.push_back({e0, e1});
    return e;
}

}  // namespace te

using namespace te;

extern "C" {

te_status te_profile_enable(int32_t on)
{
    std::lock_guard<std::mutex> lk(g_mu);
    g_on = (on & TE_PROFILE_TIME) != 0;
    g_work_on = (on & TE_PROFILE_WORK) != 0;
    return TE_OK;
}

te_status te_profile_work_all(int64_t *counts, int32_t reset)
{
    std::lock_guard<std::mutex> lk(g_mu);
    unsigned long long w[4] = {0, 0, 0, 0};
    if (g_work) {
        if (hipDeviceSynchronize() != hipSuccess ||
            hipMemcpy(w, g_work, sizeof w, hipMemcpyDeviceToHost) != hipSuccess)
            return TE_ERR_DEVICE;
        if (reset && hipMemset(g_work, 0, sizeof w) != hipSuccess)
            return TE_ERR_DEVICE;
    }
    if (counts)
        for (int i = 0; i < 4; ++i)
            counts[i] = (int64_t)w[i];
    return TE_OK;
}

te_status te_profile_work(int64_t *pass1_pairs, int64_t *pass2_pairs, int32_t reset)
{
    int64_t w[4];
    const te_status s = te_profile_work_all(w, reset);
    if (s != TE_OK)
        return s;
    if (pass1_pairs)
        *pass1_pairs = w[0];
    if (pass2_pairs)
        *pass2_pairs = w[1];
    return TE_OK;
}

te_status te_profile_read(double *search_ms, int64_t *launches, int32_t reset)
{
    std::lock_guard<std::mutex> lk(g_mu);
    for (auto &p : g_pending) {
        float ms = 0.f;
        if (hipEventSynchronize(p.b) == hipSuccess && hipEventElapsedTime(&ms, p.a, p.b) == hipSuccess) {
            g_ms += ms;
            g_launches += 1;
        }
        g_free.push_back(p.a);
        g_free.push_back(p.b);
    }
    g_pending.clear();
    if (search_ms)
        *search_ms = g_ms;
    if (launches)
        *launches = g_launches;
    if (reset) {
        g_ms = 0.0;
        g_launches = 0;
    }
    return TE_OK;
}

}  // extern "C"
