// te_noalloc.hip -- te_knn_counts_noalloc: the neighbour-count export with its
// device scratch in a static array of the library instead of a caller workspace,
// for callers that cannot allocate device memory.

#include <hip/hip_runtime.h>

#include <mutex>

#include "te.h"
#include "te_internal.h"
#include "te_runtime.h"

namespace te {

// Scratch of te_knn_counts_noalloc, one copy per device, held until the process
// ends.  In host code this name is only a stand-in for the symbol: its device
// address comes from hipGetSymbolAddress (scratch_on_current_device).
static __device__ __align__(256) unsigned char scratch[TE_NOALLOC_SCRATCH_BYTES];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void *g_ptr[kMaxDevices] = {};

// Device address of the current device's copy of `scratch`, looked up once per device.
te_status scratch_on_current_device(char **out)
{
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess)
        return hip_fail(e, "hipGetDevice");
    if (dev < 0 || dev >= kMaxDevices)
        return fail(TE_ERR_DEVICE, "device %d out of range for the scratch table", dev);
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_ptr[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return hip_fail(e != hipSuccess ? e : hipErrorInvalidSymbol, "hipGetSymbolAddress(scratch)");
        g_ptr[dev] = p;
    }
    *out = static_cast<char *>(g_ptr[dev]);
    return TE_OK;
}

}  // namespace
}  // namespace te

using namespace te;

extern "C" {

te_status te_knn_counts_noalloc(const float *pts, int64_t dim_stride, const int64_t *offsets, int32_t n_chunks,
                                int32_t d_y, int32_t d_x, int32_t k, void *hip_stream, float *eps, int32_t *counts,
                                double *te_out)
{
    clear_error();
    if (n_chunks >= 1 && offsets) {
        const size_t need = te_knn_counts_workspace_bytes(n_chunks, offsets[n_chunks]);
        if (need > (size_t)TE_NOALLOC_SCRATCH_BYTES)
            return fail(TE_ERR_NOMEM,
                        "te_knn_counts_noalloc: %d chunks of %lld points need %zu bytes of scratch; the library's "
                        "static scratch holds %zu (use te_knn_counts with a workspace)",
                        n_chunks, (long long)offsets[n_chunks], need, (size_t)TE_NOALLOC_SCRATCH_BYTES);
    }
    char *ws = nullptr;
    te_status s = scratch_on_current_device(&ws);
    if (s != TE_OK)
        return s;
    return knn_counts_run(pts, dim_stride, offsets, n_chunks, d_y, d_x, k, ws, (size_t)TE_NOALLOC_SCRATCH_BYTES,
                          (hipStream_t)hip_stream, eps, counts, te_out, false, "static scratch");
}

}  // extern "C"
