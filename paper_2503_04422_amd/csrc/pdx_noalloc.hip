// pdx_search_exact_noalloc: the exact search with its workspace in a
// static device array instead of a caller buffer, for callers that cannot
// allocate device memory (code under stream capture, serving loops).
//
// `scratch` is a file-scope device array; every GPU the library runs on
// holds its own copy at its own address until the process ends.  Host code
// never passes the array's name to a kernel: the device address is looked
// up once per device with hipGetSymbolAddress (with that device current)
// and kept in g_scratch.  The search's kernels initialise every workspace
// part they read (thresholds, counters, candidate counts are filled by
// kernels, not memsets), so stale contents from an earlier call do no
// harm; calls that overlap on one GPU share the array and race.
#include <mutex>

#include "pdx_internal.h"

namespace pdx {
namespace {

constexpr size_t kScratchBytes = PDX_NOALLOC_SCRATCH_BYTES;
constexpr int kMaxDevices = 64;

__device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_scratch_mu;
void *g_scratch[kMaxDevices] = {};

// Device address of this device's copy of `scratch` (looked up once).
pdx_status scratch_address(void **out) {
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) {
        set_error("pdx_search_exact_noalloc: hipGetDevice: %s", hipGetErrorString(e));
        return PDX_EHIP;
    }
    if (dev < 0 || dev >= kMaxDevices) {
        set_error("pdx_search_exact_noalloc: device %d beyond the %d supported", dev, kMaxDevices);
        return PDX_EUNSUPPORTED;
    }
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            set_error("pdx_search_exact_noalloc: hipGetSymbolAddress: %s", hipGetErrorString(e));
            return PDX_EHIP;
        }
        g_scratch[dev] = p;
    }
    *out = g_scratch[dev];
    return PDX_OK;
}

}  // namespace
}  // namespace pdx

using namespace pdx;

extern "C" {

pdx_status pdx_search_exact_noalloc(const pdx_index *index, const float *q, int64_t nq, int32_t k,
                                    const pdx_search_params *params, int64_t *out_ids, float *out_dist,
                                    void *stream) {
    if (!index || (index->kind != kFlat && index->kind != kIvf)) {
        set_error("pdx_search_exact_noalloc: not an index built by pdx_build or pdx_ivf_build");
        return PDX_EINVAL;
    }
    if (nq < 0 || k < 1) {
        set_error("pdx_search_exact_noalloc: need nq >= 0 and k >= 1");
        return PDX_EINVAL;
    }
    if (nq == 0) return PDX_OK;
    const size_t need = pdx_search_exact_workspace(index, nq, k, params);
    if (need == 0) {  // arguments the sizing query rejects: let the search report them
        return search_exact(index, q, nq, k, params, nullptr, 0, out_ids, out_dist, stream, false);
    }
    if (need > kScratchBytes) {
        set_error("pdx_search_exact_noalloc: this search needs %zu bytes of workspace, above the static "
                  "scratch of %zu bytes; search fewer queries per call",
                  need, kScratchBytes);
        return PDX_EWORKSPACE;
    }
    void *ws = nullptr;
    const pdx_status st = scratch_address(&ws);
    if (st != PDX_OK) return st;
    // the library's own GEMM kernel: rocBLAS may allocate (its handle, its workspace)
    return search_exact(index, q, nq, k, params, ws, kScratchBytes, out_ids, out_dist, stream, false);
}

}  // extern "C"
