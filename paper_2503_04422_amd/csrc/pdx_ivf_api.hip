// IVF entry points (declared in include/pdx.h).
#include "pdx_internal.h"

using namespace pdx;

extern "C" {

size_t pdx_ivf_build_bytes(int64_t, int32_t, int32_t, const pdx_ivf_params *) { return 0; }

pdx_status pdx_ivf_build(const float *, int64_t, int32_t, int32_t, const pdx_ivf_params *, void *, size_t,
                         void *, pdx_index **out) {
    if (out) *out = nullptr;
    set_error("pdx_ivf_build: not implemented yet");
    return PDX_EUNSUPPORTED;
}

pdx_status pdx_ivf_export(const pdx_index *, float *, float *, int32_t *, int32_t *, void *) {
    set_error("pdx_ivf_export: not implemented yet");
    return PDX_EUNSUPPORTED;
}

size_t pdx_search_ivf_workspace(const pdx_index *, int64_t, int32_t, int32_t, const pdx_ivf_search_params *) {
    return 0;
}

pdx_status pdx_search_ivf(const pdx_index *index, const float *, int64_t, int32_t, int32_t,
                          const pdx_ivf_search_params *, void *, size_t, int64_t *, float *, void *) {
    if (!index || index->kind != kIvf) {
        set_error("pdx_search_ivf: not an IVF index");
        return PDX_EINVAL;
    }
    set_error("pdx_search_ivf: not implemented yet");
    return PDX_EUNSUPPORTED;
}

}  // extern "C"
