// C ABI entry points of libpdx (declared in include/pdx.h): argument
// validation, carving of the caller's buffers, launch sequencing.
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <new>

#include "pdx_internal.h"

namespace pdx {

static thread_local char g_err[512] = "";

void set_error(const char *fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof(g_err), fmt, ap);
    va_end(ap);
}

namespace {

constexpr int32_t kMeanChunks = 256;

struct FlatLayout {
    float *pdx;
    float *means;
    double *partial;
    int32_t *flag;
    size_t bytes;
};

FlatLayout flat_layout(int64_t n, int32_t d, void *base) {
    int64_t ng = (n + kGroup - 1) / kGroup;
    Carver c(base);
    FlatLayout l{};
    l.pdx = c.take<float>(static_cast<size_t>(ng) * d * kGroup);
    l.means = c.take<float>(d);
    l.partial = c.take<double>(static_cast<size_t>(kMeanChunks) * d);
    l.flag = c.take<int32_t>(64);
    l.bytes = c.bytes();
    return l;
}

bool aligned16(const void *p) { return (reinterpret_cast<uintptr_t>(p) & 15u) == 0; }

pdx_status hip_fail(hipError_t e, const char *what) {
    set_error("%s: %s", what, hipGetErrorString(e));
    return PDX_EHIP;
}

}  // namespace
}  // namespace pdx

using namespace pdx;

extern "C" {

const char *pdx_last_error(void) { return g_err; }

const char *pdx_version(void) { return "pdx 0.1.0 gfx950"; }

void pdx_free(pdx_index *index) { delete index; }

size_t pdx_build_bytes(int64_t n, int32_t d, const pdx_build_params *params) {
    (void)params;
    if (n < 1 || d < 1 || d > PDX_MAX_DIM || n >= (int64_t(1) << 31)) return 0;
    return flat_layout(n, d, nullptr).bytes;
}

pdx_status pdx_build(const float *x, int64_t n, int32_t d, const pdx_build_params *params,
                     void *index_mem, size_t index_bytes, void *stream, pdx_index **out) {
    if (!out) {
        set_error("pdx_build: out is null");
        return PDX_EINVAL;
    }
    *out = nullptr;
    if (!x || !index_mem) {
        set_error("pdx_build: null data or index pointer");
        return PDX_EINVAL;
    }
    if (n < 1 || d < 1 || d > PDX_MAX_DIM || n >= (int64_t(1) << 31)) {
        set_error("pdx_build: need 1 <= n < 2^31 and 1 <= d <= %d (n=%lld d=%d)", PDX_MAX_DIM,
                  (long long)n, d);
        return PDX_EINVAL;
    }
    if (!aligned16(x) || !aligned16(index_mem)) {
        set_error("pdx_build: pointers must be 16-byte aligned");
        return PDX_EINVAL;
    }
    int32_t group = params && params->group ? params->group : kGroup;
    if (group != kGroup) {
        set_error("pdx_build: only vectorgroups of 64 are supported (got %d)", group);
        return PDX_EUNSUPPORTED;
    }
    int32_t start_rows = params && params->start_rows > 0 ? params->start_rows : 10000;
    FlatLayout l = flat_layout(n, d, index_mem);
    if (index_bytes < l.bytes) {
        set_error("pdx_build: index buffer has %zu bytes, needs %zu", index_bytes, l.bytes);
        return PDX_EWORKSPACE;
    }
    hipStream_t s = static_cast<hipStream_t>(stream);
    hipError_t e;
    if ((e = hipMemsetAsync(l.flag, 0, sizeof(int32_t), s)) != hipSuccess) return hip_fail(e, "pdx_build");
    if ((e = launch_finite_check(x, n * d, l.flag, s)) != hipSuccess) return hip_fail(e, "pdx_build");
    if ((e = launch_transpose_pdx(x, n, d, l.pdx, s)) != hipSuccess) return hip_fail(e, "pdx_build");
    if ((e = launch_column_means(x, n, d, l.partial, kMeanChunks, l.means, s)) != hipSuccess)
        return hip_fail(e, "pdx_build");
    int32_t hflag = 0;
    if ((e = hipMemcpyAsync(&hflag, l.flag, sizeof(int32_t), hipMemcpyDeviceToHost, s)) != hipSuccess)
        return hip_fail(e, "pdx_build");
    if ((e = hipStreamSynchronize(s)) != hipSuccess) return hip_fail(e, "pdx_build");
    if (hflag) {
        set_error("pdx_build: data holds NaN or Inf");
        return PDX_EINVAL;
    }
    pdx_index *ix = new (std::nothrow) pdx_index{};
    if (!ix) {
        set_error("pdx_build: out of host memory");
        return PDX_EINVAL;
    }
    ix->kind = kFlat;
    ix->n = n;
    ix->d = d;
    ix->group = kGroup;
    ix->ngroups = static_cast<int32_t>((n + kGroup - 1) / kGroup);
    ix->start_rows = start_rows;
    ix->pdx = l.pdx;
    ix->means = l.means;
    *out = ix;
    return PDX_OK;
}

size_t pdx_search_exact_workspace(const pdx_index *index, int64_t nq, int32_t k,
                                  const pdx_search_params *params) {
    if (!index || (index->kind != kFlat && index->kind != kIvf) || nq < 0 || k < 1 || k > PDX_MAX_K) return 0;
    if (params && (params->metric < PDX_METRIC_L2 || params->metric > PDX_METRIC_IP)) return 0;
    return exact_plan(index, nq, k, params, nullptr, nullptr);
}

pdx_status pdx_search_exact(const pdx_index *index, const float *q, int64_t nq, int32_t k,
                            const pdx_search_params *params, void *ws, size_t ws_bytes,
                            int64_t *out_ids, float *out_dist, void *stream) {
    return pdx::search_exact(index, q, nq, k, params, ws, ws_bytes, out_ids, out_dist, stream, true);
}

}  // extern "C"

namespace pdx {

pdx_status search_exact(const pdx_index *index, const float *q, int64_t nq, int32_t k,
                        const pdx_search_params *params, void *ws, size_t ws_bytes, int64_t *out_ids,
                        float *out_dist, void *stream, bool library_gemm) {
    if (!index || (index->kind != kFlat && index->kind != kIvf)) {
        set_error("pdx_search_exact: not an index built by pdx_build or pdx_ivf_build");
        return PDX_EINVAL;
    }
    if (nq < 0 || k < 1) {
        set_error("pdx_search_exact: need nq >= 0 and k >= 1");
        return PDX_EINVAL;
    }
    if (k > PDX_MAX_K) {
        set_error("pdx_search_exact: k=%d above PDX_MAX_K=%d", k, PDX_MAX_K);
        return PDX_EUNSUPPORTED;
    }
    if (params && params->mode != PDX_MODE_LINEAR && params->mode != PDX_MODE_BOND) {
        set_error("pdx_search_exact: unknown mode %d", params->mode);
        return PDX_EINVAL;
    }
    if (params && (params->metric < PDX_METRIC_L2 || params->metric > PDX_METRIC_IP)) {
        set_error("pdx_search_exact: unknown metric %d", params->metric);
        return PDX_EINVAL;
    }
    if (params && params->metric == PDX_METRIC_IP && params->mode != PDX_MODE_LINEAR) {
        set_error("pdx_search_exact: the inner product has no pruning bound; use PDX_MODE_LINEAR");
        return PDX_EUNSUPPORTED;
    }
    if (params && params->start_rows < 0) {
        set_error("pdx_search_exact: start_rows must be >= 0");
        return PDX_EINVAL;
    }
    if (params && (params->chunk < 0 || params->tile_groups < 0 ||
                   !(params->queries_per_block == 0 || params->queries_per_block == 1 ||
                     params->queries_per_block == 2 || params->queries_per_block == 4 ||
                     params->queries_per_block == 8))) {
        set_error("pdx_search_exact: bad chunk / tile_groups / queries_per_block");
        return PDX_EINVAL;
    }
    if (params && (params->rounds < 0 || params->rounds > kMaxTileRounds || params->dense_min < 0 ||
                   params->dense_min > 33)) {
        set_error("pdx_search_exact: rounds must be in [0, %d], dense_min in [0, 33]", kMaxTileRounds);
        return PDX_EINVAL;
    }
    if (nq == 0) return PDX_OK;
    if (!q || !ws || !out_ids || !out_dist) {
        set_error("pdx_search_exact: null pointer");
        return PDX_EINVAL;
    }
    if (!aligned16(q) || !aligned16(ws)) {
        set_error("pdx_search_exact: pointers must be 16-byte aligned");
        return PDX_EINVAL;
    }
    if (nq > (int64_t(1) << 31) - 1) {
        set_error("pdx_search_exact: nq too large");
        return PDX_EINVAL;
    }
    ExactPlan plan;
    size_t need = exact_plan(index, nq, k, params, ws, &plan);
    if (ws_bytes < need) {
        set_error("pdx_search_exact: workspace has %zu bytes, needs %zu", ws_bytes, need);
        return PDX_EWORKSPACE;
    }
    plan.library_gemm = library_gemm;
    hipError_t e = run_exact(index, q, plan, out_ids, out_dist, static_cast<hipStream_t>(stream));
    if (e != hipSuccess) return hip_fail(e, "pdx_search_exact");
    return PDX_OK;
}

}  // namespace pdx

extern "C" {

namespace {
struct OrderWs {
    uint32_t *tau;
    int32_t *bad;
    float *qrot;
    float *qval;
    size_t bytes;
};
OrderWs order_ws(const pdx_index *ix, int64_t nq, void *base) {
    const size_t q = static_cast<size_t>(nq > 0 ? nq : 0);
    Carver c(base);
    OrderWs w{};
    w.tau = c.take<uint32_t>(q);
    w.bad = c.take<int32_t>(q);
    w.qrot = (ix->kind == kIvf && ix->has_rot) ? c.take<float>(q * ix->d) : nullptr;
    w.qval = c.take<float>(q * ix->d);  // used when the caller does not ask for the values
    w.bytes = c.bytes();
    return w;
}
}  // namespace

size_t pdx_query_order_workspace(const pdx_index *index, int64_t nq) {
    if (!index || (index->kind != kFlat && index->kind != kIvf) || nq < 0) return 0;
    return order_ws(index, nq, nullptr).bytes;
}

pdx_status pdx_query_order(const pdx_index *index, const float *q, int64_t nq, int32_t order, int32_t *out_perm,
                           float *out_qval, uint16_t *out_tile_off, void *ws, size_t ws_bytes, void *stream) {
    if (!index || (index->kind != kFlat && index->kind != kIvf)) {
        set_error("pdx_query_order: not an index built by pdx_build or pdx_ivf_build");
        return PDX_EINVAL;
    }
    if (nq < 0 || nq > (int64_t(1) << 31) - 1) {
        set_error("pdx_query_order: need 0 <= nq < 2^31");
        return PDX_EINVAL;
    }
    if (order != PDX_ORDER_NATURAL && order != PDX_ORDER_BOND && order != PDX_ORDER_ZONES) {
        set_error("pdx_query_order: unknown order %d", order);
        return PDX_EINVAL;
    }
    if (out_tile_off && index->d * 32 >= 65536) {
        set_error("pdx_query_order: 16-bit tile offsets need d * 32 < 65536 (d=%d)", index->d);
        return PDX_EUNSUPPORTED;
    }
    if (nq == 0) return PDX_OK;
    if (!q || !out_perm || !ws) {
        set_error("pdx_query_order: null pointer");
        return PDX_EINVAL;
    }
    if (!aligned16(q) || !aligned16(ws)) {
        set_error("pdx_query_order: pointers must be 16-byte aligned");
        return PDX_EINVAL;
    }
    OrderWs w = order_ws(index, nq, ws);
    if (ws_bytes < w.bytes) {
        set_error("pdx_query_order: workspace has %zu bytes, needs %zu", ws_bytes, w.bytes);
        return PDX_EWORKSPACE;
    }
    hipError_t e = launch_query_order(index, q, nq, order, w.qrot, out_perm, out_qval ? out_qval : w.qval,
                                      out_tile_off, w.tau, w.bad, static_cast<hipStream_t>(stream));
    if (e != hipSuccess) return hip_fail(e, "pdx_query_order");
    return PDX_OK;
}

}  // extern "C"
