// IVF entry points (declared in include/pdx.h): argument validation,
// carving of the caller's buffers, build sequencing.
#include <cmath>
#include <new>

#include "pdx_internal.h"

namespace pdx {
namespace {

constexpr int32_t kMaxNlist = 4096;
constexpr int32_t kRowsPerBlock = 1024;
constexpr int32_t kMeanChunksIvf = 256;

struct IvfLayout {
    float *rot, *centroids, *pdx, *xrot, *fp8_scale, *means, *tile_rad, *tile_rad1;
    uint16_t *pdx16;
    uint8_t *pdx8;
    uint32_t *maxbits;
    int32_t *list_size, *list_goff, *stats, *assign, *slot_id, *cnt, *blk_cnt, *flag, *group_bucket;
    unsigned long long *best;
    double *sums, *acm, *qd, *v, *diag, *mean_partial;
    float *pca_part, *pca_cov, *pca_h, *pca_r2, *pca_tmp, *pca_rho, *pca_cs;  // PCA rotation scratch (pca only)
    float *xres;  // [max_groups][ntp][64] residual norms (BSA)
    float *xn16, *xn8;  // [max_groups][ceil(d / 32)][64] sub-chunk norms of the low-precision codes
    int32_t res_ntp, res_dd;
    double *pca_w64;
    int32_t *pca_perm;
    int64_t max_groups;
    size_t bytes;
};

IvfLayout ivf_layout(int64_t n, int32_t d, int32_t nlist, int32_t lowp_mask, bool pca, void *base) {
    IvfLayout l{};
    l.max_groups = (n + kGroup - 1) / kGroup + nlist;
    int64_t nblocks = (n + kRowsPerBlock - 1) / kRowsPerBlock;
    Carver c(base);
    // index proper
    l.rot = c.take<float>((size_t)d * d);
    l.centroids = c.take<float>((size_t)nlist * d);
    l.list_size = c.take<int32_t>(nlist);
    l.list_goff = c.take<int32_t>(nlist + 1);
    l.stats = c.take<int32_t>(64);
    l.assign = c.take<int32_t>(n);
    l.slot_id = c.take<int32_t>((size_t)l.max_groups * kGroup);
    l.pdx = c.take<float>((size_t)l.max_groups * d * kGroup);
    l.xrot = c.take<float>((size_t)n * d);  // kept: rows for the f32 rerank
    l.means = c.take<float>(d);             // per-dimension means of the stored rows (exact search order)
    l.group_bucket = c.take<int32_t>((size_t)l.max_groups);
    l.tile_rad = c.take<float>((size_t)l.max_groups * 2);
    l.tile_rad1 = c.take<float>((size_t)l.max_groups * 2);
    l.res_dd = d >= 128 ? 32 : (d / 4 > 0 ? d / 4 : 1);  // ADSampling's default delta_d
    l.res_ntp = res_test_points(d, l.res_dd);
    l.xres = l.res_ntp > 0 ? c.take<float>((size_t)l.max_groups * l.res_ntp * kGroup) : nullptr;
    const size_t nsub = (size_t)(d + 31) / 32;
    if (lowp_mask & (1 << PDX_DTYPE_BF16)) {
        l.pdx16 = c.take<uint16_t>((size_t)l.max_groups * d * kGroup);
        l.xn16 = c.take<float>((size_t)l.max_groups * nsub * kGroup);
    }
    if (lowp_mask & (1 << PDX_DTYPE_FP8)) {
        l.pdx8 = c.take<uint8_t>((size_t)l.max_groups * d * kGroup);
        l.xn8 = c.take<float>((size_t)l.max_groups * nsub * kGroup);
        l.fp8_scale = c.take<float>(d);
        l.maxbits = c.take<uint32_t>(d);
    }
    // build scratch
    l.best = c.take<unsigned long long>(n);
    l.sums = c.take<double>((size_t)nlist * d);
    l.cnt = c.take<int32_t>(nlist);
    l.blk_cnt = c.take<int32_t>((size_t)nblocks * nlist);
    l.acm = c.take<double>((size_t)d * d);
    l.qd = c.take<double>((size_t)d * d);
    l.v = c.take<double>(d);
    l.diag = c.take<double>(d);
    l.flag = c.take<int32_t>(64);
    l.mean_partial = c.take<double>((size_t)kMeanChunksIvf * d);
    if (pca) {
        l.pca_part = c.take<float>(pca_part_floats(n, d));
        l.pca_cov = c.take<float>((size_t)d * d);
        l.pca_h = c.take<float>((size_t)d * d);
        l.pca_r2 = c.take<float>((size_t)d * d);
        l.pca_tmp = c.take<float>((size_t)d * d);
        l.pca_w64 = c.take<double>((size_t)d * d);
        l.pca_rho = c.take<float>(d);
        l.pca_perm = c.take<int32_t>(d);
        l.pca_cs = c.take<float>((size_t)3 * d);
    }
    l.bytes = c.bytes();
    return l;
}

bool aligned16(const void *p) { return (reinterpret_cast<uintptr_t>(p) & 15u) == 0; }

pdx_status hip_fail(hipError_t e, const char *what) {
    set_error("%s: %s", what, hipGetErrorString(e));
    return PDX_EHIP;
}

__global__ void identity_kernel(float *rot, int32_t d) {
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i < (int64_t)d * d) rot[i] = (i / d == i % d) ? 1.0f : 0.0f;
}

bool valid_shape(int64_t n, int32_t d, int32_t nlist) {
    return n >= 1 && n < (int64_t(1) << 31) && d >= 1 && d <= PDX_MAX_DIM && nlist >= 1 && nlist <= kMaxNlist &&
           nlist <= n;
}

}  // namespace
}  // namespace pdx

using namespace pdx;

#define TRY(expr)                                        \
    do {                                                 \
        hipError_t e_ = (expr);                          \
        if (e_ != hipSuccess) return hip_fail(e_, what); \
    } while (0)

extern "C" {

size_t pdx_ivf_build_bytes(int64_t n, int32_t d, int32_t nlist, const pdx_ivf_params *params) {
    (void)params;
    if (!valid_shape(n, d, nlist)) return 0;
    if (params && (params->lowp_mask & ~((1 << PDX_DTYPE_BF16) | (1 << PDX_DTYPE_FP8)))) return 0;
    if (params && (params->rotation_kind < PDX_ROTATION_RANDOM || params->rotation_kind > PDX_ROTATION_PCA ||
                   params->pca_iters < 0))
        return 0;
    const bool pca = params && !params->rotation && params->rotation_kind == PDX_ROTATION_PCA;
    return ivf_layout(n, d, nlist, params ? params->lowp_mask : 0, pca, nullptr).bytes;
}

pdx_status pdx_ivf_build(const float *x, int64_t n, int32_t d, int32_t nlist, const pdx_ivf_params *params,
                         void *index_mem, size_t index_bytes, void *stream, pdx_index **out) {
    const char *what = "pdx_ivf_build";
    if (!out) {
        set_error("pdx_ivf_build: out is null");
        return PDX_EINVAL;
    }
    *out = nullptr;
    if (!x || !index_mem || !params) {
        set_error("pdx_ivf_build: null data, index or params pointer");
        return PDX_EINVAL;
    }
    if (!valid_shape(n, d, nlist)) {
        set_error("pdx_ivf_build: need 1 <= nlist <= min(n, %d), 1 <= d <= %d, n < 2^31 (n=%lld d=%d nlist=%d)",
                  kMaxNlist, PDX_MAX_DIM, (long long)n, d, nlist);
        return PDX_EINVAL;
    }
    if (!params->centroids && !params->init_rows) {
        set_error("pdx_ivf_build: init_rows is required unless centroids are given");
        return PDX_EINVAL;
    }
    if (params->assign && !params->centroids) {
        set_error("pdx_ivf_build: assign needs centroids");
        return PDX_EINVAL;
    }
    if (params->lowp_mask & ~((1 << PDX_DTYPE_BF16) | (1 << PDX_DTYPE_FP8))) {
        set_error("pdx_ivf_build: lowp_mask may only hold the bf16 and fp8 bits");
        return PDX_EINVAL;
    }
    if (!aligned16(x) || !aligned16(index_mem)) {
        set_error("pdx_ivf_build: pointers must be 16-byte aligned");
        return PDX_EINVAL;
    }
    if (params->rotation_kind < PDX_ROTATION_RANDOM || params->rotation_kind > PDX_ROTATION_PCA ||
        params->pca_iters < 0) {
        set_error("pdx_ivf_build: unknown rotation_kind %d or negative pca_iters", params->rotation_kind);
        return PDX_EINVAL;
    }
    const bool pca = !params->rotation && params->rotation_kind == PDX_ROTATION_PCA;
    IvfLayout L = ivf_layout(n, d, nlist, params->lowp_mask, pca, index_mem);
    if (index_bytes < L.bytes) {
        set_error("pdx_ivf_build: index buffer has %zu bytes, needs %zu", index_bytes, L.bytes);
        return PDX_EWORKSPACE;
    }
    const int32_t iters = params->kmeans_iters > 0 ? params->kmeans_iters : 20;
    hipStream_t s = static_cast<hipStream_t>(stream);
    TRY(launch_fill_i32(L.flag, 1, 0, s));
    TRY(launch_finite_check(x, n * d, L.flag, s));
    {
        int32_t hf = 0;
        TRY(hipMemcpyAsync(&hf, L.flag, sizeof(int32_t), hipMemcpyDeviceToHost, s));
        TRY(hipStreamSynchronize(s));
        if (hf) {
            set_error("pdx_ivf_build: data holds NaN or Inf");
            return PDX_EINVAL;
        }
    }
    // rotation
    int32_t has_rot = 1;
    if (params->rotation) {
        TRY(hipMemcpyAsync(L.rot, params->rotation, sizeof(float) * d * d, hipMemcpyDeviceToDevice, s));
    } else if (pca) {
        // the rows' column means (into the means slot, rewritten below for
        // the rotated rows), then the principal directions
        TRY(launch_column_means(x, n, d, L.mean_partial, kMeanChunksIvf, L.means, s));
        TRY(launch_pca_rotation(x, n, d, params->pca_iters > 0 ? params->pca_iters : 12, L.means, L.pca_part,
                                L.pca_cov, L.pca_h, L.pca_r2, L.pca_w64, L.acm, L.qd, L.v, L.diag, L.pca_tmp,
                                L.pca_rho, L.pca_perm, L.pca_cs, L.rot, s));
    } else if (params->gaussian) {
        TRY(launch_qr_rotation(params->gaussian, d, L.acm, L.qd, L.v, L.diag, L.rot, s));
    } else {
        has_rot = 0;
        identity_kernel<<<(unsigned)(((int64_t)d * d + 255) / 256), 256, 0, s>>>(L.rot, d);
        TRY(hipGetLastError());
    }
    if (has_rot)
        TRY(launch_sgemm_abt(x, n, L.rot, d, d, L.xrot, d, s));
    else
        TRY(hipMemcpyAsync(L.xrot, x, sizeof(float) * n * d, hipMemcpyDeviceToDevice, s));
    TRY(launch_column_means(L.xrot, n, d, L.mean_partial, kMeanChunksIvf, L.means, s));
    // centroids: given, or Lloyd iterations from the seed rows
    if (params->centroids) {
        TRY(hipMemcpyAsync(L.centroids, params->centroids, sizeof(float) * nlist * d, hipMemcpyDeviceToDevice, s));
    } else {
        TRY(launch_gather_rows(L.xrot, n, d, params->init_rows, nlist, L.centroids, L.flag, s));
        for (int32_t it = 0; it < iters; ++it) {
            TRY(launch_fill_u64(L.best, n, ~0ull, s));
            TRY(launch_pair(1, 1, L.xrot, n, L.centroids, nlist, d, nullptr, 0, L.best, s));
            TRY(launch_labels_from_keys(L.best, n, L.assign, s));
            TRY(launch_kmeans_update(L.xrot, n, d, L.assign, nlist, L.sums, L.cnt, L.centroids, s));
        }
    }
    // final assignment
    if (params->assign) {
        TRY(hipMemcpyAsync(L.assign, params->assign, sizeof(int32_t) * n, hipMemcpyDeviceToDevice, s));
        TRY(launch_check_labels(L.assign, n, nlist, L.flag, s));
    } else {
        TRY(launch_fill_u64(L.best, n, ~0ull, s));
        TRY(launch_pair(1, 1, L.xrot, n, L.centroids, nlist, d, nullptr, 0, L.best, s));
        TRY(launch_labels_from_keys(L.best, n, L.assign, s));
    }
    // the flag must be read before bucketing trusts the labels
    int32_t hflag = 0;
    TRY(hipMemcpyAsync(&hflag, L.flag, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    TRY(hipStreamSynchronize(s));
    if (hflag) {
        set_error("pdx_ivf_build: %s", (hflag & 1)   ? "data holds NaN or Inf"
                                       : (hflag & 2) ? "init_rows holds a row outside [0, n)"
                                                     : "assign holds a bucket outside [0, nlist)");
        return PDX_EINVAL;
    }
    TRY(launch_bucketize(L.xrot, n, d, L.assign, nlist, L.blk_cnt, L.list_size, L.list_goff, L.stats, L.slot_id,
                         L.max_groups * kGroup, L.pdx, L.max_groups, s));
    TRY(launch_tile_radii(L.pdx, L.slot_id, L.list_goff, nlist, L.centroids, d, L.max_groups, L.group_bucket,
                          L.tile_rad, L.tile_rad1, s));
    if (L.xres) TRY(launch_residual_norms(L.pdx, d, L.max_groups, L.stats, L.res_dd, L.xres, s));
    if (L.pdx16 || L.pdx8) {
        TRY(launch_lowp_store(L.xrot, n, d, L.slot_id, L.stats, L.max_groups, L.pdx16, L.pdx8, L.fp8_scale, L.maxbits,
                              s));
        TRY(launch_lowp_norms(L.pdx16, L.pdx8, L.fp8_scale, d, L.stats, L.max_groups, L.xn16, L.xn8, s));
    }
    int32_t hstats[2] = {0, 0};
    TRY(hipMemcpyAsync(hstats, L.stats, sizeof(hstats), hipMemcpyDeviceToHost, s));
    TRY(hipStreamSynchronize(s));
    pdx_index *ix = new (std::nothrow) pdx_index{};
    if (!ix) {
        set_error("pdx_ivf_build: out of host memory");
        return PDX_EINVAL;
    }
    ix->kind = kIvf;
    ix->n = n;
    ix->d = d;
    ix->group = kGroup;
    ix->ngroups = hstats[0];
    ix->max_list = hstats[1];
    ix->nlist = nlist;
    ix->dtype_mask = (1 << PDX_DTYPE_F32) | params->lowp_mask;
    ix->pdx_bf16 = L.pdx16;
    ix->pdx_fp8 = L.pdx8;
    ix->fp8_scale = L.fp8_scale;
    ix->xn_bf16 = L.xn16;
    ix->xn_fp8 = L.xn8;
    ix->lp_nsub = (d + 31) / 32;
    ix->xrow = L.xrot;
    ix->has_rot = has_rot;
    ix->rot = L.rot;
    ix->centroids = L.centroids;
    ix->list_goff = L.list_goff;
    ix->list_size = L.list_size;
    ix->slot_id = L.slot_id;
    ix->assign = L.assign;
    ix->pdx = L.pdx;
    ix->means = L.means;
    ix->group_bucket = L.group_bucket;
    ix->tile_rad = L.tile_rad;
    ix->tile_rad1 = L.tile_rad1;
    ix->xres = L.xres;
    ix->res_ntp = L.res_ntp;
    ix->res_dd = L.res_dd;
    *out = ix;
    return PDX_OK;
}

pdx_status pdx_ivf_export(const pdx_index *index, float *rotation, float *centroids, int32_t *assign,
                          int32_t *list_sizes, void *stream) {
    const char *what = "pdx_ivf_export";
    if (!index || index->kind != kIvf) {
        set_error("pdx_ivf_export: not an IVF index");
        return PDX_EINVAL;
    }
    hipStream_t s = static_cast<hipStream_t>(stream);
    const int32_t d = index->d;
    if (rotation) TRY(hipMemcpyAsync(rotation, index->rot, sizeof(float) * d * d, hipMemcpyDeviceToDevice, s));
    if (centroids)
        TRY(hipMemcpyAsync(centroids, index->centroids, sizeof(float) * index->nlist * d, hipMemcpyDeviceToDevice,
                           s));
    if (assign) TRY(hipMemcpyAsync(assign, index->assign, sizeof(int32_t) * index->n, hipMemcpyDeviceToDevice, s));
    if (list_sizes)
        TRY(hipMemcpyAsync(list_sizes, index->list_size, sizeof(int32_t) * index->nlist, hipMemcpyDeviceToDevice, s));
    return PDX_OK;
}

size_t pdx_search_ivf_workspace(const pdx_index *index, int64_t nq, int32_t k, int32_t nprobe,
                                const pdx_ivf_search_params *params) {
    if (!index || index->kind != kIvf || nq < 0 || k < 1 || k > PDX_MAX_K || nprobe < 1 || nprobe > index->nlist)
        return 0;
    return ivf_plan(index, nq, k, nprobe, params, nullptr, nullptr);
}

pdx_status pdx_search_ivf(const pdx_index *index, const float *q, int64_t nq, int32_t k, int32_t nprobe,
                          const pdx_ivf_search_params *params, void *ws, size_t ws_bytes, int64_t *out_ids,
                          float *out_dist, void *stream) {
    const char *what = "pdx_search_ivf";
    if (!index || index->kind != kIvf) {
        set_error("pdx_search_ivf: not an IVF index");
        return PDX_EINVAL;
    }
    if (nq < 0 || k < 1 || nprobe < 1 || nprobe > index->nlist) {
        set_error("pdx_search_ivf: need nq >= 0, k >= 1, 1 <= nprobe <= nlist (%d)", index->nlist);
        return PDX_EINVAL;
    }
    if (k > PDX_MAX_K) {
        set_error("pdx_search_ivf: k=%d above PDX_MAX_K=%d", k, PDX_MAX_K);
        return PDX_EUNSUPPORTED;
    }
    if (params && (params->delta_d < 0 || std::isnan(params->eps0) || params->eps0 < 0.0f)) {
        set_error("pdx_search_ivf: need delta_d >= 0 and eps0 >= 0");
        return PDX_EINVAL;
    }
    if (params && (params->dtype < 0 || params->dtype > PDX_DTYPE_FP8 || !((index->dtype_mask >> params->dtype) & 1))) {
        set_error("pdx_search_ivf: dtype %d is not stored in this index", params ? params->dtype : -1);
        return PDX_EUNSUPPORTED;
    }
    if (params && params->dtype != PDX_DTYPE_F32 && params->rerank > PDX_MAX_RERANK) {
        set_error("pdx_search_ivf: rerank=%d above PDX_MAX_RERANK=%d", params->rerank, PDX_MAX_RERANK);
        return PDX_EUNSUPPORTED;
    }
    if (params && params->rerank_capacity < 0) {
        set_error("pdx_search_ivf: rerank_capacity must be >= 0");
        return PDX_EINVAL;
    }
    if (params && params->dtype != PDX_DTYPE_F32 && params->rerank > PDX_MAX_K) {
        // more candidates than a wave's register list: the candidate buffer
        const int32_t r = params->rerank;
        if (params->mlp || params->prune_mlp || params->trace_features || params->trace_need ||
            params->trace_prune_features) {
            set_error("pdx_search_ivf: the learned networks and their traces need rerank <= PDX_MAX_K=%d",
                      PDX_MAX_K);
            return PDX_EUNSUPPORTED;
        }
        if (params->rerank_capacity != 0 && (params->rerank_capacity < 2 * r || params->rerank_capacity < r + 256)) {
            set_error("pdx_search_ivf: rerank_capacity must be 0 or at least max(2 rerank, rerank + 256)");
            return PDX_EINVAL;
        }
        const int32_t cap = wide_capacity(index, nprobe, r, params->rerank_capacity);
        const int32_t rounds = wide_rounds(index, nprobe, r, cap);
        if (rounds < 0 || rounds > kMaxWideRounds) {
            set_error("pdx_search_ivf: rerank_capacity %d would need %d compaction rounds (at most %d); raise it",
                      cap, rounds, kMaxWideRounds);
            return PDX_EINVAL;
        }
    }
    if (nq == 0) return PDX_OK;
    if (!q || !ws || !out_ids || !out_dist) {
        set_error("pdx_search_ivf: null pointer");
        return PDX_EINVAL;
    }
    if (!aligned16(q) || !aligned16(ws)) {
        set_error("pdx_search_ivf: pointers must be 16-byte aligned");
        return PDX_EINVAL;
    }
    if (params && params->queries_per_wave != 0 && params->queries_per_wave != 1 && params->queries_per_wave != 2 &&
        params->queries_per_wave != 4 && params->queries_per_wave != 8 && params->queries_per_wave != 16 &&
        !(params->queries_per_wave == 32 && params->engine == 2)) {
        set_error("pdx_search_ivf: queries_per_wave must be 0, 1, 2, 4, 8, 16 (or 32 with engine 2), got %d",
                  params->queries_per_wave);
        return PDX_EINVAL;
    }
    if (params && params->bucket_split != 0 && params->bucket_split != 1 && params->bucket_split != 2 &&
        params->bucket_split != 4 && params->bucket_split != 8) {
        set_error("pdx_search_ivf: bucket_split must be 0, 1, 2, 4 or 8 (got %d)", params->bucket_split);
        return PDX_EINVAL;
    }
    if (params && (params->bound < 0 || params->bound > 3)) {
        set_error("pdx_search_ivf: bound must be 0 (ADSampling), 1 (PDX-BOND), 2 (PDX-BOND, dimension zones) "
                  "or 3 (BSA)");
        return PDX_EINVAL;
    }
    if (params && (params->bound == 1 || params->bound == 2) && params->dtype != PDX_DTYPE_F32) {
        set_error("pdx_search_ivf: the PDX-BOND bound scans f32 storage only");
        return PDX_EUNSUPPORTED;
    }
    if (params && params->bound == 3) {
        const int32_t dd_def = index->d >= 128 ? 32 : (index->d / 4 > 0 ? index->d / 4 : 1);
        if (!(params->bsa_m >= 0.0f && params->bsa_m <= 1.0f)) {
            set_error("pdx_search_ivf: bsa_m must lie in [0, 1]");
            return PDX_EINVAL;
        }
        if (params->delta_d != 0 && params->delta_d != dd_def) {
            set_error("pdx_search_ivf: BSA's residual norms are stored for delta_d = %d", dd_def);
            return PDX_EUNSUPPORTED;
        }
        if (params->engine == 2) {
            set_error("pdx_search_ivf: BSA's test runs on the vector-ALU scans (engine 0 or 1)");
            return PDX_EUNSUPPORTED;
        }
        if (!index->xres && index->res_ntp > 0) {
            set_error("pdx_search_ivf: this index holds no residual norms");
            return PDX_EUNSUPPORTED;
        }
    }
    if (params && params->prune_mlp && params->bound != 0) {
        set_error("pdx_search_ivf: the learned prune multiplier replaces the ADSampling test (bound 0)");
        return PDX_EINVAL;
    }
    if (params && !(params->prune_scale >= 0.0f && params->prune_scale < INFINITY)) {
        set_error("pdx_search_ivf: prune_scale must be finite and >= 0");
        return PDX_EINVAL;
    }
    if (params && params->prune_table && !params->prune_mlp) {
        set_error("pdx_search_ivf: prune_table needs prune_mlp");
        return PDX_EINVAL;
    }
    if (params && (!params->trace_prune_features) != (!params->trace_prune_target)) {
        set_error("pdx_search_ivf: trace_prune_features and trace_prune_target go together");
        return PDX_EINVAL;
    }
    if (params && (params->engine < 0 || params->engine > 2)) {
        set_error("pdx_search_ivf: engine must be 0, 1 or 2");
        return PDX_EINVAL;
    }
    if (params && (params->bucket_order < 0 || params->bucket_order > 1)) {
        set_error("pdx_search_ivf: bucket_order must be 0 or 1");
        return PDX_EINVAL;
    }
    // item slots, padding included (at most 15 per bucket and segment of 6)
    if (nq * (int64_t)nprobe + (int64_t)15 * 6 * index->nlist + 16 >= (int64_t(1) << 31)) {
        set_error("pdx_search_ivf: nq * nprobe too large");
        return PDX_EINVAL;
    }
    IvfPlan plan;
    size_t need = ivf_plan(index, nq, k, nprobe, params, ws, &plan);
    if (ws_bytes < need) {
        set_error("pdx_search_ivf: workspace has %zu bytes, needs %zu", ws_bytes, need);
        return PDX_EWORKSPACE;
    }
    TRY(run_ivf(index, q, plan, out_ids, out_dist, static_cast<hipStream_t>(stream)));
    return PDX_OK;
}

}  // extern "C"
