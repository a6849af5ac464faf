// Scan-schedule autotuner for the IVF search (pdx_ivf_tune, include/pdx.h).
#include <cmath>

#include "pdx_internal.h"

namespace {

struct Candidate {
    int32_t engine, qpw, order, delta_d;  // delta_d 0: the search's own
};

// candidate order is part of the interface (the table is filled in it)
constexpr Candidate kCandidates[PDX_TUNE_CANDIDATES] = {
    {1, 1, 0, 0}, {1, 1, 1, 0}, {1, 2, 0, 0}, {1, 4, 0, 0}, {1, 8, 0, 0}, {2, 0, 0, 0}, {2, 0, 1, 0},
    {1, 1, 0, 64}, {1, 1, 1, 64}, {1, 2, 0, 64}, {1, 4, 0, 64}, {1, 8, 0, 64}, {2, 0, 0, 64}, {2, 0, 1, 64},
};

pdx_ivf_search_params with(const pdx_ivf_search_params &base, const Candidate &c) {
    pdx_ivf_search_params p = base;
    p.engine = c.engine;
    p.queries_per_wave = c.qpw;
    p.bucket_order = c.order;
    if (c.delta_d) p.delta_d = c.delta_d;
    p.phase_events = nullptr;
    p.counters = nullptr;
    return p;
}

bool usable(const pdx_index *index, const pdx_ivf_search_params &base, int32_t tune_delta_d, const Candidate &c) {
    // BSA's test: vector-ALU scans and the delta_d its residual norms were stored for
    if (base.bound == 3 && (c.engine == 2 || c.delta_d)) return false;
    if (!c.delta_d) return true;
    return tune_delta_d && std::isfinite(base.eps0) && c.delta_d < index->d;
}

}  // namespace

extern "C" {

size_t pdx_ivf_tune_workspace(const pdx_index *index, int64_t nq, int32_t k, int32_t nprobe,
                              const pdx_ivf_search_params *params) {
    if (!index || !params || nq < 0 || k < 1) return 0;
    size_t need = 0;
    for (const Candidate &c : kCandidates) {
        const pdx_ivf_search_params p = with(*params, c);
        const size_t w = pdx_search_ivf_workspace(index, nq, k, nprobe, &p);
        if (w > need) need = w;
    }
    // result buffers after the search workspace
    return pdx::align_up(need, 256) + pdx::align_up((size_t)nq * k * sizeof(int64_t), 256) +
           pdx::align_up((size_t)nq * k * sizeof(float), 256);
}

pdx_status pdx_ivf_tune(const pdx_index *index, const float *q, int64_t nq, int32_t k, int32_t nprobe,
                        pdx_ivf_search_params *params, int32_t tune_delta_d, int32_t reps, pdx_ivf_schedule *table,
                        void *ws, size_t ws_bytes, void *stream) {
    if (!index || !params || !q || !ws || nq < 1 || reps < 1) {
        pdx::set_error("pdx_ivf_tune: need index, params, queries, workspace, nq >= 1 and reps >= 1");
        return PDX_EINVAL;
    }
    if (params->mlp || params->trace_features || params->trace_need || params->prune_mlp || params->prune_table ||
        params->trace_prune_features || params->trace_prune_target) {
        pdx::set_error("pdx_ivf_tune: tune the search without the networks or traces");
        return PDX_EINVAL;
    }
    const size_t need = pdx_ivf_tune_workspace(index, nq, k, nprobe, params);
    if (need == 0) {
        pdx::set_error("pdx_ivf_tune: invalid index or sizes");
        return PDX_EINVAL;
    }
    if (ws_bytes < need) {
        pdx::set_error("pdx_ivf_tune: workspace has %zu bytes, needs %zu", ws_bytes, need);
        return PDX_EWORKSPACE;
    }
    hipStream_t s = static_cast<hipStream_t>(stream);
    size_t search_bytes = 0;
    for (const Candidate &c : kCandidates) {
        const pdx_ivf_search_params p = with(*params, c);
        const size_t w = pdx_search_ivf_workspace(index, nq, k, nprobe, &p);
        if (w > search_bytes) search_bytes = w;
    }
    char *base = static_cast<char *>(ws);
    const size_t off_ids = pdx::align_up(search_bytes, 256);
    int64_t *ids = reinterpret_cast<int64_t *>(base + off_ids);
    float *dist = reinterpret_cast<float *>(base + off_ids + pdx::align_up((size_t)nq * k * sizeof(int64_t), 256));
    hipEvent_t ev[2];
    if (hipEventCreate(&ev[0]) != hipSuccess) {
        pdx::set_error("pdx_ivf_tune: hipEventCreate failed");
        return PDX_EHIP;
    }
    if (hipEventCreate(&ev[1]) != hipSuccess) {
        (void)hipEventDestroy(ev[0]);  // best effort on the error path
        pdx::set_error("pdx_ivf_tune: hipEventCreate failed");
        return PDX_EHIP;
    }
    pdx_status st = PDX_OK;
    bool event_failed = false;
    int best = -1;
    float best_ms = INFINITY;
    for (int ci = 0; ci < PDX_TUNE_CANDIDATES && st == PDX_OK; ++ci) {
        const Candidate &c = kCandidates[ci];
        float ms = -1.0f;
        if (usable(index, *params, tune_delta_d, c)) {
            const pdx_ivf_search_params p = with(*params, c);
            st = pdx_search_ivf(index, q, nq, k, nprobe, &p, ws, search_bytes, ids, dist, stream);  // warm-up
            for (int r = 0; r < reps && st == PDX_OK; ++r) {
                float t = 0.0f;
                if (hipEventRecord(ev[0], s) != hipSuccess) event_failed = true;
                if (!event_failed) st = pdx_search_ivf(index, q, nq, k, nprobe, &p, ws, search_bytes, ids, dist, stream);
                if (st == PDX_OK && !event_failed &&
                    (hipEventRecord(ev[1], s) != hipSuccess || hipEventSynchronize(ev[1]) != hipSuccess ||
                     hipEventElapsedTime(&t, ev[0], ev[1]) != hipSuccess))
                    event_failed = true;
                if (event_failed) st = PDX_EHIP;
                if (st == PDX_OK && (ms < 0.0f || t < ms)) ms = t;
            }
            if (st == PDX_OK && ms < best_ms) {
                best_ms = ms;
                best = ci;
            }
        }
        if (table) table[ci] = pdx_ivf_schedule{c.engine, c.qpw, c.order, c.delta_d ? c.delta_d : params->delta_d, ms};
    }
    if (hipEventDestroy(ev[0]) != hipSuccess) event_failed = true;
    if (hipEventDestroy(ev[1]) != hipSuccess) event_failed = true;
    if (event_failed) pdx::set_error("pdx_ivf_tune: a HIP event call failed");
    if (st != PDX_OK) return st;
    const Candidate &c = kCandidates[best];
    params->engine = c.engine;
    params->queries_per_wave = c.qpw;
    params->bucket_order = c.order;
    if (c.delta_d) params->delta_d = c.delta_d;
    return PDX_OK;
}

}  // extern "C"

// ---- exact search (pdx_exact_tune) ----

namespace {

struct ExactCandidate {
    int32_t start_rows, rounds, dense_min;
};

// candidate order is part of the interface (the table is filled in it)
constexpr int32_t kStartRows[3] = {64, 128, 256};
constexpr int32_t kRoundsSet[3] = {2, 4, 8};
constexpr int32_t kDenseSet[3] = {4, 8, 16};

ExactCandidate exact_candidate(int i) {
    return ExactCandidate{kStartRows[i / 9], kRoundsSet[(i / 3) % 3], kDenseSet[i % 3]};
}

pdx_search_params exact_with(const pdx_search_params &base, const ExactCandidate &c) {
    pdx_search_params p = base;
    p.start_rows = c.start_rows;
    p.rounds = c.rounds;
    p.dense_min = c.dense_min;
    p.phase_events = nullptr;
    p.counters = nullptr;
    p.chunk_survivors = nullptr;
    return p;
}

// A candidate is timed when each of its values reaches the scan it would
// change: START's block on the bucket layout, the tile path's rounds, and
// its dense continuation on the bucket layout.  Values that change nothing
// must be the defaults, so the search is timed once per distinct schedule.
bool exact_usable(const pdx_index *index, int64_t nq, int32_t k, const pdx_search_params &base,
                  const ExactCandidate &c) {
    const pdx_search_params p = exact_with(base, c);
    pdx::ExactPlan pl;
    (void)pdx::exact_plan(index, nq, k, &p, nullptr, &pl);
    const bool start = pl.ivf && (pl.mode == PDX_MODE_BOND || (pl.metric == PDX_METRIC_IP && pl.use_tiles));
    const bool tiles = pl.use_tiles && pl.metric != PDX_METRIC_IP;
    const bool dense = tiles && pl.ivf;
    return (start || c.start_rows == 128) && (tiles || c.rounds == pdx::kDefaultRounds) &&
           (dense || c.dense_min == pdx::kDefaultDenseMin);
}

}  // namespace

extern "C" {

size_t pdx_exact_tune_workspace(const pdx_index *index, int64_t nq, int32_t k, const pdx_search_params *params) {
    if (!index || !params || nq < 0 || k < 1) return 0;
    size_t need = 0;
    for (int i = 0; i < PDX_EXACT_TUNE_CANDIDATES; ++i) {
        const pdx_search_params p = exact_with(*params, exact_candidate(i));
        const size_t w = pdx_search_exact_workspace(index, nq, k, &p);
        if (w == 0) return 0;
        if (w > need) need = w;
    }
    return pdx::align_up(need, 256) + pdx::align_up((size_t)nq * k * sizeof(int64_t), 256) +
           pdx::align_up((size_t)nq * k * sizeof(float), 256);
}

pdx_status pdx_exact_tune(const pdx_index *index, const float *q, int64_t nq, int32_t k, pdx_search_params *params,
                          int32_t reps, pdx_exact_schedule *table, void *ws, size_t ws_bytes, void *stream) {
    if (!index || !params || !q || !ws || nq < 1 || reps < 1) {
        pdx::set_error("pdx_exact_tune: need index, params, queries, workspace, nq >= 1 and reps >= 1");
        return PDX_EINVAL;
    }
    const size_t need = pdx_exact_tune_workspace(index, nq, k, params);
    if (need == 0) {
        pdx::set_error("pdx_exact_tune: invalid index, sizes or params");
        return PDX_EINVAL;
    }
    if (ws_bytes < need) {
        pdx::set_error("pdx_exact_tune: workspace has %zu bytes, needs %zu", ws_bytes, need);
        return PDX_EWORKSPACE;
    }
    hipStream_t s = static_cast<hipStream_t>(stream);
    size_t search_bytes = 0;
    for (int i = 0; i < PDX_EXACT_TUNE_CANDIDATES; ++i) {
        const pdx_search_params p = exact_with(*params, exact_candidate(i));
        const size_t w = pdx_search_exact_workspace(index, nq, k, &p);
        if (w > search_bytes) search_bytes = w;
    }
    char *base = static_cast<char *>(ws);
    const size_t off_ids = pdx::align_up(search_bytes, 256);
    int64_t *ids = reinterpret_cast<int64_t *>(base + off_ids);
    float *dist = reinterpret_cast<float *>(base + off_ids + pdx::align_up((size_t)nq * k * sizeof(int64_t), 256));
    hipEvent_t ev[2];
    if (hipEventCreate(&ev[0]) != hipSuccess) {
        pdx::set_error("pdx_exact_tune: hipEventCreate failed");
        return PDX_EHIP;
    }
    if (hipEventCreate(&ev[1]) != hipSuccess) {
        (void)hipEventDestroy(ev[0]);  // best effort on the error path
        pdx::set_error("pdx_exact_tune: hipEventCreate failed");
        return PDX_EHIP;
    }
    pdx_status st = PDX_OK;
    bool event_failed = false;
    int best = -1;
    float best_ms = INFINITY;
    for (int ci = 0; ci < PDX_EXACT_TUNE_CANDIDATES && st == PDX_OK; ++ci) {
        const ExactCandidate c = exact_candidate(ci);
        float ms = -1.0f;
        if (exact_usable(index, nq, k, *params, c)) {
            const pdx_search_params p = exact_with(*params, c);
            st = pdx_search_exact(index, q, nq, k, &p, ws, search_bytes, ids, dist, stream);  // warm-up
            for (int r = 0; r < reps && st == PDX_OK; ++r) {
                float t = 0.0f;
                if (hipEventRecord(ev[0], s) != hipSuccess) event_failed = true;
                if (!event_failed) st = pdx_search_exact(index, q, nq, k, &p, ws, search_bytes, ids, dist, stream);
                if (st == PDX_OK && !event_failed &&
                    (hipEventRecord(ev[1], s) != hipSuccess || hipEventSynchronize(ev[1]) != hipSuccess ||
                     hipEventElapsedTime(&t, ev[0], ev[1]) != hipSuccess))
                    event_failed = true;
                if (event_failed) st = PDX_EHIP;
                if (st == PDX_OK && (ms < 0.0f || t < ms)) ms = t;
            }
            if (st == PDX_OK && ms < best_ms) {
                best_ms = ms;
                best = ci;
            }
        }
        if (table) table[ci] = pdx_exact_schedule{c.start_rows, c.rounds, c.dense_min, ms};
    }
    if (hipEventDestroy(ev[0]) != hipSuccess) event_failed = true;
    if (hipEventDestroy(ev[1]) != hipSuccess) event_failed = true;
    if (event_failed) pdx::set_error("pdx_exact_tune: a HIP event call failed");
    if (st != PDX_OK) return st;
    const ExactCandidate c = exact_candidate(best);
    params->start_rows = c.start_rows;
    params->rounds = c.rounds;
    params->dense_min = c.dense_min;
    return PDX_OK;
}

}  // extern "C"
