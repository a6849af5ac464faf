// Device side of the IVF search's candidate buffer (WideSink): append,
// threshold refresh from the distance histogram, and overflow bookkeeping.
#pragma once

#include "wave_topk.h"

namespace pdx {

// Bin of a non-negative distance: 64 bins per octave (the exponent and the
// top 6 mantissa bits), shifted by the query's base, clamped at both ends.
__device__ __forceinline__ int wide_bin(float v, int32_t hb) {
    const int b = (int)(__float_as_uint(v) >> 17) - hb;
    return min(max(b, 0), kWideBins - 1);
}

// Lower tau[q] to the upper edge of the bin where the stored count reaches
// r (whole wave).  The counters only grow, so any snapshot undercounts and
// the edge found is still one with at least r stored keys strictly below.
__device__ __forceinline__ void wide_refresh(const WideSink &w, int64_t q, uint32_t *tau, int lane) {
    const uint32_t *h = w.hist + q * kWideBins + lane * (kWideBins / kWave);
    uint32_t v[kWideBins / kWave];
    uint32_t sum = 0;
#pragma unroll
    for (int i = 0; i < kWideBins / kWave; ++i) {
        v[i] = __hip_atomic_load(h + i, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        sum += v[i];
    }
    uint32_t pre = sum;  // inclusive prefix over lanes
#pragma unroll
    for (int off = 1; off < kWave; off <<= 1) {
        const uint32_t t = __shfl_up(pre, off);
        if (lane >= off) pre += t;
    }
    const unsigned long long hit = __ballot(pre >= (uint32_t)w.r);
    if (!hit) return;
    const int src = __ffsll((long long)hit) - 1;
    int bin = kWideBins;
    if (lane == src) {
        uint32_t cum = pre - sum;
#pragma unroll
        for (int i = 0; i < kWideBins / kWave; ++i) {
            cum += v[i];
            if (cum >= (uint32_t)w.r && bin == kWideBins) bin = lane * (kWideBins / kWave) + i;
        }
    }
    bin = __shfl(bin, src);
    if (bin >= kWideBins - 1) return;  // the last bin is open-ended
    const uint32_t edge = (uint32_t)(w.hbase[q] + bin + 1) << 17;
    if (lane == 0) atomicMin(tau + q, edge);
}

// A refresh after a reservation [base, base + n): when the buffer first
// holds r keys, then each time its count crosses a multiple of
// kWideRefreshStep (a refresh reads the whole histogram; between refreshes
// the threshold only stays looser, never wrong).
constexpr int kWideRefreshStep = 256;
__device__ __forceinline__ bool wide_due(int base, int n, int r) {
    const int end = base + n;
    return end >= r && (base < r || end / kWideRefreshStep != base / kWideRefreshStep);
}

// Append the keys (dist, id) of the lanes where `cand` holds for query q.
// Returns false, storing nothing, when the reservation does not fit (the
// slots of a reservation that straddles the end are marked empty); the
// caller then records where to resume.
__device__ __forceinline__ bool wide_push(const WideSink &w, int64_t q, float dist, uint32_t id, bool cand,
                                          int32_t hb, uint32_t *tau, int lane) {
    const unsigned long long m = __ballot(cand);
    if (!m) return true;
    const int n = __popcll(m);
    int base = 0;
    if (lane == 0) base = atomicAdd(w.cnt + q, n);
    base = __shfl(base, 0);
    const int pos =
        base + (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
    uint64_t *row = w.buf + q * (int64_t)w.cap;
    if (base <= w.cap - n) {
        if (cand) {
            row[pos] = make_key(dist, id);
            atomicAdd(w.hist + q * kWideBins + wide_bin(dist, hb), 1u);
        }
        if (wide_due(base, n, w.r)) wide_refresh(w, q, tau, lane);
        return true;
    }
    if (cand && pos < w.cap) row[pos] = kEmptyKey;
    return false;
}

// wide_push for up to 4 candidates per lane (vectors vid[t] at distances
// dist[t] where cand[t]): one reservation for all of them, all or nothing.
__device__ __forceinline__ bool wide_push4(const WideSink &w, int64_t q, const float (&dist)[4],
                                           const int32_t (&vid)[4], const bool (&cand)[4], int32_t hb, uint32_t *tau,
                                           int lane) {
    unsigned long long m[4];
    int pre[4];
    int n = 0;
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        m[t] = __ballot(cand[t]);
        pre[t] = n;
        n += __popcll(m[t]);
    }
    if (!n) return true;
    int base = 0;
    if (lane == 0) base = atomicAdd(w.cnt + q, n);
    base = __shfl(base, 0);
    uint64_t *row = w.buf + q * (int64_t)w.cap;
    const bool fits = base <= w.cap - n;
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        if (!cand[t]) continue;
        const int pos = base + pre[t] +
                        (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(m[t] >> 32),
                                                       __builtin_amdgcn_mbcnt_lo((uint32_t)m[t], 0u));
        if (fits) {
            row[pos] = make_key(dist[t], (uint32_t)vid[t]);
            atomicAdd(w.hist + q * kWideBins + wide_bin(dist[t], hb), 1u);
        } else if (pos < w.cap) {
            row[pos] = kEmptyKey;
        }
    }
    if (fits && wide_due(base, n, w.r)) wide_refresh(w, q, tau, lane);
    return fits;
}

// Item (q, rank) stopped at vectorgroup g: resume there; list q once per
// round for compaction.
__device__ __forceinline__ void wide_overflow(const WideSink &w, int64_t q, int32_t rank, int32_t g, int lane) {
    if (lane != 0) return;
    w.resume[q * w.nprobe + rank] = g;
    if (atomicExch(w.over + q, 1) == 0) {
        const int32_t at = atomicAdd(w.ocnt + w.round, 1);
        w.olist[(int64_t)(w.round & 1) * w.nq + at] = (int32_t)q;
    }
}

}  // namespace pdx
