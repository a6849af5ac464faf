// IVF search with ADSampling on PDX buckets.
//
//  1. queries rotated (k_pair DOT) and distances to every centroid (k_pair L2);
//  2. select: per query the nprobe nearest buckets, nearest first, ties by
//     bucket id (Section 2.1 IVF);
//  3. work items (query, probe rank) grouped by bucket so that the queries
//     reading one bucket run together (the bucket stays in L2 / MALL);
//  4. START (Section 4, PHASE 0): every query's nearest bucket is scanned
//     without pruning; its k-th distance becomes the query's threshold;
//  5. the other probed buckets are scanned chunk by chunk in the rotated
//     (natural) dimension order; after d < D dimensions a vector is dropped
//     when partial * D/d > tau * (1 + eps0/sqrt(d))^2 (ADSampling test of
//     Section 2.3), or with a learned error bound per (query, bucket) in
//     place of eps0,
//     at d = D when partial > tau; survivors enter the wave's k-best list,
//     whose k-th distance tightens the query's threshold;
//  6. merge of the per-item k-best lists.
#include "mlp_device.h"
#include "pdx_internal.h"
#include "wave_topk.h"
#include "wide_sink.h"

namespace pdx {
namespace {

// nprobe nearest buckets per query: bitonic sort of (distance, bucket)
// keys in LDS; also flags queries holding non-finite values.
__global__ __launch_bounds__(256) void select_probe_kernel(const float *__restrict__ cd, int32_t nlist,
                                                           int32_t pow2, const float *__restrict__ q,
                                                           int32_t d, int32_t nprobe,
                                                           int32_t *__restrict__ probe,
                                                           int32_t *__restrict__ bad,
                                                           uint32_t *__restrict__ tau) {
    extern __shared__ uint64_t key[];
    const int64_t qi = blockIdx.x;
    int nonfinite = 0;
    for (int j = threadIdx.x; j < d; j += blockDim.x) nonfinite |= !isfinite(q[qi * d + j]);
    nonfinite = __syncthreads_or(nonfinite);
    for (int l = threadIdx.x; l < pow2; l += blockDim.x) {
        uint64_t kk = kEmptyKey;
        if (l < nlist) kk = make_key(cd[qi * nlist + l], (uint32_t)l);
        key[l] = kk;
    }
    __syncthreads();
    for (int k2 = 2; k2 <= pow2; k2 <<= 1)
        for (int j2 = k2 >> 1; j2 > 0; j2 >>= 1) {
            for (int i = threadIdx.x; i < pow2; i += blockDim.x) {
                int ixj = i ^ j2;
                if (ixj > i) {
                    uint64_t a = key[i], b = key[ixj];
                    bool up = (i & k2) == 0;
                    if ((a > b) == up) {
                        key[i] = b;
                        key[ixj] = a;
                    }
                }
            }
            __syncthreads();
        }
    for (int r = threadIdx.x; r < nprobe; r += blockDim.x)
        probe[qi * nprobe + r] = (int32_t)(key[r] & 0xffffffffu);
    if (threadIdx.x == 0) {
        bad[qi] = nonfinite;
        tau[qi] = kInfBits;
    }
}

// Squared norm of each row of a [rows][d] matrix, one wave per row.
__global__ __launch_bounds__(64) void row_norm_kernel(const float *__restrict__ a, int32_t d,
                                                      float *__restrict__ out) {
    const int64_t i = blockIdx.x;
    float s = 0.0f;
    for (int32_t j = threadIdx.x; j < d; j += kWave) s = fmaf(a[i * d + j], a[i * d + j], s);
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off);
    if (threadIdx.x == 0) out[i] = s;
}

// The nprobe nearest buckets (nprobe <= 64) from the matrix-core products
// g[q][l] = q.c_l, one wave per query.  The expanded |q|^2 + |c|^2 - 2 q.c
// is within E = 2 (D + 64) 2^-24 (|q|^2 + |c|^2) of the exact distance, so
// every bucket of the exact nprobe best (ties by id) has a lower bound at
// or below T, the nprobe-th smallest upper bound: only those candidates
// get their exact f32 distance (each summed across the wave), and the
// nprobe best of them by (distance, id) are the probes.  g[q][l] then holds the exact distance
// of every candidate.  Too many candidates (near-equal centroid distances)
// or fewer than nprobe (NaN bounds): every bucket is summed exactly; a
// non-finite query gets buckets 0 .. nprobe-1 (it returns no result), so
// the probe ids are always buckets of the index.
constexpr int kProbeCand = 256;

__global__ __launch_bounds__(256) void probe_from_dot_kernel(float *__restrict__ g, int64_t nq, int32_t nlist,
                                                             const float *__restrict__ qsq,
                                                             const float *__restrict__ csq,
                                                             const float *__restrict__ qrot,
                                                             const float *__restrict__ cen,
                                                             const float *__restrict__ q, int32_t d, int32_t nprobe,
                                                             int32_t *__restrict__ probe, int32_t *__restrict__ bad,
                                                             uint32_t *__restrict__ tau) {
    __shared__ int32_t cand[4][kProbeCand];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int64_t qi = (int64_t)blockIdx.x * 4 + wave;
    if (qi >= nq) return;
    int nonfinite = 0;
    for (int32_t j = lane; j < d; j += kWave) nonfinite |= !isfinite(q[qi * d + j]);
    nonfinite = __any(nonfinite) ? 1 : 0;
    if (nonfinite) {  // no result; any real buckets keep the later kernels in bounds
        if (lane < nprobe) probe[qi * nprobe + lane] = lane;
        if (lane == 0) {
            bad[qi] = 1;
            tau[qi] = kInfBits;
        }
        return;
    }
    float *gq = g + qi * nlist;
    const float qn = qsq[qi], ef = (float)(d + 64) * 0x1p-23f;
    // T: the nprobe-th smallest upper bound
    uint64_t e = kEmptyKey, kth = kEmptyKey;
    for (int32_t l0 = 0; l0 < nlist; l0 += kWave) {
        const int32_t l = l0 + lane;
        uint64_t key = kEmptyKey;
        if (l < nlist) {
            const float nn = qn + csq[l];
            key = make_key(fmaxf(nn - 2.0f * gq[l] + ef * nn, 0.0f), (uint32_t)l);
        }
        topk_offer(e, kth, key, key != kEmptyKey, nprobe, lane);
    }
    const float T = kth == kEmptyKey ? INFINITY : key_dist(kth);
    // candidates: lower bound at or below T
    int32_t nc = 0;
    for (int32_t l0 = 0; l0 < nlist; l0 += kWave) {
        const int32_t l = l0 + lane;
        bool in = false;
        if (l < nlist) {
            const float nn = qn + csq[l];
            in = nn - 2.0f * gq[l] - ef * nn <= T;
        }
        const unsigned long long m = __ballot(in);
        const int at = nc + (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
        if (in && at < kProbeCand) cand[wave][at] = l;
        nc += __popcll(m);
    }
    // too many candidates, or too few (NaN bounds compare false): every
    // bucket exactly, so the probes are always real buckets
    const bool all = nc > kProbeCand || nc < nprobe;
    const int32_t ncand = all ? nlist : nc;
    // exact distances of the candidates, four at a time across the wave
    // (lane j sums dimensions j, j + 64, ...; the lane sums then reduced)
    const float *qp = qrot + qi * d;
    e = kth = kEmptyKey;
    for (int32_t i0 = 0; i0 < ncand; i0 += 4) {
        int32_t lc[4];
        float acc[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int32_t i = min(i0 + u, ncand - 1);
            lc[u] = all ? i : cand[wave][i];
            acc[u] = 0.0f;
        }
        for (int32_t j = lane; j < d; j += kWave) {
            const float qv = qp[j];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const float dd = qv - cen[(int64_t)lc[u] * d + j];
                acc[u] = fmaf(dd, dd, acc[u]);
            }
        }
        float mine = 0.0f;
#pragma unroll
        for (int u = 0; u < 4; ++u) {
#pragma unroll
            for (int off = 32; off > 0; off >>= 1) acc[u] += __shfl_xor(acc[u], off);
            if (lane == u) mine = acc[u];
        }
        const bool ok = lane < 4 && i0 + lane < ncand;
        int32_t myl = lc[0];
#pragma unroll
        for (int u = 1; u < 4; ++u) myl = lane == u ? lc[u] : myl;
        if (ok) gq[myl] = mine;
        topk_offer(e, kth, make_key(mine, (uint32_t)myl), ok, nprobe, lane);
    }
    if (lane < nprobe) probe[qi * nprobe + lane] = e != kEmptyKey ? (int32_t)(e & 0xffffffffu) : lane;
    if (lane == 0) {
        bad[qi] = 0;
        tau[qi] = kInfBits;
    }
}

// items per bucket: count, padded exclusive prefix, scatter (START items
// r = 0 and the other ranks r >= 1 in two separate lists).  Only ranks in
// [rlo, rhi) below the query's budget (if any) become items.
__device__ __forceinline__ bool item_wanted(int32_t r, int32_t rlo, int32_t rhi, const int32_t *budget,
                                            int64_t qi) {
    return r >= rlo && r < rhi && !(budget && r >= budget[qi]);
}

__global__ void item_count_kernel(const int32_t *__restrict__ probe, int64_t nq, int32_t nprobe, int32_t rlo,
                                  int32_t rhi, const int32_t *__restrict__ budget, int32_t *__restrict__ cnt0,
                                  int32_t *__restrict__ cnt1) {
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= nq * nprobe) return;
    int32_t r = (int32_t)(i % nprobe);
    if (!item_wanted(r, rlo, rhi, budget, i / nprobe)) return;
    atomicAdd((r == 0 ? cnt0 : cnt1) + probe[i], 1);
}

// Cursor where each bucket's items start, per count array (block b of the
// grid: cnt[b]).  A bucket's item count is rounded up to a
// multiple of qb so that every batch of qb consecutive items belongs to one
// bucket (the rounding slots stay padding, query id -1).  Buckets are laid
// out by id, or larger first so their long batches start early and the
// launch drains evenly; keys (size descending, id) are sorted in LDS.
// With xcd (non-null, 9 entries), the buckets are dealt to
// the 8 XCDs round-robin in that order and laid out XCD by XCD; xcd[x] is
// the first item of XCD x's range and xcd[8] the end, so a scan can keep
// every batch of a bucket on one XCD (one L2).
__global__ __launch_bounds__(1024) void batch_prefix_kernel(int32_t *__restrict__ cnt0, int32_t qb0,
                                                            int32_t *__restrict__ xcd0, int32_t *__restrict__ cnt1,
                                                            int32_t qb1, int32_t *__restrict__ xcd1, int32_t nlist,
                                                            int32_t pow2, const int32_t *__restrict__ list_size,
                                                            int32_t by_size) {
    extern __shared__ uint64_t order[];  // pow2 keys, then (xcd layout) nlist bucket ids
    __shared__ int32_t part[1024];
    __shared__ int32_t carry;
    int32_t *cnt = blockIdx.x == 0 ? cnt0 : cnt1;
    const int32_t qb = blockIdx.x == 0 ? qb0 : qb1;
    int32_t *xcd = blockIdx.x == 0 ? xcd0 : xcd1;
    int32_t *lay = reinterpret_cast<int32_t *>(order + pow2);
    for (int32_t l = threadIdx.x; l < pow2; l += blockDim.x) {
        uint64_t key = kEmptyKey;
        if (l < nlist)
            key = by_size ? (static_cast<uint64_t>(0x7fffffffu - static_cast<uint32_t>(list_size[l])) << 32) | (uint32_t)l
                          : (uint64_t)l;
        order[l] = key;
    }
    if (threadIdx.x == 0) carry = 0;
    __syncthreads();
    if (by_size)
        for (int k2 = 2; k2 <= pow2; k2 <<= 1)
            for (int j2 = k2 >> 1; j2 > 0; j2 >>= 1) {
                for (int i = threadIdx.x; i < pow2; i += blockDim.x) {
                    int ixj = i ^ j2;
                    if (ixj > i) {
                        uint64_t a = order[i], b = order[ixj];
                        bool up = (i & k2) == 0;
                        if ((a > b) == up) {
                            order[i] = b;
                            order[ixj] = a;
                        }
                    }
                }
                __syncthreads();
            }
    // bucket at layout position i
    auto base_of = [&](int32_t x) {  // first layout position of XCD x: sum of the earlier XCDs' shares
        int32_t b = 0;
        for (int32_t y = 0; y < x; ++y) b += (nlist - y + 7) / 8;
        return b;
    };
    if (xcd) {
        for (int32_t p = threadIdx.x; p < nlist; p += blockDim.x)
            lay[base_of(p & 7) + (p >> 3)] = (int32_t)(order[p] & 0xffffffffu);
        __syncthreads();
    }
    for (int32_t i0 = 0; i0 < nlist; i0 += 1024) {
        const int32_t i = i0 + threadIdx.x;
        const int32_t l = i < nlist ? (xcd ? lay[i] : (int32_t)(order[i] & 0xffffffffu)) : -1;
        const int32_t c = l >= 0 ? (cnt[l] + qb - 1) / qb * qb : 0;
        part[threadIdx.x] = c;
        __syncthreads();
        for (int off = 1; off < 1024; off <<= 1) {
            int32_t t = threadIdx.x >= off ? part[threadIdx.x - off] : 0;
            __syncthreads();
            part[threadIdx.x] += t;
            __syncthreads();
        }
        if (l >= 0) cnt[l] = carry + part[threadIdx.x] - c;
        __syncthreads();
        if (threadIdx.x == 1023) carry += part[1023];
        __syncthreads();
    }
    if (xcd && threadIdx.x < 9) {
        const int32_t b = base_of(threadIdx.x);
        xcd[threadIdx.x] = (threadIdx.x < 8 && b < nlist) ? cnt[lay[b]] : carry;
    }
}

__global__ void item_scatter_kernel(const int32_t *__restrict__ probe, int64_t nq, int32_t nprobe, int32_t rlo,
                                    int32_t rhi, const int32_t *__restrict__ budget, int32_t *__restrict__ cur0,
                                    int32_t *__restrict__ cur1, int2 *__restrict__ items0,
                                    int2 *__restrict__ items1) {
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= nq * nprobe) return;
    int32_t r = (int32_t)(i % nprobe);
    int32_t qi = (int32_t)(i / nprobe);
    if (!item_wanted(r, rlo, rhi, budget, qi)) return;
    int32_t l = probe[i];
    if (r == 0) items0[atomicAdd(cur0 + l, 1)] = make_int2(qi, r);
    else items1[atomicAdd(cur1 + l, 1)] = make_int2(qi, r);
}

// Value of dimension j of the lane's vector in group g: f32, or a bfloat16 /
// e4m3 code decoded to f32 (e4m3 times the dimension's scale).
template <int STORE>
__device__ __forceinline__ float load_val(const void *__restrict__ data, const float *__restrict__ scale, int64_t at,
                                          int32_t j) {
    if (STORE == PDX_DTYPE_F32) return static_cast<const float *>(data)[at];
    if (STORE == PDX_DTYPE_BF16) return bf16_decode(static_cast<const uint16_t *>(data)[at]);
    return e4m3_decode(static_cast<const uint8_t *>(data)[at]) * scale[j];
}

// One (query, probe rank) item from vectorgroup g0 of its bucket (-1: the
// first) for one wave: the running k-best list written to the item's slot,
// or (WIDE) the survivors appended to the query's candidate buffer.
template <bool PRUNE, int STORE, bool WIDE>
__device__ __forceinline__ void scan_item(const void *__restrict__ pdxd, const float *__restrict__ scale, int32_t d,
                                          const int32_t *__restrict__ slot_id, const int32_t *__restrict__ goff,
                                          int64_t qi, int32_t r, int32_t g0, const int32_t *__restrict__ probe,
                                          int32_t nprobe, const float *__restrict__ qrot, uint32_t *__restrict__ tau,
                                          const int32_t *__restrict__ bad, const SlotMap &slots, int32_t chunk,
                                          const PruneRule &rule, unsigned long long *__restrict__ counters,
                                          const WideSink &wide, int lane) {
    const int32_t k = slots.kk;
    if (bad[qi]) {  // non-finite query
        if (!WIDE && lane < k) slots.at(qi, r, 0)[lane] = kEmptyKey;
        return;
    }
    const int32_t l = probe[qi * nprobe + r];
    const float *qp = qrot + qi * d;
    const float eps_i = (PRUNE && rule.eps) ? rule.eps_at(qi, r, nprobe) : 0.0f;
    const int32_t hb = WIDE ? wide.hbase[qi] : 0;
    uint64_t e = kEmptyKey, kth = kEmptyKey;
    unsigned long long live_vals = 0, lane_vals = 0;
    for (int32_t g = g0 >= 0 ? g0 : goff[l]; g < goff[l + 1]; ++g) {
        float tau_eff = INFINITY;
        if (PRUNE || WIDE) {
            uint32_t tg = __hip_atomic_load(tau + qi, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            float tl = (WIDE || kth == kEmptyKey) ? INFINITY : key_dist(kth);
            tau_eff = fminf(__uint_as_float(tg), tl);
        }
        const int32_t vid = slot_id[(int64_t)g * kGroup + lane];
        bool alive = vid >= 0;
        const int64_t gbase = (int64_t)g * d * kGroup + lane;
        float partial = 0.0f;
        for (int32_t c0 = 0; c0 < d; c0 += chunk) {
            if (PRUNE && !__any(alive)) break;
            const int32_t c1 = min(c0 + chunk, d);
            if (counters) {
                live_vals += (unsigned long long)__popcll(__ballot(alive)) * (c1 - c0);
                lane_vals += 64ull * (c1 - c0);
            }
            float s = 0.0f;
            if (alive) {
                int32_t j = c0;
                for (; j + 8 <= c1; j += 8) {
                    float x[8];
#pragma unroll
                    for (int u = 0; u < 8; ++u) x[u] = load_val<STORE>(pdxd, scale, gbase + (int64_t)(j + u) * kGroup, j + u);
#pragma unroll
                    for (int u = 0; u < 8; ++u) {
                        float t = qp[j + u] - x[u];
                        s = fmaf(t, t, s);
                    }
                }
                for (; j < c1; ++j) {
                    float t = qp[j] - load_val<STORE>(pdxd, scale, gbase + (int64_t)j * kGroup, j);
                    s = fmaf(t, t, s);
                }
            }
            partial += s;
            if (PRUNE) {
                // the prune test after c1 of d dimensions (exact at c1 = d)
                if (rule.xres && c1 < d) {  // BSA: the stored residual norms of the test point
                    const int32_t tp = c0 / chunk;
                    const float xr = rule.xres[((int64_t)g * rule.ntp + tp) * kGroup + lane];
                    alive = alive && !rule.bsa_drop(partial, tau_eff, rule.qres[qi * rule.ntp + tp], xr);
                } else {
                    float thr = tau_eff;
                    if (c1 < d)
                        thr = tau_eff * (rule.eps ? PruneRule::learned(eps_i, (float)c1 / (float)d, prune_rs(c1))
                                                  : rule.ads(c1, d));
                    alive = alive && !(partial > thr);
                }
            }
        }
        if constexpr (WIDE) {
            if (!wide_push(wide, qi, partial, (uint32_t)vid, alive && partial < tau_eff, hb, tau, lane)) {
                wide_overflow(wide, qi, r, g, lane);
                break;
            }
        } else {
            topk_offer(e, kth, make_key(partial, (uint32_t)vid), alive, k, lane);
            if (PRUNE && kth != kEmptyKey) {
                float kt = key_dist(kth);
                if (kt < tau_eff && lane == 0) atomicMin(tau + qi, __float_as_uint(kt));
            }
        }
    }
    if (!WIDE && lane < k) slots.at(qi, r, 0)[lane] = e;
    if (counters && lane == 0) {
        atomicAdd(counters, live_vals);
        atomicAdd(counters + 1, lane_vals);
    }
}

// Scan of one bucket for one query per wave.  Work items are consecutive
// per bucket; workgroup ids are mapped so each XCD takes a contiguous
// range of items (and so of buckets).
template <bool PRUNE, int STORE, bool WIDE>
__global__ __launch_bounds__(256) void ivf_scan_kernel(
    const void *__restrict__ pdxd, const float *__restrict__ scale, int32_t d, const int32_t *__restrict__ slot_id,
    const int32_t *__restrict__ goff, const int2 *__restrict__ items, int64_t nitems,
    const int32_t *__restrict__ probe, int32_t nprobe, const float *__restrict__ qrot,
    uint32_t *__restrict__ tau, const int32_t *__restrict__ bad, SlotMap slots, int32_t chunk, PruneRule rule,
    unsigned long long *__restrict__ counters, uint32_t nwg, WideSink wide) {
    // grid = 8 * ceil(nwg / 8): every (xcd, index) pair is launched once
    const uint32_t per_xcd = gridDim.x >> 3;
    const uint32_t wg = (blockIdx.x & 7) * per_xcd + (blockIdx.x >> 3);
    const int32_t wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    const int64_t it = (int64_t)wg * 4 + wave;
    if (wg >= nwg || it >= nitems) return;
    const int2 item = items[it];
    scan_item<PRUNE, STORE, WIDE>(pdxd, scale, d, slot_id, goff, item.x, item.y, -1, probe, nprobe, qrot, tau, bad,
                                  slots, chunk, rule, counters, wide, lane);
}

// Resumes the items of the queries listed in round `list_round` whose
// candidate buffer filled up (after their compaction): one item per wave,
// grid-strided; START items (rank 0) unpruned.
template <int STORE>
__global__ __launch_bounds__(256) void ivf_wide_resume_kernel(
    const void *__restrict__ pdxd, const float *__restrict__ scale, int32_t d, const int32_t *__restrict__ slot_id,
    const int32_t *__restrict__ goff, const int32_t *__restrict__ probe, int32_t nprobe,
    const float *__restrict__ qrot, uint32_t *__restrict__ tau, const int32_t *__restrict__ bad, SlotMap slots,
    int32_t chunk, PruneRule rule, unsigned long long *__restrict__ counters, WideSink wide, int32_t list_round) {
    const int lane = threadIdx.x & 63;
    const int64_t nitems = (int64_t)wide.ocnt[list_round] * nprobe;
    const int32_t *list = wide.olist + (int64_t)(list_round & 1) * wide.nq;
    for (int64_t it = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6); it < nitems; it += (int64_t)gridDim.x * 4) {
        const int64_t qi = list[it / nprobe];
        const int32_t r = (int32_t)(it % nprobe);
        const int32_t g0 = wide.resume[qi * nprobe + r];
        if (g0 < 0) continue;
        if (lane == 0) wide.resume[qi * nprobe + r] = -1;
        if (r == 0)
            scan_item<false, STORE, true>(pdxd, scale, d, slot_id, goff, qi, r, g0, probe, nprobe, qrot, tau, bad,
                                          slots, chunk, rule, counters, wide, lane);
        else
            scan_item<true, STORE, true>(pdxd, scale, d, slot_id, goff, qi, r, g0, probe, nprobe, qrot, tau, bad,
                                         slots, chunk, rule, counters, wide, lane);
    }
}

// Scan of one bucket for a batch of QB queries per wave (the batch's
// items are QB consecutive slots of one bucket; padding slots have query
// id -1).  Lane = vector of the current vectorgroup; each value loaded
// (and decoded) once serves all queries of the batch.  Per query and lane:
// partial distance, alive bit, and the query's own k-best list; a query
// with no alive lane in the group skips its arithmetic (wave-uniform
// branch), and the group ends early once no (query, lane) pair is alive.
// Summation per (query, vector): each chunk summed sequentially, then
// added to the partial, as in the one-query kernel.  WIDE: survivors go to
// the queries' candidate buffers; a query whose buffer fills leaves the
// batch (its item resumes later).
template <bool PRUNE, int STORE, int QB, bool WIDE>
__global__ __launch_bounds__(256) void ivf_bscan_kernel(
    const void *__restrict__ pdxd, const float *__restrict__ scale, int32_t d, const int32_t *__restrict__ slot_id,
    const int32_t *__restrict__ goff, const int2 *__restrict__ items, int64_t nbatch,
    const int32_t *__restrict__ probe, int32_t nprobe, const float *__restrict__ qrot,
    uint32_t *__restrict__ tau, const int32_t *__restrict__ bad, SlotMap slots, int32_t chunk, PruneRule rule,
    unsigned long long *__restrict__ counters, WideSink wide) {
    const int lane = threadIdx.x & 63;
    const int32_t k = slots.kk;
    const int64_t b = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (b >= nbatch) return;
    const int2 mine = lane < QB ? items[b * QB + lane] : make_int2(-1, 0);
    int32_t qid[QB], rk[QB];
#pragma unroll
    for (int q = 0; q < QB; ++q) {
        qid[q] = __builtin_amdgcn_readlane(mine.x, q);
        rk[q] = __builtin_amdgcn_readlane(mine.y, q);
    }
    if (qid[0] < 0) return;  // a batch starts with a real item unless it is unused capacity
    const int32_t l = probe[(int64_t)qid[0] * nprobe + rk[0]];
    uint32_t use = 0;
#pragma unroll
    for (int q = 0; q < QB; ++q) {
        if (qid[q] < 0) continue;
        if (bad[qid[q]]) {  // non-finite query
            if (!WIDE && lane < k) slots.at(qid[q], rk[q], 0)[lane] = kEmptyKey;
        } else {
            use |= 1u << q;
        }
    }
    if (!use) return;
    float epsq[QB];  // learned bound of each query's item
#pragma unroll
    for (int q = 0; q < QB; ++q)
        epsq[q] = (PRUNE && rule.eps && ((use >> q) & 1u)) ? rule.eps_at(qid[q], rk[q], nprobe) : 0.0f;
    uint64_t e[QB], kth[QB];
    float part[QB], s[QB];
#pragma unroll
    for (int q = 0; q < QB; ++q) e[q] = kth[q] = kEmptyKey;
    unsigned long long live_vals = 0, lane_vals = 0;
    for (int32_t g = goff[l]; g < goff[l + 1]; ++g) {
        float teff[QB];
#pragma unroll
        for (int q = 0; q < QB; ++q) {
            teff[q] = INFINITY;
            if ((PRUNE || WIDE) && ((use >> q) & 1)) {
                uint32_t tg = __hip_atomic_load(tau + qid[q], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                float tl = (WIDE || kth[q] == kEmptyKey) ? INFINITY : key_dist(kth[q]);
                teff[q] = fminf(__uint_as_float(tg), tl);
            }
            part[q] = 0.0f;
        }
        const int32_t vid = slot_id[(int64_t)g * kGroup + lane];
        uint32_t am = vid >= 0 ? use : 0u;  // bit q: lane alive for query q
        uint32_t qa = use;                  // wave-uniform: queries with an alive lane
        const int64_t gbase = (int64_t)g * d * kGroup + lane;
        for (int32_t c0 = 0; c0 < d; c0 += chunk) {
            if (PRUNE) {
                qa = 0;
#pragma unroll
                for (int q = 0; q < QB; ++q) qa |= (__ballot((am >> q) & 1u) != 0ull ? 1u : 0u) << q;
                if (!qa) break;
            }
            const int32_t c1 = min(c0 + chunk, d);
            if (counters) {
#pragma unroll
                for (int q = 0; q < QB; ++q)
                    if ((qa >> q) & 1u) {
                        live_vals += (unsigned long long)__popcll(__ballot((am >> q) & 1u)) * (c1 - c0);
                        lane_vals += 64ull * (c1 - c0);
                    }
            }
#pragma unroll
            for (int q = 0; q < QB; ++q) s[q] = 0.0f;
            int32_t j = c0;
            for (; j + 8 <= c1; j += 8) {
                float x[8];
#pragma unroll
                for (int u = 0; u < 8; ++u) x[u] = load_val<STORE>(pdxd, scale, gbase + (int64_t)(j + u) * kGroup, j + u);
#pragma unroll
                for (int q = 0; q < QB; ++q) {
                    if ((qa >> q) & 1u) {
                        const float *qp = qrot + (int64_t)qid[q] * d + j;
#pragma unroll
                        for (int u = 0; u < 8; ++u) {
                            float t = qp[u] - x[u];
                            s[q] = fmaf(t, t, s[q]);
                        }
                    }
                }
            }
            for (; j < c1; ++j) {
                const float x = load_val<STORE>(pdxd, scale, gbase + (int64_t)j * kGroup, j);
#pragma unroll
                for (int q = 0; q < QB; ++q) {
                    if ((qa >> q) & 1u) {
                        float t = qrot[(int64_t)qid[q] * d + j] - x;
                        s[q] = fmaf(t, t, s[q]);
                    }
                }
            }
            float fac = 1.0f, cdl = 0.0f, rsl = 0.0f, xr = 0.0f;
            const bool bsa = PRUNE && c1 < d && rule.xres;
            const bool learned = PRUNE && c1 < d && rule.eps && !bsa;
            if (PRUNE && c1 < d && !rule.eps && !bsa) fac = rule.ads(c1, d);
            if (learned) {
                cdl = (float)c1 / (float)d;
                rsl = prune_rs(c1);
            }
            if (bsa) xr = rule.xres[((int64_t)g * rule.ntp + c0 / chunk) * kGroup + lane];
#pragma unroll
            for (int q = 0; q < QB; ++q) {
                if ((qa >> q) & 1u) {
                    part[q] += s[q];
                    // the prune test after c1 of d dimensions (exact at c1 = d)
                    if (bsa) {
                        if (rule.bsa_drop(part[q], teff[q], rule.qres[(int64_t)qid[q] * rule.ntp + c0 / chunk], xr))
                            am &= ~(1u << q);
                    } else {
                        const float fq = learned ? PruneRule::learned(epsq[q], cdl, rsl) : fac;
                        if (PRUNE && part[q] > teff[q] * fq) am &= ~(1u << q);
                    }
                }
            }
        }
#pragma unroll
        for (int q = 0; q < QB; ++q) {
            if (!((use >> q) & 1u)) continue;
            const bool cand = (am >> q) & 1u;
            if constexpr (WIDE) {
                if (!wide_push(wide, qid[q], part[q], (uint32_t)vid, cand && part[q] < teff[q], wide.hbase[qid[q]],
                               tau, lane)) {
                    wide_overflow(wide, qid[q], rk[q], g, lane);
                    use &= ~(1u << q);
                }
            } else {
                if (__ballot(cand)) topk_offer(e[q], kth[q], make_key(part[q], (uint32_t)vid), cand, k, lane);
                if (PRUNE && kth[q] != kEmptyKey) {
                    const float kt = key_dist(kth[q]);
                    if (kt < teff[q] && lane == 0) atomicMin(tau + qid[q], __float_as_uint(kt));
                }
            }
        }
        if (WIDE && !use) break;
    }
#pragma unroll
    for (int q = 0; q < QB; ++q)
        if (!WIDE && ((use >> q) & 1u) && lane < k) slots.at(qid[q], rk[q], 0)[lane] = e[q];
    if (counters && lane == 0) {
        atomicAdd(counters, live_vals);
        atomicAdd(counters + 1, lane_vals);
    }
}

// Learned probe budget, after START: for r = 1 .. nprobe-1 the network's
// inputs (documented with pdx_mlp_* in include/pdx.h) for "stop after r
// buckets", tau being the k-th distance of the START bucket; the query
// probes the smallest r whose logit exceeds zthr (else all nprobe).  With
// trace_f, every r's inputs are recorded ([nq][nprobe][72], row r - 1; the
// last row zero) and no budget is set.
__global__ __launch_bounds__(64) void budget_kernel(const float *__restrict__ qrot, int32_t d,
                                                    const float *__restrict__ cd, int32_t nlist,
                                                    const int32_t *__restrict__ probe, int32_t nprobe,
                                                    const uint32_t *__restrict__ tau, const int32_t *__restrict__ bad,
                                                    const __half *__restrict__ w16, float zthr,
                                                    int32_t *__restrict__ budget, float *__restrict__ trace_f) {
    __shared__ float feat[kMlpIn];
    const int64_t qi = blockIdx.x;
    const int lane = threadIdx.x;
    const float *cq = cd + qi * nlist;
    const int32_t *pq = probe + qi * nprobe;
    const float t = __uint_as_float(tau[qi]);
    const float d0 = cq[pq[0]] + 1e-20f;
    const float dl = cq[pq[nprobe - 1]] + 1e-20f;
    auto clampr = [](float v) { return fminf(fmaxf(v, 0.0f), 1.0e4f); };
    feat[lane] = lane < d ? qrot[qi * d + lane] : 0.0f;
    const bool decide = w16 && !trace_f && !bad[qi];
    int32_t chosen = nprobe;
    for (int32_t r = 1; r < nprobe; ++r) {
        const float dr = cq[pq[r]] + 1e-20f;
        if (lane < kMlpIn - 64) {
            float v = 0.0f;
            if (lane == 0) v = clampr(t / dr);
            else if (lane == 1) v = clampr(dr / d0);
            else if (lane == 2) v = clampr(dl / d0);
            else if (lane == 3) v = clampr(t / d0);
            else if (lane == 4) v = log2f((float)r) / log2f((float)nprobe);
            feat[64 + lane] = v;
        }
        __syncthreads();
        if (trace_f)
            for (int i = lane; i < kMlpIn; i += 64) trace_f[(qi * nprobe + (r - 1)) * kMlpIn + i] = feat[i];
        if (decide) {
            const float z = mlp_forward_wave(w16, feat, lane, nullptr, nullptr, nullptr, nullptr);
            if (z > zthr) {  // z is the same in every lane
                chosen = r;
                break;
            }
        }
        __syncthreads();
    }
    if (trace_f)
        for (int i = lane; i < kMlpIn; i += 64) trace_f[(qi * nprobe + (nprobe - 1)) * kMlpIn + i] = 0.0f;
    if (decide && lane == 0) budget[qi] = chosen;
}

// Buckets a query needed: 1 + the largest probe rank among the buckets of
// its final ids (0 when it has none); stopping after r buckets loses
// nothing of the result exactly when r >= this.
__global__ __launch_bounds__(64) void need_kernel(const int64_t *__restrict__ ids, int32_t k,
                                                  const int32_t *__restrict__ assign,
                                                  const int32_t *__restrict__ probe, int32_t nprobe,
                                                  int32_t *__restrict__ need) {
    const int64_t qi = blockIdx.x;
    const int lane = threadIdx.x;
    int32_t mine = 0;
    if (lane < k) {
        const int64_t id = ids[qi * k + lane];
        if (id >= 0) {
            const int32_t l = assign[id];
            for (int32_t r = 0; r < nprobe; ++r)
                if (probe[qi * nprobe + r] == l) {
                    mine = r + 1;
                    break;
                }
        }
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) mine = max(mine, __shfl_xor(mine, off));
    if (lane == 0) need[qi] = mine;
}

// Inputs 64 .. 71 of the prune network for the bucket of probe rank
// r >= 1 (inputs 0 .. 63: the rotated query's first coordinates); the same
// in every lane.
__device__ __forceinline__ void prune_inputs(float t, float d0, float dr, int32_t r, int32_t nprobe,
                                             float (&x)[8]) {
    auto clampr = [](float v) { return fminf(fmaxf(v, 0.0f), 1.0e4f); };
    x[0] = clampr(t / dr);
    x[1] = clampr(dr / d0);
    x[2] = clampr(t / d0);
    x[3] = log2f((float)r) / log2f((float)nprobe);
    x[4] = x[5] = x[6] = x[7] = 0.0f;
}

// Learned prune bounds after START: one wave per (query, rank r >= 1)
// evaluates the network once: eps = scale * z; table (optional) receives
// the multiplier prune_mult(eps, c1) of every test point c (c1 = (c + 1)
// chunk < d).  Also records the START threshold in tau0.  Non-finite
// queries are not scanned: their rows hold NaN in `table`.
__global__ __launch_bounds__(256) void prune_table_kernel(
    const float *__restrict__ qrot, int32_t d, const float *__restrict__ cd, int32_t nlist,
    const int32_t *__restrict__ probe, int32_t nprobe, const uint32_t *__restrict__ tau,
    const int32_t *__restrict__ bad, const __half *__restrict__ w16, float scale, int32_t chunk, int32_t npt,
    int64_t npairs, float *__restrict__ epsq, float *__restrict__ table, float *__restrict__ tau0) {
    __shared__ float feat[4][kMlpIn];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int64_t pr = (int64_t)blockIdx.x * 4 + wave;
    if (pr >= npairs) return;
    const int64_t qi = pr / (nprobe - 1);
    const int32_t r = (int32_t)(pr - qi * (nprobe - 1)) + 1;
    const float t = __uint_as_float(tau[qi]);
    if (tau0 && r == 1 && lane == 0) tau0[qi] = t;
    if (!w16) return;
    const size_t row = (size_t)pr * npt;
    if (bad[qi]) {
        if (table)
            for (int32_t c = lane; c < npt; c += 64) table[row + c] = __uint_as_float(0x7fc00000u);
        return;
    }
    const float *cq = cd + qi * nlist;
    const int32_t *pq = probe + qi * nprobe;
    float x[8];
    prune_inputs(t, cq[pq[0]] + 1e-20f, cq[pq[r]] + 1e-20f, r, nprobe, x);
    feat[wave][lane] = lane < d ? qrot[qi * d + lane] : 0.0f;
    float mine = 0.0f;
#pragma unroll
    for (int i = 0; i < 8; ++i) mine = lane == i ? x[i] : mine;
    if (lane < kMlpIn - 64) feat[wave][64 + lane] = mine;
    // the wave's own LDS row: a wavefront-scope hand-off between its lanes
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    const float eps = scale * mlp_forward_wave(w16, feat[wave], lane, nullptr, nullptr, nullptr, nullptr);
    if (lane == 0) epsq[pr] = eps;
    if (table)
        for (int32_t c = lane; c < npt; c += 64) table[row + c] = prune_mult(eps, prune_rs((c + 1) * chunk));
}

// Training traces of the prune network, after the result is known: one
// wave per (query, result slot i).  Target: the smallest error bound that
// keeps the i-th id at every test point, max over c of
// (sqrt(partial(c1) D / (c1 tau_k)) - 1) sqrt(c1), with partial(c1) its
// squared distance over the first c1 rotated dimensions and tau_k the
// result's k-th distance; inputs: those of (query, rank of the id's bucket)
// with the START threshold tau0.  No sample (target NaN, inputs 0): no id,
// an id of the START bucket, tau_k not positive and finite, a non-finite
// query.
__global__ __launch_bounds__(256) void prune_trace_kernel(
    const int64_t *__restrict__ ids, const float *__restrict__ dist, int32_t k, const int32_t *__restrict__ assign,
    const float *__restrict__ xrow, const float *__restrict__ qrot, int32_t d, const float *__restrict__ cd,
    int32_t nlist, const int32_t *__restrict__ probe, int32_t nprobe, const float *__restrict__ tau0,
    const int32_t *__restrict__ bad, int32_t chunk, int32_t npt, int64_t nslots, float *__restrict__ feat_out,
    float *__restrict__ target_out) {
    const int lane = threadIdx.x & 63;
    const int64_t si = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (si >= nslots) return;
    const int64_t qi = si / k;
    const int64_t id = ids[si];
    const float tk = dist[qi * k + (k - 1)];
    bool ok = !bad[qi] && id >= 0 && tk > 0.0f && tk < INFINITY;
    int32_t r = -1;
    if (ok) {
        const int32_t l = assign[id];
        for (int32_t r0 = 0; r0 < nprobe && r < 0; r0 += 64) {
            const unsigned long long hit = __ballot(r0 + lane < nprobe && probe[qi * nprobe + r0 + lane] == l);
            if (hit) r = r0 + __builtin_ctzll(hit);
        }
        ok = r >= 1;
    }
    float *fo = feat_out + (size_t)si * kMlpIn;
    if (!ok) {
        fo[lane] = 0.0f;
        if (lane < kMlpIn - 64) fo[64 + lane] = 0.0f;
        if (lane == 0) target_out[si] = __uint_as_float(0x7fc00000u);
        return;
    }
    const float *cq = cd + qi * nlist;
    const int32_t *pq = probe + qi * nprobe;
    float x[8];
    prune_inputs(tau0[qi], cq[pq[0]] + 1e-20f, cq[pq[r]] + 1e-20f, r, nprobe, x);
    float mine = 0.0f;
#pragma unroll
    for (int i = 0; i < 8; ++i) mine = lane == i ? x[i] : mine;
    fo[lane] = lane < d ? qrot[qi * d + lane] : 0.0f;
    if (lane < kMlpIn - 64) fo[64 + lane] = mine;
    const float *xv = xrow + id * d, *qp = qrot + qi * d;
    float partial = 0.0f, need = -INFINITY;
    for (int32_t c = 0; c < npt; ++c) {
        const int32_t c0 = c * chunk, c1 = c0 + chunk;
        float sum = 0.0f;
        for (int32_t j = c0 + lane; j < c1; j += 64) {
            const float t = xv[j] - qp[j];
            sum = fmaf(t, t, sum);
        }
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) sum += __shfl_xor(sum, off);
        partial += sum;
        const float sc = sqrtf((float)c1);
        need = fmaxf(need, (sqrtf(partial * (float)d / ((float)c1 * tk)) - 1.0f) * sc);
    }
    if (lane == 0) target_out[si] = need;
}

// k-best over a query's item lists: the START lists (if use0) and the lists
// of ranks 1 .. r1-1 (cut at the query's learned budget, if any); optional
// threshold / result / keys.  Each run of lists is contiguous per query.
__global__ __launch_bounds__(64) void ivf_merge_kernel(SlotMap s0, bool use0, SlotMap s1, int32_t r1,
                                                       const int32_t *__restrict__ budget, int32_t k,
                                                       const int32_t *__restrict__ bad,
                                                       uint32_t *__restrict__ tau,
                                                       int64_t *__restrict__ out_ids,
                                                       float *__restrict__ out_dist, uint64_t *__restrict__ keys_out) {
    const int64_t qi = blockIdx.x;
    const int lane = threadIdx.x;
    if (budget) r1 = min(r1, budget[qi]);  // ranks at or past the budget were not scanned
    uint64_t e = kEmptyKey, kth = kEmptyKey;
    for (int run = 0; run < 2; ++run) {
        const uint64_t *base = run == 0 ? s0.at(qi, 0, 0) : s1.at(qi, 1, 0);
        const int64_t total = run == 0 ? (use0 ? (int64_t)s0.parts * s0.kk : 0)
                                       : (r1 > 1 ? (int64_t)(r1 - 1) * s1.parts * s1.kk : 0);
        for (int64_t i0 = 0; i0 < total; i0 += kWave) {
            uint64_t kk = (i0 + lane < total) ? base[i0 + lane] : kEmptyKey;
            topk_offer(e, kth, kk, kk != kEmptyKey, k, lane);
        }
    }
    if (tau && lane == 0 && kth != kEmptyKey) tau[qi] = (uint32_t)(kth >> 32);
    if (keys_out && lane < k) keys_out[qi * k + lane] = e;
    if (out_ids && lane < k) {
        int64_t id = -1;
        float dist = INFINITY;
        if (bad[qi]) {
            dist = __uint_as_float(0x7fc00000u);
        } else if (e != kEmptyKey) {
            id = (int64_t)(e & 0xffffffffu);
            dist = key_dist(e);
        }
        out_ids[qi * k + lane] = id;
        out_dist[qi * k + lane] = dist;
    }
}

// Exact f32 distances of a query's r candidates (keys [nq][r], ordered by
// the scanned distance) from the row-major rotated rows, then the k best by
// (exact distance, id).  The summation order is the vector scans' (each
// chunk of `chunk` dimensions summed sequentially, the chunk sums added in
// order), so every engine reports the same distance for a vector.  One
// wave per query: lane c sums chunk c of 4 candidates at a time (loads
// issued 8 dimensions ahead), then the chunk sums are added in order.
__global__ __launch_bounds__(256) void rerank_kernel(const uint64_t *__restrict__ keys, int32_t r, int32_t k,
                                                     const float *__restrict__ xrow, const float *__restrict__ qrot,
                                                     int32_t d, int32_t chunk, const int32_t *__restrict__ bad,
                                                     int64_t nq, int64_t *__restrict__ out_ids,
                                                     float *__restrict__ out_dist) {
    constexpr int U = 4;  // candidates in flight
    const int64_t qi = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (qi >= nq) return;
    const float *qp = qrot + qi * d;
    const int32_t nch = (d + chunk - 1) / chunk;
    uint64_t mine = kEmptyKey;
    for (int32_t i0 = 0; i0 < r; i0 += U) {
        uint64_t key[U];
        const float *x[U];
        float partial[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            key[u] = i0 + u < r ? keys[qi * r + i0 + u] : kEmptyKey;
            // an empty key reads row 0, whose sum is discarded
            x[u] = xrow + (key[u] == kEmptyKey ? 0 : (int64_t)(key[u] & 0xffffffffu) * d);
            partial[u] = 0.0f;
        }
        if (key[0] == kEmptyKey) break;  // the list is sorted: the rest is empty too
        for (int32_t base = 0; base < nch; base += 64) {
            float s[U];
#pragma unroll
            for (int u = 0; u < U; ++u) s[u] = 0.0f;
            const int32_t c = base + lane;
            if (c < nch) {
                const int32_t j1 = min((c + 1) * chunk, d);
                int32_t j = c * chunk;
                for (; j + 8 <= j1; j += 8) {
                    float qv[8], xv[U][8];
#pragma unroll
                    for (int t = 0; t < 8; ++t) qv[t] = qp[j + t];
#pragma unroll
                    for (int u = 0; u < U; ++u)
#pragma unroll
                        for (int t = 0; t < 8; ++t) xv[u][t] = x[u][j + t];
#pragma unroll
                    for (int u = 0; u < U; ++u)
#pragma unroll
                        for (int t = 0; t < 8; ++t) {
                            const float dlt = qv[t] - xv[u][t];
                            s[u] = fmaf(dlt, dlt, s[u]);
                        }
                }
                for (; j < j1; ++j) {
                    const float qv = qp[j];
#pragma unroll
                    for (int u = 0; u < U; ++u) {
                        const float dlt = qv - x[u][j];
                        s[u] = fmaf(dlt, dlt, s[u]);
                    }
                }
            }
            const int32_t cnt = min(64, nch - base);
            for (int32_t v = 0; v < cnt; ++v)
#pragma unroll
                for (int u = 0; u < U; ++u)
                    partial[u] += __int_as_float(__builtin_amdgcn_readlane(__float_as_int(s[u]), v));
        }
#pragma unroll
        for (int u = 0; u < U; ++u)
            if (lane == i0 + u && key[u] != kEmptyKey)
                mine = make_key(partial[u], static_cast<uint32_t>(key[u] & 0xffffffffu));
    }
    uint64_t e = kEmptyKey, kth = kEmptyKey;
    topk_offer(e, kth, mine, mine != kEmptyKey, k, lane);
    if (lane < k) {
        int64_t oid = -1;
        float od = INFINITY;
        if (bad[qi]) {
            od = __uint_as_float(0x7fc00000u);
        } else if (e != kEmptyKey) {
            oid = (int64_t)(e & 0xffffffffu);
            od = key_dist(e);
        }
        out_ids[qi * k + lane] = oid;
        out_dist[qi * k + lane] = od;
    }
}

int32_t next_pow2(int32_t v) {
    int32_t p = 1;
    while (p < v) p <<= 1;
    return p;
}

}  // namespace

size_t ivf_plan(const pdx_index *ix, int64_t nq, int32_t k, int32_t nprobe, const pdx_ivf_search_params *p,
                void *ws, IvfPlan *plan) {
    IvfPlan pl{};
    pl.nq = nq;
    pl.k = k;
    pl.nprobe = nprobe;
    pl.eps0 = p ? p->eps0 : 2.1f;
    pl.dtype = p ? p->dtype : PDX_DTYPE_F32;
    pl.rerank = 0;
    if (pl.dtype != PDX_DTYPE_F32) {
        int32_t r = p ? p->rerank : 0;
        if (r == 0) r = min(4 * k, PDX_MAX_K);
        pl.rerank = r < 0 ? 0 : max(r, k);
    }
    pl.wide = pl.rerank > PDX_MAX_K ? 1 : 0;
    pl.bond = (p && (p->bound == 1 || p->bound == 2)) ? 1 : 0;
    pl.zones = (p && p->bound == 2) ? 1 : 0;
    pl.zone_rows = pl.zones ? bond_zone_rows(ix->d, p->zone_rows) : 0;
    // ADSampling's test interval (delta_d)
    const int32_t dd = (p && p->delta_d > 0) ? p->delta_d : (ix->d >= 128 ? 32 : (ix->d / 4 > 0 ? ix->d / 4 : 1));
    {
        int32_t eng = p ? p->engine : 0;
        if (eng == 0)  // automatic: matrix cores once buckets see enough queries to fill 16-row tiles
            eng = (!(p && p->queries_per_wave > 0) && (double)nq * nprobe >= 8.0 * ix->nlist) ? 2 : 1;
        // the BOND scan gathers per-query dimensions, BSA's test reads a norm
        // per vector and test point: both on the vector ALU.  Candidate
        // buffers on the matrix cores: one tile per wave over the codes'
        // bfloat16 MFMA (their norms stored, whole 32-dimension sub-chunks),
        // else the vector ALU.
        const bool wide_ok = !pl.wide || (!(p && p->queries_per_wave == 32) && dd % 32 == 0 &&
                                          (pl.dtype == PDX_DTYPE_BF16 ? ix->xn_bf16 : ix->xn_fp8) != nullptr);
        pl.matrix = (eng == 2 && !pl.bond && !(p && p->bound == 3) && wide_ok) ? 1 : 0;
    }
    // matrix-core scans report exact f32 distances of their k best
    if (pl.matrix && pl.dtype == PDX_DTYPE_F32) pl.rerank = k;
    pl.kk = (pl.rerank > 0 && !pl.wide) ? pl.rerank : k;
    pl.w16 = (p && p->mlp) ? mlp_layout(const_cast<void *>(p->mlp)).w16 : nullptr;
    pl.trace_f = p ? p->trace_features : nullptr;
    pl.trace_need = p ? p->trace_need : nullptr;
    if (pl.trace_f || pl.trace_need) pl.w16 = nullptr;  // traces probe every bucket
    {
        float th = p ? p->mlp_threshold : 0.5f;
        th = fminf(fmaxf(th, 1e-7f), 1.0f - 1e-7f);
        pl.zthr = logf(th / (1.0f - th));
    }
    if (pl.matrix) {
        // 16 queries per MFMA tile; two tiles per wave on request (each
        // loaded value then serves 32 queries, but the wave needs about
        // 330 registers: one wave per SIMD)
        const int32_t tiles = (p && p->queries_per_wave == 32) ? 2 : 1;
        pl.qb0 = pl.qb1 = 16 * tiles;
    } else if (pl.bond) {
        pl.qb0 = pl.qb1 = 1;  // one query per wave: each query visits its own dimension order
    } else {
        pl.qb0 = pl.qb1 = (p && p->queries_per_wave > 0) ? p->queries_per_wave : kDefaultQueriesPerWave;
    }
    pl.by_size = !(p && p->bucket_order == 1);
    pl.cap0 = ivf_item_capacity(nq, 1, pl.qb0, ix->nlist);
    pl.cap1 = ivf_item_capacity(nq, nprobe - 1, pl.qb1, ix->nlist);
    pl.chunk = pl.zones ? 32 : dd;  // zones: every chunk is one whole zone
    size_t q = (size_t)(nq > 0 ? nq : 0);
    Carver c(ws);
    pl.qrot = c.take<float>(q * ix->d);
    pl.cd = c.take<float>(q * ix->nlist);
    // up to 64 probes: centroid products on the matrix cores, exact sums only near the boundary
    pl.qsq = nprobe <= kWave ? c.take<float>(q) : nullptr;
    pl.csq = nprobe <= kWave ? c.take<float>((size_t)ix->nlist) : nullptr;
    pl.probe = c.take<int32_t>(q * nprobe);
    pl.bad = c.take<int32_t>(q);
    pl.tau = c.take<uint32_t>(q);
    pl.cnt0 = c.take<int32_t>(ix->nlist);
    pl.cnt1 = c.take<int32_t>(ix->nlist);
    pl.budget = c.take<int32_t>(q);
    pl.xcd = pl.matrix ? c.take<int32_t>(18) : nullptr;  // XCD ranges of the START and later-rank items
    pl.perm = pl.bond ? c.take<int32_t>(q * ix->d) : nullptr;
    pl.qperm = pl.bond ? c.take<float>(q * ix->d) : nullptr;
    pl.items0 = c.take<int2>((size_t)pl.cap0);
    pl.items1 = c.take<int2>((size_t)(pl.cap1 > 0 ? pl.cap1 : 1));
    {
        // waves per item: enough waves to fill the chip (about 8 per SIMD)
        // when a phase has few batches; matrix-core scans only
        auto parts_for = [&](int64_t items, int32_t qb_phase) -> int32_t {
            if (!pl.matrix || items <= 0 || pl.wide) return 1;  // candidate buffers: a resume point per item
            if (p && p->bucket_split > 0) return p->bucket_split;
            const int64_t batches = (items + 15) / 16 / (qb_phase / 16), want = 8 * 4 * (int64_t)device_cus();
            int32_t s_ = 1;
            while (s_ < kMaxSplit && batches * s_ < want) s_ <<= 1;
            return s_;
        };
        const int32_t s0 = parts_for(nq, pl.qb0), s1 = parts_for(nq * (int64_t)(nprobe - 1), pl.qb1);
        pl.slots0 = SlotMap{c.take<uint64_t>(q * s0 * pl.kk), 1, 0, s0, pl.kk};
        pl.slots1 = SlotMap{c.take<uint64_t>(q * (nprobe > 1 ? nprobe - 1 : 1) * s1 * pl.kk), nprobe - 1, 1, s1,
                            pl.kk};
    }
    pl.rkeys = (pl.rerank > 0 && !pl.wide) ? c.take<uint64_t>(q * pl.kk) : nullptr;
    pl.ws = WideSink{};
    pl.wide_rounds = 0;
    if (pl.wide) {
        const int32_t cap = wide_capacity(ix, nprobe, pl.rerank, p ? p->rerank_capacity : 0);
        pl.wide_rounds = wide_rounds(ix, nprobe, pl.rerank, cap);
        pl.ws.cap = cap;
        pl.ws.r = pl.rerank;
        pl.ws.nprobe = nprobe;
        pl.ws.nq = (int64_t)q;
        pl.ws.buf = c.take<uint64_t>(q * (size_t)cap);
        pl.ws.cnt = c.take<int32_t>(q);
        pl.ws.hist = c.take<uint32_t>(q * kWideBins);
        pl.ws.hbase = c.take<int32_t>(q);
        pl.ws.resume = c.take<int32_t>(q * nprobe);
        pl.ws.over = c.take<int32_t>(q);
        pl.ws.olist = c.take<int32_t>(2 * q);
        pl.ws.ocnt = c.take<int32_t>((size_t)pl.wide_rounds + 1);
    }
    // learned prune multipliers and their traces
    pl.npt = dd < ix->d ? (ix->d + dd - 1) / dd - 1 : 0;
    pl.pw16 = (p && p->prune_mlp) ? mlp_layout(const_cast<void *>(p->prune_mlp)).w16 : nullptr;
    pl.pscale = (p && p->prune_scale > 0.0f) ? p->prune_scale : 1.0f;
    pl.ptable = p ? p->prune_table : nullptr;
    pl.trace_pf = p ? p->trace_prune_features : nullptr;
    pl.trace_pt = p ? p->trace_prune_target : nullptr;
    pl.peps = (pl.pw16 && nprobe > 1 && pl.npt > 0) ? c.take<float>(q * (nprobe - 1)) : nullptr;
    pl.tau0 = (pl.trace_pf && pl.npt > 0) ? c.take<float>(q) : nullptr;
    // matrix cores over low-precision codes: bfloat16 MFMA on the codes
    // when every chunk is whole 32-dimension sub-chunks
    pl.lp = LpOperands{};
    if (pl.matrix && pl.dtype != PDX_DTYPE_F32 && pl.chunk % 32 == 0) {
        const float *xn = pl.dtype == PDX_DTYPE_BF16 ? ix->xn_bf16 : ix->xn_fp8;
        if (xn) {
            pl.lp.nsub = ix->lp_nsub;
            pl.lp.dpad = 32 * ix->lp_nsub;
            pl.lp.qs = c.take<uint16_t>(q * 3 * (size_t)pl.lp.dpad);
            pl.lp.qn = c.take<float>(q * (size_t)pl.lp.nsub);
            pl.lp.xn = xn;
        }
    }
    pl.rule = PruneRule{pl.eps0, pl.peps};
    if (p && p->bound == 3 && ix->res_ntp > 0) {  // BSA's test with the stored residual norms
        pl.qres = c.take<float>(q * ix->res_ntp);
        pl.rule.xres = ix->xres;
        pl.rule.qres = pl.qres;
        pl.rule.ntp = ix->res_ntp;
        pl.rule.m = p->bsa_m > 0.0f ? p->bsa_m : 1.0f;
        pl.rule.err = 2.0f * (float)(ix->d + 4) * 0x1p-24f;
    }
    pl.events = p ? reinterpret_cast<hipEvent_t *>(p->phase_events) : nullptr;
    pl.counters = p ? p->counters : nullptr;
    if (plan) *plan = pl;
    return c.bytes();
}

hipError_t run_ivf(const pdx_index *ix, const float *q, const IvfPlan &pl, int64_t *out_ids, float *out_dist,
                   hipStream_t s) {
    const int32_t d = ix->d;
    const int64_t nq = pl.nq;
    hipError_t e;
    auto mark = [&](int i) { return pl.events ? hipEventRecord(pl.events[i], s) : hipSuccess; };
    if ((e = mark(0)) != hipSuccess) return e;
    // 1. rotation and centroid distances
    if (ix->has_rot) {
        if ((e = launch_sgemm_abt(q, nq, ix->rot, d, d, pl.qrot, d, s)) != hipSuccess) return e;
    } else {
        if ((e = hipMemcpyAsync(pl.qrot, q, sizeof(float) * nq * d, hipMemcpyDeviceToDevice, s)) != hipSuccess)
            return e;
    }
    if (pl.csq) {  // products on the matrix cores; exact distances near the nprobe boundary (step 2)
        if ((e = launch_sgemm_abt(pl.qrot, nq, ix->centroids, ix->nlist, d, pl.cd, ix->nlist, s)) != hipSuccess)
            return e;
        row_norm_kernel<<<(unsigned)nq, 64, 0, s>>>(pl.qrot, d, pl.qsq);
        row_norm_kernel<<<(unsigned)ix->nlist, 64, 0, s>>>(ix->centroids, d, pl.csq);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    } else if ((e = launch_pair(1, 0, pl.qrot, nq, ix->centroids, ix->nlist, d, pl.cd, ix->nlist, nullptr, s)) !=
               hipSuccess) {
        return e;
    }
    if (pl.qres && (e = launch_query_residuals(pl.qrot, nq, d, pl.chunk, pl.qres, s)) != hipSuccess) return e;
    if (pl.lp.qs &&
        (e = launch_lp_query(pl.qrot, nq, d, pl.dtype == PDX_DTYPE_FP8 ? ix->fp8_scale : nullptr, pl.lp, s)) !=
            hipSuccess)
        return e;
    // 2. nearest buckets
    int32_t pow2 = next_pow2(ix->nlist);
    if (pl.csq) {
        probe_from_dot_kernel<<<(unsigned)((nq + 3) / 4), 256, 0, s>>>(pl.cd, nq, ix->nlist, pl.qsq, pl.csq, pl.qrot,
                                                                       ix->centroids, q, d, pl.nprobe, pl.probe,
                                                                       pl.bad, pl.tau);
    } else {
        select_probe_kernel<<<(unsigned)nq, 256, pow2 * sizeof(uint64_t), s>>>(pl.cd, ix->nlist, pow2, q, d,
                                                                             pl.nprobe, pl.probe, pl.bad, pl.tau);
    }
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if (pl.wide && (e = launch_wide_init(pl.ws, pl.cd, ix->nlist, pl.probe, pl.wide_rounds, s)) != hipSuccess) return e;
    // PDX-BOND: each query's dimension order by |q'_j - mean_j| (Section 5)
    if (pl.bond && (e = launch_bond_prep(pl.qrot, nq, d, ix->means, pl.zones != 0, pl.perm, pl.qperm, pl.tau, pl.bad, s)) != hipSuccess)
        return e;
    // 3. work items grouped by bucket
    if ((e = launch_fill_i32(pl.cnt0, ix->nlist, 0, s)) != hipSuccess) return e;
    if ((e = launch_fill_i32(pl.cnt1, ix->nlist, 0, s)) != hipSuccess) return e;
    if ((e = launch_fill_i32(pl.budget, nq, pl.nprobe, s)) != hipSuccess) return e;
    {  // padding slots: query id -1
        const unsigned long long pad = 0x00000000ffffffffull;
        if (pl.qb0 > 1 &&
            (e = launch_fill_u64(reinterpret_cast<unsigned long long *>(pl.items0), pl.cap0, pad, s)) != hipSuccess)
            return e;
        if (pl.qb1 > 1 && pl.cap1 > 0 &&
            (e = launch_fill_u64(reinterpret_cast<unsigned long long *>(pl.items1), pl.cap1, pad, s)) != hipSuccess)
            return e;
    }
    int64_t tot = nq * pl.nprobe;
    unsigned gb = (unsigned)((tot + 255) / 256);
    // with a learned budget the items of ranks >= 1 are built once it is known
    const bool later = pl.w16 != nullptr;
    const int32_t rhi0 = later ? 1 : pl.nprobe;
    item_count_kernel<<<gb, 256, 0, s>>>(pl.probe, nq, pl.nprobe, 0, rhi0, nullptr, pl.cnt0, pl.cnt1);
    batch_prefix_kernel<<<later ? 1 : 2, 1024, pow2 * sizeof(uint64_t) + ix->nlist * sizeof(int32_t), s>>>(
        pl.cnt0, pl.qb0, pl.xcd, pl.cnt1, pl.qb1, pl.xcd ? pl.xcd + 9 : nullptr, ix->nlist, pow2, ix->list_size,
        pl.by_size);
    item_scatter_kernel<<<gb, 256, 0, s>>>(pl.probe, nq, pl.nprobe, 0, rhi0, nullptr, pl.cnt0, pl.cnt1, pl.items0,
                                          pl.items1);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    // 4. START
    const void *data = pl.dtype == PDX_DTYPE_BF16 ? static_cast<const void *>(ix->pdx_bf16)
                       : pl.dtype == PDX_DTYPE_FP8 ? static_cast<const void *>(ix->pdx_fp8)
                                                   : static_cast<const void *>(ix->pdx);
    // `cap` item slots starting at `items`: one item per wave (qb = 1), or
    // cap / qb batches of qb items
    auto scan = [&](bool prune, const int2 *items, int64_t cap, int32_t qb, const SlotMap &sm,
                    unsigned long long *cnt, const int32_t *xr) {
        if (cap <= 0) return hipSuccess;
        if (pl.bond)
            return launch_bond_items(prune, ix, items, cap, pl.probe, pl.nprobe, pl.perm, pl.qperm, pl.tau, pl.bad,
                                     sm, pl.chunk, cnt, pl.zones != 0, pl.zone_rows, s);
        if (qb == 1) {
            const uint32_t nwg = (uint32_t)((cap + 3) / 4);
            const unsigned grid = 8u * ((nwg + 7u) / 8u);
#define PDX_SCAN(P, S, W)                                                                                       \
    ivf_scan_kernel<P, S, W><<<grid, 256, 0, s>>>(data, ix->fp8_scale, d, ix->slot_id, ix->list_goff, items, cap, \
                                                  pl.probe, pl.nprobe, pl.qrot, pl.tau, pl.bad, sm, pl.chunk,     \
                                                  pl.rule, cnt, nwg, pl.ws)
            if (pl.wide) {  // low precision only
                if (prune) {
                    if (pl.dtype == PDX_DTYPE_BF16) PDX_SCAN(true, PDX_DTYPE_BF16, true);
                    else PDX_SCAN(true, PDX_DTYPE_FP8, true);
                } else {
                    if (pl.dtype == PDX_DTYPE_BF16) PDX_SCAN(false, PDX_DTYPE_BF16, true);
                    else PDX_SCAN(false, PDX_DTYPE_FP8, true);
                }
            } else if (prune) {
                if (pl.dtype == PDX_DTYPE_BF16) PDX_SCAN(true, PDX_DTYPE_BF16, false);
                else if (pl.dtype == PDX_DTYPE_FP8) PDX_SCAN(true, PDX_DTYPE_FP8, false);
                else PDX_SCAN(true, PDX_DTYPE_F32, false);
            } else {
                if (pl.dtype == PDX_DTYPE_BF16) PDX_SCAN(false, PDX_DTYPE_BF16, false);
                else if (pl.dtype == PDX_DTYPE_FP8) PDX_SCAN(false, PDX_DTYPE_FP8, false);
                else PDX_SCAN(false, PDX_DTYPE_F32, false);
            }
#undef PDX_SCAN
            return hipGetLastError();
        }
        const int64_t nb = cap / qb;
        if (pl.matrix)
            return launch_ivf_mscan(prune, pl.dtype, qb / 16, data, ix->fp8_scale, d, ix->slot_id, ix->list_goff,
                                    ix->centroids, items, nb, xr, pl.probe, pl.nprobe, pl.qrot, pl.tau, pl.bad, sm,
                                    pl.chunk, pl.rule, cnt, pl.lp, pl.wide ? &pl.ws : nullptr, s);
        const unsigned grid = (unsigned)((nb + 3) / 4);
#define PDX_BSCAN(P, S, Q, W)                                                                                 \
    ivf_bscan_kernel<P, S, Q, W><<<grid, 256, 0, s>>>(data, ix->fp8_scale, d, ix->slot_id, ix->list_goff, items, \
                                                      nb, pl.probe, pl.nprobe, pl.qrot, pl.tau, pl.bad, sm,     \
                                                      pl.chunk, pl.rule, cnt, pl.ws)
#define PDX_BSCAN_W(P, S, W)                     \
    switch (qb) {                                \
        case 2: PDX_BSCAN(P, S, 2, W); break;    \
        case 4: PDX_BSCAN(P, S, 4, W); break;    \
        case 8: PDX_BSCAN(P, S, 8, W); break;    \
        default: PDX_BSCAN(P, S, 16, W); break;  \
    }
#define PDX_BSCAN_Q(P, S) PDX_BSCAN_W(P, S, false)
        if (pl.wide) {  // low precision only
            if (prune) {
                if (pl.dtype == PDX_DTYPE_BF16) PDX_BSCAN_W(true, PDX_DTYPE_BF16, true)
                else PDX_BSCAN_W(true, PDX_DTYPE_FP8, true)
            } else {
                if (pl.dtype == PDX_DTYPE_BF16) PDX_BSCAN_W(false, PDX_DTYPE_BF16, true)
                else PDX_BSCAN_W(false, PDX_DTYPE_FP8, true)
            }
        } else if (prune) {
            if (pl.dtype == PDX_DTYPE_BF16) PDX_BSCAN_Q(true, PDX_DTYPE_BF16)
            else if (pl.dtype == PDX_DTYPE_FP8) PDX_BSCAN_Q(true, PDX_DTYPE_FP8)
            else PDX_BSCAN_Q(true, PDX_DTYPE_F32)
        } else {
            if (pl.dtype == PDX_DTYPE_BF16) PDX_BSCAN_Q(false, PDX_DTYPE_BF16)
            else if (pl.dtype == PDX_DTYPE_FP8) PDX_BSCAN_Q(false, PDX_DTYPE_FP8)
            else PDX_BSCAN_Q(false, PDX_DTYPE_F32)
        }
#undef PDX_BSCAN_Q
#undef PDX_BSCAN_W
#undef PDX_BSCAN
        return hipGetLastError();
    };
    if ((e = scan(false, pl.items0, pl.cap0, pl.qb0, pl.slots0, pl.counters, pl.xcd)) != hipSuccess) return e;
    if (!pl.wide) {  // tau: the k-th (or R-th) distance of START (the candidate buffer keeps its own)
        ivf_merge_kernel<<<(unsigned)nq, 64, 0, s>>>(pl.slots0, true, pl.slots1, 1, nullptr, pl.kk, pl.bad, pl.tau,
                                                    nullptr, nullptr, nullptr);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    if ((e = mark(1)) != hipSuccess) return e;
    // 5. learned probe budget (or the traces of its inputs), then the
    //    pruned scan of the other probed buckets
    if ((pl.w16 || pl.trace_f) && pl.nprobe > 1) {
        budget_kernel<<<(unsigned)nq, 64, 0, s>>>(pl.qrot, d, pl.cd, ix->nlist, pl.probe, pl.nprobe, pl.tau, pl.bad,
                                                  pl.w16, pl.zthr, pl.budget, pl.trace_f);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    // learned prune bounds (and the START threshold for the traces)
    if ((pl.peps || pl.tau0) && pl.nprobe > 1) {
        const int64_t npairs = nq * (pl.nprobe - 1);
        prune_table_kernel<<<(unsigned)((npairs + 3) / 4), 256, 0, s>>>(
            pl.qrot, d, pl.cd, ix->nlist, pl.probe, pl.nprobe, pl.tau, pl.bad, pl.peps ? pl.pw16 : nullptr,
            pl.pscale, pl.chunk, pl.npt, npairs, pl.peps, pl.ptable, pl.tau0);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    if (later) {  // items of ranks 1 .. budget - 1
        item_count_kernel<<<gb, 256, 0, s>>>(pl.probe, nq, pl.nprobe, 1, pl.nprobe, pl.budget, pl.cnt0, pl.cnt1);
        batch_prefix_kernel<<<1, 1024, pow2 * sizeof(uint64_t) + ix->nlist * sizeof(int32_t), s>>>(
            pl.cnt1, pl.qb1, pl.xcd ? pl.xcd + 9 : nullptr, nullptr, 0, nullptr, ix->nlist, pow2, ix->list_size,
            pl.by_size);
        item_scatter_kernel<<<gb, 256, 0, s>>>(pl.probe, nq, pl.nprobe, 1, pl.nprobe, pl.budget, pl.cnt0, pl.cnt1,
                                              pl.items0, pl.items1);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    if (pl.trace_f && pl.nprobe == 1)
        if ((e = launch_fill_i32(reinterpret_cast<int32_t *>(pl.trace_f), nq * kMlpIn, 0, s)) != hipSuccess) return e;
    if (pl.nprobe > 1 &&
        (e = scan(true, pl.items1, pl.cap1, pl.qb1, pl.slots1, pl.counters ? pl.counters + 2 : nullptr,
                  pl.xcd ? pl.xcd + 9 : nullptr)) != hipSuccess)
        return e;
    if ((e = mark(2)) != hipSuccess) return e;
    // 6. merge
    if (pl.wide) {
        // compaction and resume rounds, then the R best re-ranked exactly
        for (int32_t rd = 0; rd < pl.wide_rounds; ++rd) {
            if ((e = launch_wide_select(pl.ws, rd, pl.tau, s)) != hipSuccess) return e;
            WideSink wr = pl.ws;
            wr.round = rd + 1;
#define PDX_RESUME(S)                                                                                             \
    ivf_wide_resume_kernel<S><<<1024, 256, 0, s>>>(data, ix->fp8_scale, d, ix->slot_id, ix->list_goff, pl.probe, \
                                                   pl.nprobe, pl.qrot, pl.tau, pl.bad, pl.slots1, pl.chunk,      \
                                                   pl.rule, pl.counters ? pl.counters + 2 : nullptr, wr, rd)
            if (pl.dtype == PDX_DTYPE_BF16) PDX_RESUME(PDX_DTYPE_BF16);
            else PDX_RESUME(PDX_DTYPE_FP8);
#undef PDX_RESUME
            if ((e = hipGetLastError()) != hipSuccess) return e;
        }
        if ((e = launch_wide_select(pl.ws, -1, pl.tau, s)) != hipSuccess) return e;
        if ((e = launch_wide_rerank(pl.ws, ix->xrow, pl.qrot, d, pl.chunk, pl.bad, pl.k, out_ids, out_dist, s)) !=
            hipSuccess)
            return e;
    } else if (pl.rerank > 0) {
        ivf_merge_kernel<<<(unsigned)nq, 64, 0, s>>>(pl.slots0, true, pl.slots1, pl.nprobe,
                                                    later ? pl.budget : nullptr, pl.kk, pl.bad, nullptr, nullptr,
                                                    nullptr, pl.rkeys);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        rerank_kernel<<<(unsigned)((nq + 3) / 4), 256, 0, s>>>(pl.rkeys, pl.kk, pl.k, ix->xrow, pl.qrot, d,
                                                               pl.chunk, pl.bad, nq, out_ids, out_dist);
    } else {
        ivf_merge_kernel<<<(unsigned)nq, 64, 0, s>>>(pl.slots0, true, pl.slots1, pl.nprobe,
                                                    later ? pl.budget : nullptr, pl.k, pl.bad, nullptr, out_ids,
                                                    out_dist, nullptr);
    }
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if (pl.trace_pf && pl.npt > 0) {
        const int64_t nslots = nq * pl.k;
        prune_trace_kernel<<<(unsigned)((nslots + 3) / 4), 256, 0, s>>>(
            out_ids, out_dist, pl.k, ix->assign, ix->xrow, pl.qrot, d, pl.cd, ix->nlist, pl.probe, pl.nprobe,
            pl.tau0, pl.bad, pl.chunk, pl.npt, nslots, pl.trace_pf, pl.trace_pt);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    if (pl.trace_need) {
        need_kernel<<<(unsigned)nq, 64, 0, s>>>(out_ids, pl.k, ix->assign, pl.probe, pl.nprobe, pl.trace_need);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    return mark(3);
}

}  // namespace pdx
