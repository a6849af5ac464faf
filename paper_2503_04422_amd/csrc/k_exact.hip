// Exact search on the flat PDX index: query preparation (PDX-BOND order),
// the chunked PDX scan with the partial-distance bound, and the k-best
// merge.
//
// Mapping (one wave = one query x one vectorgroup at a time):
//  * lane i owns vector i of the group, so every dimension is one coalesced
//    256-byte row load (the kernel listing of Section 3, vectors across
//    lanes instead of SIMD slots);
//  * dimensions are visited in chunks in the query's order; after every
//    chunk the lanes whose partial distance is strictly above the running
//    k-th distance drop out (Sections 2.3 and 5) and a group whose lanes
//    have all dropped is left (wave-level break-off, Section 4 PRUNE);
//  * survivors of the last chunk enter a register k-best list of the wave;
//    its k-th distance is published to a per-query threshold with an
//    atomic minimum, which every wave reads before each group (threshold
//    propagation between blocks, Section 4).  Any wave's k-th distance is
//    an upper bound of the final one, so pruning against the minimum over
//    waves never drops a true neighbour, and ties survive (strict test).
//  * each vector's partial sum is accumulated chunk by chunk in the query's
//    dimension order with fused multiply-adds, so its final distance is the
//    same float32 value whichever wave or launch computed it.
#include "pdx_internal.h"
#include "wave_topk.h"

namespace pdx {
namespace {

// ---------------------------------------------------------------------------
// Query preparation: visit order and permuted query values.
// PDX-BOND (Section 5): dimensions by |q_j - mean_j| descending, ties by j.
// Sort key (ascending): (~bits(|q_j - mean_j|) << 32) | j.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void prep_kernel(const float *__restrict__ q, int32_t d,
                                                   const float *__restrict__ means, int32_t mode,
                                                   int32_t pow2, int32_t *__restrict__ perm_off,
                                                   float *__restrict__ qperm,
                                                   uint32_t *__restrict__ tau,
                                                   int32_t *__restrict__ bad) {
    extern __shared__ uint64_t smem[];
    uint64_t *keys = smem;                                   // [pow2]
    float *qs = reinterpret_cast<float *>(smem + pow2);     // [d]
    const int64_t qi = blockIdx.x;
    const float *qrow = q + qi * d;
    int nonfinite = 0;
    for (int j = threadIdx.x; j < d; j += blockDim.x) {
        float v = qrow[j];
        qs[j] = v;
        nonfinite |= !isfinite(v);
    }
    nonfinite = __syncthreads_or(nonfinite);
    int32_t *po = perm_off + qi * d;
    float *qp = qperm + qi * d;
    if (mode == PDX_MODE_LINEAR) {
        for (int j = threadIdx.x; j < d; j += blockDim.x) {
            po[j] = j * kGroup;
            qp[j] = qs[j];
        }
    } else {
        for (int j = threadIdx.x; j < pow2; j += blockDim.x) {
            uint64_t key = kEmptyKey;
            if (j < d) {
                uint32_t kb = __float_as_uint(fabsf(qs[j] - means[j]));
                key = (static_cast<uint64_t>(~kb) << 32) | static_cast<uint32_t>(j);
            }
            keys[j] = key;
        }
        __syncthreads();
        for (int k2 = 2; k2 <= pow2; k2 <<= 1) {
            for (int j2 = k2 >> 1; j2 > 0; j2 >>= 1) {
                for (int i = threadIdx.x; i < pow2; i += blockDim.x) {
                    int ixj = i ^ j2;
                    if (ixj > i) {
                        uint64_t a = keys[i], b = keys[ixj];
                        bool up = (i & k2) == 0;
                        if ((a > b) == up) {
                            keys[i] = b;
                            keys[ixj] = a;
                        }
                    }
                }
                __syncthreads();
            }
        }
        for (int j = threadIdx.x; j < d; j += blockDim.x) {
            int32_t src = static_cast<int32_t>(keys[j] & 0xffffffffu);
            po[j] = src * kGroup;
            qp[j] = qs[src];
        }
    }
    if (threadIdx.x == 0) {
        tau[qi] = kInfBits;
        bad[qi] = nonfinite;
    }
}

// Sum of (q_j - x_j)^2 over dimensions [c0, c1) of the visit order, one
// fused multiply-add after the other starting from zero.
template <int UNROLL>
__device__ __forceinline__ float chunk_sum(const float *__restrict__ gp, const int32_t *__restrict__ po,
                                           const float *__restrict__ qp, int32_t c0, int32_t c1) {
    float s = 0.0f;
    int32_t j = c0;
    for (; j + UNROLL <= c1; j += UNROLL) {
        float x[UNROLL];
#pragma unroll
        for (int u = 0; u < UNROLL; ++u) x[u] = gp[po[j + u]];
#pragma unroll
        for (int u = 0; u < UNROLL; ++u) {
            float t = qp[j + u] - x[u];
            s = fmaf(t, t, s);
        }
    }
    for (; j < c1; ++j) {
        float t = qp[j] - gp[po[j]];
        s = fmaf(t, t, s);
    }
    return s;
}

// ---------------------------------------------------------------------------
// Chunked scan over vectorgroups [g_begin, g_end).
// Work item = (tile of tile_groups groups, block of qpb queries); wave w of
// a workgroup serves query qb*qpb + w.  Workgroup ids are spread so that all
// query blocks of one tile run on the same XCD (ids are dealt round-robin to
// the 8 XCDs), keeping the tile's rows in that XCD's L2.
// ---------------------------------------------------------------------------
template <bool PRUNE>
__global__ __launch_bounds__(512) void scan_kernel(
    const float *__restrict__ pdxd, int64_t n, int32_t d, int32_t g_begin, int32_t g_end,
    int32_t tile_groups, int32_t ntiles, int32_t nqb, int64_t nq, int32_t qpb,
    const int32_t *__restrict__ perm_off, const float *__restrict__ qperm, uint32_t *__restrict__ tau,
    const int32_t *__restrict__ bad, uint64_t *__restrict__ slots, int32_t nslots, int32_t slot0,
    int32_t k, int32_t chunk, unsigned long long *__restrict__ counters) {
    const uint32_t L = blockIdx.x;
    const int32_t xcd = L & 7;
    const uint32_t r = L >> 3;
    const int32_t qb = r % nqb;
    const int32_t tile = (r / nqb) * 8 + xcd;
    if (tile >= ntiles) return;
    const int32_t wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    const int64_t qi = (int64_t)qb * qpb + wave;
    if (qi >= nq) return;
    uint64_t *myslot = slots + ((size_t)qi * nslots + slot0 + tile) * k;
    if (bad[qi]) {
        if (lane < k) myslot[lane] = kEmptyKey;
        return;
    }
    const int32_t *po = perm_off + qi * d;
    const float *qp = qperm + qi * d;
    uint64_t e = kEmptyKey;    // this lane's entry of the wave's k-best list
    uint64_t kth = kEmptyKey;  // k-th entry (wave-uniform)
    const int32_t g0 = g_begin + tile * tile_groups;
    const int32_t g1 = min(g0 + tile_groups, g_end);
    unsigned long long live_vals = 0, lane_vals = 0;  // instrumentation only
    for (int32_t g = g0; g < g1; ++g) {
        float tau_eff = INFINITY;
        if (PRUNE) {
            uint32_t tg = __hip_atomic_load(tau + qi, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            float tl = kth == kEmptyKey ? INFINITY : key_dist(kth);
            tau_eff = fminf(__uint_as_float(tg), tl);
        }
        const int64_t v = (int64_t)g * kGroup + lane;
        bool alive = v < n;
        const float *gp = pdxd + (int64_t)g * d * kGroup + lane;
        float partial = 0.0f;
        for (int32_t c0 = 0; c0 < d; c0 += chunk) {
            if (PRUNE && !__any(alive)) break;
            const int32_t c1 = min(c0 + chunk, d);
            if (counters) {
                live_vals += (unsigned long long)__popcll(__ballot(alive)) * (c1 - c0);
                lane_vals += 64ull * (c1 - c0);
            }
            float s = 0.0f;
            if (alive) s = (c1 - c0 == 32) ? chunk_sum<32>(gp, po, qp, c0, c1) : chunk_sum<8>(gp, po, qp, c0, c1);
            partial += s;
            if (PRUNE) alive = alive && !(partial > tau_eff);
        }
        topk_offer(e, kth, make_key(partial, static_cast<uint32_t>(v)), alive, k, lane);
        if (PRUNE && kth != kEmptyKey) {
            float kt = key_dist(kth);
            if (kt < tau_eff && lane == 0) atomicMin(tau + qi, __float_as_uint(kt));
        }
    }
    if (lane < k) myslot[lane] = e;
    if (counters && lane == 0) {
        atomicAdd(counters, live_vals);
        atomicAdd(counters + 1, lane_vals);
    }
}

// ---------------------------------------------------------------------------
// k-best of a query's slots [slot_begin, slot_begin + slot_count).
// Writes the threshold (k-th distance) and/or the final result.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(64) void merge_kernel(const uint64_t *__restrict__ slots, int32_t nslots,
                                                   int32_t slot_begin, int32_t slot_count, int32_t k,
                                                   const int32_t *__restrict__ bad,
                                                   uint32_t *__restrict__ tau,
                                                   int64_t *__restrict__ out_ids,
                                                   float *__restrict__ out_dist) {
    const int64_t qi = blockIdx.x;
    const int lane = threadIdx.x;
    const uint64_t *base = slots + ((size_t)qi * nslots + slot_begin) * k;
    const int64_t total = (int64_t)slot_count * k;
    uint64_t e = kEmptyKey, kth = kEmptyKey;
    for (int64_t i0 = 0; i0 < total; i0 += kWave) {
        uint64_t key = (i0 + lane < total) ? base[i0 + lane] : kEmptyKey;
        topk_offer(e, kth, key, key != kEmptyKey, k, lane);
    }
    if (tau && lane == 0 && kth != kEmptyKey) tau[qi] = static_cast<uint32_t>(kth >> 32);
    if (out_ids && lane < k) {
        int64_t id = -1;
        float dist = INFINITY;
        if (bad[qi]) {
            dist = __uint_as_float(0x7fc00000u);
        } else if (e != kEmptyKey) {
            id = static_cast<int64_t>(e & 0xffffffffu);
            dist = key_dist(e);
        }
        out_ids[qi * k + lane] = id;
        out_dist[qi * k + lane] = dist;
    }
}

int32_t next_pow2(int32_t v) {
    int32_t p = 1;
    while (p < v) p <<= 1;
    return p;
}

}  // namespace

size_t exact_plan(const pdx_index *ix, int64_t nq, int32_t k, const pdx_search_params *p,
                  void *ws, ExactPlan *plan) {
    ExactPlan pl{};
    pl.nq = nq;
    pl.k = k;
    pl.mode = p ? p->mode : PDX_MODE_BOND;
    pl.chunk = (p && p->chunk > 0) ? p->chunk : 32;
    pl.tile_groups = (p && p->tile_groups > 0) ? p->tile_groups : 16;
    pl.qpb = (p && p->queries_per_block > 0) ? p->queries_per_block : 4;
    if (pl.mode == PDX_MODE_BOND) {
        int32_t sg = (ix->start_rows + kGroup - 1) / kGroup;
        pl.start_groups = sg < ix->ngroups ? sg : ix->ngroups;
    } else {
        pl.start_groups = 0;
    }
    pl.tiles_start = (pl.start_groups + pl.tile_groups - 1) / pl.tile_groups;
    pl.tiles_main = (ix->ngroups - pl.start_groups + pl.tile_groups - 1) / pl.tile_groups;
    pl.nslots = pl.tiles_start + pl.tiles_main;
    size_t q = static_cast<size_t>(nq > 0 ? nq : 0);
    Carver c(ws);
    pl.tau = c.take<uint32_t>(q);
    pl.bad = c.take<int32_t>(q);
    pl.perm_off = c.take<int32_t>(q * ix->d);
    pl.qperm = c.take<float>(q * ix->d);
    pl.slots = c.take<uint64_t>(q * pl.nslots * k);
    pl.events = p ? reinterpret_cast<hipEvent_t *>(p->phase_events) : nullptr;
    pl.counters = p ? p->counters : nullptr;
    if (plan) *plan = pl;
    return c.bytes();
}

hipError_t run_exact(const pdx_index *ix, const float *q, const ExactPlan &pl, int64_t *out_ids,
                     float *out_dist, hipStream_t s) {
    const int32_t d = ix->d;
    const int32_t pow2 = next_pow2(d);
    size_t lds = pow2 * sizeof(uint64_t) + d * sizeof(float);
    auto mark = [&](int i) { return pl.events ? hipEventRecord(pl.events[i], s) : hipSuccess; };
    hipError_t err;
    if ((err = mark(0)) != hipSuccess) return err;
    prep_kernel<<<dim3((unsigned)pl.nq), dim3(256), lds, s>>>(q, d, ix->means, pl.mode, pow2, pl.perm_off,
                                                              pl.qperm, pl.tau, pl.bad);
    err = hipGetLastError();
    if (err != hipSuccess) return err;
    const int32_t nqb = (int32_t)((pl.nq + pl.qpb - 1) / pl.qpb);
    auto scan = [&](bool prune, int32_t gb, int32_t ge, int32_t ntiles, int32_t slot0) {
        unsigned grid = 8u * (unsigned)((ntiles + 7) / 8) * (unsigned)nqb;
        dim3 block(64 * pl.qpb);
        if (prune)
            scan_kernel<true><<<grid, block, 0, s>>>(ix->pdx, ix->n, d, gb, ge, pl.tile_groups, ntiles, nqb,
                                                     pl.nq, pl.qpb, pl.perm_off, pl.qperm, pl.tau, pl.bad,
                                                     pl.slots, pl.nslots, slot0, pl.k, pl.chunk,
                                                     pl.counters ? pl.counters + 2 : nullptr);
        else
            scan_kernel<false><<<grid, block, 0, s>>>(ix->pdx, ix->n, d, gb, ge, pl.tile_groups, ntiles, nqb,
                                                      pl.nq, pl.qpb, pl.perm_off, pl.qperm, pl.tau, pl.bad,
                                                      pl.slots, pl.nslots, slot0, pl.k, pl.chunk,
                                                      pl.counters ? pl.counters + (slot0 == 0 && pl.tiles_start ? 0 : 2) : nullptr);
        return hipGetLastError();
    };
    if (pl.tiles_start > 0) {
        // START (Section 4, PHASE 0): the first block without pruning, then
        // its k-th distance becomes the initial threshold.
        if ((err = scan(false, 0, pl.start_groups, pl.tiles_start, 0)) != hipSuccess) return err;
        merge_kernel<<<dim3((unsigned)pl.nq), dim3(64), 0, s>>>(pl.slots, pl.nslots, 0, pl.tiles_start, pl.k,
                                                               pl.bad, pl.tau, nullptr, nullptr);
        if ((err = hipGetLastError()) != hipSuccess) return err;
    }
    if ((err = mark(1)) != hipSuccess) return err;
    if (pl.tiles_main > 0) {
        bool prune = pl.mode == PDX_MODE_BOND;
        if ((err = scan(prune, pl.start_groups, ix->ngroups, pl.tiles_main, pl.tiles_start)) != hipSuccess)
            return err;
    }
    if ((err = mark(2)) != hipSuccess) return err;
    merge_kernel<<<dim3((unsigned)pl.nq), dim3(64), 0, s>>>(pl.slots, pl.nslots, 0, pl.nslots, pl.k, pl.bad,
                                                           nullptr, out_ids, out_dist);
    if ((err = hipGetLastError()) != hipSuccess) return err;
    return mark(3);
}

}  // namespace pdx
