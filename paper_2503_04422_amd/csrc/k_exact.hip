// Exact search on the flat PDX index: query preparation (PDX-BOND order),
// the chunked PDX scan with the partial-distance bound, and the k-best
// merge.
//
// Every vector's distance to a query is accumulated in one fixed order:
// chunk by chunk in the query's visit order, each chunk of 32 dimensions as
// four octets (fused multiply-adds over 8 consecutive visited dimensions
// from zero) combined as (o0 + o1) + (o2 + o3), a chunk of any other
// length as (its first 16 dimensions) + (the rest), then added to the
// running partial.  Whichever kernel, wave or launch evaluates a
// (query, vector) pair therefore produces the same float32 value, and the
// partial after any chunk is a lower bound of the full distance (sums of
// non-negative terms are monotone under round-to-nearest).
//
// Two scan kernels:
//  * scan_kernel ("group" path): one wave = one query x one vectorgroup at
//    a time, lane i = vector i, so each dimension is one coalesced 256-byte
//    row (the kernel listing of Section 3 with vectors across lanes); lanes
//    drop out when their partial distance passes the threshold and the wave
//    leaves the group when all lanes have dropped.  Used for START, the
//    linear mode, shapes the tile path does not take, and as the fallback of
//    the tile path.
//  * tile_kernel ("tile" path): a workgroup stages 32 vectors x all D
//    dimensions in LDS once and scans them for every query of the batch, so
//    HBM is read once per batch instead of once per query.  The first chunk
//    is scanned densely (lanes = 16 vector pairs x 4 octets); the few
//    survivors go to an LDS queue and are finished by "persistent" lanes,
//    each lane carrying one (query, vector) pair chunk by chunk and taking a
//    new pair from the queue when its pair is pruned or complete.  Completed
//    pairs (distance <= threshold) are appended to a per-query candidate
//    buffer; between rounds of tiles the threshold becomes the k-th smallest
//    candidate (threshold propagation between blocks, Section 4).
#include "pdx_internal.h"
#include "wave_topk.h"

namespace pdx {
namespace {

constexpr int kTV = 32;       // vectors per LDS tile (half a vectorgroup)
constexpr int kTW = 16;       // waves per workgroup
constexpr int kQCap = 2048;   // survivor queue entries per tile in LDS
constexpr int kGCap = 16384;  // further entries per workgroup in global memory
constexpr int kZone = 32;     // dimensions per zone (one chunk)
constexpr int32_t kModeZones = 2;  // prep_kernel: dimension-zone order

// ---------------------------------------------------------------------------
// Query preparation: visit order and permuted query values.
// PDX-BOND (Section 5): dimensions by |q_j - mean_j| descending, ties by j.
// Sort key (ascending): (~bits(|q_j - mean_j|) << 32) | j.
// Dimension zones (Section 5, Figure "dz"; mode kModeZones): zones of kZone
// consecutive stored dimensions by sum_j |q_j - mean_j| descending (float32,
// j ascending), ties by zone; storage order inside a zone; when D is not a
// multiple of kZone the shorter last zone comes last, so every chunk of
// kZone visited dimensions is one whole zone.
// perm[j] is the j-th visited dimension; qperm[j] the query value there;
// poff[j] (optional, tile path: d kTV < 65536) its LDS tile row offset
// perm[j] * kTV, half the size of perm in the tile kernel's registers.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void prep_kernel(const float *__restrict__ q, int32_t d,
                                                   const float *__restrict__ means, int32_t mode,
                                                   int32_t pow2, int32_t *__restrict__ perm,
                                                   float *__restrict__ qperm,
                                                   uint32_t *__restrict__ tau,
                                                   int32_t *__restrict__ bad, uint16_t *__restrict__ poff) {
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
    int32_t *po = perm + qi * d;
    float *qp = qperm + qi * d;
    uint16_t *pf = poff ? poff + qi * d : nullptr;
    if (mode == PDX_MODE_LINEAR) {
        for (int j = threadIdx.x; j < d; j += blockDim.x) {
            po[j] = j;
            qp[j] = qs[j];
            if (pf) pf[j] = static_cast<uint16_t>(j * kTV);
        }
    } else {
        const bool zones = mode == kModeZones;
        const int32_t cnt = zones ? d / kZone : d;  // sort keys: zones or dimensions
        int32_t p2 = 1;
        while (p2 < cnt) p2 <<= 1;  // <= pow2
        for (int j = threadIdx.x; j < p2; j += blockDim.x) {
            uint64_t key = kEmptyKey;
            if (j < cnt) {
                float sc;
                if (zones) {
                    sc = 0.0f;
                    for (int u = 0; u < kZone; ++u) sc += fabsf(qs[j * kZone + u] - means[j * kZone + u]);
                } else {
                    sc = fabsf(qs[j] - means[j]);
                }
                key = (static_cast<uint64_t>(~__float_as_uint(sc)) << 32) | static_cast<uint32_t>(j);
            }
            keys[j] = key;
        }
        __syncthreads();
        for (int k2 = 2; k2 <= p2; k2 <<= 1) {
            for (int j2 = k2 >> 1; j2 > 0; j2 >>= 1) {
                for (int i = threadIdx.x; i < p2; i += blockDim.x) {
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
            int32_t src;
            if (zones)
                src = j < cnt * kZone ? static_cast<int32_t>(keys[j / kZone] & 0xffffffffu) * kZone + j % kZone : j;
            else
                src = static_cast<int32_t>(keys[j] & 0xffffffffu);
            po[j] = src;
            qp[j] = qs[src];
            if (pf) pf[j] = static_cast<uint16_t>(src * kTV);
        }
    }
    if (threadIdx.x == 0) {
        tau[qi] = kInfBits;
        bad[qi] = nonfinite;
    }
}

// One term of the distance: (q - x)^2 (L2) or |q - x| (L1, the kernel
// listing's second distance) added to acc.
template <bool L1>
__device__ __forceinline__ float dist_term(float acc, float t) {
    return L1 ? acc + fabsf(t) : fmaf(t, t, acc);
}

// Four octet sums of a 32-dimension chunk combined in the fixed order.
__device__ __forceinline__ float octets(float o0, float o1, float o2, float o3) { return (o0 + o1) + (o2 + o3); }

// Chunk [c0, c1) of the visit order for one lane's vector: a full chunk of
// 32 as four octets, any other length as (first 16) + (rest).
template <bool FULL32, bool L1>
__device__ __forceinline__ float chunk_sum(const float *__restrict__ gp, const int32_t *__restrict__ po,
                                           const float *__restrict__ qp, int32_t c0, int32_t c1) {
    if (FULL32) {
        float x[32];
#pragma unroll
        for (int u = 0; u < 32; ++u) x[u] = gp[po[c0 + u] * kGroup];
        float o[4];
#pragma unroll
        for (int g = 0; g < 4; ++g) {
            o[g] = 0.0f;
#pragma unroll
            for (int u = 8 * g; u < 8 * g + 8; ++u) o[g] = dist_term<L1>(o[g], qp[c0 + u] - x[u]);
        }
        return octets(o[0], o[1], o[2], o[3]);
    }
    float lo = 0.0f, hi = 0.0f;
    const int32_t mid = min(c0 + 16, c1);
    for (int32_t j = c0; j < mid; ++j) lo = dist_term<L1>(lo, qp[j] - gp[po[j] * kGroup]);
    for (int32_t j = mid; j < c1; ++j) hi = dist_term<L1>(hi, qp[j] - gp[po[j] * kGroup]);
    return lo + hi;
}

// One whole zone (kZone = 32 consecutive stored dimensions) of one row,
// read from the row-major copy as one 128-byte line (xr 16-byte aligned),
// summed exactly as chunk_sum<true, false> sums the same dimensions from
// the vectorgroup rows (four octets).
__device__ __forceinline__ float zone_sum(const float *__restrict__ xr, const float *__restrict__ qp) {
    float x[kZone];
#pragma unroll
    for (int u = 0; u < kZone / 4; ++u) {
        const float4 v = reinterpret_cast<const float4 *>(xr)[u];
        x[4 * u] = v.x;
        x[4 * u + 1] = v.y;
        x[4 * u + 2] = v.z;
        x[4 * u + 3] = v.w;
    }
    float o[4];
#pragma unroll
    for (int g = 0; g < 4; ++g) {
        o[g] = 0.0f;
#pragma unroll
        for (int u = 8 * g; u < 8 * g + 8; ++u) o[g] = dist_term<false>(o[g], qp[u] - x[u]);
    }
    return octets(o[0], o[1], o[2], o[3]);
}

// One wave scans groups [g0, g1) for query qi and writes its k-best list to
// myslot.  PRUNE: drop lanes whose partial exceeds the threshold.
// ZONES (dimension-zone order, chunk = kZone): after the first chunk, a
// vectorgroup with at most zone_rows live lanes reads each live row's zone
// from the row-major copy xrow ([n][d], by row id, d % 4 == 0) -- one line
// per survivor instead of kZone dimension rows of the group.  Both reads
// give the same bits.
// surv (optional, PRUNE only): per-chunk survivor counts, entry c0 / chunk
// += the lanes still alive after chunk [c0, c1).
template <bool PRUNE, bool L1 = false, bool ZONES = false>
__device__ __forceinline__ void scan_groups(const float *__restrict__ pdxd, int64_t n,
                                            const int32_t *__restrict__ slot_id, int32_t d, int32_t g0,
                                            int32_t g1, int64_t qi, const int32_t *__restrict__ perm,
                                            const float *__restrict__ qperm, uint32_t *__restrict__ tau,
                                            uint64_t *__restrict__ myslot, int32_t k, int32_t chunk,
                                            unsigned long long *__restrict__ counters,
                                            const float *__restrict__ xrow = nullptr, int32_t zone_rows = 0,
                                            unsigned long long *__restrict__ surv = nullptr) {
    const int lane = threadIdx.x & 63;
    const int32_t *po = perm + qi * d;
    const float *qp = qperm + qi * d;
    uint64_t e = kEmptyKey;    // this lane's entry of the wave's k-best list
    uint64_t kth = kEmptyKey;  // k-th entry (wave-uniform)
    unsigned long long live_vals = 0, lane_vals = 0;  // instrumentation only
    for (int32_t g = g0; g < g1; ++g) {
        float tau_eff = INFINITY;
        if (PRUNE) {
            uint32_t tg = __hip_atomic_load(tau + qi, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            float tl = kth == kEmptyKey ? INFINITY : key_dist(kth);
            tau_eff = fminf(__uint_as_float(tg), tl);
        }
        const int64_t v = (int64_t)g * kGroup + lane;
        // row id of this slot: the slot itself (flat), or the bucket layout's table (IVF; -1 = padding)
        const int32_t rid = slot_id ? slot_id[v] : (v < n ? (int32_t)v : -1);
        bool alive = rid >= 0;
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
            if (ZONES && c0 > 0 && c1 - c0 == kZone && __popcll(__ballot(alive)) <= zone_rows) {
                if (alive) s = zone_sum(xrow + (int64_t)rid * d + po[c0], qp + c0);
            } else if (alive) {
                s = (c1 - c0 == 32) ? chunk_sum<true, L1>(gp, po, qp, c0, c1) : chunk_sum<false, L1>(gp, po, qp, c0, c1);
            }
            partial += s;
            if (PRUNE) alive = alive && !(partial > tau_eff);
            if (PRUNE && surv) {
                const int na = __popcll(__ballot(alive));
                if (lane == 0 && na) atomicAdd(surv + c0 / chunk, (unsigned long long)na);
            }
        }
        topk_offer(e, kth, make_key(partial, static_cast<uint32_t>(rid)), alive, k, lane);
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
// Group path over vectorgroups [g_begin, g_end).
// Work item = (tile of tile_groups groups, block of qpb queries); wave w of
// a workgroup serves query qb*qpb + w.  Workgroup ids are spread so that all
// query blocks of one tile run on the same XCD (ids are dealt round-robin to
// the 8 XCDs), keeping the tile's rows in that XCD's L2.
// ---------------------------------------------------------------------------
template <bool PRUNE, bool L1>
__global__ __launch_bounds__(512) void scan_kernel(
    const float *__restrict__ pdxd, int64_t n, const int32_t *__restrict__ slot_id, int32_t d, int32_t g_begin,
    int32_t g_end,
    int32_t tile_groups, int32_t ntiles, int32_t nqb, int64_t nq, int32_t qpb,
    const int32_t *__restrict__ perm, const float *__restrict__ qperm, uint32_t *__restrict__ tau,
    const int32_t *__restrict__ bad, uint64_t *__restrict__ slots, int32_t nslots, int32_t slot0,
    int32_t k, int32_t chunk, unsigned long long *__restrict__ counters, unsigned long long *__restrict__ surv) {
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
    const int32_t g0 = g_begin + tile * tile_groups;
    const int32_t g1 = min(g0 + tile_groups, g_end);
    scan_groups<PRUNE, L1>(pdxd, n, slot_id, d, g0, g1, qi, perm, qperm, tau, myslot, k, chunk, counters, nullptr, 0,
                           surv);
}

// |row|^2 of every row of a [m][d] matrix, one wave per row.
__global__ __launch_bounds__(64) void row_sq_kernel(const float *__restrict__ a, int32_t d, float *__restrict__ sq) {
    const int64_t i = blockIdx.x;
    float s = 0.0f;
    for (int32_t j = threadIdx.x; j < d; j += kWave) s = fmaf(a[i * d + j], a[i * d + j], s);
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off);
    if (threadIdx.x == 0) sq[i] = s;
}

// Squared centroid distances from the matrix-core products g[q][l] = q.c_l
// (in place): |q|^2 + |c|^2 - 2 q.c lowered by 2 (D + 64) 2^-24
// (|q|^2 + |c|^2), twice the float32 rounding of the expanded form, and
// clamped at 0 -- a lower bound of |q - c|^2, which is all the centroid
// bound and the START choice need.
__global__ __launch_bounds__(256) void l2_from_dot_kernel(float *__restrict__ g, int64_t nq, int32_t nlist, int32_t d,
                                                          const float *__restrict__ qsq,
                                                          const float *__restrict__ csq) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nq * nlist) return;
    const int64_t q = i / nlist;
    const int32_t l = (int32_t)(i - q * nlist);
    const float nn = qsq[q] + csq[l];
    g[i] = fmaxf(nn - 2.0f * g[i] - (float)(d + 64) * 0x1p-23f * nn, 0.0f);
}

// Nearest bucket of each query (distances [nq][nlist]; ties to the lower
// bucket id), one wave per query.
__global__ __launch_bounds__(64) void nearest_kernel(const float *__restrict__ cd, int32_t nlist,
                                                     int32_t *__restrict__ nearest) {
    const int64_t qi = blockIdx.x;
    const int lane = threadIdx.x;
    uint64_t best = kEmptyKey;
    for (int32_t l = lane; l < nlist; l += kWave) {
        const uint64_t key = make_key(cd[qi * nlist + l], (uint32_t)l);
        best = key < best ? key : best;
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        const uint64_t o = (static_cast<uint64_t>(__shfl_xor(static_cast<uint32_t>(best >> 32), off)) << 32) |
                           __shfl_xor(static_cast<uint32_t>(best), off);
        best = o < best ? o : best;
    }
    if (lane == 0) nearest[qi] = static_cast<int32_t>(best & 0xffffffffu);
}

// Centroid bound inputs for the tile kernel: dql[l][q] = sqrt(cd[q][l])
// (L2; cd[q][l] itself for L1, where cd holds L1 distances) lowered by 1e-4
// (a lower bound of |q - c_l|: the float32 sum of D non-negative terms
// carries at most about D 2^-24 relative error), bucket-major so that the
// queries of one tile read one contiguous row.  32 x 32 blocks through LDS.
__global__ __launch_bounds__(256) void centroid_lo_kernel(const float *__restrict__ cd, int64_t nq, int32_t nlist,
                                                          float *__restrict__ dql, int32_t l1) {
    __shared__ float blk[32][33];
    const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;  // 32 x 8
    const int64_t q0 = (int64_t)blockIdx.x * 32;
    const int32_t l0 = blockIdx.y * 32;
    for (int r = ty; r < 32; r += 8) {
        const int64_t q = q0 + r;
        const int32_t l = l0 + tx;
        const float c = (q < nq && l < nlist) ? cd[q * nlist + l] : 0.0f;
        blk[r][tx] = (l1 ? c : sqrtf(c)) * (1.0f - 1e-4f);
    }
    __syncthreads();
    for (int r = ty; r < 32; r += 8) {
        const int32_t l = l0 + r;
        const int64_t q = q0 + tx;
        if (q < nq && l < nlist) dql[(int64_t)l * nq + q] = blk[tx][r];
    }
}

// START on a bucket layout (Section 4, PHASE 0 on the query's nearest
// bucket instead of the first rows): the first maxg vectorgroups of the
// bucket; `parts` waves per query share them, each writing its own k-best
// list.
template <bool L1>
__global__ __launch_bounds__(256) void start_bucket_kernel(
    const float *__restrict__ pdxd, const int32_t *__restrict__ slot_id, int32_t d,
    const int32_t *__restrict__ goff, const int32_t *__restrict__ nearest, int64_t nq, int32_t parts, int32_t maxg,
    const int32_t *__restrict__ perm, const float *__restrict__ qperm, uint32_t *__restrict__ tau,
    const int32_t *__restrict__ bad, uint64_t *__restrict__ slots, int32_t k, int32_t chunk,
    unsigned long long *__restrict__ counters) {
    const int64_t w = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    const int64_t qi = w / parts;
    const int32_t part = (int32_t)(w - qi * parts);
    const int lane = threadIdx.x & 63;
    if (qi >= nq) return;
    uint64_t *myslot = slots + ((size_t)qi * parts + part) * k;
    if (bad[qi]) {
        if (lane < k) myslot[lane] = kEmptyKey;
        return;
    }
    const int32_t l = nearest[qi];
    const int32_t a = goff[l], len = min(goff[l + 1] - a, maxg);
    const int32_t g0 = a + (int32_t)((int64_t)len * part / parts), g1 = a + (int32_t)((int64_t)len * (part + 1) / parts);
    scan_groups<false, L1>(pdxd, 0, slot_id, d, g0, g1, qi, perm, qperm, tau, myslot, k, chunk, counters);
}

// Group path for the queries whose candidate buffer overflowed in the tile
// path: every (listed query, group tile) pair, grid-stride.
template <bool L1>
__global__ __launch_bounds__(256) void fallback_kernel(
    const float *__restrict__ pdxd, int64_t n, const int32_t *__restrict__ slot_id, int32_t d, int32_t g_begin,
    int32_t g_end, int32_t tile_groups,
    int32_t ntiles, const int32_t *__restrict__ over_list, const int32_t *__restrict__ over_count,
    const int32_t *__restrict__ perm, const float *__restrict__ qperm, uint32_t *__restrict__ tau,
    uint64_t *__restrict__ slots, int32_t nslots, int32_t slot0, int32_t k, int32_t chunk,
    unsigned long long *__restrict__ surv) {
    const int32_t wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int64_t total = (int64_t)(*over_count) * ntiles;
    for (int64_t it = (int64_t)blockIdx.x * 4 + wave; it < total; it += (int64_t)gridDim.x * 4) {
        const int64_t qi = over_list[it / ntiles];
        const int32_t tile = (int32_t)(it % ntiles);
        const int32_t g0 = g_begin + tile * tile_groups;
        const int32_t g1 = min(g0 + tile_groups, g_end);
        scan_groups<true, L1>(pdxd, n, slot_id, d, g0, g1, qi, perm, qperm, tau,
                              slots + ((size_t)qi * nslots + slot0 + tile) * k, k, chunk, nullptr, nullptr, 0, surv);
    }
}

// ---------------------------------------------------------------------------
// k-best of a query's slots [slot_begin, slot_begin + slot_count).
// Writes the threshold (k-th distance), the result, and/or the list as
// the first k entries of the query's candidate buffer.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(64) void merge_kernel(const uint64_t *__restrict__ slots, int32_t nslots,
                                                   int32_t slot_begin, int32_t slot_count, int32_t k,
                                                   const int32_t *__restrict__ bad,
                                                   uint32_t *__restrict__ tau,
                                                   int64_t *__restrict__ out_ids,
                                                   float *__restrict__ out_dist, uint64_t *__restrict__ cand,
                                                   int32_t *__restrict__ cand_cnt, int32_t cap) {
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
    if (cand) {
        if (lane < k) cand[(size_t)qi * cap + lane] = e;
        if (lane == 0) cand_cnt[qi] = k;
    }
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

// k-best of a query's candidate buffer (for a query whose buffer
// overflowed: its first `head` entries, which hold rows outside the main
// range, and the fallback slots over the main range).  Refresh mode:
// tighten the threshold; final mode: write the result.
__global__ __launch_bounds__(64) void cand_merge_kernel(uint64_t *__restrict__ cand,
                                                        int32_t *__restrict__ cand_cnt, int32_t cap,
                                                        int32_t head, int32_t k, const int32_t *__restrict__ bad,
                                                        uint32_t *__restrict__ tau,
                                                        const uint64_t *__restrict__ slots, int32_t nslots,
                                                        int32_t slot_begin, int32_t slot_count,
                                                        int64_t *__restrict__ out_ids,
                                                        float *__restrict__ out_dist,
                                                        const float *__restrict__ qshift, int32_t compact) {
    const int64_t qi = blockIdx.x;
    const int lane = threadIdx.x;
    const int32_t cnt = cand_cnt[qi];
    const bool over = cnt > cap;
    const uint64_t *cb = cand + (size_t)qi * cap;
    uint64_t *cb_w = cand + (size_t)qi * cap;
    const int32_t nc = over && out_ids ? head : min(cnt, cap);
    uint64_t e = kEmptyKey, kth = kEmptyKey;
    for (int32_t i0 = 0; i0 < nc; i0 += kWave) {
        uint64_t key = (i0 + lane < nc) ? cb[i0 + lane] : kEmptyKey;
        topk_offer(e, kth, key, key != kEmptyKey, k, lane);
    }
    if (over && out_ids) {
        const uint64_t *base = slots + ((size_t)qi * nslots + slot_begin) * k;
        const int64_t total = (int64_t)slot_count * k;
        for (int64_t i0 = 0; i0 < total; i0 += kWave) {
            uint64_t key = (i0 + lane < total) ? base[i0 + lane] : kEmptyKey;
            topk_offer(e, kth, key, key != kEmptyKey, k, lane);
        }
    }
    if (!out_ids) {
        if (lane == 0 && kth != kEmptyKey) {
            uint32_t kb = static_cast<uint32_t>(kth >> 32);
            if (kb < tau[qi]) tau[qi] = kb;
        }
        if (compact && !over) {
            // keep only the k best: an entry with k better ones never
            // reaches the result (bucket layout only, where an overflowed
            // query keeps no buffer head)
            const unsigned long long has = __ballot(lane < k && e != kEmptyKey);
            if (lane < k && e != kEmptyKey) cb_w[lane] = e;
            if (lane == 0) cand_cnt[qi] = __popcll(has);
        }
        return;
    }
    if (lane < k) {
        int64_t id = -1;
        float dist = INFINITY;
        if (bad[qi]) {
            dist = __uint_as_float(0x7fc00000u);
        } else if (e != kEmptyKey) {
            id = static_cast<int64_t>(e & 0xffffffffu);
            dist = qshift ? key_dist(e) - qshift[qi] : key_dist(e);  // inner product: s' - B_q = -q.x
        }
        out_ids[qi * k + lane] = id;
        out_dist[qi * k + lane] = dist;
    }
}

__global__ void over_list_kernel(const int32_t *__restrict__ cand_cnt, int64_t nq, int32_t cap,
                                 int32_t *__restrict__ over_list, int32_t *__restrict__ over_count) {
    int64_t qi = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (qi < nq && cand_cnt[qi] > cap) over_list[atomicAdd(over_count, 1)] = (int32_t)qi;
}

// ---------------------------------------------------------------------------
// Tile path.
// ---------------------------------------------------------------------------
typedef float v4f __attribute__((ext_vector_type(4)));


__device__ __forceinline__ void cand_append(uint64_t *__restrict__ cand, int32_t *__restrict__ cnt, int32_t cap,
                                            int64_t qi, float dist, uint32_t id) {
    int32_t pos = atomicAdd(cnt + qi, 1);
    if (pos < cap) cand[(size_t)qi * cap + pos] = make_key(dist, id);
}

__device__ __forceinline__ int lane_rank(unsigned long long m) {
    return __builtin_amdgcn_mbcnt_hi(static_cast<uint32_t>(m >> 32),
                                     __builtin_amdgcn_mbcnt_lo(static_cast<uint32_t>(m), 0));
}

// Four LDS row offsets (tile path) from two words of 16-bit offsets.
__device__ __forceinline__ void unpack_off(uint32_t w0, uint32_t w1, int (&o)[4]) {
    o[0] = (int)(w0 & 0xffffu);
    o[1] = (int)(w0 >> 16);
    o[2] = (int)(w1 & 0xffffu);
    o[3] = (int)(w1 >> 16);
}

// Full chunk of 32 visited dimensions for vector v of the LDS tile, four
// octets of fused multiply-adds (pf: the chunk's 16-bit row offsets, qp:
// its query values; loaded 16 bytes at a time).
template <bool L1>
__device__ __forceinline__ float tile_chunk(const float *__restrict__ tile, const uint16_t *__restrict__ pf,
                                            const float *__restrict__ qp, int v) {
    const uint4 *o4 = reinterpret_cast<const uint4 *>(pf);
    const float4 *q4 = reinterpret_cast<const float4 *>(qp);
    float oc[4] = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
    for (int u = 0; u < 8; ++u) {
        const uint4 ow = o4[u >> 1];
        int o[4];
        unpack_off((u & 1) ? ow.z : ow.x, (u & 1) ? ow.w : ow.y, o);
        float4 qq = q4[u];
        float t0 = qq.x - tile[o[0] + v];
        float t1 = qq.y - tile[o[1] + v];
        float t2 = qq.z - tile[o[2] + v];
        float t3 = qq.w - tile[o[3] + v];
        float &s = oc[u >> 1];
        s = dist_term<L1>(s, t0);
        s = dist_term<L1>(s, t1);
        s = dist_term<L1>(s, t2);
        s = dist_term<L1>(s, t3);
    }
    return octets(oc[0], oc[1], oc[2], oc[3]);
}

// One octet (8 visited dimensions) of a chunk for the tile's adjacent
// vectors 2p and 2p + 1: one 8-byte LDS read per dimension serves both.
// The 16 lanes of an octet then read one whole 128-byte tile row, every
// bank once, so the four octets of a wave (four rows) never wait on one
// another's banks.  All 8 reads are issued before the first sum, so a
// chunk waits for one LDS round trip rather than one per dimension.
template <bool L1>
__device__ __forceinline__ void octet_pair(const float *__restrict__ tile, uint4 ow, float4 q0, float4 q1, int p,
                                           float &a, float &b) {
    int o[8];
    unpack_off(ow.x, ow.y, *reinterpret_cast<int(*)[4]>(o));
    unpack_off(ow.z, ow.w, *reinterpret_cast<int(*)[4]>(o + 4));
    const float qv[8] = {q0.x, q0.y, q0.z, q0.w, q1.x, q1.y, q1.z, q1.w};
    float ra[8], rb[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
        const float2 r = *reinterpret_cast<const float2 *>(tile + o[u] + 2 * p);
        ra[u] = r.x;
        rb[u] = r.y;
    }
    a = 0.0f;
    b = 0.0f;
#pragma unroll
    for (int u = 0; u < 8; ++u) {
        a = dist_term<L1>(a, qv[u] - ra[u]);
        b = dist_term<L1>(b, qv[u] - rb[u]);
    }
}

// A chunk's total for both vectors of a pair from the octet sums sa
// (the pair's first vector) and sb (its second), one per 16-lane row (octets 0..3),
// combined as (o0 + o1) + (o2 + o3) in the VALU with no LDS round trip.
// gfx950's first row swap (v_permlane16_swap) trades the odd rows of sa for
// the even rows of sb, so the two results add to o0 + o1 (row 0) and
// o2 + o3 (row 2) of vector p and the same (rows 1, 3) of vector p + 16;
// the second (v_permlane32_swap, a value with itself) adds the halves.
// Rows 0 and 2 end with the first vector's total, rows 1 and 3 with the
// second's.  The whole wave must be active.
__device__ __forceinline__ float pair_total(float sa, float sb) {
    const auto r = __builtin_amdgcn_permlane16_swap(__float_as_uint(sa), __float_as_uint(sb), false, false);
    const float t = __uint_as_float(r[0]) + __uint_as_float(r[1]);
    const auto r2 = __builtin_amdgcn_permlane32_swap(__float_as_uint(t), __float_as_uint(t), false, false);
    return __uint_as_float(r2[0]) + __uint_as_float(r2[1]);
}

// Bit p: the first vector of lane p's pair, bit 16 + p: the second (pairs
// held by lanes p of every octet; the lanes of octet 0 stand for them).
__device__ __forceinline__ uint32_t pair_mask(bool a, bool b) {
    return static_cast<uint32_t>(__ballot(a) & 0xffffull) | (static_cast<uint32_t>(__ballot(b) & 0xffffull) << 16);
}

// One query's first visited chunk as this lane's octet sees it: 8
// dimensions (16-bit LDS row offsets, query values), the threshold and the
// non-finite flag.
struct FirstChunk {
    uint4 o;
    float4 q[2];
    float tau;
    int bad;
    __device__ __forceinline__ void load(const uint16_t *__restrict__ poff, const float *__restrict__ qperm,
                                         const uint32_t *__restrict__ tau_all, const int32_t *__restrict__ bad_all,
                                         int64_t qi, int32_t d, int oct) {
        o = *reinterpret_cast<const uint4 *>(poff + qi * d + oct * 8);
        const float4 *q4 = reinterpret_cast<const float4 *>(qperm + qi * d + oct * 8);
        q[0] = q4[0];
        q[1] = q4[1];
        tau = __uint_as_float(tau_all[qi]);
        bad = bad_all[qi];
    }
};


// DENSE (bucket layout, where a query's own cluster fills whole tiles): a
// (query, tile) pair with at least dense_min first-chunk survivors is finished
// by its wave; other survivors go to the queue.  On this layout a tile's
// rows lie within radius r of their bucket's centroid c, so every row is at
// squared distance at least (|q - c| - r)^2 from the query (triangle
// inequality): a query whose threshold is below that bound skips the tile.
// The bound takes |q - c| 1e-4 low (dql, from centroid_lo_kernel) and r
// rounded up, so it never exceeds a row's distance.  Per tile, the
// queries that remain are listed in LDS, kList at a time, and the waves
// take them from the list.
constexpr int kList = 1024;
constexpr int kTileWaves = 16;  // waves per workgroup of the L2/L1 tile scan (kList is a multiple of their threads)
typedef __attribute__((address_space(3))) void lds_void_t;  // LDS destination of direct loads

// STATS (instrumentation build only): per-chunk survivor counts in surv.
// NW waves per workgroup.  Per tile three barriers: after the staging loads
// and the query list (built while the loads are in flight), before the
// survivor queue, and at the end; the counters of a tile alternate between
// two sets so the next tile's are cleared while this one's are in use.
// Waves take the listed queries from an LDS counter (the next one is
// claimed, and its first-chunk metadata loaded, while the current one is
// scanned), so a wave that meets cheap queries takes more of them.
template <bool DENSE, bool L1, bool STATS, int NW>
__global__ __launch_bounds__(NW * 64) void tile_kernel(
    const float *__restrict__ pdxd, int64_t n, const int32_t *__restrict__ slot_id, int32_t d, int32_t t_begin,
    int32_t t_end, int64_t nq,
    const uint16_t *__restrict__ poff, const float *__restrict__ qperm, const uint32_t *__restrict__ tau,
    const int32_t *__restrict__ bad, uint64_t *__restrict__ cand, int32_t *__restrict__ cand_cnt, int32_t cap,
    uint64_t *__restrict__ gqueue, unsigned long long *__restrict__ counters, const float *__restrict__ dql,
    const int32_t *__restrict__ group_bucket, const float *__restrict__ tile_rad, int32_t *__restrict__ tile_ctr,
    unsigned long long *__restrict__ surv, int32_t dense_min) {
    constexpr int NT = NW * 64;
    extern __shared__ float4 smem4[];
    float *tile = reinterpret_cast<float *>(smem4);                          // [d][32]
    uint2 *queue = reinterpret_cast<uint2 *>(tile + (size_t)d * kTV);        // [kQCap]
    __shared__ int32_t qcount[2], qhead[2], lcount[2], qnext[2], next_t[2];
    __shared__ int32_t qlist[DENSE ? kList : 1];
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int pr = lane & 15;   // vector pair (2 pr, 2 pr + 1) of the tile
    const int oct = lane >> 4;  // octet of the chunk
    const int32_t nchunks = d / 32;
    uint64_t *gq = gqueue + (size_t)blockIdx.x * kGCap;  // this workgroup's overflow entries
    unsigned long long live_vals = 0, lane_vals = 0;

    // the queries of [q0, q0 + kList) the centroid bound keeps for tile
    // (bucket tb, radius trad), appended to qlist (lcount[p] zero before)
    auto build_list = [&](int p, int64_t q0, int32_t tb, float trad) {
#pragma unroll
        for (int j = 0; j < kList / NT; ++j) {
            const int64_t qt = q0 + j * NT + threadIdx.x;
            bool keep = false;
            if (qt < nq && !bad[qt]) {
                const float gap = fmaxf(dql[(int64_t)tb * nq + qt] - trad, 0.0f);
                const float tq = __uint_as_float(__hip_atomic_load(tau + qt, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
                keep = L1 ? !(gap > tq) : !(gap * gap > tq);  // L1: the bound is the gap itself
            }
            const unsigned long long km = __ballot(keep);
            int lb = 0;
            if (lane == 0 && km) lb = atomicAdd(&lcount[p], __popcll(km));
            lb = __shfl(lb, 0);
            if (keep) qlist[lb + lane_rank(km)] = (int32_t)qt;
        }
    };

    if (threadIdx.x == 0) {
        next_t[0] = t_begin + atomicAdd(tile_ctr, 1);
        qcount[0] = qhead[0] = lcount[0] = qnext[0] = 0;
    }
    __syncthreads();
    // tiles are taken from a counter shared by the launch's workgroups, so
    // workgroups that meet cheap tiles take more (tile costs vary widely)
    for (int p = 0;; p ^= 1) {
        const int32_t t = next_t[p];
        if (t >= t_end) break;
        if (threadIdx.x == 0) {  // the other set is free: every thread passed the barrier that ended its tile
            next_t[p ^ 1] = t_begin + atomicAdd(tile_ctr, 1);
            qcount[p ^ 1] = qhead[p ^ 1] = lcount[p ^ 1] = qnext[p ^ 1] = 0;
        }
        // stage 32 vectors x d dimensions (one 128-byte half row per
        // dimension) with direct global-to-LDS loads: a wave's 64 lanes
        // bring 16 bytes each into 1 KB of contiguous LDS, 8 tile rows, with
        // no registers holding the data, so every piece is in flight at once.
        // The loads are non-temporal (cache policy 2): the rows are read
        // once per launch, and streaming them past the L2 keeps the queries'
        // visit orders and values, read again for every tile, resident.
        const float *src = pdxd + (int64_t)(t >> 1) * d * kGroup + (t & 1) * kTV;
        const int32_t nv4 = d * 8;  // a multiple of 64: whole waves
        for (int32_t iw = wave * 64; iw < nv4; iw += NT) {
            const int32_t i = iw + lane;
            __builtin_amdgcn_global_load_lds(src + (int64_t)(i >> 3) * kGroup + (i & 7) * 4,
                                             (lds_void_t *)(tile + (size_t)iw * 4), 16, 0, 2);
        }
        // while the loads are in flight: the pair's row ids (-1: padding)
        // and the first list of queries
        const int64_t vid_a = (int64_t)t * kTV + 2 * pr, vid_b = vid_a + 1;
        const int32_t rid_a = slot_id ? slot_id[vid_a] : (vid_a < n ? (int32_t)vid_a : -1);
        const int32_t rid_b = slot_id ? slot_id[vid_b] : (vid_b < n ? (int32_t)vid_b : -1);
        int32_t tb = 0;
        float trad = 0.0f;
        if (DENSE) {
            tb = group_bucket[t >> 1];
            trad = tile_rad[t];
            build_list(p, 0, tb, trad);
        }
        __syncthreads();  // tile staged, first list complete
        const uint32_t valid_m = pair_mask(rid_a >= 0, rid_b >= 0);
        const int32_t rid_v = (oct & 1) ? rid_b : rid_a;  // row id of this lane's vector

        // Phase A: first chunk of every query, lanes = 16 vector pairs x 4
        // octets.  The next query's first-chunk metadata is loaded while the
        // current one is scanned (one query per wave in flight otherwise
        // stalls on memory latency).
        for (int64_t q0 = 0; q0 < nq; q0 += (DENSE ? kList : nq)) {
          int32_t cnt = (int32_t)nq;
          if (DENSE) {
            if (q0 > 0) {  // a later block of kList queries: rebuild the list
                __syncthreads();  // the previous list is no longer read
                if (threadIdx.x == 0) lcount[p] = qnext[p] = 0;
                __syncthreads();
                build_list(p, q0, tb, trad);
                __syncthreads();
            }
            cnt = lcount[p];
          }
          auto qid = [&](int32_t e) -> int64_t { return DENSE ? (int64_t)qlist[e] : (int64_t)e; };
          auto claim = [&]() -> int32_t {
              int32_t v = 0;
              if (lane == 0) v = atomicAdd(&qnext[p], 1);
              return __builtin_amdgcn_readfirstlane(v);
          };
          FirstChunk cur, nxt;
          int32_t e = claim();
          if (e < cnt) cur.load(poff, qperm, tau, bad, qid(e), d, oct);
          while (e < cnt) {
            const int64_t qi = qid(e);
            const int32_t en = claim();
            if (en < cnt) nxt.load(poff, qperm, tau, bad, qid(en), d, oct);
            if (!cur.bad) {
                // the second chunk's metadata, needed if the pair turns out
                // dense (almost every listed pair on the bucket layout), is
                // requested before the first chunk is summed
                const uint4 *o4 = reinterpret_cast<const uint4 *>(poff + qi * d + oct * 8);
                const float4 *q4 = reinterpret_cast<const float4 *>(qperm + qi * d + oct * 8);
                uint4 oa;
                float4 qa0, qa1;
                float sa, sb;
                octet_pair<L1>(tile, cur.o, cur.q[0], cur.q[1], pr, sa, sb);
                // this lane's vector (2 pr in rows 0 and 2, 2 pr + 1 in rows 1 and 3)
                const float p1 = pair_total(sa, sb);
                const bool al1 = rid_v >= 0 && !(p1 > cur.tau);
                if (counters) {
                    live_vals += 32ull * __popc(valid_m);
                    lane_vals += 64ull * 16;
                }
                // bit b: lane b of rows 0 and 1, vector 2 (b & 15) + (b >> 4)
                const uint32_t m = static_cast<uint32_t>(__ballot(al1));
                if (STATS && lane == 0 && m) atomicAdd(surv, (unsigned long long)__popc(m));
                if (DENSE && m != 0 && nchunks > 1 && __popc(m) >= dense_min) {
                    // dense pair: this wave finishes the query on the tile,
                    // lanes = 16 vector pairs x 4 octets as in the first
                    // chunk; the next chunk's metadata is fetched while the
                    // current one is summed
                    bool al = al1;
                    float x = p1;
                    auto dense_step = [&](int32_t c, const uint4 oc, const float4 qc0, const float4 qc1) {
                        float ta, tb2;
                        if (counters) {  // the vectors still alive evaluate this chunk
                            live_vals += 32ull * __popc(static_cast<uint32_t>(__ballot(al)));
                            lane_vals += 64ull * 16;
                        }
                        octet_pair<L1>(tile, oc, qc0, qc1, pr, ta, tb2);
                        x += pair_total(ta, tb2);
                        al = al && !(x > cur.tau);
                        if (STATS) {
                            const uint32_t ms = static_cast<uint32_t>(__ballot(al));
                            if (lane == 0 && ms) atomicAdd(surv + c, (unsigned long long)__popc(ms));
                        }
                    };
                    // two metadata sets in turn (chunks c and c + 1), so a
                    // prefetched set is used where it landed, never copied
                    // (the second set is first written before its first use)
                    oa = o4[4];
                    qa0 = q4[8];
                    qa1 = q4[9];
                    uint4 ob;
                    float4 qb0, qb1;
                    for (int32_t c = 1; c < nchunks; c += 2) {
                        if (!__any(al)) break;
                        if (c + 1 < nchunks) {
                            ob = o4[4 * (c + 1)];
                            qb0 = q4[8 * (c + 1)];
                            qb1 = q4[8 * (c + 1) + 1];
                        }
                        dense_step(c, oa, qa0, qa1);
                        if (c + 1 == nchunks || !__any(al)) break;
                        if (c + 2 < nchunks) {
                            oa = o4[4 * (c + 2)];
                            qa0 = q4[8 * (c + 2)];
                            qa1 = q4[8 * (c + 2) + 1];
                        }
                        dense_step(c + 1, ob, qb0, qb1);
                    }
                    if (oct < 2 && al) cand_append(cand, cand_cnt, cap, qi, x, (uint32_t)rid_v);
                } else if (m != 0) {
                    if (nchunks == 1) {
                        if (oct < 2 && al1) cand_append(cand, cand_cnt, cap, qi, p1, (uint32_t)rid_v);
                    } else {
                        int base = 0;
                        if (lane == 0) base = atomicAdd(&qcount[p], __popc(m));
                        base = __shfl(base, 0);
                        // queue slot of lane b's vector: base + the
                        // survivors of the lanes below b; rows 0 and 1 enqueue
                        // their vectors
                        bool own = false;  // both queues are full: finish it here
                        if (oct < 2 && al1) {
                            const int vb = pr + 16 * oct, vv = 2 * pr + oct;
                            const int pos = base + __popc(m & ((1u << vb) - 1u));
                            const uint32_t key = (static_cast<uint32_t>(qi) << 5) | static_cast<uint32_t>(vv);
                            if (pos < kQCap)
                                queue[pos] = make_uint2(key, __float_as_uint(p1));
                            else if (pos < kQCap + kGCap)
                                gq[pos - kQCap] = (static_cast<uint64_t>(__float_as_uint(p1)) << 32) | key;
                            else
                                own = true;
                        }
                        if (__any(own)) {
                            const int vv = 2 * pr + (oct & 1);
                            const uint16_t *pf = poff + qi * d;
                            const float *qp = qperm + qi * d;
                            float x = p1;
                            for (int32_t c = 1; c < nchunks && __any(own); ++c) {
                                if (counters) {  // rows 0 and 1 hold the wave's vectors
                                    live_vals += 32ull * __popc(static_cast<uint32_t>(__ballot(own)));
                                    lane_vals += 64ull * 32;
                                }
                                if (own) {
                                    x += tile_chunk<L1>(tile, pf + c * 32, qp + c * 32, vv);
                                    own = !(x > cur.tau);
                                }
                                if (STATS) {  // rows 0 and 1 hold the wave's vectors
                                    const uint32_t ms = static_cast<uint32_t>(__ballot(own));
                                    if (lane == 0 && ms) atomicAdd(surv + c, (unsigned long long)__popc(ms));
                                }
                            }
                            if (own) cand_append(cand, cand_cnt, cap, qi, x, (uint32_t)rid_v);
                        }
                    }
                }
            }
            cur = nxt;
            e = en;
          }
        }
        __syncthreads();

        // Phase B: persistent lanes finish the queued (query, vector) pairs
        const int32_t total = min(qcount[p], kQCap + kGCap);
        bool act = false;
        uint32_t qv = 0;
        float pq = 0.0f, tl = 0.0f;
        int32_t c = 0;
        while (true) {
            const unsigned long long idle = __ballot(!act);
            if (idle) {
                int b = 0;
                if (lane == 0) b = atomicAdd(&qhead[p], __popcll(idle));
                b = __shfl(b, 0);
                if (!act) {
                    const int idx = b + lane_rank(idle);
                    if (idx < total) {
                        if (idx < kQCap) {
                            const uint2 en = queue[idx];
                            qv = en.x;
                            pq = __uint_as_float(en.y);
                        } else {
                            // written by other waves of this workgroup: read past the L1
                            const uint64_t en = __hip_atomic_load(gq + (idx - kQCap), __ATOMIC_RELAXED,
                                                                  __HIP_MEMORY_SCOPE_AGENT);
                            qv = static_cast<uint32_t>(en);
                            pq = __uint_as_float(static_cast<uint32_t>(en >> 32));
                        }
                        c = 1;
                        act = true;
                        tl = __uint_as_float(tau[qv >> 5]);
                    }
                }
            }
            const unsigned long long live = __ballot(act);
            if (!live) break;
            if (counters) {
                live_vals += 32ull * __popcll(live);
                lane_vals += 64ull * 32;
            }
            if (act) {
                const int64_t qi = qv >> 5;
                const int vv = qv & 31;
                pq += tile_chunk<L1>(tile, poff + qi * d + c * 32, qperm + qi * d + c * 32, vv);
                if (STATS && !(pq > tl)) atomicAdd(surv + c, 1ull);
                ++c;
                if (pq > tl) {
                    act = false;
                } else if (c == nchunks) {
                    const int64_t sv = (int64_t)t * kTV + vv;
                    cand_append(cand, cand_cnt, cap, qi, pq, (uint32_t)(slot_id ? slot_id[sv] : sv));
                    act = false;
                }
            }
        }
        __syncthreads();  // the tile, the queue and the list are free
    }
    if (counters && lane == 0) {
        atomicAdd(counters, live_vals);
        atomicAdd(counters + 1, lane_vals);
    }
}

int32_t next_pow2(int32_t v) {
    int32_t p = 1;
    while (p < v) p <<= 1;
    return p;
}

constexpr int32_t kCandCap = 2048;     // candidates per query in the tile path
constexpr int32_t kCandCapIp = 65536;  // the inner product's largest (looser START threshold)
constexpr int32_t kRoundsIp = 16;   // the inner product's least (rounds are also bounded by the buffer size)

size_t tile_lds_bytes(int32_t d) { return (size_t)d * kTV * sizeof(float) + kQCap * sizeof(uint2); }

// Largest dynamic LDS a workgroup may request on the current device.
size_t max_dynamic_lds() {
    int dev = 0, optin = 0, plain = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 0;
    if (hipDeviceGetAttribute(&optin, hipDeviceAttributeSharedMemPerBlockOptin, dev) != hipSuccess) optin = 0;
    if (hipDeviceGetAttribute(&plain, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess) plain = 0;
    size_t m = (size_t)(optin > plain ? optin : plain);
    const size_t stat = 64 + kList * sizeof(int32_t);  // room for the kernel's static LDS (scalars, query list)
    return m > stat ? m - stat : 0;
}

bool tile_path(const pdx_index *ix, const ExactPlan &pl) {
    if (pl.metric == PDX_METRIC_IP)  // inner product: the bucket layout's tile bound
        return ix->kind == kIvf && ix->d % 32 == 0 && pl.nq < (int64_t(1) << 27) && pl.tiles_main > 0 &&
               (size_t)ix->d * kTV * sizeof(float) <= max_dynamic_lds();
    // L1 only on the bucket layout, where its centroid bound applies (on the
    // flat layout the vectorgroup path is faster for it)
    return pl.mode == PDX_MODE_BOND && (pl.metric == PDX_METRIC_L2 || (pl.metric == PDX_METRIC_L1 && pl.ivf)) &&
           pl.chunk == 32 && ix->d * kTV < 65536 && ix->d % 32 == 0 && pl.nq < (int64_t(1) << 27) &&
           pl.tiles_main > 0 && tile_lds_bytes(ix->d) <= max_dynamic_lds();
}

// PDX-BOND inside IVF: one wave per (query, probe rank) work item scans
// the item's bucket in the query's BOND order (scan_groups), writing the
// item's k-best list; PRUNE drops a vector once its partial distance
// exceeds the threshold (exact within the probed buckets).  Items are
// grouped by bucket; workgroup ids map to XCD-contiguous ranges of items.
template <bool PRUNE, bool ZONES>
__global__ __launch_bounds__(256) void bond_item_kernel(
    const float *__restrict__ pdxd, const int32_t *__restrict__ slot_id, int32_t d, const int32_t *__restrict__ goff,
    const int2 *__restrict__ items, int64_t nitems, const int32_t *__restrict__ probe, int32_t nprobe,
    const int32_t *__restrict__ perm, const float *__restrict__ qperm, uint32_t *__restrict__ tau,
    const int32_t *__restrict__ bad, SlotMap slots, int32_t chunk, unsigned long long *__restrict__ counters,
    uint32_t nwg, const float *__restrict__ xrow, int32_t zone_rows) {
    const uint32_t per_xcd = gridDim.x >> 3;
    const uint32_t wg = (blockIdx.x & 7) * per_xcd + (blockIdx.x >> 3);
    const int lane = threadIdx.x & 63;
    const int64_t it = (int64_t)wg * 4 + (threadIdx.x >> 6);
    if (wg >= nwg || it >= nitems) return;
    const int2 item = items[it];
    uint64_t *myslot = slots.at(item.x, item.y, 0);
    if (bad[item.x]) {
        if (lane < slots.kk) myslot[lane] = kEmptyKey;
        return;
    }
    const int32_t l = probe[(int64_t)item.x * nprobe + item.y];
    scan_groups<PRUNE, false, ZONES>(pdxd, 0, slot_id, d, goff[l], goff[l + 1], item.x, perm, qperm, tau, myslot,
                                     slots.kk, chunk, counters, xrow, zone_rows);
}

// ---------------------------------------------------------------------------
// Inner product on the bucket layout (tile path).  A partial inner product
// bounds nothing, so a (query, tile) pair is scanned in full once kept; what
// prunes is the tile bound: for x within radius r of its bucket's centroid
// c, q.x <= q.c + |q| r (Cauchy-Schwarz).  Scores are ranked as
// s' = B_q - q.x with B_q a power of two at or above |q| M (1 + 2^-10) and
// M >= every |x| (the largest |c| + r over the tiles), so s' > 0 and the
// non-negative key and threshold machinery of the L2 path applies; the
// result reports s' - B_q.
// Every q.x is summed in the one fixed order of the other metrics (natural
// dimension order, 32-dimension chunks as four octets), so START, the tile
// kernel and the fallback agree bit for bit.
// ---------------------------------------------------------------------------

// |row| of every row of a [m][d] matrix, one wave per row.
__global__ __launch_bounds__(64) void row_norm_kernel(const float *__restrict__ a, int32_t d, float *__restrict__ nrm) {
    const int64_t i = blockIdx.x;
    float s = 0.0f;
    for (int32_t j = threadIdx.x; j < d; j += kWave) s = fmaf(a[i * d + j], a[i * d + j], s);
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off);
    if (threadIdx.x == 0) nrm[i] = sqrtf(s);
}

// M: the largest |c| + r over the stored tiles, rounded up by 2^-20 (float
// bits of a non-negative value order like the value).
__global__ __launch_bounds__(256) void ip_max_norm_kernel(const float *__restrict__ cn,
                                                          const int32_t *__restrict__ group_bucket,
                                                          const float *__restrict__ tile_rad, int32_t ngroups,
                                                          uint32_t *__restrict__ mbits) {
    float m = 0.0f;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < 2 * (int64_t)ngroups;
         t += (int64_t)gridDim.x * blockDim.x)
        m = fmaxf(m, (cn[group_bucket[t >> 1]] + tile_rad[t]) * (1.0f + 0x1p-20f));
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) m = fmaxf(m, __shfl_xor(m, off));
    if ((threadIdx.x & 63) == 0) atomicMax(mbits, __float_as_uint(m));
}

// Per query: |q| and B_q, the power of two at or above |q| M (1 + 2^-10)
// (a power of two keeps B_q - q.x exact wherever q.x is, e.g. on integer
// data, and then s' - B_q gives back -q.x exactly).
__global__ __launch_bounds__(64) void ip_query_kernel(const float *__restrict__ q, int32_t d,
                                                      const uint32_t *__restrict__ mbits, float *__restrict__ qn,
                                                      float *__restrict__ qshift) {
    const int64_t qi = blockIdx.x;
    float s = 0.0f;
    for (int32_t j = threadIdx.x; j < d; j += kWave) s = fmaf(q[qi * d + j], q[qi * d + j], s);
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off);
    if (threadIdx.x == 0) {
        const float n = sqrtf(s) * (1.0f + 0x1p-20f);
        qn[qi] = n;
        int e = 0;
        (void)frexpf(n * __uint_as_float(*mbits) * (1.0f + 0x1p-10f), &e);
        qshift[qi] = ldexpf(1.0f, e);
    }
}

// From cd[q][l] = q.c_l: cd[q][l] becomes B_q - q.c_l (>= 0; its minimum is
// the START bucket), and dql[l][q] = B_q - q.c_l - margin, bucket-major: a
// lower bound of s' over the bucket's rows before the |q| r term.  margin
// covers the float32 rounding of q.c ((D + 8) 2^-24 |q| |c|), of the fixed-
// order q.x ((10 + D/32) 2^-24 |q| M) and of s' itself (2^-23 B_q), twice
// (q.c from the matrix cores: at most about (D + 16) 2^-24 |q| |c|).
__global__ __launch_bounds__(256) void ip_bound_kernel(float *__restrict__ cd, int64_t nq, int32_t nlist, int32_t d,
                                                       const float *__restrict__ qn,
                                                       const float *__restrict__ qshift,
                                                       const float *__restrict__ cn,
                                                       const uint32_t *__restrict__ mbits,
                                                       float *__restrict__ dql) {
    __shared__ float blk[32][33];
    const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;  // 32 x 8
    const int64_t q0 = (int64_t)blockIdx.x * 32;
    const int32_t l0 = blockIdx.y * 32;
    const float m = __uint_as_float(*mbits);
    const float rel = (float)(d + 64) * 0x1p-23f;
    for (int r = ty; r < 32; r += 8) {
        const int64_t q = q0 + r;
        const int32_t l = l0 + tx;
        float v = 0.0f;
        if (q < nq && l < nlist) {
            const float sp = qshift[q] - cd[q * nlist + l];
            cd[q * nlist + l] = fmaxf(sp, 0.0f);
            v = sp - (rel * qn[q] * (cn[l] + m) + 0x1p-22f * qshift[q]);
        }
        blk[r][tx] = v;
    }
    __syncthreads();
    for (int r = ty; r < 32; r += 8) {
        const int32_t l = l0 + r;
        const int64_t q = q0 + tx;
        if (q < nq && l < nlist) dql[(int64_t)l * nq + q] = blk[tx][r];
    }
}

// One wave scans vectorgroups [g0, g1) for query qi (natural order q row
// qrow): s' = B - q.x per row, k-best list to myslot.
__device__ __forceinline__ void ip_groups(const float *__restrict__ pdxd, const int32_t *__restrict__ slot_id,
                                          int32_t d, int32_t g0, int32_t g1, const float *__restrict__ qrow,
                                          float shift, uint64_t *__restrict__ myslot, int32_t k) {
    const int lane = threadIdx.x & 63;
    uint64_t e = kEmptyKey, kth = kEmptyKey;
    for (int32_t g = g0; g < g1; ++g) {
        const int32_t rid = slot_id[(int64_t)g * kGroup + lane];
        const float *gp = pdxd + (int64_t)g * d * kGroup + lane;
        float dot = 0.0f;
        for (int32_t c0 = 0; c0 < d; c0 += 32) {
            float o[4];
#pragma unroll
            for (int gg = 0; gg < 4; ++gg) {
                o[gg] = 0.0f;
#pragma unroll
                for (int u = 8 * gg; u < 8 * gg + 8; ++u)
                    o[gg] = fmaf(qrow[c0 + u], gp[(int64_t)(c0 + u) * kGroup], o[gg]);
            }
            dot += octets(o[0], o[1], o[2], o[3]);
        }
        topk_offer(e, kth, make_key(shift - dot, static_cast<uint32_t>(rid)), rid >= 0, k, lane);
    }
    if (lane < k) myslot[lane] = e;
}

// START for the inner product: the first maxg vectorgroups of the bucket
// with the largest q.c; `parts` waves per query, each its own k-best list.
__global__ __launch_bounds__(256) void ip_start_kernel(const float *__restrict__ pdxd,
                                                       const int32_t *__restrict__ slot_id, int32_t d,
                                                       const int32_t *__restrict__ goff,
                                                       const int32_t *__restrict__ nearest, int64_t nq, int32_t parts,
                                                       int32_t maxg, const float *__restrict__ q,
                                                       const float *__restrict__ qshift,
                                                       const int32_t *__restrict__ bad, uint64_t *__restrict__ slots,
                                                       int32_t k) {
    const int64_t w = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    const int64_t qi = w / parts;
    const int32_t part = (int32_t)(w - qi * parts);
    const int lane = threadIdx.x & 63;
    if (qi >= nq) return;
    uint64_t *myslot = slots + ((size_t)qi * parts + part) * k;
    if (bad[qi]) {
        if (lane < k) myslot[lane] = kEmptyKey;
        return;
    }
    const int32_t l = nearest[qi];
    const int32_t a = goff[l], len = min(goff[l + 1] - a, maxg);
    const int32_t g0 = a + (int32_t)((int64_t)len * part / parts), g1 = a + (int32_t)((int64_t)len * (part + 1) / parts);
    ip_groups(pdxd, slot_id, d, g0, g1, q + qi * d, qshift[qi], myslot, k);
}

// Overflowed queries: every (listed query, group tile) pair in full.
__global__ __launch_bounds__(256) void ip_fallback_kernel(const float *__restrict__ pdxd,
                                                          const int32_t *__restrict__ slot_id, int32_t d,
                                                          int32_t g_end, int32_t tile_groups, int32_t ntiles,
                                                          const int32_t *__restrict__ over_list,
                                                          const int32_t *__restrict__ over_count,
                                                          const float *__restrict__ q,
                                                          const float *__restrict__ qshift,
                                                          uint64_t *__restrict__ slots, int32_t nslots, int32_t k) {
    const int32_t wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int64_t total = (int64_t)(*over_count) * ntiles;
    for (int64_t it = (int64_t)blockIdx.x * 4 + wave; it < total; it += (int64_t)gridDim.x * 4) {
        const int64_t qi = over_list[it / ntiles];
        const int32_t tile = (int32_t)(it % ntiles);
        const int32_t g0 = tile * tile_groups;
        const int32_t g1 = min(g0 + tile_groups, g_end);
        ip_groups(pdxd, slot_id, d, g0, g1, q + qi * d, qshift[qi], slots + ((size_t)qi * nslots + tile) * k, k);
    }
}

// One octet of a chunk (8 consecutive dimensions from j) for the tile's
// adjacent vectors 2p and 2p + 1 (one 8-byte read per dimension, as in
// octet_pair): q.x terms.
__device__ __forceinline__ void octet_pair_ip(const float *__restrict__ tile, int32_t j, float4 q0, float4 q1, int p,
                                              float &a, float &b) {
    const float qv[8] = {q0.x, q0.y, q0.z, q0.w, q1.x, q1.y, q1.z, q1.w};
    float ra[8], rb[8];  // all reads issued before the first product
#pragma unroll
    for (int u = 0; u < 8; ++u) {
        const float2 r = *reinterpret_cast<const float2 *>(tile + (j + u) * kTV + 2 * p);
        ra[u] = r.x;
        rb[u] = r.y;
    }
    a = 0.0f;
    b = 0.0f;
#pragma unroll
    for (int u = 0; u < 8; ++u) {
        a = fmaf(qv[u], ra[u], a);
        b = fmaf(qv[u], rb[u], b);
    }
}

// Tile kernel for the inner product: tiles staged as in tile_kernel; per
// tile the queries whose bound B_q - q.c - margin - |q| r is not above
// their threshold are listed, and each listed query's wave forms q.x for
// the 32 vectors over all chunks (lanes = 16 vector pairs x 4 octets, the
// next chunk's query values prefetched), appending rows with s' within the
// threshold.
__global__ __launch_bounds__(1024) void ip_tile_kernel(
    const float *__restrict__ pdxd, const int32_t *__restrict__ slot_id, int32_t d, int32_t t_begin, int32_t t_end,
    int64_t nq, const float *__restrict__ q, const float *__restrict__ qn, const float *__restrict__ qshift,
    const uint32_t *__restrict__ tau, const int32_t *__restrict__ bad, uint64_t *__restrict__ cand,
    int32_t *__restrict__ cand_cnt, int32_t cap, const float *__restrict__ dql,
    const int32_t *__restrict__ group_bucket, const float *__restrict__ tile_rad,
    unsigned long long *__restrict__ counters, int32_t *__restrict__ tile_ctr) {
    extern __shared__ float4 smem4[];
    float *tile = reinterpret_cast<float *>(smem4);  // [d][32]
    __shared__ int32_t lcount, next_t;
    __shared__ int32_t qlist[kList];
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int pr = lane & 15, oct = lane >> 4;
    const int32_t nchunks = d / 32;
    unsigned long long live_vals = 0, lane_vals = 0;
    for (;;) {  // tiles from the launch's shared counter, as in tile_kernel
        if (threadIdx.x == 0) next_t = t_begin + atomicAdd(tile_ctr, 1);
        __syncthreads();
        const int32_t t = next_t;
        if (t >= t_end) break;
        const float *src = pdxd + (int64_t)(t >> 1) * d * kGroup + (t & 1) * kTV;
        const int32_t nv4 = d * 8;  // non-temporal, as in tile_kernel
        for (int32_t iw = wave * 64; iw < nv4; iw += 1024) {
            const int32_t i = iw + lane;
            __builtin_amdgcn_global_load_lds(src + (int64_t)(i >> 3) * kGroup + (i & 7) * 4,
                                             (lds_void_t *)(tile + (size_t)iw * 4), 16, 0, 2);
        }
        __syncthreads();
        const int64_t vid_a = (int64_t)t * kTV + 2 * pr, vid_b = vid_a + 1;
        const int32_t rid_a = slot_id[vid_a], rid_b = slot_id[vid_b];
        const uint32_t valid_m = pair_mask(rid_a >= 0, rid_b >= 0);
        const int32_t tb = group_bucket[t >> 1];
        const float trad = tile_rad[t];
        for (int64_t q0 = 0; q0 < nq; q0 += kList) {
            __syncthreads();  // the previous list is no longer read
            if (threadIdx.x == 0) lcount = 0;
            __syncthreads();
            const int64_t qt = q0 + threadIdx.x;
            bool keep = false;
            if (threadIdx.x < kList && qt < nq && !bad[qt] && valid_m) {
                const float lb = dql[(int64_t)tb * nq + qt] - qn[qt] * trad;
                const float tq =
                    __uint_as_float(__hip_atomic_load(tau + qt, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
                keep = !(lb > tq);
            }
            const unsigned long long km = __ballot(keep);
            int lb0 = 0;
            if (lane == 0 && km) lb0 = atomicAdd(&lcount, __popcll(km));
            lb0 = __shfl(lb0, 0);
            if (keep) qlist[lb0 + lane_rank(km)] = (int32_t)qt;
            __syncthreads();
            const int32_t cnt = lcount;
            for (int32_t e = wave; e < cnt; e += kTW) {
                const int64_t qi = qlist[e];
                const float *qr = q + qi * d + oct * 8;
                float x = 0.0f;  // this lane's vector: 2 pr in rows 0 and 2, 2 pr + 1 in rows 1 and 3
                auto ip_step = [&](int32_t c, const float4 qc0, const float4 qc1) {
                    float sa, sb;
                    octet_pair_ip(tile, c * 32 + oct * 8, qc0, qc1, pr, sa, sb);
                    x += pair_total(sa, sb);
                };
                // two query-value sets in turn (chunks c and c + 1), so a
                // prefetched set is used where it landed, never copied
                float4 qa0 = *reinterpret_cast<const float4 *>(qr);
                float4 qa1 = *reinterpret_cast<const float4 *>(qr + 4);
                float4 qb0 = qa0, qb1 = qa1;
                for (int32_t c = 0; c < nchunks; c += 2) {
                    if (c + 1 < nchunks) {
                        qb0 = *reinterpret_cast<const float4 *>(qr + (c + 1) * 32);
                        qb1 = *reinterpret_cast<const float4 *>(qr + (c + 1) * 32 + 4);
                    }
                    ip_step(c, qa0, qa1);
                    if (c + 1 == nchunks) break;
                    if (c + 2 < nchunks) {
                        qa0 = *reinterpret_cast<const float4 *>(qr + (c + 2) * 32);
                        qa1 = *reinterpret_cast<const float4 *>(qr + (c + 2) * 32 + 4);
                    }
                    ip_step(c + 1, qb0, qb1);
                }
                if (counters) {
                    live_vals += (unsigned long long)d * __popc(valid_m);
                    lane_vals += 32ull * d;
                }
                const float tq = __uint_as_float(tau[qi]);
                const float sv = qshift[qi] - x;
                const int32_t rid_v = (oct & 1) ? rid_b : rid_a;
                if (oct < 2 && rid_v >= 0 && !(sv > tq)) cand_append(cand, cand_cnt, cap, qi, sv, (uint32_t)rid_v);
            }
        }
        __syncthreads();
    }
    if (counters && lane == 0) {
        atomicAdd(counters, live_vals);
        atomicAdd(counters + 1, lane_vals);
    }
}

// The listed vectors' exact distances (scan_groups' chunk order, natural
// dimension order), written back as keys (distance bits, row id).
__global__ __launch_bounds__(256) void lin_rescore_kernel(const float *__restrict__ pdxd,
                                                         const int32_t *__restrict__ slot_id, int32_t d,
                                                         const int32_t *__restrict__ perm,
                                                         const float *__restrict__ qperm,
                                                         const int32_t *__restrict__ bad, uint64_t *__restrict__ cand,
                                                         const int32_t *__restrict__ cand_cnt, int32_t cap,
                                                         int32_t chunk) {
    const int64_t qi = blockIdx.x;
    if (bad[qi]) return;
    const int32_t cnt = min(cand_cnt[qi], cap);
    const int32_t *po = perm + qi * d;
    const float *qp = qperm + qi * d;
    for (int32_t i = threadIdx.x; i < cnt; i += 256) {
        const uint32_t sv = static_cast<uint32_t>(cand[qi * cap + i]);
        const float *gp = pdxd + (int64_t)(sv / kGroup) * d * kGroup + (sv % kGroup);
        float partial = 0.0f;
        for (int32_t c0 = 0; c0 < d; c0 += chunk) {
            const int32_t c1 = min(c0 + chunk, d);
            partial += (c1 - c0 == 32) ? chunk_sum<true, false>(gp, po, qp, c0, c1)
                                       : chunk_sum<false, false>(gp, po, qp, c0, c1);
        }
        const uint32_t rid = slot_id ? static_cast<uint32_t>(slot_id[sv]) : sv;
        cand[qi * cap + i] = make_key(partial, rid);
    }
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
    pl.ivf = ix->kind == kIvf;
    pl.rounds = (p && p->rounds > 0) ? p->rounds : (pl.ivf ? kDefaultRoundsBuckets : kDefaultRounds);
    pl.dense_min = (p && p->dense_min > 0) ? p->dense_min : kDefaultDenseMin;
    pl.metric = p ? p->metric : PDX_METRIC_L2;
    if (pl.ivf) {
        pl.start_groups = 0;  // START is each query's nearest bucket
    } else if (pl.mode == PDX_MODE_BOND) {
        int32_t sg = (ix->start_rows + kGroup - 1) / kGroup;
        pl.start_groups = sg < ix->ngroups ? sg : ix->ngroups;
    } else {
        pl.start_groups = 0;
    }
    pl.tiles_start = (pl.start_groups + pl.tile_groups - 1) / pl.tile_groups;
    pl.tiles_main = (ix->ngroups - pl.start_groups + pl.tile_groups - 1) / pl.tile_groups;
    pl.nslots = pl.tiles_start + pl.tiles_main;
    pl.use_tiles = tile_path(ix, pl);
    size_t q = static_cast<size_t>(nq > 0 ? nq : 0);
    Carver c(ws);
    pl.tau = c.take<uint32_t>(q);
    pl.bad = c.take<int32_t>(q);
    pl.perm = c.take<int32_t>(q * ix->d);
    pl.qperm = c.take<float>(q * ix->d);
    const bool ip_tiles = pl.metric == PDX_METRIC_IP && pl.use_tiles;
    pl.slots = (pl.metric == PDX_METRIC_IP && !ip_tiles) ? nullptr : c.take<uint64_t>(q * pl.nslots * k);
    if (pl.ivf) {
        // START: the first start_rows rows (whole vectorgroups) of the
        // nearest bucket; waves per query about 8 per SIMD in all, at most
        // one per vectorgroup
        const int32_t sr = (p && p->start_rows > 0) ? p->start_rows : 128;
        pl.start_maxg = (int32_t)std::min<int64_t>(((int64_t)sr + kGroup - 1) / kGroup, ix->ngroups);
        int32_t sp = 1;
        while (sp < 16 && sp < pl.start_maxg && (int64_t)sp * nq < 8 * 4 * (int64_t)device_cus()) sp <<= 1;
        pl.start_parts = sp;
        pl.qrot = ix->has_rot ? c.take<float>(q * ix->d) : nullptr;
        const bool bstart = pl.mode == PDX_MODE_BOND || ip_tiles;  // START on the nearest bucket
        pl.cd = bstart ? c.take<float>(q * ix->nlist) : nullptr;
        pl.dql = bstart ? c.take<float>(q * ix->nlist) : nullptr;
        pl.nearest = bstart ? c.take<int32_t>(q) : nullptr;
        pl.start_slots = bstart ? c.take<uint64_t>(q * pl.start_parts * k) : nullptr;
        if (bstart) {  // norms: |q| and |c| (inner product) or their squares (L2 centroid distances)
            pl.qn = c.take<float>(q);
            pl.cn = c.take<float>(ix->nlist);
        }
        if (ip_tiles) {
            pl.qshift = c.take<float>(q);
            pl.mbits = c.take<uint32_t>(64);
        }
    }
    if (pl.use_tiles) {
        pl.poff = ip_tiles ? nullptr : c.take<uint16_t>(q * ix->d);
        const int32_t cus = device_cus();
        pl.tile_grid = cus;  // one workgroup per compute unit (the LDS tile fills the CU)
        pl.gqueue = c.take<uint64_t>((size_t)cus * kGCap);
        pl.tile_ctr = c.take<int32_t>(kMaxTileRounds);
        if (ip_tiles) {  // about 1 GiB of buffers at most; fewer entries mean more rounds
            const int64_t fit = ((int64_t)1 << 30) / (int64_t)sizeof(uint64_t) / std::max<int64_t>(nq, 1);
            pl.cand_cap = (int32_t)std::max<int64_t>(4096, std::min<int64_t>(kCandCapIp, fit / 64 * 64));
        } else {
            pl.cand_cap = kCandCap;
        }
        pl.cand = c.take<uint64_t>(q * pl.cand_cap);
        pl.cand_cnt = c.take<int32_t>(q);
        pl.over_list = c.take<int32_t>(q);
        pl.over_count = c.take<int32_t>(64);
    }
    if (pl.metric == PDX_METRIC_IP && !ip_tiles) {
        pl.ip_parts = ip_parts_for(nq, ix->ngroups, ix->d);
        pl.ip_slots = c.take<uint64_t>(q * pl.ip_parts * k);
    }
    // L2 linear mode on the matrix cores (the vectorgroup path when the
    // counters are asked for, or D is not a multiple of 4)
    pl.lin_mx = pl.mode == PDX_MODE_LINEAR && pl.metric == PDX_METRIC_L2 && ix->d % 4 == 0 &&
                !(p && (p->counters || p->chunk_survivors));
    if (pl.lin_mx) {
        pl.ip_parts = lin_bound_parts(nq, ix->ngroups);
        pl.lin_mins = c.take<float>(q * pl.ip_parts * 16);
        pl.qn = c.take<float>(q);
        pl.cand_cap = kCandCap;
        pl.cand = c.take<uint64_t>(q * pl.cand_cap);
        pl.cand_cnt = c.take<int32_t>(q);
        pl.over_list = c.take<int32_t>(q);
        pl.over_count = c.take<int32_t>(64);
    }
    pl.events = p ? reinterpret_cast<hipEvent_t *>(p->phase_events) : nullptr;
    pl.counters = p ? p->counters : nullptr;
    pl.surv = (p && pl.mode == PDX_MODE_BOND) ? p->chunk_survivors : nullptr;
    if (plan) *plan = pl;
    return c.bytes();
}

// Inner product on the bucket layout: bound inputs, START on the first rows
// of the bucket with the largest q.c, rounds of tiles with the threshold refreshed in between,
// the full scan for overflowed queries, and the k best with the shift undone.
template <typename Mark>
hipError_t run_ip_tiles(const pdx_index *ix, const float *qs, const ExactPlan &pl, int64_t *out_ids,
                        float *out_dist, hipStream_t s, Mark &mark) {
    const int32_t d = ix->d;
    const unsigned nqu = (unsigned)pl.nq;
    hipError_t err;
    row_norm_kernel<<<(unsigned)ix->nlist, 64, 0, s>>>(ix->centroids, d, pl.cn);
    if ((err = launch_fill_i32(reinterpret_cast<int32_t *>(pl.mbits), 1, 0, s)) != hipSuccess) return err;
    ip_max_norm_kernel<<<256, 256, 0, s>>>(pl.cn, ix->group_bucket, ix->tile_rad, ix->ngroups, pl.mbits);
    ip_query_kernel<<<nqu, 64, 0, s>>>(qs, d, pl.mbits, pl.qn, pl.qshift);
    if ((err = hipGetLastError()) != hipSuccess) return err;
    // q.c on the matrix cores, a library GEMM unless the caller cannot
    // allocate (the rounding of a D-term dot product in any summation order
    // is within ip_bound_kernel's margin)
    if ((err = (pl.library_gemm ? launch_sgemm_abt : launch_gemm_abt)(qs, pl.nq, ix->centroids, ix->nlist, d, pl.cd,
                                                                      ix->nlist, s)) != hipSuccess)
        return err;
    ip_bound_kernel<<<dim3((unsigned)((pl.nq + 31) / 32), (unsigned)((ix->nlist + 31) / 32)), 256, 0, s>>>(
        pl.cd, pl.nq, ix->nlist, d, pl.qn, pl.qshift, pl.cn, pl.mbits, pl.dql);
    nearest_kernel<<<nqu, 64, 0, s>>>(pl.cd, ix->nlist, pl.nearest);
    const int64_t waves = pl.nq * pl.start_parts;
    ip_start_kernel<<<(unsigned)((waves + 3) / 4), 256, 0, s>>>(ix->pdx, ix->slot_id, d, ix->list_goff, pl.nearest,
                                                                pl.nq, pl.start_parts, pl.start_maxg, qs, pl.qshift,
                                                                pl.bad, pl.start_slots, pl.k);
    merge_kernel<<<nqu, 64, 0, s>>>(pl.start_slots, pl.start_parts, 0, pl.start_parts, pl.k, pl.bad, pl.tau, nullptr,
                                    nullptr, nullptr, nullptr, 0);
    if ((err = hipGetLastError()) != hipSuccess) return err;
    if ((err = launch_fill_i32(pl.cand_cnt, pl.nq, 0, s)) != hipSuccess) return err;
    if ((err = mark(1)) != hipSuccess) return err;
    const size_t lds = (size_t)d * kTV * sizeof(float);
    if (lds > 64 * 1024 &&
        (err = hipFuncSetAttribute(reinterpret_cast<const void *>(ip_tile_kernel),
                                   hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds)) != hipSuccess)
        return err;
    unsigned long long *cmain = pl.counters ? pl.counters + 2 : nullptr;
    // rounds of at most cap - k rows each: with the buffer compacted to its k
    // best between rounds no buffer can overflow (the full scan stays as the
    // guard)
    const int32_t t1 = 2 * ix->ngroups;
    const int64_t tiles_per_round = std::max<int64_t>(1, (pl.cand_cap - pl.k) / kTV);
    const int32_t rounds = (int32_t)std::max<int64_t>(kRoundsIp, (t1 + tiles_per_round - 1) / tiles_per_round);
    for (int32_t r = 0; r < rounds; ++r) {
        const int32_t a = (int32_t)((int64_t)t1 * r / rounds), b = (int32_t)((int64_t)t1 * (r + 1) / rounds);
        if (b <= a) continue;
        const unsigned grid = (unsigned)min(b - a, pl.tile_grid);
        if ((err = launch_fill_i32(pl.tile_ctr, 1, 0, s)) != hipSuccess) return err;
        ip_tile_kernel<<<grid, 1024, lds, s>>>(ix->pdx, ix->slot_id, d, a, b, pl.nq, qs, pl.qn, pl.qshift, pl.tau,
                                               pl.bad, pl.cand, pl.cand_cnt, pl.cand_cap, pl.dql, ix->group_bucket,
                                               ix->tile_rad, cmain, pl.tile_ctr);
        if ((err = hipGetLastError()) != hipSuccess) return err;
        if (r + 1 < rounds) {
            cand_merge_kernel<<<nqu, 64, 0, s>>>(pl.cand, pl.cand_cnt, pl.cand_cap, 0, pl.k, pl.bad, pl.tau, nullptr, 0,
                                                 0, 0, nullptr, nullptr, nullptr, 1);
            if ((err = hipGetLastError()) != hipSuccess) return err;
        }
    }
    if ((err = launch_fill_i32(pl.over_count, 1, 0, s)) != hipSuccess) return err;
    over_list_kernel<<<(nqu + 255) / 256, 256, 0, s>>>(pl.cand_cnt, pl.nq, pl.cand_cap, pl.over_list, pl.over_count);
    ip_fallback_kernel<<<2048, 256, 0, s>>>(ix->pdx, ix->slot_id, d, ix->ngroups, pl.tile_groups, pl.tiles_main,
                                            pl.over_list, pl.over_count, qs, pl.qshift, pl.slots, pl.nslots, pl.k);
    if ((err = hipGetLastError()) != hipSuccess) return err;
    if ((err = mark(2)) != hipSuccess) return err;
    // an overflowed query keeps nothing of its buffer: the full scan covers every row
    cand_merge_kernel<<<nqu, 64, 0, s>>>(pl.cand, pl.cand_cnt, pl.cand_cap, 0, pl.k, pl.bad, pl.tau, pl.slots, pl.nslots,
                                         0, pl.tiles_main, out_ids, out_dist, pl.qshift, 0);
    if ((err = hipGetLastError()) != hipSuccess) return err;
    return mark(3);
}

hipError_t run_exact(const pdx_index *ix, const float *q, const ExactPlan &pl, int64_t *out_ids,
                     float *out_dist, hipStream_t s) {
    const int32_t d = ix->d;
    const int32_t pow2 = next_pow2(d);
    size_t lds = pow2 * sizeof(uint64_t) + d * sizeof(float);
    auto mark = [&](int i) { return pl.events ? hipEventRecord(pl.events[i], s) : hipSuccess; };
    hipError_t err;
    if ((err = mark(0)) != hipSuccess) return err;
    const int32_t *sid = pl.ivf ? ix->slot_id : nullptr;  // slot -> row id on the bucket layout
    const float *qs = q;
    if (pl.ivf && ix->has_rot) {  // the bucket layout stores rotated rows
        if ((err = launch_gemm_abt(q, pl.nq, ix->rot, d, d, pl.qrot, d, s)) != hipSuccess) return err;
        qs = pl.qrot;
    }
    prep_kernel<<<dim3((unsigned)pl.nq), dim3(256), lds, s>>>(qs, d, ix->means, pl.mode, pow2, pl.perm,
                                                              pl.qperm, pl.tau, pl.bad, pl.use_tiles ? pl.poff : nullptr);
    if ((err = hipGetLastError()) != hipSuccess) return err;
    if (pl.metric == PDX_METRIC_IP && pl.use_tiles) return run_ip_tiles(ix, qs, pl, out_ids, out_dist, s, mark);
    if (pl.metric == PDX_METRIC_IP) {  // linear inner-product scan on the matrix cores
        if ((err = mark(1)) != hipSuccess) return err;
        if ((err = launch_ip_scan(ix, qs, pl.nq, pl.bad, pl.ip_parts, pl.ip_slots, pl.k, s)) != hipSuccess)
            return err;
        if ((err = mark(2)) != hipSuccess) return err;
        if ((err = launch_ip_merge(pl.ip_slots, pl.nq, pl.ip_parts, pl.k, pl.bad, out_ids, out_dist, s)) !=
            hipSuccess)
            return err;
        return mark(3);
    }
    if (pl.lin_mx) {
        const unsigned nqu = (unsigned)pl.nq;
        if ((err = mark(1)) != hipSuccess) return err;
        row_sq_kernel<<<nqu, 64, 0, s>>>(qs, d, pl.qn);
        // the bound from every 8th vectorgroup, then the listing pass
        if ((err = launch_lin_bound(ix, sid, qs, pl.nq, pl.qn, pl.bad, pl.ip_parts, 8, pl.lin_mins, pl.k, pl.tau, s)) !=
            hipSuccess)
            return err;
        if ((err = launch_fill_i32(pl.cand_cnt, pl.nq, 0, s)) != hipSuccess) return err;
        if ((err = launch_lin_list(ix, sid, qs, pl.nq, pl.qn, pl.bad, pl.tau, pl.cand, pl.cand_cnt, pl.cand_cap, s)) !=
            hipSuccess)
            return err;
        lin_rescore_kernel<<<nqu, 256, 0, s>>>(ix->pdx, sid, d, pl.perm, pl.qperm, pl.bad, pl.cand, pl.cand_cnt,
                                             pl.cand_cap, pl.chunk);
        if ((err = hipGetLastError()) != hipSuccess) return err;
        // a query whose list overflowed: the vectorgroup path over every row,
        // pruned by the same bound
        if ((err = launch_fill_i32(pl.over_count, 1, 0, s)) != hipSuccess) return err;
        over_list_kernel<<<(nqu + 255) / 256, 256, 0, s>>>(pl.cand_cnt, pl.nq, pl.cand_cap, pl.over_list,
                                                            pl.over_count);
        fallback_kernel<false><<<2048, 256, 0, s>>>(ix->pdx, ix->n, sid, d, 0, ix->ngroups, pl.tile_groups,
                                                    pl.tiles_main, pl.over_list, pl.over_count, pl.perm, pl.qperm,
                                                    pl.tau, pl.slots, pl.nslots, pl.tiles_start, pl.k, pl.chunk,
                                                    nullptr);
        if ((err = hipGetLastError()) != hipSuccess) return err;
        if ((err = mark(2)) != hipSuccess) return err;
        cand_merge_kernel<<<nqu, 64, 0, s>>>(pl.cand, pl.cand_cnt, pl.cand_cap, 0, pl.k, pl.bad, pl.tau, pl.slots,
                                             pl.nslots, pl.tiles_start, pl.tiles_main, out_ids, out_dist, nullptr, 0);
        if ((err = hipGetLastError()) != hipSuccess) return err;
        return mark(3);
    }
    const bool l1 = pl.metric == PDX_METRIC_L1;
    const int32_t nqb = (int32_t)((pl.nq + pl.qpb - 1) / pl.qpb);
    auto scan = [&](bool prune, int32_t gb, int32_t ge, int32_t ntiles, int32_t slot0, unsigned long long *cnt) {
        unsigned grid = 8u * (unsigned)((ntiles + 7) / 8) * (unsigned)nqb;
        dim3 block(64 * pl.qpb);
#define PDX_GROUP_SCAN(P, M)                                                                                   \
    scan_kernel<P, M><<<grid, block, 0, s>>>(ix->pdx, ix->n, sid, d, gb, ge, pl.tile_groups, ntiles, nqb, pl.nq, \
                                             pl.qpb, pl.perm, pl.qperm, pl.tau, pl.bad, pl.slots, pl.nslots,     \
                                             slot0, pl.k, pl.chunk, cnt, P ? pl.surv : nullptr)
        if (prune) {
            if (l1) PDX_GROUP_SCAN(true, true);
            else PDX_GROUP_SCAN(true, false);
        } else {
            if (l1) PDX_GROUP_SCAN(false, true);
            else PDX_GROUP_SCAN(false, false);
        }
#undef PDX_GROUP_SCAN
        return hipGetLastError();
    };
    const unsigned nqu = (unsigned)pl.nq;
    if (pl.ivf && pl.mode == PDX_MODE_BOND) {
        // START on the nearest bucket: its k-th distance is the initial
        // threshold (its rows are found again by the main scan)
        // centroid distances in the search's metric: L1 on the vector ALU;
        // L2 as a lower bound from matrix-core products (expanded form)
        if (l1) {
            if ((err = launch_pair(2, 0, qs, pl.nq, ix->centroids, ix->nlist, d, pl.cd, ix->nlist, nullptr, s)) !=
                hipSuccess)
                return err;
        } else {
            row_sq_kernel<<<nqu, 64, 0, s>>>(qs, d, pl.qn);
            row_sq_kernel<<<(unsigned)ix->nlist, 64, 0, s>>>(ix->centroids, d, pl.cn);
            if ((err = hipGetLastError()) != hipSuccess) return err;
            // q.c as a library GEMM unless the caller cannot allocate (any
            // summation order is within the lower bound's margin)
            if ((err = (pl.library_gemm ? launch_sgemm_abt : launch_gemm_abt)(qs, pl.nq, ix->centroids, ix->nlist,
                                                                              d, pl.cd, ix->nlist, s)) != hipSuccess)
                return err;
            const int64_t pairs = pl.nq * ix->nlist;
            l2_from_dot_kernel<<<(unsigned)((pairs + 255) / 256), 256, 0, s>>>(pl.cd, pl.nq, ix->nlist, d, pl.qn,
                                                                               pl.cn);
        }
        nearest_kernel<<<nqu, 64, 0, s>>>(pl.cd, ix->nlist, pl.nearest);
        centroid_lo_kernel<<<dim3((unsigned)((pl.nq + 31) / 32), (unsigned)((ix->nlist + 31) / 32)), 256, 0, s>>>(
            pl.cd, pl.nq, ix->nlist, pl.dql, l1 ? 1 : 0);
        const int64_t waves = pl.nq * pl.start_parts;
        if (l1)
            start_bucket_kernel<true><<<(unsigned)((waves + 3) / 4), 256, 0, s>>>(
                ix->pdx, ix->slot_id, d, ix->list_goff, pl.nearest, pl.nq, pl.start_parts, pl.start_maxg, pl.perm, pl.qperm,
                pl.tau, pl.bad, pl.start_slots, pl.k, pl.chunk, pl.counters);
        else
            start_bucket_kernel<false><<<(unsigned)((waves + 3) / 4), 256, 0, s>>>(
                ix->pdx, ix->slot_id, d, ix->list_goff, pl.nearest, pl.nq, pl.start_parts, pl.start_maxg, pl.perm, pl.qperm,
                pl.tau, pl.bad, pl.start_slots, pl.k, pl.chunk, pl.counters);
        merge_kernel<<<nqu, 64, 0, s>>>(pl.start_slots, pl.start_parts, 0, pl.start_parts, pl.k, pl.bad, pl.tau,
                                        nullptr, nullptr, nullptr, nullptr, 0);
        if ((err = hipGetLastError()) != hipSuccess) return err;
        if (pl.use_tiles && (err = launch_fill_i32(pl.cand_cnt, pl.nq, 0, s)) != hipSuccess) return err;
    }
    if (pl.tiles_start > 0) {
        // START (Section 4, PHASE 0): the first block without pruning, then
        // its k-th distance becomes the initial threshold.
        if ((err = scan(false, 0, pl.start_groups, pl.tiles_start, 0, pl.counters)) != hipSuccess) return err;
        merge_kernel<<<nqu, 64, 0, s>>>(pl.slots, pl.nslots, 0, pl.tiles_start, pl.k, pl.bad, pl.tau, nullptr,
                                        nullptr, pl.use_tiles ? pl.cand : nullptr, pl.cand_cnt, pl.cand_cap);
        if ((err = hipGetLastError()) != hipSuccess) return err;
    }
    if ((err = mark(1)) != hipSuccess) return err;
    unsigned long long *cmain = pl.counters ? pl.counters + 2 : nullptr;
    if (!pl.use_tiles) {
        if (pl.tiles_main > 0) {
            bool prune = pl.mode == PDX_MODE_BOND;
            if ((err = scan(prune, pl.start_groups, ix->ngroups, pl.tiles_main, pl.tiles_start, cmain)) != hipSuccess)
                return err;
        }
        if ((err = mark(2)) != hipSuccess) return err;
        merge_kernel<<<nqu, 64, 0, s>>>(pl.slots, pl.nslots, 0, pl.nslots, pl.k, pl.bad, nullptr, out_ids, out_dist,
                                        nullptr, nullptr, 0);
        if ((err = hipGetLastError()) != hipSuccess) return err;
        return mark(3);
    }
    // tile path: rounds of 32-vector tiles, threshold refreshed in between
    const size_t tile_lds = tile_lds_bytes(d);
    // kernel: the centroid bound and dense pairs on the bucket layout (the
    // tile radii in the search's metric); on the flat layout every query
    // meets every tile
    const bool st = pl.surv != nullptr;  // instrumentation build of the kernel
    const void *tk;
#define PDX_TILE_FN(DN, M)                                                         \
    (st ? reinterpret_cast<const void *>(tile_kernel<DN, M, true, kTileWaves>) \
        : reinterpret_cast<const void *>(tile_kernel<DN, M, false, kTileWaves>))
    if (pl.ivf) tk = l1 ? PDX_TILE_FN(true, true) : PDX_TILE_FN(true, false);
    else tk = l1 ? PDX_TILE_FN(false, true) : PDX_TILE_FN(false, false);
#undef PDX_TILE_FN
    if (tile_lds > 64 * 1024) {
        if ((err = hipFuncSetAttribute(tk, hipFuncAttributeMaxDynamicSharedMemorySize, (int)tile_lds)) != hipSuccess)
            return err;
    }
    const int32_t t0 = 2 * pl.start_groups, t1 = 2 * ix->ngroups;
    const int cus = pl.tile_grid;
    const float *trad = pl.ivf ? (l1 ? ix->tile_rad1 : ix->tile_rad) : nullptr;
    const int32_t rounds = pl.rounds;
    if ((err = launch_fill_i32(pl.tile_ctr, rounds, 0, s)) != hipSuccess) return err;
    for (int32_t r = 0; r < rounds; ++r) {
        const int32_t a = t0 + (int32_t)((int64_t)(t1 - t0) * r / rounds);
        const int32_t b = t0 + (int32_t)((int64_t)(t1 - t0) * (r + 1) / rounds);
        if (b <= a) continue;
        const unsigned grid = (unsigned)min(b - a, cus);
#define PDX_TILE(DN, M, ST)                                                                                      \
    tile_kernel<DN, M, ST, kTileWaves><<<grid, kTileWaves * 64, tile_lds, s>>>(ix->pdx, ix->n, sid, d, a, b, pl.nq, pl.poff, pl.qperm,     \
                                                        pl.tau, pl.bad, pl.cand, pl.cand_cnt, pl.cand_cap, pl.gqueue, \
                                                        cmain, DN ? pl.dql : nullptr, DN ? ix->group_bucket : nullptr, \
                                                        trad, pl.tile_ctr + r, pl.surv, pl.dense_min)
        if (st) {
            if (pl.ivf) {
                if (l1) PDX_TILE(true, true, true);
                else PDX_TILE(true, false, true);
            } else {
                if (l1) PDX_TILE(false, true, true);
                else PDX_TILE(false, false, true);
            }
        } else if (pl.ivf) {
            if (l1) PDX_TILE(true, true, false);
            else PDX_TILE(true, false, false);
        } else {
            if (l1) PDX_TILE(false, true, false);
            else PDX_TILE(false, false, false);
        }
#undef PDX_TILE
        if ((err = hipGetLastError()) != hipSuccess) return err;
        if (r + 1 < rounds) {
            cand_merge_kernel<<<nqu, 64, 0, s>>>(pl.cand, pl.cand_cnt, pl.cand_cap, 0, pl.k, pl.bad, pl.tau, nullptr, 0,
                                                 0, 0, nullptr, nullptr, nullptr, pl.ivf ? 1 : 0);
            if ((err = hipGetLastError()) != hipSuccess) return err;
        }
    }
    // queries whose buffer overflowed: group path over the main range
    if ((err = launch_fill_i32(pl.over_count, 1, 0, s)) != hipSuccess) return err;
    over_list_kernel<<<(nqu + 255) / 256, 256, 0, s>>>(pl.cand_cnt, pl.nq, pl.cand_cap, pl.over_list, pl.over_count);
    if (l1)
        fallback_kernel<true><<<2048, 256, 0, s>>>(ix->pdx, ix->n, sid, d, pl.start_groups, ix->ngroups,
                                                   pl.tile_groups, pl.tiles_main, pl.over_list, pl.over_count,
                                                   pl.perm, pl.qperm, pl.tau, pl.slots, pl.nslots, pl.tiles_start,
                                                   pl.k, pl.chunk, pl.surv);
    else
        fallback_kernel<false><<<2048, 256, 0, s>>>(ix->pdx, ix->n, sid, d, pl.start_groups, ix->ngroups,
                                                    pl.tile_groups, pl.tiles_main, pl.over_list, pl.over_count,
                                                    pl.perm, pl.qperm, pl.tau, pl.slots, pl.nslots, pl.tiles_start,
                                                    pl.k, pl.chunk, pl.surv);
    if ((err = hipGetLastError()) != hipSuccess) return err;
    if ((err = mark(2)) != hipSuccess) return err;
    // an overflowed buffer's head: START's k best on the flat layout (rows
    // before the main range); on the bucket layout START's rows lie inside
    // the main range and the fallback finds them again, so nothing is kept
    const int32_t head = pl.ivf ? 0 : pl.k;
    cand_merge_kernel<<<nqu, 64, 0, s>>>(pl.cand, pl.cand_cnt, pl.cand_cap, head, pl.k, pl.bad, pl.tau, pl.slots,
                                         pl.nslots, pl.tiles_start, pl.tiles_main, out_ids, out_dist, nullptr, 0);
    if ((err = hipGetLastError()) != hipSuccess) return err;
    return mark(3);
}

// ---------------------------------------------------------------------------
// PDX-BOND inside IVF (pdx_search_ivf with the BOND bound)
// ---------------------------------------------------------------------------
hipError_t launch_bond_prep(const float *q, int64_t nq, int32_t d, const float *means, bool zones, int32_t *perm,
                            float *qperm, uint32_t *tau, int32_t *bad, hipStream_t s) {
    if (nq <= 0) return hipSuccess;
    const int32_t pow2 = next_pow2(d);
    const size_t lds = pow2 * sizeof(uint64_t) + d * sizeof(float);
    prep_kernel<<<dim3((unsigned)nq), dim3(256), lds, s>>>(q, d, means, zones ? kModeZones : PDX_MODE_BOND, pow2,
                                                           perm, qperm, tau, bad, nullptr);
    return hipGetLastError();
}

// The visit order of pdx_query_order: the searches' own query preparation
// (rotation of a rotated bucket layout, then prep_kernel with the index's
// means).  order: PDX_ORDER_* (the prep_kernel modes).
hipError_t launch_query_order(const pdx_index *ix, const float *q, int64_t nq, int32_t order, float *qrot,
                              int32_t *perm, float *qval, uint16_t *off, uint32_t *tau, int32_t *bad,
                              hipStream_t s) {
    if (nq <= 0) return hipSuccess;
    const int32_t d = ix->d;
    const float *qs = q;
    if (ix->kind == kIvf && ix->has_rot) {
        const hipError_t err = launch_gemm_abt(q, nq, ix->rot, d, d, qrot, d, s);
        if (err != hipSuccess) return err;
        qs = qrot;
    }
    const int32_t pow2 = next_pow2(d);
    const size_t lds = pow2 * sizeof(uint64_t) + d * sizeof(float);
    const int32_t mode = order == PDX_ORDER_ZONES ? kModeZones : (order == PDX_ORDER_BOND ? PDX_MODE_BOND : PDX_MODE_LINEAR);
    prep_kernel<<<dim3((unsigned)nq), dim3(256), lds, s>>>(qs, d, ix->means, mode, pow2, perm, qval, tau, bad, off);
    return hipGetLastError();
}

int32_t bond_zone_rows(int32_t d, int32_t requested) {
    if (d % 4 != 0 || requested < 0) return 0;  // row-major zone reads need 16-byte aligned rows
    return requested == 0 ? 32 : requested;
}

hipError_t launch_bond_items(bool prune, const pdx_index *ix, const int2 *items, int64_t nitems,
                             const int32_t *probe, int32_t nprobe, const int32_t *perm, const float *qperm,
                             uint32_t *tau, const int32_t *bad, SlotMap slots, int32_t chunk,
                             unsigned long long *counters, bool zones, int32_t zone_rows, hipStream_t s) {
    if (nitems <= 0) return hipSuccess;
    const uint32_t nwg = (uint32_t)((nitems + 3) / 4);
    const unsigned grid = 8u * ((nwg + 7u) / 8u);
    const int32_t zr = zones ? zone_rows : 0;
#define PDX_BOND_ITEMS(P, Z)                                                                                       \
    bond_item_kernel<P, Z><<<grid, 256, 0, s>>>(ix->pdx, ix->slot_id, ix->d, ix->list_goff, items, nitems, probe, \
                                                nprobe, perm, qperm, tau, bad, slots, chunk, counters, nwg, ix->xrow, zr)
    if (prune) {
        if (zones) PDX_BOND_ITEMS(true, true);
        else PDX_BOND_ITEMS(true, false);
    } else {
        PDX_BOND_ITEMS(false, false);  // no pruning: every lane stays live, zones change only the order
    }
#undef PDX_BOND_ITEMS
    return hipGetLastError();
}

}  // namespace pdx
