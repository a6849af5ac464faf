// The IVF search's re-rank of more than PDX_MAX_K candidates: the
// candidate buffer's set-up, its compaction to the R best keys, and the
// exact f32 re-rank of those R followed by the k best.
//
// A query's R best by the scanned distance are its R smallest keys
// (distance bits << 32 | row id: the (distance, id) order).  They are found
// by a radix select over the buffer (11-bit digits from the top, one
// histogram in LDS per pass, early exit once every key sharing the chosen
// prefix is selected); keys are unique per query (each probed row is
// scanned once), so "every key <= the threshold" is exactly R keys.
#include "pdx_internal.h"
#include "wave_topk.h"

namespace pdx {
namespace {

constexpr int kSelThreads = 256;
constexpr int kSelBits = 11;
constexpr int kSelBins = 1 << kSelBits;
constexpr int kSelPer = kSelBins / kSelThreads;

__global__ __launch_bounds__(256) void wide_init_kernel(WideSink w, const float *__restrict__ cd, int32_t nlist,
                                                        const int32_t *__restrict__ probe, int32_t rounds) {
    const int64_t q = blockIdx.x;
    for (int b = threadIdx.x; b < kWideBins; b += blockDim.x) w.hist[q * kWideBins + b] = 0u;
    for (int r = threadIdx.x; r < w.nprobe; r += blockDim.x) w.resume[q * w.nprobe + r] = -1;
    if (threadIdx.x == 0) {
        w.cnt[q] = 0;
        w.over[q] = 0;
        // bins centred on the farthest probed centroid's distance: the
        // window covers it times 2^-8 .. 2^8
        float far = cd[q * nlist + probe[q * w.nprobe + w.nprobe - 1]];
        if (!(far > 0.0f) || !isfinite(far)) far = 0.0f;
        w.hbase[q] = max(0, (int)(__float_as_uint(far) >> 17) - kWideBins / 2);
    }
    if (q == 0)
        for (int i = threadIdx.x; i <= rounds; i += blockDim.x) w.ocnt[i] = 0;
}

// Keeps each listed query's R best keys at the front of its buffer
// (list_round < 0: every query, the final pass, which also pads with empty
// keys up to R).  Otherwise the query's tau drops to just above its R-th
// distance (keys at that distance with a smaller id may still enter) and
// its items can resume.
__global__ __launch_bounds__(kSelThreads) void wide_select_kernel(WideSink w, int32_t list_round,
                                                                  uint32_t *__restrict__ tau) {
    extern __shared__ uint64_t sel[];  // [w.r]
    __shared__ uint32_t hist[kSelBins];
    __shared__ uint32_t tsum[kSelThreads];
    __shared__ uint32_t s_digit, s_below, s_cnt, s_n, s_real;
    __shared__ unsigned long long s_max;
    const int tid = threadIdx.x;
    const bool fin = list_round < 0;
    const int64_t nitems = fin ? w.nq : (int64_t)w.ocnt[list_round];
    const int32_t *list = fin ? nullptr : w.olist + (int64_t)(list_round & 1) * w.nq;
    for (int64_t it = blockIdx.x; it < nitems; it += gridDim.x) {
        const int64_t q = fin ? it : list[it];
        uint64_t *row = w.buf + q * (int64_t)w.cap;
        const int32_t n = min(w.cnt[q], w.cap);
        if (tid == 0) {
            s_real = 0;
            s_n = 0;
            s_max = 0;
        }
        __syncthreads();
        uint32_t real = 0;
        for (int32_t i = tid; i < n; i += kSelThreads) real += row[i] != kEmptyKey;
        atomicAdd(&s_real, real);
        __syncthreads();
        const uint32_t total = s_real;
        uint64_t t = kEmptyKey - 1;  // every real key
        if (total > (uint32_t)w.r) {
            uint64_t prefix = 0;
            int known = 0;
            uint32_t need = (uint32_t)w.r;
            for (;;) {
                const int db = min(kSelBits, 64 - known), sh = 64 - known - db;
                for (int b = tid; b < kSelBins; b += kSelThreads) hist[b] = 0u;
                __syncthreads();
                for (int32_t i = tid; i < n; i += kSelThreads) {
                    const uint64_t key = row[i];
                    if (known == 0 || (key >> (64 - known)) == (prefix >> (64 - known)))
                        atomicAdd(&hist[(uint32_t)(key >> sh) & ((1u << db) - 1u)], 1u);
                }
                __syncthreads();
                uint32_t mine = 0;
#pragma unroll
                for (int b = 0; b < kSelPer; ++b) mine += hist[tid * kSelPer + b];
                tsum[tid] = mine;
                __syncthreads();
                if (tid == 0) {
                    uint32_t acc = 0;
                    for (int i = 0; i < kSelThreads; ++i) {
                        const uint32_t v = tsum[i];
                        tsum[i] = acc;
                        acc += v;
                    }
                }
                __syncthreads();
                const uint32_t before = tsum[tid];
                if (before < need && need <= before + mine) {
                    uint32_t c = before;
                    for (int b = 0; b < kSelPer; ++b) {
                        const uint32_t h = hist[tid * kSelPer + b];
                        if (c + h >= need) {
                            s_digit = (uint32_t)(tid * kSelPer + b);
                            s_below = c;
                            s_cnt = h;
                            break;
                        }
                        c += h;
                    }
                }
                __syncthreads();
                need -= s_below;
                prefix |= (uint64_t)s_digit << sh;
                known += db;
                const bool done = s_cnt == need || known == 64;
                __syncthreads();  // every thread has read s_* before the next pass
                if (done) {
                    t = prefix | (sh ? ((1ull << sh) - 1ull) : 0ull);
                    break;
                }
            }
        }
        for (int32_t i = tid; i < n; i += kSelThreads) {
            const uint64_t key = row[i];
            if (key <= t) {
                const uint32_t at = atomicAdd(&s_n, 1u);
                if (at < (uint32_t)w.r) sel[at] = key;
                atomicMax(&s_max, (unsigned long long)key);
            }
        }
        __syncthreads();
        const int32_t m = (int32_t)min(s_n, (uint32_t)w.r);
        for (int32_t i = tid; i < m; i += kSelThreads) row[i] = sel[i];
        if (fin)
            for (int32_t i = m + tid; i < w.r; i += kSelThreads) row[i] = kEmptyKey;
        if (tid == 0) {
            w.cnt[q] = m;
            if (!fin) {
                w.over[q] = 0;
                if (m == w.r) atomicMin(tau + q, (uint32_t)(s_max >> 32) + 1u);
            }
        }
        __syncthreads();  // LDS reused by the next query
    }
}

// Exact f32 distance of each of the R candidates, written back as its key
// in place (one wave per 64 candidates of one query, a lane per candidate).
// The summation order is the vector scans': each chunk of `chunk`
// dimensions summed in order, the chunk sums added in order.  The rows are
// read a slab of 32 dimensions at a time: coalesced loads (8 lanes per
// 128-byte row segment) put the slab of the wave's 64 rows in its LDS
// (row stride 33 floats, so the lanes' reads of one dimension fall in
// distinct banks), and each lane then sums its own row's dimensions in
// order.  A lane per row reading its row alone would touch 64 lines per
// load and re-fetch each line for every 16 bytes of it.
constexpr int kSlab = 32;
constexpr int kSlabPitch = kSlab + 1;
__global__ __launch_bounds__(256) void wide_rerank_kernel(WideSink w, const float *__restrict__ xrow,
                                                          const float *__restrict__ qrot, int32_t d, int32_t chunk,
                                                          const int32_t *__restrict__ bad) {
    __shared__ float slab_all[4][kWave * kSlabPitch];
    const int lane = threadIdx.x & 63;
    const int wid = threadIdx.x >> 6;
    const int32_t nblk = (w.r + 63) / 64;
    const int64_t wv = (int64_t)blockIdx.x * 4 + wid;
    const int64_t q = __builtin_amdgcn_readfirstlane((int32_t)(wv / nblk));
    const int32_t blk = (int32_t)(wv % nblk);
    if (q >= w.nq || bad[q]) return;  // whole waves
    const int32_t i = blk * 64 + lane;
    uint64_t *row = w.buf + q * (int64_t)w.cap;
    const uint64_t key = i < w.r ? row[i] : kEmptyKey;
    const bool live = key != kEmptyKey;
    const uint32_t id = (uint32_t)(key & 0xffffffffu);
    float *sl = slab_all[wid];
    const float *qp = qrot + q * d;
    const bool vec = (d & 3) == 0;
    // the rows this lane loads: row (lane >> 3) + 8u (vector path) or
    // (lane >> 5) + 2u (scalar path) of the wave's 64
    const float *src[8];
    bool ok[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
        const int r = (lane >> 3) + 8 * u;
        ok[u] = __shfl((int)live, r) != 0;
        src[u] = xrow + (int64_t)(uint32_t)__shfl((int)id, r) * d;
    }
    float partial = 0.0f, s = 0.0f;
    int32_t cb = chunk;  // next chunk boundary
    for (int32_t j0 = 0; j0 < d; j0 += kSlab) {
        const int32_t jn = min(kSlab, d - j0);
        if (vec) {
            const int c4 = 4 * (lane & 7);
            float4 v[8];
#pragma unroll
            for (int u = 0; u < 8; ++u)
                v[u] = (ok[u] && c4 < jn) ? *reinterpret_cast<const float4 *>(src[u] + j0 + c4)
                                          : make_float4(0.0f, 0.0f, 0.0f, 0.0f);
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                float *o = sl + ((lane >> 3) + 8 * u) * kSlabPitch + c4;
                o[0] = v[u].x;
                o[1] = v[u].y;
                o[2] = v[u].z;
                o[3] = v[u].w;
            }
        } else {
            const int c = lane & 31;
            for (int u = 0; u < 32; ++u) {
                const int r = (lane >> 5) + 2 * u;
                const bool rl = __shfl((int)live, r) != 0;
                const float *xr = xrow + (int64_t)(uint32_t)__shfl((int)id, r) * d;
                sl[r * kSlabPitch + c] = (rl && c < jn) ? xr[j0 + c] : 0.0f;
            }
        }
        // the slab, written by the wave's lanes, is read by other lanes of
        // the same wave: LDS instructions of a wave are performed in order,
        // and the fences keep the compiler from moving the reads above the
        // writes (or the next slab's writes above these reads, below)
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        const float *mine = sl + lane * kSlabPitch;
        for (int32_t jj = 0; jj < jn;) {
            if (j0 + jj == cb) {  // a chunk ends: add its sum
                partial += s;
                s = 0.0f;
                cb += chunk;
            }
            const int32_t seg = min(jn, cb - j0);  // this chunk's dimensions in the slab
            for (; jj < seg; ++jj) {
                const float t = qp[j0 + jj] - mine[jj];
                s = fmaf(t, t, s);
            }
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
    partial += s;
    if (live) row[i] = make_key(partial, id);
}

// The k best of the R re-ranked keys; a non-finite query gets NaN rows, a
// query whose scan did not complete (cannot happen with the planner's
// number of rounds) ids -1 and NaN distances.
__global__ __launch_bounds__(64) void wide_topk_kernel(WideSink w, int32_t k, const int32_t *__restrict__ bad,
                                                       int64_t *__restrict__ out_ids, float *__restrict__ out_dist) {
    const int64_t q = blockIdx.x;
    const int lane = threadIdx.x;
    const bool nan_row = bad[q] || w.over[q];
    uint64_t e = kEmptyKey, kth = kEmptyKey;
    if (!nan_row) {
        const uint64_t *row = w.buf + q * (int64_t)w.cap;
        for (int32_t i0 = 0; i0 < w.r; i0 += kWave) {
            const uint64_t key = i0 + lane < w.r ? row[i0 + lane] : kEmptyKey;
            topk_offer(e, kth, key, key != kEmptyKey, k, lane);
        }
    }
    if (lane < k) {
        int64_t id = -1;
        float dist = INFINITY;
        if (nan_row) {
            dist = __uint_as_float(0x7fc00000u);
        } else if (e != kEmptyKey) {
            id = (int64_t)(e & 0xffffffffu);
            dist = key_dist(e);
        }
        out_ids[q * k + lane] = id;
        out_dist[q * k + lane] = dist;
    }
}

}  // namespace

hipError_t launch_wide_init(const WideSink &w, const float *cd, int32_t nlist, const int32_t *probe, int32_t rounds,
                            hipStream_t s) {
    if (w.nq <= 0) return hipSuccess;
    wide_init_kernel<<<(unsigned)w.nq, 256, 0, s>>>(w, cd, nlist, probe, rounds);
    return hipGetLastError();
}

hipError_t launch_wide_select(const WideSink &w, int32_t list_round, uint32_t *tau, hipStream_t s) {
    if (w.nq <= 0) return hipSuccess;
    const size_t lds = sizeof(uint64_t) * (size_t)w.r;
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(wide_select_kernel),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    const int64_t grid = list_round < 0 ? w.nq : (w.nq < 1024 ? w.nq : 1024);
    wide_select_kernel<<<(unsigned)grid, kSelThreads, lds, s>>>(w, list_round, tau);
    return hipGetLastError();
}

hipError_t launch_wide_rerank(const WideSink &w, const float *xrow, const float *qrot, int32_t d, int32_t chunk,
                              const int32_t *bad, int32_t k, int64_t *out_ids, float *out_dist, hipStream_t s) {
    if (w.nq <= 0) return hipSuccess;
    const int64_t waves = w.nq * ((w.r + 63) / 64);
    wide_rerank_kernel<<<(unsigned)((waves + 3) / 4), 256, 0, s>>>(w, xrow, qrot, d, chunk, bad);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    wide_topk_kernel<<<(unsigned)w.nq, 64, 0, s>>>(w, k, bad, out_ids, out_dist);
    return hipGetLastError();
}

}  // namespace pdx
