// Exact inner-product search (the IP kernel of Section 3's listing) as a
// linear scan on the matrix cores.  The score of a vector v for a query q
// is -q.v, so ascending scores rank the largest inner products first, ties
// by row id as for every other result.
//
// A partial inner product bounds nothing, so every value is used: the scan
// is a dense (queries x vectors x D) contraction.  A workgroup holds 64
// queries (4 waves x 16) and walks the vectorgroups of one of `parts`
// ranges; per 32-dimension sub-chunk a wave issues 32
// v_mfma_f32_16x16x4f32 (16 queries x 64 vectors).  The four waves of a
// workgroup read the same rows, and the query blocks of one range run on one
// XCD (workgroup i runs on XCD i mod 8), so a range's rows are fetched into
// that XCD's L2 once for all its query blocks.
//
// Lane layout (lane = 16 kq + col) as in the IVF matrix-core scan:
// A (16 x 4): query slot col, k index kq; B (4 x 16): k index kq, vector
// 4 col + t for MFMA t; D: lane holds query slots 4 kq + r against vector
// 4 col + t.  In K-step s of the sub-chunk starting at j0 the k index kq
// stands for dimension j0 + 8 kq + s.
//
// Scores are signed, so k-best keys use an order-preserving image of the
// float bits (non-negative: sign bit set; negative: all bits complemented).
#include "mfma_tiles.h"
#include "pdx_internal.h"
#include "wave_topk.h"

namespace pdx {
namespace {

typedef float v4f __attribute__((ext_vector_type(4)));

__device__ __forceinline__ uint32_t ord_bits(float f) {
    const uint32_t b = __float_as_uint(f);
    return (b & 0x80000000u) ? ~b : (b | 0x80000000u);
}

__device__ __forceinline__ float ord_float(uint32_t o) {
    return __uint_as_float((o & 0x80000000u) ? (o & 0x7fffffffu) : ~o);
}

constexpr int kIpQueries = 64;  // queries per workgroup (4 waves x 16)
constexpr int kIpTiles = 2;     // D % 4 == 0: 16-query tiles per wave

// grid = 8 * (parts / 8) * nqb; XCD x = blockIdx.x % 8 takes ranges
// [x parts/8, (x+1) parts/8), every query block of each.
__global__ __launch_bounds__(256) void ip_scan_kernel(const float *__restrict__ pdxd,
                                                      const int32_t *__restrict__ slot_id, int64_t n, int32_t d,
                                                      int32_t ngroups, const float *__restrict__ q, int64_t nq,
                                                      const int32_t *__restrict__ bad, int32_t parts, int32_t nqb,
                                                      uint64_t *__restrict__ slots, int32_t k) {
    __shared__ uint64_t lists[4][16][kWave];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int col = lane & 15, kq = lane >> 4;
    const int32_t per_xcd = parts / 8;
    const int32_t x = blockIdx.x & 7, idx = blockIdx.x >> 3;
    const int32_t p = x * per_xcd + idx / nqb;
    const int64_t q0 = (int64_t)(idx % nqb) * kIpQueries + wave * 16;
    if (q0 >= nq) return;
    uint64_t(*lw)[kWave] = lists[wave];
    // query slot col of this wave's tile (rows past nq or non-finite: zeros)
    const int64_t qc = q0 + col;
    const bool qok = qc < nq && !bad[qc];
    const float *qrow = q + (qok ? qc : q0) * d;
    bool rowok[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int64_t qr = q0 + 4 * kq + r;
        rowok[r] = qr < nq && !bad[qr];
    }
#pragma unroll
    for (int m = 0; m < 16; ++m) lw[m][lane] = kEmptyKey;
    uint64_t kth[16];  // wave-uniform k-th key of each query's list
#pragma unroll
    for (int m = 0; m < 16; ++m) kth[m] = kEmptyKey;
    const bool vec_ok = (d & 3) == 0;
    const int32_t g0 = (int32_t)((int64_t)ngroups * p / parts), g1 = (int32_t)((int64_t)ngroups * (p + 1) / parts);
    for (int32_t g = g0; g < g1; ++g) {
        int32_t vid[4];
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            const int64_t sv = (int64_t)g * kGroup + 4 * col + t;
            vid[t] = slot_id ? slot_id[sv] : (sv < n ? (int32_t)sv : -1);
        }
        v4f acc[4];
#pragma unroll
        for (int t = 0; t < 4; ++t) acc[t] = v4f{0.0f, 0.0f, 0.0f, 0.0f};
        const int64_t gbase = (int64_t)g * d;
        for (int32_t j0 = 0; j0 < d; j0 += 32) {
            const int32_t jl = j0 + 8 * kq;
            float a[8];
            v4f bx[8];
            if (j0 + 32 <= d && vec_ok) {
#pragma unroll
                for (int s = 0; s < 8; ++s)
                    bx[s] = *reinterpret_cast<const v4f *>(pdxd + (gbase + jl + s) * kGroup + 4 * col);
                const v4f q_lo = *reinterpret_cast<const v4f *>(qrow + jl);
                const v4f q_hi = *reinterpret_cast<const v4f *>(qrow + jl + 4);
#pragma unroll
                for (int s = 0; s < 4; ++s) {
                    a[s] = qok ? q_lo[s] : 0.0f;
                    a[s + 4] = qok ? q_hi[s] : 0.0f;
                }
            } else {
#pragma unroll
                for (int s = 0; s < 8; ++s) {
                    const int32_t j = jl + s;
                    const bool ok = j < d;
                    a[s] = (ok && qok) ? qrow[j] : 0.0f;
                    bx[s] = ok ? *reinterpret_cast<const v4f *>(pdxd + (gbase + j) * kGroup + 4 * col)
                               : v4f{0.0f, 0.0f, 0.0f, 0.0f};
                }
            }
#pragma unroll
            for (int s = 0; s < 8; ++s)
#pragma unroll
                for (int t = 0; t < 4; ++t)
                    acc[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[s], bx[s][t], acc[t], 0, 0, 0);
        }
        // offers: query slot m = 4 kq' + r is held by the 16 lanes with kq == kq'
#pragma unroll
        for (int m = 0; m < 16; ++m) {
            const int r = m & 3;
            const bool myrow = kq == (m >> 2) && rowok[r];
            uint64_t key[4];
            bool want[4];
            bool any = false;
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                const float sc = -acc[t][r] + 0.0f;  // -q.v, zero as +0
                key[t] = (static_cast<uint64_t>(ord_bits(sc)) << 32) | static_cast<uint32_t>(vid[t]);
                want[t] = myrow && vid[t] >= 0 && key[t] < kth[m];
                any |= want[t];
            }
            if (!__any(any)) continue;
            uint64_t em = lw[m][lane];
            uint64_t km = kth[m];
#pragma unroll
            for (int t = 0; t < 4; ++t) topk_offer(em, km, key[t], want[t], k, lane);
            lw[m][lane] = em;
            kth[m] = km;
        }
    }
#pragma unroll
    for (int m = 0; m < 16; ++m) {
        const int64_t qm = q0 + m;
        if (qm < nq && lane < k) slots[((size_t)qm * parts + p) * k + lane] = lw[m][lane];
    }
}

// The same scan for D % 4 == 0 with NT tiles of 16 queries per wave: each
// row value a lane loads feeds 4 NT MFMAs, a workgroup holds 4 such waves
// (64 NT queries) over one range of vectorgroups, so the range's rows are
// fetched once per 64 NT queries, and the loads run half a sub-chunk ahead
// of the MFMAs (across vectorgroups too).  A query slot that is out of
// range or non-finite reads another row of q; its products are never
// offered.  The per-query lists take 16 NT x kp keys of LDS per wave (kp:
// k rounded up to 16; dynamic LDS of 4 x 16 NT x kp keys).
template <int NT>
__global__ __launch_bounds__(256, 3) void ip_scan_mx_kernel(const float *__restrict__ pdxd,
                                                            const int32_t *__restrict__ slot_id, int64_t n, int32_t d,
                                                            int32_t ngroups, const float *__restrict__ q, int64_t nq,
                                                            const int32_t *__restrict__ bad, int32_t parts,
                                                            int32_t nqb, uint64_t *__restrict__ slots, int32_t k) {
    extern __shared__ uint64_t ip_lists[];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int col = lane & 15, kq = lane >> 4;
    const int32_t per_xcd = parts / 8;
    const int32_t x = blockIdx.x & 7, idx = blockIdx.x >> 3;
    const int32_t p = x * per_xcd + idx / nqb;
    const int64_t q0 = (int64_t)(idx % nqb) * (64 * NT) + wave * (16 * NT);
    if (q0 >= nq) return;
    const int kp = (k + 15) & ~15;
    uint64_t *lw = ip_lists + (size_t)wave * 16 * NT * kp;  // query slot m: lw[m kp .. m kp + kp)
    const float *qrow[NT];
    bool rowok[NT][4];
#pragma unroll
    for (int u = 0; u < NT; ++u) {
        const int64_t qc = q0 + 16 * u + col;
        qrow[u] = q + (qc < nq ? qc : q0) * d;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int64_t qr = q0 + 16 * u + 4 * kq + r;
            rowok[u][r] = qr < nq && !bad[qr];
        }
    }
    uint64_t kth[16 * NT];  // wave-uniform k-th key of each query's list
#pragma unroll
    for (int m = 0; m < 16 * NT; ++m) {
        if (lane < kp) lw[m * kp + lane] = kEmptyKey;
        kth[m] = kEmptyKey;
    }
    const int32_t g0 = (int32_t)((int64_t)ngroups * p / parts), g1 = (int32_t)((int64_t)ngroups * (p + 1) / parts);
    const int32_t nfull = d / 32;  // whole sub-chunks; then a partial one when 32 does not divide D
    if (g0 < g1) {
        v4f b0[4], b1[4], a0[NT], a1[NT];
        float xx[4];  // unused (no norms)
        if (nfull > 0) load_half<NT>(pdxd, (int64_t)g0 * d, 0, 0, kq, col, qrow, b0, a0);
        for (int32_t g = g0; g < g1; ++g) {
            int32_t vid[4];
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                const int64_t sv = (int64_t)g * kGroup + 4 * col + t;
                vid[t] = slot_id ? slot_id[sv] : (sv < n ? (int32_t)sv : -1);
            }
            v4f acc[NT][4];
#pragma unroll
            for (int u = 0; u < NT; ++u)
#pragma unroll
                for (int t = 0; t < 4; ++t) acc[u][t] = v4f{0.0f, 0.0f, 0.0f, 0.0f};
            const int64_t gbase = (int64_t)g * d;
            for (int32_t c = 0; c < nfull; ++c) {
                const int32_t j0 = 32 * c;
                load_half<NT>(pdxd, gbase, j0, 1, kq, col, qrow, b1, a1);
                mfma_half<NT, false>(b0, a0, acc, xx);
                // the next whole sub-chunk: of this vectorgroup, else the
                // next one's first (after the last, this one's first again)
                const bool more = c + 1 < nfull;
                const int64_t gnext = more ? gbase : (g + 1 < g1 ? gbase + d : (int64_t)g0 * d);
                load_half<NT>(pdxd, gnext, more ? j0 + 32 : 0, 0, kq, col, qrow, b0, a0);
                mfma_half<NT, false>(b1, a1, acc, xx);
            }
            if (32 * nfull < d) {
                v4f bt[4], at[NT];
                load_half_tail<NT>(pdxd, gbase, d, 32 * nfull, 0, kq, col, qrow, bt, at);
                mfma_half<NT, false>(bt, at, acc, xx);
                load_half_tail<NT>(pdxd, gbase, d, 32 * nfull, 1, kq, col, qrow, bt, at);
                mfma_half<NT, false>(bt, at, acc, xx);
            }
            // offers: query slot 16 u + 4 kq' + r is held by the 16 lanes with kq == kq'
#pragma unroll
            for (int u = 0; u < NT; ++u)
#pragma unroll
                for (int m = 0; m < 16; ++m) {
                    const int r = m & 3;
                    const bool myrow = kq == (m >> 2) && rowok[u][r];
                    uint64_t key[4];
                    bool want[4];
                    bool any = false;
#pragma unroll
                    for (int t = 0; t < 4; ++t) {
                        const float sc = -acc[u][t][r] + 0.0f;  // -q.v, zero as +0
                        key[t] = (static_cast<uint64_t>(ord_bits(sc)) << 32) | static_cast<uint32_t>(vid[t]);
                        want[t] = myrow && vid[t] >= 0 && key[t] < kth[16 * u + m];
                        any |= want[t];
                    }
                    if (!__any(any)) continue;
                    // lanes k .. 63 hold kEmptyKey and are never changed by an offer
                    uint64_t em = lane < kp ? lw[(16 * u + m) * kp + lane] : kEmptyKey;
                    uint64_t km = kth[16 * u + m];
#pragma unroll
                    for (int t = 0; t < 4; ++t) topk_offer(em, km, key[t], want[t], k, lane);
                    if (lane < kp) lw[(16 * u + m) * kp + lane] = em;
                    kth[16 * u + m] = km;
                }
        }
    }
#pragma unroll
    for (int m = 0; m < 16 * NT; ++m) {
        const int64_t qm = q0 + m;
        if (qm < nq && lane < k) slots[((size_t)qm * parts + p) * k + lane] = lw[m * kp + lane];
    }
}

// k best of a query's `parts` lists: ids and -q.v; non-finite queries get
// ids -1 and NaN, missing entries id -1 and +inf.
__global__ __launch_bounds__(64) void ip_merge_kernel(const uint64_t *__restrict__ slots, int32_t parts, int32_t k,
                                                      const int32_t *__restrict__ bad, int64_t *__restrict__ out_ids,
                                                      float *__restrict__ out_dist) {
    const int64_t qi = blockIdx.x;
    const int lane = threadIdx.x;
    if (bad[qi]) {
        if (lane < k) {
            out_ids[qi * k + lane] = -1;
            out_dist[qi * k + lane] = __uint_as_float(0x7fc00000u);
        }
        return;
    }
    uint64_t e = kEmptyKey, kth = kEmptyKey;
    const uint64_t *src = slots + (size_t)qi * parts * k;
    const int64_t total = (int64_t)parts * k;
    for (int64_t i = lane; i - lane < total; i += 64) {
        const uint64_t key = i < total ? src[i] : kEmptyKey;
        topk_offer(e, kth, key, key != kEmptyKey, k, lane);
    }
    if (lane < k) {
        const bool has = e != kEmptyKey;
        out_ids[qi * k + lane] = has ? (int64_t)(uint32_t)(e & 0xffffffffu) : -1;
        out_dist[qi * k + lane] = has ? ord_float(static_cast<uint32_t>(e >> 32)) : INFINITY;
    }
}

}  // namespace

// Ranges of vectorgroups: enough workgroups to fill the chip (about 8 waves
// per SIMD) for the query blocks at hand, a multiple of 8, at most one range
// per vectorgroup.
int32_t ip_parts_for(int64_t nq, int32_t ngroups, int32_t d) {
    const int64_t per = d % 4 == 0 ? 64 * kIpTiles : kIpQueries;
    const int64_t nqb = (nq + per - 1) / per;
    const int64_t want_wg = 8 * (int64_t)device_cus();  // 4 waves each: 8 waves per SIMD
    int64_t parts = (want_wg + nqb - 1) / (nqb > 0 ? nqb : 1);
    parts = (parts + 7) / 8 * 8;
    const int64_t cap = ((int64_t)ngroups + 7) / 8 * 8;
    if (parts > cap) parts = cap;
    return (int32_t)(parts < 8 ? 8 : parts);
}

hipError_t launch_ip_scan(const pdx_index *ix, const float *q, int64_t nq, const int32_t *bad, int32_t parts,
                          uint64_t *slots, int32_t k, hipStream_t s) {
    if (nq <= 0) return hipSuccess;
    const bool mx = ix->d % 4 == 0;
    const int64_t per = mx ? 64 * kIpTiles : kIpQueries;
    const int32_t nqb = (int32_t)((nq + per - 1) / per);
    const unsigned grid = 8u * (unsigned)(parts / 8) * (unsigned)nqb;
    const int32_t *sid = ix->kind == kIvf ? ix->slot_id : nullptr;
    if (mx) {
        const size_t lds = (size_t)4 * 16 * kIpTiles * ((k + 15) & ~15) * sizeof(uint64_t);  // at most 64 KiB
        ip_scan_mx_kernel<kIpTiles><<<grid, 256, lds, s>>>(ix->pdx, sid, ix->n, ix->d, ix->ngroups, q, nq, bad,
                                                           parts, nqb, slots, k);
    }
    else
        ip_scan_kernel<<<grid, 256, 0, s>>>(ix->pdx, sid, ix->n, ix->d, ix->ngroups, q, nq, bad, parts, nqb, slots, k);
    return hipGetLastError();
}

hipError_t launch_ip_merge(const uint64_t *slots, int64_t nq, int32_t parts, int32_t k, const int32_t *bad,
                           int64_t *out_ids, float *out_dist, hipStream_t s) {
    if (nq <= 0) return hipSuccess;
    ip_merge_kernel<<<(unsigned)nq, 64, 0, s>>>(slots, parts, k, bad, out_ids, out_dist);
    return hipGetLastError();
}

}  // namespace pdx
