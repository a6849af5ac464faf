// L2 linear mode on the matrix cores (the L2 kernel of Section 3's listing:
// every vector evaluated; exact).  Per 16 queries x 64 vectors a wave forms
// q.x with v_mfma_f32_16x16x4f32 and |x|^2 from the same loaded values, so
// each (query, vector) pair gets d' = |q|^2 + |x|^2 - 2 q.x.
//
// Margin: e = 4 (D + 64) 2^-24 (|q|^2 + |x|^2) bounds both d' - |q - x|^2
// and the fixed-order float32 sum's distance from |q - x|^2, so d' - e is
// below and d' + e above the distance every other path reports.
//
// Bound pass (every stride-th vectorgroup): each query's k smallest d' + e;
// their k-th bounds the query's k-th distance from above, since the k-th of
// a subset is no smaller.  Listing pass (every vectorgroup): the vectors
// whose d' - e is at or below that bound, a superset of the k nearest.  The
// caller sums the listed vectors exactly and merges them.
//
// Lane layout (lane = 16 kq + col): A (16 x 4) holds query slot col at k
// index kq; B (4 x 16) holds k index kq for vector 4 col + t in MFMA t; D
// gives a lane query slots 4 kq + r against vector 4 col + t.  In K-step s
// of the 32-dimension sub-chunk starting at j0, k index kq stands for
// dimension j0 + 8 kq + s.  A lane loads its four vectors of a dimension
// with one 16-byte load (vectors 4 col .. 4 col + 3 are adjacent in a
// vectorgroup).
//
// Workgroup i runs on XCD i mod 8; the query blocks of one range of
// vectorgroups are consecutive there, so the range's rows are fetched into
// that XCD's L2 once for all of them.
#include "mfma_tiles.h"
#include "pdx_internal.h"
#include "wave_topk.h"

namespace pdx {
namespace {

typedef float v4f __attribute__((ext_vector_type(4)));

constexpr int kBoundQueries = 64;  // bound pass: queries per workgroup (4 waves x 16)
constexpr int kListTiles = 4;      // listing pass: 16-query tiles per wave
constexpr int kListQueries = 4 * 16 * kListTiles;  // listing pass: queries per workgroup

__host__ __device__ inline float lin_margin(int32_t d) { return 4.0f * (float)(d + 64) * 0x1p-24f; }

// One 32-dimension sub-chunk's operands: the lane's four vectors of its 8
// dimensions, and NT query tiles' values of the same dimensions (zero past
// D).  A query slot's values reach only that query's row of the products,
// so a slot that is out of range or non-finite reads another row of q and
// its results are never used.
template <int NT>
__device__ __forceinline__ void load_subchunk(const float *__restrict__ pdxd, int64_t gbase, int32_t d, int32_t j0,
                                              int kq, int col, const float *const (&qrow)[NT], v4f (&bx)[8],
                                              v4f (&alo)[NT], v4f (&ahi)[NT]) {
    const int32_t jl = j0 + 8 * kq;
    if (j0 + 32 <= d) {
#pragma unroll
        for (int s = 0; s < 8; ++s) bx[s] = *reinterpret_cast<const v4f *>(pdxd + (gbase + jl + s) * kGroup + 4 * col);
#pragma unroll
        for (int u = 0; u < NT; ++u) {
            alo[u] = *reinterpret_cast<const v4f *>(qrow[u] + jl);
            ahi[u] = *reinterpret_cast<const v4f *>(qrow[u] + jl + 4);
        }
    } else {
#pragma unroll
        for (int s = 0; s < 8; ++s) {
            const int32_t j = jl + s;
            const bool ok = j < d;
            bx[s] = ok ? *reinterpret_cast<const v4f *>(pdxd + (gbase + j) * kGroup + 4 * col)
                       : v4f{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
            for (int u = 0; u < NT; ++u) {
                const float v = ok ? qrow[u][j] : 0.0f;
                if (s < 4) alo[u][s] = v;
                else ahi[u][s - 4] = v;
            }
        }
    }
}

// Bound pass.  A workgroup holds 64 queries (4 waves x 16) and walks the
// stride-th vectorgroups of one of `parts` ranges; each wave keeps its 16
// queries' k smallest keys (d' + e, row slot) in LDS lists, written to
// slots[q][part][0..k).
__global__ __launch_bounds__(256) void lin_bound_kernel(
    const float *__restrict__ pdxd, const int32_t *__restrict__ slot_id, int64_t n, int32_t d, int32_t ngroups,
    const float *__restrict__ q, int64_t nq, const float *__restrict__ qn, const int32_t *__restrict__ bad,
    int32_t parts, int32_t nqb, int32_t stride, uint64_t *__restrict__ slots, int32_t k) {
    __shared__ uint64_t lists[4][16][kWave];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int col = lane & 15, kq = lane >> 4;
    const int32_t per_xcd = parts / 8;
    const int32_t x = blockIdx.x & 7, idx = blockIdx.x >> 3;
    const int32_t p = x * per_xcd + idx / nqb;
    const int64_t q0 = (int64_t)(idx % nqb) * kBoundQueries + wave * 16;
    if (q0 >= nq) return;
    const float margin = lin_margin(d);
    const int64_t qc = q0 + col;
    const float *const qrow[1] = {q + (qc < nq ? qc : q0) * d};
    bool rowok[4];
    float qnr[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int64_t qr = q0 + 4 * kq + r;
        rowok[r] = qr < nq && !bad[qr];
        qnr[r] = rowok[r] ? qn[qr] : 0.0f;
    }
    uint64_t kth[16];
#pragma unroll
    for (int m = 0; m < 16; ++m) {
        lists[wave][m][lane] = kEmptyKey;
        kth[m] = kEmptyKey;
    }
    const int32_t g0 = (int32_t)((int64_t)ngroups * p / parts), g1 = (int32_t)((int64_t)ngroups * (p + 1) / parts);
    for (int32_t g = (g0 + stride - 1) / stride * stride; g < g1; g += stride) {
        int32_t sv[4];
        bool vok[4];
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            sv[t] = g * kGroup + 4 * col + t;
            vok[t] = slot_id ? slot_id[sv[t]] >= 0 : sv[t] < n;
        }
        v4f acc[4];
        float xx[4] = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
        for (int t = 0; t < 4; ++t) acc[t] = v4f{0.0f, 0.0f, 0.0f, 0.0f};
        const int64_t gbase = (int64_t)g * d;
        for (int32_t j0 = 0; j0 < d; j0 += 32) {
            v4f bx[8], alo[1], ahi[1];
            load_subchunk<1>(pdxd, gbase, d, j0, kq, col, qrow, bx, alo, ahi);
#pragma unroll
            for (int s = 0; s < 8; ++s)
#pragma unroll
                for (int t = 0; t < 4; ++t) {
                    const float a = s < 4 ? alo[0][s] : ahi[0][s - 4];
                    acc[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, bx[s][t], acc[t], 0, 0, 0);
                    xx[t] = fmaf(bx[s][t], bx[s][t], xx[t]);
                }
        }
        // |x|^2 over all dimensions: the lanes of one column hold 8 of each 32
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            xx[t] += __shfl_xor(xx[t], 16);
            xx[t] += __shfl_xor(xx[t], 32);
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
                const float nn = qnr[r] + xx[t];
                const float hi = fmaxf(nn - 2.0f * acc[t][r], 0.0f) + margin * nn;
                key[t] = make_key(hi, (uint32_t)sv[t]);
                want[t] = myrow && vok[t] && key[t] < kth[m];
                any |= want[t];
            }
            if (!__any(any)) continue;
            uint64_t em = lists[wave][m][lane];
            uint64_t km = kth[m];
#pragma unroll
            for (int t = 0; t < 4; ++t) topk_offer(em, km, key[t], want[t], k, lane);
            lists[wave][m][lane] = em;
            kth[m] = km;
        }
    }
#pragma unroll
    for (int m = 0; m < 16; ++m) {
        const int64_t qm = q0 + m;
        if (qm < nq && lane < k) slots[((size_t)qm * parts + p) * k + lane] = lists[wave][m][lane];
    }
}

// Each query's bound: the k-th smallest of its bound-pass keys (+inf when it
// has fewer than k).
__global__ __launch_bounds__(64) void lin_tau_kernel(const uint64_t *__restrict__ slots, int32_t parts, int32_t k,
                                                     uint32_t *__restrict__ tau) {
    const int64_t qi = blockIdx.x;
    const int lane = threadIdx.x;
    uint64_t e = kEmptyKey, kth = kEmptyKey;
    const uint64_t *src = slots + (size_t)qi * parts * k;
    const int64_t total = (int64_t)parts * k;
    for (int64_t i = lane; i - lane < total; i += 64) {
        const uint64_t key = i < total ? src[i] : kEmptyKey;
        topk_offer(e, kth, key, key != kEmptyKey, k, lane);
    }
    if (lane == 0) tau[qi] = kth == kEmptyKey ? kInfBits : static_cast<uint32_t>(kth >> 32);
}

// Listing pass.  A wave holds NT tiles of 16 queries, so each loaded value
// of a row feeds 4 NT MFMAs; a workgroup holds 4 waves of different queries
// over the same range of vectorgroups (the rows reach the four through the
// CU's L1).  The loads run one half sub-chunk ahead of the MFMAs, across
// vectorgroups too.  A vector whose lower bound d' - e is at or below its
// query's bound is appended to that query's list (row slot; the count runs
// on past cap when the list overflows).
template <int NT>
__global__ __launch_bounds__(256, 2) void lin_list_kernel(
    const float *__restrict__ pdxd, const int32_t *__restrict__ slot_id, int64_t n, int32_t d, int32_t ngroups,
    const float *__restrict__ q, int64_t nq, const float *__restrict__ qn, const int32_t *__restrict__ bad,
    int32_t parts, int32_t nqb, const uint32_t *__restrict__ tau, uint64_t *__restrict__ cand,
    int32_t *__restrict__ cand_cnt, int32_t cap) {
    // the workgroup's queries: squared norm and bound (-inf: out of range or
    // non-finite; a bound is never below 0 otherwise)
    __shared__ float lqn[64 * NT], lbound[64 * NT];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int col = lane & 15, kq = lane >> 4;
    const int32_t per_xcd = parts / 8;
    const int32_t x = blockIdx.x & 7, idx = blockIdx.x >> 3;
    const int32_t p = x * per_xcd + idx / nqb;
    const int64_t qblk = (int64_t)(idx % nqb) * (64 * NT);
    for (int i = threadIdx.x; i < 64 * NT; i += 256) {
        const int64_t qi = qblk + i;
        const bool ok = qi < nq && !bad[qi];
        lqn[i] = ok ? qn[qi] : 0.0f;
        lbound[i] = ok ? __uint_as_float(tau[qi]) : -INFINITY;
    }
    __syncthreads();
    const int64_t q0 = qblk + wave * (16 * NT);
    const int32_t g0 = (int32_t)((int64_t)ngroups * p / parts), g1 = (int32_t)((int64_t)ngroups * (p + 1) / parts);
    if (q0 >= nq || g0 >= g1) return;
    const float margin = lin_margin(d);
    const float *qrow[NT];
#pragma unroll
    for (int u = 0; u < NT; ++u) {
        const int64_t qc = q0 + 16 * u + col;
        qrow[u] = q + (qc < nq ? qc : q0) * d;
    }
    const int32_t nfull = d / 32;  // whole sub-chunks; then a partial one when 32 does not divide D
    v4f b0[4], b1[4], a0[NT], a1[NT];
    if (nfull > 0) load_half<NT>(pdxd, (int64_t)g0 * d, 0, 0, kq, col, qrow, b0, a0);
    for (int32_t g = g0; g < g1; ++g) {
        v4f acc[NT][4];
        float xx[4] = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
        for (int u = 0; u < NT; ++u)
#pragma unroll
            for (int t = 0; t < 4; ++t) acc[u][t] = v4f{0.0f, 0.0f, 0.0f, 0.0f};
        const int64_t gbase = (int64_t)g * d;
        for (int32_t c = 0; c < nfull; ++c) {
            const int32_t j0 = 32 * c;
            load_half<NT>(pdxd, gbase, j0, 1, kq, col, qrow, b1, a1);
            mfma_half<NT, true>(b0, a0, acc, xx);
            // the next whole sub-chunk: of this vectorgroup, else the next
            // one's first (after the last vectorgroup, this one's first again)
            const bool more = c + 1 < nfull;
            const int64_t gnext = more ? gbase : (g + 1 < g1 ? gbase + d : (int64_t)g0 * d);
            load_half<NT>(pdxd, gnext, more ? j0 + 32 : 0, 0, kq, col, qrow, b0, a0);
            mfma_half<NT, true>(b1, a1, acc, xx);
        }
        if (32 * nfull < d) {
            v4f bt[4], at[NT];
            load_half_tail<NT>(pdxd, gbase, d, 32 * nfull, 0, kq, col, qrow, bt, at);
            mfma_half<NT, true>(bt, at, acc, xx);
            load_half_tail<NT>(pdxd, gbase, d, 32 * nfull, 1, kq, col, qrow, bt, at);
            mfma_half<NT, true>(bt, at, acc, xx);
        }
        // |x|^2 over all dimensions: the lanes of one column hold 8 of each 32
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            xx[t] += __shfl_xor(xx[t], 16);
            xx[t] += __shfl_xor(xx[t], 32);
        }
        bool vok[4];
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            const int32_t sv = g * kGroup + 4 * col + t;
            vok[t] = slot_id ? slot_id[sv] >= 0 : sv < n;
        }
#pragma unroll
        for (int u = 0; u < NT; ++u)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int i = wave * (16 * NT) + 16 * u + 4 * kq + r;
                const float qq = lqn[i], bound = lbound[i];
                if (bound == -INFINITY) continue;
#pragma unroll
                for (int t = 0; t < 4; ++t) {
                    const float nn = qq + xx[t];
                    const float lo = nn - 2.0f * acc[u][t][r] - margin * nn;
                    if (vok[t] && !(lo > bound)) {
                        const int64_t qr = qblk + i;
                        const int32_t pos = atomicAdd(cand_cnt + qr, 1);
                        if (pos < cap) cand[qr * cap + pos] = (uint64_t)(uint32_t)(g * kGroup + 4 * col + t);
                    }
                }
            }
    }
}

int32_t xcd_parts(int64_t want_wg, int64_t nqb, int32_t ngroups) {
    int64_t parts = (want_wg + nqb - 1) / (nqb > 0 ? nqb : 1);
    parts = (parts + 7) / 8 * 8;
    const int64_t cap = ((int64_t)ngroups + 7) / 8 * 8;
    if (parts > cap) parts = cap;
    return (int32_t)(parts < 8 ? 8 : parts);
}

}  // namespace

// Ranges for the bound pass: about 8 workgroups per CU for the query blocks
// at hand, a multiple of 8, at most one range per vectorgroup.
int32_t lin_bound_parts(int64_t nq, int32_t ngroups) {
    return xcd_parts(8 * (int64_t)device_cus(), (nq + kBoundQueries - 1) / kBoundQueries, ngroups);
}

hipError_t launch_lin_bound(const pdx_index *ix, const int32_t *sid, const float *q, int64_t nq, const float *qn,
                            const int32_t *bad, int32_t parts, int32_t stride, uint64_t *slots, int32_t k,
                            uint32_t *tau, hipStream_t s) {
    if (nq <= 0) return hipSuccess;
    const int32_t nqb = (int32_t)((nq + kBoundQueries - 1) / kBoundQueries);
    const unsigned grid = 8u * (unsigned)(parts / 8) * (unsigned)nqb;
    lin_bound_kernel<<<grid, 256, 0, s>>>(ix->pdx, sid, ix->n, ix->d, ix->ngroups, q, nq, qn, bad, parts, nqb,
                                          stride, slots, k);
    lin_tau_kernel<<<(unsigned)nq, 64, 0, s>>>(slots, parts, k, tau);
    return hipGetLastError();
}

hipError_t launch_lin_list(const pdx_index *ix, const int32_t *sid, const float *q, int64_t nq, const float *qn,
                           const int32_t *bad, const uint32_t *tau, uint64_t *cand, int32_t *cand_cnt, int32_t cap,
                           hipStream_t s) {
    if (nq <= 0) return hipSuccess;
    // four tiles per wave once there are queries for them
    const bool wide = nq > 64;
    const int64_t per_wg = wide ? kListQueries : 64;
    const int32_t nqb = (int32_t)((nq + per_wg - 1) / per_wg);
    // ranges: about 32 workgroups per CU in all, so the last ones to finish
    // leave little of the chip idle
    const int32_t parts = xcd_parts(32 * (int64_t)device_cus(), nqb, ix->ngroups);
    const unsigned grid = 8u * (unsigned)(parts / 8) * (unsigned)nqb;
    if (wide)
        lin_list_kernel<kListTiles><<<grid, 256, 0, s>>>(ix->pdx, sid, ix->n, ix->d, ix->ngroups, q, nq, qn, bad,
                                                         parts, nqb, tau, cand, cand_cnt, cap);
    else
        lin_list_kernel<1><<<grid, 256, 0, s>>>(ix->pdx, sid, ix->n, ix->d, ix->ngroups, q, nq, qn, bad, parts, nqb,
                                                tau, cand, cand_cnt, cap);
    return hipGetLastError();
}

}  // namespace pdx
