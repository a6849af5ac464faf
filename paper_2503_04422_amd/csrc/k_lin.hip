// L2 linear mode on the matrix cores (the L2 kernel of Section 3's listing:
// every vector evaluated; exact).  Per 16 queries x 64 vectors a wave forms
// q.x with v_mfma_f32_16x16x4f32 and |x|^2 from the same loaded values, so
// each (query, vector) pair gets d' = |q|^2 + |x|^2 - 2 q.x.
//
// Margin: e = 4 (D + 64) 2^-24 (|q|^2 + |x|^2) bounds both d' - |q - x|^2
// and the fixed-order float32 sum's distance from |q - x|^2, so d' - e is
// below and d' + e above the distance every other path reports.
//
// Bound pass (every stride-th vectorgroup): each lane keeps, per query, the
// smallest d' + e over its own vectors (disjoint from every other lane's and
// range's), and a query's bound is the k-th smallest of these minima: k
// distinct vectors lie at or below it, so it bounds the query's k-th
// distance from above.  Listing pass (every vectorgroup): the vectors whose
// d' - e is at or below that bound, a superset of the k nearest.  The
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

constexpr int kTiles = 4;                  // 16-query tiles per wave once nq > 64
constexpr int kWideQueries = 4 * 16 * kTiles;  // queries per workgroup then

__host__ __device__ inline float lin_margin(int32_t d) { return 4.0f * (float)(d + 64) * 0x1p-24f; }

// The products of NT query tiles with every stride-th vectorgroup of
// [g0, g1) (g0 a multiple of stride): acc[u][t] = q.x and xx[t] = |x|^2 for
// the lane's slots, handed to epi(g, acc, xx) per vectorgroup.  The loads
// run half a sub-chunk ahead of the MFMAs, across vectorgroups too.
template <int NT, typename Epi>
__device__ __forceinline__ void scan_products(const float *__restrict__ pdxd, int32_t d, int32_t g0, int32_t g1,
                                              int32_t stride, int kq, int col, const float *const (&qrow)[NT],
                                              Epi &&epi) {
    const int32_t nfull = d / 32;  // whole sub-chunks; then a partial one when 32 does not divide D
    v4f b0[4], b1[4], a0[NT], a1[NT];
    if (nfull > 0) load_half<NT>(pdxd, (int64_t)g0 * d, 0, 0, kq, col, qrow, b0, a0);
    for (int32_t g = g0; g < g1; g += stride) {
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
            // one's first (after the last vectorgroup, the first one's first)
            const bool more = c + 1 < nfull;
            const int64_t gnext = more ? gbase : (g + stride < g1 ? gbase + (int64_t)stride * d : (int64_t)g0 * d);
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
        epi(g, acc, xx);
    }
}

// Per workgroup: its 64 NT queries' squared norms and, for the listing
// pass, bounds, staged in LDS (-inf: out of range or non-finite; a bound is
// never below 0 otherwise).
template <int NT, bool BOUNDS>
__device__ __forceinline__ void stage_queries(int64_t qblk, int64_t nq, const float *__restrict__ qn,
                                              const int32_t *__restrict__ bad, const uint32_t *__restrict__ tau,
                                              float *lqn, float *lbound) {
    for (int i = threadIdx.x; i < 64 * NT; i += 256) {
        const int64_t qi = qblk + i;
        const bool ok = qi < nq && !bad[qi];
        lqn[i] = ok ? qn[qi] : 0.0f;
        lbound[i] = !ok ? -INFINITY : (BOUNDS ? __uint_as_float(tau[qi]) : 0.0f);
    }
    __syncthreads();
}

// Bound pass.  Workgroups as in the listing pass, over every stride-th
// vectorgroup of their range; the lane's minimum of d' + e per query slot
// goes to mins[q][part][col] (+inf where the lane saw no vector).
template <int NT>
__global__ __launch_bounds__(256, 2) void lin_bound_kernel(
    const float *__restrict__ pdxd, const int32_t *__restrict__ slot_id, int64_t n, int32_t d, int32_t ngroups,
    const float *__restrict__ q, int64_t nq, const float *__restrict__ qn, const int32_t *__restrict__ bad,
    int32_t parts, int32_t nqb, int32_t stride, float *__restrict__ mins) {
    __shared__ float lqn[64 * NT], lok[64 * NT];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int col = lane & 15, kq = lane >> 4;
    const int32_t per_xcd = parts / 8;
    const int32_t x = blockIdx.x & 7, idx = blockIdx.x >> 3;
    const int32_t p = x * per_xcd + idx / nqb;
    const int64_t qblk = (int64_t)(idx % nqb) * (64 * NT);
    stage_queries<NT, false>(qblk, nq, qn, bad, nullptr, lqn, lok);
    const int64_t q0 = qblk + wave * (16 * NT);
    if (q0 >= nq) return;
    const float margin = lin_margin(d);
    const float *qrow[NT];
#pragma unroll
    for (int u = 0; u < NT; ++u) {
        const int64_t qc = q0 + 16 * u + col;
        qrow[u] = q + (qc < nq ? qc : q0) * d;
    }
    float best[NT][4];
#pragma unroll
    for (int u = 0; u < NT; ++u)
#pragma unroll
        for (int r = 0; r < 4; ++r) best[u][r] = INFINITY;
    const int32_t ga = (int32_t)((int64_t)ngroups * p / parts), g1 = (int32_t)((int64_t)ngroups * (p + 1) / parts);
    const int32_t g0 = (ga + stride - 1) / stride * stride;
    if (g0 < g1)
        scan_products<NT>(pdxd, d, g0, g1, stride, kq, col, qrow,
                          [&](int32_t g, const v4f (&acc)[NT][4], const float (&xx)[4]) {
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
                                      const float qq = lqn[wave * (16 * NT) + 16 * u + 4 * kq + r];
#pragma unroll
                                      for (int t = 0; t < 4; ++t) {
                                          const float nn = qq + xx[t];
                                          const float hi = fmaxf(nn - 2.0f * acc[u][t][r], 0.0f) + margin * nn;
                                          if (vok[t] && hi < best[u][r]) best[u][r] = hi;
                                      }
                                  }
                          });
#pragma unroll
    for (int u = 0; u < NT; ++u)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int i = wave * (16 * NT) + 16 * u + 4 * kq + r;
            const int64_t qr = qblk + i;
            if (qr < nq) mins[((size_t)qr * parts + p) * 16 + col] = lok[i] == -INFINITY ? INFINITY : best[u][r];
        }
}

// Each query's bound: the k-th smallest of its parts x 16 lane minima (+inf
// when fewer than k are finite).
__global__ __launch_bounds__(64) void lin_tau_kernel(const float *__restrict__ mins, int32_t parts, int32_t k,
                                                     uint32_t *__restrict__ tau) {
    const int64_t qi = blockIdx.x;
    const int lane = threadIdx.x;
    uint64_t e = kEmptyKey, kth = kEmptyKey;
    const float *src = mins + (size_t)qi * parts * 16;
    const int64_t total = (int64_t)parts * 16;
    for (int64_t i = lane; i - lane < total; i += 64) {
        const float v = i < total ? src[i] : INFINITY;
        const uint64_t key = make_key(v, (uint32_t)i);  // the index keeps equal minima apart
        topk_offer(e, kth, key, v < INFINITY, k, lane);
    }
    if (lane == 0) tau[qi] = kth == kEmptyKey ? kInfBits : static_cast<uint32_t>(kth >> 32);
}

// Listing pass.  A wave holds NT tiles of 16 queries, so each loaded value
// of a row feeds 4 NT MFMAs; a workgroup holds 4 waves of different queries
// over the same range of vectorgroups (the rows reach the four through the
// CU's L1).  A vector whose lower bound d' - e is at or below its query's
// bound is appended to that query's list (row slot; the count runs on past
// cap when the list overflows).
template <int NT>
__global__ __launch_bounds__(256, 2) void lin_list_kernel(
    const float *__restrict__ pdxd, const int32_t *__restrict__ slot_id, int64_t n, int32_t d, int32_t ngroups,
    const float *__restrict__ q, int64_t nq, const float *__restrict__ qn, const int32_t *__restrict__ bad,
    int32_t parts, int32_t nqb, const uint32_t *__restrict__ tau, uint64_t *__restrict__ cand,
    int32_t *__restrict__ cand_cnt, int32_t cap) {
    __shared__ float lqn[64 * NT], lbound[64 * NT];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int col = lane & 15, kq = lane >> 4;
    const int32_t per_xcd = parts / 8;
    const int32_t x = blockIdx.x & 7, idx = blockIdx.x >> 3;
    const int32_t p = x * per_xcd + idx / nqb;
    const int64_t qblk = (int64_t)(idx % nqb) * (64 * NT);
    stage_queries<NT, true>(qblk, nq, qn, bad, tau, lqn, lbound);
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
    scan_products<NT>(pdxd, d, g0, g1, 1, kq, col, qrow,
                      [&](int32_t g, const v4f (&acc)[NT][4], const float (&xx)[4]) {
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
                                          if (pos < cap)
                                              cand[qr * cap + pos] = (uint64_t)(uint32_t)(g * kGroup + 4 * col + t);
                                      }
                                  }
                              }
                      });
}

int32_t xcd_parts(int64_t want_wg, int64_t nqb, int32_t ngroups) {
    int64_t parts = (want_wg + nqb - 1) / (nqb > 0 ? nqb : 1);
    parts = (parts + 7) / 8 * 8;
    const int64_t cap = ((int64_t)ngroups + 7) / 8 * 8;
    if (parts > cap) parts = cap;
    return (int32_t)(parts < 8 ? 8 : parts);
}

}  // namespace

// Ranges of the bound pass: about 4 workgroups per CU for the query blocks
// at hand (each range then holds several of the vectorgroups it visits), a
// multiple of 8, at most one range per vectorgroup.
int32_t lin_bound_parts(int64_t nq, int32_t ngroups) {
    const int64_t per_wg = nq > 64 ? kWideQueries : 64;
    return xcd_parts(4 * (int64_t)device_cus(), (nq + per_wg - 1) / per_wg, ngroups);
}

hipError_t launch_lin_bound(const pdx_index *ix, const int32_t *sid, const float *q, int64_t nq, const float *qn,
                            const int32_t *bad, int32_t parts, int32_t stride, float *mins, int32_t k,
                            uint32_t *tau, hipStream_t s) {
    if (nq <= 0) return hipSuccess;
    const bool wide = nq > 64;  // four tiles per wave once there are queries for them
    const int64_t per_wg = wide ? kWideQueries : 64;
    const int32_t nqb = (int32_t)((nq + per_wg - 1) / per_wg);
    const unsigned grid = 8u * (unsigned)(parts / 8) * (unsigned)nqb;
    if (wide)
        lin_bound_kernel<kTiles><<<grid, 256, 0, s>>>(ix->pdx, sid, ix->n, ix->d, ix->ngroups, q, nq, qn, bad, parts,
                                                      nqb, stride, mins);
    else
        lin_bound_kernel<1><<<grid, 256, 0, s>>>(ix->pdx, sid, ix->n, ix->d, ix->ngroups, q, nq, qn, bad, parts, nqb,
                                                 stride, mins);
    lin_tau_kernel<<<(unsigned)nq, 64, 0, s>>>(mins, parts, k, tau);
    return hipGetLastError();
}

hipError_t launch_lin_list(const pdx_index *ix, const int32_t *sid, const float *q, int64_t nq, const float *qn,
                           const int32_t *bad, const uint32_t *tau, uint64_t *cand, int32_t *cand_cnt, int32_t cap,
                           hipStream_t s) {
    if (nq <= 0) return hipSuccess;
    const bool wide = nq > 64;  // four tiles per wave once there are queries for them
    const int64_t per_wg = wide ? kWideQueries : 64;
    const int32_t nqb = (int32_t)((nq + per_wg - 1) / per_wg);
    // ranges: about 32 workgroups per CU in all, so the last ones to finish
    // leave little of the chip idle
    const int32_t parts = xcd_parts(32 * (int64_t)device_cus(), nqb, ix->ngroups);
    const unsigned grid = 8u * (unsigned)(parts / 8) * (unsigned)nqb;
    if (wide)
        lin_list_kernel<kTiles><<<grid, 256, 0, s>>>(ix->pdx, sid, ix->n, ix->d, ix->ngroups, q, nq, qn, bad, parts,
                                                     nqb, tau, cand, cand_cnt, cap);
    else
        lin_list_kernel<1><<<grid, 256, 0, s>>>(ix->pdx, sid, ix->n, ix->d, ix->ngroups, q, nq, qn, bad, parts, nqb,
                                                tau, cand, cand_cnt, cap);
    return hipGetLastError();
}

}  // namespace pdx
