// IVF bucket scan on the matrix cores: 16 queries x one vectorgroup (64
// vectors) per wave, the chunk's dot products as v_mfma_f32_16x16x4f32.
//
// Same work items, thresholds, ADSampling test and per-item k-best output
// as the vector-ALU scans (k_ivf_search.hip); only the arithmetic of the
// partial distances differs.  Per chunk of dimensions C,
//     sum_{j in C} (q_j - x_j)^2 = |a|^2 + |b|^2 - 2 a.b,
//     a = q_C - c_C,  b = x_C - c_C,
// with c the bucket's centroid: centring both operands on the centroid
// keeps |a|^2 + |b|^2 of the order of the distance itself, so the f32
// cancellation error stays a few units of roundoff of the partial.  Each
// chunk's term is clamped at 0 (it is a sum of squares).
//
// Lane layout (lane = 16 * kq + col):
//   A operand (16 x 4): row = query slot col, k = kq;
//   B operand (4 x 16): k = kq, column col, one MFMA per vector quad t:
//                       vector 4 * col + t of the group;
//   D (16 x 16), per t:  lane holds rows 4 * kq + r (r = 0..3), column col,
//                       i.e. query slot 4 * kq + r against vector 4 * col + t.
// In K-step s of a 32-dimension sub-chunk starting at j0, lane k index kq
// stands for dimension j0 + 8 * kq + s, for A and B alike.
#include "pdx_internal.h"
#include "wave_topk.h"

namespace pdx {
namespace {

typedef float v4f __attribute__((ext_vector_type(4)));

// Dimension j of vectors 4c..4c+3 of a group (`at` = element index of the
// first; a multiple of 4), decoded to f32.
template <int STORE>
__device__ __forceinline__ v4f load_quad(const void *__restrict__ data, const float *__restrict__ scale, int64_t at,
                                         int32_t j) {
    if (STORE == PDX_DTYPE_F32) return *reinterpret_cast<const v4f *>(static_cast<const float *>(data) + at);
    if (STORE == PDX_DTYPE_BF16) {
        const uint2 u = *reinterpret_cast<const uint2 *>(static_cast<const uint16_t *>(data) + at);
        return v4f{bf16_decode(u.x & 0xffffu), bf16_decode(u.x >> 16), bf16_decode(u.y & 0xffffu),
                   bf16_decode(u.y >> 16)};
    }
    const int u = *reinterpret_cast<const int *>(static_cast<const uint8_t *>(data) + at);
    const float sc = scale[j];
    return v4f{__builtin_amdgcn_cvt_f32_fp8(u, 0) * sc, __builtin_amdgcn_cvt_f32_fp8(u, 1) * sc,
               __builtin_amdgcn_cvt_f32_fp8(u, 2) * sc, __builtin_amdgcn_cvt_f32_fp8(u, 3) * sc};
}

template <bool PRUNE, int STORE>
__global__ __launch_bounds__(256) void ivf_mscan_kernel(
    const void *__restrict__ pdxd, const float *__restrict__ scale, int32_t d, const int32_t *__restrict__ slot_id,
    const int32_t *__restrict__ goff, const float *__restrict__ cen, const int2 *__restrict__ items, int64_t nbatch,
    const int32_t *__restrict__ probe, int32_t nprobe, const float *__restrict__ qrot,
    uint32_t *__restrict__ tau, const int32_t *__restrict__ bad, SlotMap slots, int32_t chunk, float eps0,
    unsigned long long *__restrict__ counters) {
    const int lane = threadIdx.x & 63;
    const int col = lane & 15, kq = lane >> 4;
    const int32_t k = slots.kk;
    // wave -> (batch, part): slots.parts waves share a batch, part p scans
    // vectorgroups p, p + parts, ... of the bucket
    const int64_t wid = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    const int64_t b = wid / slots.parts;
    const int32_t part = (int32_t)(wid - b * slots.parts);
    if (b >= nbatch) return;
    const int2 mine = items[b * 16 + col];  // query slot col (same in the 4 lane rows)
    const int32_t q0 = __builtin_amdgcn_readfirstlane(mine.x);
    if (q0 < 0) return;  // unused capacity (a batch otherwise starts with a real item)
    const int32_t l = probe[(int64_t)q0 * nprobe + __builtin_amdgcn_readfirstlane(mine.y)];
    bool row_ok = mine.x >= 0 && !bad[mine.x];
    const uint32_t use = (uint32_t)(__ballot(row_ok) & 0xffffull);  // bit m: query slot m is scanned
    // items of non-finite queries get an empty list
    if (mine.x >= 0 && !row_ok && kq == 0)
        for (int i = 0; i < k; ++i) slots.at(mine.x, mine.y, part)[i] = kEmptyKey;
    if (!use) return;
    const float *qrow = qrot + (int64_t)(row_ok ? mine.x : q0) * d;
    const float *crow = cen + (int64_t)l * d;
    // query slots of this lane's D rows
    int32_t rowq[4];
    bool rowuse[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        rowq[r] = __shfl(mine.x, 4 * kq + r);
        rowuse[r] = (use >> (4 * kq + r)) & 1u;
    }
    uint64_t e[16];
    float kthr[4];  // k-th distance of the query in D row 4 * kq + r
#pragma unroll
    for (int m = 0; m < 16; ++m) e[m] = kEmptyKey;
#pragma unroll
    for (int r = 0; r < 4; ++r) kthr[r] = INFINITY;
    const bool vec_ok = (d & 3) == 0;
    unsigned long long live_vals = 0, lane_vals = 0;

    for (int32_t g = goff[l] + part; g < goff[l + 1]; g += slots.parts) {
        const int4 vq = *reinterpret_cast<const int4 *>(slot_id + (int64_t)g * kGroup + 4 * col);
        const int32_t vid[4] = {vq.x, vq.y, vq.z, vq.w};
        float teff[4];
        uint32_t alive = 0;  // bit 4 r + t: (row r, vector quad t) alive
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            teff[r] = INFINITY;
            if (PRUNE && rowuse[r]) {
                const uint32_t tg = __hip_atomic_load(tau + rowq[r], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                teff[r] = fminf(__uint_as_float(tg), kthr[r]);
            }
#pragma unroll
            for (int t = 0; t < 4; ++t)
                if (rowuse[r] && vid[t] >= 0) alive |= 1u << (4 * r + t);
        }
        float part[4][4];
#pragma unroll
        for (int r = 0; r < 4; ++r)
#pragma unroll
            for (int t = 0; t < 4; ++t) part[r][t] = 0.0f;
        const int64_t gbase = (int64_t)g * d;
        for (int32_t c0 = 0; c0 < d; c0 += chunk) {
            if (PRUNE && !__any(alive != 0u)) break;
            const int32_t c1 = min(c0 + chunk, d);
            if (counters) {  // live (query, vector) pairs, and the 1024 pairs the MFMAs compute
                int pairs = __popc(alive);
#pragma unroll
                for (int off = 1; off < 64; off <<= 1) pairs += __shfl_xor(pairs, off);
                live_vals += (unsigned long long)pairs * (c1 - c0);
                lane_vals += 1024ull * (c1 - c0);
            }
            v4f acc[4];
#pragma unroll
            for (int t = 0; t < 4; ++t) acc[t] = v4f{0.0f, 0.0f, 0.0f, 0.0f};
            float qq = 0.0f;
            float xx[4] = {0.0f, 0.0f, 0.0f, 0.0f};
            for (int32_t j0 = c0; j0 < c1; j0 += 32) {
                const int32_t jl = j0 + 8 * kq;  // this lane's first dimension of the sub-chunk
                float cv[8], a[8];
                v4f bx[8];
                if (j0 + 32 <= c1 && vec_ok && (j0 & 3) == 0) {
                    const v4f c_lo = *reinterpret_cast<const v4f *>(crow + jl);
                    const v4f c_hi = *reinterpret_cast<const v4f *>(crow + jl + 4);
                    const v4f q_lo = *reinterpret_cast<const v4f *>(qrow + jl);
                    const v4f q_hi = *reinterpret_cast<const v4f *>(qrow + jl + 4);
#pragma unroll
                    for (int s = 0; s < 8; ++s)
                        bx[s] = load_quad<STORE>(pdxd, scale, (gbase + jl + s) * kGroup + 4 * col, jl + s);
#pragma unroll
                    for (int s = 0; s < 4; ++s) {
                        cv[s] = c_lo[s];
                        cv[s + 4] = c_hi[s];
                        a[s] = q_lo[s];
                        a[s + 4] = q_hi[s];
                    }
#pragma unroll
                    for (int s = 0; s < 8; ++s) a[s] = row_ok ? a[s] - cv[s] : 0.0f;
                } else {
#pragma unroll
                    for (int s = 0; s < 8; ++s) {
                        const int32_t j = jl + s;
                        const bool ok = j < c1;
                        cv[s] = ok ? crow[j] : 0.0f;
                        a[s] = (ok && row_ok) ? qrow[j] - cv[s] : 0.0f;
                        bx[s] = ok ? load_quad<STORE>(pdxd, scale, (gbase + j) * kGroup + 4 * col, j)
                                   : v4f{cv[s], cv[s], cv[s], cv[s]};
                    }
                }
#pragma unroll
                for (int s = 0; s < 8; ++s) {
                    const v4f bs = bx[s] - cv[s];
                    qq = fmaf(a[s], a[s], qq);
#pragma unroll
                    for (int t = 0; t < 4; ++t) {
                        xx[t] = fmaf(bs[t], bs[t], xx[t]);
                        acc[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[s], bs[t], acc[t], 0, 0, 0);
                    }
                }
            }
            // |a|^2 per query slot and |b|^2 per vector over the chunk: sum the 4 k rows
            qq += __shfl_xor(qq, 16);
            qq += __shfl_xor(qq, 32);
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                xx[t] += __shfl_xor(xx[t], 16);
                xx[t] += __shfl_xor(xx[t], 32);
            }
            float fac = 1.0f;
            if (PRUNE && c1 < d) {
                const float dc = (float)c1;
                const float f = 1.0f + eps0 / sqrtf(dc);
                fac = (dc / (float)d) * f * f;
            }
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const float qn = __shfl(qq, 4 * kq + r);
#pragma unroll
                for (int t = 0; t < 4; ++t) {
                    part[r][t] += fmaxf(qn + xx[t] - 2.0f * acc[t][r], 0.0f);
                    // ADSampling test after c1 of d dimensions (exact at c1 = d)
                    if (PRUNE && part[r][t] > teff[r] * fac) alive &= ~(1u << (4 * r + t));
                }
            }
        }
        // survivors enter their query's k-best list
        if (__any(alive != 0u)) {
#pragma unroll
            for (int m = 0; m < 16; ++m) {
                if (!((use >> m) & 1u)) continue;
                const int r = m & 3;
                const bool myrow = kq == (m >> 2);
                uint64_t kth = readlane64(e[m], k - 1);
                const uint64_t before = kth;
#pragma unroll
                for (int t = 0; t < 4; ++t) {
                    const bool want = myrow && ((alive >> (4 * r + t)) & 1u);
                    if (__ballot(want)) topk_offer(e[m], kth, make_key(part[r][t], (uint32_t)vid[t]), want, k, lane);
                }
                if (kth != before) {
                    if (myrow) kthr[r] = key_dist(kth);
                    if (PRUNE && lane == 0) atomicMin(tau + __builtin_amdgcn_readlane(mine.x, m), (uint32_t)(kth >> 32));
                }
            }
        }
    }
#pragma unroll
    for (int m = 0; m < 16; ++m) {
        if (!((use >> m) & 1u)) continue;
        const int32_t qm = __builtin_amdgcn_readlane(mine.x, m), rm = __builtin_amdgcn_readlane(mine.y, m);
        if (lane < k) slots.at(qm, rm, part)[lane] = e[m];
    }
    if (counters && lane == 0) {
        atomicAdd(counters, live_vals);
        atomicAdd(counters + 1, lane_vals);
    }
}

}  // namespace

hipError_t launch_ivf_mscan(bool prune, int32_t store, const void *data, const float *scale, int32_t d,
                            const int32_t *slot_id, const int32_t *goff, const float *cen, const int2 *items,
                            int64_t nbatch, const int32_t *probe, int32_t nprobe, const float *qrot, uint32_t *tau,
                            const int32_t *bad, SlotMap slots, int32_t chunk, float eps0,
                            unsigned long long *counters, hipStream_t s) {
    if (nbatch <= 0) return hipSuccess;
    const unsigned grid = (unsigned)((nbatch * slots.parts + 3) / 4);
#define PDX_MSCAN(P, S)                                                                                            \
    ivf_mscan_kernel<P, S><<<grid, 256, 0, s>>>(data, scale, d, slot_id, goff, cen, items, nbatch, probe, nprobe, \
                                                qrot, tau, bad, slots, chunk, eps0, counters)
    if (prune) {
        if (store == PDX_DTYPE_BF16) PDX_MSCAN(true, PDX_DTYPE_BF16);
        else if (store == PDX_DTYPE_FP8) PDX_MSCAN(true, PDX_DTYPE_FP8);
        else PDX_MSCAN(true, PDX_DTYPE_F32);
    } else {
        if (store == PDX_DTYPE_BF16) PDX_MSCAN(false, PDX_DTYPE_BF16);
        else if (store == PDX_DTYPE_FP8) PDX_MSCAN(false, PDX_DTYPE_FP8);
        else PDX_MSCAN(false, PDX_DTYPE_F32);
    }
#undef PDX_MSCAN
    return hipGetLastError();
}

}  // namespace pdx
