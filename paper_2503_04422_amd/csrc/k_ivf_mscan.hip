// IVF bucket scan on the matrix cores: 16 queries x one vectorgroup (64
// vectors) per wave, the chunk's dot products as v_mfma_f32_16x16x4f32.
//
// Same work items, thresholds, prune test (ADSampling or the learned
// multipliers) and per-item k-best output
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
//
// Low-precision storage with chunks of whole 32-dimension sub-chunks (LP):
// the stored codes feed v_mfma_f32_16x16x32_bf16 directly (bfloat16 as
// stored; e4m3 converted exactly to bfloat16, its per-dimension scale
// folded into the query), one MFMA per vector quad t and query term with
// lane (kq, col) holding dimensions j0 + 8 kq .. + 7 of its row / column.
// The f32 query (times the scale for e4m3) is split into three bfloat16
// terms h + m + l (each the rounding of what the previous left), whose
// exact products accumulate in f32, so the dot products keep f32 accuracy.
// Per sub-chunk, |x_C|^2 of the decoded values is stored at build time and
// |q_C|^2 computed once per query:
//     sum_{j in C} (q_j - x_j)^2 = |q_C|^2 + |x_C|^2 - 2 q_C.x_C,
// uncentred (the codes cannot be re-centred exactly), clamped at 0.
#include "pdx_internal.h"
#include "wave_topk.h"
#include "wide_sink.h"

namespace pdx {
namespace {

typedef float v4f __attribute__((ext_vector_type(4)));
typedef __bf16 v8bf __attribute__((ext_vector_type(8)));

// Two 16-bit halves (byte selector of v_perm_b32): low halves of lo and
// hi, or high halves, packed lo | hi << 16.
constexpr uint32_t kPermLo = 0x05040100u, kPermHi = 0x07060302u;

__device__ __forceinline__ v8bf as_v8bf(uint4 u) { return __builtin_bit_cast(v8bf, u); }

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

// One (batch, part) work unit: MT tiles of 16 queries (a batch of 16 MT
// items) share every loaded value of the bucket; part p of the slots.parts
// waves sharing a batch scans vectorgroups p, p + parts, ... of the bucket.
// The queries' k-best lists live in LDS (list m, lane i = its i-th entry)
// and are read into a register only when they get offers.  WIDE (one tile,
// one wave per batch): survivors below the query's threshold go to its
// candidate buffer instead, one reservation per (query, vectorgroup); a
// query whose reservation does not fit stops there, recorded for a resume
// round, and the batch goes on without it.
template <bool PRUNE, int STORE, int MT, bool LP, bool WIDE>
__device__ __forceinline__ void mscan_unit(
    const void *__restrict__ pdxd, const float *__restrict__ scale, int32_t d, const int32_t *__restrict__ slot_id,
    const int32_t *__restrict__ goff, const float *__restrict__ cen, const int2 *__restrict__ items, int64_t b,
    int32_t part, const int32_t *__restrict__ probe, int32_t nprobe, const float *__restrict__ qrot,
    uint32_t *__restrict__ tau, const int32_t *__restrict__ bad, const SlotMap &slots, int32_t chunk,
    const PruneRule &rule, unsigned long long *__restrict__ counters, uint64_t (*lists)[kWave],
    const LpOperands &lp, const WideSink &wide) {
    static_assert(!WIDE || MT == 1, "candidate buffers: one tile per wave");
    constexpr int NQ = 16 * MT;
    const int lane = threadIdx.x & 63;
    const int col = lane & 15, kq = lane >> 4;
    const int32_t k = slots.kk;
    int2 mine[MT];  // query slot 16 mt + col (same in the 4 lane rows)
#pragma unroll
    for (int mt = 0; mt < MT; ++mt) mine[mt] = items[b * NQ + 16 * mt + col];
    const int32_t q0 = __builtin_amdgcn_readfirstlane(mine[0].x);
    if (q0 < 0) return;  // unused capacity (a batch otherwise starts with a real item)
    const int32_t l = probe[(int64_t)q0 * nprobe + __builtin_amdgcn_readfirstlane(mine[0].y)];
    bool row_ok[MT];
    uint32_t use = 0;  // bit 16 mt + m: query slot m of tile mt is scanned
#pragma unroll
    for (int mt = 0; mt < MT; ++mt) {
        row_ok[mt] = mine[mt].x >= 0 && !bad[mine[mt].x];
        use |= (uint32_t)(__ballot(row_ok[mt]) & 0xffffull) << (16 * mt);
        // items of non-finite queries get an empty list
        if (!WIDE && mine[mt].x >= 0 && !row_ok[mt] && kq == 0)
            for (int i = 0; i < k; ++i) slots.at(mine[mt].x, mine[mt].y, part)[i] = kEmptyKey;
    }
    if (!use) return;
    const float *qrow[MT];
#pragma unroll
    for (int mt = 0; mt < MT; ++mt) qrow[mt] = qrot + (int64_t)(row_ok[mt] ? mine[mt].x : q0) * d;
    const float *crow = cen + (int64_t)l * d;
    // query slots of this lane's D rows
    int32_t rowq[MT][4];
    float rowe[MT][4];  // learned bound of the row's (query, bucket)
    bool rowuse[MT][4];
    float kthr[MT][4];  // k-th distance of the query in D row 4 kq + r of tile mt
#pragma unroll
    for (int mt = 0; mt < MT; ++mt)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            rowq[mt][r] = __shfl(mine[mt].x, 4 * kq + r);
            const int32_t rr = __shfl(mine[mt].y, 4 * kq + r);
            rowuse[mt][r] = (use >> (16 * mt + 4 * kq + r)) & 1u;
            rowe[mt][r] = (PRUNE && rule.eps && rowuse[mt][r]) ? rule.eps_at(rowq[mt][r], rr, nprobe) : 0.0f;
            kthr[mt][r] = INFINITY;
        }
    if constexpr (!WIDE) {
#pragma unroll
        for (int m = 0; m < NQ; ++m) lists[m][lane] = kEmptyKey;
    }
    const bool vec_ok = (d & 3) == 0;
    unsigned long long live_vals = 0, lane_vals = 0;
    // LP: one sub-chunk's codes in registers (dimensions jl .. jl + 7 of
    // vectors 4 col .. 4 col + 3: 8 uint2 of bfloat16 or 8 words of e4m3)
    // and the vectors' norms; fetched one sub-chunk ahead
    struct LpRaw {
        uint32_t b[STORE == PDX_DTYPE_BF16 ? 16 : 8];
        v4f xn;
    };
    int64_t gbase_lp = 0, xn_row = 0;
    auto lp_fetch = [&](LpRaw &r, int32_t j0) {
        const int32_t jl = j0 + 8 * kq;
        constexpr int W = STORE == PDX_DTYPE_BF16 ? 2 : 1;   // words per lane and dimension
        constexpr int EB = STORE == PDX_DTYPE_BF16 ? 2 : 1;  // bytes per code
        constexpr int ROWW = kGroup * EB / 4;                 // words per dimension row of a group
        if (jl + 8 <= d) {  // whole: one base address, constant offsets
            const uint32_t *p = reinterpret_cast<const uint32_t *>(
                static_cast<const uint8_t *>(pdxd) + ((gbase_lp + jl) * kGroup + 4 * col) * EB);
#pragma unroll
            for (int s8 = 0; s8 < 8; ++s8)
#pragma unroll
                for (int w = 0; w < W; ++w) r.b[W * s8 + w] = p[s8 * ROWW + w];
        } else {  // the ragged end of D: clamped addresses, zeros past D
#pragma unroll
            for (int s8 = 0; s8 < 8; ++s8) {
                const bool ok = jl + s8 < d;
                const uint32_t *p = reinterpret_cast<const uint32_t *>(
                    static_cast<const uint8_t *>(pdxd) +
                    ((gbase_lp + (ok ? jl + s8 : d - 1)) * kGroup + 4 * col) * EB);
#pragma unroll
                for (int w = 0; w < W; ++w) r.b[W * s8 + w] = ok ? p[w] : 0u;
            }
        }
        r.xn = *reinterpret_cast<const v4f *>(lp.xn + (xn_row + (j0 >> 5)) * kGroup + 4 * col);
    };

    for (int32_t g = goff[l] + part; g < goff[l + 1]; g += slots.parts) {
        const int4 vq = *reinterpret_cast<const int4 *>(slot_id + (int64_t)g * kGroup + 4 * col);
        const int32_t vid[4] = {vq.x, vq.y, vq.z, vq.w};
        float teff[MT][4];
        uint32_t alive = 0;  // bit 16 mt + 4 r + t: (tile mt, row r, vector quad t) alive
#pragma unroll
        for (int mt = 0; mt < MT; ++mt)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                teff[mt][r] = INFINITY;
                if ((PRUNE || WIDE) && rowuse[mt][r]) {
                    const uint32_t tg =
                        __hip_atomic_load(tau + rowq[mt][r], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    // the candidate buffer's threshold bounds its R-th distance
                    teff[mt][r] = WIDE ? __uint_as_float(tg) : fminf(__uint_as_float(tg), kthr[mt][r]);
                }
#pragma unroll
                for (int t = 0; t < 4; ++t)
                    if (rowuse[mt][r] && vid[t] >= 0) alive |= 1u << (16 * mt + 4 * r + t);
            }
        float part_[MT][4][4];
#pragma unroll
        for (int mt = 0; mt < MT; ++mt)
#pragma unroll
            for (int r = 0; r < 4; ++r)
#pragma unroll
                for (int t = 0; t < 4; ++t) part_[mt][r][t] = 0.0f;
        const int64_t gbase = (int64_t)g * d;
        LpRaw cur;
        if constexpr (LP) {
            gbase_lp = gbase;
            xn_row = (int64_t)g * lp.nsub;
            lp_fetch(cur, 0);
        }
        for (int32_t c0 = 0; c0 < d; c0 += chunk) {
            // tiles with a live pair (wave-uniform); the others skip their MFMAs
            uint32_t tl = 0;
#pragma unroll
            for (int mt = 0; mt < MT; ++mt) tl |= (__ballot(((alive >> (16 * mt)) & 0xffffu) != 0u) ? 1u : 0u) << mt;
            if (PRUNE && !tl) break;
            const int32_t c1 = min(c0 + chunk, d);
            if (counters) {  // live (query, vector) pairs, and the pairs the MFMAs compute
                int pairs = __popc(alive);
#pragma unroll
                for (int off = 1; off < 64; off <<= 1) pairs += __shfl_xor(pairs, off);
                live_vals += (unsigned long long)pairs * (c1 - c0);
                lane_vals += 1024ull * __popc(tl) * (c1 - c0);
            }
            v4f acc[MT][4];
            float qq[MT];
            float qs[MT][4];  // LP: |q_C|^2 of the query in D row 4 kq + r
#pragma unroll
            for (int mt = 0; mt < MT; ++mt) {
                qq[mt] = 0.0f;
#pragma unroll
                for (int t = 0; t < 4; ++t) acc[mt][t] = v4f{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
                for (int r = 0; r < 4; ++r) qs[mt][r] = 0.0f;
            }
            float xx[4] = {0.0f, 0.0f, 0.0f, 0.0f};
            if constexpr (LP) {
                for (int32_t j0 = c0; j0 < c1; j0 += 32) {
                    // fetch the next sub-chunk while this one's MFMAs run
                    LpRaw nxt;
                    const bool more = j0 + 32 < d;
                    if (more) lp_fetch(nxt, j0 + 32);
                    uint32_t bw[4][4];
                    if constexpr (STORE == PDX_DTYPE_BF16) {
#pragma unroll
                        for (int p2 = 0; p2 < 4; ++p2) {
                            const uint32_t *u0 = cur.b + 4 * p2, *u1 = cur.b + 4 * p2 + 2;  // dims 2 p2, 2 p2 + 1
                            bw[0][p2] = __builtin_amdgcn_perm(u1[0], u0[0], kPermLo);
                            bw[1][p2] = __builtin_amdgcn_perm(u1[0], u0[0], kPermHi);
                            bw[2][p2] = __builtin_amdgcn_perm(u1[1], u0[1], kPermLo);
                            bw[3][p2] = __builtin_amdgcn_perm(u1[1], u0[1], kPermHi);
                        }
                    } else {
                        // e4m3 -> f32 is exact, and so is its top half as bfloat16
                        uint32_t f[8][4];
#pragma unroll
                        for (int s8 = 0; s8 < 8; ++s8) {
                            const auto lo = __builtin_amdgcn_cvt_pk_f32_fp8((int)cur.b[s8], false);
                            const auto hi = __builtin_amdgcn_cvt_pk_f32_fp8((int)cur.b[s8], true);
                            f[s8][0] = __float_as_uint(lo[0]);
                            f[s8][1] = __float_as_uint(lo[1]);
                            f[s8][2] = __float_as_uint(hi[0]);
                            f[s8][3] = __float_as_uint(hi[1]);
                        }
#pragma unroll
                        for (int t = 0; t < 4; ++t)
#pragma unroll
                            for (int p2 = 0; p2 < 4; ++p2)
                                bw[t][p2] = __builtin_amdgcn_perm(f[2 * p2 + 1][t], f[2 * p2][t], kPermHi);
                    }
#pragma unroll
                    for (int t = 0; t < 4; ++t) xx[t] += cur.xn[t];
                    const int32_t jl = j0 + 8 * kq, sub = j0 >> 5;
#pragma unroll
                    for (int mt = 0; mt < MT; ++mt) {
                        if (!((tl >> mt) & 1u)) continue;
                        const uint16_t *qa = lp.qs + (int64_t)(row_ok[mt] ? mine[mt].x : q0) * 3 * lp.dpad + jl;
                        uint4 a3[3];
#pragma unroll
                        for (int h = 0; h < 3; ++h) {
                            const uint4 v = *reinterpret_cast<const uint4 *>(qa + h * lp.dpad);
                            a3[h] = row_ok[mt] ? v : make_uint4(0u, 0u, 0u, 0u);
                        }
                        // smallest query term first; the four vector quads interleaved
#pragma unroll
                        for (int h = 2; h >= 0; --h)
#pragma unroll
                            for (int t = 0; t < 4; ++t)
                                acc[mt][t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(
                                    as_v8bf(a3[h]), as_v8bf(make_uint4(bw[t][0], bw[t][1], bw[t][2], bw[t][3])),
                                    acc[mt][t], 0, 0, 0);
#pragma unroll
                        for (int r = 0; r < 4; ++r)
                            if (rowuse[mt][r]) qs[mt][r] += lp.qn[(int64_t)rowq[mt][r] * lp.nsub + sub];
                    }
                    if (more) cur = nxt;
                }
            } else {
                for (int32_t j0 = c0; j0 < c1; j0 += 32) {
                    const int32_t jl = j0 + 8 * kq;  // this lane's first dimension of the sub-chunk
                    float cv[8], a[MT][8];
                    v4f bx[8];
                    if (j0 + 32 <= c1 && vec_ok && (j0 & 3) == 0) {
#pragma unroll
                        for (int s = 0; s < 8; ++s)
                            bx[s] = load_quad<STORE>(pdxd, scale, (gbase + jl + s) * kGroup + 4 * col, jl + s);
                        const v4f c_lo = *reinterpret_cast<const v4f *>(crow + jl);
                        const v4f c_hi = *reinterpret_cast<const v4f *>(crow + jl + 4);
#pragma unroll
                        for (int s = 0; s < 4; ++s) {
                            cv[s] = c_lo[s];
                            cv[s + 4] = c_hi[s];
                        }
#pragma unroll
                        for (int mt = 0; mt < MT; ++mt) {
                            const v4f q_lo = *reinterpret_cast<const v4f *>(qrow[mt] + jl);
                            const v4f q_hi = *reinterpret_cast<const v4f *>(qrow[mt] + jl + 4);
#pragma unroll
                            for (int s = 0; s < 4; ++s) {
                                a[mt][s] = row_ok[mt] ? q_lo[s] - cv[s] : 0.0f;
                                a[mt][s + 4] = row_ok[mt] ? q_hi[s] - cv[s + 4] : 0.0f;
                            }
                        }
                    } else {
#pragma unroll
                        for (int s = 0; s < 8; ++s) {
                            const int32_t j = jl + s;
                            const bool ok = j < c1;
                            cv[s] = ok ? crow[j] : 0.0f;
#pragma unroll
                            for (int mt = 0; mt < MT; ++mt) a[mt][s] = (ok && row_ok[mt]) ? qrow[mt][j] - cv[s] : 0.0f;
                            bx[s] = ok ? load_quad<STORE>(pdxd, scale, (gbase + j) * kGroup + 4 * col, j)
                                       : v4f{cv[s], cv[s], cv[s], cv[s]};
                        }
                    }
#pragma unroll
                    for (int s = 0; s < 8; ++s) {
                        const v4f bs = bx[s] - cv[s];
#pragma unroll
                        for (int t = 0; t < 4; ++t) xx[t] = fmaf(bs[t], bs[t], xx[t]);
#pragma unroll
                        for (int mt = 0; mt < MT; ++mt) {
                            if (!((tl >> mt) & 1u)) continue;
                            qq[mt] = fmaf(a[mt][s], a[mt][s], qq[mt]);
#pragma unroll
                            for (int t = 0; t < 4; ++t)
                                acc[mt][t] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[mt][s], bs[t], acc[mt][t], 0, 0, 0);
                        }
                    }
                }
                // |b|^2 per vector and |a|^2 per query slot over the chunk: sum the 4 k rows
#pragma unroll
                for (int t = 0; t < 4; ++t) {
                    xx[t] += __shfl_xor(xx[t], 16);
                    xx[t] += __shfl_xor(xx[t], 32);
                }
            }
            float fac = 1.0f, cdl = 0.0f, rsl = 0.0f;
            const bool learned = PRUNE && c1 < d && rule.eps;
            if (PRUNE && c1 < d && !rule.eps) fac = rule.ads(c1, d);
            if (learned) {
                cdl = (float)c1 / (float)d;
                rsl = prune_rs(c1);
            }
#pragma unroll
            for (int mt = 0; mt < MT; ++mt) {
                if (!((tl >> mt) & 1u)) continue;
                if constexpr (!LP) {
                    qq[mt] += __shfl_xor(qq[mt], 16);
                    qq[mt] += __shfl_xor(qq[mt], 32);
                }
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const float qn = LP ? qs[mt][r] : __shfl(qq[mt], 4 * kq + r);
                    const float fr = learned ? PruneRule::learned(rowe[mt][r], cdl, rsl) : fac;
#pragma unroll
                    for (int t = 0; t < 4; ++t) {
                        part_[mt][r][t] += fmaxf(qn + xx[t] - 2.0f * acc[mt][t][r], 0.0f);
                        // the prune test after c1 of d dimensions (exact at c1 = d)
                        if (PRUNE && part_[mt][r][t] > teff[mt][r] * fr) alive &= ~(1u << (16 * mt + 4 * r + t));
                    }
                }
            }
        }
        if constexpr (WIDE) {
            // survivors below the threshold go to their query's buffer
#pragma unroll
            for (int m = 0; m < NQ; ++m) {
                if (!((use >> m) & 1u)) continue;
                const int r = m & 3;
                const bool myrow = kq == (m >> 2);
                const int32_t qm = __builtin_amdgcn_readlane(mine[0].x, m);
                float dv[4];
                bool cand[4];
#pragma unroll
                for (int t = 0; t < 4; ++t) {
                    dv[t] = part_[0][r][t];
                    cand[t] = myrow && ((alive >> (4 * r + t)) & 1u) && dv[t] < teff[0][r];
                }
                if (!wide_push4(wide, qm, dv, vid, cand, wide.hbase[qm], tau, lane)) {
                    wide_overflow(wide, qm, __builtin_amdgcn_readlane(mine[0].y, m), g, lane);
                    use &= ~(1u << m);
                    if (myrow) rowuse[0][r] = false;
                }
            }
            if (!use) break;
        } else if (__any(alive != 0u)) {
            // survivors enter their query's k-best list
#pragma unroll
            for (int m = 0; m < NQ; ++m) {
                if (!((use >> m) & 1u)) continue;
                const int mt = m >> 4, mm = m & 15;
                const int r = mm & 3;
                const bool myrow = kq == (mm >> 2);
                unsigned long long any = 0;
#pragma unroll
                for (int t = 0; t < 4; ++t) any |= __ballot(myrow && ((alive >> (16 * mt + 4 * r + t)) & 1u));
                if (!any) continue;
                uint64_t em = lists[m][lane];
                uint64_t kth = readlane64(em, k - 1);
                const uint64_t before = kth;
#pragma unroll
                for (int t = 0; t < 4; ++t) {
                    const bool want = myrow && ((alive >> (16 * mt + 4 * r + t)) & 1u);
                    if (__ballot(want))
                        topk_offer(em, kth, make_key(part_[mt][r][t], (uint32_t)vid[t]), want, k, lane);
                }
                lists[m][lane] = em;
                if (kth != before) {
                    if (myrow) kthr[mt][r] = key_dist(kth);
                    if (PRUNE && lane == 0)
                        atomicMin(tau + __builtin_amdgcn_readlane(mine[mt].x, mm), (uint32_t)(kth >> 32));
                }
            }
        }
    }
    if constexpr (!WIDE) {
#pragma unroll
        for (int m = 0; m < NQ; ++m) {
            if (!((use >> m) & 1u)) continue;
            const int mt = m >> 4, mm = m & 15;
            const int32_t qm = __builtin_amdgcn_readlane(mine[mt].x, mm),
                          rm = __builtin_amdgcn_readlane(mine[mt].y, mm);
            if (lane < k) slots.at(qm, rm, part)[lane] = lists[m][lane];
        }
    }
    if (counters && lane == 0) {
        atomicAdd(counters, live_vals);
        atomicAdd(counters + 1, lane_vals);
    }
}

// Work units of XCD x (blockIdx.x % 8; workgroups are dealt to the XCDs
// round-robin) are the batches in [xcd_range[x], xcd_range[x + 1]) / 16 MT:
// all batches of a bucket run on one XCD and share its L2.  Each wave
// strides over its XCD's units.  Without xcd_range: unit = global wave index.
template <bool PRUNE, int STORE, int MT, bool LP, bool WIDE>
__global__ __launch_bounds__(256, (MT == 1 && !LP) ? 3 : 1) void ivf_mscan_kernel(
    const void *__restrict__ pdxd, const float *__restrict__ scale, int32_t d, const int32_t *__restrict__ slot_id,
    const int32_t *__restrict__ goff, const float *__restrict__ cen, const int2 *__restrict__ items, int64_t nbatch,
    const int32_t *__restrict__ xcd_range, const int32_t *__restrict__ probe, int32_t nprobe,
    const float *__restrict__ qrot, uint32_t *__restrict__ tau, const int32_t *__restrict__ bad, SlotMap slots,
    int32_t chunk, PruneRule rule, unsigned long long *__restrict__ counters, LpOperands lp, WideSink wide) {
    __shared__ uint64_t lists[4][WIDE ? 1 : 16 * MT][kWave];
    const int wave = threadIdx.x >> 6;
    const int64_t parts = slots.parts;
    if (!xcd_range) {
        const int64_t wid = (int64_t)blockIdx.x * 4 + wave;
        const int64_t b = wid / parts;
        if (b < nbatch)
            mscan_unit<PRUNE, STORE, MT, LP, WIDE>(pdxd, scale, d, slot_id, goff, cen, items, b,
                                                   (int32_t)(wid - b * parts), probe, nprobe, qrot, tau, bad, slots,
                                                   chunk, rule, counters, lists[wave], lp, wide);
        return;
    }
    const int32_t x = blockIdx.x & 7;
    const int64_t b0 = xcd_range[x] / (16 * MT), nb = xcd_range[x + 1] / (16 * MT) - b0;
    const int64_t stride = (int64_t)(gridDim.x >> 3) * 4;
    for (int64_t w = (int64_t)(blockIdx.x >> 3) * 4 + wave; w < nb * parts; w += stride) {
        const int64_t b = w / parts;
        mscan_unit<PRUNE, STORE, MT, LP, WIDE>(pdxd, scale, d, slot_id, goff, cen, items, b0 + b,
                                               (int32_t)(w - b * parts), probe, nprobe, qrot, tau, bad, slots, chunk,
                                               rule, counters, lists[wave], lp, wide);
    }
}

// Query operands of the LP scan: the three bfloat16 terms of q (times the
// e4m3 scale of each dimension when `scale` is given), zero-padded to dpad
// dimensions, and |q_C|^2 of the f32 query per 32-dimension sub-chunk.
__global__ __launch_bounds__(256) void lp_query_kernel(const float *__restrict__ qrot, int32_t d, int32_t dpad,
                                                       int32_t nsub, const float *__restrict__ scale,
                                                       uint16_t *__restrict__ qs, float *__restrict__ qn) {
    const int64_t q = blockIdx.x;
    const float *qp = qrot + q * d;
    uint16_t *o = qs + q * 3 * (int64_t)dpad;
    for (int32_t j = threadIdx.x; j < dpad; j += blockDim.x) {
        float v = j < d ? qp[j] : 0.0f;
        if (scale && j < d) v *= scale[j];
        const uint16_t h = bf16_encode(v);
        const float r1 = v - bf16_decode(h);  // exact
        const uint16_t m = bf16_encode(r1);
        const uint16_t l = bf16_encode(r1 - bf16_decode(m));
        o[j] = h;
        o[dpad + j] = m;
        o[2 * dpad + j] = l;
    }
    for (int32_t sb = threadIdx.x; sb < nsub; sb += blockDim.x) {
        float acc = 0.0f;
        for (int32_t j = 32 * sb; j < min(32 * sb + 32, d); ++j) acc = fmaf(qp[j], qp[j], acc);
        qn[q * nsub + sb] = acc;
    }
}

}  // namespace

hipError_t launch_lp_query(const float *qrot, int64_t nq, int32_t d, const float *scale, const LpOperands &lp,
                           hipStream_t s) {
    if (nq <= 0) return hipSuccess;
    lp_query_kernel<<<(unsigned)nq, 256, 0, s>>>(qrot, d, lp.dpad, lp.nsub, scale, const_cast<uint16_t *>(lp.qs),
                                                 const_cast<float *>(lp.qn));
    return hipGetLastError();
}

hipError_t launch_ivf_mscan(bool prune, int32_t store, int32_t tiles, const void *data, const float *scale,
                            int32_t d, const int32_t *slot_id, const int32_t *goff, const float *cen,
                            const int2 *items, int64_t nbatch, const int32_t *xcd_range, const int32_t *probe,
                            int32_t nprobe, const float *qrot, uint32_t *tau, const int32_t *bad, SlotMap slots,
                            int32_t chunk, PruneRule rule, unsigned long long *counters, const LpOperands &lp,
                            const WideSink *wide, hipStream_t s) {
    if (nbatch <= 0) return hipSuccess;
    // one wave per unit, or (XCD ranges) 8 equal sets of workgroups, an
    // eighth of the units each plus slack for uneven ranges
    const int64_t units = nbatch * slots.parts;
    const unsigned grid = xcd_range ? 8u * (unsigned)((units / 8 + 3) / 4 + 64) : (unsigned)((units + 3) / 4);
    const bool use_lp = lp.qs != nullptr && store != PDX_DTYPE_F32;
    if (wide) {  // candidate buffers: one tile per wave, one wave per batch, bfloat16 MFMA on the codes
        if (tiles != 1 || !use_lp || slots.parts != 1) return hipErrorInvalidValue;
#define PDX_MSCAN_W(P, S)                                                                                         \
    ivf_mscan_kernel<P, S, 1, true, true><<<grid, 256, 0, s>>>(data, scale, d, slot_id, goff, cen, items, nbatch, \
                                                               xcd_range, probe, nprobe, qrot, tau, bad, slots,    \
                                                               chunk, rule, counters, lp, *wide)
        if (prune) {
            if (store == PDX_DTYPE_BF16) PDX_MSCAN_W(true, PDX_DTYPE_BF16);
            else PDX_MSCAN_W(true, PDX_DTYPE_FP8);
        } else {
            if (store == PDX_DTYPE_BF16) PDX_MSCAN_W(false, PDX_DTYPE_BF16);
            else PDX_MSCAN_W(false, PDX_DTYPE_FP8);
        }
#undef PDX_MSCAN_W
        return hipGetLastError();
    }
    const WideSink none{};
#define PDX_MSCAN(P, S, M, L)                                                                                       \
    ivf_mscan_kernel<P, S, M, L, false><<<grid, 256, 0, s>>>(data, scale, d, slot_id, goff, cen, items, nbatch,   \
                                                             xcd_range, probe, nprobe, qrot, tau, bad, slots,      \
                                                             chunk, rule, counters, lp, none)
#define PDX_MSCAN_T(P, S, L)                \
    if (tiles == 2) PDX_MSCAN(P, S, 2, L);  \
    else PDX_MSCAN(P, S, 1, L);
    if (prune) {
        if (store == PDX_DTYPE_BF16) {
            if (use_lp) { PDX_MSCAN_T(true, PDX_DTYPE_BF16, true) }
            else { PDX_MSCAN_T(true, PDX_DTYPE_BF16, false) }
        } else if (store == PDX_DTYPE_FP8) {
            if (use_lp) { PDX_MSCAN_T(true, PDX_DTYPE_FP8, true) }
            else { PDX_MSCAN_T(true, PDX_DTYPE_FP8, false) }
        } else { PDX_MSCAN_T(true, PDX_DTYPE_F32, false) }
    } else {
        if (store == PDX_DTYPE_BF16) {
            if (use_lp) { PDX_MSCAN_T(false, PDX_DTYPE_BF16, true) }
            else { PDX_MSCAN_T(false, PDX_DTYPE_BF16, false) }
        } else if (store == PDX_DTYPE_FP8) {
            if (use_lp) { PDX_MSCAN_T(false, PDX_DTYPE_FP8, true) }
            else { PDX_MSCAN_T(false, PDX_DTYPE_FP8, false) }
        } else { PDX_MSCAN_T(false, PDX_DTYPE_F32, false) }
    }
#undef PDX_MSCAN_T
#undef PDX_MSCAN
    return hipGetLastError();
}

}  // namespace pdx
