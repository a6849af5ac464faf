// Operand loads and K-steps of the matrix-core scans whose waves hold NT
// tiles of 16 queries against one vectorgroup (v_mfma_f32_16x16x4f32).
//
// Lane layout (lane = 16 kq + col): A (16 x 4) holds query slot col at k
// index kq; B (4 x 16) holds k index kq for vector 4 col + t in MFMA t; D
// gives a lane query slots 4 kq + r against vector 4 col + t.  In K-step s
// of the 32-dimension sub-chunk starting at j0, k index kq stands for
// dimension j0 + 8 kq + s.  A lane loads its four vectors of a dimension
// with one 16-byte load (vectors 4 col .. 4 col + 3 are adjacent in a
// vectorgroup), and its query values of 4 dimensions with another (D a
// multiple of 4, so a row of q is 16-byte aligned).
#pragma once

#include "pdx_internal.h"

namespace pdx {

typedef float mx_v4f __attribute__((ext_vector_type(4)));

// Half h of a whole sub-chunk: K-steps 4h .. 4h + 3 (the lane's dimensions
// jl .. jl + 3, jl = j0 + 8 kq + 4h), its four vectors and NT query tiles'
// values.  Nothing reads the loaded values until that half's MFMAs, so the
// loads stay in flight across the other half's.
template <int NT>
__device__ __forceinline__ void load_half(const float *__restrict__ pdxd, int64_t gbase, int32_t j0, int h, int kq,
                                          int col, const float *const (&qrow)[NT], mx_v4f (&b)[4],
                                          mx_v4f (&a)[NT]) {
    const int32_t jl = j0 + 8 * kq + 4 * h;
#pragma unroll
    for (int u = 0; u < NT; ++u) a[u] = *reinterpret_cast<const mx_v4f *>(qrow[u] + jl);
#pragma unroll
    for (int s = 0; s < 4; ++s) b[s] = *reinterpret_cast<const mx_v4f *>(pdxd + (gbase + jl + s) * kGroup + 4 * col);
}

// The same for the last, partial sub-chunk (zero past D).
template <int NT>
__device__ __forceinline__ void load_half_tail(const float *__restrict__ pdxd, int64_t gbase, int32_t d, int32_t j0,
                                               int h, int kq, int col, const float *const (&qrow)[NT],
                                               mx_v4f (&b)[4], mx_v4f (&a)[NT]) {
    const int32_t jl = j0 + 8 * kq + 4 * h;
#pragma unroll
    for (int s = 0; s < 4; ++s) {
        const int32_t j = jl + s;
        const bool ok = j < d;
        b[s] = ok ? *reinterpret_cast<const mx_v4f *>(pdxd + (gbase + j) * kGroup + 4 * col)
                  : mx_v4f{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
        for (int u = 0; u < NT; ++u) a[u][s] = ok ? qrow[u][j] : 0.0f;
    }
}

// K-steps of one half: acc[u][t] += A(tile u) B(vectors 4 col + t); with
// NORMS also the vectors' squared norms (the lane's dimensions only).
template <int NT, bool NORMS>
__device__ __forceinline__ void mfma_half(const mx_v4f (&b)[4], const mx_v4f (&a)[NT], mx_v4f (&acc)[NT][4],
                                          float (&xx)[4]) {
#pragma unroll
    for (int s = 0; s < 4; ++s) {
#pragma unroll
        for (int u = 0; u < NT; ++u)
#pragma unroll
            for (int t = 0; t < 4; ++t)
                acc[u][t] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[u][s], b[s][t], acc[u][t], 0, 0, 0);
        if constexpr (NORMS) {
#pragma unroll
            for (int t = 0; t < 4; ++t) xx[t] = fmaf(b[s][t], b[s][t], xx[t]);
        }
    }
}

}  // namespace pdx
