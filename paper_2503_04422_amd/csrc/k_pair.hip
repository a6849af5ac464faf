// Tiled pairwise kernels between the rows of two row-major float32
// matrices A [m][k] and B [nb][k]:
//   DOT: C[i][j] = sum_t A[i][t] * B[j][t]      (rotation: X R^T)
//   L2 : C[i][j] = sum_t (A[i][t] - B[j][t])^2  (centroid distances)
//   L1 : C[i][j] = sum_t |A[i][t] - B[j][t]|    (L1 centroid distances)
// Output either stored (C, leading dimension ldc) or reduced per row of A
// to the nearest B row: an atomic minimum over the 64-bit key
// (distance bits << 32 | j), i.e. the smallest distance, ties to lower j
// (k-means assignment, Section 2.1 IVF).
//
// 64 x 64 output tile per 256-thread workgroup, 16-deep k slices staged in
// LDS, 4 x 4 outputs per thread, sums accumulated in k order with FMAs.
#include "pdx_internal.h"

namespace pdx {
namespace {

constexpr int TM = 64, TN = 64, TK = 16;

template <int MODE, int OUT>
__global__ __launch_bounds__(256) void pair_kernel(const float *__restrict__ A, int64_t m,
                                                   const float *__restrict__ B, int64_t nb, int32_t k,
                                                   float *__restrict__ C, int64_t ldc,
                                                   unsigned long long *__restrict__ best) {
    __shared__ float As[TK][TM + 4];
    __shared__ float Bs[TK][TN + 4];
    const int tx = threadIdx.x & 15;
    const int ty = threadIdx.x >> 4;
    const int64_t i0 = (int64_t)blockIdx.x * TM;
    const int64_t j0 = (int64_t)blockIdx.y * TN;
    float acc[4][4];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) acc[a][b] = 0.0f;
    // loader mapping: 64 rows x 16 k -> 4 values per thread
    const int lr = threadIdx.x >> 2;        // row in tile
    const int lk = (threadIdx.x & 3) * 4;   // k offset in slice
    for (int32_t t0 = 0; t0 < k; t0 += TK) {
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            int32_t t = t0 + lk + u;
            int64_t ia = i0 + lr, jb = j0 + lr;
            As[lk + u][lr] = (ia < m && t < k) ? A[ia * k + t] : 0.0f;
            Bs[lk + u][lr] = (jb < nb && t < k) ? B[jb * k + t] : 0.0f;
        }
        __syncthreads();
        const int kk_end = (k - t0) < TK ? (k - t0) : TK;
        for (int kk = 0; kk < kk_end; ++kk) {
            float a[4], b[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                a[u] = As[kk][ty + 16 * u];
                b[u] = Bs[kk][tx + 16 * u];
            }
#pragma unroll
            for (int u = 0; u < 4; ++u)
#pragma unroll
                for (int w = 0; w < 4; ++w) {
                    if (MODE == 0) {
                        acc[u][w] = fmaf(a[u], b[w], acc[u][w]);
                    } else if (MODE == 2) {
                        acc[u][w] += fabsf(a[u] - b[w]);
                    } else {
                        float dd = a[u] - b[w];
                        acc[u][w] = fmaf(dd, dd, acc[u][w]);
                    }
                }
        }
        __syncthreads();
    }
    if (OUT == 0) {
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            int64_t i = i0 + ty + 16 * u;
            if (i >= m) continue;
#pragma unroll
            for (int w = 0; w < 4; ++w) {
                int64_t j = j0 + tx + 16 * w;
                if (j < nb) C[i * ldc + j] = acc[u][w];
            }
        }
    } else {
        // per row: smallest (distance, column) among this thread's 4 columns,
        // then across the 16 threads sharing the row (lanes tx = 0..15)
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            int64_t i = i0 + ty + 16 * u;
            unsigned long long key = ~0ull;
#pragma unroll
            for (int w = 0; w < 4; ++w) {
                int64_t j = j0 + tx + 16 * w;
                if (j < nb) {
                    unsigned long long kk =
                        ((unsigned long long)__float_as_uint(acc[u][w]) << 32) | (unsigned long long)(uint32_t)j;
                    key = kk < key ? kk : key;
                }
            }
#pragma unroll
            for (int off = 1; off < 16; off <<= 1) {
                unsigned long long o = __shfl_xor(key, off, 16);
                key = o < key ? o : key;
            }
            if (tx == 0 && i < m && key != ~0ull) atomicMin(best + i, key);
        }
    }
}

}  // namespace

hipError_t launch_pair(int mode, int out, const float *A, int64_t m, const float *B, int64_t nb, int32_t k,
                       float *C, int64_t ldc, unsigned long long *best, hipStream_t s) {
    if (m <= 0 || nb <= 0) return hipSuccess;
    dim3 grid((unsigned)((m + TM - 1) / TM), (unsigned)((nb + TN - 1) / TN));
    if (mode == 0 && out == 0)
        pair_kernel<0, 0><<<grid, 256, 0, s>>>(A, m, B, nb, k, C, ldc, best);
    else if (mode == 1 && out == 0)
        pair_kernel<1, 0><<<grid, 256, 0, s>>>(A, m, B, nb, k, C, ldc, best);
    else if (mode == 1 && out == 1)
        pair_kernel<1, 1><<<grid, 256, 0, s>>>(A, m, B, nb, k, C, ldc, best);
    else if (mode == 2 && out == 0)
        pair_kernel<2, 0><<<grid, 256, 0, s>>>(A, m, B, nb, k, C, ldc, best);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

}  // namespace pdx
