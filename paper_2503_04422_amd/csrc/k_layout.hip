// Build-time kernels: finiteness check, N-ary -> PDX transposition and the
// per-dimension collection means.
//
// PDX layout (Section 3 and its kernel listing): vectorgroups of 64
// vectors; inside a group the 64 values of one dimension are contiguous,
// so a wave reads one dimension of a whole group as a single 256-byte row.
#include "pdx_internal.h"

namespace pdx {
namespace {

__global__ void finite_check_kernel(const float *__restrict__ x, int64_t count,
                                    int32_t *__restrict__ flag) {
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    int64_t stride = (int64_t)gridDim.x * blockDim.x;
    bool bad = false;
    for (; i < count; i += stride) bad |= !isfinite(x[i]);
    if (__any(bad) && (threadIdx.x & 63) == 0) atomicOr(flag, 1);
}

// One workgroup moves a 64-row x 64-dimension tile through LDS:
// coalesced 256-byte row reads in, coalesced 256-byte dimension rows out.
__global__ __launch_bounds__(256) void transpose_pdx_kernel(const float *__restrict__ x, int64_t n,
                                                            int32_t d, float *__restrict__ pdx) {
    __shared__ float tile[64][65];
    const int tx = threadIdx.x & 63;
    const int ty = threadIdx.x >> 6;
    const int64_t g = blockIdx.x;
    const int32_t c0 = blockIdx.y * 64;
#pragma unroll 4
    for (int r = 0; r < 64; r += 4) {
        int64_t row = g * 64 + r + ty;
        int32_t col = c0 + tx;
        tile[r + ty][tx] = (row < n && col < d) ? x[row * d + col] : 0.0f;
    }
    __syncthreads();
#pragma unroll 4
    for (int c = 0; c < 64; c += 4) {
        int32_t col = c0 + c + ty;
        if (col < d) pdx[(g * d + col) * 64 + tx] = tile[tx][c + ty];
    }
}

// partial[chunk][j] = sum of column j over the chunk's rows, in float64,
// rows added in increasing order (deterministic).
__global__ __launch_bounds__(256) void column_sums_kernel(const float *__restrict__ x, int64_t n,
                                                          int32_t d, int64_t rows_per_chunk,
                                                          double *__restrict__ partial) {
    int32_t j = blockIdx.x * 256 + threadIdx.x;
    int32_t c = blockIdx.y;
    if (j >= d) return;
    int64_t r0 = (int64_t)c * rows_per_chunk;
    int64_t r1 = r0 + rows_per_chunk < n ? r0 + rows_per_chunk : n;
    double s = 0.0;
    for (int64_t r = r0; r < r1; ++r) s += (double)x[r * d + j];
    partial[(int64_t)c * d + j] = s;
}

__global__ void column_means_finish_kernel(const double *__restrict__ partial, int32_t nchunks,
                                           int32_t d, int64_t n, float *__restrict__ means) {
    int32_t j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= d) return;
    double s = 0.0;
    for (int32_t c = 0; c < nchunks; ++c) s += partial[(int64_t)c * d + j];
    means[j] = (float)(s / (double)n);
}

}  // namespace

hipError_t launch_finite_check(const float *x, int64_t count, int32_t *flag, hipStream_t s) {
    if (count <= 0) return hipSuccess;
    int64_t blocks = (count + 255) / 256;
    if (blocks > 8192) blocks = 8192;
    finite_check_kernel<<<dim3((unsigned)blocks), dim3(256), 0, s>>>(x, count, flag);
    return hipGetLastError();
}

hipError_t launch_transpose_pdx(const float *x, int64_t n, int32_t d, float *pdx, hipStream_t s) {
    int64_t ng = (n + 63) / 64;
    transpose_pdx_kernel<<<dim3((unsigned)ng, (unsigned)((d + 63) / 64)), dim3(256), 0, s>>>(x, n, d,
                                                                                            pdx);
    return hipGetLastError();
}

hipError_t launch_column_means(const float *x, int64_t n, int32_t d, double *partial,
                               int32_t nchunks, float *means, hipStream_t s) {
    int64_t rows_per = (n + nchunks - 1) / nchunks;
    int32_t used = (int32_t)((n + rows_per - 1) / rows_per);
    column_sums_kernel<<<dim3((unsigned)((d + 255) / 256), (unsigned)used), dim3(256), 0, s>>>(
        x, n, d, rows_per, partial);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    column_means_finish_kernel<<<dim3((unsigned)((d + 255) / 256)), dim3(256), 0, s>>>(partial, used,
                                                                                     d, n, means);
    return hipGetLastError();
}

}  // namespace pdx
