// C = A B^T on the matrix cores: A [m][k], B [n][k] row-major float32,
// C [m][n] (leading dimension ldc).  Used for the random rotation of rows
// and queries (x -> R x, Section 2.3), a dense product where every output
// needs every input.
//
// 128 x 128 output tile per 256-thread workgroup (4 waves, 64 x 64 each as
// 4 x 4 tiles of v_mfma_f32_16x16x4f32), 32-deep k slices staged in LDS
// row-major (stride 36 floats: 16-byte rows, two passes per 16-lane read).
// In K-step s of a slice, lane row kq stands for k = 8 kq + s, for A and B
// alike, so each lane reads its 8 consecutive k values with two 16-byte LDS
// reads.  The next slice's global loads are issued before the current
// slice's MFMAs.  Rows and k beyond the matrices read as zero.
#include <rocblas/rocblas.h>

#include <mutex>

#include "pdx_internal.h"

namespace pdx {
namespace {

typedef float v4f __attribute__((ext_vector_type(4)));

constexpr int BM = 128, BN = 128, BK = 32;
constexpr int LDS_STRIDE = BK + 4;

// 128 rows x 32 k of a row-major matrix: thread t loads rows t/8 + 32 u
// (u = 0..3), k = 4 (t % 8) .. +3 (8 threads read 128 contiguous bytes).
__device__ __forceinline__ void load_slice(const float *__restrict__ M, int64_t rows, int32_t k, int64_t r0,
                                           int32_t k0, bool vec, v4f (&v)[4]) {
    const int t = threadIdx.x;
    const int kc = (t & 7) * 4;
#pragma unroll
    for (int u = 0; u < 4; ++u) {
        const int64_t r = r0 + (t >> 3) + 32 * u;
        v4f x = {0.0f, 0.0f, 0.0f, 0.0f};
        if (r < rows) {
            const float *p = M + r * k + k0 + kc;
            if (vec && k0 + kc + 4 <= k) {
                x = *reinterpret_cast<const v4f *>(p);
            } else {
#pragma unroll
                for (int e = 0; e < 4; ++e) x[e] = (k0 + kc + e < k) ? p[e] : 0.0f;
            }
        }
        v[u] = x;
    }
}

__device__ __forceinline__ void store_slice(float (*S)[LDS_STRIDE], const v4f (&v)[4]) {
    const int t = threadIdx.x;
    const int kc = (t & 7) * 4;
#pragma unroll
    for (int u = 0; u < 4; ++u) *reinterpret_cast<v4f *>(&S[(t >> 3) + 32 * u][kc]) = v[u];
}

__global__ __launch_bounds__(256) void gemm_abt_kernel(const float *__restrict__ A, int64_t m,
                                                       const float *__restrict__ B, int64_t n, int32_t k,
                                                       float *__restrict__ C, int64_t ldc) {
    __shared__ __attribute__((aligned(16))) float As[BM][LDS_STRIDE];
    __shared__ __attribute__((aligned(16))) float Bs[BN][LDS_STRIDE];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int col = lane & 15, kq = lane >> 4;
    const int wm = (wave & 1) * 64, wn = (wave >> 1) * 64;
    const int64_t m0 = (int64_t)blockIdx.x * BM, n0 = (int64_t)blockIdx.y * BN;
    const bool vec = (k & 3) == 0;
    v4f acc[4][4];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = v4f{0.0f, 0.0f, 0.0f, 0.0f};
    v4f ra[4], rb[4];
    load_slice(A, m, k, m0, 0, vec, ra);
    load_slice(B, n, k, n0, 0, vec, rb);
    for (int32_t k0 = 0; k0 < k; k0 += BK) {
        __syncthreads();  // the previous slice's reads are done
        store_slice(As, ra);
        store_slice(Bs, rb);
        __syncthreads();
        if (k0 + BK < k) {  // next slice in flight during this slice's MFMAs
            load_slice(A, m, k, m0, k0 + BK, vec, ra);
            load_slice(B, n, k, n0, k0 + BK, vec, rb);
        }
        v4f a[4][2], b[4][2];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            a[i][0] = *reinterpret_cast<const v4f *>(&As[wm + 16 * i + col][8 * kq]);
            a[i][1] = *reinterpret_cast<const v4f *>(&As[wm + 16 * i + col][8 * kq + 4]);
            b[i][0] = *reinterpret_cast<const v4f *>(&Bs[wn + 16 * i + col][8 * kq]);
            b[i][1] = *reinterpret_cast<const v4f *>(&Bs[wn + 16 * i + col][8 * kq + 4]);
        }
#pragma unroll
        for (int s = 0; s < 8; ++s)
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
                for (int j = 0; j < 4; ++j)
                    acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[i][s >> 2][s & 3], b[j][s >> 2][s & 3],
                                                                     acc[i][j], 0, 0, 0);
    }
    // D of tile (i, j): lane holds rows 4 kq + r, column col
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int64_t c = n0 + wn + 16 * j + col;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int64_t row = m0 + wm + 16 * i + 4 * kq + r;
                if (row < m && c < n) C[row * ldc + c] = acc[i][j][r];
            }
        }
}

}  // namespace

hipError_t launch_gemm_abt(const float *A, int64_t m, const float *B, int64_t n, int32_t k, float *C, int64_t ldc,
                           hipStream_t s) {
    if (m <= 0 || n <= 0) return hipSuccess;
    const dim3 grid((unsigned)((m + BM - 1) / BM), (unsigned)((n + BN - 1) / BN));
    gemm_abt_kernel<<<grid, 256, 0, s>>>(A, m, B, n, k, C, ldc);
    return hipGetLastError();
}

// The same product through rocBLAS's f32 GEMM (a plain library GEMM: the
// IVF query rotation, the query x centroid products, the build's rotation
// of the rows).  Row-major C = A B^T is column-major C^T = B^T' A^T', i.e.
// sgemm(T, N) on the column-major views of B [k][n] and A [k][m].  One
// handle per device, created on first use (it allocates); calls that share
// it are serialised around the stream binding.
namespace {
std::mutex g_blas_mu;
rocblas_handle g_blas[64] = {};
}  // namespace

hipError_t launch_sgemm_abt(const float *A, int64_t m, const float *B, int64_t n, int32_t k, float *C, int64_t ldc,
                            hipStream_t s) {
    if (m <= 0 || n <= 0) return hipSuccess;
    if (m > INT32_MAX || n > INT32_MAX || ldc > INT32_MAX) return hipErrorInvalidValue;
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= 64) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_blas_mu);
    if (!g_blas[dev] && rocblas_create_handle(&g_blas[dev]) != rocblas_status_success) {
        g_blas[dev] = nullptr;
        return hipErrorOutOfMemory;
    }
    rocblas_handle h = g_blas[dev];
    if (rocblas_set_stream(h, s) != rocblas_status_success) return hipErrorInvalidHandle;
    const float one = 1.0f, zero = 0.0f;
    const rocblas_status st = rocblas_sgemm(h, rocblas_operation_transpose, rocblas_operation_none, (rocblas_int)n,
                                            (rocblas_int)m, k, &one, B, k, A, k, &zero, C, (rocblas_int)ldc);
    return st == rocblas_status_success ? hipGetLastError() : hipErrorLaunchFailure;
}

}  // namespace pdx
