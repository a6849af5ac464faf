// Random orthogonal rotation for ADSampling (Section 2.3): float64
// Householder QR of a caller-drawn Gaussian matrix G, then the Haar sign
// fix Q <- Q diag(sign(diag(R))).  The rotation applied to a vector v is
// Q v, so rows are rotated as X Q^T.
//
// A is kept column-major (column c contiguous) so that reflecting a
// column is a contiguous dot product and update; Q is row-major so that
// accumulating Q <- Q H_j touches contiguous rows.  One reflection step
// is three launches: build v_j, reflect the trailing columns, update Q.
#include "pdx_internal.h"

namespace pdx {
namespace {

__device__ double block_sum(double v, double *red) {
    // 1024 threads: wave sums, then the first wave sums the partials
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    if (lane == 0) red[w] = v;
    __syncthreads();
    double t = 0.0;
    if (w == 0) {
        t = lane < (int)(blockDim.x >> 6) ? red[lane] : 0.0;
        for (int off = 32; off > 0; off >>= 1) t += __shfl_down(t, off);
        if (lane == 0) red[0] = t;
    }
    __syncthreads();
    t = red[0];
    __syncthreads();
    return t;
}

__global__ void qr_init_kernel(const double *__restrict__ g, int32_t d, double *__restrict__ acm,
                               double *__restrict__ q) {
    int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (idx >= (int64_t)d * d) return;
    int32_t r = (int32_t)(idx / d), c = (int32_t)(idx % d);
    acm[(int64_t)c * d + r] = g[idx];
    q[idx] = (r == c) ? 1.0 : 0.0;
}

// v = x - alpha e_0 (x = column j from row j down), alpha = -sign(x_0) |x|,
// normalised; diag[j] = alpha.  A zero column gives v = 0 (no reflection).
__global__ __launch_bounds__(1024) void qr_house_kernel(double *__restrict__ acm, int32_t d, int32_t j,
                                                        double *__restrict__ v, double *__restrict__ diag) {
    __shared__ double red[16];
    const double *col = acm + (int64_t)j * d;
    double ss = 0.0;
    for (int r = j + threadIdx.x; r < d; r += blockDim.x) ss += col[r] * col[r];
    double nrm2 = block_sum(ss, red);
    double x0 = col[j];
    double nrm = sqrt(nrm2);
    double alpha = x0 >= 0.0 ? -nrm : nrm;
    double vn2 = nrm2 - 2.0 * alpha * x0 + alpha * alpha;  // |x - alpha e0|^2
    double inv = vn2 > 0.0 ? 1.0 / sqrt(vn2) : 0.0;
    for (int r = threadIdx.x; r < d; r += blockDim.x) {
        double val = 0.0;
        if (r > j) val = col[r] * inv;
        else if (r == j) val = (x0 - alpha) * inv;
        v[r] = val;
    }
    if (threadIdx.x == 0) diag[j] = vn2 > 0.0 ? alpha : x0;
}

// trailing columns c > j: a_c <- a_c - 2 v (v . a_c); one workgroup per column
__global__ __launch_bounds__(256) void qr_apply_a_kernel(double *__restrict__ acm, int32_t d, int32_t j,
                                                         const double *__restrict__ v) {
    __shared__ double red[16];
    const int32_t c = j + 1 + blockIdx.x;
    double *col = acm + (int64_t)c * d;
    double s = 0.0;
    for (int r = j + threadIdx.x; r < d; r += blockDim.x) s += v[r] * col[r];
    double w = block_sum(s, red);
    for (int r = j + threadIdx.x; r < d; r += blockDim.x) col[r] -= 2.0 * v[r] * w;
}

// rows of Q: q_r <- q_r - 2 (q_r . v) v^T; one workgroup per row
__global__ __launch_bounds__(256) void qr_apply_q_kernel(double *__restrict__ q, int32_t d, int32_t j,
                                                         const double *__restrict__ v) {
    __shared__ double red[16];
    double *row = q + (int64_t)blockIdx.x * d;
    double s = 0.0;
    for (int i = j + threadIdx.x; i < d; i += blockDim.x) s += row[i] * v[i];
    double w = block_sum(s, red);
    for (int i = j + threadIdx.x; i < d; i += blockDim.x) row[i] -= 2.0 * w * v[i];
}

__global__ void qr_finish_kernel(const double *__restrict__ q, const double *__restrict__ acm,
                                 double *__restrict__ diag, int32_t d, float *__restrict__ rot) {
    int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (idx >= (int64_t)d * d) return;
    int32_t c = (int32_t)(idx % d);
    double dc = (c == d - 1) ? acm[(int64_t)(d - 1) * d + (d - 1)] : diag[c];
    double sgn = dc < 0.0 ? -1.0 : 1.0;
    // rot = Q diag(sign(diag(R)))
    rot[idx] = (float)(q[idx] * sgn);
}

}  // namespace

hipError_t launch_qr_rotation(const double *gauss, int32_t d, double *acm, double *q, double *v, double *diag,
                              float *rot, hipStream_t s) {
    int64_t dd = (int64_t)d * d;
    unsigned blocks = (unsigned)((dd + 255) / 256);
    qr_init_kernel<<<blocks, 256, 0, s>>>(gauss, d, acm, q);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    for (int32_t j = 0; j + 1 < d; ++j) {
        qr_house_kernel<<<1, 1024, 0, s>>>(acm, d, j, v, diag);
        qr_apply_a_kernel<<<(unsigned)(d - j - 1), 256, 0, s>>>(acm, d, j, v);
        qr_apply_q_kernel<<<(unsigned)d, 256, 0, s>>>(q, d, j, v);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    qr_finish_kernel<<<blocks, 256, 0, s>>>(q, acm, diag, d, rot);
    return hipGetLastError();
}

}  // namespace pdx
