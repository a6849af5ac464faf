// PCA rotation for the IVF index: BSA's projection (Section 2.3: a PCA of
// the collection in place of ADSampling's random orthogonal projection).
//
// The rows of the rotation R are the principal directions of the rows x,
// largest variance first, so x -> R x puts the most variance in the first
// coordinates.  Steps:
//  1. covariance C = (1/n) sum_x (x - mu)(x - mu)^T in float32: upper
//     64 x 64 tiles, each accumulated over `splits` row ranges by one
//     workgroup (centred as they are staged), the ranges then summed in a
//     fixed order and the tiles mirrored, so C is exactly symmetric and the
//     result does not depend on scheduling;
//  2. cyclic Jacobi sweeps on H = R C R^T from R = I, in float32: every
//     sweep visits each pair (p, q) once, in d - 1 rounds of disjoint pairs
//     (round-robin order); a round computes each pair's rotation from
//     H_pp, H_qq, H_pq (the symmetric 2 x 2 Schur step: tau =
//     (H_qq - H_pp) / (2 H_pq), t = sign(tau) / (|tau| + sqrt(1 + tau^2)),
//     c = 1 / sqrt(1 + t^2), s = t c) and applies all of them at once,
//     H <- J^T H J and R <- J^T R, elementwise from the previous H and R;
//     off-diagonal mass falls quadratically once it is small;
//  3. R re-orthonormalised by the float64 Householder QR of R^T (with its
//     sign fix), which removes the float32 drift of the rotations;
//  4. the rows ordered by their Rayleigh quotient r_i^T C r_i, largest first
//     (ties by row).
// Any orthogonal R preserves distances, so the searches stay as exact (or
// as approximate) as with the random rotation; the PCA only changes which
// coordinates come first.
#include "pdx_internal.h"

namespace pdx {
namespace {

constexpr int kCT = 64;  // covariance tile width

__global__ void eye_kernel(float *__restrict__ r, int32_t d) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i < (int64_t)d * d) r[i] = (i / d == i % d) ? 1.0f : 0.0f;
}

// tile pair p (row tile <= column tile) of nt tiles
__device__ __forceinline__ void tile_pair(int32_t p, int32_t nt, int32_t &ti, int32_t &tj) {
    ti = 0;
    while (p >= nt - ti) {
        p -= nt - ti;
        ++ti;
    }
    tj = ti + p;
}

// Partial sums of (x - mu)(x - mu)^T for rows [r0, r1) of split blockIdx.y
// over the 64 x 64 tile pair blockIdx.x; 16 x 16 threads hold 4 x 4 sums.
__global__ __launch_bounds__(256) void cov_partial_kernel(const float *__restrict__ x, int64_t n, int32_t d,
                                                          const float *__restrict__ mu, int32_t nt, int32_t splits,
                                                          float *__restrict__ part) {
    __shared__ float A[16][kCT + 1], B[16][kCT + 1];
    int32_t ti, tj;
    tile_pair(blockIdx.x, nt, ti, tj);
    const int32_t i0 = ti * kCT, j0 = tj * kCT;
    const int64_t r0 = n * blockIdx.y / splits, r1 = n * (blockIdx.y + 1) / splits;
    const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
    float acc[4][4] = {};
    for (int64_t rb = r0; rb < r1; rb += 16) {
        for (int e = threadIdx.x; e < 16 * kCT; e += 256) {
            const int rr = e / kCT, cc = e % kCT;
            const int64_t r = rb + rr;
            const int32_t ci = i0 + cc, cj = j0 + cc;
            A[rr][cc] = (r < r1 && ci < d) ? x[r * d + ci] - mu[ci] : 0.0f;
            B[rr][cc] = (r < r1 && cj < d) ? x[r * d + cj] - mu[cj] : 0.0f;
        }
        __syncthreads();
#pragma unroll 4
        for (int rr = 0; rr < 16; ++rr) {
            float a[4], b[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                a[u] = A[rr][4 * ty + u];
                b[u] = B[rr][4 * tx + u];
            }
#pragma unroll
            for (int u = 0; u < 4; ++u)
#pragma unroll
                for (int w = 0; w < 4; ++w) acc[u][w] = fmaf(a[u], b[w], acc[u][w]);
        }
        __syncthreads();
    }
    float *out = part + ((size_t)blockIdx.y * gridDim.x + blockIdx.x) * kCT * kCT;
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int w = 0; w < 4; ++w) out[(4 * ty + u) * kCT + 4 * tx + w] = acc[u][w];
}

// C[i][j] = sum over splits (in order) of the tile pair holding (i, j) / n;
// the lower triangle reads the mirrored upper tile.
__global__ void cov_reduce_kernel(const float *__restrict__ part, int32_t d, int32_t nt, int32_t npairs,
                                  int32_t splits, float inv_n, float *__restrict__ cov) {
    const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (e >= (int64_t)d * d) return;
    int32_t i = (int32_t)(e / d), j = (int32_t)(e % d);
    if (i / kCT > j / kCT) {  // lower tile: the mirrored entry of the upper one
        const int32_t t = i;
        i = j;
        j = t;
    }
    const int32_t ti = i / kCT, tj = j / kCT;
    const int32_t p = ti * nt - ti * (ti - 1) / 2 + (tj - ti);  // pairs before row tile ti, then the offset
    const int32_t li = i - ti * kCT, lj = j - tj * kCT;
    float s = 0.0f;
    for (int32_t sp = 0; sp < splits; ++sp) s += part[((size_t)sp * npairs + p) * kCT * kCT + li * kCT + lj];
    cov[e] = s * inv_n;
}

__global__ void to_f64_kernel(const float *__restrict__ a, int64_t count, double *__restrict__ b) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i < count) b[i] = (double)a[i];
}

// b = a^T for [d][d], 32 x 32 blocks through LDS
__global__ __launch_bounds__(256) void transpose_kernel(const float *__restrict__ a, int32_t d, float *__restrict__ b) {
    __shared__ float blk[32][33];
    const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
    const int32_t r0 = blockIdx.y * 32, c0 = blockIdx.x * 32;
    for (int r = ty; r < 32; r += 8)
        if (r0 + r < d && c0 + tx < d) blk[r][tx] = a[(int64_t)(r0 + r) * d + c0 + tx];
    __syncthreads();
    for (int r = ty; r < 32; r += 8)
        if (c0 + r < d && r0 + tx < d) b[(int64_t)(c0 + r) * d + r0 + tx] = blk[tx][r];
}

// rho_i = r_i . (C r_i) = sum_j R[i][j] W[j][i] with W = C R^T; one wave per i
__global__ __launch_bounds__(64) void rayleigh_kernel(const float *__restrict__ r, const float *__restrict__ w,
                                                      int32_t d, float *__restrict__ rho) {
    const int32_t i = blockIdx.x;
    float s = 0.0f;
    for (int32_t j = threadIdx.x; j < d; j += kWave) s = fmaf(r[(int64_t)i * d + j], w[(int64_t)j * d + i], s);
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off);
    if (threadIdx.x == 0) rho[i] = s;
}

// perm = rows by rho descending (clamped at 0), ties by row; one workgroup,
// bitonic sort of (~bits(rho) << 32 | i) in LDS (pow2 >= d keys)
__global__ __launch_bounds__(256) void order_desc_kernel(const float *__restrict__ rho, int32_t d, int32_t pow2,
                                                         int32_t *__restrict__ perm) {
    extern __shared__ uint64_t keys[];
    for (int j = threadIdx.x; j < pow2; j += blockDim.x) {
        uint64_t key = kEmptyKey;
        if (j < d) key = (static_cast<uint64_t>(~__float_as_uint(fmaxf(rho[j], 0.0f))) << 32) | (uint32_t)j;
        keys[j] = key;
    }
    __syncthreads();
    for (int k2 = 2; k2 <= pow2; k2 <<= 1) {
        for (int j2 = k2 >> 1; j2 > 0; j2 >>= 1) {
            for (int i = threadIdx.x; i < pow2; i += blockDim.x) {
                const int ixj = i ^ j2;
                if (ixj > i) {
                    const uint64_t a = keys[i], b = keys[ixj];
                    const bool up = (i & k2) == 0;
                    if ((a > b) == up) {
                        keys[i] = b;
                        keys[ixj] = a;
                    }
                }
            }
            __syncthreads();
        }
    }
    for (int j = threadIdx.x; j < d; j += blockDim.x) perm[j] = (int32_t)(keys[j] & 0xffffffffu);
}

__global__ void permute_rows_kernel(const float *__restrict__ a, const int32_t *__restrict__ perm, int32_t d,
                                    float *__restrict__ b) {
    const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (e >= (int64_t)d * d) return;
    const int32_t i = (int32_t)(e / d), j = (int32_t)(e % d);
    b[e] = a[(int64_t)perm[i] * d + j];
}

// Round r of a sweep over m (even) indices, the last one fixed: pairs
// (m - 1, r) and ((r + i) mod (m - 1), (r - i) mod (m - 1)), i = 1 .. m/2 - 1.
// Indices >= d are padding (d odd).  Per index: its partner, and the two
// entries of column i of the round's rotation J: J[i][i] = ws, J[i'][i] = wo.
__global__ void jacobi_angles_kernel(const float *__restrict__ h, int32_t d, int32_t m, int32_t r,
                                     int32_t *__restrict__ partner, float *__restrict__ ws,
                                     float *__restrict__ wo) {
    const int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= m / 2) return;
    int32_t a, b;
    if (i == 0) {
        a = m - 1;
        b = r;
    } else {
        a = (r + i) % (m - 1);
        b = (r - i + m - 1) % (m - 1);
    }
    const int32_t p = min(a, b), q = max(a, b);
    float c = 1.0f, sn = 0.0f;
    if (q < d) {
        const float hpq = h[(int64_t)p * d + q];
        if (hpq != 0.0f) {
            const float tau = (h[(int64_t)q * d + q] - h[(int64_t)p * d + p]) / (2.0f * hpq);
            const float t = copysignf(1.0f, tau) / (fabsf(tau) + sqrtf(1.0f + tau * tau));
            c = 1.0f / sqrtf(1.0f + t * t);
            sn = t * c;
        }
    }
    if (p < d) {
        partner[p] = q < d ? q : p;
        ws[p] = c;
        wo[p] = -sn;
    }
    if (q < d) {
        partner[q] = p;
        ws[q] = c;
        wo[q] = sn;
    }
}

// H1 = J^T H0 J and R1 = J^T R0 from the round's rotation (disjoint pairs):
// H1[i][j] = ws_i (ws_j H0[i][j] + wo_j H0[i][j']) + wo_i (ws_j H0[i'][j] + wo_j H0[i'][j']),
// R1[i][k] = ws_i R0[i][k] + wo_i R0[i'][k].
__global__ void jacobi_rotate_kernel(const float *__restrict__ h0, const float *__restrict__ r0, int32_t d,
                                     const int32_t *__restrict__ partner, const float *__restrict__ ws,
                                     const float *__restrict__ wo, float *__restrict__ h1, float *__restrict__ r1) {
    const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (e >= (int64_t)d * d) return;
    const int32_t i = (int32_t)(e / d), j = (int32_t)(e % d);
    const int32_t ip = partner[i], jp = partner[j];
    const float si = ws[i], oi = wo[i], sj = ws[j], oj = wo[j];
    const float *hi = h0 + (int64_t)i * d, *hip = h0 + (int64_t)ip * d;
    h1[e] = si * (sj * hi[j] + oj * hi[jp]) + oi * (sj * hip[j] + oj * hip[jp]);
    r1[e] = si * r0[(int64_t)i * d + j] + oi * r0[(int64_t)ip * d + j];
}

// |x| over [c1, d) for every test point of every vector of group g (one
// wave per group, lane = vector), summed from the last dimension down
__global__ __launch_bounds__(64) void residual_norms_kernel(const float *__restrict__ pdx, int32_t d,
                                                            const int32_t *__restrict__ ngroups, int32_t dd,
                                                            int32_t ntp, float *__restrict__ xres) {
    const int64_t g = blockIdx.x;
    if (ngroups && g >= *ngroups) return;
    const int lane = threadIdx.x;
    const float *col = pdx + g * d * kGroup + lane;
    float s = 0.0f;
    for (int32_t c = ntp - 1; c >= 0; --c) {
        const int32_t c1 = (c + 1) * dd, hi = c == ntp - 1 ? d : (c + 2) * dd;
        for (int32_t j = hi - 1; j >= c1; --j) {
            const float v = col[(int64_t)j * kGroup];
            s = fmaf(v, v, s);
        }
        xres[(g * ntp + c) * kGroup + lane] = sqrtf(s);
    }
}

// the same for queries: one wave per query (a lane per test point)
__global__ __launch_bounds__(64) void query_residual_kernel(const float *__restrict__ q, int32_t d, int32_t dd,
                                                            int32_t ntp, float *__restrict__ qres) {
    const int64_t qi = blockIdx.x;
    const float *row = q + qi * d;
    for (int32_t c = threadIdx.x; c < ntp; c += kWave) {
        float s = 0.0f;
        for (int32_t j = d - 1; j >= (c + 1) * dd; --j) s = fmaf(row[j], row[j], s);
        qres[qi * ntp + c] = sqrtf(s);
    }
}

}  // namespace

int32_t res_test_points(int32_t d, int32_t dd) { return dd > 0 && dd < d ? (d + dd - 1) / dd - 1 : 0; }

hipError_t launch_residual_norms(const float *pdx, int32_t d, int64_t ngroups, const int32_t *ngroups_dev,
                                 int32_t dd, float *xres, hipStream_t s) {
    const int32_t ntp = res_test_points(d, dd);
    if (ntp == 0 || ngroups == 0) return hipSuccess;
    residual_norms_kernel<<<(unsigned)ngroups, 64, 0, s>>>(pdx, d, ngroups_dev, dd, ntp, xres);
    return hipGetLastError();
}

hipError_t launch_query_residuals(const float *q, int64_t nq, int32_t d, int32_t dd, float *qres, hipStream_t s) {
    const int32_t ntp = res_test_points(d, dd);
    if (ntp == 0 || nq == 0) return hipSuccess;
    query_residual_kernel<<<(unsigned)nq, 64, 0, s>>>(q, d, dd, ntp, qres);
    return hipGetLastError();
}

int32_t pca_splits(int64_t n) { return n >= (int64_t)1 << 20 ? 16 : (n >= 65536 ? 8 : 1); }
int32_t pca_tiles(int32_t d) { return (d + kCT - 1) / kCT; }
size_t pca_part_floats(int64_t n, int32_t d) {
    const int32_t nt = pca_tiles(d);
    return (size_t)pca_splits(n) * (nt * (nt + 1) / 2) * kCT * kCT;
}

hipError_t launch_pca_rotation(const float *x, int64_t n, int32_t d, int32_t sweeps, const float *mu, float *part,
                               float *cov, float *h, float *r2, double *w64, double *acm, double *qd, double *v,
                               double *diag, float *tmp, float *rho, int32_t *perm, float *cs, float *rot,
                               hipStream_t s) {
    const int64_t dd = (int64_t)d * d;
    const unsigned eb = (unsigned)((dd + 255) / 256);
    const int32_t nt = pca_tiles(d), npairs = nt * (nt + 1) / 2, splits = pca_splits(n);
    cov_partial_kernel<<<dim3((unsigned)npairs, (unsigned)splits), 256, 0, s>>>(x, n, d, mu, nt, splits, part);
    cov_reduce_kernel<<<eb, 256, 0, s>>>(part, d, nt, npairs, splits, (float)(1.0 / (double)n), cov);
    eye_kernel<<<eb, 256, 0, s>>>(rot, d);
    hipError_t e = hipMemcpyAsync(h, cov, sizeof(float) * dd, hipMemcpyDeviceToDevice, s);
    if (e != hipSuccess) return e;
    if ((e = hipGetLastError()) != hipSuccess) return e;
    // Jacobi sweeps: H and R ping-pong between (h, rot) and (tmp, r2)
    const int32_t m = d + (d & 1);
    int32_t *partner = reinterpret_cast<int32_t *>(cs);
    float *ws = cs + d, *wo = cs + 2 * d;
    float *hc = h, *rc = rot, *hn = tmp, *rn = r2;
    for (int32_t sw = 0; sw < sweeps && m > 1; ++sw) {
        for (int32_t r = 0; r < m - 1; ++r) {
            jacobi_angles_kernel<<<(unsigned)((m / 2 + 255) / 256), 256, 0, s>>>(hc, d, m, r, partner, ws, wo);
            jacobi_rotate_kernel<<<eb, 256, 0, s>>>(hc, rc, d, partner, ws, wo, hn, rn);
            if ((e = hipGetLastError()) != hipSuccess) return e;
            float *t = hc;
            hc = hn;
            hn = t;
            t = rc;
            rc = rn;
            rn = t;
        }
    }
    // re-orthonormalise: QR of R^T (columns = the basis vectors), R = Q^T
    const dim3 tg((unsigned)((d + 31) / 32), (unsigned)((d + 31) / 32));
    transpose_kernel<<<tg, 256, 0, s>>>(rc, d, rn);
    to_f64_kernel<<<eb, 256, 0, s>>>(rn, dd, w64);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if ((e = launch_qr_rotation(w64, d, acm, qd, v, diag, rn, s)) != hipSuccess) return e;
    transpose_kernel<<<tg, 256, 0, s>>>(rn, d, rc);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    // Rayleigh quotients with the covariance, rows by them
    if ((e = launch_gemm_abt(cov, d, rc, d, d, rn, d, s)) != hipSuccess) return e;  // C R^T
    rayleigh_kernel<<<(unsigned)d, 64, 0, s>>>(rc, rn, d, rho);
    int32_t pow2 = 1;
    while (pow2 < d) pow2 <<= 1;
    order_desc_kernel<<<1, 256, pow2 * sizeof(uint64_t), s>>>(rho, d, pow2, perm);
    permute_rows_kernel<<<eb, 256, 0, s>>>(rc, perm, d, rn);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    return rn == rot ? hipSuccess : hipMemcpyAsync(rot, rn, sizeof(float) * dd, hipMemcpyDeviceToDevice, s);
}

}  // namespace pdx
