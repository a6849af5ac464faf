// Distance kernels with no search (Section 3's kernel listing; the kernel
// study of Section 6.4, Tables "kernels" and "block"): the L2, L1 or
// inner-product score of every vector of a collection for each query,
// over the PDX layout with blocks of G vectors, or over the row-major
// (N-ary) layout with one vector per lane.
//
// Both layouts sum a vector's terms in the same order, so they return the
// same bits: chunks of 32 dimensions, sequential inside a chunk; the chunks
// split into S consecutive segments (S depends only on n and D); a
// segment's chunk sums added in order; the segment sums added in order.
// The float32 error stays about (32 + D/32) 2^-24 of the sum of |terms|.
//
// A workgroup holds 64 vectors and S waves, wave s summing segment s (so
// small collections still fill the chip); the segment sums meet in LDS.
// PDX blocks: dimension j of the block's v-th vector at offset j G + v.
// The 64 vectors are 64/G blocks when G < 64 (lane = block-local vector),
// or one block with G/64 vectors per lane when G > 64; every dimension row
// is read as G contiguous floats.  The row-major kernel gives each lane
// one row.  The query value of a dimension is the same for all lanes.
#include "pdx_internal.h"

namespace pdx {
namespace {

constexpr int kDistChunk = 32;

template <int M>
__device__ __forceinline__ float dterm(float acc, float qv, float xv) {
    if (M == PDX_METRIC_L2) {
        const float t = qv - xv;
        return fmaf(t, t, acc);
    }
    if (M == PDX_METRIC_L1) return acc + fabsf(qv - xv);
    return fmaf(qv, xv, acc);
}

// reported score: the sum, or -sum for the inner product (zero as +0)
template <int M>
__device__ __forceinline__ float dfinish(float s) {
    return M == PDX_METRIC_IP ? -s + 0.0f : s;
}

template <int G, int M>
__global__ __launch_bounds__(1024) void pdx_dist_kernel(const float *__restrict__ data, int64_t n, int32_t d,
                                                        const float *__restrict__ q, float *__restrict__ out) {
    constexpr int R = G >= 64 ? G / 64 : 1;      // vectors per lane
    constexpr int BPW = G >= 64 ? 1 : 64 / G;    // blocks per wave
    __shared__ float part[16][R][64];
    const int lane = threadIdx.x & 63, seg = threadIdx.x >> 6, S = blockDim.x >> 6;
    const int64_t blk = (int64_t)blockIdx.x * BPW + (G >= 64 ? 0 : lane / G);
    const int v0 = G >= 64 ? lane : lane % G;
    const bool live = blk * G < n;  // some vector of this lane's block exists
    const int32_t nch = (d + kDistChunk - 1) / kDistChunk;
    const int32_t c0 = (int32_t)((int64_t)nch * seg / S), c1 = (int32_t)((int64_t)nch * (seg + 1) / S);
    const float *qrow = q + (int64_t)blockIdx.y * d;
    const float *base = data + blk * (int64_t)d * G + v0;
    float total[R];
#pragma unroll
    for (int r = 0; r < R; ++r) total[r] = 0.0f;
    for (int32_t c = live ? c0 : c1; c < c1; ++c) {
        const int32_t j0 = c * kDistChunk, j1 = min(j0 + kDistChunk, d);
        float acc[R];
#pragma unroll
        for (int r = 0; r < R; ++r) acc[r] = 0.0f;
#pragma unroll 8
        for (int32_t j = j0; j < j1; ++j) {
            const float qv = qrow[j];
            const float *row = base + (int64_t)j * G;
#pragma unroll
            for (int r = 0; r < R; ++r) acc[r] = dterm<M>(acc[r], qv, row[64 * r]);
        }
#pragma unroll
        for (int r = 0; r < R; ++r) total[r] += acc[r];
    }
    if (S > 1) {
#pragma unroll
        for (int r = 0; r < R; ++r) part[seg][r][lane] = total[r];
        __syncthreads();
        if (seg != 0) return;
#pragma unroll
        for (int r = 0; r < R; ++r) {
            total[r] = part[0][r][lane];
            for (int t = 1; t < S; ++t) total[r] += part[t][r][lane];
        }
    }
    if (!live) return;
    float *orow = out + (int64_t)blockIdx.y * n;
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int64_t vec = blk * G + v0 + 64 * r;
        if (vec < n) orow[vec] = dfinish<M>(total[r]);
    }
}

// Row-major layout, one vector per lane: the lane walks its own row
// (16-byte loads when D % 4 == 0).
template <int M>
__global__ __launch_bounds__(1024) void nary_dist_kernel(const float *__restrict__ data, int64_t n, int32_t d,
                                                         const float *__restrict__ q, float *__restrict__ out) {
    __shared__ float part[16][64];
    const int lane = threadIdx.x & 63, seg = threadIdx.x >> 6, S = blockDim.x >> 6;
    const int64_t i = (int64_t)blockIdx.x * 64 + lane;
    const bool live = i < n;
    const int32_t nch = (d + kDistChunk - 1) / kDistChunk;
    const int32_t c0 = (int32_t)((int64_t)nch * seg / S), c1 = (int32_t)((int64_t)nch * (seg + 1) / S);
    const float *qrow = q + (int64_t)blockIdx.y * d;
    const float *row = data + i * d;
    const bool vec4 = (d & 3) == 0;
    float total = 0.0f;
    for (int32_t c = live ? c0 : c1; c < c1; ++c) {
        const int32_t j0 = c * kDistChunk, j1 = min(j0 + kDistChunk, d);
        float acc = 0.0f;
        if (vec4) {
#pragma unroll 4
            for (int32_t j = j0; j < j1; j += 4) {
                const float4 x = *reinterpret_cast<const float4 *>(row + j);
                acc = dterm<M>(acc, qrow[j], x.x);
                acc = dterm<M>(acc, qrow[j + 1], x.y);
                acc = dterm<M>(acc, qrow[j + 2], x.z);
                acc = dterm<M>(acc, qrow[j + 3], x.w);
            }
        } else {
            for (int32_t j = j0; j < j1; ++j) acc = dterm<M>(acc, qrow[j], row[j]);
        }
        total += acc;
    }
    if (S > 1) {
        part[seg][lane] = total;
        __syncthreads();
        if (seg != 0) return;
        total = part[0][lane];
        for (int t = 1; t < S; ++t) total += part[t][lane];
    }
    if (live) out[(int64_t)blockIdx.y * n + i] = dfinish<M>(total);
}

// Rows -> PDX blocks of G vectors through a 64 x 64 LDS tile: reads
// coalesced along dimensions, writes coalesced along vectors; rows past n
// (the last block's padding) are written as zeros.
__global__ __launch_bounds__(256) void layout_blocks_kernel(const float *__restrict__ x, int64_t n, int32_t d,
                                                            int32_t G, int64_t npad, float *__restrict__ out) {
    __shared__ float t[64][65];
    const int64_t i0 = (int64_t)blockIdx.x * 64;
    const int32_t j0 = (int32_t)blockIdx.y * 64;
    const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
    for (int r = ty; r < 64; r += 4) {
        const int64_t i = i0 + r;
        const int32_t j = j0 + tx;
        t[r][tx] = (i < n && j < d) ? x[i * d + j] : 0.0f;
    }
    __syncthreads();
    for (int c = ty; c < 64; c += 4) {
        const int32_t j = j0 + c;
        const int64_t i = i0 + tx;
        if (j < d && i < npad) {
            const int64_t b = i / G;
            out[(b * d + j) * G + (i - b * G)] = t[tx][c];
        }
    }
}

bool block_ok(int32_t b) { return b == 16 || b == 32 || b == 64 || b == 128 || b == 256 || b == 512; }

// Segments per 64 vectors: enough waves for about 8 per SIMD over the
// collection, at most 16 (one workgroup) and at most one per chunk.  A
// function of n and D only, so both layouts sum in the same order.
int32_t dist_segments(int64_t n, int32_t d) {
    const int64_t groups = (n + 63) / 64;
    const int64_t want = 8 * 4 * (int64_t)device_cus();
    int64_t S = (want + groups - 1) / groups;
    const int64_t nch = (d + kDistChunk - 1) / kDistChunk;
    if (S > 16) S = 16;
    if (S > nch) S = nch;
    return (int32_t)(S < 1 ? 1 : S);
}

template <int M>
hipError_t launch_pdx_dist(const float *data, int32_t G, int64_t n, int32_t d, const float *q, int64_t nq, float *out,
                           hipStream_t s) {
    const int32_t S = dist_segments(n, d);
    const int64_t nblk = (n + G - 1) / G;
    const int64_t bpw = G >= 64 ? 1 : 64 / G;
    const dim3 grid((unsigned)((nblk + bpw - 1) / bpw), (unsigned)nq);
    const dim3 block(64u * (unsigned)S);
    switch (G) {
        case 16: pdx_dist_kernel<16, M><<<grid, block, 0, s>>>(data, n, d, q, out); break;
        case 32: pdx_dist_kernel<32, M><<<grid, block, 0, s>>>(data, n, d, q, out); break;
        case 64: pdx_dist_kernel<64, M><<<grid, block, 0, s>>>(data, n, d, q, out); break;
        case 128: pdx_dist_kernel<128, M><<<grid, block, 0, s>>>(data, n, d, q, out); break;
        case 256: pdx_dist_kernel<256, M><<<grid, block, 0, s>>>(data, n, d, q, out); break;
        default: pdx_dist_kernel<512, M><<<grid, block, 0, s>>>(data, n, d, q, out); break;
    }
    return hipGetLastError();
}

template <int M>
hipError_t launch_nary_dist(const float *data, int64_t n, int32_t d, const float *q, int64_t nq, float *out,
                            hipStream_t s) {
    const int32_t S = dist_segments(n, d);
    const dim3 grid((unsigned)((n + 63) / 64), (unsigned)nq);
    nary_dist_kernel<M><<<grid, dim3(64u * (unsigned)S), 0, s>>>(data, n, d, q, out);
    return hipGetLastError();
}

constexpr int64_t kMaxDistQueries = 65535;  // grid.y

}  // namespace
}  // namespace pdx

using namespace pdx;

extern "C" {

size_t pdx_layout_blocks_bytes(int64_t n, int32_t d, int32_t block) {
    if (n < 1 || d < 1 || !block_ok(block)) return 0;
    return (size_t)((n + block - 1) / block) * (size_t)block * (size_t)d * sizeof(float);
}

pdx_status pdx_layout_blocks(const float *x, int64_t n, int32_t d, int32_t block, float *out, void *stream) {
    if (n < 1 || d < 1) {
        set_error("pdx_layout_blocks: n and d must be >= 1");
        return PDX_EINVAL;
    }
    if (!block_ok(block)) {
        set_error("pdx_layout_blocks: block must be 16, 32, 64, 128, 256 or 512 (got %d)", block);
        return PDX_EINVAL;
    }
    if (!x || !out) {
        set_error("pdx_layout_blocks: null pointer");
        return PDX_EINVAL;
    }
    const int64_t npad = (n + block - 1) / block * block;
    if ((npad + 63) / 64 > 0x7fffffff || (d + 63) / 64 > 65535) {
        set_error("pdx_layout_blocks: collection too large for one launch");
        return PDX_EINVAL;
    }
    hipStream_t s = static_cast<hipStream_t>(stream);
    layout_blocks_kernel<<<dim3((unsigned)((npad + 63) / 64), (unsigned)((d + 63) / 64)), 256, 0, s>>>(
        x, n, d, block, npad, out);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) {
        set_error("pdx_layout_blocks: %s", hipGetErrorString(e));
        return PDX_EHIP;
    }
    return PDX_OK;
}

pdx_status pdx_distances(const float *data, int32_t layout, int32_t block, int64_t n, int32_t d, const float *q,
                         int64_t nq, int32_t metric, float *out, void *stream) {
    if (n < 1 || d < 1 || nq < 0 || nq > kMaxDistQueries) {
        set_error("pdx_distances: need n >= 1, d >= 1 and 0 <= nq <= %lld", (long long)kMaxDistQueries);
        return PDX_EINVAL;
    }
    if (layout != PDX_LAYOUT_NARY && layout != PDX_LAYOUT_PDX) {
        set_error("pdx_distances: unknown layout %d", layout);
        return PDX_EINVAL;
    }
    if (layout == PDX_LAYOUT_PDX && !block_ok(block)) {
        set_error("pdx_distances: block must be 16, 32, 64, 128, 256 or 512 (got %d)", block);
        return PDX_EINVAL;
    }
    if (metric != PDX_METRIC_L2 && metric != PDX_METRIC_L1 && metric != PDX_METRIC_IP) {
        set_error("pdx_distances: unknown metric %d", metric);
        return PDX_EINVAL;
    }
    if (nq == 0) return PDX_OK;
    if (!data || !q || !out) {
        set_error("pdx_distances: null pointer");
        return PDX_EINVAL;
    }
    if (layout == PDX_LAYOUT_NARY && (d & 3) == 0 && (reinterpret_cast<uintptr_t>(data) & 15u) != 0) {
        set_error("pdx_distances: row-major data must be 16-byte aligned");
        return PDX_EINVAL;
    }
    if ((n + 63) / 64 > 0x7fffffff) {  // grid.x of either kernel is at most this
        set_error("pdx_distances: collection too large for one launch");
        return PDX_EINVAL;
    }
    hipStream_t s = static_cast<hipStream_t>(stream);
    hipError_t e;
    if (layout == PDX_LAYOUT_PDX) {
        e = metric == PDX_METRIC_L2   ? launch_pdx_dist<PDX_METRIC_L2>(data, block, n, d, q, nq, out, s)
            : metric == PDX_METRIC_L1 ? launch_pdx_dist<PDX_METRIC_L1>(data, block, n, d, q, nq, out, s)
                                      : launch_pdx_dist<PDX_METRIC_IP>(data, block, n, d, q, nq, out, s);
    } else {
        e = metric == PDX_METRIC_L2   ? launch_nary_dist<PDX_METRIC_L2>(data, n, d, q, nq, out, s)
            : metric == PDX_METRIC_L1 ? launch_nary_dist<PDX_METRIC_L1>(data, n, d, q, nq, out, s)
                                      : launch_nary_dist<PDX_METRIC_IP>(data, n, d, q, nq, out, s);
    }
    if (e != hipSuccess) {
        set_error("pdx_distances: %s", hipGetErrorString(e));
        return PDX_EHIP;
    }
    return PDX_OK;
}

}  // extern "C"
