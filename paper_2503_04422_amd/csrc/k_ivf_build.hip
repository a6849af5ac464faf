// IVF build kernels (Section 2.1, IVF): Lloyd k-means steps on the rotated
// rows, and bucketing of the rows into per-bucket PDX vectorgroups
// (Figure "IVF-PDX": every bucket is a PDX block).
//
// Bucket member order is the row order (a stable counting sort), so the
// layout is deterministic for a given assignment.
#include "pdx_internal.h"

namespace pdx {
namespace {

template <typename T>
__global__ void fill_kernel(T *__restrict__ p, int64_t count, T value) {
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (; i < count; i += stride) p[i] = value;
}

// centroids[l] = rows[init[l]]; flags an out-of-range seed row
__global__ void gather_rows_kernel(const float *__restrict__ x, int64_t n, int32_t d,
                                   const int64_t *__restrict__ rows, int32_t count, float *__restrict__ out,
                                   int32_t *__restrict__ flag) {
    int32_t l = blockIdx.x;
    int64_t r = rows[l];
    if (r < 0 || r >= n) {
        if (threadIdx.x == 0) atomicOr(flag, 2);
        return;
    }
    for (int j = threadIdx.x; j < d; j += blockDim.x) out[(int64_t)l * d + j] = x[r * d + j];
}

__global__ void labels_from_keys_kernel(const unsigned long long *__restrict__ best, int64_t n,
                                        int32_t *__restrict__ lab) {
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i < n) lab[i] = (int32_t)(best[i] & 0xffffffffu);
}

// float64 member sums and counts, one workgroup per row
__global__ __launch_bounds__(256) void kmeans_accumulate_kernel(const float *__restrict__ x, int64_t n,
                                                                int32_t d, const int32_t *__restrict__ lab,
                                                                double *__restrict__ sums,
                                                                int32_t *__restrict__ cnt) {
    int64_t i = blockIdx.x;
    int32_t l = lab[i];
    const float *row = x + i * d;
    double *dst = sums + (int64_t)l * d;
    for (int j = threadIdx.x; j < d; j += blockDim.x) atomicAdd(dst + j, (double)row[j]);
    if (threadIdx.x == 0) atomicAdd(cnt + l, 1);
}

// centroid = mean of members; an empty bucket keeps its previous centroid
__global__ void kmeans_finish_kernel(const double *__restrict__ sums, const int32_t *__restrict__ cnt,
                                     int32_t nlist, int32_t d, float *__restrict__ cen) {
    int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (idx >= (int64_t)nlist * d) return;
    int32_t l = (int32_t)(idx / d);
    if (cnt[l] > 0) cen[idx] = (float)(sums[idx] / (double)cnt[l]);
}

__global__ void check_labels_kernel(const int32_t *__restrict__ lab, int64_t n, int32_t nlist,
                                    int32_t *__restrict__ flag) {
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i < n && (lab[i] < 0 || lab[i] >= nlist)) atomicOr(flag, 4);
}

// ---- stable counting sort of rows by bucket ----
constexpr int kRowsPerBlock = 1024;

// per row block: members per bucket (LDS histogram)
__global__ __launch_bounds__(1024) void block_hist_kernel(const int32_t *__restrict__ lab, int64_t n,
                                                          int32_t nlist, int32_t *__restrict__ blk_cnt) {
    extern __shared__ int32_t h[];
    for (int l = threadIdx.x; l < nlist; l += blockDim.x) h[l] = 0;
    __syncthreads();
    int64_t i = (int64_t)blockIdx.x * kRowsPerBlock + threadIdx.x;
    if (i < n) atomicAdd(&h[lab[i]], 1);
    __syncthreads();
    int32_t *out = blk_cnt + (int64_t)blockIdx.x * nlist;
    for (int l = threadIdx.x; l < nlist; l += blockDim.x) out[l] = h[l];
}

// per bucket: exclusive prefix over row blocks; bucket sizes
__global__ void block_prefix_kernel(int32_t *__restrict__ blk_cnt, int32_t nblocks, int32_t nlist,
                                    int32_t *__restrict__ size) {
    int32_t l = blockIdx.x * blockDim.x + threadIdx.x;
    if (l >= nlist) return;
    int32_t run = 0;
    for (int32_t b = 0; b < nblocks; ++b) {
        int64_t at = (int64_t)b * nlist + l;
        int32_t c = blk_cnt[at];
        blk_cnt[at] = run;
        run += c;
    }
    size[l] = run;
}

// first vectorgroup of each bucket (buckets padded to whole groups); one
// workgroup, sequential chunks of 1024 buckets
__global__ __launch_bounds__(1024) void group_offsets_kernel(const int32_t *__restrict__ size, int32_t nlist,
                                                             int32_t *__restrict__ goff,
                                                             int32_t *__restrict__ stats) {
    __shared__ int32_t s[1024];
    __shared__ int32_t carry;
    __shared__ int32_t maxsz;
    if (threadIdx.x == 0) {
        carry = 0;
        maxsz = 0;
    }
    __syncthreads();
    for (int32_t base = 0; base < nlist; base += 1024) {
        int32_t l = base + threadIdx.x;
        int32_t sz = l < nlist ? size[l] : 0;
        int32_t g = (sz + kGroup - 1) / kGroup;
        if (sz > 0) atomicMax(&maxsz, sz);
        s[threadIdx.x] = g;
        __syncthreads();
        for (int off = 1; off < 1024; off <<= 1) {  // inclusive scan
            int32_t t = threadIdx.x >= off ? s[threadIdx.x - off] : 0;
            __syncthreads();
            s[threadIdx.x] += t;
            __syncthreads();
        }
        if (l < nlist) goff[l] = carry + s[threadIdx.x] - g;
        __syncthreads();
        if (threadIdx.x == 1023) carry += s[1023];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        goff[nlist] = carry;
        stats[0] = carry;   // total vectorgroups
        stats[1] = maxsz;   // largest bucket
    }
}

// slot of every row: bucket's first slot + rank among the bucket's rows
// (earlier blocks first, then row order inside the block)
__global__ __launch_bounds__(1024) void place_rows_kernel(const int32_t *__restrict__ lab, int64_t n,
                                                          int32_t nlist, const int32_t *__restrict__ blk_off,
                                                          const int32_t *__restrict__ goff,
                                                          int32_t *__restrict__ slot_id) {
    __shared__ uint32_t key[kRowsPerBlock];
    const int t = threadIdx.x;
    const int64_t i = (int64_t)blockIdx.x * kRowsPerBlock + t;
    // key = bucket << 10 | position inside the block; padding sorts last
    key[t] = i < n ? ((uint32_t)lab[i] << 10) | (uint32_t)t : 0xffffffffu;
    __syncthreads();
    for (int k2 = 2; k2 <= kRowsPerBlock; k2 <<= 1)
        for (int j2 = k2 >> 1; j2 > 0; j2 >>= 1) {
            int ixj = t ^ j2;
            if (ixj > t) {
                uint32_t a = key[t], b = key[ixj];
                bool up = (t & k2) == 0;
                if ((a > b) == up) {
                    key[t] = b;
                    key[ixj] = a;
                }
            }
            __syncthreads();
        }
    uint32_t kk = key[t];
    if (kk == 0xffffffffu) return;
    uint32_t l = kk >> 10;
    // rank inside the block = distance to the first sorted entry of bucket l
    int lo = 0, hi = t;  // first index with key >= (l << 10)
    while (lo < hi) {
        int mid = (lo + hi) >> 1;
        if ((key[mid] >> 10) < l) lo = mid + 1;
        else hi = mid;
    }
    int32_t rank = blk_off[(int64_t)blockIdx.x * nlist + l] + (t - lo);
    int64_t row = (int64_t)blockIdx.x * kRowsPerBlock + (kk & 1023u);
    slot_id[(int64_t)goff[l] * kGroup + rank] = (int32_t)row;
}

// PDX vectorgroups of the buckets: group g gathers the rows of its 64
// slots (row tile of 64 dimensions through LDS), zero for padding slots
__global__ __launch_bounds__(256) void gather_pdx_kernel(const float *__restrict__ x, int32_t d,
                                                         const int32_t *__restrict__ slot_id,
                                                         const int32_t *__restrict__ stats,
                                                         float *__restrict__ pdx) {
    __shared__ float tile[64][65];
    const int64_t g = blockIdx.x;
    if (g >= stats[0]) return;
    const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
    const int32_t c0 = blockIdx.y * 64;
#pragma unroll 4
    for (int r = 0; r < 64; r += 4) {
        int32_t row = slot_id[g * 64 + r + ty];
        int32_t col = c0 + tx;
        tile[r + ty][tx] = (row >= 0 && col < d) ? x[(int64_t)row * d + col] : 0.0f;
    }
    __syncthreads();
#pragma unroll 4
    for (int c = 0; c < 64; c += 4) {
        int32_t col = c0 + c + ty;
        if (col < d) pdx[(g * d + col) * 64 + tx] = tile[tx][c + ty];
    }
}

}  // namespace

hipError_t launch_fill_i32(int32_t *p, int64_t count, int32_t v, hipStream_t s) {
    if (count <= 0) return hipSuccess;
    int64_t b = (count + 255) / 256;
    fill_kernel<int32_t><<<(unsigned)(b < 4096 ? b : 4096), 256, 0, s>>>(p, count, v);
    return hipGetLastError();
}
hipError_t launch_fill_u64(unsigned long long *p, int64_t count, unsigned long long v, hipStream_t s) {
    if (count <= 0) return hipSuccess;
    int64_t b = (count + 255) / 256;
    fill_kernel<unsigned long long><<<(unsigned)(b < 4096 ? b : 4096), 256, 0, s>>>(p, count, v);
    return hipGetLastError();
}
hipError_t launch_fill_f64(double *p, int64_t count, double v, hipStream_t s) {
    if (count <= 0) return hipSuccess;
    int64_t b = (count + 255) / 256;
    fill_kernel<double><<<(unsigned)(b < 4096 ? b : 4096), 256, 0, s>>>(p, count, v);
    return hipGetLastError();
}

hipError_t launch_gather_rows(const float *x, int64_t n, int32_t d, const int64_t *rows, int32_t count,
                              float *out, int32_t *flag, hipStream_t s) {
    gather_rows_kernel<<<(unsigned)count, 256, 0, s>>>(x, n, d, rows, count, out, flag);
    return hipGetLastError();
}

hipError_t launch_labels_from_keys(const unsigned long long *best, int64_t n, int32_t *lab, hipStream_t s) {
    labels_from_keys_kernel<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(best, n, lab);
    return hipGetLastError();
}

hipError_t launch_kmeans_update(const float *x, int64_t n, int32_t d, const int32_t *lab, int32_t nlist,
                                double *sums, int32_t *cnt, float *cen, hipStream_t s) {
    hipError_t e;
    if ((e = launch_fill_f64(sums, (int64_t)nlist * d, 0.0, s)) != hipSuccess) return e;
    if ((e = launch_fill_i32(cnt, nlist, 0, s)) != hipSuccess) return e;
    kmeans_accumulate_kernel<<<(unsigned)n, 256, 0, s>>>(x, n, d, lab, sums, cnt);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    int64_t tot = (int64_t)nlist * d;
    kmeans_finish_kernel<<<(unsigned)((tot + 255) / 256), 256, 0, s>>>(sums, cnt, nlist, d, cen);
    return hipGetLastError();
}

hipError_t launch_check_labels(const int32_t *lab, int64_t n, int32_t nlist, int32_t *flag, hipStream_t s) {
    check_labels_kernel<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(lab, n, nlist, flag);
    return hipGetLastError();
}

hipError_t launch_bucketize(const float *xrot, int64_t n, int32_t d, const int32_t *lab, int32_t nlist,
                            int32_t *blk_cnt, int32_t *size, int32_t *goff, int32_t *stats, int32_t *slot_id,
                            int64_t max_slots, float *pdx, int64_t max_groups, hipStream_t s) {
    int32_t nblocks = (int32_t)((n + kRowsPerBlock - 1) / kRowsPerBlock);
    hipError_t e;
    block_hist_kernel<<<(unsigned)nblocks, 1024, nlist * sizeof(int32_t), s>>>(lab, n, nlist, blk_cnt);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    block_prefix_kernel<<<(unsigned)((nlist + 255) / 256), 256, 0, s>>>(blk_cnt, nblocks, nlist, size);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    group_offsets_kernel<<<1, 1024, 0, s>>>(size, nlist, goff, stats);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if ((e = launch_fill_i32(slot_id, max_slots, -1, s)) != hipSuccess) return e;
    place_rows_kernel<<<(unsigned)nblocks, 1024, 0, s>>>(lab, n, nlist, blk_cnt, goff, slot_id);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    gather_pdx_kernel<<<dim3((unsigned)max_groups, (unsigned)((d + 63) / 64)), 256, 0, s>>>(xrot, d, slot_id,
                                                                                          stats, pdx);
    return hipGetLastError();
}

}  // namespace pdx

// ---------------------------------------------------------------------------
// Low-precision copies of the bucketed vectorgroups.
// ---------------------------------------------------------------------------
namespace pdx {
namespace {

// per-dimension max |x| (float bits of non-negative values order as unsigned)
__global__ __launch_bounds__(256) void col_absmax_kernel(const float *__restrict__ x, int64_t n, int32_t d,
                                                         int64_t rows_per, uint32_t *__restrict__ maxbits) {
    int32_t j = blockIdx.x * 256 + threadIdx.x;
    if (j >= d) return;
    int64_t r0 = (int64_t)blockIdx.y * rows_per, r1 = min(r0 + rows_per, n);
    float m = 0.0f;
    for (int64_t r = r0; r < r1; ++r) m = fmaxf(m, fabsf(x[r * d + j]));
    atomicMax(maxbits + j, __float_as_uint(m));
}

__global__ void fp8_scale_kernel(const uint32_t *__restrict__ maxbits, int32_t d, float *__restrict__ scale) {
    int32_t j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= d) return;
    float m = __uint_as_float(maxbits[j]);
    scale[j] = m == 0.0f ? 1.0f : m / 448.0f;
}

// as gather_pdx_kernel, writing codes: bfloat16 and/or e4m3(x / s_j)
__global__ __launch_bounds__(256) void gather_lowp_kernel(const float *__restrict__ x, int32_t d,
                                                          const int32_t *__restrict__ slot_id,
                                                          const int32_t *__restrict__ stats,
                                                          uint16_t *__restrict__ pdx16, uint8_t *__restrict__ pdx8,
                                                          const float *__restrict__ scale) {
    __shared__ float tile[64][65];
    const int64_t g = blockIdx.x;
    if (g >= stats[0]) return;
    const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
    const int32_t c0 = blockIdx.y * 64;
#pragma unroll 4
    for (int r = 0; r < 64; r += 4) {
        int32_t row = slot_id[g * 64 + r + ty];
        int32_t col = c0 + tx;
        tile[r + ty][tx] = (row >= 0 && col < d) ? x[(int64_t)row * d + col] : 0.0f;
    }
    __syncthreads();
#pragma unroll 4
    for (int c = 0; c < 64; c += 4) {
        int32_t col = c0 + c + ty;
        if (col >= d) continue;
        const float v = tile[tx][c + ty];
        const int64_t at = (g * d + col) * 64 + tx;
        if (pdx16) pdx16[at] = bf16_encode(v);
        if (pdx8) pdx8[at] = static_cast<uint8_t>(e4m3_encode(v / scale[col]));
    }
}

// The bucket of every stored vectorgroup (one thread per bucket).
__global__ void group_bucket_kernel(const int32_t *__restrict__ goff, int32_t nlist, int32_t *__restrict__ gb) {
    const int32_t b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= nlist) return;
    for (int32_t g = goff[b]; g < goff[b + 1]; ++g) gb[g] = b;
}

// Radius of every 32-vector tile (half a vectorgroup) around its bucket's
// centroid: the largest |x - c| (L2, or the L1 norm when L1) over the
// tile's rows, float64 sums, widened by 1e-6 and rounded up to float32 (0
// for a tile of padding only).  One wave per tile; lanes 0..31 are its
// vectors.
template <bool L1>
__global__ __launch_bounds__(256) void tile_radius_kernel(const float *__restrict__ pdx,
                                                          const int32_t *__restrict__ slot_id,
                                                          const int32_t *__restrict__ goff, int32_t nlist,
                                                          const int32_t *__restrict__ gb,
                                                          const float *__restrict__ cen, int32_t d, int64_t max_tiles,
                                                          float *__restrict__ rad) {
    const int64_t t = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (t >= max_tiles) return;
    const int32_t g = (int32_t)(t >> 1);
    if (g >= goff[nlist]) return;
    const int32_t b = gb[g];
    const int v = (int)(t & 1) * 32 + (lane & 31);
    double acc = 0.0;
    if (lane < 32 && slot_id[(int64_t)g * kGroup + v] >= 0) {
        const float *xp = pdx + (int64_t)g * d * kGroup + v;
        const float *cp = cen + (int64_t)b * d;
        for (int32_t j = 0; j < d; ++j) {
            const double e = (double)xp[(int64_t)j * kGroup] - (double)cp[j];
            acc = L1 ? acc + fabs(e) : fma(e, e, acc);
        }
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) acc = fmax(acc, __shfl_xor(acc, off));
    if (lane == 0) rad[t] = __double2float_ru((L1 ? acc : sqrt(acc)) * (1.0 + 1e-6));
}

}  // namespace

hipError_t launch_tile_radii(const float *pdx, const int32_t *slot_id, const int32_t *goff, int32_t nlist,
                             const float *cen, int32_t d, int64_t max_groups, int32_t *gb, float *rad,
                             float *rad1, hipStream_t s) {
    group_bucket_kernel<<<(unsigned)((nlist + 255) / 256), 256, 0, s>>>(goff, nlist, gb);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const int64_t tiles = 2 * max_groups;
    tile_radius_kernel<false><<<(unsigned)((tiles + 3) / 4), 256, 0, s>>>(pdx, slot_id, goff, nlist, gb, cen, d,
                                                                          tiles, rad);
    tile_radius_kernel<true><<<(unsigned)((tiles + 3) / 4), 256, 0, s>>>(pdx, slot_id, goff, nlist, gb, cen, d,
                                                                         tiles, rad1);
    return hipGetLastError();
}

hipError_t launch_lowp_store(const float *xrow, int64_t n, int32_t d, const int32_t *slot_id, const int32_t *stats,
                             int64_t max_groups, uint16_t *pdx16, uint8_t *pdx8, float *scale, uint32_t *maxbits,
                             hipStream_t s) {
    hipError_t e;
    if (pdx8) {
        if ((e = launch_fill_i32(reinterpret_cast<int32_t *>(maxbits), d, 0, s)) != hipSuccess) return e;
        int64_t chunks = 256, rows_per = (n + chunks - 1) / chunks;
        chunks = (n + rows_per - 1) / rows_per;
        col_absmax_kernel<<<dim3((unsigned)((d + 255) / 256), (unsigned)chunks), 256, 0, s>>>(xrow, n, d, rows_per,
                                                                                           maxbits);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        fp8_scale_kernel<<<(unsigned)((d + 255) / 256), 256, 0, s>>>(maxbits, d, scale);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    gather_lowp_kernel<<<dim3((unsigned)max_groups, (unsigned)((d + 63) / 64)), 256, 0, s>>>(xrow, d, slot_id, stats,
                                                                                           pdx16, pdx8, scale);
    return hipGetLastError();
}

// One wave per (vectorgroup, 32-dimension sub-chunk), lane = vector: the
// sum of squares of the decoded values, dimensions in order.
__global__ __launch_bounds__(64) void lowp_norms_kernel(const uint16_t *__restrict__ pdx16,
                                                        const uint8_t *__restrict__ pdx8,
                                                        const float *__restrict__ scale, int32_t d,
                                                        const int32_t *__restrict__ stats, float *__restrict__ xn16,
                                                        float *__restrict__ xn8) {
    const int64_t g = blockIdx.x;
    const int32_t sb = blockIdx.y, nsub = gridDim.y;
    const int lane = threadIdx.x;
    const int64_t at = (g * nsub + sb) * 64 + lane;
    if (g >= stats[0]) return;
    float a16 = 0.0f, a8 = 0.0f;
    for (int32_t j = 32 * sb; j < min(32 * sb + 32, d); ++j) {
        const int64_t e = (g * d + j) * 64 + lane;
        if (pdx16) {
            const float v = bf16_decode(pdx16[e]);
            a16 = fmaf(v, v, a16);
        }
        if (pdx8) {
            const float v = e4m3_decode(pdx8[e]) * scale[j];
            a8 = fmaf(v, v, a8);
        }
    }
    if (xn16) xn16[at] = a16;
    if (xn8) xn8[at] = a8;
}

hipError_t launch_lowp_norms(const uint16_t *pdx16, const uint8_t *pdx8, const float *scale, int32_t d,
                             const int32_t *stats, int64_t max_groups, float *xn16, float *xn8, hipStream_t s) {
    if (max_groups <= 0 || (!xn16 && !xn8)) return hipSuccess;
    const unsigned nsub = (unsigned)((d + 31) / 32);
    lowp_norms_kernel<<<dim3((unsigned)max_groups, nsub), 64, 0, s>>>(pdx16, pdx8, scale, d, stats, xn16, xn8);
    return hipGetLastError();
}

}  // namespace pdx
