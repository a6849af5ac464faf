// Internal declarations shared by the libpdx translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

#include "pdx.h"

namespace pdx {

constexpr int kGroup = 64;          // vectors per vectorgroup == wave width
constexpr int kWave = 64;
constexpr uint32_t kInfBits = 0x7f800000u;  // +inf as float bits
constexpr uint64_t kEmptyKey = ~0ull;       // empty top-k slot

enum IndexKind { kFlat = 1, kIvf = 2 };

}  // namespace pdx

struct pdx_index {
    int kind;
    int64_t n;
    int32_t d;
    int32_t group;
    int32_t ngroups;     // vectorgroups stored
    int32_t start_rows;  // flat: START block, rounded up to whole groups
    float *pdx;          // [ngroups][d][64] float32
    float *means;        // [d] float32 (flat)
    // IVF
    int32_t nlist;
    int32_t dtype_mask;  // bit i set: PDX_DTYPE i stored
    float *rot;          // [d][d] rotation (row j = j-th output coordinate)
    float *centroids;    // [nlist][d] rotated space
    int32_t *list_goff;  // [nlist+1] first vectorgroup of each bucket
    int32_t *list_size;  // [nlist]
    int32_t *slot_id;    // [ngroups*64] original row of each slot (-1 = pad)
    int32_t *assign;     // [n] bucket of each row
    uint16_t *pdx_bf16;  // [ngroups][d][64] (optional)
    uint8_t *pdx_fp8;    // [ngroups][d][64] (optional)
    float *fp8_scale;    // [d] per-dimension scale (optional)
    int32_t max_list;    // largest bucket, rows
};

namespace pdx {

void set_error(const char *fmt, ...);

inline size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

// Hands out aligned sub-ranges of one caller buffer (or only sizes them
// when base is null).
struct Carver {
    char *base;
    size_t off = 0;
    explicit Carver(void *b) : base(static_cast<char *>(b)) {}
    template <typename T>
    T *take(size_t count) {
        off = align_up(off, 256);
        T *p = base ? reinterpret_cast<T *>(base + off) : nullptr;
        off += count * sizeof(T);
        return p;
    }
    size_t bytes() const { return align_up(off, 256); }
};

// ---- launchers (each returns hipSuccess or the launch error) ----
hipError_t launch_finite_check(const float *x, int64_t count, int32_t *flag, hipStream_t s);
hipError_t launch_transpose_pdx(const float *x, int64_t n, int32_t d, float *pdx, hipStream_t s);
hipError_t launch_column_means(const float *x, int64_t n, int32_t d, double *partial,
                               int32_t nchunks, float *means, hipStream_t s);

struct ExactPlan {
    int64_t nq;
    int32_t k;
    int32_t mode;
    int32_t chunk;
    int32_t tile_groups;
    int32_t qpb;           // queries per workgroup (waves per block)
    int32_t start_groups;  // groups scanned by START
    int32_t tiles_start;
    int32_t tiles_main;
    int32_t nslots;
    // workspace parts
    uint32_t *tau;
    int32_t *bad;
    int32_t *perm_off;
    float *qperm;
    uint64_t *slots;
    hipEvent_t *events;              // optional [4]
    unsigned long long *counters;    // optional [4]
};

size_t exact_plan(const pdx_index *ix, int64_t nq, int32_t k, const pdx_search_params *p,
                  void *ws, ExactPlan *plan);
hipError_t run_exact(const pdx_index *ix, const float *q, const ExactPlan &plan,
                     int64_t *out_ids, float *out_dist, hipStream_t s);

}  // namespace pdx
