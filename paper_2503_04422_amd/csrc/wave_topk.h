// Wave-wide sorted k-best list (k <= 64) held in registers.
//
// A candidate is the 64-bit key (float bits of the distance << 32 | row id).
// For non-negative distances the unsigned order of the keys is the
// (distance, id) order used for results, so one integer compare ranks two
// candidates and ties on distance fall back to the lower id.
//
// Lane i (< k) holds the i-th smallest key; the list starts filled with
// kEmptyKey (all ones), which ranks after every real candidate.
#pragma once

#include "pdx_internal.h"

namespace pdx {

__device__ __forceinline__ uint64_t make_key(float dist, uint32_t id) {
    return (static_cast<uint64_t>(__float_as_uint(dist)) << 32) | id;
}

__device__ __forceinline__ float key_dist(uint64_t key) {
    return __uint_as_float(static_cast<uint32_t>(key >> 32));
}

__device__ __forceinline__ uint64_t readlane64(uint64_t v, int lane) {
    uint32_t lo = __builtin_amdgcn_readlane(static_cast<uint32_t>(v), lane);
    uint32_t hi = __builtin_amdgcn_readlane(static_cast<uint32_t>(v >> 32), lane);
    return (static_cast<uint64_t>(hi) << 32) | lo;
}

// value of lane-1 (lane 0 gets its own value back; it is never used)
__device__ __forceinline__ uint64_t shift_up64(uint64_t v, int lane) {
    int src = (lane == 0 ? 0 : lane - 1) << 2;
    uint32_t lo = __builtin_amdgcn_ds_bpermute(src, static_cast<int>(static_cast<uint32_t>(v)));
    uint32_t hi = __builtin_amdgcn_ds_bpermute(src, static_cast<int>(static_cast<uint32_t>(v >> 32)));
    return (static_cast<uint64_t>(hi) << 32) | lo;
}

// Insert a wave-uniform key that is smaller than the current k-th entry.
__device__ __forceinline__ void topk_insert(uint64_t &e, uint64_t key, int k, int lane) {
    unsigned long long below = __ballot(lane < k && e < key);
    int pos = __popcll(below);
    uint64_t up = shift_up64(e, lane);
    if (lane < k) {
        if (lane == pos)
            e = key;
        else if (lane > pos)
            e = up;
    }
}

// Offer every lane's key where `want` holds; keeps the k smallest.
// `kth` (wave-uniform) is the current k-th entry and is kept up to date.
__device__ __forceinline__ void topk_offer(uint64_t &e, uint64_t &kth, uint64_t key, bool want, int k,
                                           int lane) {
    unsigned long long m = __ballot(want && key < kth);
    while (m) {
        int src = __ffsll(static_cast<long long>(m)) - 1;
        m &= m - 1;
        uint64_t kk = readlane64(key, src);
        if (kk < kth) {
            topk_insert(e, kk, k, lane);
            kth = readlane64(e, k - 1);
        }
    }
}

}  // namespace pdx
