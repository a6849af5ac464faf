// Device-side forward pass of the search's networks (probe budget and
// prune multiplier), shared by the training kernels and the search.
#pragma once

#include "pdx_internal.h"

namespace pdx {

constexpr int kOffW1 = 0, kOffB1 = kMlpH * kMlpIn, kOffW2 = kOffB1 + kMlpH, kOffB2 = kOffW2 + kMlpH * kMlpH,
              kOffW3 = kOffB2 + kMlpH, kOffB3 = kOffW3 + kMlpH;

__device__ __forceinline__ float h2f(const __half *w, int i) { return __half2float(w[i]); }

// First layer's pre-activation of hidden unit `lane`, inputs i0 .. i1-1
// added to a1 in index order (a1 starts at the unit's bias).  Splitting
// the inputs into runs gives the same value as one pass.
__device__ __forceinline__ float mlp_a1_run(const __half *__restrict__ w, const float *__restrict__ x, int lane,
                                            int i0, int i1, float a1) {
    const __half *r1 = w + kOffW1 + lane * kMlpIn;
#pragma unroll 8
    for (int i = i0; i < i1; ++i) a1 = fmaf(h2f(r1, i), x[i], a1);
    return a1;
}

// Layers 2 and 3 from the first layer's pre-activation (lane j = unit j).
// Returns z (wave-uniform); h1/h2 and the pre-activations of this lane's
// units are returned through the pointers.
__device__ __forceinline__ float mlp_tail_wave(const __half *__restrict__ w, float a1, int lane, float *a1_out,
                                               float *h1_out, float *a2_out, float *h2_out) {
    const float h1 = fmaxf(a1, 0.0f);
    float a2 = h2f(w, kOffB2 + lane);
    const __half *r2 = w + kOffW2 + lane * kMlpH;
#pragma unroll 8
    for (int i = 0; i < kMlpH; ++i) a2 = fmaf(h2f(r2, i), __shfl(h1, i), a2);
    const float h2 = fmaxf(a2, 0.0f);
    float part = h2f(w, kOffW3 + lane) * h2;
    for (int off = 32; off > 0; off >>= 1) part += __shfl_xor(part, off);
    if (a1_out) {
        *a1_out = a1;
        *h1_out = h1;
        *a2_out = a2;
        *h2_out = h2;
    }
    return part + h2f(w, kOffB3);
}

// One wave evaluates one sample; lane j is hidden unit j.  x points to 72
// inputs (wave-uniform).
__device__ __forceinline__ float mlp_forward_wave(const __half *__restrict__ w, const float *__restrict__ x, int lane,
                                                  float *a1_out, float *h1_out, float *a2_out, float *h2_out) {
    const float a1 = mlp_a1_run(w, x, lane, 0, kMlpIn, h2f(w, kOffB1 + lane));
    return mlp_tail_wave(w, a1, lane, a1_out, h1_out, a2_out, h2_out);
}

}  // namespace pdx
