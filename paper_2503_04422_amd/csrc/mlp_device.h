// Device-side forward pass of the early-termination network, shared by the
// training kernels and the search's checkpoint kernel.
#pragma once

#include "pdx_internal.h"

namespace pdx {

constexpr int kOffW1 = 0, kOffB1 = kMlpH * kMlpIn, kOffW2 = kOffB1 + kMlpH, kOffB2 = kOffW2 + kMlpH * kMlpH,
              kOffW3 = kOffB2 + kMlpH, kOffB3 = kOffW3 + kMlpH;

__device__ __forceinline__ float h2f(const __half *w, int i) { return __half2float(w[i]); }

// One wave evaluates one sample; lane j is hidden unit j.  x points to 72
// inputs (wave-uniform).  Returns z (wave-uniform); h1/h2 and the
// pre-activations of this lane's units are returned through the pointers.
__device__ __forceinline__ float mlp_forward_wave(const __half *__restrict__ w, const float *__restrict__ x, int lane, float *a1_out,
                                  float *h1_out, float *a2_out, float *h2_out) {
    float a1 = h2f(w, kOffB1 + lane);
    const __half *r1 = w + kOffW1 + lane * kMlpIn;
#pragma unroll 8
    for (int i = 0; i < kMlpIn; ++i) a1 = fmaf(h2f(r1, i), x[i], a1);
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

}  // namespace pdx
