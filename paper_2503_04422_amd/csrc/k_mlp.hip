// The learned early-termination network: float16 weights, float32
// accumulation, x (72) -> relu(64) -> relu(64) -> logit.  Forward (used by
// the search's stop decision and by pdx_mlp_forward), and training kernels
// (per-sample forward/backward, deterministic gradient reduction, Adam).
//
// Parameter vector (float32 master copy and float16 deployed copy):
// W1 [64][72] | b1 [64] | W2 [64][64] | b2 [64] | w3 [64] | b3 [1], padded.
#include "mlp_device.h"
#include "pdx_internal.h"

namespace pdx {

namespace {

__global__ __launch_bounds__(256) void mlp_forward_kernel(const __half *__restrict__ w, const float *__restrict__ x,
                                                          int64_t n, float *__restrict__ z) {
    const int lane = threadIdx.x & 63;
    const int64_t s = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (s >= n) return;
    const float zz = mlp_forward_wave(w, x + s * kMlpIn, lane, nullptr, nullptr, nullptr, nullptr);
    if (lane == 0) z[s] = zz;
}

// Per sample: forward, loss term, and the backpropagated signals
//   weighted cross-entropy (w = w0):  dz = (-y (1-p) + w0 (1-y) p) / n,
//   pinball at level w:               dz = ([z > y] - w) / n,
//   dh2_j = dz w3_j [a2_j > 0],
//   dh1_i = sum_j W2[j][i] dh2_j [a1_i > 0]
// stored for the reduction kernel (H1, H2, DH1, DH2 are [n][64]).
__global__ __launch_bounds__(256) void mlp_backprop_kernel(const __half *__restrict__ w, const float *__restrict__ x,
                                                           const float *__restrict__ y, int64_t n, int32_t kind,
                                                           float w0, float *__restrict__ H1, float *__restrict__ H2,
                                                           float *__restrict__ DH1, float *__restrict__ DH2,
                                                           float *__restrict__ DZ, float *__restrict__ LS) {
    const int lane = threadIdx.x & 63;
    const int64_t s = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (s >= n) return;
    float a1, h1, a2, h2;
    const float z = mlp_forward_wave(w, x + s * kMlpIn, lane, &a1, &h1, &a2, &h2);
    const float yy = y[s];
    const float p = 1.0f / (1.0f + expf(-z));
    const float dz = kind == PDX_LOSS_PINBALL ? ((z > yy ? 1.0f : 0.0f) - w0) / (float)n
                                              : (-yy * (1.0f - p) + w0 * (1.0f - yy) * p) / (float)n;
    const float dh2 = a2 > 0.0f ? dz * h2f(w, kOffW3 + lane) : 0.0f;
    // dh1_i for i = lane: sum over j of W2[j][lane] dh2_j
    float dh1 = 0.0f;
    for (int j = 0; j < kMlpH; ++j) dh1 = fmaf(h2f(w, kOffW2 + j * kMlpH + lane), __shfl(dh2, j), dh1);
    if (!(a1 > 0.0f)) dh1 = 0.0f;
    H1[s * kMlpH + lane] = h1;
    H2[s * kMlpH + lane] = h2;
    DH1[s * kMlpH + lane] = dh1;
    DH2[s * kMlpH + lane] = dh2;
    if (lane == 0) {
        DZ[s] = dz;
        if (kind == PDX_LOSS_PINBALL) {
            const float u = yy - z;
            LS[s] = u * (u < 0.0f ? w0 - 1.0f : w0) / (float)n;
        } else {  // softplus form of the loss term
            const float spn = fmaxf(-z, 0.0f) + log1pf(expf(-fabsf(z)));
            const float spp = fmaxf(z, 0.0f) + log1pf(expf(-fabsf(z)));
            LS[s] = (yy * spn + w0 * (1.0f - yy) * spp) / (float)n;
        }
    }
}

// Gradient of every parameter: sums over samples in sample order (one
// thread per parameter).
__global__ __launch_bounds__(256) void mlp_grad_reduce_kernel(const float *__restrict__ x, int64_t n,
                                                              const float *__restrict__ H1,
                                                              const float *__restrict__ H2,
                                                              const float *__restrict__ DH1,
                                                              const float *__restrict__ DH2,
                                                              const float *__restrict__ DZ,
                                                              const float *__restrict__ LS, float *__restrict__ g,
                                                              float *__restrict__ loss) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= kMlpPad) return;
    float acc = 0.0f;
    if (p < kOffB1) {  // W1[j][i] += dh1_j x_i
        const int j = p / kMlpIn, i = p % kMlpIn;
        for (int64_t s = 0; s < n; ++s) acc = fmaf(DH1[s * kMlpH + j], x[s * kMlpIn + i], acc);
    } else if (p < kOffW2) {
        const int j = p - kOffB1;
        for (int64_t s = 0; s < n; ++s) acc += DH1[s * kMlpH + j];
    } else if (p < kOffB2) {  // W2[j][i] += dh2_j h1_i
        const int q = p - kOffW2, j = q / kMlpH, i = q % kMlpH;
        for (int64_t s = 0; s < n; ++s) acc = fmaf(DH2[s * kMlpH + j], H1[s * kMlpH + i], acc);
    } else if (p < kOffW3) {
        const int j = p - kOffB2;
        for (int64_t s = 0; s < n; ++s) acc += DH2[s * kMlpH + j];
    } else if (p < kOffB3) {  // w3_j += dz h2_j
        const int j = p - kOffW3;
        for (int64_t s = 0; s < n; ++s) acc = fmaf(DZ[s], H2[s * kMlpH + j], acc);
    } else if (p == kOffB3) {
        for (int64_t s = 0; s < n; ++s) acc += DZ[s];
        if (loss) {
            float l = 0.0f;
            for (int64_t s = 0; s < n; ++s) l += LS[s];
            *loss = l;
        }
    }
    g[p] = acc;
}

__global__ void mlp_adam_kernel(float *__restrict__ theta, float *__restrict__ m, float *__restrict__ v,
                                const float *__restrict__ g, __half *__restrict__ w16, float lr, float b1t,
                                float b2t) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= kMlpPad) return;
    if (p > kOffB3) {
        w16[p] = __float2half(0.0f);
        return;
    }
    const float gg = g[p];
    const float mm = 0.9f * m[p] + 0.1f * gg;
    const float vv = 0.999f * v[p] + 0.001f * gg * gg;
    m[p] = mm;
    v[p] = vv;
    const float th = theta[p] - lr * (mm / (1.0f - b1t)) / (sqrtf(vv / (1.0f - b2t)) + 1e-8f);
    theta[p] = th;
    w16[p] = __float2half(th);
}

__global__ void mlp_init_kernel(const float *__restrict__ theta0, float *__restrict__ theta, float *__restrict__ m,
                                float *__restrict__ v, __half *__restrict__ w16) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= kMlpPad) return;
    const float t = p <= kOffB3 ? theta0[p] : 0.0f;
    theta[p] = t;
    m[p] = 0.0f;
    v[p] = 0.0f;
    w16[p] = __float2half(t);
}

}  // namespace

MlpLayout mlp_layout(void *base) {
    Carver c(base);
    MlpLayout l{};
    l.theta = c.take<float>(kMlpPad);
    l.m = c.take<float>(kMlpPad);
    l.v = c.take<float>(kMlpPad);
    l.g = c.take<float>(kMlpPad);
    l.w16 = c.take<__half>(kMlpPad);
    l.loss = c.take<float>(64);
    l.bytes = c.bytes();
    return l;
}

hipError_t launch_mlp_init(const MlpLayout &L, const float *theta0, hipStream_t s) {
    mlp_init_kernel<<<(kMlpPad + 255) / 256, 256, 0, s>>>(theta0, L.theta, L.m, L.v, L.w16);
    return hipGetLastError();
}

hipError_t launch_mlp_forward(const __half *w16, const float *x, int64_t n, float *z, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    mlp_forward_kernel<<<(unsigned)((n + 3) / 4), 256, 0, s>>>(w16, x, n, z);
    return hipGetLastError();
}

hipError_t launch_mlp_grad(const MlpLayout &L, const float *x, const float *y, int64_t n, int32_t kind, float w0,
                           float *work, float *grad, float *loss, hipStream_t s) {
    float *H1 = work, *H2 = H1 + n * kMlpH, *DH1 = H2 + n * kMlpH, *DH2 = DH1 + n * kMlpH, *DZ = DH2 + n * kMlpH,
          *LS = DZ + n;
    mlp_backprop_kernel<<<(unsigned)((n + 3) / 4), 256, 0, s>>>(L.w16, x, y, n, kind, w0, H1, H2, DH1, DH2, DZ, LS);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    mlp_grad_reduce_kernel<<<(kMlpPad + 255) / 256, 256, 0, s>>>(x, n, H1, H2, DH1, DH2, DZ, LS, grad, loss);
    return hipGetLastError();
}

hipError_t launch_mlp_adam(const MlpLayout &L, float lr, int64_t step, hipStream_t s) {
    const float b1t = powf(0.9f, (float)step), b2t = powf(0.999f, (float)step);
    mlp_adam_kernel<<<(kMlpPad + 255) / 256, 256, 0, s>>>(L.theta, L.m, L.v, L.g, L.w16, lr, b1t, b2t);
    return hipGetLastError();
}

size_t mlp_work_floats(int64_t n) { return (size_t)n * (4 * kMlpH + 2); }

}  // namespace pdx
