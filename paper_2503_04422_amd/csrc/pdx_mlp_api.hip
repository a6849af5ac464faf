// Entry points of the learned early-termination network (include/pdx.h).
#include "pdx_internal.h"

using namespace pdx;

namespace {
bool aligned16(const void *p) { return (reinterpret_cast<uintptr_t>(p) & 15u) == 0; }
pdx_status hip_fail(hipError_t e, const char *what) {
    set_error("%s: %s", what, hipGetErrorString(e));
    return PDX_EHIP;
}
}  // namespace

#define TRY(expr)                                        \
    do {                                                 \
        hipError_t e_ = (expr);                          \
        if (e_ != hipSuccess) return hip_fail(e_, what); \
    } while (0)

extern "C" {

size_t pdx_mlp_bytes(void) { return mlp_layout(nullptr).bytes; }

size_t pdx_mlp_workspace(int64_t n) { return n < 0 ? 0 : align_up(mlp_work_floats(n) * sizeof(float), 256); }

pdx_status pdx_mlp_init(void *mlp, const float *theta0, void *stream) {
    const char *what = "pdx_mlp_init";
    if (!mlp || !theta0 || !aligned16(mlp)) {
        set_error("pdx_mlp_init: null or misaligned pointer");
        return PDX_EINVAL;
    }
    TRY(launch_mlp_init(mlp_layout(mlp), theta0, static_cast<hipStream_t>(stream)));
    return PDX_OK;
}

pdx_status pdx_mlp_forward(const void *mlp, const float *x, int64_t n, float *z, void *stream) {
    const char *what = "pdx_mlp_forward";
    if (n < 0 || (n > 0 && (!mlp || !x || !z))) {
        set_error("pdx_mlp_forward: null pointer or n < 0");
        return PDX_EINVAL;
    }
    if (n == 0) return PDX_OK;
    TRY(launch_mlp_forward(mlp_layout(const_cast<void *>(mlp)).w16, x, n, z, static_cast<hipStream_t>(stream)));
    return PDX_OK;
}

namespace {
// w: the negatives' weight w0 >= 0 (PDX_LOSS_BCE) or the level in (0, 1)
// (PDX_LOSS_PINBALL)
bool loss_ok(int32_t kind, float w) {
    if (kind == PDX_LOSS_BCE) return w >= 0.0f && w < INFINITY;
    if (kind == PDX_LOSS_PINBALL) return w > 0.0f && w < 1.0f;
    return false;
}
}  // namespace

pdx_status pdx_mlp_grad(const void *mlp, const float *x, const float *y, int64_t n, int32_t loss_kind, float w,
                        void *ws, size_t ws_bytes, float *grad, float *loss, void *stream) {
    const char *what = "pdx_mlp_grad";
    if (n < 1 || !mlp || !x || !y || !ws || !grad || !loss_ok(loss_kind, w)) {
        set_error("pdx_mlp_grad: need n >= 1, a known loss with a valid w and non-null pointers");
        return PDX_EINVAL;
    }
    if (ws_bytes < pdx_mlp_workspace(n)) {
        set_error("pdx_mlp_grad: workspace has %zu bytes, needs %zu", ws_bytes, pdx_mlp_workspace(n));
        return PDX_EWORKSPACE;
    }
    MlpLayout L = mlp_layout(const_cast<void *>(mlp));
    TRY(launch_mlp_grad(L, x, y, n, loss_kind, w, static_cast<float *>(ws), grad, loss,
                        static_cast<hipStream_t>(stream)));
    return PDX_OK;
}

pdx_status pdx_mlp_train_step(void *mlp, const float *x, const float *y, int64_t n, int32_t loss_kind, float w,
                              float lr, int64_t step, void *ws, size_t ws_bytes, float *loss, void *stream) {
    const char *what = "pdx_mlp_train_step";
    if (n < 1 || !mlp || !x || !y || !ws || step < 1 || !(lr > 0.0f) || !loss_ok(loss_kind, w)) {
        set_error("pdx_mlp_train_step: need n >= 1, step >= 1, lr > 0, a known loss with a valid w and "
                  "non-null pointers");
        return PDX_EINVAL;
    }
    if (ws_bytes < pdx_mlp_workspace(n)) {
        set_error("pdx_mlp_train_step: workspace has %zu bytes, needs %zu", ws_bytes, pdx_mlp_workspace(n));
        return PDX_EWORKSPACE;
    }
    MlpLayout L = mlp_layout(mlp);
    hipStream_t s = static_cast<hipStream_t>(stream);
    TRY(launch_mlp_grad(L, x, y, n, loss_kind, w, static_cast<float *>(ws), L.g, loss ? loss : L.loss, s));
    TRY(launch_mlp_adam(L, lr, step, s));
    return PDX_OK;
}

pdx_status pdx_mlp_export(const void *mlp, float *theta, void *stream) {
    const char *what = "pdx_mlp_export";
    if (!mlp || !theta) {
        set_error("pdx_mlp_export: null pointer");
        return PDX_EINVAL;
    }
    MlpLayout L = mlp_layout(const_cast<void *>(mlp));
    TRY(hipMemcpyAsync(theta, L.theta, sizeof(float) * kMlpPad, hipMemcpyDeviceToDevice,
                       static_cast<hipStream_t>(stream)));
    return PDX_OK;
}

}  // extern "C"
