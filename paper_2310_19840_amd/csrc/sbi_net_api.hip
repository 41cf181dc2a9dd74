// sbi_net_api.hip -- C interface of the warm-start trainer (include/sbi_net.h).
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <vector>

#include "../../include/sbi_net.h"
#include "sbi_kernels.hpp"
#include "sbi_net.hpp"

using namespace sbi;

static_assert(SBI_NET_PARAMS == kNetParams, "parameter count");
static_assert(sizeof(sbi_net_header) == 64, "blob header");

namespace {
constexpr int kWgradBlocks = 256;  // workgroups of the weight-gradient reductions

struct TrLayout {
    size_t params, acts32, acts2, part, lpart, total;
};
size_t al(size_t b) { return (b + 255) / 256 * 256; }
TrLayout tr_layout(int batch, int ny, int nx) {
    TrLayout L{};
    const size_t n = (size_t)batch * ny * nx;
    TrainDims d{batch, ny, nx, (long long)n};
    L.params = al(sizeof(float) * kNetParams);                // one parameter-sized vector
    L.acts32 = al(sizeof(float) * n * 32);                    // one 32-channel field
    L.acts2 = al(sizeof(float) * n * 2);                      // one 2-channel field
    L.part = al(sizeof(float) * tr_part_floats(kWgradBlocks));
    L.lpart = al(sizeof(float) * tr_loss_blocks(d));
    L.total = 5 * L.params + 9 * L.acts32 + 2 * L.acts2 + L.part + L.lpart;
    return L;
}
bool dims_ok(int batch, int ny, int nx) {
    return batch >= 1 && ny >= 16 && nx >= 64 && nx % 64 == 0 && (long long)batch * ny * nx < (1ll << 31);
}
}  // namespace

struct sbi_net_trainer {
    TrainDims d{};
    TrainBuffers b{};
    float *theta = nullptr, *m = nullptr, *v = nullptr, *wq = nullptr;
    hipStream_t stream = nullptr;
    int step = 0;
    bool have_grad = false;
};

extern "C" int32_t sbi_net_param_count(void) { return kNetParams; }

extern "C" size_t sbi_net_blob_bytes(void) { return sizeof(sbi_net_header) + sizeof(float) * kNetParams; }

extern "C" size_t sbi_net_trainer_bytes(int32_t batch, int32_t ny, int32_t nx) {
    if (!dims_ok(batch, ny, nx)) return 0;
    return tr_layout(batch, ny, nx).total;
}

extern "C" sbi_status sbi_net_trainer_init(sbi_net_trainer** out, int32_t batch, int32_t ny, int32_t nx,
                                           const float* theta, void* workspace, size_t ws_bytes, void* hip_stream) {
    if (!out || !theta || !workspace || !dims_ok(batch, ny, nx)) return SBI_ERR_INVALID_ARG;
    *out = nullptr;
    const TrLayout L = tr_layout(batch, ny, nx);
    if (ws_bytes < L.total) return SBI_ERR_WORKSPACE;
    for (int i = 0; i < kNetParams; ++i)
        if (!std::isfinite(theta[i])) return SBI_ERR_INVALID_ARG;
    auto* tr = new sbi_net_trainer();
    tr->d = TrainDims{batch, ny, nx, (long long)batch * ny * nx};
    tr->stream = static_cast<hipStream_t>(hip_stream);
    char* p = static_cast<char*>(workspace);
    auto take = [&](size_t bytes) {
        char* q = p;
        p += bytes;
        return reinterpret_cast<float*>(q);
    };
    tr->theta = take(L.params);
    tr->m = take(L.params);
    tr->v = take(L.params);
    tr->wq = take(L.params);
    float* grad = take(L.params);
    TrainBuffers& b = tr->b;
    b.wq = tr->wq;
    b.z1 = take(L.acts32);
    b.a1 = take(L.acts32);
    b.z2 = take(L.acts32);
    b.a2 = take(L.acts32);
    b.z3 = take(L.acts32);
    b.a3 = take(L.acts32);
    b.g1 = take(L.acts32);
    b.g2 = take(L.acts32);
    b.g3 = take(L.acts32);
    b.y = take(L.acts2);
    b.gy = take(L.acts2);
    b.part = take(L.part);
    b.lpart = take(L.lpart);
    b.grad = grad;
    b.nblk = kWgradBlocks;
    hipError_t e = hipMemcpyAsync(tr->theta, theta, sizeof(float) * kNetParams, hipMemcpyHostToDevice, tr->stream);
    if (e == hipSuccess) e = launch_fill_zero(tr->m, L.params, tr->stream);
    if (e == hipSuccess) e = launch_fill_zero(tr->v, L.params, tr->stream);
    if (e == hipSuccess) e = tr_round_weights(tr->theta, tr->wq, tr->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(tr->stream);
    if (e != hipSuccess) {
        delete tr;
        return SBI_ERR_HIP;
    }
    *out = tr;
    return SBI_OK;
}

extern "C" sbi_status sbi_net_trainer_forward(sbi_net_trainer* tr, const float* feat, float* y_out) {
    if (!tr || !feat || !y_out) return SBI_ERR_INVALID_ARG;
    if (tr_forward(tr->d, tr->b, feat, nullptr, tr->stream) != hipSuccess) return SBI_ERR_HIP;
    if (hipMemcpyAsync(y_out, tr->b.y, sizeof(float) * 2 * tr->d.npts, hipMemcpyDeviceToDevice, tr->stream) !=
        hipSuccess)
        return SBI_ERR_HIP;
    return hipStreamSynchronize(tr->stream) == hipSuccess ? SBI_OK : SBI_ERR_HIP;
}

extern "C" sbi_status sbi_net_trainer_gradient(sbi_net_trainer* tr, const float* feat, const float* target,
                                               double* loss, float* grad_out) {
    if (!tr || !feat || !target) return SBI_ERR_INVALID_ARG;
    if (tr_forward(tr->d, tr->b, feat, target, tr->stream) != hipSuccess) return SBI_ERR_HIP;
    if (tr_backward(tr->d, tr->b, feat, tr->stream) != hipSuccess) return SBI_ERR_HIP;
    tr->have_grad = true;
    if (loss) {
        const int nb = tr_loss_blocks(tr->d);
        std::vector<float> lp(nb);
        if (hipMemcpyAsync(lp.data(), tr->b.lpart, sizeof(float) * nb, hipMemcpyDeviceToHost, tr->stream) !=
            hipSuccess)
            return SBI_ERR_HIP;
        if (hipStreamSynchronize(tr->stream) != hipSuccess) return SBI_ERR_HIP;
        double s = 0.0;
        for (float v : lp) s += v;
        *loss = s / (2.0 * (double)tr->d.npts);
        if (!std::isfinite(*loss)) return SBI_ERR_NONFINITE;
    }
    if (grad_out) {
        if (hipMemcpyAsync(grad_out, tr->b.grad, sizeof(float) * kNetParams, hipMemcpyDeviceToHost, tr->stream) !=
            hipSuccess)
            return SBI_ERR_HIP;
    }
    return hipStreamSynchronize(tr->stream) == hipSuccess ? SBI_OK : SBI_ERR_HIP;
}

extern "C" sbi_status sbi_net_trainer_adam(sbi_net_trainer* tr, float lr) {
    if (!tr || !tr->have_grad || !(lr > 0.0f) || !std::isfinite(lr)) return SBI_ERR_INVALID_ARG;
    tr->step += 1;
    const double b1 = 0.9, b2 = 0.999;
    const float bc1 = (float)(1.0 - std::pow(b1, tr->step));
    const float bc2 = (float)(1.0 - std::pow(b2, tr->step));
    if (tr_adam(tr->theta, tr->m, tr->v, tr->b.grad, tr->wq, lr, (float)b1, (float)b2, 1e-8f, bc1, bc2,
                tr->stream) != hipSuccess)
        return SBI_ERR_HIP;
    return SBI_OK;
}

extern "C" sbi_status sbi_net_trainer_params(sbi_net_trainer* tr, float* theta_out) {
    if (!tr || !theta_out) return SBI_ERR_INVALID_ARG;
    if (hipMemcpyAsync(theta_out, tr->theta, sizeof(float) * kNetParams, hipMemcpyDeviceToHost, tr->stream) !=
        hipSuccess)
        return SBI_ERR_HIP;
    return hipStreamSynchronize(tr->stream) == hipSuccess ? SBI_OK : SBI_ERR_HIP;
}

extern "C" sbi_status sbi_net_trainer_destroy(sbi_net_trainer* tr) {
    if (!tr) return SBI_ERR_INVALID_ARG;
    (void)hipStreamSynchronize(tr->stream);
    delete tr;
    return SBI_OK;
}
