// sbi_net.hpp -- learned warm start of the W iteration: parameter layout, the
// packed BF16 inference weights and the launchers of the network kernels.
//
// Network (periodic in y and x, channel-last fields):
//   x  = 8 scaled features (eta, W_lin, grad eta, grad phi, delta, eta W_lin)
//   z1 = b1 + conv3x3(x; W1) 8 -> 32,   a1 = silu(z1)
//   z2 = b2 + conv3x3(a1; W2) 32 -> 32, a2 = silu(z2)
//   z3 = b3 + W3 a2 (1x1) 32 -> 32,     a3 = silu(z3)
//   y  = b4 + W4 a3 (1x1) 32 -> 2
//   seeds V0 = W_lin + out_scale[0] y[0],  phi_b0 = S phi_hat + F{out_scale[1] y[1]}
// conv3x3 is the periodic cross-correlation over the 3x3 neighbourhood
// p + (t / 3 - 1, t % 3 - 1), t = 0..8.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

namespace sbi {

constexpr int kNetCin = 8;
constexpr int kNetWidth = 32;
// offsets in the FP32 parameter vector W1[32][9][8], b1, W2[32][9][32], b2,
// W3[32][32], b3, W4[2][32], b4[2]
constexpr int kOffW1 = 0;
constexpr int kOffB1 = kOffW1 + 32 * 9 * 8;
constexpr int kOffW2 = kOffB1 + 32;
constexpr int kOffB2 = kOffW2 + 32 * 9 * 32;
constexpr int kOffW3 = kOffB2 + 32;
constexpr int kOffB3 = kOffW3 + 32 * 32;
constexpr int kOffW4 = kOffB3 + 32;
constexpr int kOffB4 = kOffW4 + 2 * 32;
constexpr int kNetParams = kOffB4 + 2;

// packed inference weights: BF16 rows of K contiguous values per output
// channel (the B operand of the matrix-core products), row strides padded so
// that the 16 rows read by a quarter wave fall on distinct LDS banks
constexpr int kL1K = 96, kL1S = 104;   // 9 taps x 8 channels, zero-padded to 3 K-steps of 32
constexpr int kL2K = 288, kL2S = 296;  // 9 taps x 32 channels
constexpr int kL3K = 32, kL3S = 40;
struct NetPacked {
    uint16_t w1[32 * kL1S];
    uint16_t w2[32 * kL2S];
    uint16_t w3[32 * kL3S];
    uint16_t w4[2 * 32];
    float b1[32], b2[32], b3[32];
    float b4[2], out_scale[2];
    float in_scale[8];
    float pad[4];
};

struct NetInferParams {
    const float* feat;   // [batch][ny][nx][8] scaled features
    const void* wlin;    // [batch][ny][nx] W_lin in the working precision
    void* out;           // [batch][ny][nx] seed V0 in the working precision
    void* out_b;         // [batch][ny][nx] bottom-potential correction
    const NetPacked* w;
    int ny, nx;
    long long s_phys;    // member stride of the physical fields (points)
};
hipError_t launch_net_infer(int fp64, const NetInferParams& p, int batch, hipStream_t s);

// ---------------------------------------------------------------------------
// training (FP32 forward with the BF16-rounded weights, FP32 backward)
// ---------------------------------------------------------------------------
struct TrainDims {
    int batch, ny, nx;
    long long npts;      // batch * ny * nx
};
struct TrainBuffers {
    const float* wq;     // forward copy of the parameters (weights BF16-rounded)
    float *z1, *a1, *z2, *a2, *z3, *a3, *g1, *g2, *g3;
    float *y, *gy;       // [point][2]
    float* part;         // per-workgroup partial sums of the weight gradients
    float* lpart;        // per-workgroup partial sums of the squared residual
    float* grad;         // [kNetParams]
    int nblk;            // workgroups of the weight-gradient reductions
};
int tr_loss_blocks(const TrainDims& d);
size_t tr_part_floats(int nblk);
hipError_t tr_forward(const TrainDims& d, const TrainBuffers& b, const float* feat, const float* target,
                      hipStream_t s);
hipError_t tr_backward(const TrainDims& d, const TrainBuffers& b, const float* feat, hipStream_t s);
hipError_t tr_adam(float* theta, float* m, float* v, const float* g, float* wq, float lr, float beta1,
                   float beta2, float eps, float bc1, float bc2, hipStream_t s);
hipError_t tr_round_weights(const float* theta, float* wq, hipStream_t s);

}  // namespace sbi
