// sbi_net.hip -- kernels of the learned warm start: fused BF16 matrix-core
// inference (all four layers per 16x16 tile, activations in LDS) and the FP32
// training kernels (forward, backward, weight-gradient reductions, Adam).
#include <hip/hip_runtime.h>

#include "sbi_net.hpp"

namespace sbi {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

// round to nearest even BF16 (finite inputs)
__device__ __forceinline__ uint32_t bf16_bits(float f) {
    uint32_t u = __float_as_uint(f);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return u >> 16;
}
__device__ __forceinline__ float bf16_round(float f) { return __uint_as_float(bf16_bits(f) << 16); }
__device__ __forceinline__ float bf16_value(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }
__device__ __forceinline__ float silu(float z) { return z / (1.0f + expf(-z)); }
__device__ __forceinline__ float dsilu(float z) {
    const float s = 1.0f / (1.0f + expf(-z));
    return s * (1.0f + z * (1.0f - s));
}
__device__ __forceinline__ f32x4 mfma16x16x32(uint4 a, uint4 b, f32x4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, a), __builtin_bit_cast(bf16x8, b), c,
                                                   0, 0, 0);
}

// ---------------------------------------------------------------------------
// Inference: one workgroup (4 waves) per 16x16 output tile at a time.
//   input tile 20x20 (halo 2) -> layer 1 on 18x18 -> layer 2 on 16x16 ->
//   layers 3, 4 pointwise.  Matrix-core products 16 points x 16 channels x
//   32 K per instruction; lane l supplies A row l%16 (a point) and B column
//   l%16 (an output channel) for K values 8(l/16)..8(l/16)+7, and receives
//   D rows 4(l/16)..4(l/16)+3 of column l%16.
// ---------------------------------------------------------------------------
constexpr int kT = 16;            // output tile edge
constexpr int kIn = kT + 4;       // input tile edge
constexpr int kA1 = kT + 2;       // layer-1 tile edge
constexpr int kA1Pts = 336;       // 18 * 18 = 324 points padded to 21 M-blocks of 16
constexpr int kPS = 40;           // activation point stride (BF16): 80 bytes, conflict-free rows

template <typename RO>
__global__ void __launch_bounds__(256) k_net_infer(const NetInferParams p) {
    __shared__ __attribute__((aligned(16))) uint16_t sW1[32 * kL1S];
    __shared__ __attribute__((aligned(16))) uint16_t sW2[32 * kL2S];
    __shared__ __attribute__((aligned(16))) uint16_t sW3[32 * kL3S];
    __shared__ __attribute__((aligned(16))) uint16_t sIn[kIn * kIn * 8];
    __shared__ __attribute__((aligned(16))) uint16_t sA1[kA1Pts * kPS];
    __shared__ __attribute__((aligned(16))) uint16_t sA2[kT * kT * kPS];
    __shared__ float sB1[32], sB2[32], sB3[32], sW4[64];

    const int t = threadIdx.x;
    const int wave = t >> 6, lane = t & 63;
    const int lr = lane & 15, lg = lane >> 4;
    {
        const uint4* s1 = reinterpret_cast<const uint4*>(p.w->w1);
        uint4* d1 = reinterpret_cast<uint4*>(sW1);
        for (int i = t; i < 32 * kL1S / 8; i += 256) d1[i] = s1[i];
        const uint4* s2 = reinterpret_cast<const uint4*>(p.w->w2);
        uint4* d2 = reinterpret_cast<uint4*>(sW2);
        for (int i = t; i < 32 * kL2S / 8; i += 256) d2[i] = s2[i];
        const uint4* s3 = reinterpret_cast<const uint4*>(p.w->w3);
        uint4* d3 = reinterpret_cast<uint4*>(sW3);
        for (int i = t; i < 32 * kL3S / 8; i += 256) d3[i] = s3[i];
        if (t < 32) {
            sB1[t] = p.w->b1[t];
            sB2[t] = p.w->b2[t];
            sB3[t] = p.w->b3[t];
        }
        if (t < 64) sW4[t] = bf16_value(p.w->w4[t]);
    }
    const float b40 = p.w->b4[0], b41 = p.w->b4[1];
    const float osc0 = p.w->out_scale[0], osc1 = p.w->out_scale[1];
    const int mem = blockIdx.y;
    const int tiles_x = p.nx / kT, tiles = tiles_x * (p.ny / kT);
    const long long mbase = (long long)mem * p.s_phys;
    const RO* wlin = static_cast<const RO*>(p.wlin) + mbase;
    RO* out = static_cast<RO*>(p.out) + mbase;
    RO* out_b = static_cast<RO*>(p.out_b) + mbase;

    for (int tile = blockIdx.x; tile < tiles; tile += gridDim.x) {
        const int ty0 = (tile / tiles_x) * kT, tx0 = (tile % tiles_x) * kT;
        __syncthreads();  // weights staged / previous tile's readers done
        for (int i = t; i < kIn * kIn; i += 256) {
            const int r = i / kIn, c = i % kIn;
            const int gy = (ty0 - 2 + r + p.ny) % p.ny, gx = (tx0 - 2 + c + p.nx) % p.nx;
            const float4* src = reinterpret_cast<const float4*>(p.feat + (mbase + (long long)gy * p.nx + gx) * 8);
            const float4 u = src[0], v = src[1];
            uint4 pk;
            pk.x = bf16_bits(u.x) | (bf16_bits(u.y) << 16);
            pk.y = bf16_bits(u.z) | (bf16_bits(u.w) << 16);
            pk.z = bf16_bits(v.x) | (bf16_bits(v.y) << 16);
            pk.w = bf16_bits(v.z) | (bf16_bits(v.w) << 16);
            *reinterpret_cast<uint4*>(sIn + i * 8) = pk;
        }
        __syncthreads();
        // layer 1: 18x18 points, K = 9 taps x 8 channels in 3 steps of 32
        for (int mb = wave; mb < kA1Pts / 16; mb += 4) {
            f32x4 acc0 = {0.f, 0.f, 0.f, 0.f}, acc1 = {0.f, 0.f, 0.f, 0.f};
            const int pm = mb * 16 + lr;
            const bool pv = pm < kA1 * kA1;
            const int a = pv ? pm / kA1 : 0, b = pv ? pm % kA1 : 0;
#pragma unroll
            for (int s = 0; s < 3; ++s) {
                const int tap = 4 * s + lg;
                uint4 av = make_uint4(0u, 0u, 0u, 0u);
                if (pv && tap < 9) av = *reinterpret_cast<const uint4*>(sIn + ((a + tap / 3) * kIn + b + tap % 3) * 8);
                const uint4 bv0 = *reinterpret_cast<const uint4*>(sW1 + lr * kL1S + 32 * s + 8 * lg);
                const uint4 bv1 = *reinterpret_cast<const uint4*>(sW1 + (16 + lr) * kL1S + 32 * s + 8 * lg);
                acc0 = mfma16x16x32(av, bv0, acc0);
                acc1 = mfma16x16x32(av, bv1, acc1);
            }
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int pt = mb * 16 + 4 * lg + q;
                sA1[pt * kPS + lr] = (uint16_t)bf16_bits(silu(acc0[q] + sB1[lr]));
                sA1[pt * kPS + 16 + lr] = (uint16_t)bf16_bits(silu(acc1[q] + sB1[16 + lr]));
            }
        }
        __syncthreads();
        // layer 2: 16x16 points, K = 9 taps x 32 channels
        for (int mb = wave; mb < kT * kT / 16; mb += 4) {
            f32x4 acc0 = {0.f, 0.f, 0.f, 0.f}, acc1 = {0.f, 0.f, 0.f, 0.f};
            const int pm = mb * 16 + lr;
            const int a = pm / kT, b = pm % kT;
#pragma unroll
            for (int s = 0; s < 9; ++s) {
                const uint4 av =
                    *reinterpret_cast<const uint4*>(sA1 + ((a + s / 3) * kA1 + b + s % 3) * kPS + 8 * lg);
                const uint4 bv0 = *reinterpret_cast<const uint4*>(sW2 + lr * kL2S + 32 * s + 8 * lg);
                const uint4 bv1 = *reinterpret_cast<const uint4*>(sW2 + (16 + lr) * kL2S + 32 * s + 8 * lg);
                acc0 = mfma16x16x32(av, bv0, acc0);
                acc1 = mfma16x16x32(av, bv1, acc1);
            }
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int pt = mb * 16 + 4 * lg + q;
                sA2[pt * kPS + lr] = (uint16_t)bf16_bits(silu(acc0[q] + sB2[lr]));
                sA2[pt * kPS + 16 + lr] = (uint16_t)bf16_bits(silu(acc1[q] + sB2[16 + lr]));
            }
        }
        __syncthreads();
        // layers 3 and 4
        for (int mb = wave; mb < kT * kT / 16; mb += 4) {
            const f32x4 zero = {0.f, 0.f, 0.f, 0.f};
            const uint4 av = *reinterpret_cast<const uint4*>(sA2 + (mb * 16 + lr) * kPS + 8 * lg);
            const uint4 bv0 = *reinterpret_cast<const uint4*>(sW3 + lr * kL3S + 8 * lg);
            const uint4 bv1 = *reinterpret_cast<const uint4*>(sW3 + (16 + lr) * kL3S + 8 * lg);
            const f32x4 z0 = mfma16x16x32(av, bv0, zero);
            const f32x4 z1 = mfma16x16x32(av, bv1, zero);
            float y0[4], y1[4];
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const float s0 = silu(z0[q] + sB3[lr]), s1 = silu(z1[q] + sB3[16 + lr]);
                y0[q] = s0 * sW4[lr] + s1 * sW4[16 + lr];
                y1[q] = s0 * sW4[32 + lr] + s1 * sW4[48 + lr];
            }
#pragma unroll
            for (int off = 1; off < 16; off <<= 1)
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    y0[q] += __shfl_xor(y0[q], off);
                    y1[q] += __shfl_xor(y1[q], off);
                }
            if (lr == 0) {
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const int pt = mb * 16 + 4 * lg + q;
                    const long long gi = (long long)(ty0 + pt / kT) * p.nx + tx0 + pt % kT;
                    out[gi] = wlin[gi] + (RO)(osc0 * (y0[q] + b40));
                    out_b[gi] = (RO)(osc1 * (y1[q] + b41));
                }
            }
        }
    }
}

hipError_t launch_net_infer(int fp64, const NetInferParams& p, int batch, hipStream_t s) {
    if (p.nx % kT || p.ny % kT) return hipErrorInvalidValue;
    int tiles = (p.nx / kT) * (p.ny / kT);
    const unsigned gx = (unsigned)(tiles < 1024 ? tiles : 1024);
    if (fp64)
        hipLaunchKernelGGL(k_net_infer<double>, dim3(gx, batch), dim3(256), 0, s, p);
    else
        hipLaunchKernelGGL(k_net_infer<float>, dim3(gx, batch), dim3(256), 0, s, p);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Training kernels (FP32).  Fields are channel-last [point][channel] with
// points ordered (member, y, x); one thread per point in the pointwise and
// convolution kernels.
// ---------------------------------------------------------------------------
__device__ __forceinline__ long long nbr(const TrainDims& d, long long p, int dy, int dx) {
    const int x = (int)(p % d.nx);
    const int y = (int)((p / d.nx) % d.ny);
    const long long base = p - (long long)y * d.nx - x;
    return base + (long long)((y + dy + d.ny) % d.ny) * d.nx + (x + dx + d.nx) % d.nx;
}

// z = b + sum_t sum_c W[o][t][c] in[p + off(t)][c],  a = silu(z)
template <int CIN>
__global__ void __launch_bounds__(256) k_tr_conv3(const float* __restrict__ in, const float* __restrict__ w,
                                                  const float* __restrict__ bias, float* __restrict__ z,
                                                  float* __restrict__ a, TrainDims d) {
    constexpr int COUT = 32;
    __shared__ float sw[9 * CIN * COUT];  // [t][c][o]
    for (int i = threadIdx.x; i < 9 * CIN * COUT; i += 256) {
        const int o = i % COUT, tc = i / COUT;
        sw[i] = w[o * 9 * CIN + tc];
    }
    __syncthreads();
    const long long p = (long long)blockIdx.x * 256 + threadIdx.x;
    if (p >= d.npts) return;
    float acc[COUT];
#pragma unroll
    for (int o = 0; o < COUT; ++o) acc[o] = bias[o];
    for (int tap = 0; tap < 9; ++tap) {
        const float4* src = reinterpret_cast<const float4*>(in + nbr(d, p, tap / 3 - 1, tap % 3 - 1) * CIN);
#pragma unroll
        for (int c4 = 0; c4 < CIN / 4; ++c4) {
            const float4 v = src[c4];
            const float vv[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const float* wr = sw + (tap * CIN + c4 * 4 + e) * COUT;
#pragma unroll
                for (int o = 0; o < COUT; ++o) acc[o] = fmaf(vv[e], wr[o], acc[o]);
            }
        }
    }
#pragma unroll
    for (int o = 0; o < COUT; ++o) {
        z[p * COUT + o] = acc[o];
        a[p * COUT + o] = silu(acc[o]);
    }
}

// layers 3 and 4, residuals and dL/dy; per-workgroup partial of sum (y - t)^2
__global__ void __launch_bounds__(256) k_tr_head(const float* __restrict__ a2, const float* __restrict__ wq,
                                                 const float* __restrict__ target, float* __restrict__ z3,
                                                 float* __restrict__ a3, float* __restrict__ y,
                                                 float* __restrict__ gy, float* __restrict__ lpart, TrainDims d) {
    __shared__ float sw3[32 * 32];  // [c][o]
    __shared__ float sb3[32], sw4[64];
    __shared__ double red[256];
    for (int i = threadIdx.x; i < 1024; i += 256) sw3[i] = wq[kOffW3 + (i % 32) * 32 + i / 32];
    if (threadIdx.x < 32) sb3[threadIdx.x] = wq[kOffB3 + threadIdx.x];
    if (threadIdx.x < 64) sw4[threadIdx.x] = wq[kOffW4 + threadIdx.x];
    __syncthreads();
    const long long p = (long long)blockIdx.x * 256 + threadIdx.x;
    double r2 = 0.0;
    if (p < d.npts) {
        float acc[32];
#pragma unroll
        for (int o = 0; o < 32; ++o) acc[o] = sb3[o];
        const float4* src = reinterpret_cast<const float4*>(a2 + p * 32);
#pragma unroll
        for (int c4 = 0; c4 < 8; ++c4) {
            const float4 v = src[c4];
            const float vv[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
            for (int e = 0; e < 4; ++e)
#pragma unroll
                for (int o = 0; o < 32; ++o) acc[o] = fmaf(vv[e], sw3[(c4 * 4 + e) * 32 + o], acc[o]);
        }
        float out0 = wq[kOffB4], out1 = wq[kOffB4 + 1];
#pragma unroll
        for (int o = 0; o < 32; ++o) {
            const float s = silu(acc[o]);
            z3[p * 32 + o] = acc[o];
            a3[p * 32 + o] = s;
            out0 = fmaf(sw4[o], s, out0);
            out1 = fmaf(sw4[32 + o], s, out1);
        }
        y[2 * p] = out0;
        y[2 * p + 1] = out1;
        if (target) {
            // L = mean over points and both outputs of (y - t)^2
            const float r0 = out0 - target[2 * p], r1 = out1 - target[2 * p + 1];
            const float sc = 2.0f / (2.0f * (float)d.npts);
            gy[2 * p] = sc * r0;
            gy[2 * p + 1] = sc * r1;
            r2 = (double)r0 * (double)r0 + (double)r1 * (double)r1;
        }
    }
    red[threadIdx.x] = r2;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0 && lpart) lpart[blockIdx.x] = (float)red[0];
}

// dL/dz3 = (W4^T gy) silu'(z3);  dL/dz2 = (W3^T dL/dz3) silu'(z2)
__global__ void __launch_bounds__(256) k_tr_head_bwd(const float* __restrict__ gy, const float* __restrict__ z3,
                                                     const float* __restrict__ z2, const float* __restrict__ wq,
                                                     float* __restrict__ g3, float* __restrict__ g2, TrainDims d) {
    __shared__ float sw3[32 * 32];  // [o][c]
    __shared__ float sw4[64];
    for (int i = threadIdx.x; i < 1024; i += 256) sw3[i] = wq[kOffW3 + i];
    if (threadIdx.x < 64) sw4[threadIdx.x] = wq[kOffW4 + threadIdx.x];
    __syncthreads();
    const long long p = (long long)blockIdx.x * 256 + threadIdx.x;
    if (p >= d.npts) return;
    const float gp0 = gy[2 * p], gp1 = gy[2 * p + 1];
    float acc[32];
#pragma unroll
    for (int c = 0; c < 32; ++c) acc[c] = 0.f;
    for (int o = 0; o < 32; ++o) {
        const float g = (gp0 * sw4[o] + gp1 * sw4[32 + o]) * dsilu(z3[p * 32 + o]);
        g3[p * 32 + o] = g;
#pragma unroll
        for (int c = 0; c < 32; ++c) acc[c] = fmaf(g, sw3[o * 32 + c], acc[c]);
    }
#pragma unroll
    for (int c = 0; c < 32; ++c) g2[p * 32 + c] = acc[c] * dsilu(z2[p * 32 + c]);
}

// dL/dz1(q)[c] = silu'(z1(q)[c]) sum_t sum_o dL/dz2(q - off(t))[o] W2[o][t][c]
__global__ void __launch_bounds__(256) k_tr_conv3_bwd(const float* __restrict__ g2, const float* __restrict__ wq,
                                                      const float* __restrict__ z1, float* __restrict__ g1,
                                                      TrainDims d) {
    __shared__ float sw[9 * 32 * 32];  // [t][o][c]
    for (int i = threadIdx.x; i < 9 * 32 * 32; i += 256) {
        const int c = i % 32, o = (i / 32) % 32, tap = i / 1024;
        sw[i] = wq[kOffW2 + (o * 9 + tap) * 32 + c];
    }
    __syncthreads();
    const long long p = (long long)blockIdx.x * 256 + threadIdx.x;
    if (p >= d.npts) return;
    float acc[32];
#pragma unroll
    for (int c = 0; c < 32; ++c) acc[c] = 0.f;
    for (int tap = 0; tap < 9; ++tap) {
        const float4* src = reinterpret_cast<const float4*>(g2 + nbr(d, p, 1 - tap / 3, 1 - tap % 3) * 32);
        for (int o4 = 0; o4 < 8; ++o4) {
            const float4 v = src[o4];
            const float vv[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const float* wr = sw + (tap * 32 + o4 * 4 + e) * 32;
#pragma unroll
                for (int c = 0; c < 32; ++c) acc[c] = fmaf(vv[e], wr[c], acc[c]);
            }
        }
    }
#pragma unroll
    for (int c = 0; c < 32; ++c) g1[p * 32 + c] = acc[c] * dsilu(z1[p * 32 + c]);
}

// Weight gradients of one layer: dW[o][t][c] = sum_p g(p)[o] a(p + off(t))[c],
// db[o] = sum_p g(p)[o].  Workgroup b sums the 64-point runs b, b + nblk, ...
// (runs lie inside one row).  Thread t owns output channel o = t % COUT and
// input channels c = t / COUT + j * (256 / COUT) for every tap, so its LDS
// offsets are compile-time constants.  part[b][NP + COUT] holds the partial
// sums in the order ((t * CIN + c) * COUT + o), then the biases.
constexpr int kRun = 64;
template <int TAPS, int CIN, int COUT>
__global__ void __launch_bounds__(256) k_tr_wgrad(const float* __restrict__ g, const float* __restrict__ a,
                                                  float* __restrict__ part, TrainDims d) {
    constexpr int NP = TAPS * CIN * COUT;
    constexpr int G = 256 / COUT;               // threads per output channel
    constexpr int NJ = (CIN + G - 1) / G;       // input channels per thread
    constexpr int ROWS = TAPS == 9 ? 3 : 1;
    constexpr int HALO = TAPS == 9 ? 1 : 0;
    constexpr int AW = kRun + 2 * HALO;
    __shared__ float sg[kRun * COUT];
    __shared__ float sa[ROWS * AW * CIN];
    const int t = threadIdx.x;
    const int o = t % COUT, w = t / COUT;
    float acc[TAPS][NJ];
#pragma unroll
    for (int k = 0; k < TAPS; ++k)
#pragma unroll
        for (int j = 0; j < NJ; ++j) acc[k][j] = 0.f;
    float bacc = 0.f;
    const long long nrun = d.npts / kRun;
    for (long long run = blockIdx.x; run < nrun; run += gridDim.x) {
        const long long p0 = run * kRun;
        __syncthreads();
        for (int i = t; i < kRun * COUT; i += 256) sg[i] = g[p0 * COUT + i];
        for (int i = t; i < ROWS * AW * CIN; i += 256) {
            const int c = i % CIN, xx = (i / CIN) % AW, rr = i / (CIN * AW);
            sa[i] = a[nbr(d, p0, rr - HALO, xx - HALO) * CIN + c];
        }
        __syncthreads();
        if (w < CIN) {
            for (int pp = 0; pp < kRun; ++pp) {
                const float gv = sg[pp * COUT + o];
                const float* ar = sa + pp * CIN + w;
#pragma unroll
                for (int k = 0; k < TAPS; ++k) {
                    const int dy = TAPS == 9 ? k / 3 : 0, dx = TAPS == 9 ? k % 3 : 0;
#pragma unroll
                    for (int j = 0; j < NJ; ++j)
                        if (w + j * G < CIN) acc[k][j] = fmaf(gv, ar[(dy * AW + dx) * CIN + j * G], acc[k][j]);
                }
            }
        }
        if (t < COUT) {
            float s = 0.f;
            for (int pp = 0; pp < kRun; ++pp) s += sg[pp * COUT + t];
            bacc += s;
        }
    }
    float* out = part + (size_t)blockIdx.x * (NP + COUT);
#pragma unroll
    for (int k = 0; k < TAPS; ++k)
#pragma unroll
        for (int j = 0; j < NJ; ++j) {
            const int c = w + j * G;
            if (c < CIN) out[(k * CIN + c) * COUT + o] = acc[k][j];
        }
    if (t < COUT) out[NP + t] = bacc;
}

// sum the partials over workgroups (fixed order, FP64) into the gradient
// vector at the layer's offsets (weights [o][t][c], biases [o])
__global__ void k_tr_reduce(const float* __restrict__ part, int nblk, int taps, int cin, int cout,
                            float* __restrict__ gw, float* __restrict__ gb) {
    const int np = taps * cin * cout;
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= np + cout) return;
    double s = 0.0;
    for (int b = 0; b < nblk; ++b) s += (double)part[(size_t)b * (np + cout) + i];
    if (i < np) {
        const int o = i % cout, tc = i / cout;
        gw[o * taps * cin + tc] = (float)s;
    } else {
        gb[i - np] = (float)s;
    }
}

__device__ __forceinline__ bool is_bias(int i) {
    return (i >= kOffB1 && i < kOffW2) || (i >= kOffB2 && i < kOffW3) || (i >= kOffB3 && i < kOffW4) ||
           i >= kOffB4;
}

__global__ void k_tr_adam(float* theta, float* m, float* v, const float* g, float* wq, float lr, float b1,
                          float b2, float eps, float bc1, float bc2) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= kNetParams) return;
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.0f - b1) * gi;
    const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    const float th = theta[i] - lr * (mi / bc1) / (sqrtf(vi / bc2) + eps);
    theta[i] = th;
    wq[i] = is_bias(i) ? th : bf16_round(th);
}

__global__ void k_tr_round(const float* theta, float* wq) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= kNetParams) return;
    wq[i] = is_bias(i) ? theta[i] : bf16_round(theta[i]);
}

// ---------------------------------------------------------------------------
// host launchers
// ---------------------------------------------------------------------------
int tr_loss_blocks(const TrainDims& d) { return (int)((d.npts + 255) / 256); }
size_t tr_part_floats(int nblk) { return (size_t)nblk * (9 * 32 * 32 + 32); }

hipError_t tr_forward(const TrainDims& d, const TrainBuffers& b, const float* feat, const float* target,
                      hipStream_t s) {
    const dim3 grid((unsigned)tr_loss_blocks(d)), block(256);
    hipLaunchKernelGGL(k_tr_conv3<8>, grid, block, 0, s, feat, b.wq + kOffW1, b.wq + kOffB1, b.z1, b.a1, d);
    hipLaunchKernelGGL(k_tr_conv3<32>, grid, block, 0, s, b.a1, b.wq + kOffW2, b.wq + kOffB2, b.z2, b.a2, d);
    hipLaunchKernelGGL(k_tr_head, grid, block, 0, s, b.a2, b.wq, target, b.z3, b.a3, b.y, b.gy, b.lpart, d);
    return hipGetLastError();
}

template <int TAPS, int CIN, int COUT>
static void wgrad(const TrainDims& d, const TrainBuffers& b, const float* g, const float* a, int off_w, int off_b,
                  hipStream_t s) {
    hipLaunchKernelGGL((k_tr_wgrad<TAPS, CIN, COUT>), dim3(b.nblk), dim3(256), 0, s, g, a, b.part, d);
    const int n = TAPS * CIN * COUT + COUT;
    hipLaunchKernelGGL(k_tr_reduce, dim3((n + 255) / 256), dim3(256), 0, s, (const float*)b.part, b.nblk, TAPS, CIN,
                       COUT, b.grad + off_w, b.grad + off_b);
}

hipError_t tr_backward(const TrainDims& d, const TrainBuffers& b, const float* feat, hipStream_t s) {
    if (d.nx % kRun) return hipErrorInvalidValue;
    const dim3 grid((unsigned)tr_loss_blocks(d)), block(256);
    hipLaunchKernelGGL(k_tr_head_bwd, grid, block, 0, s, (const float*)b.gy, (const float*)b.z3,
                       (const float*)b.z2, b.wq, b.g3, b.g2, d);
    wgrad<1, 32, 2>(d, b, b.gy, b.a3, kOffW4, kOffB4, s);
    wgrad<1, 32, 32>(d, b, b.g3, b.a2, kOffW3, kOffB3, s);
    wgrad<9, 32, 32>(d, b, b.g2, b.a1, kOffW2, kOffB2, s);
    hipLaunchKernelGGL(k_tr_conv3_bwd, grid, block, 0, s, (const float*)b.g2, b.wq, (const float*)b.z1, b.g1, d);
    wgrad<9, 8, 32>(d, b, b.g1, feat, kOffW1, kOffB1, s);
    return hipGetLastError();
}

hipError_t tr_adam(float* theta, float* m, float* v, const float* g, float* wq, float lr, float beta1,
                   float beta2, float eps, float bc1, float bc2, hipStream_t s) {
    hipLaunchKernelGGL(k_tr_adam, dim3((kNetParams + 255) / 256), dim3(256), 0, s, theta, m, v, g, wq, lr, beta1,
                       beta2, eps, bc1, bc2);
    return hipGetLastError();
}

hipError_t tr_round_weights(const float* theta, float* wq, hipStream_t s) {
    hipLaunchKernelGGL(k_tr_round, dim3((kNetParams + 255) / 256), dim3(256), 0, s, theta, wq);
    return hipGetLastError();
}

}  // namespace sbi
