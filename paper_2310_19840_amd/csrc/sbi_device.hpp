// sbi_device.hpp -- device helpers shared by the kernel sources: order-
// preserving bit keys of doubles, block-wide maxima of 64-bit keys, and the
// decision rule of an iterated W solve.
#pragma once
#include <hip/hip_runtime.h>

#include "sbi_internal.hpp"

namespace sbi {

__device__ __forceinline__ unsigned long long ord_bits(double x) {
    unsigned long long b = (unsigned long long)__double_as_longlong(x);
    return (b >> 63) ? ~b : (b | 0x8000000000000000ull);
}
__device__ __forceinline__ double unord_bits(unsigned long long o) {
    unsigned long long b = (o >> 63) ? (o & 0x7fffffffffffffffull) : ~o;
    return __longlong_as_double((long long)b);
}
__device__ __forceinline__ unsigned long long abs_bits(double x) {
    return (unsigned long long)__double_as_longlong(fabs(x));
}
__device__ __forceinline__ double bits_to_double(unsigned long long b) {
    return __longlong_as_double((long long)b);
}
// Block-wide max/min of 64-bit keys (order-independent, so every block size
// and schedule gives the same bits).  Whole wavefronts reduce by lane
// exchanges and meet in one LDS slot per wavefront; blocks that are not a
// whole number of wavefronts (narrow grids, at most 256 threads) fold
// through LDS.  Every thread must call it.
template <bool MAX>
__device__ __forceinline__ unsigned long long block_reduce_u64(unsigned long long v) {
    __shared__ unsigned long long red[256];
    const int t = threadIdx.x;
    const int n = blockDim.x;
    auto pick = [](unsigned long long a, unsigned long long b) { return MAX ? (a > b ? a : b) : (a < b ? a : b); };
    __syncthreads();  // a previous call's readers are done with red
    if (n % 64 == 0) {
#pragma unroll
        for (int off = 32; off >= 1; off >>= 1) v = pick(v, __shfl_xor(v, off, 64));
        if ((t & 63) == 0) red[t >> 6] = v;
        __syncthreads();
        unsigned long long r = red[0];
        for (int w = 1; w < n / 64; ++w) r = pick(r, red[w]);
        return r;
    }
    red[t] = v;
    __syncthreads();
    for (int s = 1; s < n; s <<= 1) {
        if ((t & (2 * s - 1)) == 0 && t + s < n) red[t] = pick(red[t], red[t + s]);
        __syncthreads();
    }
    return red[0];
}

// Block-wide maxima of two 64-bit keys at once (one pair of barriers); the
// same contract as block_reduce_u64.
__device__ __forceinline__ void block_reduce2_max_u64(unsigned long long& a, unsigned long long& b) {
    __shared__ unsigned long long red2[2][16];
    const int t = threadIdx.x;
    const int n = blockDim.x;
    if (n % 64 != 0) {
        a = block_reduce_u64<true>(a);
        b = block_reduce_u64<true>(b);
        return;
    }
    auto mx = [](unsigned long long x, unsigned long long y) { return x > y ? x : y; };
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
        a = mx(a, __shfl_xor(a, off, 64));
        b = mx(b, __shfl_xor(b, off, 64));
    }
    __syncthreads();  // a previous call's readers are done with red2
    if ((t & 63) == 0) {
        red2[0][t >> 6] = a;
        red2[1][t >> 6] = b;
    }
    __syncthreads();
    a = red2[0][0];
    b = red2[1][0];
    for (int w = 1; w < n / 64; ++w) {
        a = mx(a, red2[0][w]);
        b = mx(b, red2[1][w]);
    }
}

// record the end of a member's solve: status, sweeps, last residual, and the
// totals of the captured-run statistics
__device__ __forceinline__ void ctl_commit(Ctl* ctl, int st, int sweeps, double r) {
    ctl->status = st;
    ctl->sweeps = sweeps;
    ctl->residual = r;
    ctl->done = 1;
    ctl->acc_solves += 1;
    ctl->acc_sweeps += sweeps;
    ctl->acc_sweeps_max = max(ctl->acc_sweeps_max, sweeps);
    ctl->acc_residual_max = fmax(ctl->acc_residual_max, r);
    const int w = ctl->acc_worst;
    if (st < 0 ? (w >= 0 || st < w) : (w >= 0 && st > w)) ctl->acc_worst = st;
}

// decision of a sweep pass from the completed residual of the previous sweep.
// returns 0 to continue, else the terminating sbi_status + 100 (so 0 is free).
__device__ __forceinline__ int sweep_decision(Ctl* ctl, int n, int M, double tol, double* r_out, double* rmin_out) {
    *r_out = 0.0;
    *rmin_out = ctl->rmin;
    if (n == 0) return 0;
    const double num = bits_to_double(ctl->slots->num[n - 1]);
    const double den = bits_to_double(ctl->slots->den[n - 1]);
    if (!isfinite(num) || !isfinite(den)) {
        *r_out = __longlong_as_double(0x7ff8000000000000ll);
        return 100 - 5;  // SBI_ERR_NONFINITE
    }
    const double r = (num == 0.0) ? 0.0 : (den > 0.0 ? num / den : INFINITY);
    *r_out = r;
    if (r <= tol) return 100;  // converged: SBI_OK
    double rmin = fmin(ctl->rmin, r);
    *rmin_out = rmin;
    if (r > 1e6 || ((n - 1) >= 3 && r > 10.0 * rmin)) return 100 - 6;  // SBI_ERR_DIVERGED
    if (n >= M) return 100 + 1;                                        // SBI_WARN_NOT_CONVERGED
    return 0;
}

}  // namespace sbi
