// sbi_fft.hpp -- register/LDS Stockham FFT building blocks for gfx950.
//
// A length-N complex transform is carried by P = N/E threads that each hold E
// elements in registers; thread j holds x[j + q*P] in v[q].  Every radix-R
// pass performs E/R butterflies per thread and exchanges through LDS; the last
// pass leaves y[j + q*P] in v[q] again, so the first pass reads coalesced and
// the last pass writes coalesced.  Forward uses exp(-2 pi i/N) (unnormalised),
// inverse exp(+2 pi i/N) (unscaled; callers apply 1/N).
//
// LDS addressing is lds[idx * LS + lo]: LS = 1 for a row held contiguously,
// LS = C for C interleaved columns (lo = column within the tile) so that
// consecutive threads touch consecutive LDS words.
#pragma once
#include <hip/hip_runtime.h>

namespace sbi {

template <typename R> struct cplx_of;
template <> struct cplx_of<double> { using type = double2; };
template <> struct cplx_of<float> { using type = float2; };

template <typename V> __device__ __forceinline__ V cx(decltype(V::x) a, decltype(V::x) b) { V r; r.x = a; r.y = b; return r; }
template <typename V> __device__ __forceinline__ V operator_add(V a, V b) { return cx<V>(a.x + b.x, a.y + b.y); }

template <typename V> __device__ __forceinline__ V cadd(V a, V b) { return cx<V>(a.x + b.x, a.y + b.y); }
template <typename V> __device__ __forceinline__ V csub(V a, V b) { return cx<V>(a.x - b.x, a.y - b.y); }
template <typename V> __device__ __forceinline__ V cmul(V a, V b) {
    return cx<V>(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
template <typename V> __device__ __forceinline__ V cconj(V a) { return cx<V>(a.x, -a.y); }
template <typename V> __device__ __forceinline__ V cscale(V a, decltype(V::x) s) { return cx<V>(a.x * s, a.y * s); }
// multiply by -i (forward) or +i (inverse)
template <bool INV, typename V> __device__ __forceinline__ V mul_mi(V a) {
    return INV ? cx<V>(-a.y, a.x) : cx<V>(a.y, -a.x);
}
template <typename V> __device__ __forceinline__ V mul_i(V a) { return cx<V>(-a.y, a.x); }

template <int R, bool INV, typename V> struct Dft;

template <bool INV, typename V> struct Dft<1, INV, V> {
    static __device__ __forceinline__ void run(V*) {}
};

template <bool INV, typename V> struct Dft<2, INV, V> {
    static __device__ __forceinline__ void run(V* a) {
        V t = a[0];
        a[0] = cadd(t, a[1]);
        a[1] = csub(t, a[1]);
    }
};

template <bool INV, typename V> struct Dft<4, INV, V> {
    static __device__ __forceinline__ void run(V* a) {
        V s02 = cadd(a[0], a[2]), d02 = csub(a[0], a[2]);
        V s13 = cadd(a[1], a[3]), d13 = mul_mi<INV>(csub(a[1], a[3]));
        a[0] = cadd(s02, s13);
        a[2] = csub(s02, s13);
        a[1] = cadd(d02, d13);
        a[3] = csub(d02, d13);
    }
};

template <bool INV, typename V> struct Dft<8, INV, V> {
    static __device__ __forceinline__ void run(V* a) {
        using T = decltype(V::x);
        const T r2 = T(0.70710678118654752440084436210484903928);
        V e[4] = {a[0], a[2], a[4], a[6]};
        V o[4] = {a[1], a[3], a[5], a[7]};
        Dft<4, INV, V>::run(e);
        Dft<4, INV, V>::run(o);
        // twiddles W8^k, W8 = exp(-i pi/4) forward, exp(+i pi/4) inverse
        V o1, o3;
        if (INV) {
            o1 = cx<V>((o[1].x - o[1].y) * r2, (o[1].x + o[1].y) * r2);
            o3 = cx<V>((-o[3].x - o[3].y) * r2, (o[3].x - o[3].y) * r2);
        } else {
            o1 = cx<V>((o[1].x + o[1].y) * r2, (o[1].y - o[1].x) * r2);
            o3 = cx<V>((o[3].y - o[3].x) * r2, (-o[3].x - o[3].y) * r2);
        }
        V o2 = mul_mi<INV>(o[2]);
        a[0] = cadd(e[0], o[0]);
        a[4] = csub(e[0], o[0]);
        a[1] = cadd(e[1], o1);
        a[5] = csub(e[1], o1);
        a[2] = cadd(e[2], o2);
        a[6] = csub(e[2], o2);
        a[3] = cadd(e[3], o3);
        a[7] = csub(e[3], o3);
    }
};

__host__ __device__ constexpr int cmin(int a, int b) { return a < b ? a : b; }

// Elements per thread for a length-N transform.
template <int N> struct FftShape {
    static constexpr int E = N >= 8 ? 8 : N;
    static constexpr int P = N / E;
};

// One Stockham pass of radix R with current span Ns (product of earlier radices).
// tw: table of length N with tw[m] = exp(-2 pi i m / N) (host FP64 values).
template <typename V, int N, int E, int R, int Ns, bool INV, bool LAST, int LS>
__device__ __forceinline__ void stockham_pass(V (&v)[E], V* lds, int lo, int j, const V* __restrict__ tw) {
    constexpr int P = N / E;
    constexpr int B = E / R;
#pragma unroll
    for (int s = 0; s < B; ++s) {
        const int b = j + s * P;
        const int k = b & (Ns - 1);
        V u[R];
#pragma unroll
        for (int r = 0; r < R; ++r) u[r] = v[s + r * B];
        if (Ns > 1) {
#pragma unroll
            for (int r = 1; r < R; ++r) {
                V w = tw[(r * k) * (N / (Ns * R))];
                if (INV) w.y = -w.y;
                u[r] = cmul(u[r], w);
            }
        }
        Dft<R, INV, V>::run(u);
        if (LAST) {
#pragma unroll
            for (int r = 0; r < R; ++r) v[s + r * B] = u[r];
        } else {
            const int base = (b - k) * R + k;
#pragma unroll
            for (int r = 0; r < R; ++r) lds[(base + r * Ns) * LS + lo] = u[r];
        }
    }
    if (!LAST) {
        __syncthreads();
#pragma unroll
        for (int q = 0; q < E; ++q) v[q] = lds[(j + q * P) * LS + lo];
        __syncthreads();
    }
}

template <typename V, int N, int E, int Ns, bool INV, int LS>
struct StockhamRun {
    static constexpr int REM = N / Ns;
    static constexpr int R = REM >= E ? E : REM;
    static constexpr bool LAST = (Ns * R == N);
    static __device__ __forceinline__ void run(V (&v)[E], V* lds, int lo, int j, const V* __restrict__ tw) {
        stockham_pass<V, N, E, R, Ns, INV, LAST, LS>(v, lds, lo, j, tw);
        if constexpr (!LAST) StockhamRun<V, N, E, Ns * R, INV, LS>::run(v, lds, lo, j, tw);
    }
};

// Full transform.  All threads of the workgroup must call it (it synchronises).
template <typename V, int N, bool INV, int LS>
__device__ __forceinline__ void fft(V (&v)[FftShape<N>::E], V* lds, int lo, int j, const V* __restrict__ tw) {
    if constexpr (N > 1) StockhamRun<V, N, FftShape<N>::E, 1, INV, LS>::run(v, lds, lo, j, tw);
}

}  // namespace sbi
