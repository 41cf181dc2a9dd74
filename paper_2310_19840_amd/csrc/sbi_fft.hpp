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

// Workgroup barrier that orders LDS only: outstanding global loads (prefetch)
// stay in flight across it.
__device__ __forceinline__ void lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}
// LDS exchange among the lanes of one wavefront: a wave's LDS operations
// complete in order, so ordering the wave's own accesses is enough when every
// thread of a transform sits in the same wavefront
__device__ __forceinline__ void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront", "local");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront", "local");
}
template <bool WAVE> __device__ __forceinline__ void xfer_sync() {
    if constexpr (WAVE)
        wave_lds_sync();
    else
        lds_sync();
}

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

// a * W16^e, W16 = exp(-i pi/8) forward, exp(+i pi/8) inverse, given
// c = cos(pi e/8) and s = sin(pi e/8)
template <bool INV, typename V> __device__ __forceinline__ V rot16(V a, decltype(V::x) c, decltype(V::x) s) {
    return INV ? cx<V>(a.x * c - a.y * s, a.y * c + a.x * s) : cx<V>(a.x * c + a.y * s, a.y * c - a.x * s);
}

// 16 points as 4 x 4: DFTs of length 4 over the stride-4 subsequences, the
// twiddles W16^(n2 k1), then DFTs of length 4 across them; output in natural
// order.
template <bool INV, typename V> struct Dft<16, INV, V> {
    static __device__ __forceinline__ void run(V* a) {
        using T = decltype(V::x);
        const T c1 = T(0.92387953251128675612818318939678828682);  // cos(pi/8)
        const T s1 = T(0.38268343236508977172845998403039886676);  // sin(pi/8)
        const T r2 = T(0.70710678118654752440084436210484903928);
        V y[4][4];
#pragma unroll
        for (int n2 = 0; n2 < 4; ++n2) {
#pragma unroll
            for (int n1 = 0; n1 < 4; ++n1) y[n2][n1] = a[n2 + 4 * n1];
            Dft<4, INV, V>::run(y[n2]);
        }
        y[1][1] = rot16<INV>(y[1][1], c1, s1);
        y[1][2] = rot16<INV>(y[1][2], r2, r2);
        y[1][3] = rot16<INV>(y[1][3], s1, c1);
        y[2][1] = rot16<INV>(y[2][1], r2, r2);
        y[2][2] = mul_mi<INV>(y[2][2]);
        y[2][3] = rot16<INV>(y[2][3], -r2, r2);
        y[3][1] = rot16<INV>(y[3][1], s1, c1);
        y[3][2] = rot16<INV>(y[3][2], -r2, r2);
        y[3][3] = rot16<INV>(y[3][3], -c1, -s1);
#pragma unroll
        for (int k1 = 0; k1 < 4; ++k1) {
            V z[4] = {y[0][k1], y[1][k1], y[2][k1], y[3][k1]};
            Dft<4, INV, V>::run(z);
#pragma unroll
            for (int k2 = 0; k2 < 4; ++k2) a[k1 + 4 * k2] = z[k2];
        }
    }
};

__host__ __device__ constexpr int cmin(int a, int b) { return a < b ? a : b; }

// Elements per thread for a length-N transform (at most EMAX, a power of two
// in {2, 4, 8, 16}).
template <int N, int EMAX = 8> struct FftShape {
    static constexpr int E = N >= EMAX ? EMAX : N;
    static constexpr int P = N / E;
};

// Pass sequence of a length-N transform with E elements per thread: radix
// R_i = min(E, N / Ns_i), Ns_0 = 1, Ns_(i+1) = Ns_i R_i.  Passes with Ns > 1
// need one base twiddle per butterfly (E / R per thread); TwCount/TwOffset
// size and index the per-thread twiddle cache.
template <int N, int E, int Ns> struct PassInfo {
    static constexpr int REM = N / Ns;
    static constexpr int R = REM >= E ? E : REM;
    static constexpr bool LAST = (Ns * R == N);
    static constexpr int B = E / R;
    static constexpr int NEED = (Ns > 1) ? B : 0;
    static constexpr int NEXT = Ns * R;
};
template <int N, int E, int Ns, bool DONE = (Ns >= N)> struct TwCountFrom {
    static constexpr int value = PassInfo<N, E, Ns>::NEED + TwCountFrom<N, E, PassInfo<N, E, Ns>::NEXT>::value;
};
template <int N, int E, int Ns> struct TwCountFrom<N, E, Ns, true> {
    static constexpr int value = 0;
};
// offset of pass Ns in the cache = twiddles of all earlier passes
template <int N, int E, int Ns, int Cur = 1, bool AT = (Cur == Ns)> struct TwOffset {
    static constexpr int value = PassInfo<N, E, Cur>::NEED + TwOffset<N, E, Ns, PassInfo<N, E, Cur>::NEXT>::value;
};
template <int N, int E, int Ns, int Cur> struct TwOffset<N, E, Ns, Cur, true> {
    static constexpr int value = 0;
};

// Per-thread twiddle cache: the base twiddles of every pass for thread j,
// loaded once and reused by every transform of the same length.
template <typename V, int N, int E> struct Twid {
    static constexpr bool ALL = false;
    static constexpr int NT = TwCountFrom<N, E, 1>::value;
    V w[NT > 0 ? NT : 1];
    // tw: table of exp(-2 pi i m / (N stride)), read at every stride-th entry
    template <int Ns> __device__ __forceinline__ void load_from(const V* __restrict__ tw, int j, int stride) {
        if constexpr (Ns < N) {
            using PI = PassInfo<N, E, Ns>;
            if constexpr (Ns > 1) {
                constexpr int off = TwOffset<N, E, Ns>::value;
                constexpr int P = N / E;
#pragma unroll
                for (int s = 0; s < PI::B; ++s) {
                    const int b = j + s * P;
                    const int k = b & (Ns - 1);
                    w[off + s] = tw[stride * k * (N / (Ns * PI::R))];
                }
            }
            load_from<PI::NEXT>(tw, j, stride);
        }
    }
    __device__ __forceinline__ void load(const V* __restrict__ tw, int j, int stride = 1) { load_from<1>(tw, j, stride); }
};

// Per-thread cache of every twiddle power a pass uses: for each butterfly of
// each pass with Ns > 1, the R - 1 powers w^1 .. w^(R-1) of its base twiddle,
// read from the table rather than formed by recurrence.  It takes R - 1 times
// the registers of Twid and saves the R - 2 complex products per butterfly
// that the recurrence spends; a launch plan chooses between the two.
template <int N, int E, int Ns, bool DONE = (Ns >= N)> struct TwAllCountFrom {
    using PI = PassInfo<N, E, Ns>;
    static constexpr int value = (Ns > 1 ? PI::B * (PI::R - 1) : 0) + TwAllCountFrom<N, E, PI::NEXT>::value;
};
template <int N, int E, int Ns> struct TwAllCountFrom<N, E, Ns, true> {
    static constexpr int value = 0;
};
template <int N, int E, int Ns, int Cur = 1, bool AT = (Cur == Ns)> struct TwAllOffset {
    using PI = PassInfo<N, E, Cur>;
    static constexpr int value = (Cur > 1 ? PI::B * (PI::R - 1) : 0) + TwAllOffset<N, E, Ns, PI::NEXT>::value;
};
template <int N, int E, int Ns, int Cur> struct TwAllOffset<N, E, Ns, Cur, true> {
    static constexpr int value = 0;
};
template <typename V, int N, int E> struct TwidAll {
    static constexpr bool ALL = true;
    static constexpr int NT = TwAllCountFrom<N, E, 1>::value;
    V w[NT > 0 ? NT : 1];
    template <int Ns> __device__ __forceinline__ void load_from(const V* __restrict__ tw, int j, int stride) {
        if constexpr (Ns < N) {
            using PI = PassInfo<N, E, Ns>;
            if constexpr (Ns > 1) {
                constexpr int off = TwAllOffset<N, E, Ns>::value;
                constexpr int P = N / E;
#pragma unroll
                for (int s = 0; s < PI::B; ++s) {
                    const int k = (j + s * P) & (Ns - 1);
                    // r k < R Ns, so the index stays inside the length-N table
#pragma unroll
                    for (int r = 1; r < PI::R; ++r) w[off + s * (PI::R - 1) + r - 1] = tw[stride * r * k * (N / (Ns * PI::R))];
                }
            }
            load_from<PI::NEXT>(tw, j, stride);
        }
    }
    __device__ __forceinline__ void load(const V* __restrict__ tw, int j, int stride = 1) { load_from<1>(tw, j, stride); }
};

// LDS slot of transform element idx: the first Stockham pass writes with a
// stride of E elements (E x 16 B in FP64), which folds a wavefront onto a few
// LDS banks; one pad slot per E elements spreads every pass over all banks.
template <int E> __device__ __forceinline__ int lds_slot(int idx) { return E >= 2 ? idx + idx / E : idx; }
// LDS elements one transform of length N with E elements per thread needs
template <int N, int E> __host__ __device__ constexpr int fft_lds_elems() { return E >= 2 ? N + N / E : N; }

// One Stockham pass of radix R with current span Ns (product of earlier radices).
// WAVE: all threads of the transform are in one wavefront (exchanges need no
// workgroup barrier).
template <typename V, int N, int E, int R, int Ns, bool INV, bool LAST, int LS, bool WAVE, typename TW>
__device__ __forceinline__ void stockham_pass(V (&v)[E], V* lds, int lo, int j, const TW& tw) {
    constexpr int P = N / E;
    constexpr int B = E / R;
#pragma unroll
    for (int s = 0; s < B; ++s) {
        const int b = j + s * P;
        const int k = b & (Ns - 1);
        V u[R];
#pragma unroll
        for (int r = 0; r < R; ++r) u[r] = v[s + r * B];
        if constexpr (Ns > 1 && TW::ALL) {
            // every power from the cache
            constexpr int off = TwAllOffset<N, E, Ns>::value;
#pragma unroll
            for (int r = 1; r < R; ++r) {
                V wr = tw.w[off + s * (R - 1) + r - 1];
                if (INV) wr.y = -wr.y;
                u[r] = cmul(u[r], wr);
            }
        } else if constexpr (Ns > 1) {
            // base twiddle from the cache; higher powers by recurrence
            V w1 = tw.w[TwOffset<N, E, Ns>::value + s];
            if constexpr (E >= 8) {
                // the powers of every pass (up to 15 in a radix-16 pass) would
                // otherwise be hoisted out of the caller's loops and held in
                // registers for the whole kernel
                asm volatile("" : "+v"(w1.x), "+v"(w1.y));
            }
            if (INV) w1.y = -w1.y;
            V wr = w1;
            u[1] = cmul(u[1], w1);
#pragma unroll
            for (int r = 2; r < R; ++r) {
                wr = cmul(wr, w1);
                u[r] = cmul(u[r], wr);
            }
        }
        Dft<R, INV, V>::run(u);
        if (LAST) {
#pragma unroll
            for (int r = 0; r < R; ++r) v[s + r * B] = u[r];
        } else {
            const int base = (b - k) * R + k;
#pragma unroll
            for (int r = 0; r < R; ++r) lds[lds_slot<E>(base + r * Ns) * LS + lo] = u[r];
        }
    }
    if (!LAST) {
        xfer_sync<WAVE>();
#pragma unroll
        for (int q = 0; q < E; ++q) v[q] = lds[lds_slot<E>(j + q * P) * LS + lo];
        xfer_sync<WAVE>();
    }
}

template <typename V, int N, int E, int Ns, bool INV, int LS, bool WAVE>
struct StockhamRun {
    using PI = PassInfo<N, E, Ns>;
    template <typename TW>
    static __device__ __forceinline__ void run(V (&v)[E], V* lds, int lo, int j, const TW& tw) {
        stockham_pass<V, N, E, PI::R, Ns, INV, PI::LAST, LS, WAVE>(v, lds, lo, j, tw);
        if constexpr (!PI::LAST) StockhamRun<V, N, E, PI::NEXT, INV, LS, WAVE>::run(v, lds, lo, j, tw);
    }
};

// Full transform.  All threads of the workgroup must call it (it synchronises;
// with WAVE only the wavefront holding the transform does).  On return every
// thread of the transform has passed the last read of its exchange area only
// when WAVE is false.
template <typename V, int N, bool INV, int LS, int EMAX = 8, bool WAVE = false, typename TW>
__device__ __forceinline__ void fft(V (&v)[(FftShape<N, EMAX>::E)], V* lds, int lo, int j, const TW& tw) {
    if constexpr (N > 1) StockhamRun<V, N, FftShape<N, EMAX>::E, 1, INV, LS, WAVE>::run(v, lds, lo, j, tw);
}

}  // namespace sbi
