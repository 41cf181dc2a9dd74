// sbi_kernels.hip -- gfx950 kernels of the SBI wave solver.
//
// Every 2D transform is split into a row pass (real <-> half form, one row per
// group of P threads, half-length complex FFT plus the standard real/complex
// twist) and a column pass (C adjacent columns per workgroup, length-ny complex
// FFT).  The products of the method (eta^j V, delta^j grad phi_b, ...) are
// formed in registers inside the row pass; the Fourier multipliers of the
// method (k^j/j! tanh(kh), sech(kh), i k, ...) are applied and summed inside
// the column pass, which then runs the inverse column transforms of the new
// iterate directly from registers.  Only kept modes are ever written, so the
// spectra in memory are 1/4 (2D) of the full size.
#include <math.h>
#include <type_traits>
#include "sbi_device.hpp"
#include "sbi_fft.hpp"
#include "sbi_kernels.hpp"

#ifndef SBI_REAL
#error "compile with -DSBI_REAL=double or -DSBI_REAL=float"
#endif

namespace sbi {

// ---------------------------------------------------------------------------
// small helpers
// ---------------------------------------------------------------------------

__device__ __forceinline__ double sech_d(double x) {
    double e = exp(-fabs(x));
    return 2.0 * e / (1.0 + e * e);
}

template <typename V> __device__ __forceinline__ V rmul(V a, V b) {  // componentwise real product
    return cx<V>(a.x * b.x, a.y * b.y);
}

// ---------------------------------------------------------------------------
// Row pass helpers: real row of length NX <-> kept half spectrum F[0..Mx]
// via the length-NX/2 complex transform of z[n] = f[2n] + i f[2n+1].
// ---------------------------------------------------------------------------
// Per-thread view of a row-pass workgroup: rpw rows of P threads each.
struct RowCtx {
    int t, nthr, j, rl, y0, rpw, rsh, ny, ldh, Mx, mem;  // rpw = 1 << rsh rows per workgroup
    bool valid;
};

// LDS pitch of a row (elements): room for the padded transform, rounded up so
// that consecutive rows start 16 banks apart -- the staging loops read and
// write (row, mode) with the row index fastest, and a quarter wave of 16-byte
// (half wave of 8-byte) accesses then covers distinct banks
constexpr int row_pitch(int e0, int vbytes) {
    const int unit = 256 / vbytes, want = 64 / vbytes;
    int ls = e0;
    while (ls % unit != want) ++ls;
    return ls;
}

// EM: elements per thread of the row transform (its radix sequence: 8 gives
// radix-8 passes, 16 radix-16 ones); TWC: every twiddle power held in
// registers instead of formed by recurrence.  Both are launch-plan choices.
template <typename R, int NX, int EM = 8, bool TWC = false> struct Row {
    using V = typename cplx_of<R>::type;
    static constexpr int N = NX / 2;
    static constexpr int E = FftShape<N, EM>::E;
    static constexpr int P = FftShape<N, EM>::P;
    static constexpr int LS = row_pitch(fft_lds_elems<N, E>(), (int)sizeof(V));
    // a row of up to 64 threads lies in one wavefront: its transform's LDS
    // exchanges need only wave-level ordering
    static constexpr bool WAVE = P <= 64;

    // v <- z = inverse row transform of (G + c2 G2) for the thread's row.
    // G, G2: member base of a half form [m_x][ny]; all rows of the workgroup
    // stage their kept spectra through LDS with coalesced column segments.
    // z[n] = f[2n] + i f[2n+1] has Z[m] = (F[m] + conj F[N-m]) / 2
    //   + i (F[m] - conj F[N-m]) / 2 * exp(+2 pi i m / NX).
    using TW = typename std::conditional<TWC, TwidAll<V, N, E>, Twid<V, N, E>>::type;
    static __device__ __forceinline__ void inverse(V (&v)[E], const V* __restrict__ G, const V* __restrict__ G2,
                                                   R c2, const RowCtx& rc, V* lds_all,
                                                   const TW& twN, const V* __restrict__ twX, R scale) {
        V* lds = lds_all + rc.rl * LS;
        lds_sync();  // other rows' transforms are done with the area the staging loop writes
        // a thread stages modes k0, k0 + kstep, ... of row r2 of the workgroup
        // (the block is a whole number of rows, and ny a multiple of rpw)
        const int r2 = rc.t & (rc.rpw - 1);
        const int k0 = rc.t >> rc.rsh, kstep = rc.nthr >> rc.rsh;
        V* const zr = lds_all + r2 * LS;
        const V* const Gr = G + rc.y0 + r2;
        const V* const G2r = G2 ? G2 + rc.y0 + r2 : nullptr;
        if (2 * rc.Mx < N) {
            // kept band below N/2: F[k] alone gives Z[k] and Z[N-k], Z is zero
            // between them; the staging loop writes Z directly
            const int K = rc.Mx + 1;
#pragma unroll 4
            for (int k = k0; k < K; k += kstep) {
                V f = Gr[k * rc.ldh];
                if (G2r) {
                    const V f2 = G2r[k * rc.ldh];
                    f = cx<V>(f.x + c2 * f2.x, f.y + c2 * f2.y);
                }
                const V h = cscale(f, R(0.5));
                zr[k] = cadd(h, mul_i(cmul(h, cconj(twX[k]))));
                if (k > 0) {
                    const V hc = cconj(h);
                    const V w = mul_i(cmul(hc, cconj(twX[N - k])));
                    zr[N - k] = cx<V>(hc.x - w.x, hc.y - w.y);
                }
            }
            for (int k = K + k0; k <= N - K; k += kstep) zr[k] = cx<V>(R(0), R(0));
            lds_sync();
#pragma unroll
            for (int q = 0; q < E; ++q) v[q] = lds[rc.j + q * P];
        } else {
#pragma unroll 4
            for (int m = k0; m < N; m += kstep) {
                V f = cx<V>(R(0), R(0));
                if (m <= rc.Mx) {
                    f = Gr[m * rc.ldh];
                    if (G2r) {
                        const V f2 = G2r[m * rc.ldh];
                        f = cx<V>(f.x + c2 * f2.x, f.y + c2 * f2.y);
                    }
                }
                zr[m] = f;
            }
            lds_sync();
#pragma unroll
            for (int q = 0; q < E; ++q) {
                const int m = rc.j + q * P;
                V fm = lds[m];
                V fc = (m == 0) ? cx<V>(R(0), R(0)) : cconj(lds[N - m]);
                V ev = cx<V>(R(0.5) * (fm.x + fc.x), R(0.5) * (fm.y + fc.y));
                V od = cx<V>(R(0.5) * (fm.x - fc.x), R(0.5) * (fm.y - fc.y));
                od = cmul(od, cconj(twX[m]));           // exp(+2 pi i m / NX)
                v[q] = cadd(ev, mul_i(od));
            }
        }
        xfer_sync<WAVE>();  // the row's staged values are in registers before the exchanges reuse them
        fft<V, N, true, 1, EM, WAVE>(v, lds, 0, rc.j, twN);
#pragma unroll
        for (int q = 0; q < E; ++q) v[q] = cscale(v[q], scale);
    }

    // H[kept m][row] <- forward row transform of the real pairs in v (v is
    // destroyed): F[m] = (Z[m] + conj Z[N-m]) / 2 - i (Z[m] - conj Z[N-m]) / 2
    // * exp(-2 pi i m / NX), formed by the cooperative column-segment store.
    static __device__ __forceinline__ void forward(V (&v)[E], V* __restrict__ H, const RowCtx& rc, V* lds_all,
                                                   const TW& twN, const V* __restrict__ twX) {
        V* lds = lds_all + rc.rl * LS;
        // other rows touch this row's LDS only in the staging and store loops,
        // each closed by a workgroup barrier
        fft<V, N, false, 1, EM, WAVE>(v, lds, 0, rc.j, twN);
        xfer_sync<WAVE>();  // the row's last exchange reads are done before it is overwritten
#pragma unroll
        for (int q = 0; q < E; ++q) lds[rc.j + q * P] = v[q];
        lds_sync();
        // a thread stores modes m0, m0 + mstep, ... of row r2 of the workgroup
        const int r2 = rc.t & (rc.rpw - 1);
        const V* const zr = lds_all + r2 * LS;
        V* const Hr = H + rc.y0 + r2;
        const int mstep = rc.nthr >> rc.rsh;
#pragma unroll 4
        for (int m = rc.t >> rc.rsh; m <= rc.Mx; m += mstep) {
            const V zm = zr[m];
            const V zc = cconj(zr[(N - m) & (N - 1)]);
            const V ev = cx<V>(R(0.5) * (zm.x + zc.x), R(0.5) * (zm.y + zc.y));
            const V od = mul_mi<false>(cx<V>(R(0.5) * (zm.x - zc.x), R(0.5) * (zm.y - zc.y)));
            Hr[m * rc.ldh] = cadd(ev, cmul(twX[m], od));
        }
        lds_sync();
    }

    static __device__ __forceinline__ void load(V (&v)[E], const R* __restrict__ row, int j, bool valid) {
        const V* r2 = reinterpret_cast<const V*>(row);
#pragma unroll
        for (int q = 0; q < E; ++q) v[q] = valid ? r2[j + q * P] : cx<V>(R(0), R(0));
    }
    static __device__ __forceinline__ void store(const V (&v)[E], R* __restrict__ row, int j, bool valid) {
        if (!valid) return;
        V* r2 = reinterpret_cast<V*>(row);
#pragma unroll
        for (int q = 0; q < E; ++q) r2[j + q * P] = v[q];
    }
};

// threads per row-pass workgroup: rows of P threads packed up to 256 threads
template <int NX, int EM = 8> __host__ __device__ constexpr int row_threads() {
    return FftShape<NX / 2, EM>::P > 256 ? FftShape<NX / 2, EM>::P : 256;
}

// Row transform of launch-plan variant VAR of the sweep and SA kernels:
// 0 radix-8 passes with twiddle recurrence, 1 the same with every twiddle
// power cached, 2 radix-16 passes, 3 radix-4 passes
template <typename R, int NX, int VAR> struct RowVarT {
    using type = Row<R, NX, VAR == 2 ? 16 : (VAR == 3 ? 4 : 8), VAR == 1>;
};
template <typename R, int NX, int VAR> using RowVar = typename RowVarT<R, NX, VAR>::type;

// Workgroups are dealt to the 8 XCDs round-robin by launch order, and each
// XCD has its own L2.  Neighbouring row groups read neighbouring pieces of the
// same cache lines of the column-major half forms, so they are mapped to the
// same XCD: launch index b runs row group (b % 8) * (G / 8) + b / 8.
__device__ __forceinline__ int xcd_row_group(int b, int G) {
    constexpr int kXcd = 8;
    return (G % kXcd) ? b : (b % kXcd) * (G / kXcd) + b / kXcd;
}

template <int P> __device__ __forceinline__ RowCtx row_ctx(const GridDev& g) {
    RowCtx r;
    r.t = threadIdx.x;
    r.nthr = blockDim.x;
    r.j = r.t % P;
    r.rl = r.t / P;
    r.rpw = blockDim.x / P;  // a power of two (grid sizes are)
    r.rsh = __builtin_ctz((unsigned)r.rpw);
    r.y0 = xcd_row_group(blockIdx.x, gridDim.x) * r.rpw;
    r.ny = g.ny;
    r.ldh = g.ldh;
    r.Mx = g.Mx;
    r.mem = blockIdx.z;
    r.valid = r.y0 + r.rl < g.ny;
    return r;
}

#define ROW_PROLOGUE_T(...)                                              \
    using RW = __VA_ARGS__;                                              \
    using V = typename RW::V;                                            \
    constexpr int E = RW::E;                                             \
    extern __shared__ __attribute__((aligned(16))) unsigned char smem_raw[];                          \
    const RowCtx rc = row_ctx<RW::P>(p.g);                               \
    const struct {                                                       \
        int j, mem;                                                      \
        bool valid;                                                      \
    } ri = {rc.j, rc.mem, rc.valid};                                     \
    V* lds_all = reinterpret_cast<V*>(smem_raw);                         \
    const long long hb = (long long)rc.mem * p.g.s_half;                 \
    const long long po = rc.mem * p.g.s_phys + (long long)(rc.valid ? rc.y0 + rc.rl : 0) * p.g.nx; \
    const R iscale = R(1.0 / ((double)RW::N * (double)p.g.ny));          \
    typename RW::TW twN;                                                 \
    twN.load(twN_tab, rc.j);                                             \
    /* the twist table exp(-2 pi i m / NX), m < N, staged after the rows'  \
       areas: the staging and store loops then read it from LDS (a global  \
       read there would wait behind the loop's own stores) */             \
    V* const twX = lds_all + rc.rpw * RW::LS;                            \
    for (int i_ = rc.t; i_ < RW::N; i_ += rc.nthr) twX[i_] = twX_tab[i_]; \
    (void)po; (void)iscale; (void)hb;
#define ROW_PROLOGUE(R, NX) ROW_PROLOGUE_T(Row<R, NX>)

// ---------------------------------------------------------------------------
// Row kernels
// ---------------------------------------------------------------------------
template <typename R, int NX>
__global__ void __launch_bounds__(row_threads<NX>()) k_row_fwd(const RowFwdParams p, const typename cplx_of<R>::type* twN_tab,
                          const typename cplx_of<R>::type* twX_tab) {
    ROW_PROLOGUE(R, NX)
    for (int f = 0; f < p.nf; ++f) {
        V v[E];
        RW::load(v, static_cast<const R*>(p.in[f]) + po, ri.j, ri.valid);
        RW::forward(v, static_cast<V*>(p.out[f]) + hb, rc, lds_all, twN, twX);
    }
}

template <typename R, int NX>
__global__ void __launch_bounds__(row_threads<NX>()) k_row_inv(const RowInvParams p, const typename cplx_of<R>::type* twN_tab,
                          const typename cplx_of<R>::type* twX_tab) {
    ROW_PROLOGUE(R, NX)
    for (int f = 0; f < p.nf; ++f) {
        V v[E];
        const V* g2 = p.in2[f] ? static_cast<const V*>(p.in2[f]) + hb : nullptr;
        R c2 = R(0);
        if (g2) c2 = R(1.0 - p.ctl[ri.mem].omega);
        RW::inverse(v, static_cast<const V*>(p.in[f]) + hb, g2, c2, rc, lds_all, twN, twX, iscale);
        RW::store(v, static_cast<R*>(p.out[f]) + po, ri.j, ri.valid);
    }
}

template <typename R, int NX>
__global__ void __launch_bounds__(row_threads<NX>()) k_row_setup(const RowSetupParams p, const typename cplx_of<R>::type* twN_tab,
                            const typename cplx_of<R>::type* twX_tab) {
    ROW_PROLOGUE(R, NX)
    const bool two_d = p.g.ny > 1;
    // with two families (p.nfam = 2, 2D iteration) workgroup row y = 1 takes
    // the y component: its own copy of eta, d_y phi and their products, formed
    // by the same operations as in one family
    const int fam = blockIdx.y;
    const bool want_x = fam == 0;
    const bool want_y = two_d && (p.nfam < 2 || fam == 1);
    V e[E];
    if (p.g_eta) {
        RW::inverse(e, static_cast<const V*>(p.g_eta) + hb, nullptr, R(0), rc, lds_all, twN, twX, iscale);
    } else {
        RW::load(e, static_cast<const R*>(p.eta_in) + po, ri.j, ri.valid);
    }
    int bad = 0;
    if (fam == 0) {
        if (p.eta_out) RW::store(e, static_cast<R*>(p.eta_out) + po, ri.j, ri.valid);
        // extrema of eta (relaxation weight)
        unsigned long long mx = 0ull, mn = ~0ull;
        if (ri.valid) {
#pragma unroll
            for (int q = 0; q < E; ++q) {
                unsigned long long a = ord_bits((double)e[q].x), b = ord_bits((double)e[q].y);
                mx = a > mx ? a : mx;
                mx = b > mx ? b : mx;
                mn = a < mn ? a : mn;
                mn = b < mn ? b : mn;
            }
        }
        mx = block_reduce_u64<true>(mx);
        mn = block_reduce_u64<false>(mn);
        if (threadIdx.x == 0 && p.ctl) {
            atomicMax(&p.ctl[ri.mem].eta_max, mx);
            atomicMin(&p.ctl[ri.mem].eta_min, mn);
        }
        if (ri.valid) {
#pragma unroll
            for (int q = 0; q < E; ++q) bad |= !isfinite((double)e[q].x) || !isfinite((double)e[q].y);
        }
    }
    V px[E], py[E];
    if (want_x) {
        RW::inverse(px, static_cast<const V*>(p.g_px) + hb, nullptr, R(0), rc, lds_all, twN, twX, iscale);
        if (p.px_out) RW::store(px, static_cast<R*>(p.px_out) + po, ri.j, ri.valid);
    }
    if (want_y) {
        RW::inverse(py, static_cast<const V*>(p.g_py) + hb, nullptr, R(0), rc, lds_all, twN, twX, iscale);
        if (p.py_out) RW::store(py, static_cast<R*>(p.py_out) + po, ri.j, ri.valid);
    }
    if (ri.valid) {
#pragma unroll
        for (int q = 0; q < E; ++q) {
            if (want_x) bad |= !isfinite((double)px[q].x) || !isfinite((double)px[q].y);
            if (want_y) bad |= !isfinite((double)py[q].x) || !isfinite((double)py[q].y);
        }
    }
    if (bad && p.ctl) atomicOr(&p.ctl[ri.mem].nonfinite, 1);
    if (p.nprod > 0) {
        V ep[E];
#pragma unroll
        for (int q = 0; q < E; ++q) ep[q] = e[q];
        for (int l = 2; l <= p.g.order; ++l) {
            if (l > 2) {
#pragma unroll
                for (int q = 0; q < E; ++q) ep[q] = rmul(ep[q], e[q]);
            }
            // products of order l: x at 2 (l - 2), y at 2 (l - 2) + 1 (1D: l - 2)
            const int idx = two_d ? 2 * (l - 2) : l - 2;
            V w[E];
            if (want_x) {
#pragma unroll
                for (int q = 0; q < E; ++q) w[q] = rmul(ep[q], px[q]);
                RW::forward(w, static_cast<V*>(p.h[idx]) + hb, rc, lds_all, twN, twX);
            }
            if (want_y) {
#pragma unroll
                for (int q = 0; q < E; ++q) w[q] = rmul(ep[q], py[q]);
                RW::forward(w, static_cast<V*>(p.h[idx + 1]) + hb, rc, lds_all, twN, twX);
            }
        }
    }
}

template <typename R, int NX, bool AA, int VAR>
__device__ __forceinline__ void row_sweep_body(const RowSweepParams& p, const typename cplx_of<R>::type* twN_tab,
                                               const typename cplx_of<R>::type* twX_tab) {
    Ctl* ctl = p.ctl + blockIdx.z;
    if (ctl->done) return;  // block-uniform: the member's solve is decided
    ROW_PROLOGUE_T(RowVar<R, NX, VAR>)
    const int fam = blockIdx.y;  // product family of this workgroup
    if (fam == 0) {
        V vv[E];
        // the iterate: for its products, and for the residual's denominator
        // of the relaxed update (a residual-only Anderson pass needs neither)
        if (!AA || p.products)
            RW::inverse(vv, static_cast<const V*>(p.gV) + hb, nullptr, R(0), rc, lds_all, twN, twX, iscale);
        if (p.residual) {
            V dd[E];
            RW::inverse(dd, static_cast<const V*>(p.gD) + hb, nullptr, R(0), rc, lds_all, twN, twX, iscale);
            const double c = 1.0 - ctl->omega;
            unsigned long long nu = 0ull, de = 0ull;
            if (ri.valid) {
#pragma unroll
                for (int q = 0; q < E; ++q) {
                    const double d0 = (double)dd[q].x, d1 = (double)dd[q].y;
                    unsigned long long a = abs_bits(d0), b = abs_bits(d1);
                    nu = a > nu ? a : nu;
                    nu = b > nu ? b : nu;
                    if constexpr (!AA) {
                        // denominator T(V_(n-1)) = V_n + (1 - omega) D from the relaxed update
                        a = abs_bits((double)vv[q].x + c * d0);
                        b = abs_bits((double)vv[q].y + c * d1);
                        de = a > de ? a : de;
                        de = b > de ? b : de;
                    }
                }
            }
            if constexpr (AA) {
                // denominator T(V_(n-1)) given as its own half form (in D's registers)
                RW::inverse(dd, static_cast<const V*>(p.gT) + hb, nullptr, R(0), rc, lds_all, twN, twX, iscale);
                if (ri.valid) {
#pragma unroll
                    for (int q = 0; q < E; ++q) {
                        const unsigned long long a = abs_bits((double)dd[q].x), b = abs_bits((double)dd[q].y);
                        de = a > de ? a : de;
                        de = b > de ? b : de;
                    }
                }
            }
            block_reduce2_max_u64(nu, de);
            if (threadIdx.x == 0) {
                atomicMax(&ctl->slots->num[p.slot], nu);
                atomicMax(&ctl->slots->den[p.slot], de);
            }
        }
        if (!p.products) return;
        // eta^j V as a running product (vv <- vv eta before each transform)
        V ev[E];
        RW::load(ev, static_cast<const R*>(p.eta) + po, ri.j, ri.valid);
        for (int jj = 1; jj <= p.J; ++jj) {
            V w[E];
#pragma unroll
            for (int q = 0; q < E; ++q) {
                vv[q] = rmul(vv[q], ev[q]);
                w[q] = vv[q];
            }
            RW::forward(w, static_cast<V*>(p.h[jj - 1]) + hb, rc, lds_all, twN, twX);
        }
        return;
    }
    // families 1, 2: delta^j d_x phi_b, delta^j d_y phi_b
    if (!p.products || !p.vd) return;
    const int comp = fam - 1;
    V gb[E];
    RW::inverse(gb, static_cast<const V*>(comp == 0 ? p.gbx : p.gby) + hb, nullptr, R(0), rc, lds_all, twN, twX, iscale);
    V dv[E];
    RW::load(dv, static_cast<const R*>(p.delta) + po, ri.j, ri.valid);
    for (int jj = 1; jj <= p.J; ++jj) {
        V w[E];
#pragma unroll
        for (int q = 0; q < E; ++q) {
            gb[q] = rmul(gb[q], dv[q]);  // running product delta^j d phi_b
            w[q] = gb[q];
        }
        RW::forward(w, static_cast<V*>(p.h[fam * p.J + jj - 1]) + hb, rc, lds_all, twN, twX);
    }
}

template <typename R, int NX, int VAR>
__global__ void __launch_bounds__((row_threads<NX, RowVar<R, NX, VAR>::E>()), 3)
    k_row_sweep(const RowSweepParams p, const typename cplx_of<R>::type* twN_tab,
                const typename cplx_of<R>::type* twX_tab) {
    row_sweep_body<R, NX, false, VAR>(p, twN_tab, twX_tab);
}

// the same with the residual's denominator given as a third half form (Anderson mixing)
template <typename R, int NX, int VAR>
__global__ void __launch_bounds__((row_threads<NX, RowVar<R, NX, VAR>::E>()), 3)
    k_row_sweep_aa(const RowSweepParams p, const typename cplx_of<R>::type* twN_tab,
                   const typename cplx_of<R>::type* twX_tab) {
    row_sweep_body<R, NX, true, VAR>(p, twN_tab, twX_tab);
}

template <typename R, int NX, int VAR>
__global__ void __launch_bounds__((row_threads<NX, RowVar<R, NX, VAR>::E>()))
    k_row_sa(const RowSaParams p, const typename cplx_of<R>::type* twN_tab,
             const typename cplx_of<R>::type* twX_tab) {
    ROW_PROLOGUE_T(RowVar<R, NX, VAR>)
    const int l = p.l;
    if (p.split > 0) {
        // few rows (a 1D grid, a small 2D one): each product of the order in a
        // workgroup of its own (blockIdx.y), in the order of the sequential
        // form below and formed by the same operations: eta^j V_(l-j) for
        // j < l; over a variable bed delta^j d_x phi_b,(l-j), then (2D)
        // delta^j d_y phi_b,(l-j); then eta^(l-1) d_x phi_s (and d_y phi_s)
        const int nv = l - 1;
        const int ncomp = p.g.ny > 1 ? 2 : 1;
        const int nb = p.vd ? ncomp * nv : 0;
        const int part = blockIdx.y;
        // fam 0: V; 1: bed component comp; 2: forcing component comp
        const int fam = part < nv ? 0 : (part < nv + nb ? 1 : 2);
        const int comp = fam == 1 ? (part - nv) / nv : (fam == 2 ? part - nv - nb : 0);
        V base[E], pw[E], src[E];
        RW::load(base, static_cast<const R*>(fam == 1 ? p.delta : p.eta) + po, ri.j, ri.valid);
#pragma unroll
        for (int q = 0; q < E; ++q) pw[q] = base[q];
        if (fam < 2) {
            const int jj = (fam == 0 ? part : (part - nv) % nv) + 1;
            if (jj == 1) {
                const void* g = fam == 0 ? p.gV : (comp == 0 ? p.gbx : p.gby);
                RW::inverse(src, static_cast<const V*>(g) + hb, nullptr, R(0), rc, lds_all, twN, twX, iscale);
                void* outp = fam == 0 ? p.V_out : (comp == 0 ? p.bx_out : p.by_out);
                if (outp) RW::store(src, static_cast<R*>(outp) + po, ri.j, ri.valid);
            } else {
                for (int i = 2; i <= jj; ++i) {
#pragma unroll
                    for (int q = 0; q < E; ++q) pw[q] = rmul(pw[q], base[q]);
                }
                const void* const* phys = fam == 0 ? p.Vphys : (comp == 0 ? p.bxphys : p.byphys);
                RW::load(src, static_cast<const R*>(phys[l - jj]) + po, ri.j, ri.valid);
            }
#pragma unroll
            for (int q = 0; q < E; ++q) src[q] = rmul(pw[q], src[q]);
            const int idx = fam == 0 ? jj - 1 : nv + comp * nv + jj - 1;
            RW::forward(src, static_cast<V*>(p.h[idx]) + hb, rc, lds_all, twN, twX);
        } else {
            for (int i = 2; i <= nv; ++i) {
#pragma unroll
                for (int q = 0; q < E; ++q) pw[q] = rmul(pw[q], base[q]);
            }
            RW::load(src, static_cast<const R*>(comp == 0 ? p.phx : p.phy) + po, ri.j, ri.valid);
#pragma unroll
            for (int q = 0; q < E; ++q) src[q] = rmul(pw[q], src[q]);
            RW::forward(src, static_cast<V*>(p.h[nv + nb + comp]) + hb, rc, lds_all, twN, twX);
        }
        return;
    }
    int idx = 0;
    V a[E], base[E], pw[E];
    // eta^j V_(l-j)
    RW::inverse(a, static_cast<const V*>(p.gV) + hb, nullptr, R(0), rc, lds_all, twN, twX, iscale);
    if (p.V_out) RW::store(a, static_cast<R*>(p.V_out) + po, ri.j, ri.valid);
    RW::load(base, static_cast<const R*>(p.eta) + po, ri.j, ri.valid);
#pragma unroll
    for (int q = 0; q < E; ++q) pw[q] = base[q];
    for (int jj = 1; jj <= l - 1; ++jj) {
        V src[E], w[E];
        if (jj == 1) {
#pragma unroll
            for (int q = 0; q < E; ++q) src[q] = a[q];
        } else {
#pragma unroll
            for (int q = 0; q < E; ++q) pw[q] = rmul(pw[q], base[q]);
            RW::load(src, static_cast<const R*>(p.Vphys[l - jj]) + po, ri.j, ri.valid);
        }
#pragma unroll
        for (int q = 0; q < E; ++q) w[q] = rmul(pw[q], src[q]);
        RW::forward(w, static_cast<V*>(p.h[idx++]) + hb, rc, lds_all, twN, twX);
    }
    // delta^j grad phi_b,(l-j)
    if (p.vd) {
        const int ncomp = p.g.ny > 1 ? 2 : 1;
        for (int comp = 0; comp < ncomp; ++comp) {
            const void* gsrc = comp == 0 ? p.gbx : p.gby;
            void* outp = comp == 0 ? p.bx_out : p.by_out;
            const void* const* phys = comp == 0 ? p.bxphys : p.byphys;
            RW::inverse(a, static_cast<const V*>(gsrc) + hb, nullptr, R(0), rc, lds_all, twN, twX, iscale);
            if (outp) RW::store(a, static_cast<R*>(outp) + po, ri.j, ri.valid);
            RW::load(base, static_cast<const R*>(p.delta) + po, ri.j, ri.valid);
#pragma unroll
            for (int q = 0; q < E; ++q) pw[q] = base[q];
            for (int jj = 1; jj <= l - 1; ++jj) {
                V src[E], w[E];
                if (jj == 1) {
#pragma unroll
                    for (int q = 0; q < E; ++q) src[q] = a[q];
                } else {
#pragma unroll
                    for (int q = 0; q < E; ++q) pw[q] = rmul(pw[q], base[q]);
                    RW::load(src, static_cast<const R*>(phys[l - jj]) + po, ri.j, ri.valid);
                }
#pragma unroll
                for (int q = 0; q < E; ++q) w[q] = rmul(pw[q], src[q]);
                RW::forward(w, static_cast<V*>(p.h[idx++]) + hb, rc, lds_all, twN, twX);
            }
        }
    }
    // forcing eta^(l-1) grad phi_s
    RW::load(base, static_cast<const R*>(p.eta) + po, ri.j, ri.valid);
#pragma unroll
    for (int q = 0; q < E; ++q) pw[q] = base[q];
    for (int jj = 2; jj <= l - 1; ++jj) {
#pragma unroll
        for (int q = 0; q < E; ++q) pw[q] = rmul(pw[q], base[q]);
    }
    const int ncomp = p.g.ny > 1 ? 2 : 1;
    for (int comp = 0; comp < ncomp; ++comp) {
        V w[E];
        RW::load(a, static_cast<const R*>(comp == 0 ? p.phx : p.phy) + po, ri.j, ri.valid);
#pragma unroll
        for (int q = 0; q < E; ++q) w[q] = rmul(pw[q], a[q]);
        RW::forward(w, static_cast<V*>(p.h[idx++]) + hb, rc, lds_all, twN, twX);
    }
}

// nonlinear term of the potential equation; TANK adds the wave tank's surface
// pressures (a separate instance, so that the plain one keeps its registers)
template <typename R, int NX, bool TANK>
__device__ __forceinline__ void row_nphi_body(const RowNphiParams& p, const typename cplx_of<R>::type* twN_tab,
                                              const typename cplx_of<R>::type* twX_tab) {
    ROW_PROLOGUE(R, NX)
    V q[E], gg[E], pp[E], a[E], b[E];
    const V* gD = p.gD ? static_cast<const V*>(p.gD) + hb : nullptr;
    const R c2 = gD ? R(1.0 - p.ctl[ri.mem].omega) : R(0);
    RW::inverse(q, static_cast<const V*>(p.gV) + hb, gD, c2, rc, lds_all, twN, twX, iscale);
    RW::inverse(a, static_cast<const V*>(p.gex) + hb, nullptr, R(0), rc, lds_all, twN, twX, iscale);
    RW::inverse(b, static_cast<const V*>(p.gpx) + hb, nullptr, R(0), rc, lds_all, twN, twX, iscale);
    const double dx = p.g.lx / p.g.nx;
    // damping weight mu(x) of the wave tank times a potential gradient, in
    // place (the gradient is spent by then) -> forward half form
    auto damped = [&](V (&grad)[E], void* out) {
#pragma unroll
        for (int k = 0; k < E; ++k) {
            const int n = ri.j + k * RW::P;
            double mv[2];
#pragma unroll
            for (int hh = 0; hh < 2; ++hh) {
                const double d = fmod((2 * n + hh) * dx - p.dmp_x0 + 1.5 * p.g.lx, p.g.lx) - 0.5 * p.g.lx;
                mv[hh] = exp(-(d / p.dmp_w) * (d / p.dmp_w));
            }
            grad[k] = cx<V>(R(mv[0] * (double)grad[k].x), R(mv[1] * (double)grad[k].y));
        }
        RW::forward(grad, static_cast<V*>(out) + hb, rc, lds_all, twN, twX);
    };
#pragma unroll
    for (int k = 0; k < E; ++k) {
        q[k] = cx<V>(q[k].x + a[k].x * b[k].x, q[k].y + a[k].y * b[k].y);
        gg[k] = rmul(a[k], a[k]);
        pp[k] = rmul(b[k], b[k]);
    }
    if (p.g.ny > 1) {
        if constexpr (TANK)
            if (p.dmp_w > 0.0) damped(b, p.hdx);
        RW::inverse(a, static_cast<const V*>(p.gey) + hb, nullptr, R(0), rc, lds_all, twN, twX, iscale);
        RW::inverse(b, static_cast<const V*>(p.gpy) + hb, nullptr, R(0), rc, lds_all, twN, twX, iscale);
#pragma unroll
        for (int k = 0; k < E; ++k) {
            q[k] = cx<V>(q[k].x + a[k].x * b[k].x, q[k].y + a[k].y * b[k].y);
            gg[k] = cx<V>(gg[k].x + a[k].x * a[k].x, gg[k].y + a[k].y * a[k].y);
            pp[k] = cx<V>(pp[k].x + b[k].x * b[k].x, pp[k].y + b[k].y * b[k].y);
        }
    }
#pragma unroll
    for (int k = 0; k < E; ++k) {
        q[k] = cx<V>(R(0.5) * (q[k].x * q[k].x / (R(1) + gg[k].x) - pp[k].x),
                     R(0.5) * (q[k].y * q[k].y / (R(1) + gg[k].y) - pp[k].y));
    }
    // the last potential gradient (d_x phi in 1D, d_y phi in 2D), after the
    // products, when only q is live beside it
    if constexpr (TANK)
        if (p.dmp_w > 0.0) damped(b, p.g.ny > 1 ? p.hdy : p.hdx);
    if (TANK && p.wm_n > 0) {
        // pneumatic wavemaker: bell-shaped pressures centred on x = 0, i.e. split
        // over both ends of the periodic domain; the prefactor
        // a_j sqrt(e/(2 pi)) (1 + 2 k_j h / sinh(2 k_j h)) radiates waves of amplitude a_j
        const double hg = p.wm_h > 0.0 ? p.wm_h : p.g.href[ri.mem];
        double amp[kMaxWavemaker];
#pragma unroll
        for (int c = 0; c < kMaxWavemaker; ++c) {
            amp[c] = 0.0;
            if (c < p.wm_n) {
                const double kh2 = 2.0 * p.wm[c][1] * hg;
                const double G = kh2 < 700.0 ? kh2 / sinh(kh2) : 0.0;
                amp[c] = p.wm[c][0] * sqrt(M_E / (2.0 * M_PI)) * (1.0 + G) * sin(p.wm[c][2] * p.t + p.wm[c][3]);
            }
        }
#pragma unroll
        for (int k = 0; k < E; ++k) {
            const int n = ri.j + k * RW::P;
            double pg[2] = {0.0, 0.0};
#pragma unroll
            for (int hh = 0; hh < 2; ++hh) {
                const double x = (2 * n + hh) * dx;
                const double xs = x < 0.5 * p.g.lx ? x : x - p.g.lx;
#pragma unroll
                for (int c = 0; c < kMaxWavemaker; ++c) {
                    if (c < p.wm_n) {
                        const double kx = p.wm[c][1] * xs;
                        pg[hh] += amp[c] * exp(-0.5 * kx * kx);
                    }
                }
            }
            q[k] = cx<V>(R((double)q[k].x - pg[0]), R((double)q[k].y - pg[1]));
        }
    }
    RW::forward(q, static_cast<V*>(p.h) + hb, rc, lds_all, twN, twX);
}

template <typename R, int NX>
__global__ void __launch_bounds__(row_threads<NX>()) k_row_nphi(const RowNphiParams p, const typename cplx_of<R>::type* twN_tab,
                           const typename cplx_of<R>::type* twX_tab) {
    row_nphi_body<R, NX, false>(p, twN_tab, twX_tab);
}

template <typename R, int NX>
__global__ void __launch_bounds__(row_threads<NX>()) k_row_nphi_tank(const RowNphiParams p,
                                                                     const typename cplx_of<R>::type* twN_tab,
                                                                     const typename cplx_of<R>::type* twX_tab) {
    row_nphi_body<R, NX, true>(p, twN_tab, twX_tab);
}

template <typename R, int NX>
__global__ void __launch_bounds__(row_threads<NX>()) k_row_blend(const RowBlendParams p, const typename cplx_of<R>::type* twN_tab,
                            const typename cplx_of<R>::type* twX_tab) {
    ROW_PROLOGUE(R, NX)
    const double dx = p.g.lx / p.g.nx;
    const double r = p.t < p.ramp_time ? 0.5 * (1.0 - cos(M_PI * p.t / p.ramp_time)) : 1.0;
    // the zones' reciprocal lengths, once: a division per point, unrolled over
    // the row's elements, would hold more registers than the transforms
    const double igen = p.gen > 0.0 ? 1.0 / p.gen : 0.0, iabs = p.absl > 0.0 ? 1.0 / p.absl : 0.0;
    // one field at a time (eta against a r cos, phi against a r / om sin), so
    // that a single row of values is live
    auto blend = [&](const void* in, void* out, bool pot) {
        V v[E];
        RW::inverse(v, static_cast<const V*>(in) + hb, nullptr, R(0), rc, lds_all, twN, twX, iscale);
        const double amp = pot ? p.a * r / p.om : p.a * r;
        // target a r cos(k x - om t) for eta and a r / om cos(k x - om t - pi/2)
        // for phi: one sincos at the thread's first point 2j, then rotations by
        // k dx (to point 2n + 1) and by 2 P k dx (to the next element), each
        // exact to rounding (the two fields' phases differ, so that the first
        // field's rotated values are not kept for the second)
        double c0, s0, ch, sh, cq, sq;
        sincos(p.k * (2 * ri.j) * dx - p.om * p.t - (pot ? 0.5 * M_PI : 0.0), &s0, &c0);
        sincos(p.k * dx, &sh, &ch);
        sincos(p.k * (2 * RW::P) * dx, &sq, &cq);
#pragma unroll
        for (int q = 0; q < E; ++q) {
            const int n = ri.j + q * RW::P;
            double fv[2] = {(double)v[q].x, (double)v[q].y};
            double c = c0, sn = s0;
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                const double x = (2 * n + h) * dx;
                double wg = 0.0, wa = 0.0;
                if (x < p.gen) {
                    const double s = x * igen;
                    wg = 1.0 - (3 * s * s - 2 * s * s * s);
                }
                if (x > p.g.lx - p.absl) {
                    const double s = (p.g.lx - x) * iabs;
                    wa = 1.0 - (3 * s * s - 2 * s * s * s);
                }
                fv[h] = (1.0 - wg) * fv[h] + wg * (amp * c);
                fv[h] *= (1.0 - wa);
                const double cn = c * ch - sn * sh;
                sn = sn * ch + c * sh;
                c = cn;
            }
            const double cn = c0 * cq - s0 * sq;
            s0 = s0 * cq + c0 * sq;
            c0 = cn;
            v[q] = cx<V>(R(fv[0]), R(fv[1]));
        }
        RW::forward(v, static_cast<V*>(out) + hb, rc, lds_all, twN, twX);
    };
    blend(p.ge, p.he, false);
    blend(p.gp, p.hp, true);
}

// Learned-warm-start features of each point, channel-last FP32:
// (eta, W_lin, d_x eta, d_y eta, d_x phi, d_y phi, delta, eta * W_lin), each
// multiplied by its channel scale in the working precision before rounding.
template <typename R, int NX>
__global__ void __launch_bounds__(row_threads<NX>()) k_row_feat(const RowFeatParams p, const typename cplx_of<R>::type* twN_tab,
                           const typename cplx_of<R>::type* twX_tab) {
    ROW_PROLOGUE(R, NX)
    V wl[E], a[E];
    RW::inverse(wl, static_cast<const V*>(p.gV) + hb, nullptr, R(0), rc, lds_all, twN, twX, iscale);
    if (p.wlin) RW::store(wl, static_cast<R*>(p.wlin) + po, ri.j, ri.valid);
    float2 fe[4][E];
    const void* src[4] = {p.gex, p.gey, p.gpx, p.gpy};
    const int ch[4] = {2, 3, 4, 5};
#pragma unroll
    for (int f = 0; f < 4; ++f) {
        RW::inverse(a, static_cast<const V*>(src[f]) + hb, nullptr, R(0), rc, lds_all, twN, twX, iscale);
        const R sc = R(p.scale[ch[f]]);
#pragma unroll
        for (int q = 0; q < E; ++q) fe[f][q] = make_float2((float)(a[q].x * sc), (float)(a[q].y * sc));
    }
    if (!ri.valid) return;  // after the last workgroup barrier
    V ev[E], dv[E];
    RW::load(ev, static_cast<const R*>(p.eta) + po, ri.j, true);
    RW::load(dv, static_cast<const R*>(p.delta) + po, ri.j, true);
    const R s0 = R(p.scale[0]), s1 = R(p.scale[1]), s6 = R(p.scale[6]), s7 = R(p.scale[7]);
    float4* out = reinterpret_cast<float4*>(p.feat + po * 8);
#pragma unroll
    for (int q = 0; q < E; ++q) {
        const int n = ri.j + q * RW::P;  // points 2n and 2n + 1 of the row
        out[4 * n + 0] = make_float4((float)(ev[q].x * s0), (float)(wl[q].x * s1), fe[0][q].x, fe[1][q].x);
        out[4 * n + 1] = make_float4(fe[2][q].x, fe[3][q].x, (float)(dv[q].x * s6), (float)(ev[q].x * wl[q].x * s7));
        out[4 * n + 2] = make_float4((float)(ev[q].y * s0), (float)(wl[q].y * s1), fe[0][q].y, fe[1][q].y);
        out[4 * n + 3] = make_float4(fe[2][q].y, fe[3][q].y, (float)(dv[q].y * s6), (float)(ev[q].y * wl[q].y * s7));
    }
}

// ---------------------------------------------------------------------------
// Column pass: forward column transforms of the products, multiplier sums,
// relaxation, compact outputs, inverse column transforms of the results.
// ---------------------------------------------------------------------------
// Shape of a column pass.  QB ("quarter band"): the kept band |m_y| <= My lies
// below NY/4, so of the E values a thread transforms (modes j + qP) only the
// first and last E/4 can be kept; the accumulators of the others are never
// formed.  Elements per thread: 8, or 4 in FP64 without QB (the accumulators of
// all E modes then share the registers); columns of 128 or more threads get a
// workgroup of their own, shorter ones are packed to 256 threads per lane (half
// forms are column-major, so each column is one contiguous run); product
// lanes (threads transforming different products of the same columns) fill up
// to 512 threads, at most 2 in FP64 without QB and 4 otherwise.
// WV ("wave lanes", QB at NY = 1024 with at most 2 accumulators in FP64):
// 16 elements per thread, so a single wavefront owns a whole column
// transform; one column per workgroup and up to 8 product lanes of one
// wavefront each, which never wait on one another until their sums are
// combined.  (Four FP64 accumulators of 16 elements do not fit in registers.)
// WAVE: every column transform lies within one wavefront, so its exchanges
// order only that wavefront.
template <typename R, int NY, bool QB, int NACC> struct ColCfg {
    static constexpr bool WV = QB && NY == 1024 && (sizeof(R) == 4 || NACC <= 2);
    static constexpr int CE = WV ? 16 : ((sizeof(R) == 8 && !QB) ? 4 : 8);
    static constexpr int E = FftShape<NY, CE>::E;
    static constexpr int P = FftShape<NY, CE>::P;
    static constexpr int C = NY == 1 ? 64 : ((WV || P >= 128) ? 1 : 256 / P);
    static constexpr int LMAX = WV ? 8 : ((sizeof(R) == 8 && !QB) ? 2 : 4);
    static constexpr int FIT = 512 / (C * P);
    // 1D grids: eight wavefront lanes share a tile's products (each "column"
    // is one value, so a lane's rounds are one dependent load each)
    static constexpr int PL = NY == 1 ? 8 : (FIT < 1 ? 1 : (FIT < LMAX ? FIT : LMAX));
    static constexpr int THREADS = PL * C * P;
    static constexpr bool WAVE = P <= 64;
    // the next round's column is loaded during the current transform, except
    // in FP64 wave lanes, whose registers cannot hold a second column (the
    // other wavefront of the SIMD covers the load instead)
    static constexpr bool PREFETCH = !(WV && sizeof(R) == 8);
    // LDS: the transform exchange area of every lane and column (for 1D
    // grids, whose "columns" are single values, one value per lane and column
    // to combine the lanes' sums), then the mode-geometry table of C * Ky
    // entries of 4 reals
    static constexpr int XFORM = PL * C * fft_lds_elems<NY, E>();
    static constexpr size_t lds_bytes(int Ky) {
        return (size_t)XFORM * sizeof(typename cplx_of<R>::type) + (size_t)C * Ky * 4 * sizeof(R);
    }
    static constexpr bool keepable(int q) { return !QB || q < E / 4 || q >= E - E / 4; }
};


// Sweep control of a column pass: decides the solve from the previous
// sweep's residual (false: this launch has nothing to do) and gives the
// relaxation weight; the leader thread updates the control header.
__device__ __forceinline__ bool col_control(const ColParams& p, Ctl* ctl, bool leader, double* omega) {
    const GridDev& g = p.g;
    if (p.ctl_mode == CTL_SWEEP) {
        if (ctl->done) return false;
        double r, rmin;
        const int dec = sweep_decision(ctl, p.sweep, p.max_sweeps, p.tol, &r, &rmin);
        if (dec) {
            if (leader) ctl_commit(ctl, dec - 100, p.sweep, r);
            return false;
        }
        if (leader) {
            ctl->rmin = rmin;
            ctl->residual = r;
        }
        *omega = ctl->omega;
    } else if (p.ctl_mode == CTL_SKIP) {
        if (ctl->done) return false;
        *omega = ctl->omega;
    } else if (p.ctl_mode == CTL_OMEGA) {
        // relaxation weight from the local symbol sum_{j<=J} (k eta)^j / j!
        const double emax = unord_bits(ctl->eta_max), emin = unord_bits(ctl->eta_min);
        const int J = g.order - 1;
        double w = 1.0;
        if (g.relax && J >= 1) {
            double lmax = 0.0, lmin = 0.0, tmax = 1.0, tmin = 1.0;
            const double xmax = g.kband * emax, xmin = g.kband * emin;
            for (int jj = 0; jj <= J; ++jj) {
                if (jj > 0) {
                    tmax *= xmax / jj;
                    tmin *= xmin / jj;
                }
                lmax += tmax;
                lmin += tmin;
            }
            const double s = lmin + lmax;
            if (isfinite(s) && s > 0.0) w = fmin(1.0, 2.0 / s);
        }
        *omega = w;
        if (leader) ctl->omega = w;
    }
    return true;
}

// Stage a column pass's term table and the geometry of its C columns' kept
// modes in LDS: geo[(c * Ky + r) * 4 + {0, 1, 2, 3}] = {k, tanh(k h), sech(k h),
// k_y} (the caller synchronises).
template <typename R>
__device__ __forceinline__ void col_stage_tables(const ColParams& p, int x0, int C, double href, R* geo_all,
                                                 ColTerm* s_term, short* s_toff) {
    const GridDev& g = p.g;
    const int t = threadIdx.x;
    for (int i = t; i < p.nterm; i += blockDim.x) s_term[i] = p.term[i];
    for (int i = t; i <= p.nprod + p.ncin; i += blockDim.x) s_toff[i] = p.toff[i];
    for (int idx = t; idx < C * g.Ky; idx += blockDim.x) {
        const int c2 = idx / g.Ky, r2 = idx % g.Ky;
        const int my = r2 <= g.My ? r2 : r2 - g.Ky;
        const double kx2 = 2.0 * M_PI * (double)(x0 + c2) / g.lx;
        const double ky = (g.ny == 1) ? 0.0 : 2.0 * M_PI * (double)my / g.ly;
        const double k = sqrt(kx2 * kx2 + ky * ky);
        R* gq = geo_all + idx * 4;
        gq[0] = R(k);
        gq[1] = R(tanh(k * href));
        gq[2] = R(sech_d(k * href));
        gq[3] = R(ky);
    }
}

// multiplier sum of one source into the accumulators (kept modes only)
// toff, term: the pass's term table, staged in LDS; geo: the column's mode
// geometry (col_stage_tables)
template <typename R, typename V, int E, int NACC>
__device__ __forceinline__ void col_apply_terms(const short* toff, const ColTerm* term, int src, const V (&v)[E],
                                                V (&acc)[NACC][E], const int (&crow)[E], const R* __restrict__ geo,
                                                R kxr) {
    // modes outer, terms inner: only one mode's geometry is live at a time
    // (each accumulator still sums its terms in table order)
    const int t0 = toff[src], t1 = toff[src + 1];
#pragma unroll
    for (int q = 0; q < E; ++q) {
        if (crow[q] < 0) continue;
        const R* gq = geo + crow[q] * 4;
        const R kq = gq[0];
        for (int ti = t0; ti < t1; ++ti) {
            const ColTerm tm = term[ti];
            R m = R(tm.coef);
            if (tm.fn == FN_T) m *= gq[1];
            else if (tm.fn == FN_S) m *= gq[2];
            if (tm.pw >= 0) {
                for (int e = 0; e < tm.pw; ++e) m *= kq;
            } else {
                m = kq > R(0) ? m / kq : R(0);
            }
            V val = cscale(v[q], m);
            if (tm.dv == DV_X) val = mul_i(cscale(val, kxr));
            else if (tm.dv == DV_Y) val = mul_i(cscale(val, gq[3]));
#pragma unroll
            for (int a = 0; a < NACC; ++a)
                if (a == tm.acc) acc[a][q] = cadd(acc[a][q], val);
        }
    }
}

// value of output source `src` at the thread's mode q (crow >= 0)
template <typename R, typename V, int E, int NACC>
__device__ __forceinline__ V col_source(const ColParams& p, int src, int q, const V (&acc)[NACC][E], int crow,
                                        int mem, int mx, double omega) {
    if (src <= SRC_ACC3) {
        V r = cx<V>(R(0), R(0));
#pragma unroll
        for (int a = 0; a < NACC; ++a)
            if (a == src) r = acc[a][q];
        return r;
    }
    const int a = (src == SRC_NEW0 || src == SRC_DIFF0) ? 0 : 1;
    V cur = cx<V>(R(0), R(0));
#pragma unroll
    for (int k = 0; k < NACC; ++k)
        if (k == a) cur = acc[k][q];
    V pv = cx<V>(R(0), R(0));
    const int pi = p.relax_prev[a];
    if (pi >= 0)
        pv = static_cast<const V*>(p.cin[pi])[mem * p.g.s_cmp + (long long)mx * p.g.Ky + crow];
    const V d = csub(cur, pv);
    if (src == SRC_DIFF0 || src == SRC_DIFF1) return d;
    return cadd(pv, cscale(d, R(omega)));
}

// entry i of a register array, with i known only at run time: a chain of
// selects, so the array is never placed in memory
static __device__ __forceinline__ double aa_sel(const double (&v)[kAASlots], int i) {
    double r = 0.0;
#pragma unroll
    for (int q = 0; q < kAASlots; ++q) r = q == i ? v[q] : r;
    return r;
}

// Anderson mixing of the relaxed sweep: from dots[i] = <F_i, f_n> over the
// ring slots of sweep n, complete the Gram matrix of the residual history,
// solve the normal equations of min |f_n - sum_a gamma_a dF_a|,
// dF_a = F_(a+1) - F_a over the history in sweep order (regularised by
// 1e-12 trace / k; gamma = 0 when they fail), and write to w the weights of
// x_(n+1) = g_n - sum_a gamma_a (G_(a+1) - G_a) on the history slots.
// commit: store the new Gram entries (row and column of slot n) in the
// control block.  The entries read here that are not in that row and column
// were stored by earlier sweeps, so workgroups of one pass that solve
// side by side while one of them commits read the same values.
// dots and w are indexed with compile-time indices only (registers); the
// history slots in sweep order are H_a = (n - k + a) mod kAASlots, a <= k
static __device__ void aa_weights(Ctl* ctl, int n, const double (&dots)[kAASlots], double (&w)[kAASlots],
                                  bool commit) {
    static_assert(kAADepth == 2, "the elimination below is written out for two residual differences");
    const int s = n % kAASlots, k = n < kAADepth ? n : kAADepth;
    const int H0 = (n - k) % kAASlots, H1 = (n - k + 1) % kAASlots, H2 = (n - k + 2) % kAASlots;
    // the new row and column of slot s (over the slots of the history) come
    // from dots; the other entries were stored by earlier sweeps
    if (commit) {
#pragma unroll
        for (int i = 0; i < kAASlots; ++i) {
            const bool hi = i == H0 || (k >= 1 && i == H1) || (k >= 2 && i == H2);
            if (hi) {
                ctl->aa_gram[s][i] = aa_sel(dots, i);
                ctl->aa_gram[i][s] = aa_sel(dots, i);
            }
        }
    }
    auto M = [&](int a, int b) {
        const int r = a == 0 ? H0 : (a == 1 ? H1 : H2), c = b == 0 ? H0 : (b == 1 ? H1 : H2);
        if (r == s) return aa_sel(dots, c);
        if (c == s) return aa_sel(dots, r);
        return ctl->aa_gram[r][c];
    };
    double gam0 = 0.0, gam1 = 0.0;
    if (k == 1) {
        double A00 = M(1, 1) - M(1, 0) - M(0, 1) + M(0, 0);
        const double y0 = M(1, 1) - M(0, 1);
        const double tr = A00;
        A00 += 1e-12 * tr;
        const bool ok = tr > 0.0 && isfinite(tr) && fabs(A00) > 0.0;
        gam0 = ok ? y0 / A00 : 0.0;
        if (!isfinite(gam0)) gam0 = 0.0;
    } else if (k == 2) {
        double A00 = M(1, 1) - M(1, 0) - M(0, 1) + M(0, 0);
        double A01 = M(1, 2) - M(1, 1) - M(0, 2) + M(0, 1);
        double A10 = M(2, 1) - M(2, 0) - M(1, 1) + M(1, 0);
        double A11 = M(2, 2) - M(2, 1) - M(1, 2) + M(1, 1);
        double y0 = M(1, 2) - M(0, 2), y1 = M(2, 2) - M(1, 2);
        const double tr = A00 + A11;
        const double reg = 1e-12 * tr / 2;
        A00 += reg;
        A11 += reg;
        bool ok = tr > 0.0 && isfinite(tr);
        // Gaussian elimination with partial pivoting on the first column
        if (fabs(A10) > fabs(A00)) {
            double t = A00; A00 = A10; A10 = t;
            t = A01; A01 = A11; A11 = t;
            t = y0; y0 = y1; y1 = t;
        }
        ok = ok && fabs(A00) > 0.0;
        if (ok) {
            const double f = A10 / A00;
            A11 -= f * A01;
            y1 -= f * y0;
            ok = fabs(A11) > 0.0;
        }
        if (ok) {
            gam1 = y1 / A11;
            gam0 = (y0 - A01 * gam1) / A00;
            ok = isfinite(gam0) && isfinite(gam1);
        }
        if (!ok) gam0 = gam1 = 0.0;
    }
    // x_(n+1) = G_k - sum_a gamma_a (G_(a+1) - G_a): weights of the history slots
    const double c0 = k == 0 ? 1.0 : gam0;
    const double c1 = k == 1 ? 1.0 - gam0 : gam1 - gam0;
    const double c2 = 1.0 - gam1;
#pragma unroll
    for (int i = 0; i < kAASlots; ++i)
        w[i] = i == H0 ? c0 : ((k >= 1 && i == H1) ? c1 : ((k >= 2 && i == H2) ? c2 : 0.0));
}

// the weights inside a column-pass workgroup: the partials of the member are
// added in a fixed order (strided per thread, then across the wavefront, then
// wavefront by wavefront), so every workgroup forms the same weights; s_red
// holds kAASlots reals per wavefront (<= 16), s_w receives the weights
static __device__ void aa_block_weights(const ColParams& p, Ctl* ctl, int mem, bool commit, double* s_red, double* s_w) {
    double d[kAASlots];
#pragma unroll
    for (int i = 0; i < kAASlots; ++i) d[i] = 0.0;
    const double* part = p.aa_partial + (long long)mem * p.aa_nblk * kAASlots;
    for (int b = threadIdx.x; b < p.aa_nblk; b += blockDim.x)
#pragma unroll
        for (int i = 0; i < kAASlots; ++i) d[i] += part[b * kAASlots + i];
#pragma unroll
    for (int i = 0; i < kAASlots; ++i)
        for (int off = 32; off > 0; off >>= 1) d[i] += __shfl_xor(d[i], off, 64);
    const int wv = threadIdx.x / 64;
    if ((threadIdx.x & 63) == 0)
#pragma unroll
        for (int i = 0; i < kAASlots; ++i) s_red[wv * kAASlots + i] = d[i];
    __syncthreads();
    if (threadIdx.x == 0) {
        double tot[kAASlots], w[kAASlots];
#pragma unroll
        for (int i = 0; i < kAASlots; ++i) tot[i] = 0.0;
        const int nw = (blockDim.x + 63) / 64;
        for (int v = 0; v < nw; ++v)
#pragma unroll
            for (int i = 0; i < kAASlots; ++i) tot[i] += s_red[v * kAASlots + i];
        aa_weights(ctl, p.aa_sweep, tot, w, commit);
#pragma unroll
        for (int i = 0; i < kAASlots; ++i) s_w[i] = w[i];
    }
    __syncthreads();
}

// product lanes of a column-pass workgroup: independent thread groups that
// transform alternate products of the same columns (more waves per CU to hide
// memory latency); their partial sums are combined through LDS
template <typename R, int NY, int NACC, bool QB>
__global__ void __launch_bounds__((ColCfg<R, NY, QB, NACC>::THREADS))
k_col(const ColParams p, const typename cplx_of<R>::type* __restrict__ twY) {
    using V = typename cplx_of<R>::type;
    using CF = ColCfg<R, NY, QB, NACC>;
    constexpr int N = NY;
    constexpr int CE = CF::CE;
    constexpr int E = CF::E;
    constexpr int P = CF::P;
    constexpr int C = CF::C;
    constexpr int PL = CF::PL;
    constexpr int REG = fft_lds_elems<N, E>();  // LDS elements of one column transform
    extern __shared__ __attribute__((aligned(16))) unsigned char smem_raw[];
    const int t = threadIdx.x;
    // a lane is a whole number of wavefronts: make its index wave-uniform, so
    // that the per-product parameters it selects are scalar loads (a vector
    // load would also wait for the next product's prefetched column)
    const int lane = (C * P) % 64 == 0 ? __builtin_amdgcn_readfirstlane(t / (C * P)) : t / (C * P);
    const int tl = t % (C * P);
    const int c = tl / P;  // column of the tile
    const int j = tl % P;  // thread within the column
    V* lds = reinterpret_cast<V*>(smem_raw) + (lane * C + c) * REG;
    const int mem = blockIdx.z;
    const int grp = blockIdx.y;
    const int x0 = blockIdx.x * C;
    const int mx = x0 + c;
    const GridDev& g = p.g;
    Ctl* ctl = p.ctl ? p.ctl + mem : nullptr;

    double omega = 1.0;
    if (!col_control(p, ctl, blockIdx.x == 0 && grp == 0 && t == 0, &omega)) return;
    __shared__ double s_aa[(16 + 1) * kAASlots];  // wavefront sums, then the Anderson weights
    if (p.aa_partial) aa_block_weights(p, ctl, mem, blockIdx.x == 0 && grp == 0, s_aa, s_aa + 16 * kAASlots);

    Twid<V, N, E> twc;
    twc.load(twY, j);

    // mode geometry: the compact row of each value this thread owns (m_y index
    // n = j + q P) and an LDS table of k, tanh(kh), sech(kh), k_y per kept mode
    const double href = g.href[mem];
    const double kx = 2.0 * M_PI * (double)mx / g.lx;
    int crow[E];  // compact row, -1 if not kept
#pragma unroll
    for (int q = 0; q < E; ++q) {
        const int n = j + q * P;
        const int my = (n <= N / 2) ? n : n - N;
        const bool keep = CF::keepable(q) && (mx < g.Kx) && (my <= g.My) && (my >= -g.My);
        crow[q] = keep ? (my >= 0 ? my : my + g.Ky) : -1;
    }
    // the pass's term table in LDS: its per-product reads then wait on LDS
    // only, never on the prefetched column in flight
    __shared__ ColTerm s_term[kMaxTerms];
    __shared__ short s_toff[kMaxProd + kMaxCin + 1];
    R* geo_all = reinterpret_cast<R*>(reinterpret_cast<V*>(smem_raw) + CF::XFORM);
    col_stage_tables<R>(p, x0, C, href, geo_all, s_term, s_toff);
    __syncthreads();
    const R* geo = geo_all + c * g.Ky * 4;
    const R kxr = R(kx);

    V acc[NACC][E];  // entries of modes that cannot be kept are never used
#pragma unroll
    for (int a = 0; a < NACC; ++a)
#pragma unroll
        for (int q = 0; q < E; ++q) acc[a][q] = cx<V>(R(0), R(0));

    // jobs of this workgroup: its products (forward column transforms), then,
    // in the first product group only, the compact inputs, whose kept values
    // enter the same multiplier sums without a transform.  Lane L takes jobs
    // L, L + PL, ...; every lane runs the same number of rounds (slots that
    // are not products transform zeros so that workgroup barriers line up,
    // or skip the transform when it synchronises per wavefront).  The next
    // round's column is loaded before the current transform runs.
    const int s0 = p.ngroup > 1 ? p.gstart[grp] : 0;
    const int s1 = p.ngroup > 1 ? p.gstart[grp + 1] : p.nprod;
    const int nps = s1 - s0;
    const int njob = nps + (grp == 0 ? p.ncin : 0);
    const int rounds = (njob + PL - 1) / PL;
    auto load_col = [&](int jb, V (&dst)[E]) __attribute__((always_inline)) {
        if (jb < nps) {
            const int s = s0 + jb;
            const long long st = p.hin_stride[s] ? p.hin_stride[s] : g.s_half;
            const V* H = static_cast<const V*>(p.hin[s]) + mem * st + (long long)mx * g.ldh;
#pragma unroll
            for (int q = 0; q < E; ++q) dst[q] = H[j + q * P];
        } else {
#pragma unroll
            for (int q = 0; q < E; ++q) dst[q] = cx<V>(R(0), R(0));
        }
    };
    V v[E];
    if constexpr (CF::PREFETCH) {
        if (rounds > 0) load_col(lane, v);
    }
    for (int rd = 0; rd < rounds; ++rd) {
        const int jb = rd * PL + lane;
        const bool prod = jb < nps;
        const int src = prod ? s0 + jb : p.nprod + (jb - nps);  // row of the term table
        const bool live = jb < njob && s_toff[src] < s_toff[src + 1];
        V vn[E];
        if constexpr (CF::PREFETCH) {
            if (rd + 1 < rounds) load_col(jb + PL, vn);
        } else {
            if (CF::WAVE && jb >= njob) break;
            load_col(jb, v);
        }
        if (prod || !CF::WAVE) fft<V, N, false, 1, CE, CF::WAVE>(v, lds, 0, j, twc);
        if (live && !prod) {
            const V* Ci = static_cast<const V*>(p.cin[jb - nps]) + mem * g.s_cmp + (long long)mx * g.Ky;
            const int wi = p.cin_widx[jb - nps];
            const R cw = wi >= 0 ? R(s_aa[16 * kAASlots + wi]) : R(1);
#pragma unroll
            for (int q = 0; q < E; ++q) v[q] = crow[q] >= 0 ? cscale(Ci[crow[q]], cw) : cx<V>(R(0), R(0));
        }
        if (live) col_apply_terms<R, V, E, NACC>(s_toff, s_term, src, v, acc, crow, geo, kxr);
        if constexpr (CF::PREFETCH) {
#pragma unroll
            for (int q = 0; q < E; ++q) v[q] = vn[q];
        }
    }
    // combine the lanes' partial sums into lane 0
    if (PL > 1 && rounds > 0) {
#pragma unroll
        for (int a = 0; a < NACC; ++a) {
            lds_sync();
            if (lane > 0) {
#pragma unroll
                for (int q = 0; q < E; ++q)
                    if (CF::keepable(q)) lds[j + q * P] = acc[a][q];
            }
            lds_sync();
            if (lane == 0) {
#pragma unroll
                for (int l2 = 1; l2 < PL; ++l2) {
                    const V* o = reinterpret_cast<const V*>(smem_raw) + (l2 * C + c) * REG;
#pragma unroll
                    for (int q = 0; q < E; ++q)
                        if (CF::keepable(q)) acc[a][q] = cadd(acc[a][q], o[j + q * P]);
                }
            }
        }
    }
    if (p.ngroup > 1) {
        // publish this group's partial sums; the last workgroup of the tile
        // continues with their sum in group order (deterministic)
        V* part = static_cast<V*>(p.part);
        const long long gs = (long long)g.Ky * g.Kxp;
        if (lane == 0) {
#pragma unroll
            for (int a = 0; a < NACC; ++a)
#pragma unroll
                for (int q = 0; q < E; ++q)
                    if (crow[q] >= 0)
                        part[(((long long)mem * kMaxGroups + grp) * 4 + a) * gs + (long long)mx * g.Ky + crow[q]] =
                            acc[a][q];
        }
        __shared__ int last_flag;
        __threadfence();
        __syncthreads();
        if (t == 0) {
            const int old = atomicAdd(&p.cnt[(long long)mem * kMaxTiles + blockIdx.x], 1);
            last_flag = (old == p.ngroup - 1);
        }
        __syncthreads();
        if (!last_flag) return;
        __threadfence();
        if (t == 0) p.cnt[(long long)mem * kMaxTiles + blockIdx.x] = 0;
        if (lane == 0) {
#pragma unroll
            for (int a = 0; a < NACC; ++a)
#pragma unroll
                for (int q = 0; q < E; ++q) {
                    if (!CF::keepable(q)) continue;
                    V sum = cx<V>(R(0), R(0));
                    if (crow[q] >= 0) {
                        for (int gg = 0; gg < p.ngroup; ++gg) {
                            const R* ps = reinterpret_cast<const R*>(
                                part + (((long long)mem * kMaxGroups + gg) * 4 + a) * gs + (long long)mx * g.Ky +
                                crow[q]);
                            sum = cadd(sum,
                                       cx<V>(__builtin_nontemporal_load(ps), __builtin_nontemporal_load(ps + 1)));
                        }
                    }
                    acc[a][q] = sum;
                }
        }
    }
    // broadcast the final sums to every lane
    if (PL > 1 && p.ninv > 1) {
#pragma unroll
        for (int a = 0; a < NACC; ++a) {
            lds_sync();
            if (lane == 0) {
#pragma unroll
                for (int q = 0; q < E; ++q)
                    if (CF::keepable(q)) lds[j + q * P] = acc[a][q];
            }
            lds_sync();
            if (lane > 0) {
                const V* o = reinterpret_cast<const V*>(smem_raw) + c * REG;
#pragma unroll
                for (int q = 0; q < E; ++q)
                    if (CF::keepable(q)) acc[a][q] = o[j + q * P];
            }
        }
    }
    // the exchange areas were last read across lanes (sums combined or
    // broadcast): every lane is past those reads before it transforms again
    if (PL > 1) lds_sync();
    // inverse column transforms, spread over the lanes (before any compact
    // output is written: NEW/DIFF sources re-read the previous iterate)
    const int lanes_used = (PL > 1 && p.ninv > 1) ? PL : 1;
    const int irounds = (p.ninv + lanes_used - 1) / lanes_used;
    for (int rd = 0; rd < irounds; ++rd) {
        const int o = rd * lanes_used + (lanes_used > 1 ? lane : 0);
        const bool mine = (lanes_used > 1 || lane == 0) && o < p.ninv;
        if (CF::WAVE && !mine) continue;
        V vi[E];
        const int src = mine ? p.inv_src[o] : 0;
        const int dv = mine ? p.inv_dv[o] : 0;
#pragma unroll
        for (int q = 0; q < E; ++q) {
            V sv = cx<V>(R(0), R(0));
            if (mine && crow[q] >= 0) sv = col_source<R, V, E, NACC>(p, src, q, acc, crow[q], mem, mx, omega);
            if (crow[q] >= 0) {
                if (dv == DV_X) sv = mul_i(cscale(sv, kxr));
                else if (dv == DV_Y) sv = mul_i(cscale(sv, geo[crow[q] * 4 + 3]));
            }
            vi[q] = sv;
        }
        fft<V, N, true, 1, CE, CF::WAVE>(vi, lds, 0, j, twc);
        if (mine) {
            V* G = static_cast<V*>(p.inv[o]) + mem * g.s_half + (long long)mx * g.ldh;
#pragma unroll
            for (int q = 0; q < E; ++q) G[j + q * P] = vi[q];
        }
    }
    if (PL > 1) __syncthreads();  // inverse outputs (read prev) before compact outputs (write)
    // compact outputs: the previous iterates the relaxed sources need are read
    // before any output is written, so an output may overwrite an input of
    // the same pass in place
    if (lane == 0) {
        V pv[2][E];
#pragma unroll
        for (int a = 0; a < 2; ++a) {
            const int pi = p.relax_prev[a];
            const V* Pp = pi >= 0 ? static_cast<const V*>(p.cin[pi]) + mem * p.g.s_cmp + (long long)mx * p.g.Ky
                                  : nullptr;
#pragma unroll
            for (int q = 0; q < E; ++q)
                pv[a][q] = (Pp && crow[q] >= 0) ? Pp[crow[q]] : cx<V>(R(0), R(0));
        }
        for (int o = 0; o < p.ncout; ++o) {
            const int src = p.cout_src[o];
            const bool relaxed = src >= SRC_NEW0;
            const int a = relaxed ? ((src == SRC_NEW0 || src == SRC_DIFF0) ? 0 : 1) : src;
            const bool diff = src >= SRC_DIFF0;
            V* out = static_cast<V*>(p.cout[o]) + mem * g.s_cmp + (long long)mx * g.Ky;
#pragma unroll
            for (int q = 0; q < E; ++q) {
                if (crow[q] < 0) continue;
                V cur = cx<V>(R(0), R(0));
#pragma unroll
                for (int k = 0; k < NACC; ++k)
                    if (k == a) cur = acc[k][q];
                V val = cur;
                if (relaxed) {
                    const V pq = a == 0 ? pv[0][q] : pv[1][q];
                    const V d = csub(cur, pq);
                    val = diff ? d : cadd(pq, cscale(d, R(omega)));
                }
                out[crow[q]] = val;
            }
        }
    }
}

// ---------------------------------------------------------------------------
// Column pass in wave pairs (1024 rows, quarter band, at most two
// accumulators, one product group).  Decimation in frequency splits a
// 1024-point column transform into the 512-point transforms of its even and
// odd outputs: wave 0 of a pair transforms u0[n] = x[n] + x[n + 512] and
// wave 1 u1[n] = (x[n] - x[n + 512]) W^n, W = exp(-2 pi i / 1024), so that
// X[2k] = U0[k] and X[2k + 1] = U1[k].  Both waves read the whole column (the
// second read is served by the cache) and transform with wave-level
// ordering only; a thread of wave h holds the modes 2 (j + 64 q) + h.  The
// inverse runs the other way: each wave inverts its half of the modes, the
// odd half is multiplied by W^-n, and the pair forms x[n] = e[n] + o[n] and
// x[n + 512] = e[n] - o[n] through LDS.  Seven pairs (14 wavefronts, at most
// 128 registers each) share the workgroup of one column.
// ---------------------------------------------------------------------------
struct ColPairCfg {
    static constexpr int N = 1024, NH = 512, E = 8, P = 64;
    static constexpr int PL = 7;
    static constexpr int THREADS = PL * 2 * P;
    static constexpr int REG = fft_lds_elems<NH, E>();  // LDS elements of one wave's exchange area
    static constexpr bool keepable(int q) { return q < E / 4 || q >= E - E / 4; }
    template <typename R> static constexpr size_t lds_bytes(int Ky) {
        return (size_t)PL * 2 * REG * sizeof(typename cplx_of<R>::type) + (size_t)Ky * 4 * sizeof(R);
    }
};

template <typename R, int NACC>
__global__ void __launch_bounds__(ColPairCfg::THREADS)
k_colp(const ColParams p, const typename cplx_of<R>::type* __restrict__ twY) {
    using V = typename cplx_of<R>::type;
    using CF = ColPairCfg;
    constexpr int N = CF::N, NH = CF::NH, E = CF::E, P = CF::P, PL = CF::PL, REG = CF::REG;
    extern __shared__ __attribute__((aligned(16))) unsigned char smem_raw[];
    const int t = threadIdx.x;
    const int wv = __builtin_amdgcn_readfirstlane(t / P);
    const int lane = wv >> 1;  // pair
    const int h = wv & 1;      // 0: even outputs, 1: odd outputs
    const int j = t % P;
    V* const xch = reinterpret_cast<V*>(smem_raw);
    V* lds = xch + wv * REG;
    const int mem = blockIdx.z;
    const int mx = blockIdx.x;
    const GridDev& g = p.g;
    Ctl* ctl = p.ctl ? p.ctl + mem : nullptr;

    // tables and twiddles are requested before the sweep decision, whose
    // chain of dependent control reads then overlaps them; a launch after
    // the member's solve was decided returns before any table work
    Twid<V, NH, E> twc;
    twc.load(twY, j, 2);  // the 512-point twiddles are every other 1024-point one
    if (p.ctl_mode == CTL_SWEEP && ctl->done) return;
    const double href = g.href[mem];
    const double kx = 2.0 * M_PI * (double)mx / g.lx;
    int crow[E];  // compact row of mode 2 (j + qP) + h, -1 if not kept
#pragma unroll
    for (int q = 0; q < E; ++q) {
        const int n = 2 * (j + q * P) + h;
        const int my = (n <= N / 2) ? n : n - N;
        const bool keep = CF::keepable(q) && (mx < g.Kx) && (my <= g.My) && (my >= -g.My);
        crow[q] = keep ? (my >= 0 ? my : my + g.Ky) : -1;
    }
    __shared__ ColTerm s_term[kMaxTerms];
    __shared__ short s_toff[kMaxProd + kMaxCin + 1];
    R* geo = reinterpret_cast<R*>(xch + PL * 2 * REG);
    col_stage_tables<R>(p, mx, 1, href, geo, s_term, s_toff);
    const V wj = twY[j], wP = twY[P];  // W^(j + qP) = W^j (W^P)^q
    double omega = 1.0;
    // the decision is the same in every thread (the leader's header updates
    // cannot change it), so the workgroup returns as a whole
    if (!col_control(p, ctl, blockIdx.x == 0 && t == 0, &omega)) return;
    __shared__ double s_aa[(16 + 1) * kAASlots];  // wavefront sums, then the Anderson weights
    if (p.aa_partial) aa_block_weights(p, ctl, mem, blockIdx.x == 0, s_aa, s_aa + 16 * kAASlots);
    __syncthreads();
    const R kxr = R(kx);

    V acc[NACC][E];  // entries of modes that cannot be kept are never used
#pragma unroll
    for (int a = 0; a < NACC; ++a)
#pragma unroll
        for (int q = 0; q < E; ++q) acc[a][q] = cx<V>(R(0), R(0));

    // jobs: the products (forward transforms), then the compact inputs; job
    // jb is row jb of the term table.  Round rd deals jobs rd PL .. rd PL +
    // PL - 1 to the pairs in alternating direction, so the cheap compact-input
    // jobs of the last rounds go to pairs with fewer transforms.
    const int nps = p.nprod;
    const int njob = nps + p.ncin;
    const int rounds = (njob + PL - 1) / PL;
    for (int rd = 0; rd < rounds; ++rd) {
        const int jb = rd * PL + ((rd & 1) ? PL - 1 - lane : lane);
        if (jb >= njob) continue;
        if (s_toff[jb] == s_toff[jb + 1]) continue;  // no term reads it
        V v[E];
        if (jb < nps) {
            const long long st = p.hin_stride[jb] ? p.hin_stride[jb] : g.s_half;
            const V* H = static_cast<const V*>(p.hin[jb]) + mem * st + (long long)mx * g.ldh;
            if (h == 0) {
#pragma unroll
                for (int q = 0; q < E; ++q) v[q] = cadd(H[j + q * P], H[j + q * P + NH]);
            } else {
                V w = wj;
                asm volatile("" : "+v"(w.x), "+v"(w.y));  // powers formed here, not held across rounds
#pragma unroll
                for (int q = 0; q < E; ++q) {
                    v[q] = cmul(csub(H[j + q * P], H[j + q * P + NH]), w);
                    w = cmul(w, wP);
                }
            }
            fft<V, NH, false, 1, E, true>(v, lds, 0, j, twc);
        } else {
            const V* Ci = static_cast<const V*>(p.cin[jb - nps]) + mem * g.s_cmp + (long long)mx * g.Ky;
            const int wi = p.cin_widx[jb - nps];
            const R cw = wi >= 0 ? R(s_aa[16 * kAASlots + wi]) : R(1);
#pragma unroll
            for (int q = 0; q < E; ++q) v[q] = crow[q] >= 0 ? cscale(Ci[crow[q]], cw) : cx<V>(R(0), R(0));
        }
        col_apply_terms<R, V, E, NACC>(s_toff, s_term, jb, v, acc, crow, geo, kxr);
    }
    // combine the pairs' partial sums into pair 0 (the same half of every pair
    // holds the same modes), every accumulator in one exchange: the kept slots
    // of NACC <= 2 accumulators fill NACC * E/2 * P <= 512 of an area's slots
    static_assert(NACC * (E / 2) * P <= REG, "the accumulators exceed an exchange area");
    auto slot = [&](int a, int q) { return (a * (E / 2) + (q < E / 4 ? q : q - E / 2)) * P + j; };
    if (rounds > 0) {
        lds_sync();
        if (lane > 0) {
#pragma unroll
            for (int a = 0; a < NACC; ++a)
#pragma unroll
                for (int q = 0; q < E; ++q)
                    if (CF::keepable(q)) lds[slot(a, q)] = acc[a][q];
        }
        lds_sync();
        if (lane == 0) {
#pragma unroll
            for (int l2 = 1; l2 < PL; ++l2) {
                const V* o = xch + (2 * l2 + h) * REG;
#pragma unroll
                for (int a = 0; a < NACC; ++a)
#pragma unroll
                    for (int q = 0; q < E; ++q)
                        if (CF::keepable(q)) acc[a][q] = cadd(acc[a][q], o[slot(a, q)]);
            }
        }
    }
    // broadcast the final sums to every pair
    if (p.ninv > 1) {
        lds_sync();
        if (lane == 0) {
#pragma unroll
            for (int a = 0; a < NACC; ++a)
#pragma unroll
                for (int q = 0; q < E; ++q)
                    if (CF::keepable(q)) lds[slot(a, q)] = acc[a][q];
        }
        lds_sync();
        if (lane > 0) {
            const V* o = xch + h * REG;
#pragma unroll
            for (int a = 0; a < NACC; ++a)
#pragma unroll
                for (int q = 0; q < E; ++q)
                    if (CF::keepable(q)) acc[a][q] = o[slot(a, q)];
        }
    }
    lds_sync();  // every pair is past the reads above before the areas are reused
    // compact outputs, mode by mode: a mode's previous iterates are read before
    // any output of that mode is written, so an output may overwrite an input
    // of the same pass in place
    auto compact_outputs = [&]() __attribute__((always_inline)) {
        const long long co = mem * g.s_cmp + (long long)mx * g.Ky;
        const V* P0 = p.relax_prev[0] >= 0 ? static_cast<const V*>(p.cin[p.relax_prev[0]]) + co : nullptr;
        const V* P1 = p.relax_prev[1] >= 0 ? static_cast<const V*>(p.cin[p.relax_prev[1]]) + co : nullptr;
#pragma unroll
        for (int q = 0; q < E; ++q) {
            if (crow[q] < 0) continue;
            const V pv0 = P0 ? P0[crow[q]] : cx<V>(R(0), R(0));
            const V pv1 = P1 ? P1[crow[q]] : cx<V>(R(0), R(0));
            for (int o = 0; o < p.ncout; ++o) {
                const int src = p.cout_src[o];
                const bool relaxed = src >= SRC_NEW0;
                const int a = relaxed ? ((src == SRC_NEW0 || src == SRC_DIFF0) ? 0 : 1) : src;
                V cur = cx<V>(R(0), R(0));
#pragma unroll
                for (int k = 0; k < NACC; ++k)
                    if (k == a) cur = acc[k][q];
                V val = cur;
                if (relaxed) {
                    const V pq = a == 0 ? pv0 : pv1;
                    const V d = csub(cur, pq);
                    val = src >= SRC_DIFF0 ? d : cadd(pq, cscale(d, R(omega)));
                }
                static_cast<V*>(p.cout[o])[co + crow[q]] = val;
            }
        }
    };
    // inverse column transforms of the outputs, one per pair and round.  When
    // they take a single round and leave a pair idle (which then holds the
    // broadcast sums too), that pair writes the compact outputs while the
    // others transform, once every pair has read the previous iterates its
    // sources need; otherwise pair 0 writes them at the end.
    const int lanes_used = p.ninv > 1 ? PL : 1;
    const int irounds = (p.ninv + lanes_used - 1) / lanes_used;
    const bool overlap = p.ninv > 1 && irounds == 1 && p.ninv < PL;
    for (int rd = 0; rd < irounds; ++rd) {
        const int o = rd * lanes_used + (lanes_used > 1 ? lane : 0);
        const bool mine = (lanes_used > 1 || lane == 0) && o < p.ninv;
        V v[E];
        if (mine) {
            const int isrc = p.inv_src[o], dv = p.inv_dv[o];
#pragma unroll
            for (int q = 0; q < E; ++q) {
                V sv = cx<V>(R(0), R(0));
                if (crow[q] >= 0) {
                    sv = col_source<R, V, E, NACC>(p, isrc, q, acc, crow[q], mem, mx, omega);
                    if (dv == DV_X) sv = mul_i(cscale(sv, kxr));
                    else if (dv == DV_Y) sv = mul_i(cscale(sv, geo[crow[q] * 4 + 3]));
                }
                v[q] = sv;
            }
        }
        if (overlap) {
            __syncthreads();  // every source above has been formed from the previous iterates
            if (lane == PL - 1) compact_outputs();
        }
        if (mine) {
            fft<V, NH, true, 1, E, true>(v, lds, 0, j, twc);
            if (h == 1) {
                V w = cconj(wj);
                asm volatile("" : "+v"(w.x), "+v"(w.y));
                const V wPc = cconj(wP);
#pragma unroll
                for (int q = 0; q < E; ++q) {
                    v[q] = cmul(v[q], w);
                    w = cmul(w, wPc);
                }
            }
#pragma unroll
            for (int q = 0; q < E; ++q) lds[j + q * P] = v[q];
        }
        lds_sync();
        if (mine) {
            const V* ev = xch + (2 * lane) * REG;
            const V* od = xch + (2 * lane + 1) * REG;
            V* G = static_cast<V*>(p.inv[o]) + mem * g.s_half + (long long)mx * g.ldh + h * NH;
#pragma unroll
            for (int q = 0; q < E; ++q) {
                const int n = j + q * P;
                G[n] = h == 0 ? cadd(ev[n], od[n]) : csub(ev[n], od[n]);
            }
        }
        lds_sync();
    }
    // every inverse transform above has read its sources (the last barrier)
    if (!overlap && lane == 0) compact_outputs();
}

// ---------------------------------------------------------------------------
// Pointwise spectral kernels
// ---------------------------------------------------------------------------
struct ModeGeo {
    int r, mx;
    bool valid;
    double kx, ky, k;
};
__device__ __forceinline__ ModeGeo mode_geo(const GridDev& g, long long idx) {
    ModeGeo m;
    m.mx = (int)(idx / g.Ky);
    m.r = (int)(idx % g.Ky);
    m.valid = m.r < g.Ky && m.mx < g.Kx;
    const int my = m.r <= g.My ? m.r : m.r - g.Ky;
    m.kx = 2.0 * M_PI * m.mx / g.lx;
    m.ky = g.ny == 1 ? 0.0 : 2.0 * M_PI * my / g.ly;
    m.k = sqrt(m.kx * m.kx + m.ky * m.ky);
    return m;
}

template <typename R>
__global__ void k_rk(const RkParams p) {
    using V = typename cplx_of<R>::type;
    const int mem = blockIdx.y;
    const long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= p.g.s_cmp) return;
    const ModeGeo m = mode_geo(p.g, idx);
    if (!m.valid) return;
    const long long o = mem * p.g.s_cmp + idx;
    const double href = p.g.href[mem];
    const double om2 = m.k * tanh(m.k * href);
    const double om = sqrt(om2);
    const double h = p.h;
    V* eh = static_cast<V*>(p.eh);
    V* ph = static_cast<V*>(p.ph);
    V* es = static_cast<V*>(p.es);
    V* ps = static_cast<V*>(p.ps);
    V* ae = static_cast<V*>(p.ae);
    V* ap = static_cast<V*>(p.ap);
    const V vh = static_cast<const V*>(p.Vh)[o];
    const V nph = static_cast<const V*>(p.Nph)[o];
    const V psv = ps[o];
    // derivative of the stage: (W_hat - omega^2 phi_hat, N_phi [- p_d_hat])
    const double de_r = (double)vh.x - om2 * (double)psv.x, de_i = (double)vh.y - om2 * (double)psv.y;
    double dp_r = (double)nph.x, dp_i = (double)nph.y;
    if (p.Pdiv && m.k > 0.0) {
        const V pd = static_cast<const V*>(p.Pdiv)[o];
        dp_r += (double)pd.x / (m.k * m.k);
        dp_i += (double)pd.y / (m.k * m.k);
    }
    const double u_er = (double)eh[o].x, u_ei = (double)eh[o].y;
    const double u_pr = (double)ph[o].x, u_pi = (double)ph[o].y;
    auto prop = [&](double tau, double er, double ei, double pr, double pi_, double* oer, double* oei, double* opr,
                    double* opi) {
        const double c = cos(om * tau), s = sin(om * tau);
        const double sw = om > 0.0 ? s / om : tau;
        *oer = c * er + om * s * pr;
        *oei = c * ei + om * s * pi_;
        *opr = -sw * er + c * pr;
        *opi = -sw * ei + c * pi_;
    };
    double a_er, a_ei, a_pr, a_pi;   // accumulator
    double n_er, n_ei, n_pr, n_pi;   // next stage state
    if (p.stage == 0) {
        prop(h, de_r, de_i, dp_r, dp_i, &a_er, &a_ei, &a_pr, &a_pi);
        prop(0.5 * h, u_er + 0.5 * h * de_r, u_ei + 0.5 * h * de_i, u_pr + 0.5 * h * dp_r, u_pi + 0.5 * h * dp_i,
             &n_er, &n_ei, &n_pr, &n_pi);
    } else if (p.stage == 1 || p.stage == 2) {
        double b_er, b_ei, b_pr, b_pi;
        prop(0.5 * h, de_r, de_i, dp_r, dp_i, &b_er, &b_ei, &b_pr, &b_pi);
        a_er = (double)ae[o].x + 2.0 * b_er;
        a_ei = (double)ae[o].y + 2.0 * b_ei;
        a_pr = (double)ap[o].x + 2.0 * b_pr;
        a_pi = (double)ap[o].y + 2.0 * b_pi;
        if (p.stage == 1) {
            prop(0.5 * h, u_er, u_ei, u_pr, u_pi, &n_er, &n_ei, &n_pr, &n_pi);
            n_er += 0.5 * h * de_r;
            n_ei += 0.5 * h * de_i;
            n_pr += 0.5 * h * dp_r;
            n_pi += 0.5 * h * dp_i;
        } else {
            prop(h, u_er, u_ei, u_pr, u_pi, &n_er, &n_ei, &n_pr, &n_pi);
            n_er += h * b_er;
            n_ei += h * b_ei;
            n_pr += h * b_pr;
            n_pi += h * b_pi;
        }
    } else {
        prop(h, u_er, u_ei, u_pr, u_pi, &n_er, &n_ei, &n_pr, &n_pi);
        n_er += h / 6.0 * ((double)ae[o].x + de_r);
        n_ei += h / 6.0 * ((double)ae[o].y + de_i);
        n_pr += h / 6.0 * ((double)ap[o].x + dp_r);
        n_pi += h / 6.0 * ((double)ap[o].y + dp_i);
        if (p.fb1 > 0.0 && p.fb2 > 0.0) {
            const double lam = exp(-pow(fabs(m.k / p.fb1), p.fb2));
            n_er *= lam;
            n_ei *= lam;
            n_pr *= lam;
            n_pi *= lam;
        }
        eh[o] = cx<V>(R(n_er), R(n_ei));
        ph[o] = cx<V>(R(n_pr), R(n_pi));
        es[o] = cx<V>(R(n_er), R(n_ei));
        ps[o] = cx<V>(R(n_pr), R(n_pi));
        return;
    }
    ae[o] = cx<V>(R(a_er), R(a_ei));
    ap[o] = cx<V>(R(a_pr), R(a_pi));
    es[o] = cx<V>(R(n_er), R(n_ei));
    ps[o] = cx<V>(R(n_pr), R(n_pi));
}

// Six-stage fifth-order pair with an embedded fourth-order solution (Sec. 2.2),
// the coefficients of Cash & Karp (ACM TOMS 16, 1990): nodes, stage matrix,
// fifth-order weights and the weight differences fifth minus fourth order.
static __constant__ double kPairC[6] = {0.0, 1.0 / 5.0, 3.0 / 10.0, 3.0 / 5.0, 1.0, 7.0 / 8.0};
static __constant__ double kPairA[6][5] = {
    {0.0, 0.0, 0.0, 0.0, 0.0},
    {1.0 / 5.0, 0.0, 0.0, 0.0, 0.0},
    {3.0 / 40.0, 9.0 / 40.0, 0.0, 0.0, 0.0},
    {3.0 / 10.0, -9.0 / 10.0, 6.0 / 5.0, 0.0, 0.0},
    {-11.0 / 54.0, 5.0 / 2.0, -70.0 / 27.0, 35.0 / 27.0, 0.0},
    {1631.0 / 55296.0, 175.0 / 512.0, 575.0 / 13824.0, 44275.0 / 110592.0, 253.0 / 4096.0}};
static __constant__ double kPairB[6] = {37.0 / 378.0, 0.0, 250.0 / 621.0, 125.0 / 594.0, 0.0, 512.0 / 1771.0};
static __constant__ double kPairE[6] = {37.0 / 378.0 - 2825.0 / 27648.0, 0.0,  250.0 / 621.0 - 18575.0 / 48384.0,
                                 125.0 / 594.0 - 13525.0 / 55296.0, -277.0 / 14336.0, 512.0 / 1771.0 - 0.25};

// One stage of the pair in Lawson form, per kept mode.  With E(tau) the exact
// linear propagator (eta, phi) -> (cos eta + om sin phi, -sin/om eta + cos phi)
// and N_i = (W - om^2 phi, N_phi [- p_d]) at stage state U_i, the stage derivative is
// kept as K_i = E(-c_i h) N_i (carried back to t_n), so that
//   U_{i+1} = E(c_{i+1} h) (u_n + h sum_j a_{i+1,j} K_j),
//   u_5     = E(h) (u_n + h sum_j b_j K_j),   u_5 - u_4 = E(h) h sum_j e_j K_j.
// E preserves |eta|^2 + om^2 |phi|^2 per mode, so the linear-energy norms of
// the difference and of the candidate are summed in the frame of t_n; the last
// stage writes per-block partial sums of both (weights 2 for m_x > 0: the half
// spectrum stands for its conjugate).
template <typename R>
__global__ void k_rk54(const Rk54Params p) {
    using V = typename cplx_of<R>::type;
    __shared__ double red[2][256];
    const int mem = blockIdx.y;
    const int i = p.stage;
    const double h = p.h;
    const double href = p.g.href[mem];
    double num = 0.0, den = 0.0;
    for (long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x; idx < p.g.s_cmp;
         idx += (long long)gridDim.x * blockDim.x) {
        const ModeGeo m = mode_geo(p.g, idx);
        if (!m.valid) continue;
        const long long o = mem * p.g.s_cmp + idx;
        const double om2 = m.k * tanh(m.k * href);
        const double om = sqrt(om2);
        // (er, ei, pr, pi) -> E(tau) applied
        auto prop = [&](double tau, double& er, double& ei, double& pr, double& pi_) {
            const double c = cos(om * tau), s = sin(om * tau);
            const double sw = om > 0.0 ? s / om : tau;
            const double a = c * er + om * s * pr, b = c * ei + om * s * pi_;
            pr = -sw * er + c * pr;
            pi_ = -sw * ei + c * pi_;
            er = a;
            ei = b;
        };
        const V vh = static_cast<const V*>(p.Vh)[o];
        const V nph = static_cast<const V*>(p.Nph)[o];
        const V psv = static_cast<const V*>(p.ps)[o];
        double ker = (double)vh.x - om2 * (double)psv.x, kei = (double)vh.y - om2 * (double)psv.y;
        double kpr = (double)nph.x, kpi = (double)nph.y;
        if (p.Pdiv && m.k > 0.0) {
            // damping pressure of the wave tank: -p_d_hat = i k . MF{mu grad phi} / k^2
            const V pd = static_cast<const V*>(p.Pdiv)[o];
            kpr += (double)pd.x / (m.k * m.k);
            kpi += (double)pd.y / (m.k * m.k);
        }
        prop(-kPairC[i] * h, ker, kei, kpr, kpi);
        static_cast<V*>(p.ke[i])[o] = cx<V>(R(ker), R(kei));
        static_cast<V*>(p.kp[i])[o] = cx<V>(R(kpr), R(kpi));
        const V ue = static_cast<const V*>(p.eh)[o];
        const V up = static_cast<const V*>(p.ph)[o];
        // the stored value (rounded to R) enters the sums, as it does when read back
        const V kse = cx<V>(R(ker), R(kei)), ksp = cx<V>(R(kpr), R(kpi));
        const double* w = i < 5 ? kPairA[i + 1] : kPairB;
        double ser = 0.0, sei = 0.0, spr = 0.0, spi = 0.0;   // sum_j w_j K_j
        double der = 0.0, dei = 0.0, dpr = 0.0, dpi = 0.0;   // sum_j e_j K_j (last stage)
        for (int j = 0; j <= i; ++j) {
            const V ke = j == i ? kse : static_cast<const V*>(p.ke[j])[o];
            const V kp = j == i ? ksp : static_cast<const V*>(p.kp[j])[o];
            ser += w[j] * (double)ke.x;
            sei += w[j] * (double)ke.y;
            spr += w[j] * (double)kp.x;
            spi += w[j] * (double)kp.y;
            if (i == 5) {
                der += kPairE[j] * (double)ke.x;
                dei += kPairE[j] * (double)ke.y;
                dpr += kPairE[j] * (double)kp.x;
                dpi += kPairE[j] * (double)kp.y;
            }
        }
        double ner = (double)ue.x + h * ser, nei = (double)ue.y + h * sei;
        double npr = (double)up.x + h * spr, npi = (double)up.y + h * spi;
        if (i == 5) {
            const double wt = m.mx == 0 ? 1.0 : 2.0;
            num += wt * h * h * (der * der + dei * dei + om2 * (dpr * dpr + dpi * dpi));
            den += wt * (ner * ner + nei * nei + om2 * (npr * npr + npi * npi));
        }
        prop((i < 5 ? kPairC[i + 1] : 1.0) * h, ner, nei, npr, npi);
        if (i == 5 && p.fb1 > 0.0 && p.fb2 > 0.0) {
            const double lam = exp(-pow(fabs(m.k / p.fb1), p.fb2));
            ner *= lam;
            nei *= lam;
            npr *= lam;
            npi *= lam;
        }
        static_cast<V*>(p.es)[o] = cx<V>(R(ner), R(nei));
        static_cast<V*>(p.ps)[o] = cx<V>(R(npr), R(npi));
    }
    if (i < 5) return;
    red[0][threadIdx.x] = num;
    red[1][threadIdx.x] = den;
    __syncthreads();
    for (int s = blockDim.x / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) {
            red[0][threadIdx.x] += red[0][threadIdx.x + s];
            red[1][threadIdx.x] += red[1][threadIdx.x + s];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        p.partial[((long long)mem * p.nblk + blockIdx.x) * 2 + 0] = red[0][0];
        p.partial[((long long)mem * p.nblk + blockIdx.x) * 2 + 1] = red[1][0];
    }
}

// ---------------------------------------------------------------------------
// Anderson mixing of the relaxed sweep (iteration mode)
// ---------------------------------------------------------------------------
// The sweep's column pass stores f_n = T(x_n) - x_n and g_n = x_n + omega f_n
// in ring slot n mod kAASlots; k_aa_dot forms per-workgroup partial sums of
// <F_i, f_n> over the k + 1 = min(n, kAADepth) + 1 history slots (real inner
// product of the real fields: half-spectrum modes weighted 2 for m_x > 0).
// The column pass that forms the next iterate adds them and solves for its
// weights in every workgroup (aa_block_weights).
template <typename R>
__global__ void __launch_bounds__(kAADotThreads) k_aa_dot(const AaParams p) {
    using V = typename cplx_of<R>::type;
    __shared__ double red[kAASlots][16];
    const int mem = blockIdx.y;
    const Ctl* ctl = p.ctl + mem;
    if (ctl->done) return;
    const GridDev& g = p.g;
    const int n = p.sweep, k = n < kAADepth ? n : kAADepth;
    const int ncmp = (int)g.s_cmp;
    double d[kAASlots];
#pragma unroll
    for (int i = 0; i < kAASlots; ++i) d[i] = 0.0;
    for (int idx = blockIdx.x * blockDim.x + threadIdx.x; idx < ncmp; idx += gridDim.x * blockDim.x) {
        const int mx = idx / g.Ky;
        if (mx >= g.Kx) continue;
        const long long o = mem * g.s_cmp + idx;
        const double wt = mx == 0 ? 1.0 : 2.0;
#pragma unroll
        for (int part = 0; part < 2; ++part) {
            if (part == 1 && !p.vd) break;
            V fo[kAASlots];
#pragma unroll
            for (int j = 0; j <= kAADepth; ++j)
                if (j <= k) {
                    const int si = (n - j) % kAASlots;
                    fo[j] = static_cast<const V*>(part ? p.fb[si] : p.fv[si])[o];
                }
#pragma unroll
            for (int j = 0; j <= kAADepth; ++j) {
                if (j > k) break;
                const int si = (n - j) % kAASlots;
                const double v = wt * ((double)fo[j].x * (double)fo[0].x + (double)fo[j].y * (double)fo[0].y);
#pragma unroll
                for (int i = 0; i < kAASlots; ++i)
                    if (i == si) d[i] += v;
            }
        }
    }
    // across the wavefront, then wavefront by wavefront (<= 16 of them)
#pragma unroll
    for (int i = 0; i < kAASlots; ++i)
        for (int off = 32; off > 0; off >>= 1) d[i] += __shfl_xor(d[i], off, 64);
    const int wv = threadIdx.x / 64;
    if ((threadIdx.x & 63) == 0)
#pragma unroll
        for (int i = 0; i < kAASlots; ++i) red[i][wv] = d[i];
    __syncthreads();
    if (threadIdx.x < kAASlots) {
        double v = 0.0;
        const int nw = (blockDim.x + 63) / 64;
        for (int w = 0; w < nw; ++w) v += red[threadIdx.x][w];
        p.partial[((long long)mem * p.nblk + blockIdx.x) * kAASlots + threadIdx.x] = v;
    }
}

template <typename R>
__global__ void k_diag(const DiagParams p) {
    using V = typename cplx_of<R>::type;
    __shared__ double red[2][256];
    const int mem = blockIdx.y;
    double se = 0.0, sm = 0.0;
    for (long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x; idx < p.g.s_cmp;
         idx += (long long)gridDim.x * blockDim.x) {
        const ModeGeo m = mode_geo(p.g, idx);
        if (!m.valid) continue;
        const long long o = mem * p.g.s_cmp + idx;
        const V e = static_cast<const V*>(p.eh)[o];
        const V f = static_cast<const V*>(p.ph)[o];
        const V w = static_cast<const V*>(p.Vh)[o];
        const double wt = m.mx == 0 ? 1.0 : 2.0;
        se += wt * ((double)w.x * (double)f.x + (double)w.y * (double)f.y + (double)e.x * (double)e.x +
                    (double)e.y * (double)e.y);
        if (idx == 0) sm += (double)e.x;
    }
    red[0][threadIdx.x] = se;
    red[1][threadIdx.x] = sm;
    __syncthreads();
    for (int s = blockDim.x / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) {
            red[0][threadIdx.x] += red[0][threadIdx.x + s];
            red[1][threadIdx.x] += red[1][threadIdx.x + s];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        p.partial[((long long)mem * p.nblk + blockIdx.x) * 2 + 0] = red[0][0];
        p.partial[((long long)mem * p.nblk + blockIdx.x) * 2 + 1] = red[1][0];
    }
}

// ---------------------------------------------------------------------------
// launchers (size dispatch)
// ---------------------------------------------------------------------------
// workgroups along y of a row pass: the sweep splits its product families
template <typename PT> static int row_families(const PT&) { return 1; }
static int row_families(const RowSweepParams& p) { return p.nfam > 0 ? p.nfam : 1; }
static int row_families(const RowSaParams& p) { return p.split > 0 ? p.split : 1; }
static int row_families(const RowSetupParams& p) { return p.nfam > 1 ? p.nfam : 1; }

template <typename RWT> struct RowLaunch {
    using V = typename RWT::V;
    // rpw_req: rows per workgroup asked for by the launch plan (0: as many as
    // fit 256 threads); it is a power of two, as ny is, which the row
    // kernels rely on, and capped by the kernels' launch bounds
    static void shape(int ny, dim3* grid, dim3* block, size_t* lds, int batch, int nfam, int rpw_req = 0) {
        constexpr int P = RWT::P;
        const int cap = P >= 256 ? 1 : 256 / P;
        int rpw = (rpw_req > 0 && rpw_req < cap) ? rpw_req : cap;
        if (rpw > ny) rpw = ny;
        *block = dim3(P * rpw);
        *grid = dim3((ny + rpw - 1) / rpw, nfam, batch);
        *lds = ((size_t)rpw * RWT::LS + RWT::N) * sizeof(V);
    }
};

#define SBI_ROW_NX_SWITCH(KNAME, PTYPE)                                                                    \
    template <typename R>                                                                                  \
    static hipError_t KNAME##_nx(const PTYPE& p, int batch, const Twiddles& tw, hipStream_t s) {           \
        switch (p.g.nx) {                                                                                  \
            case 16: return KNAME##_go<R, 16>(p, batch, tw, s);                                            \
            case 32: return KNAME##_go<R, 32>(p, batch, tw, s);                                            \
            case 64: return KNAME##_go<R, 64>(p, batch, tw, s);                                            \
            case 128: return KNAME##_go<R, 128>(p, batch, tw, s);                                          \
            case 256: return KNAME##_go<R, 256>(p, batch, tw, s);                                          \
            case 512: return KNAME##_go<R, 512>(p, batch, tw, s);                                          \
            case 1024: return KNAME##_go<R, 1024>(p, batch, tw, s);                                        \
            case 2048: return KNAME##_go<R, 2048>(p, batch, tw, s);                                        \
            case 4096: return KNAME##_go<R, 4096>(p, batch, tw, s);                                        \
            case 8192: return KNAME##_go<R, 8192>(p, batch, tw, s);                                        \
            default: return hipErrorInvalidValue;                                                          \
        }                                                                                                  \
    }

#define SBI_ROW_LAUNCH(KNAME, PTYPE)                                                                       \
    template <typename R, int NX>                                                                          \
    static hipError_t KNAME##_go(const PTYPE& p, int batch, const Twiddles& tw, hipStream_t s) {           \
        using V = typename cplx_of<R>::type;                                                               \
        dim3 grid, block;                                                                                  \
        size_t lds;                                                                                        \
        RowLaunch<Row<R, NX>>::shape(p.g.ny, &grid, &block, &lds, batch, row_families(p));                  \
        hipLaunchKernelGGL((KNAME<R, NX>), grid, block, lds, s, p, (const V*)tw.tn, (const V*)tw.tx);      \
        return hipGetLastError();                                                                          \
    }                                                                                                      \
    SBI_ROW_NX_SWITCH(KNAME, PTYPE)

// kernels with launch-plan variants: p.g.row_var picks the transform's
// radix and twiddle mode, p.g.row_rpw the rows per workgroup
// Only variants that compile without register spills are built: the sweep
// kernels (three workgroups per CU) take the cached twiddle powers in FP32
// only and radix-16 rows only at 512 points; the SA kernel takes both in
// FP32 from 512 points (radix 16 needs two radix-16 passes in the
// half-length row) and the cached powers in FP64 too, below 8192 points.
template <typename R, int NX, int VAR, bool SWEEP> constexpr bool row_var_built() {
    constexpr bool f32 = std::is_same<R, float>::value;
    if constexpr (VAR == 0) return true;
    if constexpr (VAR == 1) return f32 || (!SWEEP && NX < 8192);
    if constexpr (VAR == 2) return f32 && (SWEEP ? NX == 512 : NX >= 512);
    // radix 4 (4 values per thread): a row spans two or more wavefronts, so
    // its exchanges take workgroup barriers; from 256-point rows
    if constexpr (VAR == 3) return NX >= 256 && NX <= 4096;
    return false;
}
#define SBI_ROW_LAUNCH_VAR(KNAME, PTYPE, SWEEP)                                                            \
    template <typename R, int NX, int VAR>                                                                 \
    static hipError_t KNAME##_gv(const PTYPE& p, int batch, const Twiddles& tw, hipStream_t s) {           \
        if constexpr (!row_var_built<R, NX, VAR, SWEEP>()) {                                               \
            return hipErrorInvalidValue;                                                                   \
        } else {                                                                                           \
            using V = typename cplx_of<R>::type;                                                           \
            dim3 grid, block;                                                                              \
            size_t lds;                                                                                    \
            RowLaunch<RowVar<R, NX, VAR>>::shape(p.g.ny, &grid, &block, &lds, batch, row_families(p),      \
                                                 p.g.row_rpw);                                             \
            hipLaunchKernelGGL((KNAME<R, NX, VAR>), grid, block, lds, s, p, (const V*)tw.tn,               \
                               (const V*)tw.tx);                                                           \
            return hipGetLastError();                                                                      \
        }                                                                                                  \
    }                                                                                                      \
    template <typename R, int NX>                                                                          \
    static hipError_t KNAME##_go(const PTYPE& p, int batch, const Twiddles& tw, hipStream_t s) {           \
        switch (p.g.row_var) {                                                                             \
            case 0: return KNAME##_gv<R, NX, 0>(p, batch, tw, s);                                          \
            case 1: return KNAME##_gv<R, NX, 1>(p, batch, tw, s);                                          \
            case 2: return KNAME##_gv<R, NX, 2>(p, batch, tw, s);                                          \
            case 3: return KNAME##_gv<R, NX, 3>(p, batch, tw, s);                                          \
            default: return hipErrorInvalidValue;                                                          \
        }                                                                                                  \
    }                                                                                                      \
    SBI_ROW_NX_SWITCH(KNAME, PTYPE)

SBI_ROW_LAUNCH(k_row_fwd, RowFwdParams)
SBI_ROW_LAUNCH(k_row_inv, RowInvParams)
SBI_ROW_LAUNCH(k_row_setup, RowSetupParams)
SBI_ROW_LAUNCH_VAR(k_row_sweep, RowSweepParams, true)
SBI_ROW_LAUNCH_VAR(k_row_sweep_aa, RowSweepParams, true)
SBI_ROW_LAUNCH_VAR(k_row_sa, RowSaParams, false)
SBI_ROW_LAUNCH(k_row_nphi, RowNphiParams)
SBI_ROW_LAUNCH(k_row_nphi_tank, RowNphiParams)
SBI_ROW_LAUNCH(k_row_blend, RowBlendParams)
SBI_ROW_LAUNCH(k_row_feat, RowFeatParams)

template <typename R, int NY, int NACC, bool QB>
static hipError_t col_go(const ColParams& p, int batch, const Twiddles& tw, hipStream_t s) {
    using V = typename cplx_of<R>::type;
    using CF = ColCfg<R, NY, QB, NACC>;
    if (p.g.col_C != CF::C) return hipErrorInvalidValue;  // the layout was made for another tile
    dim3 block(CF::THREADS);
    dim3 grid(p.g.Kxp / CF::C, p.ngroup > 0 ? p.ngroup : 1, batch);
    const size_t lds = CF::lds_bytes(p.g.Ky);
    if (lds > kMaxLdsBytes) return hipErrorInvalidValue;
    if constexpr (NY == 1024 && QB && NACC <= 2) {
        if (p.ngroup <= 1) {
            const size_t lp = ColPairCfg::lds_bytes<R>(p.g.Ky);
            if (lp > kMaxLdsBytes) return hipErrorInvalidValue;
            hipLaunchKernelGGL((k_colp<R, NACC>), dim3(p.g.Kxp, 1, batch), dim3(ColPairCfg::THREADS), lp, s, p,
                               (const V*)tw.ty);
            return hipGetLastError();
        }
    }
    hipLaunchKernelGGL((k_col<R, NY, NACC, QB>), grid, block, lds, s, p, (const V*)tw.ty);
    return hipGetLastError();
}
template <typename R, int NY, bool QB>
static hipError_t col_acc_qb(const ColParams& p, int batch, const Twiddles& tw, hipStream_t s) {
    if (p.nacc <= 1) return col_go<R, NY, 1, QB>(p, batch, tw, s);
    if (p.nacc <= 2) return col_go<R, NY, 2, QB>(p, batch, tw, s);
    return col_go<R, NY, 4, QB>(p, batch, tw, s);
}
// the quarter-band variant serves grids of 128 or more rows whose kept band
// lies below NY/4
template <typename R, int NY>
static hipError_t col_acc(const ColParams& p, int batch, const Twiddles& tw, hipStream_t s) {
    if constexpr (NY >= 128) {
        if (p.g.qb) return col_acc_qb<R, NY, true>(p, batch, tw, s);
    }
    return col_acc_qb<R, NY, false>(p, batch, tw, s);
}
template <typename R>
static hipError_t col_ny(const ColParams& p, int batch, const Twiddles& tw, hipStream_t s) {
    switch (p.g.ny) {
        case 1: return col_acc<R, 1>(p, batch, tw, s);
        case 16: return col_acc<R, 16>(p, batch, tw, s);
        case 32: return col_acc<R, 32>(p, batch, tw, s);
        case 64: return col_acc<R, 64>(p, batch, tw, s);
        case 128: return col_acc<R, 128>(p, batch, tw, s);
        case 256: return col_acc<R, 256>(p, batch, tw, s);
        case 512: return col_acc<R, 512>(p, batch, tw, s);
        case 1024: return col_acc<R, 1024>(p, batch, tw, s);
        case 2048: return col_acc<R, 2048>(p, batch, tw, s);
        default: return hipErrorInvalidValue;
    }
}
// ---------------------------------------------------------------------------
// Learned history seed: per mode, the nonlinear part of the solve at RK stage
// s is predicted from the backward differences d_q of the last K fixed-step
// solves' parts (newest first) with complex weights w[P][s][b][q] of the
// mode's radial bin b = min(floor(|k| / dk), nb - 1); FP32 weights,
// arithmetic in FP64.
// ---------------------------------------------------------------------------
__device__ __forceinline__ int hist_bin(double k, double dk, int nb) {
    const double f = floor(k / dk);
    return f >= (double)(nb - 1) ? nb - 1 : (int)f;
}
__device__ __forceinline__ int hist_widx(int P, int s, int b, int q, int nb, int K) {
    return (((P * kHistStages + s) * nb + b) * K + q) * 2;
}
// backward differences of the history of part P at element o: d_q = sum_(j<=q) (-1)^j C(q, j) h_j
template <typename V>
__device__ __forceinline__ void hist_diffs(const HistParams& p, int P, long long o, double (&dr)[kHistTaps],
                                           double (&di)[kHistTaps]) {
    double hr[kHistTaps], hi[kHistTaps];
    for (int q = 0; q < p.K; ++q) {
        const V h = static_cast<const V*>(P == 0 ? p.hv[q] : p.hb[q])[o];
        hr[q] = (double)h.x;
        hi[q] = (double)h.y;
    }
    for (int q = 0; q < p.K; ++q) {
        double c = 1.0, ar = 0.0, ai = 0.0;  // c = (-1)^j C(q, j)
        for (int j = 0; j <= q; ++j) {
            ar += c * hr[j];
            ai += c * hi[j];
            c = -c * (double)(q - j) / (double)(j + 1);
        }
        dr[q] = ar;
        di[q] = ai;
    }
}

// pv/pb <- predictions of the V and phi_b parts (zero outside the kept modes)
template <typename R>
__global__ void k_hist_seed(const HistParams p) {
    using V = typename cplx_of<R>::type;
    const int mem = blockIdx.y;
    const long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= p.g.s_cmp) return;
    const long long o = mem * p.g.s_cmp + idx;
    const ModeGeo m = mode_geo(p.g, idx);
    const int nparts = p.vd ? 2 : 1;
    for (int P = 0; P < nparts; ++P) {
        double re = 0.0, im = 0.0;
        if (m.valid) {
            const int b = hist_bin(m.k, p.dk, p.nb);
            double dr[kHistTaps], di[kHistTaps];
            hist_diffs<V>(p, P, o, dr, di);
            for (int q = 0; q < p.K; ++q) {
                const int wi = hist_widx(P, p.stage, b, q, p.nb, p.K);
                const double wr = (double)p.dev->w[wi], wm = (double)p.dev->w[wi + 1];
                re += wr * dr[q] - wm * di[q];
                im += wr * di[q] + wm * dr[q];
            }
        }
        static_cast<V*>(P == 0 ? p.pv : p.pb)[o] = cx<V>(R(re), R(im));
    }
}

// history shift: h_q <- h_(q-1) for q = K-1 .. 1, h_0 <- the new entry
template <typename R>
__global__ void k_hist_push(const HistParams p) {
    using V = typename cplx_of<R>::type;
    const int mem = blockIdx.y;
    const long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= p.g.s_cmp) return;
    const long long o = mem * p.g.s_cmp + idx;
    const int nparts = p.vd ? 2 : 1;
    for (int P = 0; P < nparts; ++P) {
        void* const* h = P == 0 ? p.hv : p.hb;
        for (int q = p.K - 1; q >= 1; --q) static_cast<V*>(h[q])[o] = static_cast<const V*>(h[q - 1])[o];
        static_cast<V*>(h[0])[o] = static_cast<const V*>(P == 0 ? p.tv : p.tb)[o];
    }
}

// offsets of a member's per-block partials (layout for the pass's K and nb)
__device__ __forceinline__ int hist_part_tri(const HistParams& p) { return 2 * p.nb * p.K * 2; }
__device__ __forceinline__ int hist_part_ed(const HistParams& p) {
    return hist_part_tri(p) + 2 * p.nb * (p.K * (p.K + 1) / 2) * 2;
}

// loss gradient and Gram sums of predicting the target (tv, tb) from the
// history at stage s: per workgroup, S[P][b][q] = sum c conj(d_q) r,
// T[P][b][q <= r] = sum c conj(d_q) d_r, E_P = sum c |r|^2, D_P = sum c |y|^2
// over its modes (r = pred - y, c = 1 at m_x = 0 else 2), summed in LDS and
// written as the workgroup's partials
template <typename R>
__global__ void __launch_bounds__(256) k_hist_grad(const HistParams p) {
    using V = typename cplx_of<R>::type;
    __shared__ double acc[kHistPart];
    const int mem = blockIdx.y;
    const int oT = hist_part_tri(p), oE = hist_part_ed(p);
    const int ntri = p.K * (p.K + 1) / 2;
    for (int i = threadIdx.x; i < kHistPart; i += blockDim.x) acc[i] = 0.0;
    __syncthreads();
    const int nparts = p.vd ? 2 : 1;
    for (long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x; idx < p.g.s_cmp;
         idx += (long long)gridDim.x * blockDim.x) {
        const ModeGeo m = mode_geo(p.g, idx);
        if (!m.valid) continue;
        const long long o = mem * p.g.s_cmp + idx;
        const int b = hist_bin(m.k, p.dk, p.nb);
        const double c = m.mx == 0 ? 1.0 : 2.0;
        for (int P = 0; P < nparts; ++P) {
            const V y = static_cast<const V*>(P == 0 ? p.tv : p.tb)[o];
            double dr[kHistTaps], di[kHistTaps];
            hist_diffs<V>(p, P, o, dr, di);
            double re = 0.0, im = 0.0;
            for (int q = 0; q < p.K; ++q) {
                const int wi = hist_widx(P, p.stage, b, q, p.nb, p.K);
                const double wr = (double)p.dev->w[wi], wm = (double)p.dev->w[wi + 1];
                re += wr * dr[q] - wm * di[q];
                im += wr * di[q] + wm * dr[q];
            }
            const double rr = re - (double)y.x, ri = im - (double)y.y;
            atomicAdd(&acc[oE + P], c * (rr * rr + ri * ri));
            atomicAdd(&acc[oE + 2 + P], c * ((double)y.x * y.x + (double)y.y * y.y));
            int t = 0;
            for (int q = 0; q < p.K; ++q) {
                // conj(d_q) r
                const int si = ((P * p.nb + b) * p.K + q) * 2;
                atomicAdd(&acc[si], c * (dr[q] * rr + di[q] * ri));
                atomicAdd(&acc[si + 1], c * (dr[q] * ri - di[q] * rr));
                for (int r = q; r < p.K; ++r, ++t) {
                    // conj(d_q) d_r
                    const int ti = oT + ((P * p.nb + b) * ntri + t) * 2;
                    atomicAdd(&acc[ti], c * (dr[q] * dr[r] + di[q] * di[r]));
                    atomicAdd(&acc[ti + 1], c * (dr[q] * di[r] - di[q] * dr[r]));
                }
            }
        }
    }
    __syncthreads();
    double* out = p.partial + ((long long)mem * gridDim.x + blockIdx.x) * kHistPart;
    for (int i = threadIdx.x; i < kHistPart; i += blockDim.x) out[i] = acc[i];
}

// ---------------------------------------------------------------------------
// per-precision entry points (this file is compiled once per precision with
// SBI_REAL defined; sbi_dispatch.hip selects between them)
// ---------------------------------------------------------------------------
using Real = SBI_REAL;
template <> hipError_t launch_row_fwd_t<Real>(const RowFwdParams& p, int b, const Twiddles& tw, hipStream_t s) {
    return k_row_fwd_nx<Real>(p, b, tw, s);
}
template <> hipError_t launch_row_inv_t<Real>(const RowInvParams& p, int b, const Twiddles& tw, hipStream_t s) {
    return k_row_inv_nx<Real>(p, b, tw, s);
}
template <> hipError_t launch_row_setup_t<Real>(const RowSetupParams& p, int b, const Twiddles& tw, hipStream_t s) {
    return k_row_setup_nx<Real>(p, b, tw, s);
}
template <typename R, int NX, bool SWEEP> static int row_var_mask_nx() {
    return (row_var_built<R, NX, 0, SWEEP>() ? 1 : 0) | (row_var_built<R, NX, 1, SWEEP>() ? 2 : 0) |
           (row_var_built<R, NX, 2, SWEEP>() ? 4 : 0) | (row_var_built<R, NX, 3, SWEEP>() ? 8 : 0);
}
template <typename R, int NX> static int row_var_mask_k(int sweep) {
    return sweep ? row_var_mask_nx<R, NX, true>() : row_var_mask_nx<R, NX, false>();
}
template <> int row_var_mask_t<Real>(int sweep, int nx) {
    switch (nx) {
        case 16: return row_var_mask_k<Real, 16>(sweep);
        case 32: return row_var_mask_k<Real, 32>(sweep);
        case 64: return row_var_mask_k<Real, 64>(sweep);
        case 128: return row_var_mask_k<Real, 128>(sweep);
        case 256: return row_var_mask_k<Real, 256>(sweep);
        case 512: return row_var_mask_k<Real, 512>(sweep);
        case 1024: return row_var_mask_k<Real, 1024>(sweep);
        case 2048: return row_var_mask_k<Real, 2048>(sweep);
        case 4096: return row_var_mask_k<Real, 4096>(sweep);
        case 8192: return row_var_mask_k<Real, 8192>(sweep);
        default: return 0;
    }
}
template <> int row_rows_cap_t<Real>(int nx, int var) {
    // rows per workgroup that fill 256 threads (the launch bound)
    const int n = nx / 2;
    const int em = var == 2 ? 16 : (var == 3 ? 4 : 8);
    const int e = n >= em ? em : n;
    const int P = n / e;
    return P >= 256 ? 1 : 256 / P;
}
template <> hipError_t launch_row_sweep_t<Real>(const RowSweepParams& p, int b, const Twiddles& tw, hipStream_t s) {
    return p.gT ? k_row_sweep_aa_nx<Real>(p, b, tw, s) : k_row_sweep_nx<Real>(p, b, tw, s);
}
template <> hipError_t launch_row_sa_t<Real>(const RowSaParams& p, int b, const Twiddles& tw, hipStream_t s) {
    return k_row_sa_nx<Real>(p, b, tw, s);
}
template <> hipError_t launch_row_nphi_t<Real>(const RowNphiParams& p, int b, const Twiddles& tw, hipStream_t s) {
    return (p.wm_n > 0 || p.dmp_w > 0.0) ? k_row_nphi_tank_nx<Real>(p, b, tw, s) : k_row_nphi_nx<Real>(p, b, tw, s);
}
template <> hipError_t launch_row_blend_t<Real>(const RowBlendParams& p, int b, const Twiddles& tw, hipStream_t s) {
    return k_row_blend_nx<Real>(p, b, tw, s);
}
template <> hipError_t launch_row_feat_t<Real>(const RowFeatParams& p, int b, const Twiddles& tw, hipStream_t s) {
    return k_row_feat_nx<Real>(p, b, tw, s);
}
template <> hipError_t launch_col_t<Real>(const ColParams& p, int b, const Twiddles& tw, hipStream_t s) {
    return col_ny<Real>(p, b, tw, s);
}
template <> hipError_t launch_rk_t<Real>(const RkParams& p, int batch, hipStream_t s) {
    dim3 block(256), grid((unsigned)((p.g.s_cmp + 255) / 256), batch);
    hipLaunchKernelGGL(k_rk<Real>, grid, block, 0, s, p);
    return hipGetLastError();
}
template <> hipError_t launch_rk54_t<Real>(const Rk54Params& p, int batch, hipStream_t s) {
    // the last stage reduces over a fixed number of workgroups per member
    const unsigned nb = p.stage == 5 ? (unsigned)p.nblk : (unsigned)((p.g.s_cmp + 255) / 256);
    dim3 block(256), grid(nb, batch);
    hipLaunchKernelGGL(k_rk54<Real>, grid, block, 0, s, p);
    return hipGetLastError();
}
template <> hipError_t launch_aa_dot_t<Real>(const AaParams& p, int batch, hipStream_t s) {
    dim3 block(kAADotThreads), grid((unsigned)p.nblk, batch);
    hipLaunchKernelGGL(k_aa_dot<Real>, grid, block, 0, s, p);
    return hipGetLastError();
}
template <> hipError_t launch_hist_seed_t<Real>(const HistParams& p, int batch, hipStream_t s) {
    dim3 block(256), grid((unsigned)((p.g.s_cmp + 255) / 256), batch);
    hipLaunchKernelGGL(k_hist_seed<Real>, grid, block, 0, s, p);
    return hipGetLastError();
}
template <> hipError_t launch_hist_push_t<Real>(const HistParams& p, int batch, hipStream_t s) {
    dim3 block(256), grid((unsigned)((p.g.s_cmp + 255) / 256), batch);
    hipLaunchKernelGGL(k_hist_push<Real>, grid, block, 0, s, p);
    return hipGetLastError();
}
template <> hipError_t launch_hist_grad_t<Real>(const HistParams& p, int batch, hipStream_t s) {
    dim3 block(256), grid(kHistBlocks, batch);
    hipLaunchKernelGGL(k_hist_grad<Real>, grid, block, 0, s, p);
    return hipGetLastError();
}
template <> hipError_t launch_diag_t<Real>(const DiagParams& p, int batch, hipStream_t s) {
    dim3 block(256), grid(p.nblk, batch);
    hipLaunchKernelGGL(k_diag<Real>, grid, block, 0, s, p);
    return hipGetLastError();
}

}  // namespace sbi
