// sbi_dispatch.hip -- precision dispatch of the kernel launchers and the
// precision-independent control kernels.
#include "sbi_device.hpp"
#include "sbi_full.hpp"
#include "sbi_kernels.hpp"

namespace sbi {

// columns per column-pass workgroup (equals ColCfg<R, NY, QB, NACC>::C of the kernels;
// the launcher checks it)
int col_tile(int ny, int fp64, int qb) {
    if (ny == 1) return 64;
    if (qb && ny == 1024) return 1;  // one wavefront per column transform
    int e = (fp64 && !qb) ? 4 : 8;
    if (e > ny) e = ny;
    const int P = ny / e;
    return P >= 128 ? 1 : 256 / P;
}

int col_quarter_band(int ny, int My) { return (ny >= 128 && 4 * My < ny) ? 1 : 0; }

__global__ void k_ctl_reset(Ctl* ctl, int slots) {
    Ctl* c = ctl + blockIdx.x;
    CtlSlots* sl = c->slots;
    for (int i = threadIdx.x; i < slots; i += blockDim.x) {
        sl->num[i] = 0ull;
        sl->den[i] = 0ull;
    }
    if (threadIdx.x == 0) {
        c->eta_max = 0ull;
        c->eta_min = ~0ull;
        c->nonfinite = 0;
        c->done = 0;
        c->status = 0;
        c->sweeps = 0;
        c->sweeps_inner = 0;
        c->omega = 1.0;
        c->residual = 0.0;
        c->rmin = INFINITY;
    }
}

__global__ void k_ctl_acc_reset(Ctl* ctl) {
    Ctl* c = ctl + blockIdx.x;
    if (threadIdx.x == 0) {
        c->acc_solves = 0;
        c->acc_sweeps = 0;
        c->acc_sweeps_max = 0;
        c->acc_worst = 0;
        c->acc_residual_max = 0.0;
    }
}

hipError_t launch_ctl_acc_reset(Ctl* ctl, int batch, hipStream_t s) {
    hipLaunchKernelGGL(k_ctl_acc_reset, dim3(batch), dim3(64), 0, s, ctl);
    return hipGetLastError();
}

__global__ void k_fill_zero(uint4* p, size_t n16) {
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n16; i += (size_t)gridDim.x * blockDim.x)
        p[i] = make_uint4(0u, 0u, 0u, 0u);
}

// ---------------------------------------------------------------------------
// mixed precision (SBI_MIXED): the hand-over between the FP64 refinement of
// x = T(x) and the FP32 solve of its correction equation d = A d + r
// ---------------------------------------------------------------------------
// stopping decision after FP64 refinement sweep n (its residual norms in slot
// n - 1), with the rules of the plain iteration; the sweeps counted are the
// FP64 ones plus the FP32 correction sweeps so far
__global__ void k_ctl_decide(Ctl* ctl, int n, int M, double tol) {
    Ctl* c = ctl + blockIdx.x;
    if (threadIdx.x != 0 || c->done) return;
    double r, rmin;
    const int dec = sweep_decision(c, n, M, tol, &r, &rmin);
    if (dec) {
        ctl_commit(c, dec - 100, n + c->sweeps_inner, r);
    } else {
        c->rmin = rmin;
        c->residual = r;
    }
}

// FP64 residual r (compact spectra of its V and phi_b parts) -> forcing b and
// first iterate d = r of the FP32 correction solve (d = T_r(0)); the
// relaxation weight carries over, and members already decided stay decided.
// The n = Kx*Ky kept modes of a member come first in either layout (columns
// of Ky modes); so and si are the member strides of the FP64 and FP32 sides.
__global__ void k_mixed_down(const Ctl* outer, Ctl* inner, const double2* rv, const double2* rb, float2* bv,
                             float2* vn, float2* bb, float2* bn, long long n, long long so, long long si, int vd) {
    const int m = blockIdx.y;
    const Ctl* o = outer + m;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        inner[m].omega = o->omega;
        inner[m].done = o->done;
    }
    if (o->done) return;
    const long long oo = (long long)m * so, oi = (long long)m * si;
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x) {
        const double2 a = rv[oo + i];
        const float2 f = make_float2((float)a.x, (float)a.y);
        bv[oi + i] = f;
        vn[oi + i] = f;
        if (vd) {
            const double2 q = rb[oo + i];
            const float2 g = make_float2((float)q.x, (float)q.y);
            bb[oi + i] = g;
            bn[oi + i] = g;
        }
    }
}

// x += d (FP64 += FP32) for the members the correction solve ran for; a
// correction solve that failed (diverged, non-finite) ends the member's solve
// with its status after n FP64 sweeps
__global__ void k_mixed_up(Ctl* outer, const Ctl* inner, double2* vn, double2* bn, const float2* dv,
                           const float2* db, long long n, long long so, long long si, int vd, int nsweep) {
    const int m = blockIdx.y;
    const Ctl* in = inner + m;
    if (in->sweeps == 0) return;  // decided before this correction solve
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        Ctl* o = outer + m;
        o->sweeps_inner += in->sweeps;
        const int st = in->nonfinite ? -5 : in->status;
        if (st < 0) ctl_commit(o, st, nsweep + o->sweeps_inner, in->residual);
    }
    const long long oo = (long long)m * so, oi = (long long)m * si;
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x) {
        const float2 d = dv[oi + i];
        double2 x = vn[oo + i];
        x.x += (double)d.x;
        x.y += (double)d.y;
        vn[oo + i] = x;
        if (vd) {
            const float2 e = db[oi + i];
            double2 y = bn[oo + i];
            y.x += (double)e.x;
            y.y += (double)e.y;
            bn[oo + i] = y;
        }
    }
}

// the same update for the half forms the next row pass reads (they are
// linear in the iterate: half(x + d) = half(x) + half(d)); a half form holds
// column k < kx of row y at k * ldh + y, ldh and the member stride differ
// between the two sides; nf fields (V, d_x phi_b, d_y phi_b)
struct MixedHalf {
    double2* out[3];
    const float2* in[3];
    int nf, kx, ny, ldh_o, ldh_i;
    long long so, si;
};
__global__ void k_mixed_up_half(const Ctl* inner, const MixedHalf h) {
    const int m = blockIdx.y;
    if (inner[m].sweeps == 0) return;  // decided before this correction solve
    const long long n = (long long)h.kx * h.ny;
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x) {
        const long long k = i / h.ny, y = i - k * h.ny;
        const long long oo = m * h.so + k * h.ldh_o + y, oi = m * h.si + k * h.ldh_i + y;
        for (int f = 0; f < h.nf; ++f) {
            const float2 d = h.in[f][oi];
            double2 x = h.out[f][oo];
            x.x += (double)d.x;
            x.y += (double)d.y;
            h.out[f][oo] = x;
        }
    }
}

__global__ void k_to_float(const double* src, float* dst, long long n) {
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
        dst[i] = (float)src[i];
}

static unsigned elem_blocks(long long n) {
    long long nb = (n + 255) / 256;
    return (unsigned)(nb < 1 ? 1 : (nb > 1024 ? 1024 : nb));
}

hipError_t launch_ctl_decide(Ctl* ctl, int batch, int n, int M, double tol, hipStream_t s) {
    hipLaunchKernelGGL(k_ctl_decide, dim3(batch), dim3(64), 0, s, ctl, n, M, tol);
    return hipGetLastError();
}

hipError_t launch_mixed_down(const Ctl* outer, Ctl* inner, int batch, const void* rv, const void* rb, void* bv,
                             void* vn, void* bb, void* bn, long long n, long long so, long long si, int vd,
                             hipStream_t s) {
    hipLaunchKernelGGL(k_mixed_down, dim3(elem_blocks(n), batch), dim3(256), 0, s, outer, inner,
                       static_cast<const double2*>(rv), static_cast<const double2*>(rb), static_cast<float2*>(bv),
                       static_cast<float2*>(vn), static_cast<float2*>(bb), static_cast<float2*>(bn), n, so, si, vd);
    return hipGetLastError();
}

hipError_t launch_mixed_up(Ctl* outer, const Ctl* inner, int batch, void* vn, void* bn, const void* dv,
                           const void* db, long long n, long long so, long long si, int vd, int nsweep,
                           hipStream_t s) {
    hipLaunchKernelGGL(k_mixed_up, dim3(elem_blocks(n), batch), dim3(256), 0, s, outer, inner,
                       static_cast<double2*>(vn), static_cast<double2*>(bn), static_cast<const float2*>(dv),
                       static_cast<const float2*>(db), n, so, si, vd, nsweep);
    return hipGetLastError();
}

hipError_t launch_mixed_up_half(const Ctl* inner, int batch, void* const* out, const void* const* in, int nf, int kx,
                                int ny, int ldh_o, int ldh_i, long long so, long long si, hipStream_t s) {
    MixedHalf h{};
    for (int f = 0; f < nf && f < 3; ++f) {
        h.out[f] = static_cast<double2*>(out[f]);
        h.in[f] = static_cast<const float2*>(in[f]);
    }
    h.nf = nf < 3 ? nf : 3;
    h.kx = kx;
    h.ny = ny;
    h.ldh_o = ldh_o;
    h.ldh_i = ldh_i;
    h.so = so;
    h.si = si;
    hipLaunchKernelGGL(k_mixed_up_half, dim3(elem_blocks((long long)kx * ny), batch), dim3(256), 0, s, inner, h);
    return hipGetLastError();
}

hipError_t launch_to_float(const void* src, void* dst, long long n, hipStream_t s) {
    hipLaunchKernelGGL(k_to_float, dim3(elem_blocks(n)), dim3(256), 0, s, static_cast<const double*>(src),
                       static_cast<float*>(dst), n);
    return hipGetLastError();
}

hipError_t launch_ctl_reset(Ctl* ctl, int batch, int slots, hipStream_t s) {
    hipLaunchKernelGGL(k_ctl_reset, dim3(batch), dim3(256), 0, s, ctl, slots);
    return hipGetLastError();
}

hipError_t launch_fill_zero(void* ptr, size_t bytes, hipStream_t s) {
    const size_t n16 = bytes / 16;
    if (n16 == 0) return hipSuccess;
    unsigned nb = (unsigned)((n16 + 255) / 256);
    if (nb > 4096) nb = 4096;
    hipLaunchKernelGGL(k_fill_zero, dim3(nb), dim3(256), 0, s, (uint4*)ptr, n16);
    return hipGetLastError();
}

#define SBI_DISPATCH(NAME, PTYPE)                                                                   \
    hipError_t NAME(int fp64, const PTYPE& p, int b, const Twiddles& tw, hipStream_t s) {           \
        return fp64 ? NAME##_t<double>(p, b, tw, s) : NAME##_t<float>(p, b, tw, s);                 \
    }
SBI_DISPATCH(launch_row_fwd, RowFwdParams)
SBI_DISPATCH(launch_row_inv, RowInvParams)
SBI_DISPATCH(launch_row_setup, RowSetupParams)
SBI_DISPATCH(launch_row_sweep, RowSweepParams)
SBI_DISPATCH(launch_row_sa, RowSaParams)
SBI_DISPATCH(launch_row_nphi, RowNphiParams)
SBI_DISPATCH(launch_row_blend, RowBlendParams)
SBI_DISPATCH(launch_row_feat, RowFeatParams)
SBI_DISPATCH(launch_col, ColParams)

hipError_t launch_full(int fp64, const FullParams& p, int what, hipStream_t s) {
    return fp64 ? launch_full_t<double>(p, what, s) : launch_full_t<float>(p, what, s);
}
int row_var_mask(int fp64, int sweep, int nx) {
    return fp64 ? row_var_mask_t<double>(sweep, nx) : row_var_mask_t<float>(sweep, nx);
}
int row_rows_cap(int fp64, int nx, int var) {
    return fp64 ? row_rows_cap_t<double>(nx, var) : row_rows_cap_t<float>(nx, var);
}

hipError_t launch_rk(int fp64, const RkParams& p, int batch, hipStream_t s) {
    return fp64 ? launch_rk_t<double>(p, batch, s) : launch_rk_t<float>(p, batch, s);
}
hipError_t launch_rk54(int fp64, const Rk54Params& p, int batch, hipStream_t s) {
    return fp64 ? launch_rk54_t<double>(p, batch, s) : launch_rk54_t<float>(p, batch, s);
}
hipError_t launch_aa_dot(int fp64, const AaParams& p, int batch, hipStream_t s) {
    return fp64 ? launch_aa_dot_t<double>(p, batch, s) : launch_aa_dot_t<float>(p, batch, s);
}
hipError_t launch_diag(int fp64, const DiagParams& p, int batch, hipStream_t s) {
    return fp64 ? launch_diag_t<double>(p, batch, s) : launch_diag_t<float>(p, batch, s);
}
hipError_t launch_hist_seed(int fp64, const HistParams& p, int batch, hipStream_t s) {
    return fp64 ? launch_hist_seed_t<double>(p, batch, s) : launch_hist_seed_t<float>(p, batch, s);
}
hipError_t launch_hist_push(int fp64, const HistParams& p, int batch, hipStream_t s) {
    return fp64 ? launch_hist_push_t<double>(p, batch, s) : launch_hist_push_t<float>(p, batch, s);
}
hipError_t launch_hist_grad(int fp64, const HistParams& p, int batch, hipStream_t s) {
    return fp64 ? launch_hist_grad_t<double>(p, batch, s) : launch_hist_grad_t<float>(p, batch, s);
}

// Gradient and Gram accumulation of the history layer: per entry (thread),
// the sums of the members' workgroup partials in a fixed order, each member's
// parts normalised by its D_P (parts with D_P = 0 contribute nothing), added
// into the accumulators of the pass's stage (Gram triangles expanded to the
// full Hermitian matrices); the loss and sample counts likewise.
__global__ void k_hist_reduce(const HistParams p, int batch) {
    const int K = p.K, nb = p.nb;
    const int ntri = K * (K + 1) / 2;
    const int nS = 2 * nb * K * 2;
    const int oT = nS, oE = nS + 2 * nb * ntri * 2;
    const int nall = nS + 2 * nb * ntri * 2;
    for (int e = threadIdx.x; e < nall; e += blockDim.x) {
        const bool tri = e >= oT;
        const int f = tri ? e - oT : e;
        const int P = tri ? f / (nb * ntri * 2) : f / (nb * K * 2);
        double tot = 0.0;
        for (int mem = 0; mem < batch; ++mem) {
            const double* base = p.partial + (long long)mem * kHistBlocks * kHistPart;
            double S = 0.0, D = 0.0;
            for (int blk = 0; blk < kHistBlocks; ++blk) {
                S += base[blk * kHistPart + e];
                D += base[blk * kHistPart + oE + 2 + P];
            }
            if (D > 0.0) tot += S / D;
        }
        if (!tri) {
            const int rest = f % (nb * K * 2);
            const int b = rest / (K * 2), q = (rest / 2) % K, ri = rest & 1;
            p.dev->acc[(((P * kHistStages + p.stage) * nb + b) * K + q) * 2 + ri] += 2.0 * tot;
        } else {
            const int rest = f % (nb * ntri * 2);
            const int b = rest / (ntri * 2), t = (rest / 2) % ntri, ri = rest & 1;
            int q = 0, rem = t;
            while (rem >= K - q) {
                rem -= K - q;
                ++q;
            }
            const int r = q + rem;
            const long long base = ((long long)(P * kHistStages + p.stage) * nb + b) * K * K;
            p.dev->gram[(base + q * K + r) * 2 + ri] += tot;
            if (r != q) p.dev->gram[(base + r * K + q) * 2 + ri] += ri ? -tot : tot;  // conj
        }
    }
    if (threadIdx.x == 0) {
        for (int mem = 0; mem < batch; ++mem) {
            const double* base = p.partial + (long long)mem * kHistBlocks * kHistPart;
            for (int P = 0; P < (p.vd ? 2 : 1); ++P) {
                double E = 0.0, D = 0.0;
                for (int blk = 0; blk < kHistBlocks; ++blk) {
                    E += base[blk * kHistPart + oE + P];
                    D += base[blk * kHistPart + oE + 2 + P];
                }
                if (D > 0.0) p.dev->loss += E / D;
            }
            p.dev->samples += 1.0;
        }
    }
}

hipError_t launch_hist_reduce(const HistParams& p, int batch, hipStream_t s) {
    hipLaunchKernelGGL(k_hist_reduce, dim3(1), dim3(1024), 0, s, p, batch);
    return hipGetLastError();
}

// clear the accumulators and leave (mean loss, samples) of what they held in
// dev->out (a single workgroup; every thread has read what it needs)
__device__ __forceinline__ void hist_clear(HistDev* d, int np, int ng, double n) {
    for (int i = threadIdx.x; i < np; i += blockDim.x) d->acc[i] = 0.0;
    for (int i = threadIdx.x; i < ng; i += blockDim.x) d->gram[i] = 0.0;
    __syncthreads();
    if (threadIdx.x == 0) {
        d->out[0] = n > 0.0 ? d->loss / n : 0.0;
        d->out[1] = n;
        d->loss = 0.0;
        d->samples = 0.0;
    }
}

// Gauss-Newton step of the layer: per (part, stage, bin) system (one thread
// each), w <- w - (G + lam tr(G)/K I)^-1 gamma with G the accumulated Gram
// matrix and gamma = acc/2 the complex derivative, by a complex Cholesky
// factorisation; systems with tr(G) = 0 (no samples) keep their weights.
__global__ void k_hist_newton(const HistParams p, double lam) {
    HistDev* d = p.dev;
    const int K = p.K, nb = p.nb;
    const double n = d->samples;
    const int nsys = 2 * kHistStages * nb;
    for (int sys = threadIdx.x; sys < nsys && n > 0.0; sys += blockDim.x) {
        const double* G = d->gram + (long long)sys * K * K * 2;
        double tr = 0.0;
        for (int q = 0; q < K; ++q) tr += G[(q * K + q) * 2];
        if (!(tr > 0.0)) continue;
        // lower factor L (complex), A = L L^H
        double Lr[kHistTaps][kHistTaps], Li[kHistTaps][kHistTaps];
        bool ok = true;
        for (int i = 0; i < K && ok; ++i) {
            for (int j = 0; j <= i; ++j) {
                // A_ij - sum_k L_ik conj(L_jk)
                double ar = G[(i * K + j) * 2] + (i == j ? lam * tr / K : 0.0);
                double ai = G[(i * K + j) * 2 + 1];
                for (int k = 0; k < j; ++k) {
                    ar -= Lr[i][k] * Lr[j][k] + Li[i][k] * Li[j][k];
                    ai -= Li[i][k] * Lr[j][k] - Lr[i][k] * Li[j][k];
                }
                if (i == j) {
                    if (!(ar > 0.0)) {
                        ok = false;
                        break;
                    }
                    Lr[i][i] = sqrt(ar);
                    Li[i][i] = 0.0;
                } else {
                    Lr[i][j] = ar / Lr[j][j];
                    Li[i][j] = ai / Lr[j][j];
                }
            }
        }
        if (!ok) continue;
        // gamma = acc / 2; solve L y = gamma, then L^H x = y
        const int w0 = sys * K * 2;
        double yr[kHistTaps], yi[kHistTaps];
        for (int i = 0; i < K; ++i) {
            double br = 0.5 * d->acc[w0 + 2 * i], bi = 0.5 * d->acc[w0 + 2 * i + 1];
            for (int k = 0; k < i; ++k) {
                br -= Lr[i][k] * yr[k] - Li[i][k] * yi[k];
                bi -= Lr[i][k] * yi[k] + Li[i][k] * yr[k];
            }
            yr[i] = br / Lr[i][i];
            yi[i] = bi / Lr[i][i];
        }
        for (int i = K - 1; i >= 0; --i) {
            double br = yr[i], bi = yi[i];
            for (int k = i + 1; k < K; ++k) {
                // conj(L_ki) x_k
                br -= Lr[k][i] * yr[k] + Li[k][i] * yi[k];
                bi -= Lr[k][i] * yi[k] - Li[k][i] * yr[k];
            }
            yr[i] = br / Lr[i][i];
            yi[i] = bi / Lr[i][i];
        }
        for (int i = 0; i < K; ++i) {
            d->w[w0 + 2 * i] = (float)((double)d->w[w0 + 2 * i] - yr[i]);
            d->w[w0 + 2 * i + 1] = (float)((double)d->w[w0 + 2 * i + 1] - yi[i]);
        }
    }
    __syncthreads();
    hist_clear(d, 2 * kHistStages * nb * K * 2, 2 * kHistStages * nb * K * K * 2, n);
}

hipError_t launch_hist_newton(const HistParams& p, double lam, hipStream_t s) {
    hipLaunchKernelGGL(k_hist_newton, dim3(1), dim3(256), 0, s, p, lam);
    return hipGetLastError();
}

// One Adam step (beta1 0.9, beta2 0.999, eps 1e-8, bias-corrected) of the
// layer's weights with the mean accumulated gradient; clears the accumulator
// and leaves (mean loss, samples) in dev->out.  A single workgroup.
__global__ void k_hist_adam(const HistParams p) {
    HistDev* d = p.dev;
    const double n = d->samples;
    const int t = d->adam_t + 1;
    const int np = 2 * kHistStages * p.nb * p.K * 2;
    if (n > 0.0) {
        const double b1 = 0.9, b2 = 0.999, eps = 1e-8;
        const double c1 = 1.0 - pow(b1, (double)t), c2 = 1.0 - pow(b2, (double)t);
        for (int i = threadIdx.x; i < np; i += blockDim.x) {
            const double g = d->acc[i] / n;
            const double m = b1 * d->m[i] + (1.0 - b1) * g;
            const double v = b2 * d->v[i] + (1.0 - b2) * g * g;
            d->m[i] = m;
            d->v[i] = v;
            d->w[i] = (float)((double)d->w[i] - p.lr * (m / c1) / (sqrt(v / c2) + eps));
        }
    }
    __syncthreads();
    if (threadIdx.x == 0 && n > 0.0) d->adam_t = t;
    hist_clear(d, np, 2 * kHistStages * p.nb * p.K * p.K * 2, n);
}

hipError_t launch_hist_adam(const HistParams& p, hipStream_t s) {
    hipLaunchKernelGGL(k_hist_adam, dim3(1), dim3(1024), 0, s, p);
    return hipGetLastError();
}

}  // namespace sbi
