// sbi_dispatch.hip -- precision dispatch of the kernel launchers and the
// precision-independent control kernels.
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

}  // namespace sbi
