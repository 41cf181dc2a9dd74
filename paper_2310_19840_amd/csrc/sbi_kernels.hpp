// sbi_kernels.hpp -- parameter blocks of the row passes and pointwise kernels,
// and the size-dispatching launch functions implemented in sbi_kernels.hip.
#pragma once
#include <hip/hip_runtime.h>
#include "sbi_internal.hpp"

namespace sbi {

struct RowFwdParams {
    GridDev g;
    int nf;
    const void* in[4];   // physical [ny][nx]
    void* out[4];        // half form
};

struct RowInvParams {
    GridDev g;
    int nf;
    const void* in[8];   // half form
    const void* in2[8];  // optional second half form added with (1 - omega)
    void* out[8];        // physical
    Ctl* ctl;
};

struct RowSetupParams {
    GridDev g;
    const void* g_eta;        // half form of eta (or null when eta_in is given)
    const void* eta_in;       // physical eta given by the caller (or null)
    void* eta_out;            // physical eta written (may be null when eta_in)
    const void* g_px;         // half forms of the potential gradient
    const void* g_py;
    void* px_out;             // physical gradient (SA mode), may be null
    void* py_out;
    int nprod;                // forcing products eta^(l-1) grad phi, l = 2..L
    void* h[kMaxProd];
    Ctl* ctl;
    int nfam;                 // 2: the x and y components in workgroups of their own (blockIdx.y)
};

struct RowSweepParams {
    GridDev g;
    const void* gV;     // half form of the current iterate V_n
    const void* gD;     // half form of D_(n-1) = T(V_(n-1)) - V_(n-1)
    const void* gT;     // half form of T(V_(n-1)) (Anderson mixing; NULL: V_n + (1 - omega) D_(n-1))
    const void* gbx;    // half forms of grad phi_b,n (variable depth)
    const void* gby;
    const void* eta;    // physical
    const void* delta;  // physical
    int J;              // convolution orders of the sweep
    int residual;       // compute the residual of the previous sweep into slot
    int products;       // form the products of this sweep
    int vd;             // variable depth
    int slot;
    int nfam;           // workgroups along y: 0 eta^j V (+ residual), 1/2 delta^j d_x/d_y phi_b
    void* h[kMaxProd];
    Ctl* ctl;
};

struct RowSaParams {
    GridDev g;
    int l;              // order being formed
    int vd;
    const void* gV;     // half form of V_(l-1)
    const void* gbx;    // half forms of grad phi_b,(l-1) (vd and l-1 <= L-1)
    const void* gby;
    void* V_out;        // physical V_(l-1) (kept for higher orders), may be null
    void* bx_out;
    void* by_out;
    const void* Vphys[8];   // physical V_m, m < l-1
    const void* bxphys[8];
    const void* byphys[8];
    const void* eta;
    const void* delta;
    const void* phx;    // physical grad phi_s
    const void* phy;
    void* h[kMaxProd];
    int split;          // > 0: workgroups per row block, one product each (blockIdx.y)
};

constexpr int kMaxWavemaker = 8;   // pneumatic wavemaker components

struct RowNphiParams {
    GridDev g;
    const void* gV;
    const void* gD;     // optional: V' = V + (1-omega) D
    const void* gex;
    const void* gey;
    const void* gpx;
    const void* gpy;
    void* h;
    Ctl* ctl;
    // surface pressure of the wave tank (Sec. 3.2), subtracted in the dynamic condition
    int wm_n;                       // wavemaker components (0: none)
    double wm[kMaxWavemaker][4];    // a_j, k_j, omega_j, theta_j
    double wm_h;                    // depth of the generator's factor (<= 0: the member's reference depth)
    double t;                       // stage time
    double dmp_x0, dmp_w;           // damping weight exp(-((x - x0)/w)^2) (periodic distance); w <= 0: none
    void* hdx;                      // forward half forms of mu d_x phi, mu d_y phi (damping only)
    void* hdy;
};

// features of the learned warm start (channel-last, FP32, scaled per channel):
// (eta, W_lin, d_x eta, d_y eta, d_x phi, d_y phi, delta, eta * W_lin)
struct RowFeatParams {
    GridDev g;
    const void* gV;     // half form of W_lin = F^-1{k tanh(kh) phi_hat}
    const void* gex;    // half forms of grad eta
    const void* gey;
    const void* gpx;    // half forms of grad phi
    const void* gpy;
    const void* eta;    // physical eta as the solve sees it
    const void* delta;  // physical delta
    float scale[8];
    float* feat;        // [batch][ny][nx][8]
    void* wlin;         // physical W_lin, optional
};

struct RowBlendParams {
    GridDev g;
    const void* ge;
    const void* gp;
    void* he;
    void* hp;
    double a, k, om, gen, absl, ramp_time, t;
};

struct RkParams {
    GridDev g;
    int stage;
    double h;
    void* eh;        // u_n (updated at stage 3)
    void* ph;
    void* es;        // stage state in / next stage state out
    void* ps;
    const void* Vh;  // W spectrum at the stage state
    const void* Nph; // nonlinear term of the potential equation
    const void* Pdiv;// optional: i k . MF{mu grad phi} of the damping pressure (added as Pdiv / k^2)
    void* ae;        // accumulator
    void* ap;
    double fb1, fb2; // filter
};

// one stage of the embedded fifth/fourth-order pair in integrating-factor form
struct Rk54Params {
    GridDev g;
    int stage;       // 0..5: the stage whose W and N_phi are given
    double h;
    const void* eh;  // u_n
    const void* ph;
    void* es;        // stage state in / next stage state out (the fifth-order candidate after stage 5)
    void* ps;
    const void* Vh;  // W spectrum at the stage state
    const void* Nph; // nonlinear term of the potential equation at the stage state
    const void* Pdiv;// optional: i k . MF{mu grad phi} of the damping pressure (added as Pdiv / k^2)
    void* ke[6];     // stage derivatives carried back to t_n (written at their stage, read after)
    void* kp[6];
    double fb1, fb2; // filter (applied to the candidate)
    double* partial; // [batch][nblk][2]: error and state norms (stage 5)
    int nblk;
};

// Anderson mixing of the relaxed sweep (iteration mode): partial inner
// products of the residual history (k_aa_dot), which the next column pass
// turns into the weights of the next iterate
struct AaParams {
    GridDev g;
    Ctl* ctl;
    int sweep;                 // n
    int vd;                    // phi_b is iterated too (variable bed)
    const void* fv[kAASlots];  // residual history f_i = T(x_i) - x_i (V and phi_b parts)
    const void* fb[kAASlots];
    double* partial;           // [batch][nblk][kAASlots]
    int nblk;
};

// learned history seed: prediction, history push, loss gradient, reduction, Adam
struct HistParams {
    GridDev g;
    int K, nb, stage, vd;
    double dk;                      // radial bin width: bin = min(floor(|k| / dk), nb - 1)
    HistDev* dev;                   // weights, moments, accumulators
    void* hv[kHistTaps];            // history of the V part, newest first (compact)
    void* hb[kHistTaps];            // history of the phi_b part
    const void* tv;                 // new entry / target: V part (compact)
    const void* tb;                 //   phi_b part
    void* pv;                       // prediction out (compact)
    void* pb;
    double* partial;                // [batch][kHistBlocks][kHistPart]
    double lr;                      // Adam step size
};

struct DiagParams {
    GridDev g;
    const void* eh;
    const void* ph;
    const void* Vh;
    double* partial;  // [batch][nblk][2]
    int nblk;
};


struct Twiddles {
    const void* tx;   // length nx
    const void* tn;   // length nx/2
    const void* ty;   // length ny
};

int col_tile(int ny, int fp64, int qb);   // column-tile width C for a grid
int col_quarter_band(int ny, int My);     // 1 if the quarter-band column pass applies

// per-precision launchers (defined in sbi_kernels.hip, one object per precision)
template <typename R> hipError_t launch_row_fwd_t(const RowFwdParams&, int, const Twiddles&, hipStream_t);
template <typename R> hipError_t launch_row_inv_t(const RowInvParams&, int, const Twiddles&, hipStream_t);
template <typename R> hipError_t launch_row_setup_t(const RowSetupParams&, int, const Twiddles&, hipStream_t);
template <typename R> hipError_t launch_row_sweep_t(const RowSweepParams&, int, const Twiddles&, hipStream_t);
template <typename R> hipError_t launch_row_sa_t(const RowSaParams&, int, const Twiddles&, hipStream_t);
template <typename R> hipError_t launch_row_nphi_t(const RowNphiParams&, int, const Twiddles&, hipStream_t);
template <typename R> hipError_t launch_row_blend_t(const RowBlendParams&, int, const Twiddles&, hipStream_t);
template <typename R> hipError_t launch_row_feat_t(const RowFeatParams&, int, const Twiddles&, hipStream_t);
template <typename R> hipError_t launch_col_t(const ColParams&, int, const Twiddles&, hipStream_t);
template <typename R> hipError_t launch_rk_t(const RkParams&, int, hipStream_t);
template <typename R> hipError_t launch_rk54_t(const Rk54Params&, int, hipStream_t);
template <typename R> hipError_t launch_aa_dot_t(const AaParams&, int, hipStream_t);
template <typename R> hipError_t launch_diag_t(const DiagParams&, int, hipStream_t);
template <typename R> hipError_t launch_hist_seed_t(const HistParams&, int, hipStream_t);
template <typename R> hipError_t launch_hist_push_t(const HistParams&, int, hipStream_t);
template <typename R> hipError_t launch_hist_grad_t(const HistParams&, int, hipStream_t);
// launch-plan variants of the row sweep (sweep = 1) or SA (sweep = 0) kernels
// built for a row length: bit v set when variant v is available
template <typename R> int row_var_mask_t(int sweep, int nx);
// rows per workgroup of a row variant at its 256-thread launch bound
template <typename R> int row_rows_cap_t(int nx, int var);
int row_var_mask(int fp64, int sweep, int nx);
int row_rows_cap(int fp64, int nx, int var);

hipError_t launch_row_fwd(int fp64, const RowFwdParams& p, int batch, const Twiddles& tw, hipStream_t s);
hipError_t launch_row_inv(int fp64, const RowInvParams& p, int batch, const Twiddles& tw, hipStream_t s);
hipError_t launch_row_setup(int fp64, const RowSetupParams& p, int batch, const Twiddles& tw, hipStream_t s);
hipError_t launch_row_sweep(int fp64, const RowSweepParams& p, int batch, const Twiddles& tw, hipStream_t s);
hipError_t launch_row_sa(int fp64, const RowSaParams& p, int batch, const Twiddles& tw, hipStream_t s);
hipError_t launch_row_nphi(int fp64, const RowNphiParams& p, int batch, const Twiddles& tw, hipStream_t s);
hipError_t launch_row_blend(int fp64, const RowBlendParams& p, int batch, const Twiddles& tw, hipStream_t s);
hipError_t launch_row_feat(int fp64, const RowFeatParams& p, int batch, const Twiddles& tw, hipStream_t s);
hipError_t launch_col(int fp64, const ColParams& p, int batch, const Twiddles& tw, hipStream_t s);
hipError_t launch_rk(int fp64, const RkParams& p, int batch, hipStream_t s);
hipError_t launch_rk54(int fp64, const Rk54Params& p, int batch, hipStream_t s);
hipError_t launch_aa_dot(int fp64, const AaParams& p, int batch, hipStream_t s);
hipError_t launch_diag(int fp64, const DiagParams& p, int batch, hipStream_t s);
hipError_t launch_hist_seed(int fp64, const HistParams& p, int batch, hipStream_t s);
hipError_t launch_hist_push(int fp64, const HistParams& p, int batch, hipStream_t s);
hipError_t launch_hist_grad(int fp64, const HistParams& p, int batch, hipStream_t s);
hipError_t launch_hist_reduce(const HistParams& p, int batch, hipStream_t s);
hipError_t launch_hist_adam(const HistParams& p, hipStream_t s);
hipError_t launch_hist_newton(const HistParams& p, double lam, hipStream_t s);
hipError_t launch_ctl_reset(Ctl* ctl, int batch, int slots, hipStream_t s);
hipError_t launch_fill_zero(void* ptr, size_t bytes, hipStream_t s);
hipError_t launch_ctl_acc_reset(Ctl* ctl, int batch, hipStream_t s);
// mixed precision: decision of an FP64 refinement sweep, the hand-over of its
// residual to the FP32 correction solve (rv, rb FP64 compact -> bv, vn, bb, bn
// FP32 compact; the n kept modes per member, member strides so (FP64) and si
// (FP32)), the FP64 update x += d, and eta -> FP32
hipError_t launch_ctl_decide(Ctl* ctl, int batch, int n, int M, double tol, hipStream_t s);
hipError_t launch_mixed_down(const Ctl* outer, Ctl* inner, int batch, const void* rv, const void* rb, void* bv,
                             void* vn, void* bb, void* bn, long long n, long long so, long long si, int vd,
                             hipStream_t s);
hipError_t launch_mixed_up(Ctl* outer, const Ctl* inner, int batch, void* vn, void* bn, const void* dv,
                           const void* db, long long n, long long so, long long si, int vd, int nsweep,
                           hipStream_t s);
hipError_t launch_mixed_up_half(const Ctl* inner, int batch, void* const* out, const void* const* in, int nf, int kx,
                                int ny, int ldh_o, int ldh_i, long long so, long long si, hipStream_t s);
hipError_t launch_to_float(const void* src, void* dst, long long n, hipStream_t s);

}  // namespace sbi
