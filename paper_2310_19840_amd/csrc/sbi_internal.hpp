// sbi_internal.hpp -- structures shared by the host orchestration and the
// gfx950 kernels of the SBI solver.
//
// Spectral layouts (per batch member), complex values of the run precision,
// both column-major so a column pass reads and writes contiguous runs:
//   half form  [Kxp][ldh] : x transformed (kept m_x = 0..Mx), y physical;
//                           ldh = ny + pad, so columns do not all start on the
//                           same memory channel.
//                           Row-pass output / column-pass input ("H" and "G");
//                           row passes stage rows through LDS to access it in
//                           segments of several consecutive y.
//   compact    [Kxp][Ky]  : both axes transformed, only the kept rectangle
//                           |m_x| <= Mx, |m_y| <= My.  Entry r holds m_y = r for
//                           r <= My and m_y = r - Ky for r > My.
// Kx = Mx + 1 and Kxp rounds Kx up to the column-tile width; Ky = 2 My + 1
// (1 when ny == 1).  Every spectrum of the method lives inside the kept
// rectangle, so the compact form is exact, not an approximation.
#pragma once
#include <stdint.h>

namespace sbi {

constexpr int kMaxSweepSlots = 1024;   // max_sweeps <= 1000
constexpr int kMaxProd = 24;           // forward inputs of one column pass
constexpr int kMaxCin = 8;             // compact inputs of one column pass
constexpr int kMaxTerms = 48;
constexpr int kMaxCout = 6;
constexpr int kMaxInv = 8;
constexpr int kMaxGroups = 8;          // product groups of one column pass
constexpr int kMaxTiles = 4096;        // column tiles per member (ticket counters)
constexpr size_t kMaxLdsBytes = 160 * 1024;  // LDS of one gfx950 workgroup

// Per-member control block in device memory: a small header the host reads
// for all members with one contiguous copy, plus a pointer to the member's
// residual slots.
struct CtlSlots {
    unsigned long long num[kMaxSweepSlots];  // bits of max|W'-W| (non-negative doubles)
    unsigned long long den[kMaxSweepSlots];  // bits of max|W'|
};
constexpr int kAADepth = 2;              // residual differences kept by the Anderson mixing
constexpr int kAASlots = kAADepth + 1;   // history ring of residuals and relaxed sweeps
constexpr int kAADotThreads = 512;       // threads of an inner-product workgroup (<= 1024)

// Learned history seed (a spectral layer of the learned warm start): the
// nonlinear part of a fixed-step solve at RK stage s is predicted from the
// backward differences d_q = sum_(j<=q) (-1)^j C(q, j) h_j of those of the K
// solves before it (h_0 newest), pred(k) = sum_q w[P][s][bin(|k|)][q] d_q(k),
// with complex weights per part P (V, phi_b), stage, radial bin and order.
constexpr int kHistTaps = 8;                                   // K <= kHistTaps
constexpr int kHistBins = 32;                                  // nb <= kHistBins
constexpr int kHistStages = 4;
constexpr int kHistParams = 2 * kHistStages * kHistBins * kHistTaps * 2;  // FP32 values, [P][s][b][q][re,im]
constexpr int kHistTri = kHistTaps * (kHistTaps + 1) / 2;       // upper triangle of a K x K Gram matrix
constexpr int kHistGram = 2 * kHistStages * kHistBins * kHistTaps * kHistTaps * 2;  // [P][s][b][q][r][re,im]
constexpr int kHistBlocks = 64;                                // workgroups per member of the gradient pass
// per-block partials of one member's gradient pass (layout for K, nb):
// S[P][b][q] (re, im) = sum c conj(d_q) r, the Gram triangles
// T[P][b][q <= r] (re, im) = sum c conj(d_q) d_r, then E_P = sum c |r|^2 and
// D_P = sum c |y|^2 for both parts
constexpr int kHistPart = 2 * kHistBins * kHistTaps * 2 + 2 * kHistBins * kHistTri * 2 + 4;
// weights, optimiser state and accumulators of the layer (device)
struct HistDev {
    float w[kHistParams];
    double m[kHistParams], v[kHistParams];  // Adam moments
    double acc[kHistParams];   // gradient sums over the accumulated solves
    double gram[kHistGram];    // Gram sums (full Hermitian matrices)
    double loss;               // loss sum
    double samples;            // solves accumulated
    double out[2];             // mean loss and samples of the last optimiser step
    int adam_t;
};

struct Ctl {
    int done;                                // iteration finished (any reason)
    int status;                              // sbi_status of the solve
    int sweeps;                              // sweep-operator applications
    int nonfinite;                           // a non-finite input value was seen
    int sweeps_inner;                        // FP32 correction sweeps of a mixed-precision solve
    double omega;                            // relaxation weight
    double residual;                         // last residual
    double rmin;                             // smallest residual seen so far
    unsigned long long eta_max;              // order-preserving bits of max(eta)
    unsigned long long eta_min;              // order-preserving bits of min(eta)
    CtlSlots* slots;                         // this member's residual slots
    // totals over the solves since the last accumulator reset, written by the
    // workgroup that decides each solve (host-free statistics of captured runs)
    long long acc_solves, acc_sweeps;
    int acc_sweeps_max, acc_worst;
    double acc_residual_max;
    // Anderson mixing: inner products of the residual history (ring slots)
    double aa_gram[kAASlots][kAASlots];
};

struct GridDev {
    int nx, ny, Mx, My, Kx, Kxp, Ky, order;
    int ldh;            // column pitch of a half form (ny + pad: spreads columns over memory channels)
    double lx, ly, kband;
    long long s_phys;   // reals per member of a physical field
    long long s_half;   // complex per member of a half-form field
    long long s_cmp;    // complex per member of a compact field
    const double* href; // [batch] reference depth
    int relax;
    int qb;             // kept band below ny/4 and ny >= 128: the quarter-band column pass
    int col_C;          // columns per column-pass workgroup (Kxp is a multiple)
    // launch plan of the row sweep and SA kernels (the autotuner's choice):
    // row_var 0 radix-8 with twiddle recurrence, 1 radix-8 with every twiddle
    // power cached, 2 radix-16 (FP32, rows of 512 or more); row_rpw rows per
    // workgroup (0: as many as fit 256 threads)
    int row_var, row_rpw;
};

// Multiplier of one contribution to a column-pass accumulator:
//   coef * fn(k) * k^pw * dv,  fn in {1, tanh(kh), sech(kh)}, dv in {1, i kx, i ky}
// (k^-1 and i k terms vanish at k = 0).
struct ColTerm {
    double coef;
    short src;      // product index (< nprod) or nprod + compact-input index
    signed char acc, fn, pw, dv;
    signed char pad[2];
};

enum { FN_ONE = 0, FN_T = 1, FN_S = 2 };
enum { DV_NONE = 0, DV_X = 1, DV_Y = 2 };
// sources of column-pass outputs
enum { SRC_ACC0 = 0, SRC_ACC1 = 1, SRC_ACC2 = 2, SRC_ACC3 = 3, SRC_NEW0 = 4, SRC_NEW1 = 5,
       SRC_DIFF0 = 6, SRC_DIFF1 = 7 };
// control modes of a column pass
enum { CTL_NONE = 0, CTL_OMEGA = 1, CTL_SWEEP = 2, CTL_SKIP = 3 };  // CTL_SKIP: return once the solve is decided

struct ColParams {
    GridDev g;
    int nprod, ncin, nterm, nacc;
    const void* hin[kMaxProd];
    long long hin_stride[kMaxProd];   // per-member stride override (0 = g.s_half)
    const void* cin[kMaxCin];
    signed char cin_widx[kMaxCin];     // Anderson weight (history slot) scaling each compact input, -1: none
    // Anderson weights formed in the pass itself: when aa_partial is set, each
    // workgroup adds the inner-product partials of sweep aa_sweep
    // ([batch][aa_nblk][kAASlots]) and solves for the weights of the history
    // slots; the first workgroup of a member stores the new Gram entries
    const double* aa_partial;
    int aa_nblk, aa_sweep;
    short toff[kMaxProd + kMaxCin + 1]; // terms sorted by source: [toff[s], toff[s+1])
    ColTerm term[kMaxTerms];
    int relax_prev[2];                 // compact-input index of the previous iterate of acc0/acc1, -1 none
    int ncout;
    int cout_src[kMaxCout];
    void* cout[kMaxCout];
    int ninv;
    int inv_src[kMaxInv];
    int inv_dv[kMaxInv];
    void* inv[kMaxInv];
    Ctl* ctl;
    int ctl_mode;
    int sweep;        // sweep index n of this pass (CTL_SWEEP)
    int max_sweeps;
    double tol;
    // products split over workgroups along y: group g transforms products
    // [gstart[g], gstart[g+1]); partial sums go to `part` and the last
    // workgroup of a tile (ticket in `cnt`) adds them in group order.
    int ngroup;
    int gstart[kMaxGroups + 1];
    void* part;       // [batch][kMaxGroups][4][Ky][Kxp] complex
    int* cnt;         // [batch][kMaxTiles]
};

}  // namespace sbi
