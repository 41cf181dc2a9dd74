// sbi_api.hip -- C interface and host orchestration of the SBI wave solver.
//
// Host code only decides what to launch; every step of the computation runs
// in the kernels of sbi_kernels.hip.  The W solve (Sec. 2.4 / App. C) is one
// of two kernel sequences:
//   SA mode   : orders l = 2..L, each a row pass forming the products of
//               Appendix C and a column pass applying its multipliers;
//   ITER mode : the same expansion summed over orders, iterated from the
//               linear guess of Sec. 2.4; each sweep is one row pass and one
//               column pass, and the column pass decides convergence from the
//               residual reduced by the row pass before it (device side), so
//               the host only polls a small status header between chunks of
//               sweeps.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstdio>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/sbi.h"
#include "../../include/sbi_batch.h"
#include "../../include/sbi_net.h"
#include "sbi_full.hpp"
#include "sbi_kernels.hpp"
#include "sbi_net.hpp"

using namespace sbi;

namespace {

// compact spectral buffers
enum {
    C_EH, C_PH,          // state u_n
    C_ES, C_PS,          // stage state
    C_AE, C_AP,          // Runge-Kutta accumulator
    C_VH,                // W spectrum (SA sum)
    C_BV, C_BB,          // constant parts of the summed operator
    C_VN, C_BN,          // current iterate (V, phi_b)
    C_VP,                // T(V_n): candidate answer of the iteration
    C_NP,                // nonlinear term of the potential equation
    C_DV, C_DB,          // nonlinear part (V* - kT phi, phi_b - S phi) of the last solve
    C_PD,                // i k . MF{mu grad phi} of the wave tank's damping pressure
    C_AFV0,              // residual history f_i (V part), kAASlots ring slots
    C_AFB0 = C_AFV0 + kAASlots,  //   (phi_b part)
    C_AGV0 = C_AFB0 + kAASlots,  // relaxed-sweep history g_i (V part)
    C_AGB0 = C_AGV0 + kAASlots,  //   (phi_b part)
    C_KE0 = C_AGB0 + kAASlots,  // stage derivatives of the adaptive pair: eta part K_0..K_5
    C_KP0 = C_KE0 + 6,   //   potential part
    C_HV0 = C_KP0 + 6,   // learned history seed: nonlinear parts of the last fixed-step solves, newest first (V)
    C_HB0 = C_HV0 + kHistTaps,  //   (phi_b)
    C_PV = C_HB0 + kHistTaps,   // its prediction for the current solve (V, phi_b)
    C_PB,
    C_COUNT
};
// half-form buffers
enum {
    H_ETA, H_EX, H_EY, H_PX, H_PY,  // state and its gradients
    H_GV, H_GD, H_GBX, H_GBY,       // iterate / order fields
    H_GT,                           // T(V_n) of the Anderson-mixed iteration (residual denominator)
    H_PROD0,                        // products H_PROD0 .. H_PROD0 + kMaxProd - 1
    H_COUNT = H_PROD0 + kMaxProd
};
// physical buffers
enum {
    P_ETA, P_DELTA, P_PX, P_PY,
    P_V0,                 // SA orders V_1..V_7 at P_V0 + (l-1)
    P_BX0 = P_V0 + 7,     // SA orders grad phi_b,1..6 (x)
    P_BY0 = P_BX0 + 7,
    P_COUNT = P_BY0 + 7
};

constexpr int kAABlocks = 256;  // workgroups per member of the Anderson inner products

struct Stats {
    double launches = 0, syncs = 0, sweeps = 0;
};

// kernel classes timed by the optional profiler
enum {
    K_ROW_FWD, K_ROW_INV, K_ROW_SETUP, K_ROW_SWEEP, K_ROW_SA, K_ROW_NPHI, K_ROW_BLEND,
    K_COL_STATE, K_COL_FORCING, K_COL_SWEEP, K_COL_SA, K_COL_OTHER, K_RK, K_DIAG, K_NET, K_FULL_PAIRS,
    K_FULL_APPLY, K_ROW_SWEEP32, K_COL_SWEEP32, K_COUNT
};
const char* const kKernelNames[K_COUNT] = {
    "row_fwd", "row_inv", "row_setup", "row_sweep", "row_sa", "row_nphi", "row_blend",
    "col_state", "col_forcing", "col_sweep", "col_sa", "col_other", "rk", "diag", "net", "full_pairs",
    "full_apply", "row_sweep_fp32", "col_sweep_fp32"};

struct Profiler {
    bool on = false;
    unsigned mask = 0;                  // kernel classes timed (bit per class)
    std::vector<hipEvent_t> pool;       // free events
    struct Pending { int cls; hipEvent_t a, b; };
    std::vector<Pending> pending;
    double total_ms[K_COUNT] = {};
    long long count[K_COUNT] = {};
};

}  // namespace

struct sbi_ctx {
    sbi_grid grid;
    int batch = 1;
    int fp64 = 1;
    hipStream_t stream = nullptr;
    GridDev gd{};
    size_t rsz = 8, csz = 16;
    char* ws = nullptr;
    bool own_ws = false;
    size_t ws_bytes = 0;
    void* comp[C_COUNT] = {};
    void* half[H_COUNT] = {};
    void* phys[P_COUNT] = {};
    void* tx = nullptr;
    void* tn = nullptr;
    void* ty = nullptr;
    double* href_dev = nullptr;
    Ctl* ctl = nullptr;
    double* diag_partial = nullptr;
    double* aa_partial = nullptr;   // [batch][kAABlocks][kAASlots] inner-product partials
    void* part = nullptr;    // partial sums of grouped column passes
    int* cnt = nullptr;      // tile tickets of grouped column passes
    int col_C = 1;
    int group_target = 0;    // workgroups a column pass should reach by splitting products (0: never split)
    int diag_nblk = 64;
    std::vector<double> href;
    bool vd = false;         // some member has a non-flat bed
    bool depth_warn = false;
    bool relax_on = false;
    bool have_prev = false;  // C_DV/C_DB hold the last solve's nonlinear part (SBI_SEED_PREV)
    NetPacked* net = nullptr;  // learned warm start: packed weights (device)
    bool net_loaded = false;
    float net_scale[8] = {1, 1, 1, 1, 1, 1, 1, 1};
    float* feat = nullptr;     // feature field [batch][ny][nx][8] (SBI_SEED_NET)
    int fallbacks = 0;         // solves of the current call restarted from the linear guess
    // learned history seed (SBI_SEED_NET): weights and training state in
    // hist_dev; hist_count fixed-step solves are held in C_HV/C_HB
    HistDev* hist_dev = nullptr;
    double* hist_partial = nullptr;
    // fully nonlinear solve (SBI_MODE_FULL): tables (S0^-1 per member, eta_x
    // and eta_xx circulants, sin^2) and the slices of its pair passes
    void* full_c0 = nullptr;
    void* full_d1 = nullptr;
    void* full_d2 = nullptr;
    void* full_s2 = nullptr;
    void* full_s2a = nullptr;
    void* full_rs2 = nullptr;
    void* full_rhs = nullptr;
    void* full_lfl = nullptr;
    void* full_w = nullptr;
    void* full_part = nullptr;
    // two-boundary form of the fully nonlinear solve (variable beds)
    void* full_bz = nullptr;
    void* full_bx = nullptr;
    void* full_bxx = nullptr;
    void* full_cm = nullptr;
    void* full_rb = nullptr;
    void* full_pb[2] = {nullptr, nullptr};
    int* full_bed = nullptr;    // [batch] device flags
    bool full_bed_any = false;
    bool full_bed_all = false;  // every member two-boundary: no image-form surface pass
    int full_pred = 0;          // launches the last fully nonlinear solve took (0: none yet)
    // mixed precision (SBI_MIXED): the FP32 context that solves the correction
    // equations, in the tail of this context's workspace, on the same stream
    sbi_ctx* inner = nullptr;
    int hist_K = 0, hist_nb = 0;
    double hist_dk = 0.0;
    bool hist_loaded = false;
    bool hist_train = false;
    int hist_count = 0;
    // sweeps enqueued per solve by an iteration without host polling
    // (iterate_fixed); 0 or >= max_sweeps: the full max_sweeps + 1 launches
    int budget = 0;
    double rz[6] = {0, 0, 0, 0, 0, 0};
    // wave tank (Sec. 3.2): pneumatic wavemaker components and damping pressure
    int wm_n = 0;
    double wm[kMaxWavemaker][4] = {};
    double wm_h = 0.0;
    double dmp_x0 = 0.0, dmp_w = 0.0;  // dmp_w <= 0: no damping
    Stats st;
    Profiler prof;
    Ctl* head = nullptr;     // pinned host copy of the control headers
    hipEvent_t poll = nullptr;  // marks a header copy the host waits for while sweeps run on
    // transient context of sbi_vertical_velocity_noalloc: workspace in the
    // library's static device scratch, headers in ordinary host memory, no
    // poll event (the iteration waits on the stream instead)
    bool transient = false;
    std::vector<Ctl> head_host;
    sbi_step_info step_acc{};
};

static void prof_flush(sbi_ctx* c);

static const char* kStatusNames[] = {"SBI_OK",
                                     "SBI_WARN_NOT_CONVERGED: iteration reached max_sweeps",
                                     "SBI_WARN_DEPTH_CRITERION: k_band*max(delta) exceeds 2.4",
                                     "SBI_WARN_FALLBACK_USED: learned seed rejected",
                                     "SBI_WARN_STEP_LIMIT: max_steps reached before t_end"};
static const char* kErrNames[] = {"",
                                  "SBI_ERR_INVALID_ARG: invalid argument",
                                  "SBI_ERR_UNSUPPORTED: unsupported size or option",
                                  "SBI_ERR_WORKSPACE: workspace missing or too small",
                                  "SBI_ERR_HIP: HIP runtime error",
                                  "SBI_ERR_NONFINITE: non-finite input",
                                  "SBI_ERR_DIVERGED: iteration diverged"};

static bool is_pow2(int n) { return n > 0 && (n & (n - 1)) == 0; }

static sbi_status hip_ok(hipError_t e) { return e == hipSuccess ? SBI_OK : SBI_ERR_HIP; }

#define SBI_TRY(expr)                          \
    do {                                       \
        sbi_status _s = (expr);                \
        if (_s < 0) return _s;                 \
    } while (0)
#define SBI_HIP(expr)                          \
    do {                                       \
        hipError_t _e = (expr);                \
        if (_e != hipSuccess) return SBI_ERR_HIP; \
    } while (0)

// ---------------------------------------------------------------------------
// sizes and layout
// ---------------------------------------------------------------------------
struct Layout {
    int Mx, My, Kx, Kxp, Ky, C, qb, ldh;
    size_t rsz, csz;
    long long s_phys, s_half, s_cmp;
    size_t bytes_comp, bytes_half, bytes_phys, bytes_tw, bytes_misc, bytes_net, bytes_full, bytes_inner, total;
};

// the FP32 context of a mixed-precision context: same grid and options, FP32
// fields; seeds come from the FP64 side
static sbi_grid inner_grid(const sbi_grid* g) {
    sbi_grid gi = *g;
    gi.precision = SBI_FP32;
    gi.seed = SBI_SEED_LINEAR;
    return gi;
}

constexpr int kFullSplitMax = 16;  // source-point slices of a pair pass of the fully nonlinear solve
// slices the pair passes of a fully nonlinear solve may write: the split passes'
// and the symmetric single-layer pass's (one per tile block)
static int full_slices(int nx) { return std::max(kFullSplitMax, nx / kFullSymTile); }

static bool grid_valid(const sbi_grid* g) {
    if (!g) return false;
    if (!is_pow2(g->nx) || g->nx < 16 || g->nx > 8192) return false;
    if (!(g->ny == 1 || (is_pow2(g->ny) && g->ny >= 16 && g->ny <= 2048))) return false;
    if (!(g->lx > 0) || (g->ny > 1 && !(g->ly > 0))) return false;
    if (g->order < 1 || g->order > 7) return false;
    if (!(g->dealias > 0.0 && g->dealias < 1.0)) return false;
    if (g->precision != SBI_FP64 && g->precision != SBI_FP32 && g->precision != SBI_MIXED) return false;
    if (g->precision == SBI_MIXED && g->mode != SBI_MODE_ITER) return false;  // refines an iteration
    if (g->mode != SBI_MODE_ITER && g->mode != SBI_MODE_SA && g->mode != SBI_MODE_FULL) return false;
    if (g->mode == SBI_MODE_FULL && g->ny != 1) return false;  // the exact surface equation: one dimension
    if (g->max_sweeps < 1 || g->max_sweeps > 1000) return false;
    if (g->seed < SBI_SEED_LINEAR || g->seed > SBI_SEED_USER) return false;
    if (g->accel != SBI_ACCEL_NONE && g->accel != SBI_ACCEL_ANDERSON) return false;
    return true;
}

// pad (bytes) appended to every half-form column; SBI_HALF_PAD_BYTES overrides
static int half_pad_bytes() {
    static int v = [] {
        const char* e = std::getenv("SBI_HALF_PAD_BYTES");
        return e ? std::max(0, std::atoi(e)) : 256;
    }();
    return v;
}

static Layout layout(const sbi_grid* g, int batch) {
    Layout L{};
    const bool f64 = g->precision != SBI_FP32;
    L.rsz = f64 ? 8 : 4;
    L.csz = 2 * L.rsz;
    // kept modes |m| < alpha n / 2 (strict)
    L.Mx = (int)std::ceil(g->dealias * g->nx / 2.0 - 1e-9) - 1;
    L.My = g->ny == 1 ? 0 : (int)std::ceil(g->dealias * g->ny / 2.0 - 1e-9) - 1;
    L.Kx = L.Mx + 1;
    L.qb = col_quarter_band(g->ny, L.My);
    L.C = col_tile(g->ny, f64, L.qb);
    L.Kxp = (L.Kx + L.C - 1) / L.C * L.C;
    L.Ky = g->ny == 1 ? 1 : 2 * L.My + 1;
    L.s_phys = (long long)g->nx * g->ny;
    L.ldh = g->ny == 1 ? 1 : g->ny + (int)(half_pad_bytes() / L.csz);
    L.s_half = (long long)L.ldh * L.Kxp;
    L.s_cmp = (long long)L.Ky * L.Kxp;
    auto al = [](size_t b) { return (b + 255) / 256 * 256; };
    L.bytes_comp = al((size_t)L.s_cmp * L.csz * batch) * C_COUNT;
    L.bytes_half = al((size_t)L.s_half * L.csz * batch) * H_COUNT;
    L.bytes_phys = al((size_t)L.s_phys * L.rsz * batch) * P_COUNT;
    L.bytes_tw = al((size_t)g->nx * L.csz) + al((size_t)(g->nx / 2) * L.csz) + al((size_t)g->ny * L.csz);
    L.bytes_misc = al(sizeof(double) * batch) + al(sizeof(Ctl) * batch) + al(sizeof(CtlSlots) * batch) +
                   al(sizeof(double) * 2 * 64 * batch) + al(sizeof(double) * kAASlots * kAABlocks * batch) +
                   al(sizeof(double) * kAASlots * batch) +
                   al((size_t)L.s_cmp * L.csz * batch * kMaxGroups * 4) + al(sizeof(int) * (size_t)kMaxTiles * batch);
    // learned warm start: packed weights, and the feature field when it seeds the iteration
    L.bytes_net = al(sizeof(NetPacked)) +
                  ((g->seed == SBI_SEED_NET && g->ny > 1) ? al((size_t)L.s_phys * 8 * sizeof(float) * batch) : 0) +
                  (g->seed == SBI_SEED_NET
                       ? al(sizeof(HistDev)) + al(sizeof(double) * kHistPart * kHistBlocks * (size_t)batch)
                       : 0);
    // fully nonlinear solve (FP64 in both precisions): tables [batch + 5][nx]
    // and [batch][nx], right-hand side and source term [batch][nx], pair
    // slices [full_slices(nx)][batch][nx]; for beds kept as a boundary, the bed
    // geometry (3 tables), its circulant, its right-hand side and two phi_b
    // iterates [batch][nx], and the per-member flags
    L.bytes_full = g->mode == SBI_MODE_FULL
                       ? 16 * al((size_t)g->nx * 8 * batch) + al((size_t)full_slices(g->nx) * g->nx * 8 * batch) +
                             al(sizeof(int) * batch)
                       : 0;
    // mixed precision: the FP32 context's workspace at the end
    if (g->precision == SBI_MIXED) {
        const sbi_grid gi = inner_grid(g);
        L.bytes_inner = layout(&gi, batch).total;
    }
    L.total = L.bytes_comp + L.bytes_half + L.bytes_phys + L.bytes_tw + L.bytes_misc + L.bytes_net + L.bytes_full +
              L.bytes_inner;
    return L;
}

extern "C" void sbi_grid_defaults(sbi_grid* g) {
    if (!g) return;
    std::memset(g, 0, sizeof(*g));
    g->nx = 256;
    g->ny = 1;
    g->lx = 2.0 * M_PI;
    g->ly = 2.0 * M_PI;
    g->order = 7;
    g->dealias = 0.5;
    g->precision = SBI_FP64;
    g->mode = SBI_MODE_ITER;
    g->seed = SBI_SEED_LINEAR;
    g->max_sweeps = 64;
    g->relax = 1;
    g->filter_beta1 = 0.0;
    g->filter_beta2 = 0.0;
    g->accel = SBI_ACCEL_NONE;
}

extern "C" size_t sbi_workspace_bytes(const sbi_grid* g, int32_t batch) {
    if (!grid_valid(g) || batch < 1) return 0;
    return layout(g, batch).total;
}

extern "C" const char* sbi_status_string(sbi_status s) {
    if (s >= 0 && s <= 4) return kStatusNames[s];
    if (s <= -1 && s >= -6) return kErrNames[-s];
    return "unknown sbi_status";
}

// ---------------------------------------------------------------------------
// upload helpers
// ---------------------------------------------------------------------------
static std::vector<char> to_prec(const double* src, size_t n, int fp64) {
    std::vector<char> out(n * (fp64 ? 8 : 4));
    if (fp64) std::memcpy(out.data(), src, n * 8);
    else {
        float* f = reinterpret_cast<float*>(out.data());
        for (size_t i = 0; i < n; ++i) f[i] = (float)src[i];
    }
    return out;
}

static std::vector<double> twiddle_table(int n) {
    std::vector<double> t(2 * (size_t)n);
    for (int m = 0; m < n; ++m) {
        // exp(-2 pi i m/n) with octant-symmetric argument reduction for accuracy
        const double a = -2.0 * M_PI * (double)m / (double)n;
        t[2 * m] = std::cos(a);
        t[2 * m + 1] = std::sin(a);
    }
    return t;
}

static sbi_status full_tables(sbi_ctx* c);

static sbi_status set_depth(sbi_ctx* c, const double* depth, double h_ref) {
    const sbi_grid& g = c->grid;
    const size_t npt = (size_t)g.nx * g.ny;
    std::vector<double> delta(npt * c->batch);
    c->href.assign(c->batch, 0.0);
    c->vd = false;
    double kdmax = 0.0;
    for (int b = 0; b < c->batch; ++b) {
        const double* d = depth + b * npt;
        double dmax = 0.0;
        for (size_t i = 0; i < npt; ++i) {
            if (!std::isfinite(d[i])) return SBI_ERR_NONFINITE;
            if (!(d[i] > 0.0)) return SBI_ERR_INVALID_ARG;
            dmax = std::max(dmax, d[i]);
        }
        const double h = h_ref > 0.0 ? h_ref : dmax;
        c->href[b] = h;
        for (size_t i = 0; i < npt; ++i) {
            // seabed at z = -h + delta (Sec. 2.1)
            delta[b * npt + i] = h - d[i];
            if (delta[b * npt + i] != 0.0) c->vd = true;
            kdmax = std::max(kdmax, std::fabs(delta[b * npt + i]));
        }
    }
    c->depth_warn = c->gd.kband * kdmax > 2.4;
    std::vector<char> dv = to_prec(delta.data(), delta.size(), c->fp64);
    SBI_HIP(hipMemcpyAsync(c->phys[P_DELTA], dv.data(), dv.size(), hipMemcpyHostToDevice, c->stream));
    SBI_HIP(hipMemcpyAsync(c->href_dev, c->href.data(), sizeof(double) * c->batch, hipMemcpyHostToDevice, c->stream));
    if (g.mode == SBI_MODE_FULL) {
        // the fully nonlinear solve keeps a variable bed as a boundary of its
        // own unless it is too deep to matter (k_1 times the smallest depth
        // beyond 18, where the image form drops the image); heights b = -h + delta
        std::vector<int> bed(c->batch, 0);
        std::vector<double> bz(npt * c->batch);
        const double k1 = 2.0 * M_PI / g.lx;
        c->full_bed_any = false;
        c->full_bed_all = true;
        for (int b = 0; b < c->batch; ++b) {
            bool var = false;
            double dmax = 0.0;
            for (size_t i = 0; i < npt; ++i) {
                const double dl = delta[b * npt + i];
                var = var || dl != 0.0;
                dmax = std::max(dmax, dl);
                bz[b * npt + i] = -c->href[b] + dl;
            }
            bed[b] = var && !(k1 * (c->href[b] - dmax) > 18.0);
            c->full_bed_any = c->full_bed_any || bed[b];
            c->full_bed_all = c->full_bed_all && bed[b];
        }
        SBI_HIP(hipMemcpyAsync(c->full_bz, bz.data(), sizeof(double) * bz.size(), hipMemcpyHostToDevice, c->stream));
        SBI_HIP(hipMemcpyAsync(c->full_bed, bed.data(), sizeof(int) * c->batch, hipMemcpyHostToDevice, c->stream));
        SBI_TRY(full_tables(c));
        SBI_HIP(hipStreamSynchronize(c->stream));  // the host vectors above go out of scope
    }
    SBI_HIP(hipStreamSynchronize(c->stream));
    if (c->inner) SBI_TRY(set_depth(c->inner, depth, h_ref));
    return SBI_OK;
}

// release what a context holds (not the context itself)
static void ctx_release(sbi_ctx* c) {
    if (c->inner) {
        prof_flush(c->inner);
        for (hipEvent_t e : c->inner->prof.pool) (void)hipEventDestroy(e);
        ctx_release(c->inner);
        delete c->inner;
        c->inner = nullptr;
    }
    if (c->transient) return;  // nothing was allocated
    if (c->head) (void)hipHostFree(c->head);
    if (c->poll) (void)hipEventDestroy(c->poll);
    if (c->own_ws) (void)hipFree(c->ws);
}

// Set up context c (grid, layout, workspace, tables, depth).  transient: the
// workspace is given and nothing is allocated on the device or pinned on the
// host (headers in c->head_host, no poll event).
static sbi_status ctx_setup(sbi_ctx* c, const sbi_grid* g, int32_t batch, const double* depth, double h_ref,
                            void* workspace, size_t ws_bytes, void* hip_stream, bool transient) {
    const Layout L = layout(g, batch);
    if (workspace && ws_bytes < L.total) return SBI_ERR_WORKSPACE;
    if (transient && !workspace) return SBI_ERR_WORKSPACE;
    if (transient && g->precision == SBI_MIXED) return SBI_ERR_UNSUPPORTED;
    c->transient = transient;
    c->grid = *g;
    c->batch = batch;
    c->fp64 = g->precision != SBI_FP32;
    c->stream = static_cast<hipStream_t>(hip_stream);
    c->rsz = L.rsz;
    c->csz = L.csz;
    GridDev& gd = c->gd;
    gd.nx = g->nx;
    gd.ny = g->ny;
    gd.Mx = L.Mx;
    gd.My = L.My;
    gd.Kx = L.Kx;
    gd.Kxp = L.Kxp;
    gd.Ky = L.Ky;
    gd.order = g->order;
    gd.lx = g->lx;
    gd.ly = g->ny == 1 ? 1.0 : g->ly;
    gd.kband = std::hypot(2.0 * M_PI * L.Mx / g->lx, g->ny == 1 ? 0.0 : 2.0 * M_PI * L.My / g->ly);
    gd.s_phys = L.s_phys;
    gd.s_half = L.s_half;
    gd.ldh = L.ldh;
    gd.s_cmp = L.s_cmp;
    gd.relax = g->relax;
    if (workspace) {
        c->ws = static_cast<char*>(workspace);
        c->ws_bytes = ws_bytes;
    } else {
        // the only device allocation of the library: a context created without
        // a caller workspace owns one, made here and freed by sbi_destroy
        if (hipMalloc(&c->ws, L.total) != hipSuccess) return SBI_ERR_HIP;
        c->own_ws = true;
        c->ws_bytes = L.total;
    }
    auto al = [](size_t b) { return (b + 255) / 256 * 256; };
    char* p = c->ws;
    for (int i = 0; i < C_COUNT; ++i) {
        c->comp[i] = p;
        p += al((size_t)L.s_cmp * L.csz * batch);
    }
    for (int i = 0; i < H_COUNT; ++i) {
        c->half[i] = p;
        p += al((size_t)L.s_half * L.csz * batch);
    }
    for (int i = 0; i < P_COUNT; ++i) {
        c->phys[i] = p;
        p += al((size_t)L.s_phys * L.rsz * batch);
    }
    c->tx = p;
    p += al((size_t)g->nx * L.csz);
    c->tn = p;
    p += al((size_t)(g->nx / 2) * L.csz);
    c->ty = p;
    p += al((size_t)g->ny * L.csz);
    c->href_dev = reinterpret_cast<double*>(p);
    p += al(sizeof(double) * batch);
    c->ctl = reinterpret_cast<Ctl*>(p);
    p += al(sizeof(Ctl) * batch);
    CtlSlots* slots = reinterpret_cast<CtlSlots*>(p);
    p += al(sizeof(CtlSlots) * batch);
    c->diag_partial = reinterpret_cast<double*>(p);
    p += al(sizeof(double) * 2 * 64 * batch);
    c->aa_partial = reinterpret_cast<double*>(p);
    p += al(sizeof(double) * kAASlots * kAABlocks * batch);
    c->part = p;
    p += al((size_t)L.s_cmp * L.csz * batch * kMaxGroups * 4);
    c->cnt = reinterpret_cast<int*>(p);
    p += al(sizeof(int) * (size_t)kMaxTiles * batch);
    c->net = reinterpret_cast<NetPacked*>(p);
    p += al(sizeof(NetPacked));
    if (g->seed == SBI_SEED_NET && g->ny > 1) {
        c->feat = reinterpret_cast<float*>(p);
        p += al((size_t)L.s_phys * 8 * sizeof(float) * batch);
    }
    if (g->seed == SBI_SEED_NET) {
        c->hist_dev = reinterpret_cast<HistDev*>(p);
        p += al(sizeof(HistDev));
        c->hist_partial = reinterpret_cast<double*>(p);
        p += al(sizeof(double) * kHistPart * kHistBlocks * (size_t)batch);
    }
    if (g->mode == SBI_MODE_FULL) {
        const size_t tb = al((size_t)g->nx * 8 * batch);
        c->full_c0 = p;
        c->full_d1 = p + tb;
        c->full_d2 = p + 2 * tb;
        c->full_s2 = p + 3 * tb;
        c->full_rhs = p + 4 * tb;
        c->full_lfl = p + 5 * tb;
        c->full_w = p + 6 * tb;
        c->full_bz = p + 7 * tb;
        c->full_bx = p + 8 * tb;
        c->full_bxx = p + 9 * tb;
        c->full_cm = p + 10 * tb;
        c->full_rb = p + 11 * tb;
        c->full_pb[0] = p + 12 * tb;
        c->full_pb[1] = p + 13 * tb;
        c->full_s2a = p + 14 * tb;
        c->full_rs2 = p + 15 * tb;
        c->full_part = p + 16 * tb;
        c->full_bed = reinterpret_cast<int*>(p + 16 * tb + al((size_t)full_slices(g->nx) * g->nx * 8 * batch));
    }
    c->col_C = L.C;
    gd.col_C = L.C;
    gd.qb = L.qb;
    gd.href = c->href_dev;
    if (transient) {
        c->head_host.assign(batch, Ctl{});
        c->head = c->head_host.data();
    } else {
        if (hipHostMalloc(reinterpret_cast<void**>(&c->head), sizeof(Ctl) * batch, hipHostMallocDefault) !=
            hipSuccess) {
            c->head = nullptr;
            return SBI_ERR_HIP;
        }
        if (hipEventCreateWithFlags(&c->poll, hipEventDisableTiming) != hipSuccess) {
            c->poll = nullptr;
            return SBI_ERR_HIP;
        }
    }
    // SBI_COL_GROUP_TARGET: workgroups a column pass aims for by splitting its
    // products over workgroups (tuning knob; 0 = one workgroup per tile)
    if (const char* e = std::getenv("SBI_COL_GROUP_TARGET")) c->group_target = std::atoi(e);

    sbi_status st = hip_ok(launch_fill_zero(c->ws, L.total, c->stream));
    if (st == SBI_OK) {
        auto up = [&](void* dst, int n) -> sbi_status {
            std::vector<double> t = twiddle_table(n);
            std::vector<char> v = to_prec(t.data(), t.size(), c->fp64);
            sbi_status r = hip_ok(hipMemcpyAsync(dst, v.data(), v.size(), hipMemcpyHostToDevice, c->stream));
            if (r == SBI_OK) r = hip_ok(hipStreamSynchronize(c->stream));
            return r;
        };
        if (st == SBI_OK) st = up(c->tx, g->nx);
        if (st == SBI_OK) st = up(c->tn, g->nx / 2);
        if (st == SBI_OK) st = up(c->ty, g->ny);
        if (st == SBI_OK) {
            for (int b = 0; b < batch; ++b) {
                std::memset(&c->head[b], 0, sizeof(Ctl));
                c->head[b].slots = slots + b;
            }
            st = hip_ok(hipMemcpyAsync(c->ctl, c->head, sizeof(Ctl) * batch, hipMemcpyHostToDevice, c->stream));
            if (st == SBI_OK) st = hip_ok(hipStreamSynchronize(c->stream));
        }
        if (st == SBI_OK) st = hip_ok(launch_ctl_reset(c->ctl, batch, kMaxSweepSlots, c->stream));
        if (st == SBI_OK) st = set_depth(c, depth, h_ref);
    }
    if (st >= 0 && g->precision == SBI_MIXED) {
        const sbi_grid gi = inner_grid(g);
        c->inner = new sbi_ctx();
        const sbi_status si = ctx_setup(c->inner, &gi, batch, depth, h_ref, c->ws + (L.total - L.bytes_inner),
                                        L.bytes_inner, hip_stream, false);
        if (si < 0) st = si;
    }
    if (st < 0) return st;
    return c->depth_warn ? SBI_WARN_DEPTH_CRITERION : SBI_OK;
}

extern "C" sbi_status sbi_init(sbi_ctx** out, const sbi_grid* g, int32_t batch, const double* depth, double h_ref,
                               void* workspace, size_t ws_bytes, void* hip_stream) {
    if (!out || !grid_valid(g) || batch < 1 || !depth) return SBI_ERR_INVALID_ARG;
    *out = nullptr;
    if (g->seed == SBI_SEED_NET && g->ny == 1) return SBI_ERR_UNSUPPORTED;  // the network is 2D
    sbi_ctx* c = new sbi_ctx();
    const sbi_status st = ctx_setup(c, g, batch, depth, h_ref, workspace, ws_bytes, hip_stream, false);
    if (st < 0) {
        (void)hipStreamSynchronize(c->stream);  // work enqueued before the failure ends before any free
        ctx_release(c);
        delete c;
        return st;
    }
    *out = c;
    return st;
}

extern "C" sbi_status sbi_destroy(sbi_ctx* c) {
    if (!c) return SBI_ERR_INVALID_ARG;
    (void)hipStreamSynchronize(c->stream);
    prof_flush(c);
    for (hipEvent_t e : c->prof.pool) (void)hipEventDestroy(e);
    ctx_release(c);
    delete c;
    return SBI_OK;
}

extern "C" sbi_status sbi_set_depth(sbi_ctx* c, const double* depth, double h_ref) {
    if (!c || !depth) return SBI_ERR_INVALID_ARG;
    SBI_TRY(set_depth(c, depth, h_ref));
    c->hist_count = 0;  // the learned history belongs to the old bed
    return c->depth_warn ? SBI_WARN_DEPTH_CRITERION : SBI_OK;
}

extern "C" sbi_status sbi_set_relaxation(sbi_ctx* c, const double* params, int32_t n) {
    if (!c) return SBI_ERR_INVALID_ARG;
    if (n == 0) {
        c->relax_on = false;
        return SBI_OK;
    }
    if (n != 6 || !params || c->grid.ny != 1) return SBI_ERR_INVALID_ARG;
    for (int i = 0; i < 6; ++i) {
        if (!std::isfinite(params[i])) return SBI_ERR_INVALID_ARG;
        c->rz[i] = params[i];
    }
    if (!(c->rz[2] > 0 && c->rz[3] > 0 && c->rz[4] > 0 && c->rz[5] > 0)) return SBI_ERR_INVALID_ARG;
    c->relax_on = true;
    return SBI_OK;
}

extern "C" sbi_status sbi_set_wavemaker(sbi_ctx* c, const double* comps, int32_t ncomp, double h_gen,
                                        double damp_x0, double damp_width) {
    if (!c || ncomp < 0 || ncomp > kMaxWavemaker || (ncomp > 0 && !comps)) return SBI_ERR_INVALID_ARG;
    if (!std::isfinite(h_gen) || !std::isfinite(damp_x0) || !std::isfinite(damp_width)) return SBI_ERR_INVALID_ARG;
    for (int j = 0; j < ncomp; ++j) {
        for (int e = 0; e < 4; ++e)
            if (!std::isfinite(comps[4 * j + e])) return SBI_ERR_INVALID_ARG;
        if (!(comps[4 * j + 1] > 0.0) || comps[4 * j + 2] < 0.0) return SBI_ERR_INVALID_ARG;
    }
    c->wm_n = ncomp;
    for (int j = 0; j < ncomp; ++j)
        for (int e = 0; e < 4; ++e) c->wm[j][e] = comps[4 * j + e];
    c->wm_h = h_gen;
    c->dmp_x0 = damp_x0;
    c->dmp_w = damp_width > 0.0 ? damp_width : 0.0;
    return SBI_OK;
}

extern "C" int32_t sbi_last_stats(const sbi_ctx* c, double* out, int32_t n) {
    if (!c || !out) return 0;
    const double v[3] = {c->st.launches, c->st.syncs, c->st.sweeps};
    int k = std::min<int>(n, 3);
    for (int i = 0; i < k; ++i) out[i] = v[i];
    return k;
}

// ---------------------------------------------------------------------------
// column-pass builder
// ---------------------------------------------------------------------------
struct ColBuilder {
    ColParams p{};
    std::vector<ColTerm> terms;
    std::vector<const void*> prods, cins;
    std::vector<int> cin_w;
    std::vector<long long> prod_stride;
    explicit ColBuilder(const GridDev& g) {
        p.g = g;
        p.relax_prev[0] = p.relax_prev[1] = -1;
        p.nacc = 1;
    }
    int prod(const void* h, long long stride = 0) {
        prods.push_back(h);
        prod_stride.push_back(stride);
        return (int)prods.size() - 1;
    }
    // widx >= 0: the input is scaled by the Anderson weight of history slot
    // widx, which the pass solves for itself (p.aa_partial must be set)
    int cin(const void* c, int widx = -1) {
        cins.push_back(c);
        cin_w.push_back(widx);
        return -(int)cins.size();  // resolved at build: nprod + index
    }
    void term(int src, int acc, double coef, int fn, int pw, int dv) {
        ColTerm t{};
        t.coef = coef;
        t.src = (short)src;
        t.acc = (signed char)acc;
        t.fn = (signed char)fn;
        t.pw = (signed char)pw;
        t.dv = (signed char)dv;
        terms.push_back(t);
        p.nacc = std::max(p.nacc, acc + 1);
    }
    void cout(int src, void* dst) {
        p.cout_src[p.ncout] = src;
        p.cout[p.ncout++] = dst;
    }
    void inv(int src, int dv, void* dst) {
        p.inv_src[p.ninv] = src;
        p.inv_dv[p.ninv] = dv;
        p.inv[p.ninv++] = dst;
    }
    bool build() {
        p.nprod = (int)prods.size();
        p.ncin = (int)cins.size();
        if (p.nprod > kMaxProd || p.ncin > kMaxCin || (int)terms.size() > kMaxTerms) return false;
        for (auto& t : terms)
            if (t.pw > 6 || t.pw < -1) return false;  // the column pass forms k^-1 .. k^6
        for (int i = 0; i < p.nprod; ++i) {
            p.hin[i] = prods[i];
            p.hin_stride[i] = prod_stride[i];
        }
        for (int i = 0; i < p.ncin; ++i) p.cin[i] = cins[i];
        for (int i = 0; i < kMaxCin; ++i) {
            p.cin_widx[i] = (signed char)(i < p.ncin ? cin_w[i] : -1);
            if (p.cin_widx[i] >= kAASlots || (p.cin_widx[i] >= 0 && !p.aa_partial)) return false;
        }
        for (auto& t : terms)
            if (t.src < 0) t.src = (short)(p.nprod + (-t.src - 1));
        std::stable_sort(terms.begin(), terms.end(), [](const ColTerm& a, const ColTerm& b) { return a.src < b.src; });
        const int nsrc = p.nprod + p.ncin;
        int k = 0;
        for (int s = 0; s <= nsrc; ++s) {
            while (k < (int)terms.size() && terms[k].src < s) ++k;
            p.toff[s] = (short)k;
        }
        p.nterm = (int)terms.size();
        for (int i = 0; i < p.nterm; ++i) p.term[i] = terms[i];
        return true;
    }
};

static hipEvent_t prof_event(sbi_ctx* c) {
    if (!c->prof.pool.empty()) {
        hipEvent_t e = c->prof.pool.back();
        c->prof.pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    (void)hipEventCreate(&e);
    return e;
}
// Accumulate the durations of completed launches (call after a stream sync).
static void prof_flush(sbi_ctx* c) {
    for (auto& q : c->prof.pending) {
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, q.a, q.b) == hipSuccess) {
            c->prof.total_ms[q.cls] += ms;
            c->prof.count[q.cls] += 1;
        }
        c->prof.pool.push_back(q.a);
        c->prof.pool.push_back(q.b);
    }
    c->prof.pending.clear();
}
struct ProfScope {
    sbi_ctx* c;
    int cls;
    hipEvent_t a = nullptr;
    ProfScope(sbi_ctx* cc, int k) : c(cc), cls(k) {
        if (c->prof.on && ((c->prof.mask >> k) & 1u)) {
            a = prof_event(c);
            (void)hipEventRecord(a, c->stream);
        }
    }
    ~ProfScope() {
        if (c->prof.on && a) {
            hipEvent_t b = prof_event(c);
            (void)hipEventRecord(b, c->stream);
            c->prof.pending.push_back({cls, a, b});
        }
    }
};

static double fact(int n) {
    double f = 1.0;
    for (int i = 2; i <= n; ++i) f *= i;
    return f;
}
static int Tfn(int n) { return (n & 1) ? FN_T : FN_ONE; }   // tanh^<n/2>(kh)

static Twiddles tw_of(const sbi_ctx* c) {
    Twiddles t;
    t.tx = c->tx;
    t.tn = c->tn;
    t.ty = c->ty;
    return t;
}

// pointer to the start of buffer i; member stride is applied in the kernels
#define CMP(i) (c->comp[(i)])
#define HALF(i) (c->half[(i)])
#define PHYS(i) (c->phys[(i)])

// Split the products of a column pass over workgroups along y when the tiles
// alone cannot fill the GPU (~512 workgroups wanted).
static void set_groups(sbi_ctx* c, ColParams& p) {
    p.ngroup = 1;
    p.part = c->part;
    p.cnt = c->cnt;
    const int np = p.nprod;
    if (np <= 1 || c->grid.ny == 1 || c->group_target <= 0) return;
    const int tiles = c->gd.Kxp / c->col_C;
    int want = (c->group_target + tiles * c->batch - 1) / (tiles * c->batch);
    want = std::max(1, std::min(want, std::min(np, kMaxGroups)));
    p.ngroup = want;
    for (int g = 0; g <= want; ++g) p.gstart[g] = (g * np) / want;
}

static sbi_status run_col(sbi_ctx* c, ColBuilder& b, int cls = K_COL_OTHER) {
    if (!b.build()) return SBI_ERR_UNSUPPORTED;
    set_groups(c, b.p);
    c->st.launches += 1;
    ProfScope ps(c, cls);
    return hip_ok(launch_col(c->fp64, b.p, c->batch, tw_of(c), c->stream));
}

// ---------------------------------------------------------------------------
// stage pieces
// ---------------------------------------------------------------------------
// physical (eta, phi) -> compact state (writes C_EH/C_PH and C_ES/C_PS)
static sbi_status to_spectral(sbi_ctx* c, const void* eta, const void* phi, bool state_too) {
    RowFwdParams rp{};
    rp.g = c->gd;
    rp.nf = 0;
    if (eta) {
        rp.in[rp.nf] = eta;
        rp.out[rp.nf++] = HALF(H_PROD0);
    }
    rp.in[rp.nf] = phi;
    rp.out[rp.nf++] = HALF(H_PROD0 + 1);
    c->st.launches += 1;
    {
        ProfScope ps_(c, K_ROW_FWD);
        SBI_TRY(hip_ok(launch_row_fwd(c->fp64, rp, c->batch, tw_of(c), c->stream)));
    }
    ColBuilder b(c->gd);
    int se = eta ? b.prod(HALF(H_PROD0)) : -1;
    int sp = b.prod(HALF(H_PROD0 + 1));
    if (eta) {
        b.term(se, 0, 1.0, FN_ONE, 0, DV_NONE);
        b.cout(SRC_ACC0, CMP(C_ES));
        if (state_too) b.cout(SRC_ACC0, CMP(C_EH));
    }
    b.term(sp, 1, 1.0, FN_ONE, 0, DV_NONE);
    b.cout(SRC_ACC1, CMP(C_PS));
    if (state_too) b.cout(SRC_ACC1, CMP(C_PH));
    return run_col(c, b);
}

// compact stage state (C_ES, C_PS) -> half forms of eta, grad eta, grad phi, and
// the linear-guess seeds (Sec. 2.4 initiation) of the iteration / SA order 1.
static sbi_status stage_state_pass(sbi_ctx* c, bool need_eta, bool allow_prev = true, bool hist_seed = false) {
    const bool two_d = c->grid.ny > 1;
    ColBuilder b(c->gd);
    int se = b.cin(CMP(C_ES));
    int sp = b.cin(CMP(C_PS));
    b.term(se, 0, 1.0, FN_ONE, 0, DV_NONE);
    b.term(sp, 1, 1.0, FN_ONE, 0, DV_NONE);
    b.term(sp, 2, 1.0, FN_T, 1, DV_NONE);  // k tanh(kh) phi_hat
    if (c->vd) b.term(sp, 3, 1.0, FN_S, 0, DV_NONE);  // sech(kh) phi_hat
    if (need_eta) {
        b.inv(SRC_ACC0, DV_NONE, HALF(H_ETA));
        b.inv(SRC_ACC0, DV_X, HALF(H_EX));
        if (two_d) b.inv(SRC_ACC0, DV_Y, HALF(H_EY));
    }
    b.inv(SRC_ACC1, DV_X, HALF(H_PX));
    if (two_d) b.inv(SRC_ACC1, DV_Y, HALF(H_PY));
    b.inv(SRC_ACC2, DV_NONE, HALF(H_GV));
    if (c->vd) {
        b.inv(SRC_ACC3, DV_X, HALF(H_GBX));
        if (two_d) b.inv(SRC_ACC3, DV_Y, HALF(H_GBY));
    }
    if (c->grid.mode == SBI_MODE_SA) {
        b.cout(SRC_ACC2, CMP(C_VH));
    } else {
        if (hist_seed) {
            // learned history seed: linear guess + the layer's prediction
            b.term(b.cin(CMP(C_PV)), 2, 1.0, FN_ONE, 0, DV_NONE);
            if (c->vd) b.term(b.cin(CMP(C_PB)), 3, 1.0, FN_ONE, 0, DV_NONE);
        } else if (allow_prev && (c->grid.seed == SBI_SEED_PREV || c->grid.seed == SBI_SEED_NET) && c->have_prev) {
            // previous-solve seed: linear guess + the last solve's nonlinear part
            b.term(b.cin(CMP(C_DV)), 2, 1.0, FN_ONE, 0, DV_NONE);
            if (c->vd) b.term(b.cin(CMP(C_DB)), 3, 1.0, FN_ONE, 0, DV_NONE);
        }
        b.cout(SRC_ACC2, CMP(C_VN));
        if (c->vd) b.cout(SRC_ACC3, CMP(C_BN));
    }
    if (!c->vd && b.p.nacc < 3) b.p.nacc = 3;
    return run_col(c, b, K_COL_STATE);
}

static sbi_status row_setup(sbi_ctx* c, const void* eta_user) {
    const bool two_d = c->grid.ny > 1;
    const bool sa = c->grid.mode == SBI_MODE_SA;
    const bool iter = c->grid.mode == SBI_MODE_ITER;
    RowSetupParams rp{};
    rp.g = c->gd;
    rp.g_eta = eta_user ? nullptr : HALF(H_ETA);
    rp.eta_in = eta_user;
    rp.eta_out = eta_user ? nullptr : PHYS(P_ETA);
    rp.g_px = HALF(H_PX);
    rp.g_py = HALF(H_PY);
    rp.px_out = sa ? PHYS(P_PX) : nullptr;
    rp.py_out = (sa && two_d) ? PHYS(P_PY) : nullptr;
    rp.nprod = iter ? (c->grid.order - 1) * (two_d ? 2 : 1) : 0;
    for (int i = 0; i < rp.nprod; ++i) rp.h[i] = HALF(H_PROD0 + i);
    rp.ctl = c->ctl;
    // the two components' product chains in workgroups of their own
    rp.nfam = (two_d && rp.nprod > 0) ? 2 : 1;
    c->st.launches += 1;
    {
        ProfScope ps_(c, K_ROW_SETUP);
        return hip_ok(launch_row_setup(c->fp64, rp, c->batch, tw_of(c), c->stream));
    }
}

// constant parts b_V, b_phi of the summed operator; also fixes omega (CTL_OMEGA)
static sbi_status col_forcing(sbi_ctx* c) {
    const bool two_d = c->grid.ny > 1;
    const int L = c->grid.order;
    ColBuilder b(c->gd);
    int idx = 0;
    std::vector<int> sx(L + 1, -1), sy(L + 1, -1);
    for (int l = 2; l <= L; ++l) {
        sx[l] = b.prod(HALF(H_PROD0 + idx++));
        if (two_d) sy[l] = b.prod(HALF(H_PROD0 + idx++));
    }
    int sp = b.cin(CMP(C_PS));
    b.term(sp, 0, 1.0, FN_T, 1, DV_NONE);
    if (c->vd) b.term(sp, 1, 1.0, FN_S, 0, DV_NONE);
    for (int l = 2; l <= L; ++l) {
        const double cv = -1.0 / fact(l - 1);
        b.term(sx[l], 0, cv, Tfn(l), l - 2, DV_X);
        if (two_d) b.term(sy[l], 0, cv, Tfn(l), l - 2, DV_Y);
        if (c->vd && (l & 1)) {
            b.term(sx[l], 1, cv, FN_S, l - 3, DV_X);
            if (two_d) b.term(sy[l], 1, cv, FN_S, l - 3, DV_Y);
        }
    }
    b.cout(SRC_ACC0, CMP(C_BV));
    if (c->vd) b.cout(SRC_ACC1, CMP(C_BB));
    b.p.ctl = c->ctl;
    b.p.ctl_mode = CTL_OMEGA;
    return run_col(c, b, K_COL_FORCING);
}

// Anderson mixing after the column pass of sweep n (which stored f_n and g_n
// in the history ring): partial inner products, then one column pass whose
// workgroups each solve for the weights w_i of the next iterate and form
// x_(n+1) = sum_i w_i g_i from the history (compact) and its inverse column
// transforms (V, grad phi_b) for the next row pass
static sbi_status anderson_mix(sbi_ctx* c, int n) {
    const bool two_d = c->grid.ny > 1;
    const int k = std::min(n, kAADepth);
    AaParams ap{};
    ap.g = c->gd;
    ap.ctl = c->ctl;
    ap.sweep = n;
    ap.vd = c->vd;
    for (int i = 0; i < kAASlots; ++i) {
        ap.fv[i] = CMP(C_AFV0 + i);
        ap.fb[i] = CMP(C_AFB0 + i);
    }
    ap.partial = c->aa_partial;
    ap.nblk = kAABlocks;
    c->st.launches += 1;
    {
        ProfScope ps_(c, K_COL_OTHER);
        SBI_TRY(hip_ok(launch_aa_dot(c->fp64, ap, c->batch, c->stream)));
    }
    ColBuilder b(c->gd);
    for (int a = 0; a <= k; ++a) {
        const int si = (n - k + a) % kAASlots;
        const int sv = b.cin(CMP(C_AGV0 + si), si);
        b.term(sv, 0, 1.0, FN_ONE, 0, DV_NONE);
        if (c->vd) {
            const int sb = b.cin(CMP(C_AGB0 + si), si);
            b.term(sb, 1, 1.0, FN_ONE, 0, DV_NONE);
        }
    }
    // every workgroup of the pass adds the partials and solves for the weights
    b.p.aa_partial = c->aa_partial;
    b.p.aa_nblk = kAABlocks;
    b.p.aa_sweep = n;
    b.cout(SRC_ACC0, CMP(C_VN));
    b.inv(SRC_ACC0, DV_NONE, HALF(H_GV));
    if (c->vd) {
        b.cout(SRC_ACC1, CMP(C_BN));
        b.inv(SRC_ACC1, DV_X, HALF(H_GBX));
        if (two_d) b.inv(SRC_ACC1, DV_Y, HALF(H_GBY));
    }
    b.p.ctl = c->ctl;
    b.p.ctl_mode = CTL_SKIP;
    return run_col(c, b, K_COL_OTHER);
}

// row pass of a sweep: the residual norms of the previous sweep into slot
// `slot` (residual), and the products of the iterate (products); gT selects
// the residual whose denominator is given as a half form
static RowSweepParams sweep_row_params(sbi_ctx* c, const void* eta_phys, bool residual, bool products, int slot,
                                       bool gT) {
    const bool two_d = c->grid.ny > 1;
    const int J = c->grid.order - 1;
    RowSweepParams rp{};
    rp.g = c->gd;
    rp.gV = HALF(H_GV);
    rp.gD = HALF(H_GD);
    rp.gT = gT ? HALF(H_GT) : nullptr;
    rp.gbx = HALF(H_GBX);
    rp.gby = HALF(H_GBY);
    rp.eta = eta_phys;
    rp.delta = PHYS(P_DELTA);
    rp.J = J;
    rp.residual = residual;
    rp.products = products && J >= 1;
    rp.vd = c->vd;
    rp.slot = slot;
    rp.nfam = rp.products ? 1 + (c->vd ? (two_d ? 2 : 1) : 0) : 1;
    if (rp.products) {
        const int np = J * (1 + (c->vd ? (two_d ? 2 : 1) : 0));
        for (int i = 0; i < np; ++i) rp.h[i] = HALF(H_PROD0 + i);
    }
    rp.ctl = c->ctl;
    return rp;
}

static sbi_status run_row_sweep(sbi_ctx* c, const RowSweepParams& rp) {
    c->st.launches += 1;
    ProfScope ps_(c, K_ROW_SWEEP);
    return hip_ok(launch_row_sweep(c->fp64, rp, c->batch, tw_of(c), c->stream));
}

// terms of T(x) = b + A x in a column pass: the forcing (C_BV, C_BB) and, with
// products, the summed operator applied to the iterate's products; *cvn and
// *cbn are the inputs that hold the iterate x itself (C_VN, C_BN)
static void sweep_col_terms(sbi_ctx* c, ColBuilder& b, bool products, int* cvn, int* cbn) {
    const bool two_d = c->grid.ny > 1;
    const int J = c->grid.order - 1;
    std::vector<int> se(J + 1), sbx(J + 1), sby(J + 1);
    if (products) {
        int idx = 0;
        for (int j = 1; j <= J; ++j) se[j] = b.prod(HALF(H_PROD0 + idx++));
        if (c->vd) {
            for (int j = 1; j <= J; ++j) sbx[j] = b.prod(HALF(H_PROD0 + idx++));
            if (two_d)
                for (int j = 1; j <= J; ++j) sby[j] = b.prod(HALF(H_PROD0 + idx++));
        }
    }
    int cbv = b.cin(CMP(C_BV));
    *cvn = b.cin(CMP(C_VN));
    int cbb = -1;
    *cbn = -1;
    if (c->vd) {
        cbb = b.cin(CMP(C_BB));
        *cbn = b.cin(CMP(C_BN));
    }
    b.term(cbv, 0, 1.0, FN_ONE, 0, DV_NONE);
    if (c->vd) b.term(cbb, 1, 1.0, FN_ONE, 0, DV_NONE);
    if (products) {
        for (int j = 1; j <= J; ++j) {
            const double f = 1.0 / fact(j);
            // V equation: -T_j k^j/j! F{eta^j V} + <j> S k^(j-1)/j! ik.F{delta^j grad phi_b}
            b.term(se[j], 0, -f, Tfn(j), j, DV_NONE);
            if (c->vd) {
                if (j & 1) {
                    b.term(sbx[j], 0, f, FN_S, j - 1, DV_X);
                    if (two_d) b.term(sby[j], 0, f, FN_S, j - 1, DV_Y);
                }
                // phi_b equation: -<j> S k^(j-1)/j! F{eta^j V} + (-1)^j T_j k^(j-2)/j! ik.F{delta^j grad phi_b}
                if (j & 1) b.term(se[j], 1, -f, FN_S, j - 1, DV_NONE);
                const double sg = (j & 1) ? -f : f;
                b.term(sbx[j], 1, sg, Tfn(j), j - 2, DV_X);
                if (two_d) b.term(sby[j], 1, sg, Tfn(j), j - 2, DV_Y);
            }
        }
    }
}

static sbi_status launch_sweep(sbi_ctx* c, const void* eta_phys, int n, double tol) {
    const bool two_d = c->grid.ny > 1;
    const int M = c->grid.max_sweeps;
    const bool aa = c->grid.accel == SBI_ACCEL_ANDERSON;
    const RowSweepParams rp = sweep_row_params(c, eta_phys, n >= 1, n < M, n >= 1 ? n - 1 : 0, aa);
    SBI_TRY(run_row_sweep(c, rp));

    ColBuilder b(c->gd);
    int cvn, cbn;
    sweep_col_terms(c, b, rp.products, &cvn, &cbn);
    if (aa) {
        // T_V(x_n); the residual f_n and the relaxed sweep g_n into the history
        // ring; the half forms of the residual test (f_n and T_V(x_n)).  The
        // next iterate follows once the inner products over the whole spectrum
        // are known.
        const int s = n % kAASlots;
        b.p.relax_prev[0] = -cvn - 1;
        if (c->vd) b.p.relax_prev[1] = -cbn - 1;
        b.cout(SRC_ACC0, CMP(C_VP));
        b.cout(SRC_DIFF0, CMP(C_AFV0 + s));
        b.cout(SRC_NEW0, CMP(C_AGV0 + s));
        if (c->vd) {
            b.cout(SRC_DIFF1, CMP(C_AFB0 + s));
            b.cout(SRC_NEW1, CMP(C_AGB0 + s));
        }
        b.inv(SRC_DIFF0, DV_NONE, HALF(H_GD));
        b.inv(SRC_ACC0, DV_NONE, HALF(H_GT));
    } else {
        b.p.relax_prev[0] = -cvn - 1;  // resolved in build(): encoded as cin index
        if (c->vd) b.p.relax_prev[1] = -cbn - 1;
        b.cout(SRC_ACC0, CMP(C_VP));
        b.cout(SRC_NEW0, CMP(C_VN));
        if (c->vd) b.cout(SRC_NEW1, CMP(C_BN));
        b.inv(SRC_NEW0, DV_NONE, HALF(H_GV));
        b.inv(SRC_DIFF0, DV_NONE, HALF(H_GD));
        if (c->vd) {
            b.inv(SRC_NEW1, DV_X, HALF(H_GBX));
            if (two_d) b.inv(SRC_NEW1, DV_Y, HALF(H_GBY));
        }
    }
    b.p.ctl = c->ctl;
    b.p.ctl_mode = CTL_SWEEP;
    b.p.sweep = n;
    b.p.max_sweeps = M;
    b.p.tol = tol;
    if (b.p.nacc < (c->vd ? 2 : 1)) b.p.nacc = c->vd ? 2 : 1;
    SBI_TRY(run_col(c, b, K_COL_SWEEP));
    // the next iterate is mixed after every sweep but the last, also when the
    // sweep forms no products (order 1: T is the constant b_V)
    if (!aa || n >= M) return SBI_OK;
    return anderson_mix(c, n);
}

static sbi_status read_heads(sbi_ctx* c) {
    SBI_HIP(hipMemcpyAsync(c->head, c->ctl, sizeof(Ctl) * c->batch, hipMemcpyDeviceToHost, c->stream));
    SBI_HIP(hipStreamSynchronize(c->stream));
    c->st.syncs += 1;
    if (c->prof.on) prof_flush(c);
    return SBI_OK;
}

// iteration: device-side convergence decisions, host polls in predicted
// chunks.  At each poll the control headers are copied behind the chunk and
// kAhead more sweeps are enqueued before the host waits for the copy, so the
// device keeps sweeping while the host decides; sweeps enqueued after a
// member's solve was decided return at once.
static sbi_status iterate(sbi_ctx* c, const void* eta_phys, double tol) {
    constexpr int kAhead = 1;
    const int M = c->grid.max_sweeps;
    int n = 0;  // next sweep to enqueue
    int chunk = 4;
    bool final_heads = false;  // c->head reflects every enqueued sweep
    std::vector<double> r_prev(c->batch, -1.0);
    std::vector<int> n_prev(c->batch, 0);
    while (n <= M) {
        for (int i = 0; i < chunk && n <= M; ++i, ++n) SBI_TRY(launch_sweep(c, eta_phys, n, tol));
        const int np = n;  // sweeps the header copy follows
        SBI_HIP(hipMemcpyAsync(c->head, c->ctl, sizeof(Ctl) * c->batch, hipMemcpyDeviceToHost, c->stream));
        if (c->poll) SBI_HIP(hipEventRecord(c->poll, c->stream));
        for (int i = 0; i < kAhead && n <= M; ++i, ++n) SBI_TRY(launch_sweep(c, eta_phys, n, tol));
        // a transient context has no event: it waits for the look-ahead too
        SBI_HIP(c->poll ? hipEventSynchronize(c->poll) : hipStreamSynchronize(c->stream));
        c->st.syncs += 1;
        bool all_done = true;
        int want = 1;
        for (int b = 0; b < c->batch; ++b) {
            const Ctl& h = c->head[b];
            if (h.done) continue;
            all_done = false;
            // residual r_(np-2) is the latest decided one; predict the remaining sweeps
            const double r = h.residual;
            int rem = 4;
            if (r_prev[b] > 0.0 && r > 0.0 && r < r_prev[b] && np - 2 > n_prev[b]) {
                const double rho = std::pow(r / r_prev[b], 1.0 / (double)(np - 2 - n_prev[b]));
                if (rho > 0.0 && rho < 1.0) rem = (int)std::ceil(std::log(tol / r) / std::log(rho)) + 1;
            }
            r_prev[b] = r;
            n_prev[b] = np - 2;
            want = std::max(want, rem);
        }
        if (all_done) {
            final_heads = true;  // later sweeps returned at once and changed no header
            break;
        }
        chunk = std::min(std::max(want - (n - np), 1), 64);
    }
    // the look-ahead sweeps after the last poll may have decided the solves
    if (!final_heads) SBI_TRY(read_heads(c));
    return SBI_OK;
}

// iteration without host polling (capturable): sweep launches 0..B are
// enqueued, B = the context's budget (max_sweeps when unset); after the column
// pass that decides a member's solve, that member's later launches return at
// once.  A solve that needs more than B sweeps stays undecided (its device
// statistics do not count it), which the ensemble step detects and redoes.
static sbi_status iterate_fixed(sbi_ctx* c, const void* eta_phys, double tol) {
    const int M = c->grid.max_sweeps;
    const int B = (c->budget > 0 && c->budget < M) ? c->budget : M;
    for (int n = 0; n <= B; ++n) SBI_TRY(launch_sweep(c, eta_phys, n, tol));
    return SBI_OK;
}

// ---------------------------------------------------------------------------
// mixed precision (SBI_MIXED): iterative refinement of the fixed point
// x = T(x) = A x + b of the iteration (x = (V, phi_b), T affine).  FP64 sweeps
// form r_k = T(x_k) - x_k and take the iteration's stopping decision on it;
// between them the FP32 context solves d = A d + r_k -- the same sweeps with
// the forcing b replaced by r_k, from d = r_k -- and x_(k+1) = x_k + d in
// FP64.  The new residual r_(k+1) = T(x_k + d) - x_k - d = A d + r_k - d is
// the correction solve's own residual, so a correction solved to relative
// residual tau leaves |r_(k+1)| ~ tau |d|: each FP64 sweep gains what the FP32
// sweeps reached, and the FP64 test ends the solve at the FP64 tolerance.
// ---------------------------------------------------------------------------
constexpr int kMixedRefine = 10;        // FP64 sweeps per solve at most
constexpr double kMixedTauMin = 1e-5;   // correction tolerances: above the FP32 floor (~1e-6)
constexpr double kMixedTauMax = 0.1;
constexpr double kMixedHalfAdd = 1e4;   // residuals up to this * tol update the half forms by addition

// half forms of the iterate (C_VN, C_BN) for the next row pass
static sbi_status iterate_half_forms(sbi_ctx* c) {
    const bool two_d = c->grid.ny > 1;
    ColBuilder b(c->gd);
    b.term(b.cin(CMP(C_VN)), 0, 1.0, FN_ONE, 0, DV_NONE);
    b.inv(SRC_ACC0, DV_NONE, HALF(H_GV));
    if (c->vd) {
        b.term(b.cin(CMP(C_BN)), 1, 1.0, FN_ONE, 0, DV_NONE);
        b.inv(SRC_ACC1, DV_X, HALF(H_GBX));
        if (two_d) b.inv(SRC_ACC1, DV_Y, HALF(H_GBY));
    }
    return run_col(c, b, K_COL_OTHER);
}

// FP64 sweep k of the refinement from the iterate x_k (C_VN, C_BN and their
// half forms): T_V(x_k) into C_VP, r_k into C_AFV0 / C_AFB0 (the Anderson ring
// is free: the FP64 side does not mix), the half forms of the residual test,
// and the row pass that reduces the test's norms into slot k
static sbi_status refine_sweep(sbi_ctx* c, const void* eta_phys, int k) {
    SBI_TRY(run_row_sweep(c, sweep_row_params(c, eta_phys, false, true, 0, false)));
    ColBuilder b(c->gd);
    int cvn, cbn;
    sweep_col_terms(c, b, c->grid.order > 1, &cvn, &cbn);
    b.p.relax_prev[0] = -cvn - 1;
    if (c->vd) b.p.relax_prev[1] = -cbn - 1;
    b.cout(SRC_ACC0, CMP(C_VP));
    b.cout(SRC_DIFF0, CMP(C_AFV0));
    if (c->vd) b.cout(SRC_DIFF1, CMP(C_AFB0));
    b.inv(SRC_DIFF0, DV_NONE, HALF(H_GD));
    b.inv(SRC_ACC0, DV_NONE, HALF(H_GT));
    b.p.ctl = c->ctl;
    b.p.ctl_mode = CTL_SKIP;  // decided members keep their result
    if (b.p.nacc < (c->vd ? 2 : 1)) b.p.nacc = c->vd ? 2 : 1;
    SBI_TRY(run_col(c, b, K_COL_SWEEP));
    return run_row_sweep(c, sweep_row_params(c, eta_phys, true, false, k, true));
}

static sbi_status iterate_mixed(sbi_ctx* c, const void* eta_phys, double tol) {
    sbi_ctx* in = c->inner;
    const bool two_d = c->grid.ny > 1;
    const int R = std::min(c->grid.max_sweeps, kMixedRefine);
    const long long nk = (long long)c->gd.Kx * c->gd.Ky;  // kept modes per member
    // the half forms the FP64 row pass reads, and their FP32 counterparts
    void* hout[3] = {HALF(H_GV), HALF(H_GBX), HALF(H_GBY)};
    const void* hin[3] = {in->half[H_GV], in->half[H_GBX], in->half[H_GBY]};
    const int nf = c->vd ? (two_d ? 3 : 2) : 1;
    // the FP32 sweeps' eta (fixed over the solve)
    c->st.launches += 1;
    SBI_TRY(hip_ok(launch_to_float(eta_phys, in->phys[P_ETA], c->gd.s_phys * c->batch, c->stream)));
    for (int k = 0;; ++k) {
        SBI_TRY(refine_sweep(c, eta_phys, k));
        c->st.launches += 1;
        SBI_TRY(hip_ok(launch_ctl_decide(c->ctl, c->batch, k + 1, R, tol, c->stream)));
        SBI_HIP(hipMemcpyAsync(c->head, c->ctl, sizeof(Ctl) * c->batch, hipMemcpyDeviceToHost, c->stream));
        if (c->poll) SBI_HIP(hipEventRecord(c->poll, c->stream));
        // while the host waits for the decision, the next correction solve is
        // set up (members the decision ended are skipped)
        SBI_TRY(hip_ok(launch_ctl_reset(in->ctl, in->batch, in->grid.max_sweeps + 2, c->stream)));
        SBI_TRY(hip_ok(launch_mixed_down(c->ctl, in->ctl, c->batch, CMP(C_AFV0), CMP(C_AFB0), in->comp[C_BV],
                                         in->comp[C_VN], in->comp[C_BB], in->comp[C_BN], nk, c->gd.s_cmp,
                                         in->gd.s_cmp, c->vd, c->stream)));
        SBI_TRY(iterate_half_forms(in));
        SBI_HIP(c->poll ? hipEventSynchronize(c->poll) : hipStreamSynchronize(c->stream));
        c->st.syncs += 1;
        if (c->prof.on) prof_flush(c);
        double rho = 0.0;
        bool all_done = true;
        for (int b = 0; b < c->batch; ++b) {
            if (c->head[b].done) continue;
            all_done = false;
            rho = std::max(rho, c->head[b].residual);
        }
        if (all_done) break;
        // a correction solved to tau leaves a residual ~ tau rho: aim below
        // tol, within what the FP32 sweeps reach
        const double tau = std::min(kMixedTauMax, std::max(kMixedTauMin, 0.3 * tol / rho));
        SBI_TRY(iterate(in, in->phys[P_ETA], tau));
        SBI_TRY(hip_ok(launch_mixed_up(c->ctl, in->ctl, c->batch, CMP(C_VN), CMP(C_BN), in->comp[C_VN],
                                       in->comp[C_BN], nk, c->gd.s_cmp, in->gd.s_cmp, c->vd, k + 1, c->stream)));
        // the half forms of x + d: the FP32 half forms of d carry FP32 rounding
        // of the column transforms, ~1e-7 |d| ~ 1e-7 rho |V|, which the
        // iteration never removes -- taken only when that is far below tol
        // (late corrections); early ones transform x + d again in FP64
        if (rho > kMixedHalfAdd * tol) {
            SBI_TRY(iterate_half_forms(c));
        } else {
            c->st.launches += 1;
            SBI_TRY(hip_ok(launch_mixed_up_half(in->ctl, c->batch, hout, hin, nf, c->gd.Kx, c->grid.ny, c->gd.ldh,
                                                in->gd.ldh, c->gd.s_half, in->gd.s_half, c->stream)));
        }
        c->st.launches += 3 + in->st.launches;
        c->st.syncs += in->st.syncs;
        in->st = Stats();
    }
    c->st.launches += 2 + in->st.launches;  // the set-up enqueued behind the last decision
    in->st = Stats();
    return SBI_OK;
}

static sbi_status run_sa(sbi_ctx* c, const void* eta_phys) {
    const bool two_d = c->grid.ny > 1;
    const int L = c->grid.order;
    for (int l = 2; l <= L; ++l) {
        RowSaParams rp{};
        rp.g = c->gd;
        rp.l = l;
        rp.vd = c->vd;
        rp.gV = HALF(H_GV);
        rp.gbx = HALF(H_GBX);
        rp.gby = HALF(H_GBY);
        rp.V_out = PHYS(P_V0 + (l - 2));      // V_(l-1)
        rp.bx_out = c->vd ? PHYS(P_BX0 + (l - 2)) : nullptr;
        rp.by_out = (c->vd && two_d) ? PHYS(P_BY0 + (l - 2)) : nullptr;
        for (int m = 1; m < l; ++m) {
            rp.Vphys[m] = PHYS(P_V0 + (m - 1));
            rp.bxphys[m] = PHYS(P_BX0 + (m - 1));
            rp.byphys[m] = PHYS(P_BY0 + (m - 1));
        }
        rp.eta = eta_phys;
        rp.delta = PHYS(P_DELTA);
        rp.phx = PHYS(P_PX);
        rp.phy = PHYS(P_PY);
        const int np = (l - 1) * (1 + (c->vd ? (two_d ? 2 : 1) : 0)) + (two_d ? 2 : 1);
        if (np > kMaxProd) return SBI_ERR_UNSUPPORTED;
        for (int i = 0; i < np; ++i) rp.h[i] = HALF(H_PROD0 + i);
        // few rows (a 1D grid, or up to 1024 rows over all members): one
        // workgroup per product, so that the pass is not one long chain of
        // transforms per row block
        rp.split = (!two_d || (long long)c->grid.ny * c->batch <= 1024) ? np : 0;
        c->st.launches += 1;
        {
        ProfScope ps_(c, K_ROW_SA);
        SBI_TRY(hip_ok(launch_row_sa(c->fp64, rp, c->batch, tw_of(c), c->stream)));
    }

        ColBuilder b(c->gd);
        int idx = 0;
        std::vector<int> se(l), sbx(l), sby(l);
        for (int j = 1; j <= l - 1; ++j) se[j] = b.prod(HALF(H_PROD0 + idx++));
        if (c->vd) {
            for (int j = 1; j <= l - 1; ++j) sbx[j] = b.prod(HALF(H_PROD0 + idx++));
            if (two_d)
                for (int j = 1; j <= l - 1; ++j) sby[j] = b.prod(HALF(H_PROD0 + idx++));
        }
        int fx = b.prod(HALF(H_PROD0 + idx++));
        int fy = two_d ? b.prod(HALF(H_PROD0 + idx++)) : -1;
        int cvh = b.cin(CMP(C_VH));
        const bool want_b = c->vd && l <= L - 1;
        // acc0 = V_l, acc1 = phi_b,l, acc2 = running sum of V
        auto both = [&](int src, double coef, int fn, int pw, int dv) {
            b.term(src, 0, coef, fn, pw, dv);
            b.term(src, 2, coef, fn, pw, dv);
        };
        for (int j = 1; j <= l - 1; ++j) {
            const double f = 1.0 / fact(j);
            both(se[j], -f, Tfn(j), j, DV_NONE);
            if (want_b && (j & 1)) b.term(se[j], 1, -f, FN_S, j - 1, DV_NONE);
            if (c->vd) {
                if (j & 1) {
                    both(sbx[j], f, FN_S, j - 1, DV_X);
                    if (two_d) both(sby[j], f, FN_S, j - 1, DV_Y);
                }
                if (want_b) {
                    const double sg = (j & 1) ? -f : f;
                    b.term(sbx[j], 1, sg, Tfn(j), j - 2, DV_X);
                    if (two_d) b.term(sby[j], 1, sg, Tfn(j), j - 2, DV_Y);
                }
            }
        }
        const double fl = -1.0 / fact(l - 1);
        both(fx, fl, Tfn(l), l - 2, DV_X);
        if (two_d) both(fy, fl, Tfn(l), l - 2, DV_Y);
        if (want_b && (l & 1)) {
            b.term(fx, 1, fl, FN_S, l - 3, DV_X);
            if (two_d) b.term(fy, 1, fl, FN_S, l - 3, DV_Y);
        }
        b.term(cvh, 2, 1.0, FN_ONE, 0, DV_NONE);
        b.p.nacc = 3;
        b.cout(SRC_ACC2, CMP(C_VH));
        if (l < L) {
            b.inv(SRC_ACC0, DV_NONE, HALF(H_GV));
            if (want_b) {
                b.inv(SRC_ACC1, DV_X, HALF(H_GBX));
                if (two_d) b.inv(SRC_ACC1, DV_Y, HALF(H_GBY));
            }
        } else {
            b.inv(SRC_ACC2, DV_NONE, HALF(H_GV));
        }
        SBI_TRY(run_col(c, b, K_COL_SA));
    }
    return SBI_OK;
}

// W solve at the stage state held in (C_ES, C_PS) [or physical eta_user with
// C_PS]; leaves the W spectrum in *vh_buf and its half form in H_GV (+ H_GD).
// seed of the iteration from a physical field: V_0 = mask F{w_seed}
static sbi_status seed_from_physical(sbi_ctx* c, const void* w_seed) {
    RowFwdParams rp{};
    rp.g = c->gd;
    rp.nf = 1;
    rp.in[0] = w_seed;
    rp.out[0] = HALF(H_PROD0);
    c->st.launches += 1;
    {
        ProfScope ps_(c, K_ROW_FWD);
        SBI_TRY(hip_ok(launch_row_fwd(c->fp64, rp, c->batch, tw_of(c), c->stream)));
    }
    ColBuilder b(c->gd);
    int s = b.prod(HALF(H_PROD0));
    b.term(s, 0, 1.0, FN_ONE, 0, DV_NONE);
    b.cout(SRC_ACC0, CMP(C_VN));
    b.inv(SRC_ACC0, DV_NONE, HALF(H_GV));
    return run_col(c, b);
}

// features of the learned warm start at the stage state: reads the half forms
// left by stage_state_pass (W_lin in H_GV, gradients in H_EX/H_EY/H_PX/H_PY)
static sbi_status row_features(sbi_ctx* c, const void* eta_phys, float* feat, void* wlin) {
    RowFeatParams fp{};
    fp.g = c->gd;
    fp.gV = HALF(H_GV);
    fp.gex = HALF(H_EX);
    fp.gey = HALF(H_EY);
    fp.gpx = HALF(H_PX);
    fp.gpy = HALF(H_PY);
    fp.eta = eta_phys;
    fp.delta = PHYS(P_DELTA);
    for (int i = 0; i < 8; ++i) fp.scale[i] = c->net_scale[i];
    fp.feat = feat;
    fp.wlin = wlin;
    c->st.launches += 1;
    ProfScope ps_(c, K_NET);
    return hip_ok(launch_row_feat(c->fp64, fp, c->batch, tw_of(c), c->stream));
}

static sbi_status net_infer(sbi_ctx* c, const float* feat, const void* wlin, void* out, void* out_b) {
    NetInferParams ip{};
    ip.feat = feat;
    ip.wlin = wlin;
    ip.out = out;
    ip.out_b = out_b;
    ip.w = c->net;
    ip.ny = c->grid.ny;
    ip.nx = c->grid.nx;
    ip.s_phys = c->gd.s_phys;
    c->st.launches += 1;
    ProfScope ps_(c, K_NET);
    return hip_ok(launch_net_infer(c->fp64, ip, c->batch, c->stream));
}

// learned seeds: V0 = W_lin + out_scale[0] y[0] and phi_b0 = S phi_hat +
// mask F{out_scale[1] y[1]} set as the iterate (runs after stage_state_pass,
// which left the linear guesses in C_VN / C_BN)
static sbi_status net_seed(sbi_ctx* c, const void* eta_phys) {
    if (!c->net_loaded || !c->feat) return SBI_ERR_INVALID_ARG;
    SBI_TRY(row_features(c, eta_phys, c->feat, PHYS(P_V0)));
    SBI_TRY(net_infer(c, c->feat, PHYS(P_V0), PHYS(P_V0 + 1), PHYS(P_V0 + 2)));
    RowFwdParams rp{};
    rp.g = c->gd;
    rp.nf = c->vd ? 2 : 1;
    rp.in[0] = PHYS(P_V0 + 1);
    rp.out[0] = HALF(H_PROD0);
    rp.in[1] = PHYS(P_V0 + 2);
    rp.out[1] = HALF(H_PROD0 + 1);
    c->st.launches += 1;
    {
        ProfScope ps_(c, K_NET);
        SBI_TRY(hip_ok(launch_row_fwd(c->fp64, rp, c->batch, tw_of(c), c->stream)));
    }
    ColBuilder b(c->gd);
    int sv = b.prod(HALF(H_PROD0));
    b.term(sv, 0, 1.0, FN_ONE, 0, DV_NONE);
    b.cout(SRC_ACC0, CMP(C_VN));
    b.inv(SRC_ACC0, DV_NONE, HALF(H_GV));
    if (c->vd) {
        const bool two_d = c->grid.ny > 1;
        int sb = b.prod(HALF(H_PROD0 + 1));
        int cb = b.cin(CMP(C_BN));
        b.term(sb, 1, 1.0, FN_ONE, 0, DV_NONE);
        b.term(cb, 1, 1.0, FN_ONE, 0, DV_NONE);
        b.cout(SRC_ACC1, CMP(C_BN));
        b.inv(SRC_ACC1, DV_X, HALF(H_GBX));
        if (two_d) b.inv(SRC_ACC1, DV_Y, HALF(H_GBY));
    }
    return run_col(c, b, K_NET);
}

// keeps (V* - kT phi_hat, phi_b - S phi_hat) of the finished solve: the seed of
// the next one adds them to its own linear guess.  phi_b is the iterate after
// the relaxed update of the last sweep.
static sbi_status save_nonlinear_part(sbi_ctx* c) {
    ColBuilder b(c->gd);
    int sv = b.cin(CMP(C_VP));
    int sp = b.cin(CMP(C_PS));
    b.term(sv, 0, 1.0, FN_ONE, 0, DV_NONE);
    b.term(sp, 0, -1.0, FN_T, 1, DV_NONE);
    b.cout(SRC_ACC0, CMP(C_DV));
    if (c->vd) {
        int sb = b.cin(CMP(C_BN));
        b.term(sb, 1, 1.0, FN_ONE, 0, DV_NONE);
        b.term(sp, 1, -1.0, FN_S, 0, DV_NONE);
        b.cout(SRC_ACC1, CMP(C_DB));
    }
    SBI_TRY(run_col(c, b));
    c->have_prev = true;
    return SBI_OK;
}

static HistParams hist_params(sbi_ctx* c, int stage) {
    HistParams hp{};
    hp.g = c->gd;
    hp.K = c->hist_K;
    hp.nb = c->hist_nb;
    hp.dk = c->hist_dk;
    hp.stage = stage;
    hp.vd = c->vd;
    hp.dev = c->hist_dev;
    for (int q = 0; q < kHistTaps; ++q) {
        hp.hv[q] = CMP(C_HV0 + q);
        hp.hb[q] = CMP(C_HB0 + q);
    }
    hp.tv = CMP(C_DV);
    hp.tb = CMP(C_DB);
    hp.pv = CMP(C_PV);
    hp.pb = CMP(C_PB);
    hp.partial = c->hist_partial;
    return hp;
}

// After a solve of a context with the learned history layer: a fixed-step
// solve (stage >= 0) adds its nonlinear part (C_DV, C_DB) to the history --
// first, when training, accumulating the gradient of predicting it from the
// history; any other solve empties the history.
static sbi_status hist_after_solve(sbi_ctx* c, int stage, bool capture_safe) {
    if (!c->hist_loaded || c->grid.mode != SBI_MODE_ITER) return SBI_OK;
    if (stage < 0) {
        c->hist_count = 0;
        return SBI_OK;
    }
    const HistParams hp = hist_params(c, stage);
    if (c->hist_train && !capture_safe && c->hist_count >= c->hist_K) {
        c->st.launches += 2;
        SBI_TRY(hip_ok(launch_hist_grad(c->fp64, hp, c->batch, c->stream)));
        SBI_TRY(hip_ok(launch_hist_reduce(hp, c->batch, c->stream)));
    }
    c->st.launches += 1;
    SBI_TRY(hip_ok(launch_hist_push(c->fp64, hp, c->batch, c->stream)));
    c->hist_count = std::min(c->hist_count + 1, kHistTaps);
    return SBI_OK;
}

// W solve at the stage state.  stage: the RK4 stage (0..3) of a fixed-step
// solve, -1 for any other solve.  capture_safe: no host synchronisation
// (fixed sweep launches, no fallback from a failed learned seed).
// ---------------------------------------------------------------------------
// Fully nonlinear W (SBI_MODE_FULL, one dimension): the boundary-integral
// equations with the remaining integrals kept (sbi_full.hip) -- over a flat
// bed by its image, over a variable bed with the bed as a second boundary
// ---------------------------------------------------------------------------
// physical work fields of the solve (the SA order slots, unused in this mode)
enum { PF_PHI = P_V0, PF_EX, PF_EXX, PF_V, PF_B0, PF_B1 };

static FullParams full_params(sbi_ctx* c) {
    FullParams p{};
    p.n = c->grid.nx;
    p.batch = c->batch;
    p.lx = c->grid.lx;
    p.s_phys = c->gd.s_phys;
    p.href = c->href_dev;
    p.c0 = c->full_c0;
    p.d1 = c->full_d1;
    p.d2 = c->full_d2;
    p.s2 = c->full_s2;
    p.s2a = c->full_s2a;
    p.rs2 = c->full_rs2;
    p.part = c->full_part;
    p.phi = PHYS(PF_PHI);
    p.ex = PHYS(PF_EX);
    p.exx = PHYS(PF_EXX);
    p.rhs = c->full_rhs;
    p.lfl = c->full_lfl;
    p.w = c->full_w;
    p.vbuf[0] = PHYS(PF_B0);
    p.vbuf[1] = PHYS(PF_B1);
    p.vfinal = PHYS(PF_V);
    p.ctl = c->ctl;
    p.max_sweeps = c->grid.max_sweeps;
    p.bed = c->full_bed_any ? c->full_bed : nullptr;
    p.bz = c->full_bz;
    p.bx = c->full_bx;
    p.bxx = c->full_bxx;
    p.cm = c->full_cm;
    p.rb = c->full_rb;
    // source-point slices: enough workgroups to fill the GPU (about 256)
    const int tiles = (p.n + 255) / 256;
    p.nsplit = std::max(1, std::min(kFullSplitMax, 256 / std::max(1, tiles * c->batch)));
    return p;
}

static sbi_status full_tables(sbi_ctx* c) {
    FullParams p = full_params(c);
    c->st.launches += 1;
    SBI_TRY(hip_ok(launch_full(c->fp64, p, FULL_TABLES, c->stream)));
    if (!c->full_bed_any) return SBI_OK;
    c->st.launches += 1;
    return hip_ok(launch_full(c->fp64, p, FULL_BEDGEOM, c->stream));  // b_x, b_xx from the d1, d2 tables
}

static sbi_status full_solve(sbi_ctx* c, const void* eta_phys, double tol) {
    // phi_s at the points (the band-limited stage potential)
    {
        ColBuilder b(c->gd);
        b.term(b.cin(CMP(C_PS)), 0, 1.0, FN_ONE, 0, DV_NONE);
        b.inv(SRC_ACC0, DV_NONE, HALF(H_PROD0));
        SBI_TRY(run_col(c, b));
        RowInvParams ip{};
        ip.g = c->gd;
        ip.nf = 1;
        ip.in[0] = HALF(H_PROD0);
        ip.out[0] = PHYS(PF_PHI);
        ip.ctl = c->ctl;
        c->st.launches += 1;
        ProfScope ps_(c, K_ROW_INV);
        SBI_TRY(hip_ok(launch_row_inv(c->fp64, ip, c->batch, tw_of(c), c->stream)));
    }
    FullParams p = full_params(c);
    p.eta = eta_phys;
    p.tol = tol;
    c->st.launches += 3;
    SBI_TRY(hip_ok(launch_full(c->fp64, p, FULL_GEOM, c->stream)));
    SBI_TRY(hip_ok(launch_full(c->fp64, p, FULL_DOUBLE, c->stream)));
    SBI_TRY(hip_ok(launch_full(c->fp64, p, FULL_RHS, c->stream)));
    const bool bed = c->full_bed_any;
    // the image form's single layer by its symmetric pass (each pair once) where
    // the grid holds two tiles or more
    const bool sym = p.n >= 2 * kFullSymTile;
    p.nsym = sym ? p.n / kFullSymTile : 0;
    if (bed) {
        // the bed's right-hand side -D_BS[phi_s] of the two-boundary members
        c->st.launches += 2;
        SBI_TRY(hip_ok(launch_full(c->fp64, p, FULL_RHSB, c->stream)));
        SBI_TRY(hip_ok(launch_full(c->fp64, p, FULL_RB, c->stream)));
    }
    // launch n: the pair pass decides from the residual of launch n - 1 and
    // forms (S - S0)[V_n]; the apply pass forms V_(n+1) and its residual.
    // Two-boundary members first update phi_b (the bed pass, which then
    // decides, and the phi_b pass), and their surface pass runs from the first
    // launch (phi_b is not zero there).  V_0 = 0, V_n lives in vbuf[n & 1],
    // phi_b of launch n in pb[n & 1]; the host polls after a first chunk as
    // long as the last solve took (and one launch more), then every kChunk.
    const int M = c->grid.max_sweeps;
    constexpr int kChunk = 8;
    int chunk = c->full_pred > 0 ? c->full_pred + 1 : kChunk;
    bool all = false;
    for (int n0 = 0; n0 <= M; n0 += chunk, chunk = kChunk) {
        for (int n = n0; n <= M && n < n0 + chunk; ++n) {
            p.sweep = n;
            p.vin = n == 0 ? nullptr : p.vbuf[n & 1];
            p.vout = const_cast<void*>(p.vbuf[(n + 1) & 1]);
            p.pbin = n == 0 ? nullptr : c->full_pb[n & 1];
            p.pbout = c->full_pb[(n + 1) & 1];
            if (bed) {
                ProfScope ps_(c, K_FULL_PAIRS);
                if (n > 0) {
                    c->st.launches += 1;
                    SBI_TRY(hip_ok(launch_full(c->fp64, p, FULL_BED, c->stream)));
                }
                c->st.launches += 2;
                SBI_TRY(hip_ok(launch_full(c->fp64, p, FULL_PB, c->stream)));
                SBI_TRY(hip_ok(launch_full(c->fp64, p, FULL_SURF, c->stream)));
            }
            if (n > 0 && !c->full_bed_all) {
                ProfScope ps_(c, K_FULL_PAIRS);
                c->st.launches += 1;
                SBI_TRY(hip_ok(launch_full(c->fp64, p, sym ? FULL_SYM : FULL_SINGLE, c->stream)));
            }
            c->st.launches += 3;
            ProfScope ps2_(c, K_FULL_APPLY);
            SBI_TRY(hip_ok(launch_full(c->fp64, p, FULL_COMBINE, c->stream)));
            SBI_TRY(hip_ok(launch_full(c->fp64, p, FULL_APPLY, c->stream)));
        }
        SBI_TRY(read_heads(c));
        all = true;
        for (int b = 0; b < c->batch; ++b) all = all && c->head[b].done;
        if (all) break;
    }
    if (all) {
        // the deciding launch of each member is its sweep count
        int last = 0;
        for (int b = 0; b < c->batch; ++b) last = std::max(last, c->head[b].sweeps);
        c->full_pred = last + 1;
    }
    c->st.launches += 1;
    SBI_TRY(hip_ok(launch_full(c->fp64, p, FULL_SELECT, c->stream)));
    // the spectrum of W (kept band) and its half form
    RowFwdParams rp{};
    rp.g = c->gd;
    rp.nf = 1;
    rp.in[0] = PHYS(PF_V);
    rp.out[0] = HALF(H_PROD0);
    c->st.launches += 1;
    {
        ProfScope ps_(c, K_ROW_FWD);
        SBI_TRY(hip_ok(launch_row_fwd(c->fp64, rp, c->batch, tw_of(c), c->stream)));
    }
    ColBuilder b(c->gd);
    b.term(b.prod(HALF(H_PROD0)), 0, 1.0, FN_ONE, 0, DV_NONE);
    b.cout(SRC_ACC0, CMP(C_VH));
    b.inv(SRC_ACC0, DV_NONE, HALF(H_GV));
    return run_col(c, b);
}

static sbi_status solve_stage(sbi_ctx* c, const void* eta_user, double tol, bool need_eta_grad, int* vh_buf,
                              const void* w_seed = nullptr, bool capture_safe = false, int stage = -1) {
    SBI_TRY(hip_ok(launch_ctl_reset(c->ctl, c->batch, c->grid.max_sweeps + 2, c->stream)));
    c->st.launches += 1;
    const bool iter = c->grid.mode == SBI_MODE_ITER;
    const bool netseed = iter && c->grid.seed == SBI_SEED_NET;
    // the learned history layer seeds fixed-step solves with a full history;
    // the network seeds solves that have no previous solve to start from
    const bool hist = netseed && c->hist_loaded && stage >= 0 && c->hist_count >= c->hist_K && !w_seed;
    const bool net = netseed && c->net_loaded && !hist && !c->have_prev && !w_seed;
    if (hist) {
        c->st.launches += 1;
        ProfScope ps_(c, K_NET);
        SBI_TRY(hip_ok(launch_hist_seed(c->fp64, hist_params(c, stage), c->batch, c->stream)));
    }
    SBI_TRY(stage_state_pass(c, need_eta_grad || !eta_user || net, true, hist));
    SBI_TRY(row_setup(c, eta_user));
    const void* eta_phys = eta_user ? eta_user : PHYS(P_ETA);
    if (c->grid.mode == SBI_MODE_SA) {
        SBI_TRY(run_sa(c, eta_phys));
        *vh_buf = C_VH;
    } else if (c->grid.mode == SBI_MODE_FULL) {
        SBI_TRY(full_solve(c, eta_phys, tol));
        *vh_buf = C_VH;
    } else {
        SBI_TRY(col_forcing(c));
        if (net) SBI_TRY(net_seed(c, eta_phys));
        if (w_seed) SBI_TRY(seed_from_physical(c, w_seed));
        if (capture_safe) {
            SBI_TRY(iterate_fixed(c, eta_phys, tol));
        } else if (c->inner) {
            SBI_TRY(iterate_mixed(c, eta_phys, tol));
        } else {
            SBI_TRY(iterate(c, eta_phys, tol));
        }
        if ((net || hist) && !capture_safe) {
            // the linear guess is the fallback when a learned seed fails
            bool failed = false;
            for (int b = 0; b < c->batch; ++b) failed |= c->head[b].status < 0 || c->head[b].nonfinite;
            if (failed) {
                c->fallbacks += 1;
                SBI_TRY(hip_ok(launch_ctl_reset(c->ctl, c->batch, c->grid.max_sweeps + 2, c->stream)));
                SBI_TRY(stage_state_pass(c, false, false, false));
                SBI_TRY(row_setup(c, eta_user));
                SBI_TRY(col_forcing(c));
                SBI_TRY(c->inner ? iterate_mixed(c, eta_phys, tol) : iterate(c, eta_phys, tol));
            }
        }
        *vh_buf = C_VP;
        if (c->grid.seed == SBI_SEED_PREV || c->grid.seed == SBI_SEED_NET) SBI_TRY(save_nonlinear_part(c));
        SBI_TRY(hist_after_solve(c, stage, capture_safe));
    }
    return SBI_OK;
}

static sbi_status solve_status(sbi_ctx* c, sbi_solve_info* info, bool fresh) {
    if (!fresh) SBI_TRY(read_heads(c));
    sbi_status worst = SBI_OK;
    for (int b = 0; b < c->batch; ++b) {
        const Ctl& h = c->head[b];
        int s = c->grid.mode == SBI_MODE_SA ? 0 : h.status;
        if (h.nonfinite) s = SBI_ERR_NONFINITE;
        if (info) {
            info[b].sweeps = c->grid.mode == SBI_MODE_SA ? 0 : h.sweeps;
            info[b].status = s;
            info[b].residual = h.residual;
            info[b].omega = h.omega;
            info[b].sweeps_fp32 = c->grid.mode == SBI_MODE_SA ? 0 : h.sweeps_inner;
        }
        c->st.sweeps += c->grid.mode == SBI_MODE_SA ? 0 : h.sweeps;
        if (s < 0) worst = (worst < 0) ? worst : (sbi_status)s;
        else if (worst >= 0 && s > worst) worst = (sbi_status)s;
    }
    if (worst < 0) {
        c->have_prev = false;  // a failed solve seeds nothing
        c->hist_count = 0;
    }
    return worst;
}

static sbi_status vertical_velocity(sbi_ctx* c, const void* eta, const void* phi_s, const double* h, double tol,
                                    const void* w_seed, void* w_out, sbi_solve_info* info);

extern "C" sbi_status sbi_vertical_velocity(sbi_ctx* c, const void* eta, const void* phi_s, const double* h,
                                            double tol, const void* w_seed, void* w_out, sbi_solve_info* info) {
    if (!c) return SBI_ERR_INVALID_ARG;
    return vertical_velocity(c, eta, phi_s, h, tol, w_seed, w_out, info);
}

// ---------------------------------------------------------------------------
// W solve without any allocation (sbi_vertical_velocity_noalloc)
// ---------------------------------------------------------------------------
namespace {
// Device scratch of the allocation-free entry point: its transient context's
// workspace.  Each device holds its own copy for the life of the process; in
// host code `scratch` only names the symbol, its device address comes from
// hipGetSymbolAddress (per device, cached in scratch_dev).
constexpr size_t kScratchBytes = size_t(64) << 20;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];
constexpr int kScratchDevices = 64;
std::mutex scratch_mu;
void* scratch_dev[kScratchDevices] = {};
}  // namespace

// address of this device's scratch array (the current device), looked up once
static sbi_status scratch_ptr(void** out) {
    int dev = -1;
    SBI_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= kScratchDevices) return SBI_ERR_UNSUPPORTED;
    std::lock_guard<std::mutex> lock(scratch_mu);
    if (!scratch_dev[dev]) {
        void* p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return SBI_ERR_HIP;
        scratch_dev[dev] = p;
    }
    *out = scratch_dev[dev];
    return SBI_OK;
}

extern "C" sbi_status sbi_vertical_velocity_noalloc(const sbi_grid* g, int32_t batch, const double* depth,
                                                    double h_ref, const void* eta, const void* phi_s, double tol,
                                                    const void* w_seed, void* w_out, sbi_solve_info* info,
                                                    void* hip_stream) {
    if (!grid_valid(g) || batch < 1 || !depth || !eta || !phi_s || !w_out) return SBI_ERR_INVALID_ARG;
    if (g->seed == SBI_SEED_NET) return SBI_ERR_UNSUPPORTED;  // needs loaded weights: a lasting context
    if (g->precision == SBI_MIXED) return SBI_ERR_UNSUPPORTED;  // a second context for the FP32 sweeps
    const size_t need = layout(g, batch).total;
    if (need > kScratchBytes) return SBI_ERR_WORKSPACE;
    // the stream must belong to the current device, whose scratch is used
    if (hip_stream) {
        int sdev = -1, dev = -1;
        SBI_HIP(hipStreamGetDevice(static_cast<hipStream_t>(hip_stream), &sdev));
        SBI_HIP(hipGetDevice(&dev));
        if (sdev != dev) return SBI_ERR_INVALID_ARG;
    }
    void* ws = nullptr;
    SBI_TRY(scratch_ptr(&ws));
    sbi_ctx c;
    // the setup clears the whole workspace with a fill kernel before use, so
    // nothing of an earlier call's contents is read
    sbi_status st = ctx_setup(&c, g, batch, depth, h_ref, ws, kScratchBytes, hip_stream, true);
    const sbi_status warn = st;
    if (st >= 0) st = vertical_velocity(&c, eta, phi_s, nullptr, tol, w_seed, w_out, info);
    (void)hipStreamSynchronize(c.stream);
    if (st < 0) return st;
    return st != SBI_OK ? st : warn;
}

static sbi_status vertical_velocity(sbi_ctx* c, const void* eta, const void* phi_s, const double* h, double tol,
                                    const void* w_seed, void* w_out, sbi_solve_info* info) {
    if (!eta || !phi_s || !w_out) return SBI_ERR_INVALID_ARG;
    if (c->grid.mode != SBI_MODE_SA && !(tol >= 0.0)) return SBI_ERR_INVALID_ARG;
    if (c->grid.seed == SBI_SEED_USER && !w_seed) return SBI_ERR_INVALID_ARG;
    c->st = Stats();
    sbi_status warn = SBI_OK;
    if (h) {
        SBI_TRY(set_depth(c, h, -1.0));
        if (c->depth_warn) warn = SBI_WARN_DEPTH_CRITERION;
    }
    // the learned seed needs the masked spectrum of eta for its gradient features
    const bool net = c->grid.seed == SBI_SEED_NET && c->grid.mode == SBI_MODE_ITER && !c->have_prev &&
                     c->net_loaded;
    c->fallbacks = 0;
    SBI_TRY(to_spectral(c, net ? eta : nullptr, phi_s, false));
    int vh = 0;
    SBI_TRY(solve_stage(c, eta, tol, false, &vh,
                        (c->grid.seed == SBI_SEED_USER && c->grid.mode == SBI_MODE_ITER) ? w_seed : nullptr));
    sbi_status st = solve_status(c, info, false);
    if (st < 0) return st;
    // W = T_V(V_n) of the deciding sweep: in half form for the mixed iteration,
    // else V_(n+1) + (1 - omega) D_n from the relaxed update
    const bool iter = c->grid.mode == SBI_MODE_ITER;
    const bool aa = iter && c->grid.accel == SBI_ACCEL_ANDERSON;
    RowInvParams ip{};
    ip.g = c->gd;
    ip.nf = 1;
    ip.in[0] = aa ? HALF(H_GT) : HALF(H_GV);
    ip.in2[0] = iter && !aa ? HALF(H_GD) : nullptr;
    ip.out[0] = w_out;
    ip.ctl = c->ctl;
    c->st.launches += 1;
    {
        ProfScope ps_(c, K_ROW_INV);
        SBI_TRY(hip_ok(launch_row_inv(c->fp64, ip, c->batch, tw_of(c), c->stream)));
    }
    SBI_HIP(hipStreamSynchronize(c->stream));
    if (st == SBI_OK && c->fallbacks > 0) st = SBI_WARN_FALLBACK_USED;
    return st != SBI_OK ? st : warn;
}

// nonlinear term of the potential equation at the stage state and time t -> C_NP
// (with the wave tank's wavemaker pressure; its damping pressure -> C_PD)
static sbi_status nonlinear_term(sbi_ctx* c, double t) {
    const bool iter = c->grid.mode == SBI_MODE_ITER;
    const bool damp = c->dmp_w > 0.0;
    // W at the stage state as in sbi_vertical_velocity
    const bool aa = iter && c->grid.accel == SBI_ACCEL_ANDERSON;
    RowNphiParams np{};
    np.g = c->gd;
    np.gV = aa ? HALF(H_GT) : HALF(H_GV);
    np.gD = iter && !aa ? HALF(H_GD) : nullptr;
    np.gex = HALF(H_EX);
    np.gey = HALF(H_EY);
    np.gpx = HALF(H_PX);
    np.gpy = HALF(H_PY);
    np.h = HALF(H_PROD0);
    np.ctl = c->ctl;
    np.wm_n = c->wm_n;
    std::memcpy(np.wm, c->wm, sizeof(np.wm));
    np.wm_h = c->wm_h;
    np.t = t;
    np.dmp_x0 = c->dmp_x0;
    np.dmp_w = damp ? c->dmp_w : 0.0;
    np.hdx = damp ? HALF(H_PROD0 + 1) : nullptr;
    np.hdy = damp && c->grid.ny > 1 ? HALF(H_PROD0 + 2) : nullptr;
    c->st.launches += 1;
    {
        ProfScope ps_(c, K_ROW_NPHI);
        SBI_TRY(hip_ok(launch_row_nphi(c->fp64, np, c->batch, tw_of(c), c->stream)));
    }
    ColBuilder b(c->gd);
    int s = b.prod(HALF(H_PROD0));
    b.term(s, 0, 1.0, FN_ONE, 0, DV_NONE);
    b.cout(SRC_ACC0, CMP(C_NP));
    if (damp) {
        // divergence i k . MF{mu grad phi}; the stage kernels divide it by k^2
        int sx = b.prod(HALF(H_PROD0 + 1));
        b.term(sx, 1, 1.0, FN_ONE, 0, DV_X);
        if (c->grid.ny > 1) {
            int sy = b.prod(HALF(H_PROD0 + 2));
            b.term(sy, 1, 1.0, FN_ONE, 0, DV_Y);
        }
        b.cout(SRC_ACC1, CMP(C_PD));
    }
    return run_col(c, b);
}

// nonlinear term and RK stage update after a solve; t: time at the start of the step
static sbi_status stage_update(sbi_ctx* c, int stage, double dt, int vh_buf, double t) {
    static const double kStageNode[4] = {0.0, 0.5, 0.5, 1.0};
    SBI_TRY(nonlinear_term(c, t + kStageNode[stage] * dt));
    RkParams rp{};
    rp.g = c->gd;
    rp.stage = stage;
    rp.h = dt;
    rp.eh = CMP(C_EH);
    rp.ph = CMP(C_PH);
    rp.es = CMP(C_ES);
    rp.ps = CMP(C_PS);
    rp.Vh = CMP(vh_buf);
    rp.Nph = CMP(C_NP);
    rp.Pdiv = c->dmp_w > 0.0 ? CMP(C_PD) : nullptr;
    rp.ae = CMP(C_AE);
    rp.ap = CMP(C_AP);
    rp.fb1 = c->grid.filter_beta1;
    rp.fb2 = c->grid.filter_beta2;
    c->st.launches += 1;
    {
        ProfScope ps_(c, K_RK);
        return hip_ok(launch_rk(c->fp64, rp, c->batch, c->stream));
    }
}

static sbi_status relax_zone(sbi_ctx* c, double t) {
    ColBuilder b(c->gd);
    int se = b.cin(CMP(C_EH));
    int sp = b.cin(CMP(C_PH));
    b.term(se, 0, 1.0, FN_ONE, 0, DV_NONE);
    b.term(sp, 1, 1.0, FN_ONE, 0, DV_NONE);
    b.inv(SRC_ACC0, DV_NONE, HALF(H_PROD0));
    b.inv(SRC_ACC1, DV_NONE, HALF(H_PROD0 + 1));
    SBI_TRY(run_col(c, b));
    RowBlendParams rp{};
    rp.g = c->gd;
    rp.ge = HALF(H_PROD0);
    rp.gp = HALF(H_PROD0 + 1);
    rp.he = HALF(H_PROD0 + 2);
    rp.hp = HALF(H_PROD0 + 3);
    rp.a = c->rz[0];
    rp.k = c->rz[1];
    rp.om = c->rz[2];
    rp.gen = c->rz[3];
    rp.absl = c->rz[4];
    rp.ramp_time = c->rz[5] * 2.0 * M_PI / c->rz[2];
    rp.t = t;
    c->st.launches += 1;
    {
        ProfScope ps_(c, K_ROW_BLEND);
        SBI_TRY(hip_ok(launch_row_blend(c->fp64, rp, c->batch, tw_of(c), c->stream)));
    }
    ColBuilder b2(c->gd);
    int he = b2.prod(HALF(H_PROD0 + 2));
    int hp = b2.prod(HALF(H_PROD0 + 3));
    b2.term(he, 0, 1.0, FN_ONE, 0, DV_NONE);
    b2.term(hp, 1, 1.0, FN_ONE, 0, DV_NONE);
    b2.cout(SRC_ACC0, CMP(C_EH));
    b2.cout(SRC_ACC0, CMP(C_ES));
    b2.cout(SRC_ACC1, CMP(C_PH));
    b2.cout(SRC_ACC1, CMP(C_PS));
    return run_col(c, b2);
}

static sbi_status to_physical(sbi_ctx* c, void* eta, void* phi) {
    ColBuilder b(c->gd);
    int se = b.cin(CMP(C_EH));
    int sp = b.cin(CMP(C_PH));
    b.term(se, 0, 1.0, FN_ONE, 0, DV_NONE);
    b.term(sp, 1, 1.0, FN_ONE, 0, DV_NONE);
    b.inv(SRC_ACC0, DV_NONE, HALF(H_PROD0));
    b.inv(SRC_ACC1, DV_NONE, HALF(H_PROD0 + 1));
    SBI_TRY(run_col(c, b));
    RowInvParams ip{};
    ip.g = c->gd;
    ip.nf = 2;
    ip.in[0] = HALF(H_PROD0);
    ip.in[1] = HALF(H_PROD0 + 1);
    ip.out[0] = eta;
    ip.out[1] = phi;
    ip.ctl = c->ctl;
    c->st.launches += 1;
    {
        ProfScope ps_(c, K_ROW_INV);
        return hip_ok(launch_row_inv(c->fp64, ip, c->batch, tw_of(c), c->stream));
    }
}

static void acc_info(sbi_ctx* c, sbi_step_info* si) {
    for (int b = 0; b < c->batch; ++b) {
        const Ctl& h = c->head[b];
        si->solves += 1;
        const int sw = c->grid.mode == SBI_MODE_SA ? 0 : h.sweeps;
        si->sweeps_total += sw;
        si->sweeps_max = std::max(si->sweeps_max, sw);
        si->sweeps_fp32_total += c->grid.mode == SBI_MODE_SA ? 0 : h.sweeps_inner;
        si->max_residual = std::max(si->max_residual, c->grid.mode == SBI_MODE_SA ? 0.0 : h.residual);
    }
}

extern "C" sbi_status sbi_step(sbi_ctx* c, sbi_state* state, double dt, int32_t n, double tol, sbi_step_info* info) {
    if (!c || !state || !state->eta || !state->phi_s || n < 0 || !std::isfinite(dt)) return SBI_ERR_INVALID_ARG;
    if (c->grid.mode != SBI_MODE_SA && !(tol >= 0.0)) return SBI_ERR_INVALID_ARG;
    c->st = Stats();
    c->fallbacks = 0;
    sbi_step_info si{};
    SBI_TRY(to_spectral(c, state->eta, state->phi_s, true));
    sbi_status worst = SBI_OK;
    double t = state->t;
    for (int s = 0; s < n; ++s) {
        for (int stage = 0; stage < 4; ++stage) {
            int vh = 0;
            SBI_TRY(solve_stage(c, nullptr, tol, true, &vh, nullptr, false, stage));
            if (c->grid.mode != SBI_MODE_SA) {
                // the iteration already read the control headers at its last poll
                sbi_status st = solve_status(c, nullptr, true);
                if (st < 0) return st;
                if (st > worst) worst = st;
                acc_info(c, &si);
            } else {
                si.solves += c->batch;
            }
            SBI_TRY(stage_update(c, stage, dt, vh, t));
        }
        t += dt;
        if (c->relax_on) SBI_TRY(relax_zone(c, t));
    }
    if (c->grid.mode == SBI_MODE_SA) {
        // SA mode has no residual; non-finite values surface through the last setup
        SBI_TRY(read_heads(c));
        for (int b = 0; b < c->batch; ++b)
            if (c->head[b].nonfinite) return SBI_ERR_NONFINITE;
    }
    SBI_TRY(to_physical(c, state->eta, state->phi_s));
    SBI_HIP(hipStreamSynchronize(c->stream));
    state->t = t;
    si.fallbacks = c->fallbacks;
    if (info) *info = si;
    if (worst == SBI_OK && c->fallbacks > 0) worst = SBI_WARN_FALLBACK_USED;
    return worst;
}

// stage `stage` of the embedded pair after its solve (t: time at the start of
// the step); the last stage leaves the fifth-order candidate in (C_ES, C_PS)
// and returns the largest relative difference of the two solutions over the
// members in *err
static sbi_status pair_stage(sbi_ctx* c, int stage, double h, int vh_buf, double t, double* err) {
    // nodes of the Cash-Karp pair (the stage kernel holds the whole table)
    static const double kPairNode[6] = {0.0, 1.0 / 5.0, 3.0 / 10.0, 3.0 / 5.0, 1.0, 7.0 / 8.0};
    SBI_TRY(nonlinear_term(c, t + kPairNode[stage] * h));
    Rk54Params rp{};
    rp.g = c->gd;
    rp.stage = stage;
    rp.h = h;
    rp.eh = CMP(C_EH);
    rp.ph = CMP(C_PH);
    rp.es = CMP(C_ES);
    rp.ps = CMP(C_PS);
    rp.Vh = CMP(vh_buf);
    rp.Nph = CMP(C_NP);
    rp.Pdiv = c->dmp_w > 0.0 ? CMP(C_PD) : nullptr;
    for (int j = 0; j < 6; ++j) {
        rp.ke[j] = CMP(C_KE0 + j);
        rp.kp[j] = CMP(C_KP0 + j);
    }
    rp.fb1 = c->grid.filter_beta1;
    rp.fb2 = c->grid.filter_beta2;
    rp.partial = c->diag_partial;
    rp.nblk = c->diag_nblk;
    c->st.launches += 1;
    {
        ProfScope ps_(c, K_RK);
        SBI_TRY(hip_ok(launch_rk54(c->fp64, rp, c->batch, c->stream)));
    }
    if (stage < 5) return SBI_OK;
    std::vector<double> part((size_t)c->batch * rp.nblk * 2);
    SBI_HIP(hipMemcpyAsync(part.data(), c->diag_partial, part.size() * sizeof(double), hipMemcpyDeviceToHost,
                           c->stream));
    SBI_HIP(hipStreamSynchronize(c->stream));
    c->st.syncs += 1;
    double e = 0.0;
    for (int b = 0; b < c->batch; ++b) {
        double num = 0.0, den = 0.0;
        for (int k = 0; k < rp.nblk; ++k) {
            num += part[((size_t)b * rp.nblk + k) * 2];
            den += part[((size_t)b * rp.nblk + k) * 2 + 1];
        }
        // both solutions vanish: nothing to control; a vanishing candidate alone: reject
        const double eb = num == 0.0 ? 0.0 : den > 0.0 ? std::sqrt(num / den) : HUGE_VAL;
        e = std::isnan(eb) || std::isnan(e) ? NAN : std::max(e, eb);
    }
    *err = e;
    return SBI_OK;
}

static sbi_status copy_state(sbi_ctx* c, int de, int dp, int se, int sp) {
    const size_t bytes = (size_t)c->gd.s_cmp * c->csz * c->batch;
    SBI_HIP(hipMemcpyAsync(CMP(de), CMP(se), bytes, hipMemcpyDeviceToDevice, c->stream));
    SBI_HIP(hipMemcpyAsync(CMP(dp), CMP(sp), bytes, hipMemcpyDeviceToDevice, c->stream));
    return SBI_OK;
}

extern "C" sbi_status sbi_step_adaptive(sbi_ctx* c, sbi_state* state, double t_end, double dt, double rk_tol,
                                        double tol, int32_t max_steps, sbi_adapt_info* info) {
    if (!c || !state || !state->eta || !state->phi_s || max_steps < 1) return SBI_ERR_INVALID_ARG;
    if (!std::isfinite(state->t) || !std::isfinite(t_end) || !(t_end >= state->t)) return SBI_ERR_INVALID_ARG;
    if (!(dt > 0.0) || !std::isfinite(dt) || !(rk_tol > 0.0) || !std::isfinite(rk_tol)) return SBI_ERR_INVALID_ARG;
    if (c->grid.mode != SBI_MODE_SA && !(tol >= 0.0)) return SBI_ERR_INVALID_ARG;
    // step-size controller: growth limits and safety factor of the usual
    // embedded-pair control, exponent 1/5 (the local error of the fourth-order
    // solution is O(h^5))
    const double kSafety = 0.9, kFacMin = 0.2, kFacMax = 5.0;
    c->st = Stats();
    c->fallbacks = 0;
    sbi_adapt_info ai{};
    SBI_TRY(to_spectral(c, state->eta, state->phi_s, true));
    sbi_status worst = SBI_OK;
    const double t0 = state->t;
    double t = t0, h = dt;
    bool last_rejected = false;
    while (t < t_end) {
        if (ai.accepted + ai.rejected >= max_steps) {
            worst = std::max(worst, SBI_WARN_STEP_LIMIT);
            break;
        }
        // a step whose trial size reaches t_end (within a relative 1e-9) lands on it
        const bool final = t_end - t <= h * (1.0 + 1e-9);
        const double hs = final ? t_end - t : h;
        double err = 0.0;
        for (int stage = 0; stage < 6; ++stage) {
            int vh = 0;
            SBI_TRY(solve_stage(c, nullptr, tol, true, &vh));
            if (c->grid.mode != SBI_MODE_SA) {
                sbi_status st = solve_status(c, nullptr, true);
                if (st < 0) return st;
                if (st > worst) worst = st;
                acc_info(c, &ai.solve);
            } else {
                ai.solve.solves += c->batch;
            }
            SBI_TRY(pair_stage(c, stage, hs, vh, t, &err));
        }
        const double fmax = last_rejected ? 1.0 : kFacMax;
        double fac;
        if (!std::isfinite(err)) fac = kFacMin;
        else if (err == 0.0) fac = fmax;
        else fac = std::min(fmax, std::max(kFacMin, kSafety * std::pow(rk_tol / err, 0.2)));
        ai.err_last = err;
        if (err <= rk_tol) {
            SBI_TRY(copy_state(c, C_EH, C_PH, C_ES, C_PS));
            t = final ? t_end : t + hs;
            ai.accepted += 1;
            ai.err_max = std::max(ai.err_max, err);
            last_rejected = false;
            if (c->relax_on) SBI_TRY(relax_zone(c, t));
            h = final ? std::max(hs * fac, h) : hs * fac;
        } else {
            SBI_TRY(copy_state(c, C_ES, C_PS, C_EH, C_PH));
            ai.rejected += 1;
            last_rejected = true;
            h = hs * fac;
            if (h < 1e-12 * std::max(t_end - t0, std::fabs(t))) return SBI_ERR_DIVERGED;
        }
    }
    if (c->grid.mode == SBI_MODE_SA) {
        SBI_TRY(read_heads(c));
        for (int b = 0; b < c->batch; ++b)
            if (c->head[b].nonfinite) return SBI_ERR_NONFINITE;
    }
    SBI_TRY(to_physical(c, state->eta, state->phi_s));
    SBI_HIP(hipStreamSynchronize(c->stream));
    state->t = t;
    ai.dt_next = h;
    ai.solve.fallbacks = c->fallbacks;
    if (info) *info = ai;
    if (worst == SBI_OK && c->fallbacks > 0) worst = SBI_WARN_FALLBACK_USED;
    return worst;
}

extern "C" sbi_status sbi_diagnostics(sbi_ctx* c, const sbi_state* state, double tol, double* mass, double* energy) {
    if (!c || !state || !state->eta || !state->phi_s || !mass || !energy) return SBI_ERR_INVALID_ARG;
    c->st = Stats();
    SBI_TRY(to_spectral(c, state->eta, state->phi_s, false));
    int vh = 0;
    SBI_TRY(solve_stage(c, nullptr, tol, false, &vh));
    sbi_status st = solve_status(c, nullptr, c->grid.mode != SBI_MODE_SA);
    if (st < 0) return st;
    DiagParams dp{};
    dp.g = c->gd;
    dp.eh = CMP(C_ES);
    dp.ph = CMP(C_PS);
    dp.Vh = CMP(vh);
    dp.partial = c->diag_partial;
    dp.nblk = c->diag_nblk;
    {
        ProfScope ps_(c, K_DIAG);
        SBI_TRY(hip_ok(launch_diag(c->fp64, dp, c->batch, c->stream)));
    }
    std::vector<double> part((size_t)c->batch * dp.nblk * 2);
    SBI_HIP(hipMemcpyAsync(part.data(), c->diag_partial, part.size() * sizeof(double), hipMemcpyDeviceToHost,
                           c->stream));
    SBI_HIP(hipStreamSynchronize(c->stream));
    const sbi_grid& g = c->grid;
    const double dA = (g.lx / g.nx) * (g.ny > 1 ? g.ly / g.ny : 1.0);
    const double ntot = (double)g.nx * g.ny;
    for (int b = 0; b < c->batch; ++b) {
        double se = 0.0, sm = 0.0;
        for (int k = 0; k < dp.nblk; ++k) {
            se += part[((size_t)b * dp.nblk + k) * 2];
            sm += part[((size_t)b * dp.nblk + k) * 2 + 1];
        }
        // Parseval on the kept half spectrum: sum_i f_i g_i = (1/N) sum_m w_m Re(F_m conj G_m)
        energy[b] = 0.5 * dA * se / ntot;
        mass[b] = dA * sm;
    }
    return st;
}

extern "C" sbi_status sbi_profile_enable(sbi_ctx* c, int32_t enable) {
    if (!c || (enable != SBI_PROFILE_OFF && enable != SBI_PROFILE_ALL && enable != SBI_PROFILE_SWEEPS))
        return SBI_ERR_INVALID_ARG;
    SBI_HIP(hipStreamSynchronize(c->stream));
    prof_flush(c);
    c->prof.on = enable != SBI_PROFILE_OFF;
    c->prof.mask = enable == SBI_PROFILE_SWEEPS ? ((1u << K_ROW_SWEEP) | (1u << K_COL_SWEEP)) : ~0u;
    for (int k = 0; k < K_COUNT; ++k) {
        c->prof.total_ms[k] = 0.0;
        c->prof.count[k] = 0;
    }
    if (c->inner) return sbi_profile_enable(c->inner, enable);
    return SBI_OK;
}

extern "C" int32_t sbi_profile_read(sbi_ctx* c, const char** names, double* total_ms, int64_t* launches, int32_t n) {
    if (!c) return 0;
    if (hipStreamSynchronize(c->stream) != hipSuccess) return 0;
    prof_flush(c);
    double tot[K_COUNT];
    long long cnt[K_COUNT];
    for (int i = 0; i < K_COUNT; ++i) {
        tot[i] = c->prof.total_ms[i];
        cnt[i] = c->prof.count[i];
    }
    if (c->inner) {
        // the FP32 correction sweeps under their own names, the rest of the
        // FP32 context's kernels with their classes
        sbi_ctx* in = c->inner;
        prof_flush(in);
        for (int i = 0; i < K_COUNT; ++i) {
            const int j = i == K_ROW_SWEEP ? K_ROW_SWEEP32 : (i == K_COL_SWEEP ? K_COL_SWEEP32 : i);
            tot[j] += in->prof.total_ms[i];
            cnt[j] += in->prof.count[i];
        }
    }
    const int k = std::min<int>(n, K_COUNT);
    for (int i = 0; i < k; ++i) {
        if (names) names[i] = kKernelNames[i];
        if (total_ms) total_ms[i] = tot[i];
        if (launches) launches[i] = cnt[i];
    }
    return k;
}

// ---------------------------------------------------------------------------
// learned warm start
// ---------------------------------------------------------------------------
static uint16_t host_bf16(float f) {  // round to nearest even (finite values)
    uint32_t u;
    std::memcpy(&u, &f, 4);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

extern "C" sbi_status sbi_net_load(sbi_ctx* c, const void* weights, size_t bytes) {
    if (!c || !weights || bytes != sbi_net_blob_bytes()) return SBI_ERR_INVALID_ARG;
    sbi_net_header h;
    std::memcpy(&h, weights, sizeof(h));
    if (std::memcmp(h.magic, "SBIW", 4) != 0 || h.version != 1 || h.cin != kNetCin || h.width != kNetWidth ||
        h.nparams != kNetParams)
        return SBI_ERR_INVALID_ARG;
    for (float v : h.out_scale)
        if (!std::isfinite(v)) return SBI_ERR_INVALID_ARG;
    std::vector<float> th(kNetParams);
    std::memcpy(th.data(), static_cast<const char*>(weights) + sizeof(h), sizeof(float) * kNetParams);
    for (float v : th)
        if (!std::isfinite(v)) return SBI_ERR_INVALID_ARG;
    for (float v : h.in_scale)
        if (!std::isfinite(v)) return SBI_ERR_INVALID_ARG;
    auto pk = std::make_unique<NetPacked>();
    std::memset(pk.get(), 0, sizeof(NetPacked));
    for (int o = 0; o < 32; ++o) {
        for (int k = 0; k < 9 * 8; ++k) pk->w1[o * kL1S + k] = host_bf16(th[kOffW1 + o * 72 + k]);
        for (int k = 0; k < 9 * 32; ++k) pk->w2[o * kL2S + k] = host_bf16(th[kOffW2 + o * 288 + k]);
        for (int k = 0; k < 32; ++k) pk->w3[o * kL3S + k] = host_bf16(th[kOffW3 + o * 32 + k]);
        pk->w4[o] = host_bf16(th[kOffW4 + o]);
        pk->w4[32 + o] = host_bf16(th[kOffW4 + 32 + o]);
        pk->b1[o] = th[kOffB1 + o];
        pk->b2[o] = th[kOffB2 + o];
        pk->b3[o] = th[kOffB3 + o];
    }
    for (int k = 0; k < 2; ++k) {
        pk->b4[k] = th[kOffB4 + k];
        pk->out_scale[k] = h.out_scale[k];
    }
    for (int i = 0; i < 8; ++i) pk->in_scale[i] = h.in_scale[i];
    SBI_HIP(hipMemcpyAsync(c->net, pk.get(), sizeof(NetPacked), hipMemcpyHostToDevice, c->stream));
    SBI_HIP(hipStreamSynchronize(c->stream));
    for (int i = 0; i < 8; ++i) c->net_scale[i] = h.in_scale[i];
    c->net_loaded = true;
    return SBI_OK;
}

extern "C" int32_t sbi_net_hist_param_count(int32_t taps, int32_t bins) {
    if (taps < 1 || taps > kHistTaps || bins < 1 || bins > kHistBins) return 0;
    return 2 * kHistStages * bins * taps * 2;
}

extern "C" sbi_status sbi_net_hist_load(sbi_ctx* c, int32_t taps, int32_t bins, double dk, const float* w) {
    if (!c || !w || sbi_net_hist_param_count(taps, bins) == 0 || !(dk > 0.0) || !std::isfinite(dk))
        return SBI_ERR_INVALID_ARG;
    if (c->grid.seed != SBI_SEED_NET || !c->hist_dev) return SBI_ERR_INVALID_ARG;
    const int n = sbi_net_hist_param_count(taps, bins);
    for (int i = 0; i < n; ++i)
        if (!std::isfinite(w[i])) return SBI_ERR_INVALID_ARG;
    // weights, cleared moments and accumulators
    SBI_HIP(hipStreamSynchronize(c->stream));
    auto hd = std::make_unique<HistDev>();
    std::memset(hd.get(), 0, sizeof(HistDev));
    std::memcpy(hd->w, w, sizeof(float) * n);
    SBI_HIP(hipMemcpyAsync(c->hist_dev, hd.get(), sizeof(HistDev), hipMemcpyHostToDevice, c->stream));
    SBI_HIP(hipStreamSynchronize(c->stream));
    c->hist_K = taps;
    c->hist_nb = bins;
    c->hist_dk = dk;
    c->hist_loaded = true;
    c->hist_count = 0;
    return SBI_OK;
}

extern "C" sbi_status sbi_net_hist_train(sbi_ctx* c, int32_t enable) {
    if (!c || !c->hist_loaded) return SBI_ERR_INVALID_ARG;
    c->hist_train = enable != 0;
    return SBI_OK;
}

extern "C" sbi_status sbi_net_hist_gradient(sbi_ctx* c, double* loss_sum, int32_t* samples, double* grad_sum,
                                            double* gram_sum) {
    if (!c || !c->hist_loaded) return SBI_ERR_INVALID_ARG;
    auto hd = std::make_unique<HistDev>();
    SBI_HIP(hipMemcpyAsync(hd.get(), c->hist_dev, sizeof(HistDev), hipMemcpyDeviceToHost, c->stream));
    SBI_HIP(hipStreamSynchronize(c->stream));
    if (loss_sum) *loss_sum = hd->loss;
    if (samples) *samples = (int32_t)hd->samples;
    if (grad_sum) {
        const int n = sbi_net_hist_param_count(c->hist_K, c->hist_nb);
        for (int i = 0; i < n; ++i) grad_sum[i] = hd->acc[i];
    }
    if (gram_sum) {
        const int n = 2 * kHistStages * c->hist_nb * c->hist_K * c->hist_K * 2;
        for (int i = 0; i < n; ++i) gram_sum[i] = hd->gram[i];
    }
    return SBI_OK;
}

extern "C" sbi_status sbi_net_hist_newton(sbi_ctx* c, double lam, double* loss_mean, int32_t* samples) {
    if (!c || !c->hist_loaded || !(lam >= 0.0) || !std::isfinite(lam)) return SBI_ERR_INVALID_ARG;
    const HistParams hp = hist_params(c, 0);
    SBI_TRY(hip_ok(launch_hist_newton(hp, lam, c->stream)));
    double out[2] = {0.0, 0.0};
    SBI_HIP(hipMemcpyAsync(out, c->hist_dev->out, sizeof(out), hipMemcpyDeviceToHost, c->stream));
    SBI_HIP(hipStreamSynchronize(c->stream));
    if (loss_mean) *loss_mean = out[0];
    if (samples) *samples = (int32_t)out[1];
    return SBI_OK;
}

extern "C" sbi_status sbi_net_hist_adam(sbi_ctx* c, float lr, double* loss_mean, int32_t* samples) {
    if (!c || !c->hist_loaded || !(lr >= 0.0f) || !std::isfinite(lr)) return SBI_ERR_INVALID_ARG;
    HistParams hp = hist_params(c, 0);
    hp.lr = lr;
    SBI_TRY(hip_ok(launch_hist_adam(hp, c->stream)));
    double out[2] = {0.0, 0.0};
    SBI_HIP(hipMemcpyAsync(out, c->hist_dev->out, sizeof(out), hipMemcpyDeviceToHost, c->stream));
    SBI_HIP(hipStreamSynchronize(c->stream));
    if (loss_mean) *loss_mean = out[0];
    if (samples) *samples = (int32_t)out[1];
    return SBI_OK;
}

extern "C" sbi_status sbi_net_hist_params(sbi_ctx* c, float* w_out) {
    if (!c || !c->hist_loaded || !w_out) return SBI_ERR_INVALID_ARG;
    const int n = sbi_net_hist_param_count(c->hist_K, c->hist_nb);
    SBI_HIP(hipMemcpyAsync(w_out, c->hist_dev->w, sizeof(float) * n, hipMemcpyDeviceToHost, c->stream));
    SBI_HIP(hipStreamSynchronize(c->stream));
    return SBI_OK;
}

extern "C" sbi_status sbi_net_features(sbi_ctx* c, const void* eta, const void* phi_s, float* feat_out,
                                       void* wlin_out) {
    if (!c || !eta || !phi_s || !feat_out) return SBI_ERR_INVALID_ARG;
    if (c->grid.ny == 1) return SBI_ERR_UNSUPPORTED;
    c->st = Stats();
    SBI_TRY(to_spectral(c, eta, phi_s, false));
    SBI_TRY(stage_state_pass(c, true, false));
    SBI_TRY(row_features(c, eta, feat_out, wlin_out));
    SBI_HIP(hipStreamSynchronize(c->stream));
    return SBI_OK;
}

extern "C" sbi_status sbi_net_infer(sbi_ctx* c, const float* feat, const void* wlin, void* seed_out,
                                    void* dphib_out) {
    if (!c || !feat || !wlin || !seed_out || !dphib_out) return SBI_ERR_INVALID_ARG;
    if (c->grid.ny == 1) return SBI_ERR_UNSUPPORTED;
    if (!c->net_loaded) return SBI_ERR_INVALID_ARG;
    SBI_TRY(net_infer(c, feat, wlin, seed_out, dphib_out));
    SBI_HIP(hipStreamSynchronize(c->stream));
    return SBI_OK;
}

extern "C" sbi_status sbi_last_correction(sbi_ctx* c, void* dv_out, void* dphib_out) {
    if (!c || !dv_out || !dphib_out) return SBI_ERR_INVALID_ARG;
    if ((c->grid.seed != SBI_SEED_PREV && c->grid.seed != SBI_SEED_NET) || c->grid.mode != SBI_MODE_ITER ||
        !c->have_prev)
        return SBI_ERR_INVALID_ARG;
    c->st = Stats();
    ColBuilder b(c->gd);
    b.term(b.cin(CMP(C_DV)), 0, 1.0, FN_ONE, 0, DV_NONE);
    b.inv(SRC_ACC0, DV_NONE, HALF(H_PROD0));
    if (c->vd) {
        b.term(b.cin(CMP(C_DB)), 1, 1.0, FN_ONE, 0, DV_NONE);
        b.inv(SRC_ACC1, DV_NONE, HALF(H_PROD0 + 1));
    }
    SBI_TRY(run_col(c, b));
    RowInvParams ip{};
    ip.g = c->gd;
    ip.nf = c->vd ? 2 : 1;
    ip.in[0] = HALF(H_PROD0);
    ip.out[0] = dv_out;
    ip.in[1] = HALF(H_PROD0 + 1);
    ip.out[1] = dphib_out;
    ip.ctl = c->ctl;
    c->st.launches += 1;
    SBI_TRY(hip_ok(launch_row_inv(c->fp64, ip, c->batch, tw_of(c), c->stream)));
    if (!c->vd) SBI_TRY(hip_ok(launch_fill_zero(dphib_out, (size_t)c->gd.s_phys * c->rsz * c->batch, c->stream)));
    SBI_HIP(hipStreamSynchronize(c->stream));
    return SBI_OK;
}

// ---------------------------------------------------------------------------
// ensembles of uneven grids (sbi_batch.h)
// ---------------------------------------------------------------------------
namespace {

bool same_grid(const sbi_grid& a, const sbi_grid& b) {
    return a.nx == b.nx && a.ny == b.ny && a.lx == b.lx && (a.ny == 1 || a.ly == b.ly) && a.order == b.order &&
           a.dealias == b.dealias && a.precision == b.precision && a.mode == b.mode && a.seed == b.seed &&
           a.max_sweeps == b.max_sweeps && a.relax == b.relax && a.filter_beta1 == b.filter_beta1 &&
           a.filter_beta2 == b.filter_beta2;
}

// members grouped by identical grids, in order of first appearance
std::vector<std::vector<int>> group_members(int m, const sbi_grid* grids) {
    std::vector<std::vector<int>> out;
    for (int i = 0; i < m; ++i) {
        bool placed = false;
        for (auto& g : out)
            if (same_grid(grids[g[0]], grids[i])) {
                g.push_back(i);
                placed = true;
                break;
            }
        if (!placed) out.push_back({i});
    }
    return out;
}

size_t al256(size_t b) { return (b + 255) / 256 * 256; }

// compact buffers a context carries from one call to the next: the
// previous-solve parts (C_DV, C_DB) and the learned history (C_HV0 .. C_HB0 +
// kHistTaps - 1), two contiguous runs of the workspace
constexpr int kCarriedCmp = 2 + 2 * kHistTaps;
constexpr int kBudgetMargin = 3;  // sweeps beyond the largest count seen, in a speculative budget

size_t staging_bytes(const sbi_grid& g, int count) {
    const size_t rsz = g.precision == SBI_FP64 ? 8 : 4;
    const Layout L = layout(&g, count);
    // staging of the members' states, a backup of them and of the carried
    // compact buffers (for the redo of a step whose sweep budget ran out)
    return 4 * al256((size_t)g.nx * g.ny * rsz * count) +
           (size_t)kCarriedCmp * al256((size_t)L.s_cmp * L.csz * count);
}

}  // namespace

struct sbi_batch {
    struct Group {
        sbi_ctx* c = nullptr;
        std::vector<int> members;
        hipStream_t s = nullptr;
        hipEvent_t done = nullptr;
        char* st_eta = nullptr;  // contiguous [count][ny][nx] staging of the members' states
        char* st_phi = nullptr;
        size_t field_bytes = 0;  // one member's field
        char* bk_state = nullptr;  // backup of the members' (eta, phi) at the start of a step call
        char* bk_cmp = nullptr;    // backup of the carried compact buffers
        size_t cmp_bytes = 0;      // one compact buffer of the group (all members)
        bool bk_have_prev = false;
        int bk_hist_count = 0;
    };
    int m = 0;
    int flags = 0;
    hipStream_t stream = nullptr;  // caller's stream
    hipStream_t cap = nullptr;     // the batch's own stream: work is forked from and joined to it
    hipEvent_t fork = nullptr;
    hipEvent_t in = nullptr, out = nullptr;  // caller's stream -> cap -> caller's stream
    std::vector<Group> g;
    // instantiated graphs of the parts of a step call, with what each was
    // captured for; least recently used first out
    struct Graph {
        hipGraphExec_t exec = nullptr;
        int part = 0, n = 0;
        double dt = 0.0, tol = 0.0;
        std::vector<const void*> ptrs;
        std::vector<int> prev, budget;
        unsigned long long used = 0;
    };
    std::vector<Graph> graphs;
    unsigned long long clock = 0;
    int redos = 0;  // step calls redone with a larger sweep budget (since init)
};

static void batch_free(sbi_batch* b) {
    if (!b) return;
    for (auto& gg : b->graphs)
        if (gg.exec) (void)hipGraphExecDestroy(gg.exec);
    for (auto& gr : b->g) {
        if (gr.c) sbi_destroy(gr.c);
        if (gr.done) (void)hipEventDestroy(gr.done);
        if (gr.s) (void)hipStreamDestroy(gr.s);
    }
    if (b->fork) (void)hipEventDestroy(b->fork);
    if (b->in) (void)hipEventDestroy(b->in);
    if (b->out) (void)hipEventDestroy(b->out);
    if (b->cap) (void)hipStreamDestroy(b->cap);
    delete b;
}

extern "C" size_t sbi_batch_workspace_bytes(int32_t m, const sbi_grid* grids) {
    if (m < 1 || !grids) return 0;
    for (int i = 0; i < m; ++i)
        if (!grid_valid(&grids[i])) return 0;
    size_t total = 0;
    for (auto& gm : group_members(m, grids)) {
        const sbi_grid& g = grids[gm[0]];
        total += al256(layout(&g, (int)gm.size()).total) + staging_bytes(g, (int)gm.size());
    }
    return total;
}

// ---------------------------------------------------------------------------
// Launch plans and the autotuner
// ---------------------------------------------------------------------------
static int plan_variants(const sbi_ctx* c) {
    return row_var_mask(c->fp64, c->grid.mode == SBI_MODE_ITER ? 1 : 0, c->grid.nx);
}

static bool pow2(int v) { return v > 0 && (v & (v - 1)) == 0; }

static sbi_status plan_apply(sbi_ctx* c, const sbi_plan& p) {
    if (p.row_variant < 0 || p.row_variant > 3 || !((plan_variants(c) >> p.row_variant) & 1))
        return SBI_ERR_UNSUPPORTED;
    if (p.row_rows < 0 || (p.row_rows > 0 && !pow2(p.row_rows)) || p.col_split < 0) return SBI_ERR_INVALID_ARG;
    c->gd.row_var = p.row_variant;
    c->gd.row_rpw = p.row_rows;
    c->group_target = p.col_split;
    return SBI_OK;
}

// one unit of the context's work under the current plan: a sweep of the
// iteration (products, column pass, mixing), or a whole SA solve
static sbi_status tune_unit(sbi_ctx* c) {
    if (c->grid.mode == SBI_MODE_SA) return run_sa(c, PHYS(P_ETA));
    // sweep index 0: no residual test, so no launch is ever skipped
    return launch_sweep(c, PHYS(P_ETA), 0, 1e-30);
}

// microseconds per unit: 2 units of warm-up, then the better of two rounds
// of 5 timed with events on the context's stream
static sbi_status tune_time(sbi_ctx* c, hipEvent_t e0, hipEvent_t e1, float* us) {
    constexpr int kWarm = 2, kRounds = 2, kReps = 5;
    SBI_TRY(hip_ok(launch_ctl_reset(c->ctl, c->batch, c->grid.max_sweeps + 2, c->stream)));
    for (int r = 0; r < kWarm; ++r) SBI_TRY(tune_unit(c));
    float best = 1e30f;
    for (int round = 0; round < kRounds; ++round) {
        SBI_HIP(hipEventRecord(e0, c->stream));
        for (int r = 0; r < kReps; ++r) SBI_TRY(tune_unit(c));
        SBI_HIP(hipEventRecord(e1, c->stream));
        SBI_HIP(hipEventSynchronize(e1));
        float ms = 0.f;
        SBI_HIP(hipEventElapsedTime(&ms, e0, e1));
        best = std::min(best, 1e3f * ms / kReps);
    }
    *us = best;
    return SBI_OK;
}

struct TuneCache {
    std::mutex mu;
    std::map<std::string, sbi_plan> plans;
};
static TuneCache& tune_cache() {
    static TuneCache tc;
    return tc;
}

// device name and architecture, grid, batch, precision, mode, acceleration,
// order and variable bed: everything the fastest plan can depend on
static sbi_status tune_key(const sbi_ctx* c, std::string* key) {
    int dev = 0;
    SBI_HIP(hipStreamGetDevice(c->stream, &dev));
    hipDeviceProp_t prop;
    SBI_HIP(hipGetDeviceProperties(&prop, dev));
    std::string d = std::string(prop.name) + "/" + prop.gcnArchName;
    for (char& ch : d)
        if (ch == ' ' || ch == '\t' || ch == '|') ch = '_';
    char buf[256];
    std::snprintf(buf, sizeof buf, "|%dx%d|b%d|%s|%s|a%d|o%d|vd%d", c->grid.nx, c->grid.ny, c->batch,
                  c->fp64 ? "fp64" : "fp32", c->grid.mode == SBI_MODE_SA ? "sa" : "iter", (int)c->grid.accel,
                  c->grid.order, c->vd ? 1 : 0);
    *key = d + buf;
    return SBI_OK;
}

// the plans the tuner tries: every built row variant, rows per workgroup from
// the launch bound down to a quarter of it, column splits of 2D grids
static std::vector<sbi_plan> plan_candidates(const sbi_ctx* c) {
    std::vector<sbi_plan> out;
    const int mask = plan_variants(c);
    std::vector<int> splits = {0};
    if (c->grid.ny > 1) splits = {0, 1024, 2048, 4096};
    for (int v = 0; v < 4; ++v) {
        if (!((mask >> v) & 1)) continue;
        const int cap = std::min(row_rows_cap(c->fp64, c->grid.nx, v), c->grid.ny);
        for (int rows = cap; rows >= 1 && rows * 4 >= cap; rows /= 2)
            for (int sp : splits) out.push_back(sbi_plan{v, rows, sp, 0.f, 0});
    }
    return out;
}

static sbi_status autotune(sbi_ctx* c, int32_t flags, sbi_plan* out) {
    if (c->grid.mode == SBI_MODE_FULL) {
        // its pair kernels have no launch-plan choices: the default plan stays
        if (out) *out = sbi_plan{c->gd.row_var, c->gd.row_rpw, c->group_target, 0.f, 0};
        return SBI_OK;
    }
    // mixed precision: the FP32 correction sweeps have plans of their own
    if (c->inner) SBI_TRY(autotune(c->inner, flags, nullptr));
    std::string key;
    SBI_TRY(tune_key(c, &key));
    if (!(flags & SBI_TUNE_FORCE)) {
        TuneCache& tc = tune_cache();
        std::lock_guard<std::mutex> lk(tc.mu);
        auto it = tc.plans.find(key);
        if (it != tc.plans.end() && plan_apply(c, it->second) == SBI_OK) {
            if (out) {
                *out = it->second;
                out->cached = 1;
            }
            return SBI_OK;
        }
    }
    hipEvent_t e0, e1;
    SBI_HIP(hipEventCreate(&e0));
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return SBI_ERR_HIP;
    }
    const sbi_plan before = {c->gd.row_var, c->gd.row_rpw, c->group_target, 0.f, 0};
    sbi_plan best = before;
    best.us = 1e30f;
    sbi_status st = SBI_OK;
    for (const sbi_plan& cand : plan_candidates(c)) {
        st = plan_apply(c, cand);
        float us = 0.f;
        if (st == SBI_OK) st = tune_time(c, e0, e1, &us);
        if (st != SBI_OK) break;
        if (us < best.us) {
            best = cand;
            best.us = us;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    // the tuning ran the kernels on the workspace: nothing carried is valid
    c->have_prev = false;
    c->hist_count = 0;
    if (st != SBI_OK) {
        (void)plan_apply(c, before);
        return st;
    }
    SBI_TRY(plan_apply(c, best));
    {
        TuneCache& tc = tune_cache();
        std::lock_guard<std::mutex> lk(tc.mu);
        tc.plans[key] = best;
    }
    if (out) *out = best;
    return hip_ok(launch_ctl_reset(c->ctl, c->batch, c->grid.max_sweeps + 2, c->stream));
}

extern "C" int32_t sbi_plan_variants(const sbi_ctx* c) { return c ? plan_variants(c) : 0; }

extern "C" sbi_status sbi_plan_get(const sbi_ctx* c, sbi_plan* out) {
    if (!c || !out) return SBI_ERR_INVALID_ARG;
    *out = sbi_plan{c->gd.row_var, c->gd.row_rpw, c->group_target, 0.f, 0};
    return SBI_OK;
}

extern "C" sbi_status sbi_plan_set(sbi_ctx* c, const sbi_plan* plan) {
    if (!c || !plan) return SBI_ERR_INVALID_ARG;
    return plan_apply(c, *plan);
}

extern "C" sbi_status sbi_autotune(sbi_ctx* c, int32_t flags, sbi_plan* out) {
    if (!c) return SBI_ERR_INVALID_ARG;
    return autotune(c, flags, out);
}

extern "C" sbi_status sbi_tune_cache_load(const char* path, int32_t* count) {
    if (count) *count = 0;
    if (!path) return SBI_ERR_INVALID_ARG;
    FILE* f = std::fopen(path, "r");
    if (!f) return SBI_ERR_INVALID_ARG;
    std::map<std::string, sbi_plan> got;
    char line[1024];
    while (std::fgets(line, sizeof line, f)) {
        if (line[0] == '#') continue;
        char key[512];
        sbi_plan p{};
        if (std::sscanf(line, "%511s %d %d %d %f", key, &p.row_variant, &p.row_rows, &p.col_split, &p.us) != 5)
            continue;
        if (p.row_variant < 0 || p.row_variant > 3 || p.row_rows < 0 || p.col_split < 0) continue;
        got[key] = p;
    }
    std::fclose(f);
    TuneCache& tc = tune_cache();
    std::lock_guard<std::mutex> lk(tc.mu);
    for (auto& kv : got) tc.plans[kv.first] = kv.second;
    if (count) *count = (int32_t)got.size();
    return SBI_OK;
}

extern "C" sbi_status sbi_tune_cache_save(const char* path, int32_t* count) {
    if (count) *count = 0;
    if (!path) return SBI_ERR_INVALID_ARG;
    TuneCache& tc = tune_cache();
    std::lock_guard<std::mutex> lk(tc.mu);
    FILE* f = std::fopen(path, "w");
    if (!f) return SBI_ERR_INVALID_ARG;
    bool ok = std::fprintf(f, "# sbi launch plans: key row_variant row_rows col_split us\n") > 0;
    for (auto& kv : tc.plans)
        ok = ok && std::fprintf(f, "%s %d %d %d %.3f\n", kv.first.c_str(), kv.second.row_variant,
                                kv.second.row_rows, kv.second.col_split, kv.second.us) > 0;
    ok = (std::fclose(f) == 0) && ok;
    if (!ok) return SBI_ERR_INVALID_ARG;
    if (count) *count = (int32_t)tc.plans.size();
    return SBI_OK;
}

// Plans of an ensemble: its groups run concurrently, so a group's plan is
// timed with every group running (one unit of each on its own stream, forked
// from and joined to the batch's stream), group by group (coordinate
// descent from the default plans).  A single group is the context's own
// tuning.  The plan cache keys an ensemble's plans by all its groups' keys.
static sbi_status ensemble_time(sbi_batch* b, hipEvent_t e0, hipEvent_t e1, float* us) {
    constexpr int kRounds = 2, kReps = 3;
    auto unit = [&]() -> sbi_status {
        SBI_HIP(hipEventRecord(b->fork, b->cap));
        for (auto& gr : b->g) {
            SBI_HIP(hipStreamWaitEvent(gr.s, b->fork, 0));
            SBI_TRY(hip_ok(launch_ctl_reset(gr.c->ctl, gr.c->batch, gr.c->grid.max_sweeps + 2, gr.s)));
            SBI_TRY(tune_unit(gr.c));
            SBI_HIP(hipEventRecord(gr.done, gr.s));
            SBI_HIP(hipStreamWaitEvent(b->cap, gr.done, 0));
        }
        return SBI_OK;
    };
    SBI_TRY(unit());  // warm-up
    float best = 1e30f;
    for (int r = 0; r < kRounds; ++r) {
        SBI_HIP(hipEventRecord(e0, b->cap));
        for (int k = 0; k < kReps; ++k) SBI_TRY(unit());
        SBI_HIP(hipEventRecord(e1, b->cap));
        SBI_HIP(hipEventSynchronize(e1));
        float ms = 0.f;
        SBI_HIP(hipEventElapsedTime(&ms, e0, e1));
        best = std::min(best, 1e3f * ms / kReps);
    }
    *us = best;
    return SBI_OK;
}

static sbi_status batch_autotune(sbi_batch* b) {
    if (b->g.size() == 1) return autotune(b->g[0].c, 0, nullptr);
    std::string ens = "ens";
    std::vector<std::string> keys;
    for (auto& gr : b->g) {
        std::string k;
        SBI_TRY(tune_key(gr.c, &k));
        keys.push_back(k);
        ens += ";" + k;
    }
    auto gkey = [&](size_t i) { return ens + "#g" + std::to_string(i); };
    {
        TuneCache& tc = tune_cache();
        std::lock_guard<std::mutex> lk(tc.mu);
        bool all = true;
        for (size_t i = 0; i < b->g.size() && all; ++i) all = tc.plans.count(gkey(i)) > 0;
        if (all) {
            bool ok = true;
            for (size_t i = 0; i < b->g.size(); ++i) ok = ok && plan_apply(b->g[i].c, tc.plans[gkey(i)]) == SBI_OK;
            if (ok) return SBI_OK;
        }
    }
    hipEvent_t e0, e1;
    SBI_HIP(hipEventCreate(&e0));
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return SBI_ERR_HIP;
    }
    sbi_status st = SBI_OK;
    std::vector<sbi_plan> best(b->g.size());
    for (size_t i = 0; i < b->g.size(); ++i) {
        sbi_ctx* c = b->g[i].c;
        best[i] = sbi_plan{c->gd.row_var, c->gd.row_rpw, c->group_target, 0.f, 0};
    }
    float cur = 0.f;
    if (st == SBI_OK) st = ensemble_time(b, e0, e1, &cur);
    for (size_t i = 0; i < b->g.size() && st == SBI_OK; ++i) {
        sbi_ctx* c = b->g[i].c;
        if (c->grid.mode == SBI_MODE_FULL) continue;
        for (const sbi_plan& cand : plan_candidates(c)) {
            st = plan_apply(c, cand);
            float us = 0.f;
            if (st == SBI_OK) st = ensemble_time(b, e0, e1, &us);
            if (st != SBI_OK) break;
            if (us < cur) {
                cur = us;
                best[i] = cand;
            }
        }
        if (st == SBI_OK) st = plan_apply(c, best[i]);
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (st != SBI_OK) return st;
    for (size_t i = 0; i < b->g.size(); ++i) {
        sbi_ctx* c = b->g[i].c;
        c->have_prev = false;
        c->hist_count = 0;
        best[i].us = cur;
        SBI_TRY(hip_ok(launch_ctl_reset(c->ctl, c->batch, c->grid.max_sweeps + 2, c->stream)));
    }
    TuneCache& tc = tune_cache();
    std::lock_guard<std::mutex> lk(tc.mu);
    for (size_t i = 0; i < b->g.size(); ++i) tc.plans[gkey(i)] = best[i];
    return SBI_OK;
}

extern "C" sbi_status sbi_batch_init(sbi_batch** out, int32_t m, const sbi_grid* grids, const double* const* depths,
                                     double h_ref, void* workspace, size_t ws_bytes, void* hip_stream,
                                     int32_t flags) {
    if (!out || m < 1 || !grids || !depths || !workspace) return SBI_ERR_INVALID_ARG;
    *out = nullptr;
    for (int i = 0; i < m; ++i)
        if (!grid_valid(&grids[i]) || !depths[i]) return SBI_ERR_INVALID_ARG;
    for (int i = 0; i < m; ++i)
        // the fully nonlinear solve and the mixed-precision refinement poll the host
        if (grids[i].mode == SBI_MODE_FULL || grids[i].precision == SBI_MIXED) return SBI_ERR_UNSUPPORTED;
    const size_t need = sbi_batch_workspace_bytes(m, grids);
    if (ws_bytes < need) return SBI_ERR_WORKSPACE;
    auto* b = new sbi_batch();
    b->m = m;
    b->flags = flags;
    b->stream = static_cast<hipStream_t>(hip_stream);
    if (hipEventCreateWithFlags(&b->fork, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&b->in, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&b->out, hipEventDisableTiming) != hipSuccess ||
        hipStreamCreateWithFlags(&b->cap, hipStreamNonBlocking) != hipSuccess) {
        batch_free(b);
        return SBI_ERR_HIP;
    }
    char* p = static_cast<char*>(workspace);
    sbi_status warn = SBI_OK;
    for (auto& gm : group_members(m, grids)) {
        sbi_batch::Group gr;
        gr.members = gm;
        const sbi_grid& g = grids[gm[0]];
        const int count = (int)gm.size();
        const size_t npt = (size_t)g.nx * g.ny;
        gr.field_bytes = npt * (g.precision == SBI_FP64 ? 8 : 4);
        if (hipStreamCreateWithFlags(&gr.s, hipStreamNonBlocking) != hipSuccess ||
            hipEventCreateWithFlags(&gr.done, hipEventDisableTiming) != hipSuccess) {
            b->g.push_back(gr);
            batch_free(b);
            return SBI_ERR_HIP;
        }
        std::vector<double> dep(npt * count);
        for (int k = 0; k < count; ++k) std::memcpy(&dep[npt * k], depths[gm[k]], sizeof(double) * npt);
        const size_t wsb = al256(layout(&g, count).total);
        sbi_status st = sbi_init(&gr.c, &g, count, dep.data(), h_ref, p, wsb, gr.s);
        p += wsb;
        gr.st_eta = p;
        gr.st_phi = p + al256(gr.field_bytes * count);
        gr.bk_state = p + 2 * al256(gr.field_bytes * count);
        gr.bk_cmp = p + 4 * al256(gr.field_bytes * count);
        p += staging_bytes(g, count);
        b->g.push_back(gr);
        if (st < 0) {
            batch_free(b);
            return st;
        }
        if (st == SBI_WARN_DEPTH_CRITERION) warn = st;
        b->g.back().cmp_bytes = (size_t)(static_cast<char*>(b->g.back().c->comp[C_DB]) -
                                         static_cast<char*>(b->g.back().c->comp[C_DV]));
    }
    if (flags & SBI_BATCH_AUTOTUNE) {
        const sbi_status st = batch_autotune(b);
        if (st < 0) {
            batch_free(b);
            return st;
        }
    }
    *out = b;
    return warn;
}

// enqueue n steps of every group on streams forked from b->cap and joined
// back to it (capture-safe: no host synchronisation)
// The parts of a step call: the prologue copies the members' states in and
// transforms them, a steps part advances the spectral states n steps, the
// epilogue transforms back and copies out.  Each part forks the groups onto
// their streams and joins them back to b->cap.
enum { PART_PROLOGUE = 0, PART_STEPS = 1, PART_EPILOGUE = 2 };

static sbi_status batch_enqueue_part(sbi_batch* b, sbi_state* states, int part, double dt, int n, double tol,
                                     double toff) {
    // nothing enqueued here may depend on the state time: a captured graph is
    // replayed at later times, and a group's members need not share one t.
    // Time-dependent forcing (wavemaker, relaxation zones) is therefore not
    // available to ensembles (no setter reaches a group's context).
    for (auto& gr : b->g)
        if (gr.c->relax_on || gr.c->wm_n > 0 || gr.c->dmp_w > 0.0) return SBI_ERR_UNSUPPORTED;
    SBI_HIP(hipEventRecord(b->fork, b->cap));
    for (auto& gr : b->g) {
        sbi_ctx* c = gr.c;
        SBI_HIP(hipStreamWaitEvent(gr.s, b->fork, 0));
        if (part == PART_PROLOGUE) {
            SBI_TRY(hip_ok(launch_ctl_acc_reset(c->ctl, c->batch, gr.s)));
            for (size_t k = 0; k < gr.members.size(); ++k) {
                const sbi_state& s = states[gr.members[k]];
                SBI_HIP(hipMemcpyAsync(gr.st_eta + k * gr.field_bytes, s.eta, gr.field_bytes,
                                       hipMemcpyDeviceToDevice, gr.s));
                SBI_HIP(hipMemcpyAsync(gr.st_phi + k * gr.field_bytes, s.phi_s, gr.field_bytes,
                                       hipMemcpyDeviceToDevice, gr.s));
            }
            SBI_TRY(to_spectral(c, gr.st_eta, gr.st_phi, true));
        } else if (part == PART_STEPS) {
            double t = states[gr.members[0]].t + toff;
            for (int step = 0; step < n; ++step) {
                for (int stage = 0; stage < 4; ++stage) {
                    int vh = 0;
                    SBI_TRY(solve_stage(c, nullptr, tol, true, &vh, nullptr, true, stage));
                    SBI_TRY(stage_update(c, stage, dt, vh, t));
                }
                t += dt;
                if (c->relax_on) SBI_TRY(relax_zone(c, t));
            }
        } else {
            SBI_TRY(to_physical(c, gr.st_eta, gr.st_phi));
            for (size_t k = 0; k < gr.members.size(); ++k) {
                const sbi_state& s = states[gr.members[k]];
                SBI_HIP(hipMemcpyAsync(s.eta, gr.st_eta + k * gr.field_bytes, gr.field_bytes,
                                       hipMemcpyDeviceToDevice, gr.s));
                SBI_HIP(hipMemcpyAsync(s.phi_s, gr.st_phi + k * gr.field_bytes, gr.field_bytes,
                                       hipMemcpyDeviceToDevice, gr.s));
            }
        }
        SBI_HIP(hipEventRecord(gr.done, gr.s));
        SBI_HIP(hipStreamWaitEvent(b->cap, gr.done, 0));
    }
    return SBI_OK;
}

// backup (save) or restore of what a step call changes: the members' states
// and the carried compact buffers (previous-solve parts, learned history),
// plus their host-side flags; on the batch's stream
static sbi_status batch_keep(sbi_batch* b, sbi_state* states, bool save) {
    for (auto& gr : b->g) {
        sbi_ctx* c = gr.c;
        for (size_t k = 0; k < gr.members.size(); ++k) {
            const sbi_state& st = states[gr.members[k]];
            char* be = gr.bk_state + (2 * k) * gr.field_bytes;
            char* bp = gr.bk_state + (2 * k + 1) * gr.field_bytes;
            SBI_HIP(hipMemcpyAsync(save ? be : st.eta, save ? st.eta : be, gr.field_bytes, hipMemcpyDeviceToDevice,
                                   b->cap));
            SBI_HIP(hipMemcpyAsync(save ? bp : st.phi_s, save ? st.phi_s : bp, gr.field_bytes,
                                   hipMemcpyDeviceToDevice, b->cap));
        }
        if (c->grid.seed == SBI_SEED_PREV || c->grid.seed == SBI_SEED_NET) {
            char* d0 = static_cast<char*>(c->comp[C_DV]);   // C_DV, C_DB
            char* h0 = static_cast<char*>(c->comp[C_HV0]);  // C_HV0 .. C_HB0 + kHistTaps - 1
            SBI_HIP(hipMemcpyAsync(save ? gr.bk_cmp : d0, save ? d0 : gr.bk_cmp, 2 * gr.cmp_bytes,
                                   hipMemcpyDeviceToDevice, b->cap));
            SBI_HIP(hipMemcpyAsync(save ? gr.bk_cmp + 2 * gr.cmp_bytes : h0, save ? h0 : gr.bk_cmp + 2 * gr.cmp_bytes,
                                   2 * kHistTaps * gr.cmp_bytes, hipMemcpyDeviceToDevice, b->cap));
        }
        if (save) {
            gr.bk_have_prev = c->have_prev;
            gr.bk_hist_count = c->hist_count;
        } else {
            c->have_prev = gr.bk_have_prev;
            c->hist_count = gr.bk_hist_count;
        }
    }
    return SBI_OK;
}

// enqueue one step call on the batch's stream: replay the instantiated graph
// (captured again when its key changed) or the eager launches
// Steps per captured graph of a step call.  Replaying short graphs is
// faster per step than one long one: the 96-member ragged SA ensemble runs
// 7.3 ms per step from graphs of 4 steps, 8.1 from 16 and 8.8 from one graph
// of 64 steps (no drift over 256 steps of 4-step graphs, so not a clock
// effect); graphs of 4 steps also keep capture and instantiation short.
constexpr int kGraphSteps = 4;
constexpr size_t kMaxGraphs = 8;

// enqueue one part as a captured graph (looked up, else captured and
// instantiated) or directly
static sbi_status batch_part(sbi_batch* b, sbi_state* states, int part, double dt, int n, double tol, double toff) {
    if (!(b->flags & SBI_BATCH_GRAPH)) return batch_enqueue_part(b, states, part, dt, n, tol, toff);
    std::vector<const void*> ptrs;
    std::vector<int> prev, budget;
    if (part != PART_STEPS)
        for (int i = 0; i < b->m; ++i) {
            ptrs.push_back(states[i].eta);
            ptrs.push_back(states[i].phi_s);
        }
    // what the captured solves are seeded from: the previous solve, and how
    // many history entries the learned layer holds; and the sweep budgets
    if (part == PART_STEPS)
        for (auto& gr : b->g) {
            prev.push_back((gr.c->have_prev ? 1 : 0) + 2 * std::min(gr.c->hist_count, gr.c->hist_K));
            budget.push_back(gr.c->budget);
        }
    const bool steps = part == PART_STEPS;
    sbi_batch::Graph* hit = nullptr;
    for (auto& gg : b->graphs)
        if (gg.part == part && gg.ptrs == ptrs && (!steps || (gg.n == n && gg.dt == dt && gg.tol == tol &&
                                                               gg.prev == prev && gg.budget == budget))) {
            hit = &gg;
            break;
        }
    if (!hit) {
        if (b->graphs.size() >= kMaxGraphs) {
            auto lru = std::min_element(b->graphs.begin(), b->graphs.end(),
                                        [](const sbi_batch::Graph& x, const sbi_batch::Graph& y) {
                                            return x.used < y.used;
                                        });
            (void)hipGraphExecDestroy(lru->exec);
            b->graphs.erase(lru);
        }
        std::vector<int> saved_prof;
        for (auto& gr : b->g) {
            saved_prof.push_back(gr.c->prof.on ? 1 : 0);
            gr.c->prof.on = false;  // no timing events inside a capture
        }
        SBI_HIP(hipStreamBeginCapture(b->cap, hipStreamCaptureModeThreadLocal));
        sbi_status st = batch_enqueue_part(b, states, part, dt, n, tol, toff);
        hipGraph_t graph = nullptr;
        hipError_t e = hipStreamEndCapture(b->cap, &graph);
        for (size_t k = 0; k < b->g.size(); ++k) b->g[k].c->prof.on = saved_prof[k] != 0;
        if (st < 0) {
            if (graph) (void)hipGraphDestroy(graph);
            return st;
        }
        if (e != hipSuccess) return SBI_ERR_HIP;
        sbi_batch::Graph gg;
        e = hipGraphInstantiate(&gg.exec, graph, nullptr, nullptr, 0);
        (void)hipGraphDestroy(graph);
        if (e != hipSuccess) return SBI_ERR_HIP;
        gg.part = part;
        gg.n = steps ? n : 0;
        gg.dt = steps ? dt : 0.0;
        gg.tol = steps ? tol : 0.0;
        gg.ptrs = ptrs;
        gg.prev = prev;
        gg.budget = budget;
        b->graphs.push_back(gg);
        hit = &b->graphs.back();
    }
    hit->used = ++b->clock;
    SBI_HIP(hipGraphLaunch(hit->exec, b->cap));
    return SBI_OK;
}

// a whole step call: prologue, the steps in parts of at most kGraphSteps,
// epilogue (the spectral states stay in the workspace between parts, so the
// result does not depend on the split)
static sbi_status batch_launch(sbi_batch* b, sbi_state* states, double dt, int n, double tol) {
    SBI_TRY(batch_part(b, states, PART_PROLOGUE, dt, 0, tol, 0.0));
    for (int done = 0; done < n; done += kGraphSteps) {
        const int k = std::min(kGraphSteps, n - done);
        SBI_TRY(batch_part(b, states, PART_STEPS, dt, k, tol, done * dt));
    }
    return batch_part(b, states, PART_EPILOGUE, dt, 0, tol, 0.0);
}

extern "C" sbi_status sbi_batch_step(sbi_batch* b, sbi_state* states, double dt, int32_t n, double tol,
                                     sbi_step_info* info) {
    if (!b || !states || n < 0 || !std::isfinite(dt)) return SBI_ERR_INVALID_ARG;
    for (int i = 0; i < b->m; ++i)
        if (!states[i].eta || !states[i].phi_s) return SBI_ERR_INVALID_ARG;
    for (auto& gr : b->g) {
        if (gr.c->grid.mode != SBI_MODE_SA && !(tol >= 0.0)) return SBI_ERR_INVALID_ARG;
        if (gr.c->grid.seed == SBI_SEED_NET && !gr.c->net_loaded && !gr.c->hist_loaded) return SBI_ERR_INVALID_ARG;
        gr.c->st = Stats();
        gr.c->fallbacks = 0;
    }
    // the caller's work before this call happens first
    SBI_HIP(hipEventRecord(b->in, b->stream));
    SBI_HIP(hipStreamWaitEvent(b->cap, b->in, 0));
    // Iterations run on a speculative sweep budget (the largest sweep count
    // of the last call plus a margin): when a solve outruns it, the call is
    // redone from its saved inputs with the budget doubled, so the results
    // are those of the full max_sweeps budget.
    bool speculative = false;
    for (auto& gr : b->g)
        speculative |= gr.c->grid.mode == SBI_MODE_ITER && gr.c->budget > 0 && gr.c->budget < gr.c->grid.max_sweeps;
    for (;;) {
        if (speculative) SBI_TRY(batch_keep(b, states, true));
        SBI_TRY(batch_launch(b, states, dt, n, tol));
        SBI_HIP(hipStreamSynchronize(b->cap));
        bool redo = false;
        for (auto& gr : b->g) {
            sbi_ctx* c = gr.c;
            SBI_HIP(hipMemcpy(c->head, c->ctl, sizeof(Ctl) * c->batch, hipMemcpyDeviceToHost));
            if (c->grid.mode != SBI_MODE_ITER) continue;
            bool undecided = false;
            for (size_t k = 0; k < gr.members.size(); ++k) undecided |= c->head[k].acc_solves < 4ll * n;
            if (undecided) {
                // only a budget below max_sweeps leaves a solve undecided
                c->budget = std::min(2 * c->budget, c->grid.max_sweeps);
                redo = true;
            }
        }
        if (!redo) break;
        b->redos += 1;
        SBI_TRY(batch_keep(b, states, false));
        speculative = true;
    }
    SBI_HIP(hipEventRecord(b->out, b->cap));
    SBI_HIP(hipStreamWaitEvent(b->stream, b->out, 0));
    sbi_status worst = SBI_OK;
    for (auto& gr : b->g) {
        sbi_ctx* c = gr.c;
        const bool iter = c->grid.mode == SBI_MODE_ITER;
        int smax = 0;
        for (size_t k = 0; k < gr.members.size(); ++k) {
            const Ctl& h = c->head[k];
            int st = iter ? h.acc_worst : 0;
            if (h.nonfinite) st = SBI_ERR_NONFINITE;
            const int mi = gr.members[k];
            states[mi].t += n * dt;
            if (info) {
                sbi_step_info& si = info[mi];
                si = sbi_step_info{};
                si.solves = iter ? h.acc_solves : 4ll * n;
                si.sweeps_total = iter ? h.acc_sweeps : 0;
                si.sweeps_max = iter ? h.acc_sweeps_max : 0;
                si.max_residual = iter ? h.acc_residual_max : 0.0;
            }
            smax = std::max(smax, h.acc_sweeps_max);
            if (st < 0) worst = (worst < 0 && worst < st) ? worst : (sbi_status)st;
            else if (worst >= 0 && st > worst) worst = (sbi_status)st;
        }
        if (worst < 0) {
            c->have_prev = false;
            c->hist_count = 0;
        }
        // next budget: the largest sweep count of this call plus a margin;
        // changed only when it moves by more than the margin (each change is
        // a new capture)
        if (iter && n > 0) {
            const int want = std::min(c->grid.max_sweeps, smax + kBudgetMargin);
            if (c->budget <= 0 || want > c->budget || want + kBudgetMargin < c->budget) c->budget = want;
        }
    }
    return worst;
}

extern "C" sbi_status sbi_batch_net_load(sbi_batch* b, const void* weights, size_t bytes) {
    if (!b || !weights) return SBI_ERR_INVALID_ARG;
    for (auto& gr : b->g)
        if (gr.c->grid.seed == SBI_SEED_NET) SBI_TRY(sbi_net_load(gr.c, weights, bytes));
    return SBI_OK;
}

extern "C" sbi_status sbi_batch_net_hist_load(sbi_batch* b, int32_t taps, int32_t bins, double dk, const float* w) {
    if (!b || !w) return SBI_ERR_INVALID_ARG;
    for (auto& gr : b->g)
        if (gr.c->grid.seed == SBI_SEED_NET) SBI_TRY(sbi_net_hist_load(gr.c, taps, bins, dk, w));
    return SBI_OK;
}

extern "C" int32_t sbi_batch_groups(const sbi_batch* b, int32_t* members_out, int32_t* split_out, int32_t n) {
    if (!b) return 0;
    const int ng = (int)b->g.size();
    for (int i = 0; i < ng && i < n; ++i) {
        if (members_out) members_out[i] = (int32_t)b->g[i].members.size();
        if (split_out) split_out[i] = b->g[i].c->group_target;
    }
    return ng;
}

extern "C" sbi_status sbi_batch_plan(const sbi_batch* b, int32_t g, sbi_plan* out) {
    if (!b || !out || g < 0 || g >= (int32_t)b->g.size()) return SBI_ERR_INVALID_ARG;
    return sbi_plan_get(b->g[g].c, out);
}

extern "C" int32_t sbi_batch_budgets(const sbi_batch* b, int32_t* budget_out, int32_t n) {
    if (!b) return 0;
    const int ng = (int)b->g.size();
    for (int i = 0; i < ng && i < n; ++i)
        if (budget_out) {
            const sbi_ctx* c = b->g[i].c;
            budget_out[i] = (c->budget > 0 && c->budget < c->grid.max_sweeps) ? c->budget : c->grid.max_sweeps;
        }
    return b->redos;
}

extern "C" sbi_status sbi_batch_destroy(sbi_batch* b) {
    if (!b) return SBI_ERR_INVALID_ARG;
    (void)hipStreamSynchronize(b->cap);
    for (auto& gr : b->g) (void)hipStreamSynchronize(gr.s);
    batch_free(b);
    return SBI_OK;
}
