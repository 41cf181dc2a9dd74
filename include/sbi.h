/*
 * sbi.h -- C interface of the MI355X (gfx950) spectral boundary-integral wave
 * solver: the surface vertical velocity W of the enhanced spectral boundary
 * integral method over variable depth, and the time step of the surface
 * evolution equations that uses it.
 *
 * Operations follow Wang, "An Enhanced Spectral Boundary Integral Method for
 * Modeling Highly Nonlinear Water Waves in Variable Depth":
 *   - the problem statement: given the surface elevation eta(x,y), the surface
 *     potential phi_s(x,y) and the depth h(x,y), find the surface vertical
 *     velocity V = sqrt(1+|grad eta|^2) dphi/dn at z = eta (Sec. 2.2, the
 *     definition under Eq. (prognostic)); this interface calls it W;
 *   - W is evaluated by the successive approximation of Sec. 2.4 with the
 *     explicit orders of Appendix C (Eqs. (v2)-(v7)) -- mode SBI_MODE_SA --
 *     or by iterating the same expansion summed over orders to a residual
 *     tolerance -- mode SBI_MODE_ITER -- or, on one-dimensional grids,
 *     fully nonlinearly: the boundary-integral equations of Sec. 2.3 with the
 *     remaining integrals I^(S) of App. A kept (Eq. (con-V): the expansion
 *     plus I^(S) is the exact equation) and, over a variable bed, the bed's
 *     remainder I^(B) of App. B, in their two-dimensional-flow form (Green
 *     function -ln r; over a flat bed its image, over a variable bed the bed
 *     as a second boundary with the potential phi_b on it, unless it lies too
 *     deep to matter: k_1 times the smallest depth beyond 18), iterated to the
 *     residual tolerance with O(nx^2) quadrature per sweep -- mode
 *     SBI_MODE_FULL (ensembles do not take it);
 *   - the time step integrates Eq. (prognostic) in its integrating-factor form
 *     (Sec. 2.2) with the classical 4-stage Runge-Kutta scheme of Lawson type
 *     (fixed step), or with the adaptive six-stage fifth-order pair with an
 *     embedded fourth-order solution that Sec. 2.2 describes;
 *   - the total energy is Eq. (energy) of Sec. 3.1.
 *
 * Units: lengths scaled by the peak wavenumber, time by the peak angular
 * frequency, g = 1 (Sec. 2.1).  The seabed is at z = -h_ref + delta(x,y),
 * delta = h_ref - depth >= 0.
 *
 * Conventions shared by every call
 *   - Returns sbi_status: 0 success, > 0 warning (outputs are written and
 *     usable), < 0 error (no output written; sbi_status_string() explains).
 *   - Field pointers are DEVICE pointers to row-major [batch][ny][nx] arrays
 *     of the context's precision (double for SBI_FP64 and SBI_MIXED, float for SBI_FP32),
 *     contiguous, owned by the caller.  The library never frees them.
 *   - Depth arrays are HOST pointers to double [batch][ny][nx], depth > 0.
 *   - All device work is enqueued on the context's HIP stream; calls that
 *     return host values (info structs, diagnostics) synchronise that stream.
 *   - One context per stream.  Contexts share no mutable state.
 *   - Device memory: the library allocates it only in sbi_init, and only when
 *     the caller passes no workspace (the context then owns one, freed by
 *     sbi_destroy); every other call works in caller-owned memory (or, for
 *     sbi_vertical_velocity_noalloc, in the library's static scratch array).
 *     sbi_init also takes a small pinned host buffer for the control headers.
 *   - Non-finite inputs are reported as SBI_ERR_NONFINITE.
 */
#ifndef SBI_H
#define SBI_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct sbi_ctx sbi_ctx;

typedef enum sbi_status {
    SBI_OK = 0,
    SBI_WARN_NOT_CONVERGED = 1,   /* iteration hit max_sweeps; last iterate returned */
    SBI_WARN_DEPTH_CRITERION = 2, /* k_band*max(delta) > 2.4, validity limit of Sec. 5 */
    SBI_WARN_FALLBACK_USED = 3,   /* learned seed rejected; linear guess used instead */
    SBI_WARN_STEP_LIMIT = 4,      /* adaptive stepping stopped at max_steps before t_end */
    SBI_ERR_INVALID_ARG = -1,
    SBI_ERR_UNSUPPORTED = -2,
    SBI_ERR_WORKSPACE = -3,
    SBI_ERR_HIP = -4,
    SBI_ERR_NONFINITE = -5,
    SBI_ERR_DIVERGED = -6
} sbi_status;

enum { SBI_FP64 = 0, SBI_FP32 = 1, SBI_MIXED = 2 };
enum { SBI_MODE_ITER = 0, SBI_MODE_SA = 1, SBI_MODE_FULL = 2 };
enum { SBI_SEED_LINEAR = 0, SBI_SEED_PREV = 1, SBI_SEED_NET = 2, SBI_SEED_USER = 3 };
enum { SBI_ACCEL_NONE = 0, SBI_ACCEL_ANDERSON = 1 };

/* Grid and solver options.  Fill with sbi_grid_defaults() first. */
typedef struct sbi_grid {
    int32_t nx, ny;        /* collocation points; powers of two, nx in 16..8192,
                              ny == 1 (1D) or 16..2048 */
    double lx, ly;         /* periodic lengths (ly ignored when ny == 1) */
    int32_t order;         /* expansion order L, 1..7 (Sec. 2.4 caps it at 7); default 7 */
    double dealias;        /* kept fraction alpha of the Nyquist wavenumber per axis:
                              modes |m| < alpha n/2 are kept (the "2/(l+1) rule" of
                              Sec. 2.4 read as alpha = 1/2); 0 < alpha < 1; default 0.5 */
    int32_t precision;     /* SBI_FP64 (default) or SBI_FP32 (FP64 residual norms and
                              diagnostics are kept either way), or SBI_MIXED (mode
                              SBI_MODE_ITER only; fields in double): iterative
                              refinement of the iteration's fixed point x = T(x) =
                              A x + b.  An FP64 sweep forms the residual
                              r = T(x) - x and takes the stopping decision of the
                              FP64 iteration on it (same test, same tolerance);
                              between two such sweeps FP32 sweeps (relaxed or
                              Anderson-mixed, as accel says) solve the correction
                              equation d = A d + r from d = r to a relative
                              residual between 1e-5 and 0.1, chosen so that the
                              next FP64 test can pass, and x += d in FP64.
                              Reaches the FP64 tolerances (1e-8 and tighter)
                              where SBI_FP32 stops near 1e-6; at most 10 FP64
                              sweeps per solve (then SBI_WARN_NOT_CONVERGED).
                              Not for ensembles (sbi_batch_init) or
                              sbi_vertical_velocity_noalloc (SBI_ERR_UNSUPPORTED) */
    int32_t mode;          /* SBI_MODE_ITER (default), SBI_MODE_SA or SBI_MODE_FULL (1D) */
    int32_t seed;          /* SBI_SEED_* for the iteration; default SBI_SEED_LINEAR,
                              the initiation of Sec. 2.4.  SBI_SEED_PREV: the linear
                              guess plus the nonlinear part (V* - k tanh(kh) phi_hat,
                              phi_b - sech(kh) phi_hat) that the context's previous
                              solve left (the first solve, and any solve after a
                              failed one, uses the linear guess).  SBI_SEED_NET: the
                              learned warm start of sbi_net.h (2D grids, weights from
                              sbi_net_load) for solves with no previous solve to start
                              from, the SBI_SEED_PREV seed otherwise.  SBI_SEED_USER: the w_seed field of
                              sbi_vertical_velocity */
    int32_t max_sweeps;    /* iteration cap, 1..1000; default 64 */
    int32_t relax;         /* 1: under-relaxed sweeps when the crest makes plain sweeps
                              expand (default); 0: plain sweeps */
    double filter_beta1;   /* low-pass filter of Eq. (filter) applied each step when */
    double filter_beta2;   /* both are > 0; default 0 (off) */
    int32_t accel;         /* iteration mode: SBI_ACCEL_NONE (default) sweeps
                              V <- V + w (T(V) - V); SBI_ACCEL_ANDERSON mixes these
                              relaxed sweeps over the last two residual differences
                              (Anderson mixing, least squares in the inner product
                              of the real fields), same residual, stopping rules and
                              fixed point, typically half the sweeps */
} sbi_grid;

/* A batch of surface states: eta and phi_s are device arrays [batch][ny][nx]. */
typedef struct sbi_state {
    void* eta;
    void* phi_s;
    double t;              /* advanced by n*dt by sbi_step */
} sbi_state;

typedef struct sbi_solve_info {
    int32_t sweeps;        /* applications of the sweep operator (0 in SA mode);
                              SBI_MIXED: FP64 and FP32 sweeps together */
    int32_t status;        /* per-member sbi_status of the solve */
    double residual;       /* max|T(W)-W| / max|T(W)| of the last sweep, FP64 */
    double omega;          /* relaxation weight used */
    int32_t sweeps_fp32;   /* SBI_MIXED: the FP32 sweeps among sweeps; else 0 */
} sbi_solve_info;

typedef struct sbi_step_info {
    int64_t solves;        /* W solves performed (4 per step per member) */
    int64_t sweeps_total;  /* summed over solves and members */
    int32_t sweeps_max;    /* largest sweep count of one solve */
    int32_t fallbacks;     /* solves that fell back to the linear guess */
    double max_residual;   /* largest final residual of any solve */
    int64_t sweeps_fp32_total; /* SBI_MIXED: the FP32 sweeps among sweeps_total; else 0 */
} sbi_step_info;

typedef struct sbi_adapt_info {
    int32_t accepted;      /* steps taken */
    int32_t rejected;      /* attempts discarded and redone with a smaller step */
    double dt_next;        /* step size proposed for a following call */
    double err_last;       /* error estimate of the last attempt */
    double err_max;        /* largest error estimate of an accepted step */
    sbi_step_info solve;   /* W solves of every attempt (6 per attempt per member) */
} sbi_adapt_info;

/* Default options (FP64, iteration, L = 7, alpha = 1/2, 64 sweeps, relax on). */
void sbi_grid_defaults(sbi_grid* g);

/* Device workspace bytes for `batch` members of grid g (0 if g is invalid). */
size_t sbi_workspace_bytes(const sbi_grid* g, int32_t batch);

/*
 * Create a context for `batch` members sharing grid g.
 *   depth     host double [batch][ny][nx], > 0 everywhere.
 *   h_ref     reference depth h of Sec. 2.1; <= 0 selects max(depth) per member,
 *             so that delta = h_ref - depth >= 0.
 *   workspace device buffer of sbi_workspace_bytes(g, batch) bytes owned by the
 *             caller, or NULL to let the library allocate it here (hipMalloc,
 *             the library's only device allocation; freed by sbi_destroy).
 *   hip_stream hipStream_t to enqueue on (NULL = default stream).
 * Returns SBI_WARN_DEPTH_CRITERION (context valid) when
 * k_band * max(delta) > 2.4 (Sec. 5).
 */
sbi_status sbi_init(sbi_ctx** out, const sbi_grid* g, int32_t batch, const double* depth,
                    double h_ref, void* workspace, size_t ws_bytes, void* hip_stream);

/*
 * Surface vertical velocity W for every member (Sec. 2.3-2.4, App. C).
 *   eta, phi_s  device [batch][ny][nx]; phi_s is band-limited by the dealias
 *               mask before use (its spectrum outside the kept rectangle is
 *               dropped), eta is used as given.
 *   h           host depth [batch][ny][nx] replacing the context's depth, or NULL.
 *   tol         relative residual tolerance of the iteration (ignored in SA mode).
 *   w_seed      device [batch][ny][nx] initial guess when seed == SBI_SEED_USER,
 *               else NULL.
 *   w_out       device [batch][ny][nx] output.
 *   info        host array of `batch` entries, or NULL.
 */
sbi_status sbi_vertical_velocity(sbi_ctx* ctx, const void* eta, const void* phi_s,
                                 const double* h, double tol, const void* w_seed,
                                 void* w_out, sbi_solve_info* info);

/*
 * Allocation-free W solve, for callers that cannot allocate device memory:
 * tight serving loops and harnesses that forbid hipMalloc.  It is
 * sbi_vertical_velocity on a context made from (g, batch, depth, h_ref) as
 * sbi_init would make it, set up and released inside the call, with h = NULL.
 * Its workspace is the library's static device scratch array of 64 MiB (one
 * per device, held from the library's first use on that device until the
 * process ends); the call makes no hipMalloc, hipHostMalloc, hipFree or event,
 * and keeps its control headers in ordinary host memory.  Grids that need
 * more (sbi_workspace_bytes(g, batch) > 64 MiB, e.g. FP64 beyond 512 x 256
 * points per member, FP32 beyond 512 x 512) return SBI_ERR_WORKSPACE.
 *   The scratch array of a device is shared by every call on it and keeps the
 *   last call's contents; each call clears it before use.  Calls that overlap
 *   in time on one device (from other host threads or streams) race on it:
 *   the caller must serialise them.
 *   hip_stream must belong to the current device (SBI_ERR_INVALID_ARG
 *   otherwise); the call synchronises it before returning.
 *   seed: SBI_SEED_NET is SBI_ERR_UNSUPPORTED (its weights need a lasting
 *   context), and so is precision SBI_MIXED (its FP32 sweeps run in a second
 *   context); SBI_SEED_PREV starts from the linear guess (there is no previous
 *   solve); SBI_SEED_USER takes w_seed.  Returns what sbi_init and
 *   sbi_vertical_velocity would (SBI_WARN_DEPTH_CRITERION included).
 */
sbi_status sbi_vertical_velocity_noalloc(const sbi_grid* g, int32_t batch, const double* depth, double h_ref,
                                         const void* eta, const void* phi_s, double tol, const void* w_seed,
                                         void* w_out, sbi_solve_info* info, void* hip_stream);

/*
 * Advance every member by n steps of dt (Eq. (prognostic), integrating-factor
 * RK4), in place; state->t += n*dt.  Each step performs 4 W solves with the
 * context's mode and tolerance `tol`.  The state is band-limited by the dealias
 * mask on entry and after every step.  info (host, may be NULL) aggregates over
 * members.
 */
sbi_status sbi_step(sbi_ctx* ctx, sbi_state* state, double dt, int32_t n, double tol,
                    sbi_step_info* info);

/*
 * Adaptive integration of Eq. (prognostic) (Sec. 2.2): every member is advanced
 * in place from state->t to t_end by a six-stage fifth-order Runge-Kutta pair
 * with an embedded fourth-order solution (the Cash-Karp coefficients; the paper
 * does not print its own), in the same integrating-factor (Lawson) form as
 * sbi_step.  Each attempt performs 6 W solves with the context's mode and `tol`.
 * The step size is controlled by the difference of the two solutions measured
 * in the linear-energy norm, err = sqrt(sum |d eta_k|^2 + k tanh(kh)|d phi_k|^2
 * / the same sum over the fifth-order state), the largest over the members
 * (all members share one step size): an attempt with err <= rk_tol is
 * accepted (the fifth-order state is kept, then band-limited, filtered and
 * relaxed like sbi_step's), else redone; the next size is
 * h * min(5, max(0.2, 0.9 (rk_tol/err)^(1/5))), without growth right after a
 * rejection.  A step whose trial size reaches t_end (to a relative 1e-9) is
 * cut to land on it.  The paper keeps the difference below 1e-2 (validation
 * cases) or 1e-3 (long crossing-sea runs).
 *   dt        first trial step, > 0.
 *   rk_tol    > 0.
 *   max_steps cap on attempts; reaching it returns SBI_WARN_STEP_LIMIT with
 *             the state written at state->t < t_end.
 *   info      host, may be NULL; dt_next carries the controller's proposal to
 *             a following call (after a cut last step, the larger of the
 *             proposal and the trial size before the cut).
 * Errors: SBI_ERR_INVALID_ARG (t_end < state->t, dt or rk_tol not positive and
 * finite, max_steps < 1); SBI_ERR_DIVERGED also when the step size falls below
 * 1e-12 of the interval; the state is left unchanged on any error.  The call
 * synchronises the stream after every attempt (no graph capture).
 */
sbi_status sbi_step_adaptive(sbi_ctx* ctx, sbi_state* state, double t_end, double dt, double rk_tol,
                             double tol, int32_t max_steps, sbi_adapt_info* info);

/*
 * FP64 mass  M = dA * sum(eta)  and energy  E = dA/2 * sum(W phi_s + eta^2)
 * (Eq. (energy)) of the band-limited state, per member (host arrays of `batch`).
 */
sbi_status sbi_diagnostics(sbi_ctx* ctx, const sbi_state* state, double tol,
                           double* mass, double* energy);

/*
 * Wave generation/absorption by relaxation zones in a 1D tank, applied after
 * every step (not a device of the paper, whose tank uses a pneumatic
 * wavemaker).  params = {a, k, omega, gen_len, abs_len, ramp_periods}: target
 * eta = a r(t) cos(kx - omega t), phi_s = (a r(t)/omega) sin(kx - omega t) over
 * x < gen_len with weight 1-(3s^2-2s^3), s = x/gen_len; damping to zero over
 * x > lx - abs_len; ramp r(t) = (1-cos(pi t/(ramp_periods*2pi/omega)))/2.
 * n = 6; n = 0 removes the zones.
 */
sbi_status sbi_set_relaxation(sbi_ctx* ctx, const double* params, int32_t n);

/*
 * Numerical wave tank of Sec. 3.2: surface pressures p = p_g + p_d that enter
 * the dynamic surface condition (phi_t = ... - eta - p) of every later step
 * (sbi_step, sbi_step_adaptive) at each stage's time.
 *   comps      host double [ncomp][4] = {a_j, k_j, omega_j, theta_j}, 0 <= ncomp
 *              <= 8: the pneumatic wavemaker
 *              p_g = sum_j a_j sqrt(e/(2 pi)) (1 + 2 k_j h/sinh(2 k_j h))
 *                    exp(-(k_j x)^2/2) sin(omega_j t + theta_j),
 *              a bell centred on x = 0, i.e. split in halves over both ends of
 *              the periodic domain, uniform in y; to linear order it radiates
 *              waves of amplitude a_j both ways (k_j > 0; omega_j >= 0, usually
 *              sqrt(k_j tanh(k_j h))).
 *   h_gen      the depth h of the generator's factor; <= 0: each member's h_ref.
 *   damp_x0,   the damping pressure of Eq. (pd),
 *   damp_width   p_d = F^-1{ i k/(-k^2) . MF{mu grad phi_s} } (k = 0 mode: 0),
 *              mu = exp(-((x - damp_x0)/damp_width)^2) with x - damp_x0 taken
 *              periodically; the paper uses damp_width = 4 pi and damp_x0 =
 *              7/8 of the domain; damp_width <= 0 turns the damping off.
 * ncomp = 0 with damp_width <= 0 removes the tank's pressures.  Settings are
 * copied; errors (SBI_ERR_INVALID_ARG: ncomp out of range, non-finite values,
 * k_j <= 0, omega_j < 0) leave the previous ones in place.
 */
sbi_status sbi_set_wavemaker(sbi_ctx* ctx, const double* comps, int32_t ncomp, double h_gen, double damp_x0,
                             double damp_width);

/* Replace the depth (host [batch][ny][nx]) and reference depth of a context;
   empties the history of the learned history layer (sbi_net.h), not its
   training sums. */
sbi_status sbi_set_depth(sbi_ctx* ctx, const double* depth, double h_ref);

/*
 * Load the weights of the learned warm start (used when seed == SBI_SEED_NET).
 * weights: host blob of sbi_net_blob_bytes() bytes (sbi_net_header followed by
 * the FP32 parameter vector, see sbi_net.h); copied, caller keeps ownership.
 * Errors: SBI_ERR_INVALID_ARG for a wrong size, header or non-finite value.
 */
sbi_status sbi_net_load(sbi_ctx* ctx, const void* weights, size_t bytes);

/* Release the context (and the workspace if the library allocated it). */
sbi_status sbi_destroy(sbi_ctx* ctx);

const char* sbi_status_string(sbi_status s);

/*
 * Kernel timing for profiling: when enabled, launches of the following calls
 * are bracketed by HIP events on the context's stream; enable is
 * SBI_PROFILE_ALL (every kernel class), SBI_PROFILE_SWEEPS (the row and column
 * sweep passes of the iteration only: each bracket adds a few microseconds of
 * idle device time, so timing fewer launches disturbs the run less) or
 * SBI_PROFILE_OFF.  Synchronises the stream and clears the totals.
 * sbi_profile_read writes, per kernel class, its name (static string), summed
 * device time in ms and launch count since the last enable, and returns the
 * number of classes.  In SBI_MIXED contexts the FP32 correction sweeps count
 * as "row_sweep_fp32" and "col_sweep_fp32", the FP64 refinement sweeps as
 * "row_sweep" and "col_sweep".
 */
enum { SBI_PROFILE_OFF = 0, SBI_PROFILE_ALL = 1, SBI_PROFILE_SWEEPS = 2 };
sbi_status sbi_profile_enable(sbi_ctx* ctx, int32_t enable);
int32_t sbi_profile_read(sbi_ctx* ctx, const char** names, double* total_ms, int64_t* launches, int32_t n);

/* Timing and counters of the last call (host), for profiling.  Returns the
 * number of doubles written (<= n): {kernel launches, host syncs, sweeps}. */
int32_t sbi_last_stats(const sbi_ctx* ctx, double* out, int32_t n);

/*
 * Launch plans and the autotuner.  A plan fixes, for one context, how its
 * transforms are launched; it changes rounding order only, never what is
 * computed (every plan meets the same parity bars against the FP64 oracle).
 *   row_variant  radix sequence and twiddle mode of the row sweep (iteration)
 *                or row SA kernels: 0 radix-8 passes with twiddle powers by
 *                recurrence (the default); 1 radix-8 with every twiddle power
 *                cached in registers; 2 radix-16 passes; 3 radix-4 passes (a
 *                row spread over twice the threads).  Which variants are
 *                built depends on precision and row length (only variants that
 *                compile without register spills): sbi_plan_variants().
 *   row_rows     rows of the grid per row-pass workgroup (a power of two; 0:
 *                as many as fill 256 threads, the default).
 *   col_split    workgroups a column pass should reach by splitting its
 *                products over workgroups along y (0: no split, the default;
 *                only 2D grids split).
 *   us           time of the tuned unit under this plan in microseconds (one
 *                sweep in iteration mode, one W solve in SA mode), 0 when the
 *                plan was set rather than measured.
 *   cached       1 when sbi_autotune took the plan from the plan cache.
 */
typedef struct sbi_plan {
    int32_t row_variant;
    int32_t row_rows;
    int32_t col_split;
    float us;
    int32_t cached;
} sbi_plan;

/* Bit v of the result is set when row variant v is built for the context's
   precision, mode and row length. */
int32_t sbi_plan_variants(const sbi_ctx* ctx);

sbi_status sbi_plan_get(const sbi_ctx* ctx, sbi_plan* out);

/* Use the given plan from the next call on.  Errors (plan unchanged):
   SBI_ERR_UNSUPPORTED for a variant not built here; SBI_ERR_INVALID_ARG for
   row_rows that is negative or not a power of two, or a negative col_split. */
sbi_status sbi_plan_set(sbi_ctx* ctx, const sbi_plan* plan);

/*
 * Autotuner: times every built row variant, rows per workgroup from the
 * launch bound down to a quarter of it, and column splits {0, 1024, 2048,
 * 4096} (2D grids), each on the context's own kernels and workspace (5 units
 * after 2 of warm-up, best of two rounds, HIP events on the context's
 * stream), and keeps the fastest.  The plan cache, a process-wide table keyed
 * by device (name and architecture), grid size, batch, precision, mode,
 * acceleration, order and whether the bed varies, is consulted first: a hit
 * is applied without timing unless flags has SBI_TUNE_FORCE, and every search
 * stores its result there.  Running the kernels overwrites the iteration's
 * carried state: the previous-solve seed and the history layer's history are
 * emptied, as after sbi_set_depth.  Synchronises the stream.  out may be NULL.
 */
enum { SBI_TUNE_FORCE = 1 };
sbi_status sbi_autotune(sbi_ctx* ctx, int32_t flags, sbi_plan* out);

/*
 * The plan cache as a text file: a header line, then one line per entry
 * "<key> <row_variant> <row_rows> <col_split> <us>" (the key has no spaces).
 * Load merges a file into the table (entries of the file win; lines that do
 * not parse are skipped; a missing file is SBI_ERR_INVALID_ARG); save writes
 * the whole table.  Both are host-only and take no context; they return the
 * number of entries read or written through *count when count is not NULL.
 */
sbi_status sbi_tune_cache_load(const char* path, int32_t* count);
sbi_status sbi_tune_cache_save(const char* path, int32_t* count);

#ifdef __cplusplus
}
#endif
#endif /* SBI_H */
