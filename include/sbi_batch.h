/*
 * sbi_batch.h -- ensembles of independent sea states of uneven grid sizes,
 * stepped together.
 *
 * Every member is an independent problem of sbi.h (its own grid, depth and
 * state); nothing couples members.  Members with identical grids are grouped
 * into one context whose kernels carry the members along their batch
 * dimension; the groups run concurrently on streams forked from the caller's
 * stream.  With SBI_BATCH_GRAPH a step call runs as captured HIP graphs: a
 * prologue (states in, to spectral space), the steps in parts of at most 4
 * (short graphs replay faster per step than one long graph), and an epilogue
 * (back to physical space, states out); the spectral states stay in the
 * workspace between parts, so the result does not depend on the split.  Each
 * part is captured once and replayed by later calls with the same (dt, n,
 * tol, state pointers, seeds and sweep budgets); up to 8 instantiated graphs
 * are kept, least recently used first out.  With SBI_BATCH_AUTOTUNE each
 * group's launch plan (row-transform radix and twiddle mode, rows per row
 * workgroup, column-pass product split; sbi.h, sbi_plan) is chosen at init:
 * one group is tuned like a context (sbi_autotune); with several, each
 * group's candidates are timed while every group runs its unit of work
 * concurrently (group by group, from the default plans), since the fastest
 * plan of a group alone need not be the fastest beside the others.  The
 * process's plan cache is consulted first (sbi_tune_cache_load / _save
 * persist it; an ensemble's entries are keyed by all its groups).
 *
 * Iterations run without host polling: each solve enqueues the sweep
 * launches of a budget B and a member's launches after the pass that decides
 * its solve return at once; sweep statistics are accumulated on the device.
 * The first call of a group uses B = max_sweeps; later calls use the largest
 * sweep count of the previous call plus a margin of 3 (changed only when it
 * moves by more than the margin, each change being a new capture).  When a
 * solve outruns B the device statistics show it undecided, and the call is
 * redone from a device copy of its inputs and of the carried seeds with B
 * doubled, until every solve is decided, so results equal those of the full
 * max_sweeps budget while the launches scale with the sweeps the solves need.
 * A learned seed (SBI_SEED_NET) that fails is reported, not redone.
 *
 * Nothing a batch step computes depends on the state time t (each member's
 * t is only advanced by n*dt): time-dependent forcing -- the wave tank's
 * pressures and relaxation zones of sbi.h -- is not available to ensembles,
 * which is what lets a captured graph be replayed at any later time.
 *
 * Conventions are those of sbi.h.
 */
#ifndef SBI_BATCH_H
#define SBI_BATCH_H

#include "sbi.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct sbi_batch sbi_batch;

enum { SBI_BATCH_GRAPH = 1, SBI_BATCH_AUTOTUNE = 2 };

/* Device workspace bytes for m members with grids[m]; 0 if a grid is invalid. */
size_t sbi_batch_workspace_bytes(int32_t m, const sbi_grid* grids);

/*
 * m members: grids[m], depths[m] (host [ny][nx] arrays, depth > 0), one
 * reference depth rule h_ref for all (<= 0: each member's max depth).
 * workspace: caller-owned device memory of sbi_batch_workspace_bytes bytes.
 * flags: SBI_BATCH_GRAPH | SBI_BATCH_AUTOTUNE.
 * Returns SBI_WARN_DEPTH_CRITERION when any member exceeds the Sec. 5 limit,
 * and SBI_ERR_UNSUPPORTED for a member in mode SBI_MODE_FULL or precision
 * SBI_MIXED (both decide their solves on the host between passes).
 */
sbi_status sbi_batch_init(sbi_batch** out, int32_t m, const sbi_grid* grids, const double* const* depths,
                          double h_ref, void* workspace, size_t ws_bytes, void* hip_stream, int32_t flags);

/*
 * Advance every member by n steps of dt.  states[m]: each member's device
 * eta / phi_s arrays [ny][nx] (its grid's precision), updated in place, and
 * its time t (advanced by n dt).  info: host [m] per-member statistics, or
 * NULL.  Returns the worst member status (errors < 0 take precedence).
 */
sbi_status sbi_batch_step(sbi_batch* b, sbi_state* states, double dt, int32_t n, double tol, sbi_step_info* info);

/* Load the learned warm start (sbi_net.h blob) into every group whose seed is
   SBI_SEED_NET; SBI_ERR_INVALID_ARG if the blob is rejected. */
sbi_status sbi_batch_net_load(sbi_batch* b, const void* weights, size_t bytes);

/* Load the learned history layer (sbi_net_hist_load) into every group whose
   seed is SBI_SEED_NET. */
sbi_status sbi_batch_net_hist_load(sbi_batch* b, int32_t taps, int32_t bins, double dk, const float* w);

/* Number of member groups and, per group (g < groups), its member count and
   the column-pass split of its plan (0: none). */
int32_t sbi_batch_groups(const sbi_batch* b, int32_t* members_out, int32_t* split_out, int32_t n);

/* Launch plan of group g (sbi.h, sbi_plan; us and cached are 0). */
sbi_status sbi_batch_plan(const sbi_batch* b, int32_t g, sbi_plan* out);

/* Current sweep budget of each group (host int32 [n]; max_sweeps when none is
   set); returns the number of step calls redone with a larger budget since
   init. */
int32_t sbi_batch_budgets(const sbi_batch* b, int32_t* budget_out, int32_t n);

sbi_status sbi_batch_destroy(sbi_batch* b);

#ifdef __cplusplus
}
#endif

#endif /* SBI_BATCH_H */
