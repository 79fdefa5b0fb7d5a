/*
 * liblbm batched form: many independent problems of uneven size and
 * parameters advanced together (Riemann lines along x with ny = 1, thermal
 * Couette columns along y with nx = 1, and two-dimensional problems such as
 * the shock/interface and shock-bubble set-ups; Sec. IV of the paper for the
 * problems, Sec. II-III for the step). Conventions as in lbm.h.
 *
 * Layout: instance i owns nodes [lbm_batch_offset(b, i), lbm_batch_offset(b,
 * i + 1)) of every concatenated field array (its own [ny][nx] order), and
 * 16 * (its node count) entries of a concatenated distribution array
 * ([16][ny][nx] per instance, instances back to back).
 *
 * Execution: one-dimensional Lax-Wendroff instances ("lines"; a periodic one
 * only up to 128 nodes) are cut into chunks; a workgroup owns one chunk plus a halo of
 * h nodes, advances it h steps in LDS and writes the chunk back, so K steps
 * are ceil(K/h) launches over every chunk. The other instances ("tiled") are
 * cut into 64-column tiles of a common height and take one launch per step
 * and per (equilibrium version, variant: plain, NEQ walls, flux-limited)
 * group, every tile of every such instance in the same launch; in two-step mode
 * (lbm_batch_set_two_step) the plain ones (Lax-Wendroff, no NEQ walls) take two steps per launch
 * through the two-step kernel of lbm_set_variant(4). In the persistent form
 * (lbm_batch_set_persistent) the line instances of one equilibrium version take ONE launch for
 * all ceil(K/h) blocks: as many workgroups as are resident at once take (block, chunk) tickets in
 * order, and a chunk starts a block once the chunks whose nodes lie within h of its own have
 * finished the block before (bounded waits on per-chunk epochs, no grid-wide barrier). One call
 * of lbm_batch_step(b, K) is
 * captured once in a hipGraph and replayed on later calls with the same K.
 * Results equal those of lbm_step on each instance alone: with the fused kernel (variant 0)
 * bitwise for tiled instances (in two-step mode the plain ones with variant 4, bitwise), within
 * rounding (the same arithmetic, multiply-adds contracted differently) for lines.
 */
#ifndef LBM_BATCH_H_
#define LBM_BATCH_H_

#include "lbm.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct lbm_batch lbm_batch;

/* Device workspace for n instances (two arenas, a backup arena used by the
 * tuner, descriptors, chunk and tile lists, budgets, status); 0 if n < 1 or
 * any instance is invalid (lbm_create's rules). Instances with the
 * flux-limited scheme (scheme 1) are advanced tile by tile, whatever their
 * shape. */
size_t lbm_batch_workspace_bytes(const lbm_params* inst, int32_t n);

/* Binds a batch to caller-owned workspace and stream (as lbm_create). */
lbm_status lbm_batch_create(const lbm_params* inst, int32_t n, void* d_workspace, size_t ws_bytes, void* hip_stream,
                            lbm_batch** out);

/* First node of instance i in concatenated field arrays; i == n gives the
 * total node count; -1 if out of range. */
int64_t lbm_batch_offset(const lbm_batch* b, int32_t i);

/* f = M^-1 f^eq(rho, u, T) for every instance (Sec. II, Eqs. 14a-14i);
 * concatenated device field arrays. */
lbm_status lbm_batch_init(lbm_batch* b, const double* d_rho, const double* d_ux, const double* d_uy,
                          const double* d_T);

/* Optional per-instance step budgets (host array of n, NULL = no limit):
 * during one lbm_batch_step(b, K) instance i advances min(K, steps[i]) steps. */
lbm_status lbm_batch_set_budgets(lbm_batch* b, const int64_t* steps);

/* Advances every instance nsteps time steps (Eq. 3, scheme of Sec. III). */
lbm_status lbm_batch_step(lbm_batch* b, int64_t nsteps);

/* rho, u_x, u_y, T, p of every instance, concatenated (any may be NULL). */
lbm_status lbm_batch_moments(lbm_batch* b, double* d_rho, double* d_ux, double* d_uy, double* d_T, double* d_p);

/* Current distributions, [16][ny][nx] per instance, concatenated. */
lbm_status lbm_batch_get_f(lbm_batch* b, double* d_f);

/* Schedule of the line instances: region = nodes per workgroup (128 or
 * 256), steps_per_launch = h (region - 2 h >= 32); use_graph = capture
 * lbm_batch_step in a hipGraph (all instances). nchunks counts line chunks. */
lbm_status lbm_batch_set_schedule(lbm_batch* b, int32_t region, int32_t steps_per_launch, int32_t use_graph);
lbm_status lbm_batch_get_schedule(const lbm_batch* b, int32_t* region, int32_t* steps_per_launch, int32_t* nchunks);

/* Launch form of the line instances: persistent = 1, one launch per equilibrium version for the
 * whole of an lbm_batch_step call (grid = min(chunks, workgroups resident on the device), chunks
 * taken in ticket order, each waiting for its neighbours' previous block); 0, one launch per
 * block (the form at creation). Results are bitwise the same. timeout_ms in [0, 60000] bounds each
 * wait (wall clock; 0: the first dependency check of a call with two or more blocks raises the
 * error, for tests of the error path): a wait that runs out
 * raises a device error word, every workgroup leaves, and lbm_batch_check then returns
 * LBM_ETIMEOUT (the state is invalid; re-initialise). Overlapping calls on one batch race.
 * grid (get): workgroups of the largest persistent launch of the current schedule. */
lbm_status lbm_batch_set_persistent(lbm_batch* b, int32_t persistent, double timeout_ms);
lbm_status lbm_batch_get_persistent(lbm_batch* b, int32_t* persistent, int32_t* grid);

/* Tile height of the tiled instances (rows per tile, a multiple of 4 in
 * [4, 4096]; an instance shorter than that is one tile high). Results do not
 * depend on it. ntiles = tiles per step over all tiled instances. */
lbm_status lbm_batch_set_tile_rows(lbm_batch* b, int32_t rows);
lbm_status lbm_batch_get_tile_rows(const lbm_batch* b, int32_t* rows, int32_t* ntiles);

/* Two-step mode of the plain tiled instances: on = 1, two steps per launch with `rows` output
 * rows per two-step tile (even, in [2, 4096]; results do not depend on it); 0, one step per
 * launch (the mode at creation). Can change between calls. ntiles = two-step tiles. */
lbm_status lbm_batch_set_two_step(lbm_batch* b, int32_t on, int32_t rows);
lbm_status lbm_batch_get_two_step(const lbm_batch* b, int32_t* on, int32_t* rows, int32_t* ntiles);

/* Autotuner: times every admissible (region, h), each in both launch forms, for probe_steps
 * steps of the line instances, then tile heights 8 ... 128 (one step per launch) and, with
 * plain tiled instances, two-step tile heights 8 ... 128 for probe_steps steps of the tiled
 * instances, on the current state (synchronising the stream); restores the state and keeps
 * the fastest of each; *best_ms receives the sum of the two best times. An error left by earlier
 * calls (what lbm_batch_check would return) is returned first, and nothing is tuned. */
lbm_status lbm_batch_tune(lbm_batch* b, int64_t probe_steps, double* best_ms);

/* As lbm_check, for the batch; LBM_ETIMEOUT (checked first, then cleared) if a persistent
 * launch's wait timed out since the last check. */
lbm_status lbm_batch_check(lbm_batch* b);

void lbm_batch_destroy(lbm_batch* b);

#ifdef __cplusplus
}
#endif

#endif /* LBM_BATCH_H_ */
