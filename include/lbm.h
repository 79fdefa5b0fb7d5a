/*
 * liblbm -- C ABI of the MI355X (gfx950) implementation of the compressible
 * two-dimensional 16-velocity multiple-relaxation-time finite-difference
 * lattice Boltzmann model with the energy-flux collision modification
 * (Chen, Xu, Zhang, Li: "Prandtl number effects in MRT lattice Boltzmann
 * models for shocked and unshocked compressible fluids").
 *
 * Conventions shared by every entry point
 *   - Units are the paper's non-dimensional ones with R = 1 (Sec. IV): the
 *     velocities are cyc(+-1,0), (+-1,+-1), cyc(+-2,0), (+-2,+-2) (Sec. II,
 *     Fig. 1), the gas has e = rho (T + u^2/2) and p = rho T.
 *   - Distributions are FP64, 16 planes in the paper's velocity order.
 *     Dense field arrays passed in or out are row-major [ny][nx] (x fastest);
 *     dense distribution arrays are [16][ny][nx].
 *   - Every pointer named d_* is device memory on the device that was
 *     current when the handle was created; the caller owns it, the library
 *     never frees caller memory.
 *   - Every call only enqueues work on the handle's HIP stream (asynchronous
 *     with respect to the host) unless its comment says it synchronises.
 *   - Errors are returned as lbm_status; lbm_last_error() then holds a
 *     message for the calling thread. No call aborts or throws.
 */
#ifndef LBM_H_
#define LBM_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  LBM_OK = 0,
  LBM_EINVAL = -1,      /* invalid argument (message says which) */
  LBM_ENOMEM = -2,      /* workspace too small */
  LBM_EHIP = -3,        /* a HIP runtime call failed */
  LBM_ESTATE = -4,      /* call not valid in the handle's current state */
  LBM_ENONFINITE = -5,  /* the device health flag saw rho <= 0, T <= 0 or NaN */
  LBM_ETIMEOUT = -6     /* a bounded device-side wait gave up (lbm_batch.h); the state is invalid */
} lbm_status;

/* Boundary kind of one side of the domain. */
typedef enum {
  LBM_BC_PERIODIC = 0,      /* wrap; both sides of the axis must be periodic */
  LBM_BC_ZERO_GRADIENT = 1, /* ghost = boundary node (extrapolation outflow, Sec. IV.B(b)) */
  LBM_BC_SPECULAR = 2,      /* ghost = boundary node with the normal velocity
                               component negated (reflecting wall, Sec. IV.B(b)) */
  LBM_BC_NEQ_WALL = 3,      /* non-equilibrium extrapolation wall on the first/last
                               node of the axis (Sec. IV.A); uses wall[side] = (-, ux, uy, T) */
  LBM_BC_DIRICHLET_EQ = 4   /* ghost = equilibrium of the fixed state wall[side] =
                               (rho, ux, uy, T) (fixed inflow, Sec. IV.B(b)) */
} lbm_bc;

/* Sides, in the order of lbm_params.bc and lbm_params.wall. */
enum { LBM_SIDE_XLO = 0, LBM_SIDE_XHI = 1, LBM_SIDE_YLO = 2, LBM_SIDE_YHI = 3 };

/* Problem description (Sec. II-IV).
 *   nx, ny      nodes; an axis of extent 1 must be periodic (exact 1-D problem)
 *   dx, dy, dt  grid spacings and time step (> 0)
 *   s[16]       relaxation rates s_1..s_16 of the diagonal S^ (Sec. II, Eq. 3);
 *               s_1..s_4 act on conserved moments and have no effect
 *   eq_version  free equilibrium moments 12, 15, 16 (Sec. II): 1 zeros,
 *               2 the printed polynomials, 3 moments of the sampled Maxwellian
 *   modified    0: unmodified collision; 1: energy-flux modification with the
 *               Q_8 normal-stress term u_y (d_y u_y - d_x u_x), for which the
 *               recovered energy equation is Eq. (5); 2: the same modification
 *               with that term's sign exactly as printed (Sec. II)
 *   bc[4]       lbm_bc per side (x_lo, x_hi, y_lo, y_hi); NEQ walls may be on
 *               one axis only and that axis needs >= 3 nodes
 *   wall[4][4]  per side (rho, ux, uy, T), used by NEQ_WALL and DIRICHLET_EQ
 *   scheme      convection: 0 the central Lax-Wendroff update (Sec. III, the
 *               paper's scheme, default); 1 the same update with a minmod
 *               limiter on its anti-diffusive flux (total variation
 *               diminishing, radius 2, two ghost layers: the second
 *               zero-gradient layer repeats the boundary node, the second
 *               mirror layer mirrors the node next to it). Scheme 1 takes
 *               sharp discontinuities without smoothing; it is not available
 *               with NEQ walls or in the adjoint form. */
typedef struct {
  int32_t nx, ny;
  double dx, dy, dt;
  double s[16];
  int32_t eq_version;
  int32_t modified;
  int32_t bc[4];
  double wall[4][4];
  int32_t scheme;
} lbm_params;

typedef struct lbm_handle lbm_handle;

/* Bytes of device workspace lbm_create needs for p: two pitched
 * distribution buffers [16][ny][pitch] (pitch = nx rounded up to 64 doubles)
 * and a small status block, 256-byte aligned. 0 if p is invalid. */
size_t lbm_workspace_bytes(const lbm_params* p);

/* Validates p and binds a handle to caller-owned workspace d_workspace
 * (>= lbm_workspace_bytes(p) bytes, 256-byte aligned) and to hip_stream
 * (a hipStream_t, or NULL for the null stream). Rejects with LBM_EINVAL:
 * nx or ny < 1, dx, dy or dt <= 0, s_k <= 0 for k >= 5, max_k s_k dt > 2
 * (explicit relaxation unstable), unpaired periodic sides, NEQ walls on both
 * axes or on an axis with < 3 nodes, eq_version not in {1,2,3}, modified not
 * in {0,1,2}, scheme not in {0,1} or scheme 1 with NEQ walls; LBM_ENOMEM if
 * ws_bytes is too small. The handle owns only host metadata. */
lbm_status lbm_create(const lbm_params* p, void* d_workspace, size_t ws_bytes, void* hip_stream,
                      lbm_handle** out);

/* Initial state f = M^-1 f^eq(rho, u, T) at every node (Sec. II equilibria,
 * Eqs. 14a-14i, with the handle's eq_version). Inputs are device [ny][nx]. */
lbm_status lbm_init(lbm_handle* h, const double* d_rho, const double* d_ux, const double* d_uy,
                    const double* d_T);

/* Advance nsteps >= 0 time steps of Eq. (3): per node, moments f^ = M f,
 * Q_k = s_k (f^_k - f^eq_k) plus the energy-flux modification of Q_7, Q_8
 * (Sec. II), collision -dt M^-1 Q, and per-axis central Lax-Wendroff
 * convection with forward-Euler time stepping (the scheme whose amplification
 * matrix is G_ij, Sec. III; with scheme 1 its minmod flux-limited form).
 * Velocity gradients in the modification are central differences of nodal
 * velocities at the old time level. */
lbm_status lbm_step(lbm_handle* h, int64_t nsteps);

/* rho, u_x, u_y, T = e/rho - u^2/2 and p = rho T of the current state
 * (Sec. II, conserved moments; R = 1). Device [ny][nx]; any may be NULL. */
lbm_status lbm_moments(lbm_handle* h, double* d_rho, double* d_ux, double* d_uy, double* d_T, double* d_p);

/* Copy the current distributions to / from a dense device array [16][ny][nx]
 * (checkpoint and restore: f and the parameters determine the state). */
lbm_status lbm_get_f(lbm_handle* h, double* d_f);
lbm_status lbm_set_f(lbm_handle* h, const double* d_f);

/* Synchronises the stream and reads the device health flag: LBM_OK, or
 * LBM_ENONFINITE if any step since the last check produced rho <= 0,
 * T <= 0 or a NaN; the flag is then cleared. */
lbm_status lbm_check(lbm_handle* h);

/* Kernel variant used by lbm_step:
 *   0 the fused LDS-staged kernel, one launch per step (default for grids of
 *     more than 512 nodes and more than 16 rows, and for scheme 1);
 *   1 the plain one-thread-per-node global-memory kernel (a reference for
 *     race and indexing checks);
 *   2 the small-grid kernel (default when nx ny <= 512 and scheme 0;
 *     LBM_EINVAL otherwise): one workgroup holds the whole grid in LDS and
 *     takes up to 65536 steps per launch;
 *   3 the windowed kernel (scheme 0 and nx ny > 512, LBM_EINVAL otherwise;
 *     default when ny <= 16): workgroups hold overlapping windows of the grid
 *     in LDS (lbm_set_window) and take several steps per launch,
 *     recomputing the overlap;
 *   4 the fused kernel taking two time steps per launch (scheme 0 without
 *     NEQ walls, LBM_EINVAL otherwise; default when the two distribution
 *     buffers take more than 512 MB): the intermediate level stays in LDS,
 *     so each node's distributions cross HBM once per two steps; an odd
 *     last step of a call takes variant 0.
 * Variants 2 and 3 take many steps per launch, so small and narrow grids are
 * not bound by launch cost. All variants give the same results to rounding.
 * lbm_set_tile sets the tile shape of the current variant (0, or 4 for the
 * two-step kernel, whose shape is kept separately): rows per workgroup tile
 * (1..1024, rounded up to a multiple of waves) and wavefronts per workgroup
 * (2 or 4; variant 0 with NEQ walls or scheme 1 always uses 4).
 * Results do not depend on the tile shape. */
lbm_status lbm_set_variant(lbm_handle* h, int32_t variant);
lbm_status lbm_get_variant(const lbm_handle* h, int32_t* variant);
lbm_status lbm_set_tile(lbm_handle* h, int32_t rows, int32_t waves);

/* Stores of the fused kernel (variant 0): nontemporal = 1 marks the new
 * distributions as not to be kept in the caches, 0 uses ordinary stores
 * (better while both distribution buffers fit in the caches, so the next
 * step reads them back from there). Default: 0 when the two buffers take
 * between 32 and 512 MB, else 1; lbm_tune times both. Results do not
 * depend on it. */
lbm_status lbm_set_store_mode(lbm_handle* h, int32_t nontemporal);
lbm_status lbm_get_store_mode(const lbm_handle* h, int32_t* nontemporal);

/* Window shape of variant 3: cols x rows nodes held per workgroup (at most
 * 512), steps = most time steps per launch. An axis no longer than the
 * window is held whole; a longer one is cut into windows that overlap by
 * `steps` nodes on each cut side, each writing its middle (extent - 2 steps)
 * nodes, so cut extents must exceed 2 steps. Default: grids of <= 16 rows
 * take every row and 64 columns (32 when ny > 8) with steps = columns / 8;
 * other grids 32 x 16 with 2 steps. Results do not depend on the shape
 * beyond rounding. */
lbm_status lbm_set_window(lbm_handle* h, int32_t cols, int32_t rows, int32_t steps);
lbm_status lbm_get_window(const lbm_handle* h, int32_t* cols, int32_t* rows, int32_t* steps);

/* Tuner: times probe_steps steps for each candidate fused tile shape
 * (wavefronts per workgroup x tile height x store mode) and keeps the
 * fastest. When the handle uses variant 0, 3 or 4, it also times the
 * two-step kernel's tile shapes where that kernel applies (over probe_steps
 * rounded up to even) and window shapes where the windowed kernel applies
 * (every row for grids of <= 16 rows, two-dimensional windows otherwise),
 * and then uses whichever kernel and shape was fastest (lbm_get_variant,
 * lbm_get_tile, lbm_get_window). Variants 1 and 2 are kept. Synchronises
 * the stream. rows_out, waves_out: the tile shape of the kernel kept (the
 * fused kernel's if the windowed one won); best_ms: the best
 * time of probe_steps steps over all candidates (each may be NULL). With
 * d_scratch (device, >= 16 ny pitch doubles) the state is saved and
 * restored; with NULL the state advances. */
lbm_status lbm_tune(lbm_handle* h, int64_t probe_steps, double* d_scratch, size_t scratch_bytes, int32_t* rows_out,
                    int32_t* waves_out, double* best_ms);
/* Current tile shape of variant 0, or of variant 4 while the handle uses it
 * (either pointer may be NULL). */
lbm_status lbm_get_tile(const lbm_handle* h, int32_t* rows, int32_t* waves);

/* Diagnostic, not part of the method: copies the 16 pitched planes of an
 * nx-by-ny field laid out like the distributions ([16][ny][pitch], pitch = nx
 * rounded up to 64 doubles, padding included) from d_src to d_dst on
 * hip_stream, with the step kernel's HBM access pattern and no arithmetic.
 * Its bandwidth is the ceiling for a kernel with that access pattern.
 * Both buffers hold 16 ny pitch doubles and must not overlap. */
lbm_status lbm_stream_copy(const double* d_src, double* d_dst, int32_t nx, int32_t ny, void* hip_stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * time stepping as lbm_create + lbm_set_f + lbm_step(nsteps) + lbm_get_f,
 * with the kernel and tile shape lbm_create picks by default, but with no
 * workspace argument and no allocation of any kind. The two pitched
 * distribution buffers, the coefficients and the health flag live in one
 * fixed device array of the library (64 MiB + 64.25 KiB, held on every device
 * the call runs on until the process ends), so the grid may take at most
 * LBM_NOALLOC_MAX_NODES stored nodes, counting rows padded to a multiple of
 * 64 (e.g. 1024 x 256); larger grids are rejected with LBM_EINVAL before
 * anything is enqueued.
 *   d_f_in   device [16][ny][nx] distributions of the initial state (read)
 *   d_f_out  device [16][ny][nx], the state after nsteps >= 0 steps (may be
 *            d_f_in: the input is copied into the array before any step)
 *   d_status device int32 or NULL: receives LBM_OK, or LBM_ENONFINITE if a
 *            step produced rho <= 0, T <= 0 or NaN
 * Enqueued on hip_stream; nothing is synchronised. Every call on one device
 * shares that device's array and overwrites it (the coefficients and the
 * flag are rewritten by each call), so calls whose work overlaps on one
 * device - other streams, other host threads - race and must be serialised
 * by the caller. Same validation as lbm_create. */
#define LBM_NOALLOC_MAX_NODES 262144
lbm_status lbm_run_noalloc(const lbm_params* p, const double* d_f_in, double* d_f_out, int64_t nsteps,
                           int32_t* d_status, void* hip_stream);

/* Message of the last failed call on this thread ("" if none). */
const char* lbm_last_error(void);

/* Releases the handle (NULL-safe); does not touch the workspace. */
void lbm_destroy(lbm_handle* h);

#ifdef __cplusplus
}
#endif

#endif /* LBM_H_ */
