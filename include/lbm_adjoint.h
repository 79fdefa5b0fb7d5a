/*
 * liblbm adjoint form: gradients of a scalar function of the final fields
 * with respect to the relaxation rates s_1..s_16 and the initial fields
 * (rho, u_x, u_y, T), through nsteps time steps of the MRT FD-LBM update
 * (Eq. 3 with the scheme of Sec. III and the energy-flux modification of
 * Sec. II; the step's Jacobian is the matrix G_ij of Sec. III in Fourier
 * space). Conventions as in lbm.h.
 *
 * Memory: the forward sweep keeps a checkpoint every ckpt_interval steps;
 * the reverse sweep recomputes each segment from its checkpoint into a
 * segment store and runs the hand-written adjoint step backwards through it
 * (about sqrt(nsteps) states each). Supported boundaries: periodic,
 * zero-gradient, specular, fixed-state ghosts and non-equilibrium
 * extrapolation walls (Sec. IV.A; their transpose is applied before each
 * adjoint step); equilibrium versions 1-3; modified 0-2; scheme 0 only.
 */
#ifndef LBM_ADJOINT_H_
#define LBM_ADJOINT_H_

#include "lbm.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct lbm_adjoint lbm_adjoint;

/* Device workspace for p, nsteps and a checkpoint interval (0 = round(sqrt(nsteps))):
 * checkpoints, segment store, two adjoint buffers, two per-node record buffers, the
 * s-gradient partials and constants; 0 if invalid (lbm_create's rules, or scheme 1). */
size_t lbm_adjoint_workspace_bytes(const lbm_params* p, int64_t nsteps, int32_t ckpt_interval);

lbm_status lbm_adjoint_create(const lbm_params* p, int64_t nsteps, int32_t ckpt_interval, void* d_workspace,
                              size_t ws_bytes, void* hip_stream, lbm_adjoint** out);

/* Forward sweep: f^0 = M^-1 f^eq(rho0, u0, T0), then nsteps steps, keeping
 * checkpoints. Inputs are device [ny][nx]. */
lbm_status lbm_adjoint_forward(lbm_adjoint* a, const double* d_rho0, const double* d_ux0, const double* d_uy0,
                               const double* d_T0);

/* Fields of the final state (after lbm_adjoint_forward); any may be NULL. */
lbm_status lbm_adjoint_final_moments(lbm_adjoint* a, double* d_rho, double* d_ux, double* d_uy, double* d_T,
                                     double* d_p);

/* Reverse sweep. Inputs: the same initial fields as the forward call and
 * dL/d(final rho, u_x, u_y, T) (device [ny][nx], NULL = zero). Outputs:
 * dL/d(initial rho, u_x, u_y, T) (device [ny][nx], NULL = not wanted) and
 * dL/ds_1..s_16 (device, 16 doubles; entries 1-4 are 0). The s-gradient sum
 * is taken in a fixed order (deterministic). */
lbm_status lbm_adjoint_backward(lbm_adjoint* a, const double* d_rho0, const double* d_ux0, const double* d_uy0,
                                const double* d_T0, const double* d_g_rho, const double* d_g_ux,
                                const double* d_g_uy, const double* d_g_T, double* d_grad_rho0,
                                double* d_grad_ux0, double* d_grad_uy0, double* d_grad_T0, double* d_grad_s);

/* Kernel of the adjoint step: 0 the LDS-staged form (64-column tiles
 * marching up the grid, lambda^{n+1} and the records entering an LDS ring
 * once, ghost rules applied on entry; the default on large grids); 1 one
 * thread per node gathering its neighbours' lambda and records from global
 * memory (the default on small grids, where every tile would be a few rows
 * tall). Both give the same results to rounding. */
lbm_status lbm_adjoint_set_variant(lbm_adjoint* a, int32_t variant);

/* Synchronises the stream and reads the device health flag of every step
 * the forward and reverse sweeps ran since the last check (the checkpointed
 * forward steps and the recomputed segments): LBM_OK, or LBM_ENONFINITE if
 * one of them produced rho <= 0, T <= 0 or a NaN (the gradients of such a
 * trajectory are meaningless); the flag is then cleared. */
lbm_status lbm_adjoint_check(lbm_adjoint* a);

void lbm_adjoint_destroy(lbm_adjoint* a);

#ifdef __cplusplus
}
#endif

#endif /* LBM_ADJOINT_H_ */
