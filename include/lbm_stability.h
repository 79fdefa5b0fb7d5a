/*
 * liblbm stability tool: von Neumann analysis of the step (Sec. III of the
 * paper, Fig. 2). Conventions as in lbm.h.
 *
 * About a uniform state (rho, u_x, u_y, T), one linearised time step maps a
 * Fourier mode f_i e^{i (theta_x x / dx + theta_y y / dy)} to G(theta) times
 * itself. G is the paper's coefficient matrix G_ij (Sec. III): the per-axis
 * Lax-Wendroff convection symbol
 *   1 - i c sin(theta) + c^2 (cos(theta) - 1),  c = v_i,alpha dt / dx_alpha,
 * on the diagonal, the collision term -dt M^-1 S (M - d f^eq / d f) with the
 * equilibrium moments differentiated through (rho, u, T), and, when
 * `modified` is 1 or 2, the derivative of the extra Q_7 and Q_8 terms of the
 * energy-flux modification (Sec. II), whose velocity gradients (central
 * differences, as in the step) have the symbol i sin(theta) / dx_alpha.
 * |omega|_max(theta) is the largest eigenvalue modulus of G (Fig. 2); the
 * step is von Neumann stable at theta when it is <= 1.
 *
 * Parameter sets are lbm_params: only dx, dy, dt, s, eq_version and modified
 * are used (nx, ny, bc and wall are ignored); scheme must be 0 (the
 * flux-limited scheme is not linear). The relaxation-stability bound of
 * lbm_create (max s_k dt <= 2) is not applied, so unstable parameters can be
 * analysed.
 *
 * The library works with G in the moment basis, M G M^-1 (M as in Sec. II),
 * which has the same eigenvalues; lbm_stability_matrix returns that form.
 */
#ifndef LBM_STABILITY_H_
#define LBM_STABILITY_H_

#include "lbm.h"

#ifdef __cplusplus
extern "C" {
#endif

/* Base state of the linearisation. */
typedef struct {
  double rho, ux, uy, T;
} lbm_state;

/* Device workspace for nsets parameter sets (their coefficient blocks,
 * about 10 KB each); 0 if nsets < 1. */
size_t lbm_stability_workspace_bytes(int32_t nsets);

/* G(theta) in the moment basis for every (set s, point t):
 *   sets, states   host arrays of nsets (parameters; base states, rho > 0, T > 0);
 *   d_theta        device [npts][2] FP64, (theta_x, theta_y) = (k_x dx, k_y dy);
 *   d_G            device [nsets][npts][2][16][16] FP64: real part, then
 *                  imaginary part, row-major, row k = moment k + 1.
 * Enqueued on hip_stream; the host arrays may be reused when the call returns
 * (the call waits for their upload). LBM_EINVAL on a bad set or size,
 * LBM_ENOMEM if ws_bytes is too small. */
lbm_status lbm_stability_matrix(const lbm_params* sets, const lbm_state* states, int32_t nsets,
                                const double* d_theta, int32_t npts, void* d_workspace, size_t ws_bytes,
                                double* d_G, void* hip_stream);

/* |omega|_max for every (set s, point t) into d_radius [nsets][npts] (device,
 * FP64). Computed from Gelfand's formula, rho(G) = lim ||G^N||^(1/N), with
 * N = 2^squarings (1 <= squarings <= 60; 0 selects 48): G is squared
 * `squarings` times on the FP64 matrix cores, rescaled by a power of two
 * after each product (exact), and the exponents are summed. Arguments as in
 * lbm_stability_matrix. */
lbm_status lbm_stability_radius(const lbm_params* sets, const lbm_state* states, int32_t nsets,
                                const double* d_theta, int32_t npts, int32_t squarings, void* d_workspace,
                                size_t ws_bytes, double* d_radius, void* hip_stream);

#ifdef __cplusplus
}
#endif

#endif /* LBM_STABILITY_H_ */
