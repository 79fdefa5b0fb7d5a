// Von Neumann stability tool (declarations and contracts in
// include/lbm_stability.h): the amplification matrix G(theta) of the step
// (Sec. III) in the moment basis and its spectral radius |omega|_max.
//
// In the moment basis M G M^-1 the matrix is
//   P0 + (cos tx - 1) Bx + (cos ty - 1) By + i (sin tx Qx + sin ty Qy)
// with, per parameter set,
//   P0 = I - dt S (I - D)        D = d f^eq / d f^ (non-zero in columns 1..4)
//   Bx = M diag(c_x^2) M^-1      c_x,i = v_x,i dt / dx   (likewise By)
//   Qx = -M diag(c_x) M^-1 - (dt / dx) (e_7 a_7^T + e_8 a_8^T)
// where a_7, a_8 (and b_7, b_8 for Qy) are the derivatives of the extra Q_7,
// Q_8 terms (Sec. II) with respect to the moments, per unit of the gradient
// symbol i sin(theta) / dx. k_stab_setup builds these five real 16 x 16
// matrices once per set; the point kernels combine them per wavenumber.
//
// Spectral radius: repeated squaring on the FP64 matrix cores. One wavefront
// per point holds X (16 x 16 complex) in the MFMA accumulator layout, stages
// it through LDS into the operand layouts, and forms X^2 with sixteen
// 16x16x4 FP64 MFMAs (four real products per 4-wide slice of the inner
// dimension); after every product X is rescaled by a power of two and the
// exponents are summed with weights 2^-j (Gelfand's formula). The moment
// basis keeps the powers far closer to normal than the velocity basis, so
// the rounding of the products perturbs the radius no more than the
// rounding of G's own entries does.
#include <hip/hip_runtime.h>

#include <climits>
#include <cmath>
#include <cstring>
#include <vector>

#include "../../include/lbm_stability.h"
#include "lbm_dual.h"
#include "lbm_internal.h"
#include "lbm_node.h"

using namespace lbm;

namespace {

struct StabSet {
  double dx, dy, dt;
  double s[16];
  double rho, ux, uy, T;
  int version, modified;
};

struct StabCoef {
  double P0[256], Bx[256], By[256], Qx[256], Qy[256];  // row-major, row = moment index
};

constexpr int DEFAULT_SQUARINGS = 48;
constexpr int LDS_PITCH = 17;  // padded rows: column reads hit distinct banks

size_t set_bytes(int n) { return ((size_t)n * sizeof(StabSet) + 255) / 256 * 256; }

// d q_k / d (rho, j_x, j_y, e)_c for the equilibrium moments q (Eqs. 14a-14i
// and the version's free moments), by a dual number seeded on component c.
template <int VER>
__device__ double deq(int k, int c, double rho, double jx, double jy, double e) {
  Dual a[4] = {Dual(rho), Dual(jx), Dual(jy), Dual(e)};
  a[c].d = 1.0;
  Dual q[16];
  equilibrium_moments<VER, Dual>(a[0], a[1], a[2], a[3], q);
  return q[k].d;
}

// Row i of M diag(w) M^-1 e_j: the moment image of velocity-space scaling.
__device__ double scaled_transform(int i, int j, const double* w) {
  double m[16], f[16];
  for (int k = 0; k < 16; ++k) m[k] = (k == j) ? 1.0 : 0.0;
  f_from_moments(m, f);
  for (int k = 0; k < 16; ++k) f[k] *= w[k];
  moments_from_f(f, m);
  return m[i];
}

// One workgroup (256 threads) per parameter set; thread t builds entry
// (t / 16, t % 16) of the five matrices.
__global__ __launch_bounds__(256) void k_stab_setup(const StabSet* __restrict__ sets, StabCoef* __restrict__ coef) {
  const StabSet S = sets[blockIdx.x];
  StabCoef& C = coef[blockIdx.x];
  const int t = threadIdx.x, i = t >> 4, j = t & 15;
  const double rho = S.rho, ux = S.ux, uy = S.uy, T = S.T;
  const double jx = rho * ux, jy = rho * uy, e = rho * (T + 0.5 * (ux * ux + uy * uy));
  // collision: I - dt S (I - D); rows 1..4 (conserved) are identity rows
  double p0 = (i == j) ? 1.0 : 0.0;
  if (i >= 4) {
    double d = 0.0;
    if (j < 4) d = S.version == 2 ? deq<2>(i, j, rho, jx, jy, e)
                 : S.version == 3 ? deq<3>(i, j, rho, jx, jy, e)
                                  : deq<1>(i, j, rho, jx, jy, e);
    p0 -= S.dt * S.s[i] * (((i == j) ? 1.0 : 0.0) - d);
  }
  // convection symbols
  double cx[16], cx2[16], cy[16], cy2[16];
  for (int k = 0; k < 16; ++k) {
    cx[k] = VX[k] * S.dt / S.dx;
    cy[k] = VY[k] * S.dt / S.dy;
    cx2[k] = cx[k] * cx[k];
    cy2[k] = cy[k] * cy[k];
  }
  double qx = -scaled_transform(i, j, cx), qy = -scaled_transform(i, j, cy);
  // energy-flux modification: rows 7 and 8, columns rho, j_x, j_y
  if (S.modified && (i == 6 || i == 7) && j < 3) {
    const double s5 = S.s[4], s6 = S.s[5], s7 = S.s[6], s8 = S.s[7];
    const double rT = rho * T;
    const double dux = (j == 0) ? -ux / rho : (j == 1) ? 1.0 / rho : 0.0;  // d u_x / d(rho, j_x, j_y)
    const double duy = (j == 0) ? -uy / rho : (j == 2) ? 1.0 / rho : 0.0;
    double a, b;
    if (i == 6) {
      const double ka = s7 / s5 - 1.0, kb = s7 / s6 - 1.0;
      a = ka * rT * ux * dux + kb * rT * uy * duy;
      b = -ka * rT * ux * duy + kb * rT * uy * dux;
    } else {
      const double ka = s8 / s6 - 1.0, kb = ((S.modified == 2) ? 1.0 : -1.0) * (s8 / s5 - 1.0);
      a = ka * rT * ux * duy + kb * rT * uy * dux;
      b = ka * rT * ux * dux - kb * rT * uy * duy;
    }
    qx -= S.dt / S.dx * a;
    qy -= S.dt / S.dy * b;
  }
  C.P0[t] = p0;
  C.Bx[t] = scaled_transform(i, j, cx2);
  C.By[t] = scaled_transform(i, j, cy2);
  C.Qx[t] = qx;
  C.Qy[t] = qy;
}

// Entry (i, j) of G(theta) for set C.
__device__ __forceinline__ void g_entry(const StabCoef& C, int idx, double cxm1, double cym1, double sx, double sy,
                                        double& re, double& im) {
  re = C.P0[idx] + cxm1 * C.Bx[idx] + cym1 * C.By[idx];
  im = sx * C.Qx[idx] + sy * C.Qy[idx];
}

// One workgroup per point, thread t writes entry (t / 16, t % 16).
__global__ __launch_bounds__(256) void k_stab_matrix(const StabCoef* __restrict__ coef, const double* __restrict__ theta,
                                                      int npts, double* __restrict__ out) {
  const long long p = blockIdx.x;  // point index over all sets
  const int set = (int)(p / npts), t = (int)(p % npts);
  const double tx = theta[2 * t], ty = theta[2 * t + 1];
  double sx, cxx, sy, cyy;
  sincos(tx, &sx, &cxx);
  sincos(ty, &sy, &cyy);
  double re, im;
  g_entry(coef[set], threadIdx.x, cxx - 1.0, cyy - 1.0, sx, sy, re, im);
  out[p * 512 + threadIdx.x] = re;
  out[p * 512 + 256 + threadIdx.x] = im;
}

typedef double v4d __attribute__((ext_vector_type(4)));

__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) v = fmax(v, __shfl_xor(v, m));
  return v;
}

// |omega|_max by repeated squaring; one wavefront (= one workgroup) per point
// at a time, grid-stride over all (set, point) pairs.
//
// Layouts of v_mfma_f64_16x16x4f64 (lane l, q = l / 16, c = l % 16):
//   A (16 x 4): A[c][q];  B (4 x 16): B[q][c];  C/D (16 x 16): D[q + 4 r][c], r = 0..3
// (checked on the device against a host product).
__global__ __launch_bounds__(64) void k_stab_radius(const StabCoef* __restrict__ coef,
                                                     const double* __restrict__ theta, int npts, long long total,
                                                     int squarings, double* __restrict__ out) {
  __shared__ double Lr[16 * LDS_PITCH], Li[16 * LDS_PITCH];
  const int lane = threadIdx.x, q = lane >> 4, c = lane & 15;
  for (long long p = blockIdx.x; p < total; p += gridDim.x) {
    const int set = (int)(p / npts), t = (int)(p % npts);
    const StabCoef& C = coef[set];
    double sx, cxx, sy, cyy;
    sincos(theta[2 * t], &sx, &cxx);
    sincos(theta[2 * t + 1], &sy, &cyy);
    v4d xr, xi;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      double re, im;
      g_entry(C, (q + 4 * r) * 16 + c, cxx - 1.0, cyy - 1.0, sx, sy, re, im);
      xr[r] = re;
      xi[r] = im;
    }
    double L = 0.0, frac = 1.0;
    bool zero = false;
    for (int j = 0; j <= squarings; ++j) {
      if (j > 0) {
        // X <- X^2 through LDS: write the accumulator layout, read the operand layouts
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          Lr[(q + 4 * r) * LDS_PITCH + c] = xr[r];
          Li[(q + 4 * r) * LDS_PITCH + c] = xi[r];
        }
        __syncthreads();
        v4d ar4 = {0.0, 0.0, 0.0, 0.0}, ai4 = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int kb = 0; kb < 4; ++kb) {
          const double are = Lr[c * LDS_PITCH + 4 * kb + q], aim = Li[c * LDS_PITCH + 4 * kb + q];
          const double bre = Lr[(4 * kb + q) * LDS_PITCH + c], bim = Li[(4 * kb + q) * LDS_PITCH + c];
          ar4 = __builtin_amdgcn_mfma_f64_16x16x4f64(are, bre, ar4, 0, 0, 0);
          ar4 = __builtin_amdgcn_mfma_f64_16x16x4f64(-aim, bim, ar4, 0, 0, 0);
          ai4 = __builtin_amdgcn_mfma_f64_16x16x4f64(are, bim, ai4, 0, 0, 0);
          ai4 = __builtin_amdgcn_mfma_f64_16x16x4f64(aim, bre, ai4, 0, 0, 0);
        }
        __syncthreads();  // every lane has read X before the next write
        xr = ar4;
        xi = ai4;
      }
      double m = 0.0;
#pragma unroll
      for (int r = 0; r < 4; ++r) m = fmax(m, fmax(fabs(xr[r]), fabs(xi[r])));
      m = wave_max(m);
      if (!(m > 0.0)) {  // zero matrix (nilpotent G), or NaN
        zero = m == 0.0;
        L = zero ? 0.0 : m;
        break;
      }
      const int ex = ilogb(m);
      const double sc = ldexp(1.0, -ex);
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        xr[r] *= sc;
        xi[r] *= sc;
      }
      L += ldexp((double)ex, -j);
      frac = m * sc;
    }
    if (lane == 0) {
      double rad;
      if (zero) rad = 0.0;
      else if (L != L) rad = L;
      else rad = exp2(L + log2(frac) * ldexp(1.0, -squarings));
      out[p] = rad;
    }
  }
}

lbm_status check_sets(const lbm_params* sets, const lbm_state* states, int32_t nsets, const double* d_theta,
                      int32_t npts, void* d_ws, size_t ws_bytes, void* d_out) {
  if (!sets || !states || nsets < 1) return fail(LBM_EINVAL, "need at least one parameter set and state");
  if (!d_theta || npts < 1) return fail(LBM_EINVAL, "need at least one wavenumber point");
  if (!d_out) return fail(LBM_EINVAL, "output is NULL");
  if ((long long)nsets * npts > (1LL << 40)) return fail(LBM_EINVAL, "too many points");
  if (!d_ws || ((uintptr_t)d_ws) % 256) return fail(LBM_EINVAL, "workspace must be 256-byte aligned");
  if (ws_bytes < lbm_stability_workspace_bytes(nsets))
    return fail(LBM_ENOMEM, "workspace has %zu bytes, needs %zu", ws_bytes, lbm_stability_workspace_bytes(nsets));
  for (int k = 0; k < nsets; ++k) {
    const lbm_params& p = sets[k];
    if (!(p.dx > 0) || !(p.dy > 0) || !(p.dt > 0)) return fail(LBM_EINVAL, "set %d: dx, dy, dt must be > 0", k);
    for (int i = 4; i < 16; ++i)
      if (!(p.s[i] > 0)) return fail(LBM_EINVAL, "set %d: s_%d must be > 0", k, i + 1);
    if (p.eq_version < 1 || p.eq_version > 3) return fail(LBM_EINVAL, "set %d: eq_version must be 1, 2 or 3", k);
    if (p.modified < 0 || p.modified > 2) return fail(LBM_EINVAL, "set %d: modified must be 0, 1 or 2", k);
    if (p.scheme != 0) return fail(LBM_EINVAL, "set %d: the stability tool linearises scheme 0 only", k);
    const lbm_state& s = states[k];
    if (!(s.rho > 0) || !(s.T > 0) || !std::isfinite(s.rho) || !std::isfinite(s.T) || !std::isfinite(s.ux) ||
        !std::isfinite(s.uy))
      return fail(LBM_EINVAL, "set %d: base state needs rho > 0, T > 0 and finite u", k);
  }
  return LBM_OK;
}

// Uploads the sets and builds their coefficient blocks.
lbm_status setup(const lbm_params* sets, const lbm_state* states, int32_t nsets, void* d_ws, hipStream_t st,
                 StabCoef** coef) {
  std::vector<StabSet> h(nsets);
  for (int k = 0; k < nsets; ++k) {
    StabSet& S = h[k];
    std::memset(&S, 0, sizeof(S));
    S.dx = sets[k].dx;
    S.dy = sets[k].dy;
    S.dt = sets[k].dt;
    for (int i = 0; i < 16; ++i) S.s[i] = sets[k].s[i];
    S.rho = states[k].rho;
    S.ux = states[k].ux;
    S.uy = states[k].uy;
    S.T = states[k].T;
    S.version = sets[k].eq_version;
    S.modified = sets[k].modified;
  }
  StabSet* d_sets = (StabSet*)d_ws;
  *coef = (StabCoef*)((char*)d_ws + set_bytes(nsets));
  hipError_t e = hipMemcpyAsync(d_sets, h.data(), nsets * sizeof(StabSet), hipMemcpyHostToDevice, st);
  if (e == hipSuccess) {
    hipLaunchKernelGGL(k_stab_setup, dim3(nsets), dim3(256), 0, st, d_sets, *coef);
    e = hipGetLastError();
  }
  if (e == hipSuccess) e = hipStreamSynchronize(st);  // h is the copy source
  if (e != hipSuccess) return hip_fail(e, "stability set-up");
  return LBM_OK;
}

}  // namespace

extern "C" {

size_t lbm_stability_workspace_bytes(int32_t nsets) {
  if (nsets < 1) return 0;
  return set_bytes(nsets) + (size_t)nsets * sizeof(StabCoef);
}

lbm_status lbm_stability_matrix(const lbm_params* sets, const lbm_state* states, int32_t nsets,
                                const double* d_theta, int32_t npts, void* d_workspace, size_t ws_bytes,
                                double* d_G, void* hip_stream) {
  lbm_status st = check_sets(sets, states, nsets, d_theta, npts, d_workspace, ws_bytes, d_G);
  if (st != LBM_OK) return st;
  if ((long long)nsets * npts > INT_MAX) return fail(LBM_EINVAL, "too many points for the matrix output");
  hipStream_t s = (hipStream_t)hip_stream;
  StabCoef* coef = nullptr;
  st = setup(sets, states, nsets, d_workspace, s, &coef);
  if (st != LBM_OK) return st;
  hipLaunchKernelGGL(k_stab_matrix, dim3((unsigned)(nsets * npts)), dim3(256), 0, s, coef, d_theta, npts, d_G);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(e, "k_stab_matrix launch");
  clear_error();
  return LBM_OK;
}

lbm_status lbm_stability_radius(const lbm_params* sets, const lbm_state* states, int32_t nsets,
                                const double* d_theta, int32_t npts, int32_t squarings, void* d_workspace,
                                size_t ws_bytes, double* d_radius, void* hip_stream) {
  lbm_status st = check_sets(sets, states, nsets, d_theta, npts, d_workspace, ws_bytes, d_radius);
  if (st != LBM_OK) return st;
  if (squarings == 0) squarings = DEFAULT_SQUARINGS;
  if (squarings < 1 || squarings > 60) return fail(LBM_EINVAL, "squarings must be in [1, 60] (0 = default)");
  hipStream_t s = (hipStream_t)hip_stream;
  StabCoef* coef = nullptr;
  st = setup(sets, states, nsets, d_workspace, s, &coef);
  if (st != LBM_OK) return st;
  const long long total = (long long)nsets * npts;
  const long long grid = total < 16384 ? total : 16384;
  hipLaunchKernelGGL(k_stab_radius, dim3((unsigned)grid), dim3(64), 0, s, coef, d_theta, npts, total, squarings,
                     d_radius);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(e, "k_stab_radius launch");
  clear_error();
  return LBM_OK;
}

}  // extern "C"
