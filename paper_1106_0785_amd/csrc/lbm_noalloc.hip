// Allocation-free form of lbm_create + lbm_init-from-f + lbm_step + lbm_get_f
// (contract in include/lbm.h, lbm_run_noalloc): the two pitched
// distribution buffers, the problem coefficients and the health flag live in
// a fixed device array of this translation unit instead of a caller-provided
// workspace.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <mutex>

#include "../../include/lbm.h"
#include "lbm_internal.h"

using namespace lbm;

namespace {

// Layout of the array: [coefficients | health flag | f buffer 0 | f buffer 1].
constexpr size_t CONSTS_SLOT = 64 * 1024;  // >= sizeof(Consts), 256-byte multiple
constexpr size_t FLAG_SLOT = 256;
constexpr size_t F_BYTES = (size_t)LBM_NOALLOC_MAX_NODES * 16 * sizeof(double);  // one buffer at the maximum
constexpr size_t SCRATCH_BYTES = CONSTS_SLOT + FLAG_SLOT + 2 * F_BYTES;
static_assert(sizeof(Consts) <= CONSTS_SLOT, "coefficient slot too small");

// The array itself. Host code never passes this name to a kernel or a copy:
// on the host it is only a handle for hipGetSymbolAddress, which gives each
// device's own copy's address.
__device__ __align__(256) unsigned char scratch[SCRATCH_BYTES];

constexpr int MAX_DEVICES = 64;
std::mutex g_mu;
unsigned char* g_ptr[MAX_DEVICES] = {};

// Device address of this device's copy of the array (looked up once per
// device, with that device current).
lbm_status scratch_of(int dev, unsigned char** out) {
  if (dev < 0 || dev >= MAX_DEVICES) return fail(LBM_EINVAL, "device %d out of range", dev);
  std::lock_guard<std::mutex> lock(g_mu);
  if (!g_ptr[dev]) {
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(scratch)");
    if (!ptr || ((uintptr_t)ptr) % 256) return fail(LBM_EHIP, "scratch array has no usable device address");
    g_ptr[dev] = (unsigned char*)ptr;
  }
  *out = g_ptr[dev];
  return LBM_OK;
}

// Writes the coefficients (passed by value) into the array's slot, so no host
// buffer has to outlive the call.
template <int U>
__global__ void k_put_consts(Consts c, Consts* dst) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *dst = c;
}

template <int U>
__global__ void k_clear_flag(int* flag) {
  if (threadIdx.x == 0 && blockIdx.x == 0) flag[0] = 0;
}

template <int U>
__global__ void k_report_flag(const int* flag, int32_t* out) {
  if (threadIdx.x == 0 && blockIdx.x == 0) out[0] = flag[0] ? (int32_t)LBM_ENONFINITE : (int32_t)LBM_OK;
}

}  // namespace

extern "C" {

lbm_status lbm_run_noalloc(const lbm_params* p, const double* d_f_in, double* d_f_out, int64_t nsteps,
                           int32_t* d_status, void* hip_stream) {
  lbm_status st = validate(p);
  if (st != LBM_OK) return st;
  if (!d_f_in || !d_f_out) return fail(LBM_EINVAL, "distribution arrays must not be NULL");
  if (nsteps < 0) return fail(LBM_EINVAL, "nsteps must be >= 0");
  const long long pitch = row_pitch(p->nx);
  const long long nodes = pitch * p->ny;
  if (nodes > LBM_NOALLOC_MAX_NODES)
    return fail(LBM_EINVAL,
                "%d x %d grid needs %lld stored nodes (rows padded to %lld); lbm_run_noalloc holds at most %d",
                p->nx, p->ny, nodes, pitch, LBM_NOALLOC_MAX_NODES);
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
  unsigned char* base = nullptr;
  st = scratch_of(dev, &base);
  if (st != LBM_OK) return st;
  const hipStream_t s = (hipStream_t)hip_stream;
  Consts* consts = (Consts*)base;
  int* flag = (int*)(base + CONSTS_SLOT);
  double* f[2] = {(double*)(base + CONSTS_SLOT + FLAG_SLOT), (double*)(base + CONSTS_SLOT + FLAG_SLOT + F_BYTES)};
  const long long plane = pitch * p->ny;

  Consts host;
  make_coef(p, &host.hot, &host.cold);
  hipLaunchKernelGGL(k_put_consts<0>, dim3(1), dim3(64), 0, s, host, consts);
  hipLaunchKernelGGL(k_clear_flag<0>, dim3(1), dim3(64), 0, s, flag);
  e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(e, "set-up launch");
  // both buffers take the initial state (NEQ wall nodes are then defined in
  // either, as after lbm_set_f)
  for (int b = 0; b < 2; ++b) {
    e = hipMemcpy2DAsync(f[b], pitch * sizeof(double), d_f_in, p->nx * sizeof(double), p->nx * sizeof(double),
                         (size_t)16 * p->ny, hipMemcpyDeviceToDevice, s);
    if (e != hipSuccess) return hip_fail(e, "copying the initial distributions in");
  }
  // the kernel lbm_create picks for this problem, with its default shape
  const int variant = default_variant(p);
  const bool walls = has_walls(p);
  const WinGeom win = default_window(p);
  const TileShape tile = default_tile(p->nx, p->ny), tile2 = default_tile2(p->nx, p->ny);
  int cur = 0;
  int64_t n = 0;
  while (n < nsteps) {
    Field F;
    F.fin = f[cur];
    F.fout = f[cur ^ 1];
    F.nx = p->nx;
    F.ny = p->ny;
    F.pitch = pitch;
    F.plane = plane;
    int64_t k = 1;
    if (variant == 2) {
      k = std::min<int64_t>(1 << 16, nsteps - n);
      e = launch_small(F, &consts->hot, &consts->cold, p->eq_version, walls, (int)k, flag, s);
    } else if (variant == 3) {
      k = std::min<int64_t>(win.h, nsteps - n);
      e = launch_window(F, &consts->hot, &consts->cold, p->eq_version, walls, win, (int)k, flag, s);
    } else if (variant == 4 && nsteps - n >= 2) {
      k = 2;
      e = launch_step2(F, &consts->hot, &consts->cold, p->eq_version, tile2, flag, s);
    } else {
      e = launch_step(F, &consts->hot, &consts->cold, p->eq_version, walls, p->scheme, 0, tile, flag, s);
    }
    if (e != hipSuccess) return hip_fail(e, "step kernel launch");
    cur ^= 1;
    n += k;
  }
  e = hipMemcpy2DAsync(d_f_out, p->nx * sizeof(double), f[cur], pitch * sizeof(double), p->nx * sizeof(double),
                       (size_t)16 * p->ny, hipMemcpyDeviceToDevice, s);
  if (e != hipSuccess) return hip_fail(e, "copying the distributions out");
  if (d_status) {
    hipLaunchKernelGGL(k_report_flag<0>, dim3(1), dim3(64), 0, s, flag, d_status);
    e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "status launch");
  }
  clear_error();
  return LBM_OK;
}

}  // extern "C"
