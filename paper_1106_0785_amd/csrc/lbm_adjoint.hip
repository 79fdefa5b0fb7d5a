// Checkpointed forward sweep and reverse (adjoint) sweep; contracts in
// include/lbm_adjoint.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>

#include "../../include/lbm_adjoint.h"
#include "lbm_adjoint_fused.h"
#include "lbm_internal.h"

using namespace lbm;

namespace {

size_t a256(size_t x) { return (x + 255) / 256 * 256; }

struct AdjLayout {
  int C, K;               // checkpoint interval, segments
  long long pitch, plane;  // distribution layout
  int gx, gy;             // adjoint launch grid
  size_t consts, adj, ckpt, seg, lam, rec, partials, red, red_bytes, flag, total;
};

lbm_status adj_layout(const lbm_params* p, int64_t nsteps, int32_t ckpt, AdjLayout* L) {
  lbm_status st = validate(p);
  if (st != LBM_OK) return st;
  if (p->scheme != 0) return fail(LBM_EINVAL, "the adjoint form supports scheme 0 (Lax-Wendroff) only");
  if (nsteps < 1) return fail(LBM_EINVAL, "nsteps must be >= 1");
  if (ckpt < 0) return fail(LBM_EINVAL, "checkpoint interval must be >= 0");
  L->C = ckpt > 0 ? ckpt : std::max(1, (int)std::lround(std::sqrt((double)nsteps)));
  L->C = (int)std::min<int64_t>(L->C, nsteps);
  L->K = (int)((nsteps + L->C - 1) / L->C);
  L->pitch = row_pitch(p->nx);
  L->plane = L->pitch * p->ny;
  L->gx = (p->nx + 63) / 64;
  L->gy = (p->ny + 3) / 4;
  const size_t state = (size_t)16 * L->plane * sizeof(double);
  size_t off = 0;
  L->consts = off;
  off += a256(sizeof(Consts));
  L->adj = off;
  off += a256(sizeof(AdjCoef));
  L->ckpt = off;
  off += (size_t)(L->K + 1) * state;
  L->seg = off;
  off += (size_t)std::max(L->C, 2) * state;
  L->lam = off;
  off += 2 * state;
  L->rec = off;
  off += 2 * a256((size_t)NREC * L->plane * sizeof(double));
  L->partials = off;
  off += a256((size_t)L->gx * L->gy * 12 * sizeof(double));
  // two ping-pong buffers for the chunked reduction of the partials
  L->red = off;
  L->red_bytes = a256((size_t)((L->gx * L->gy + ADJ_CHUNK - 1) / ADJ_CHUNK) * 12 * sizeof(double));
  off += 2 * L->red_bytes;
  L->flag = off;
  off += 256;
  L->total = off;
  return LBM_OK;
}

}  // namespace

struct lbm_adjoint {
  lbm_params p;
  AdjLayout L;
  int64_t nsteps;
  hipStream_t stream;
  char* base;
  Consts host;
  AdjCoef adj;
  bool forward_done;
  int variant;  // adjoint step: 0 LDS-staged tiles, 1 one thread per node, global gathers
  double* state(size_t off, int i) { return (double*)(base + off) + (size_t)i * 16 * L.plane; }
  double* ckpt(int k) { return state(L.ckpt, k); }
  double* seg(int j) { return state(L.seg, j); }
  double* lam(int j) { return state(L.lam, j); }
  const Hot* dhot() { return &((Consts*)(base + L.consts))->hot; }
  const Cold* dcold() { return &((Consts*)(base + L.consts))->cold; }
  const AdjCoef* dadj() { return (const AdjCoef*)(base + L.adj); }
  double* rec(int j) {
    return (double*)(base + L.rec + (size_t)j * a256((size_t)NREC * L.plane * sizeof(double)));
  }
  double* partials() { return (double*)(base + L.partials); }
  double* red(int j) { return (double*)(base + L.red + (size_t)j * L.red_bytes); }
  int* flag() { return (int*)(base + L.flag); }
  Field field(const double* fin, double* fout) {
    Field F;
    F.fin = fin;
    F.fout = fout;
    F.nx = p.nx;
    F.ny = p.ny;
    F.pitch = L.pitch;
    F.plane = L.plane;
    return F;
  }
};

static hipError_t step_into(lbm_adjoint* a, const double* fin, double* fout) {
  return launch_step(a->field(fin, fout), a->dhot(), a->dcold(), a->p.eq_version, has_walls(&a->p), 0, 0,
                     default_tile(a->p.nx, a->p.ny), a->flag(), a->stream);
}

extern "C" {

size_t lbm_adjoint_workspace_bytes(const lbm_params* p, int64_t nsteps, int32_t ckpt_interval) {
  AdjLayout L;
  if (adj_layout(p, nsteps, ckpt_interval, &L) != LBM_OK) return 0;
  return L.total;
}

lbm_status lbm_adjoint_create(const lbm_params* p, int64_t nsteps, int32_t ckpt_interval, void* d_workspace,
                              size_t ws_bytes, void* hip_stream, lbm_adjoint** out) {
  if (!out) return fail(LBM_EINVAL, "out is NULL");
  *out = nullptr;
  AdjLayout L;
  lbm_status st = adj_layout(p, nsteps, ckpt_interval, &L);
  if (st != LBM_OK) return st;
  if (!d_workspace || ((uintptr_t)d_workspace) % 256) return fail(LBM_EINVAL, "workspace must be 256-byte aligned");
  if (ws_bytes < L.total) return fail(LBM_ENOMEM, "workspace has %zu bytes, needs %zu", ws_bytes, L.total);
  lbm_adjoint* a = new (std::nothrow) lbm_adjoint;
  if (!a) return fail(LBM_ENOMEM, "host allocation failed");
  a->p = *p;
  a->L = L;
  a->nsteps = nsteps;
  a->stream = (hipStream_t)hip_stream;
  a->base = (char*)d_workspace;
  a->forward_done = false;
  // the LDS-staged step where its tiles are tall (large grids: at 4096 x 1024
  // it takes 507 us per step against 598 for the gather form); small grids
  // give each tile one row per wavefront, and the gather form is faster
  // there (12.9 against 15.8 us per step at 512 x 128)
  a->variant = default_tile(p->nx, p->ny).rows >= 16 ? 0 : 1;
  make_coef(p, &a->host.hot, &a->host.cold);
  std::memset(&a->adj, 0, sizeof(a->adj));
  const double dt = p->dt, s5 = p->s[4], s6 = p->s[5], s7 = p->s[6], s8 = p->s[7];
  a->adj.mdt = -dt;
  if (p->modified) {
    const double sgn = (p->modified == 2) ? 1.0 : -1.0;
    a->adj.dcm[0] = dt * s7 / (s5 * s5);  // d cm0 / d s5
    a->adj.dcm[1] = -dt / s5;             // d cm0 / d s7
    a->adj.dcm[2] = dt * s7 / (s6 * s6);  // d cm1 / d s6
    a->adj.dcm[3] = -dt / s6;             // d cm1 / d s7
    a->adj.dcm[4] = dt * s8 / (s6 * s6);  // d cm2 / d s6
    a->adj.dcm[5] = -dt / s6;             // d cm2 / d s8
    a->adj.dcm[6] = dt * sgn * s8 / (s5 * s5);  // d cm3 / d s5
    a->adj.dcm[7] = -dt * sgn / s5;             // d cm3 / d s8
  }
  hipError_t e = hipMemcpyAsync(a->base + L.consts, &a->host, sizeof(Consts), hipMemcpyHostToDevice, a->stream);
  if (e == hipSuccess) e = hipMemcpyAsync(a->base + L.adj, &a->adj, sizeof(AdjCoef), hipMemcpyHostToDevice, a->stream);
  if (e == hipSuccess) e = hipMemsetAsync(a->flag(), 0, 256, a->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(a->stream);
  if (e != hipSuccess) {
    delete a;
    return hip_fail(e, "uploading adjoint constants");
  }
  *out = a;
  clear_error();
  return LBM_OK;
}

lbm_status lbm_adjoint_forward(lbm_adjoint* a, const double* d_rho0, const double* d_ux0, const double* d_uy0,
                               const double* d_T0) {
  if (!a || !d_rho0 || !d_ux0 || !d_uy0 || !d_T0) return fail(LBM_EINVAL, "NULL argument");
  const int ver = a->p.eq_version;
  {
    Field F = a->field(nullptr, a->ckpt(0));
    dim3 grid((a->p.nx + 63) / 64, a->p.ny);
    auto k = ver == 2 ? k_init<2> : ver == 3 ? k_init<3> : k_init<1>;
    hipLaunchKernelGGL(k, grid, dim3(64), 0, a->stream, F, d_rho0, d_ux0, d_uy0, d_T0);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "k_init launch");
  }
  const int C = a->L.C, K = a->L.K;
  // between checkpoints no intermediate state is kept, so where the problem
  // takes the two-step kernel by default, steps go two per launch
  const bool two = default_variant(&a->p) == 4;
  const TileShape t2 = default_tile2(a->p.nx, a->p.ny);
  for (int k = 0; k < K; ++k) {
    const int64_t n0 = (int64_t)k * C, n1 = std::min<int64_t>(n0 + C, a->nsteps);
    const double* fin = a->ckpt(k);
    int j = 0;
    for (int64_t n = n0; n < n1;) {
      const int64_t take = (two && n1 - n >= 2) ? 2 : 1;
      double* fout = (n + take == n1) ? a->ckpt(k + 1) : a->seg(j);
      hipError_t e = take == 2 ? launch_step2(a->field(fin, fout), a->dhot(), a->dcold(), a->p.eq_version, t2,
                                              a->flag(), a->stream)
                               : step_into(a, fin, fout);
      if (e != hipSuccess) return hip_fail(e, "forward step launch");
      fin = fout;
      j ^= 1;
      n += take;
    }
  }
  a->forward_done = true;
  return LBM_OK;
}

lbm_status lbm_adjoint_final_moments(lbm_adjoint* a, double* d_rho, double* d_ux, double* d_uy, double* d_T,
                                     double* d_p) {
  if (!a) return fail(LBM_EINVAL, "adjoint handle is NULL");
  if (!a->forward_done) return fail(LBM_ESTATE, "run lbm_adjoint_forward first");
  Field F = a->field(a->ckpt(a->L.K), nullptr);
  dim3 grid((a->p.nx + 63) / 64, a->p.ny);
  hipLaunchKernelGGL(k_moments<0>, grid, dim3(64), 0, a->stream, F, d_rho, d_ux, d_uy, d_T, d_p);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(e, "k_moments launch");
  return LBM_OK;
}

lbm_status lbm_adjoint_backward(lbm_adjoint* a, const double* d_rho0, const double* d_ux0, const double* d_uy0,
                                const double* d_T0, const double* d_g_rho, const double* d_g_ux,
                                const double* d_g_uy, const double* d_g_T, double* d_grad_rho0,
                                double* d_grad_ux0, double* d_grad_uy0, double* d_grad_T0, double* d_grad_s) {
  if (!a || !d_rho0 || !d_ux0 || !d_uy0 || !d_T0) return fail(LBM_EINVAL, "NULL argument");
  if (!a->forward_done) return fail(LBM_ESTATE, "run lbm_adjoint_forward first");
  const int ver = a->p.eq_version;
  const AdjLayout& L = a->L;
  const dim3 grow((a->p.nx + 63) / 64, a->p.ny);
  const dim3 gblk(L.gx, L.gy), bblk(64, 4);
  int cur = 0, rc = 0;
  // lambda^T from the gradients of the final fields
  hipLaunchKernelGGL(k_adj_final<0>, grow, dim3(64), 0, a->stream, a->field(a->ckpt(L.K), nullptr), d_g_rho, d_g_ux,
                     d_g_uy, d_g_T, a->lam(cur));
  const long long np = (long long)L.gx * L.gy * 12;
  hipLaunchKernelGGL(k_zero<0>, dim3((unsigned)((np + 255) / 256)), dim3(256), 0, a->stream, a->partials(), np);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(e, "adjoint set-up launch");
  auto krec = ver == 2 ? k_adj_records<2> : ver == 3 ? k_adj_records<3> : k_adj_records<1>;
  auto kwall = ver == 2 ? k_adj_walls<2> : ver == 3 ? k_adj_walls<3> : k_adj_walls<1>;
  const bool walls = has_walls(&a->p);
  // grids of more than 2048 blocks (8 per CU) take the two-blocks-per-CU form
  const bool wide = (long long)L.gx * L.gy > 2048;
  auto kstep = wide ? (ver == 2 ? k_adj_step<2, true> : ver == 3 ? k_adj_step<3, true> : k_adj_step<1, true>)
                    : (ver == 2 ? k_adj_step<2, false> : ver == 3 ? k_adj_step<3, false> : k_adj_step<1, false>);
  // the LDS-staged step: 64-column tiles of 4 waves (at least 4 rows each, so
  // there are no more tiles than the per-block partial slots)
  auto kfused = ver == 2 ? k_adj_fused<2, 4, true> : ver == 3 ? k_adj_fused<3, 4, true> : k_adj_fused<1, 4, true>;
  const MarchGeom ag = march_geom(a->p.nx, a->p.ny, TileShape{std::max(4, default_tile(a->p.nx, a->p.ny).rows), 4, 1});
  for (int k = L.K - 1; k >= 0; --k) {
    const int64_t n0 = (int64_t)k * L.C, n1 = std::min<int64_t>(n0 + L.C, a->nsteps);
    // recompute f^{n0+1} .. f^{n1-1} into the segment store (f^{n0} is the checkpoint)
    for (int64_t n = n0 + 1; n < n1; ++n) {
      const double* fin = (n - 1 == n0) ? a->ckpt(k) : a->seg((int)(n - 1 - n0));
      e = step_into(a, fin, a->seg((int)(n - n0)));
      if (e != hipSuccess) return hip_fail(e, "recompute step launch");
    }
    // Each adjoint step n needs the records (dL/dA, dL/dB, velocity) of
    // every node at level n; step n writes those of step n - 1 as it
    // produces lambda^n, except across a segment boundary, where level
    // n - 1 is not recomputed yet and a records pass runs first.
    for (int64_t n = n1 - 1; n >= n0; --n) {
      const double* fn = (n == n0) ? a->ckpt(k) : a->seg((int)(n - n0));
      // with NEQ walls lambda^{n+1} first takes the walls' transpose, so the
      // records of every step come from a separate pass after it
      const double* fprev =
          (walls || n - 1 < n0) ? nullptr : (n - 1 == n0) ? a->ckpt(k) : a->seg((int)(n - 1 - n0));
      Field F = a->field(fn, nullptr);
      if (walls) {
        const double* fnext = (n + 1 == n1) ? a->ckpt(k + 1) : a->seg((int)(n + 1 - n0));
        const int along = (a->p.bc[2] == LBM_BC_NEQ_WALL || a->p.bc[3] == LBM_BC_NEQ_WALL) ? a->p.nx : a->p.ny;
        hipLaunchKernelGGL(kwall, dim3((along + 63) / 64), dim3(64), 0, a->stream, a->field(fnext, nullptr),
                           a->lam(cur), a->dhot(), a->dcold());
      }
      if (walls || n == n1 - 1)
        hipLaunchKernelGGL(krec, gblk, bblk, 0, a->stream, F, a->lam(cur), a->rec(rc), a->dhot());
      if (a->variant == 0)
        hipLaunchKernelGGL(kfused, dim3(8 * ag.per_xcd), dim3(256), 0, a->stream, F, a->lam(cur), a->lam(cur ^ 1),
                           a->rec(rc), a->dhot(), a->dcold(), a->dadj(), a->partials(), fprev, a->rec(rc ^ 1), ag);
      else
        hipLaunchKernelGGL(kstep, gblk, bblk, 0, a->stream, F, a->lam(cur), a->lam(cur ^ 1), a->rec(rc), a->dhot(),
                           a->dcold(), a->dadj(), a->partials(), fprev, a->rec(rc ^ 1));
      e = hipGetLastError();
      if (e != hipSuccess) return hip_fail(e, "adjoint step launch");
      cur ^= 1;
      if (fprev) rc ^= 1;
    }
  }
  // initial-state adjoint and the s-gradient
  auto kinit = ver == 2 ? k_adj_init<2> : ver == 3 ? k_adj_init<3> : k_adj_init<1>;
  hipLaunchKernelGGL(kinit, grow, dim3(64), 0, a->stream, a->field(a->ckpt(0), nullptr), a->lam(cur), d_rho0, d_ux0,
                     d_uy0, d_T0, d_grad_rho0, d_grad_ux0, d_grad_uy0, d_grad_T0);
  if (d_grad_s) {
    // fixed-order reduction of the per-block partials: chunks of ADJ_CHUNK
    // rows, repeated until one row is left
    const double* in = a->partials();
    long long rows = (long long)L.gx * L.gy;
    int j = 0;
    do {
      const long long nout = (rows + ADJ_CHUNK - 1) / ADJ_CHUNK;
      hipLaunchKernelGGL(k_adj_reduce<0>, dim3((unsigned)((nout * 12 + 255) / 256)), dim3(256), 0, a->stream, in,
                         (int)rows, a->red(j));
      in = a->red(j);
      j ^= 1;
      rows = nout;
    } while (rows > 1);
    hipLaunchKernelGGL(k_adj_grad<0>, dim3(1), dim3(64), 0, a->stream, in, d_grad_s);
  }
  e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(e, "adjoint finish launch");
  return LBM_OK;
}

lbm_status lbm_adjoint_set_variant(lbm_adjoint* a, int32_t variant) {
  if (!a) return fail(LBM_EINVAL, "adjoint handle is NULL");
  if (variant != 0 && variant != 1) return fail(LBM_EINVAL, "adjoint variant must be 0 or 1");
  a->variant = variant;
  return LBM_OK;
}

lbm_status lbm_adjoint_check(lbm_adjoint* a) {
  if (!a) return fail(LBM_EINVAL, "adjoint handle is NULL");
  int flag = 0;
  hipError_t e = hipMemcpyAsync(&flag, a->flag(), sizeof(int), hipMemcpyDeviceToHost, a->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(a->stream);
  if (e != hipSuccess) return hip_fail(e, "reading the health flag");
  if (flag) {
    e = hipMemsetAsync(a->flag(), 0, sizeof(int), a->stream);
    if (e != hipSuccess) return hip_fail(e, "hipMemsetAsync");
    return fail(LBM_ENONFINITE, "a forward step produced rho <= 0, T <= 0 or NaN");
  }
  return LBM_OK;
}

void lbm_adjoint_destroy(lbm_adjoint* a) { delete a; }

}  // extern "C"
