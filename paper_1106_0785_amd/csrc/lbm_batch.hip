// C ABI of the batched form (declarations and contracts in include/lbm_batch.h).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <cstring>
#include <new>
#include <vector>

#include "../../include/lbm_batch.h"
#include "lbm_batch_kernels.h"
#include "lbm_internal.h"

using namespace lbm;

namespace {

constexpr int MIN_CHUNK = 32;

// Device status words of a batch, each in a line of its own: health flag at
// byte 0, the persistent launches' time-out error at 64 and ticket counter
// at 128 (the persistent kernel finds them from the flag's address).
constexpr size_t STATUS_BYTES = 256;
static_assert(STATUS_BYTES % 256 == 0, "the backup arena after the status words stays 256-byte aligned");

struct Schedule {
  int region;  // 128 or 256 nodes per workgroup region
  int h;       // time steps per launch
};

bool schedule_ok(const Schedule& s) {
  return (s.region == 128 || s.region == 256) && s.h >= 1 && s.region - 2 * s.h >= MIN_CHUNK;
}

template <int VER, int REGION>
void launch_line(const double* A, double* B, const LineInst* insts, const LineChunk* chunks, int nchunks,
                 const int* budget, int n0, int h, int* flag, hipStream_t st) {
  hipLaunchKernelGGL((k_batch_line<VER, REGION>), dim3(nchunks), dim3(REGION), 0, st, A, B, insts, chunks, budget, n0, h,
                     flag);
}

// Persistent line kernel of (version, region), as a function pointer.
typedef void (*PersistentKernel)(double*, double*, const LineInst*, const LineChunk*, int, const int*, int, int, int*,
                                 int*, long long);

PersistentKernel persistent_kernel(int ver, int region) {
  if (region == 256)
    return ver == 2 ? k_batch_line_persistent<2, 256> : ver == 3 ? k_batch_line_persistent<3, 256>
                                                                 : k_batch_line_persistent<1, 256>;
  return ver == 2 ? k_batch_line_persistent<2, 128> : ver == 3 ? k_batch_line_persistent<3, 128>
                                                               : k_batch_line_persistent<1, 128>;
}

// Default bound on one wait of a persistent launch for the chunks another
// depends on (each takes well under a millisecond).
constexpr double DEFAULT_BARRIER_TIMEOUT_MS = 2000.0;

}  // namespace

struct lbm_batch {
  int n;
  std::vector<lbm_params> params;
  std::vector<int> tiled;            // 1: advanced tile by tile (TileInst), 0: as a line (LineInst)
  std::vector<LineInst> host_insts;  // indexed by instance (entries of tiled instances unused)
  std::vector<TileInst> host_tinsts;
  std::vector<int> tindex;           // instance -> index in host_tinsts, or -1
  std::vector<long long> node_off;   // offset of instance i in concatenated field arrays
  long long total_nodes;
  long long arena_doubles;
  hipStream_t stream;
  hipStream_t capture;  // private stream the graph is captured on (the caller's may be the null stream)
  double* arena[2];
  double* backup;
  LineInst* insts;
  LineChunk* chunks;
  TileInst* tinsts;
  int2* tile_inst;  // tile list entries (index in tinsts, tile of the instance), grouped by (version, variant)
  int ntiles;       // tiles at the current tile height
  int max_tiles;    // room in tile_inst (tiles at the smallest height, padding included)
  int tile_rows;    // rows per tile of the tiled instances
  int tbegin[4][3], tend[4][3];  // entries of each [version][variant: 0 plain, 1 NEQ walls, 2 flux-limited]
                                 // (a multiple of 8, padding included)
  // two steps per launch for the plain tiled instances (k_batch_tiles2)
  int pairs;        // 1: plain tiled instances advance two steps per launch
  int2* tile_inst2;  // two-step tile list entries (index in tinsts, tile of the instance), grouped by version
  int ntiles2, max_tiles2, tile_rows2;
  int t2begin[4], t2end[4];  // entries of each version (a multiple of 8, padding included)
  std::vector<int> host_budget;
  int max_chunks;
  int* budget;
  int* flag;       // health flag (flag[0]), first of the STATUS_BYTES status words
  unsigned long long* ctr;  // chunk ticket counter of the persistent launches
  int* epoch;               // per chunk: the last block a persistent launch has finished
  int persistent;  // line instances: 1 one persistent launch per version, 0 one launch per h steps
  long long timeout_ticks;  // bound on one wait of a persistent launch, wall-clock ticks
  int resident[4][2];       // resident workgroups of the persistent kernel [version][region 128, 256]; 0 unknown
  int cur;   // current buffer of the line instances
  int cur2;  // current buffer of the tiled instances with walls or the flux-limited scheme
  int cur3;  // current buffer of the plain tiled instances
  Schedule sched;
  int use_graph;
  // chunk ranges per equilibrium version (1..3): [begin, end)
  int vbegin[4], vend[4];
  // cached graphs, one per (cur, cur2, cur3)
  hipGraphExec_t graph[8];
  int64_t graph_steps[8];
};

static long long line_len(const lbm_params& p) { return (long long)p.nx * p.ny; }

static size_t align256(size_t x) { return (x + 255) / 256 * 256; }

// A problem runs through the line kernel when it is one-dimensional, uses the
// Lax-Wendroff scheme and, if periodic, fits one line region; otherwise tile
// by tile.
static bool is_line(const lbm_params& p) {
  if (p.scheme != 0) return false;
  if (p.nx != 1 && p.ny != 1) return false;
  const int axis = (p.ny == 1 && p.nx > 1) ? 0 : 1;
  return !(p.bc[2 * axis] == LBM_BC_PERIODIC && line_len(p) > 128);
}

// Rows per tile of the tiled instances: the tallest of 64, 32, ... 4 that
// still gives the whole batch ~1024 tiles (taller tiles re-read fewer halo rows).
static int batch_tile_rows(const lbm_params* inst, int32_t n) {
  int rows = 64;
  for (; rows > WAVES; rows /= 2) {
    long long tiles = 0;
    for (int i = 0; i < n; ++i)
      if (!is_line(inst[i])) tiles += march_geom(inst[i].nx, inst[i].ny, TileShape{rows, WAVES}).ntiles;
    if (tiles >= 1024) break;
  }
  return rows;
}

// Tile-kernel variant of a tiled instance: 0 plain, 1 NEQ walls, 2 flux-limited.
static int tile_variant(const lbm_params& p) { return p.scheme == 1 ? 2 : (has_walls(&p) ? 1 : 0); }

struct Layout {
  size_t arena_bytes, insts_off, chunks_off, epoch_off, tinsts_off, tiles_off, tiles2_off, budget_off, flag_off,
      backup_off, total;
  long long arena_doubles;
  int max_chunks, ntiled, ntiles, ntiles2;  // ntiles, ntiles2: at the smallest tile heights
  int rows;  // default rows per tile of the tiled instances
  std::vector<long long> off;  // arena offset (doubles) of each instance
};

static lbm_status layout_of(const lbm_params* inst, int32_t n, Layout* L) {
  if (!inst || n < 1) return fail(LBM_EINVAL, "need at least one instance");
  long long dbl = 0, maxc = 0;
  int ntiled = 0, ntiles = 0, ntiles2 = 0;
  L->off.assign(n, 0);
  for (int i = 0; i < n; ++i) {
    lbm_status st = validate(&inst[i]);
    if (st != LBM_OK) return fail(st, "instance %d: %s", i, lbm_last_error());
  }
  L->rows = batch_tile_rows(inst, n);
  for (int i = 0; i < n; ++i) {
    const lbm_params& p = inst[i];
    if (is_line(p)) {
      const long long N = line_len(p);
      dbl = (dbl + 15) / 16 * 16;
      L->off[i] = dbl;
      dbl += 16 * ((N + 15) / 16 * 16);
      maxc += (N + MIN_CHUNK - 1) / MIN_CHUNK + 1;
    } else {
      dbl = (dbl + 63) / 64 * 64;  // 512-byte aligned rows
      L->off[i] = dbl;
      dbl += 16 * row_pitch(p.nx) * p.ny;
      const MarchGeom g = march_geom(p.nx, p.ny, TileShape{WAVES, WAVES});  // most tiles any height gives
      ++ntiled;
      if ((long long)ntiles + g.ntiles > INT_MAX / 2) return fail(LBM_EINVAL, "batch has too many tiles");
      ntiles += g.ntiles;
      if (tile_variant(p) == 0) {
        const March2Geom g2 = march2_geom(p.nx, p.ny, TileShape{2, 2});
        if ((long long)ntiles2 + g2.ntiles > INT_MAX / 2) return fail(LBM_EINVAL, "batch has too many tiles");
        ntiles2 += g2.ntiles;
      }
    }
  }
  L->arena_doubles = dbl;
  L->max_chunks = (int)maxc;
  L->ntiled = ntiled;
  L->ntiles = ntiles;
  L->ntiles2 = ntiles2;
  L->arena_bytes = align256((size_t)dbl * sizeof(double));
  L->insts_off = 2 * L->arena_bytes;
  L->chunks_off = L->insts_off + align256((size_t)n * sizeof(LineInst));
  L->epoch_off = L->chunks_off + align256((size_t)std::max<long long>(maxc, 1) * sizeof(LineChunk));
  L->tinsts_off = L->epoch_off + align256((size_t)std::max<long long>(maxc, 1) * sizeof(int));
  L->tiles_off = L->tinsts_off + align256((size_t)std::max(ntiled, 1) * sizeof(TileInst));
  L->tiles2_off = L->tiles_off + align256((size_t)(ntiles + 72 + 1) * sizeof(int2));
  L->budget_off = L->tiles2_off + align256((size_t)(ntiles2 + 24 + 1) * sizeof(int2));
  L->flag_off = L->budget_off + align256((size_t)n * sizeof(int));
  L->backup_off = L->flag_off + STATUS_BYTES;
  L->total = L->backup_off + L->arena_bytes;
  return LBM_OK;
}

static void drop_graphs(lbm_batch* b) {
  for (int k = 0; k < 8; ++k) {
    if (b->graph[k]) (void)hipGraphExecDestroy(b->graph[k]);
    b->graph[k] = nullptr;
    b->graph_steps[k] = -1;
  }
}

// Builds the chunk list for the schedule (grouped by equilibrium version) and uploads it.
static lbm_status build_chunks(lbm_batch* b, const Schedule& s) {
  std::vector<LineChunk> ch;
  for (int ver = 1; ver <= 3; ++ver) {
    b->vbegin[ver] = (int)ch.size();
    for (int i = 0; i < b->n; ++i) {
      if (b->params[i].eq_version != ver || b->tiled[i]) continue;
      const int N = b->host_insts[i].N;
      const int first = (int)ch.size();
      if (N <= s.region) {
        ch.push_back(LineChunk{i, 0, N, 0, 0, {0, 0, 0}});
      } else {
        const int C = s.region - 2 * s.h;
        // A NEQ wall node takes its fluid neighbour's value of the same step,
        // so the chunk that writes the last node (a wall when the line has
        // walls) also writes the node before it: no one-node last chunk.
        int st = 0;
        while (st < N) {
          int len = std::min(C, N - st);
          if (b->host_insts[i].walls && N - st - len == 1) --len;
          ch.push_back(LineChunk{i, st, len, 0, 0, {0, 0, 0}});
          st += len;
        }
      }
      // chunks of this line whose nodes lie within h of chunk c's (list
      // indices relative to the version's first chunk)
      const int end = (int)ch.size();
      for (int c = first; c < end; ++c) {
        int lo = c, hi = c;
        while (lo > first && ch[lo - 1].start + ch[lo - 1].len > ch[c].start - s.h) --lo;
        while (hi + 1 < end && ch[hi + 1].start < ch[c].start + ch[c].len + s.h) ++hi;
        ch[c].dlo = lo - b->vbegin[ver];
        ch[c].dhi = hi - b->vbegin[ver];
      }
    }
    b->vend[ver] = (int)ch.size();
  }
  if ((int)ch.size() > b->max_chunks) return fail(LBM_EINVAL, "schedule needs more chunks than reserved");
  hipError_t e = hipMemcpyAsync(b->chunks, ch.data(), ch.size() * sizeof(LineChunk), hipMemcpyHostToDevice, b->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
  if (e != hipSuccess) return hip_fail(e, "uploading the chunk list");
  b->sched = s;
  drop_graphs(b);
  return LBM_OK;
}

// Appends one launch group's tiles to a tile list: (instance, tile) entries
// with the height each tile owns, ordered by decreasing height and dealt
// round-robin to the eight per-XCD runs the kernels' block mapping reads
// (entry (b mod 8) per_xcd + b / 8 for workgroup b), so that every XCD
// starts with its tallest tiles and the short tops of instances fill the
// tail; padding entries (-1) fill the group to a multiple of 8. Returns the
// number of real tiles.
static long long append_group(std::vector<int2>& list, const std::vector<int2>& v, const std::vector<int>& h) {
  std::vector<int> order(v.size());
  for (size_t k = 0; k < order.size(); ++k) order[k] = (int)k;
  std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return h[x] > h[y]; });
  const size_t per_xcd = (v.size() + 7) / 8, begin = list.size();
  list.resize(begin + 8 * per_xcd, int2{-1, 0});
  for (size_t k = 0; k < order.size(); ++k) list[begin + (k % 8) * per_xcd + k / 8] = v[order[k]];
  return (long long)v.size();
}

// Cuts the tiled instances into tiles of `rows` rows, builds the tile list
// grouped by (equilibrium version, variant) and uploads descriptors and list.
static lbm_status build_tiles(lbm_batch* b, int rows) {
  std::vector<int2> list;
  long long real = 0;
  for (TileInst& T : b->host_tinsts) T.geom = march_geom(T.nx, T.ny, TileShape{rows, WAVES});
  for (int ver = 1; ver <= 3; ++ver)
    for (int w = 0; w < 3; ++w) {
      std::vector<int2> v;
      std::vector<int> h;
      for (size_t j = 0; j < b->host_tinsts.size(); ++j) {
        const TileInst& T = b->host_tinsts[j];
        const lbm_params& p = b->params[T.gidx];
        if (p.eq_version != ver || tile_variant(p) != w) continue;
        for (int t = 0; t < T.geom.ntiles; ++t) {
          v.push_back(int2{(int)j, t});
          h.push_back(std::min(T.geom.rows, T.ny - (t / T.geom.nstrips) * T.geom.rows));
        }
      }
      b->tbegin[ver][w] = (int)list.size();
      real += append_group(list, v, h);
      b->tend[ver][w] = (int)list.size();
    }
  if ((long long)list.size() > b->max_tiles) return fail(LBM_EINVAL, "tile height needs more tiles than reserved");
  hipError_t e = hipSuccess;
  if (!b->host_tinsts.empty())
    e = hipMemcpyAsync(b->tinsts, b->host_tinsts.data(), b->host_tinsts.size() * sizeof(TileInst),
                       hipMemcpyHostToDevice, b->stream);
  if (e == hipSuccess && !list.empty())
    e = hipMemcpyAsync(b->tile_inst, list.data(), list.size() * sizeof(int2), hipMemcpyHostToDevice, b->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(b->stream);  // the host vectors are the copy sources
  if (e != hipSuccess) return hip_fail(e, "uploading the tile list");
  b->ntiles = (int)real;
  b->tile_rows = rows;
  drop_graphs(b);
  return LBM_OK;
}

// Cuts the plain tiled instances into the two-step kernel's strips with
// `rows` output rows per tile, builds their tile list grouped by equilibrium
// version (ordered as append_group orders) and uploads descriptors and list.
static lbm_status build_tiles2(lbm_batch* b, int rows) {
  std::vector<int2> list;
  long long real = 0;
  for (TileInst& T : b->host_tinsts) T.geom2 = march2_geom(T.nx, T.ny, TileShape{rows, 2});
  for (int ver = 1; ver <= 3; ++ver) {
    std::vector<int2> v;
    std::vector<int> h;
    for (size_t j = 0; j < b->host_tinsts.size(); ++j) {
      const TileInst& T = b->host_tinsts[j];
      const lbm_params& p = b->params[T.gidx];
      if (p.eq_version != ver || tile_variant(p) != 0) continue;
      for (int t = 0; t < T.geom2.ntiles; ++t) {
        v.push_back(int2{(int)j, t});
        h.push_back(std::min(T.geom2.rows, T.ny - (t / T.geom2.nstrips) * T.geom2.rows));
      }
    }
    b->t2begin[ver] = (int)list.size();
    real += append_group(list, v, h);
    b->t2end[ver] = (int)list.size();
  }
  if ((long long)list.size() > b->max_tiles2) return fail(LBM_EINVAL, "tile height needs more tiles than reserved");
  hipError_t e = hipSuccess;
  if (!b->host_tinsts.empty())
    e = hipMemcpyAsync(b->tinsts, b->host_tinsts.data(), b->host_tinsts.size() * sizeof(TileInst),
                       hipMemcpyHostToDevice, b->stream);
  if (e == hipSuccess && !list.empty())
    e = hipMemcpyAsync(b->tile_inst2, list.data(), list.size() * sizeof(int2), hipMemcpyHostToDevice, b->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
  if (e != hipSuccess) return hip_fail(e, "uploading the two-step tile list");
  b->ntiles2 = (int)real;
  b->tile_rows2 = rows;
  drop_graphs(b);
  return LBM_OK;
}

// Output rows per two-step tile: the tallest even height of 128, 64, ... 8
// that still gives the plain tiled instances ~1024 tiles.
static int batch_tile_rows2(const lbm_batch* b) {
  int rows = 128;
  for (; rows > 8; rows /= 2) {
    long long tiles = 0;
    for (const TileInst& T : b->host_tinsts)
      if (tile_variant(b->params[T.gidx]) == 0) tiles += march2_geom(T.nx, T.ny, TileShape{rows, 2}).ntiles;
    if (tiles >= 1024) break;
  }
  return rows;
}

// Workgroups of the persistent kernel of (version, region) resident on the
// stream's device at once (all its compute units, the kernel alone).
static hipError_t resident_workgroups(lbm_batch* b, int ver, int region, int* out) {
  int& r = b->resident[ver][region == 256 ? 1 : 0];
  if (r == 0) {
    int dev = 0, ncu = 0, per_cu = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev);
    if (e == hipSuccess)
      e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, reinterpret_cast<const void*>(persistent_kernel(ver, region)),
                                                       region, 0);
    if (e != hipSuccess) return e;
    if (ncu < 1 || per_cu < 1) return hipErrorInvalidConfiguration;
    r = ncu * per_cu;
  }
  *out = r;
  return hipSuccess;
}

// Enqueues nsteps steps of every instance: the line instances as
// ceil(nsteps / h) temporal-blocking launches starting from buffer
// start_cur; the tiled instances with walls or the flux-limited scheme as
// one launch per step and group starting from buffer start_cur2; the plain
// tiled instances from buffer start_cur3, one launch per step, or in pair
// mode two launches (two-step tiles, then the one-step tiles for instances
// with one step left) per pair of steps. `what` selects lines (1), tiled
// instances (2) or both.
static hipError_t enqueue_steps(lbm_batch* b, int64_t nsteps, int start_cur, int start_cur2, int start_cur3,
                                hipStream_t stream, int what = 3) {
  int cur = start_cur;
  const bool lines = (what & 1) && b->vend[3] > b->vbegin[1];
  if (lines && b->persistent) {
    // one launch per version runs every block; afterwards the lines' state
    // is where ceil(nsteps / h) one-block launches would have left it
    for (int ver = 1; ver <= 3; ++ver) {
      const int nc = b->vend[ver] - b->vbegin[ver];
      if (nc == 0) continue;
      int cap = 0;
      hipError_t e = resident_workgroups(b, ver, b->sched.region, &cap);
      if (e != hipSuccess) return e;
      hipLaunchKernelGGL(k_persist_reset, dim3((nc + 255) / 256), dim3(256), 0, stream, b->ctr,
                         b->epoch + b->vbegin[ver], nc);
      hipLaunchKernelGGL(persistent_kernel(ver, b->sched.region), dim3(std::min(nc, cap)), dim3(b->sched.region), 0,
                         stream, b->arena[start_cur], b->arena[start_cur ^ 1], b->insts, b->chunks + b->vbegin[ver],
                         nc, b->budget, (int)nsteps, b->sched.h, b->epoch + b->vbegin[ver], b->flag,
                         b->timeout_ticks);
      e = hipGetLastError();
      if (e != hipSuccess) return e;
    }
  }
  for (int64_t n0 = 0; lines && !b->persistent && n0 < nsteps; n0 += b->sched.h) {
    const int h = (int)std::min<int64_t>(b->sched.h, nsteps - n0);
    for (int ver = 1; ver <= 3; ++ver) {
      const int nc = b->vend[ver] - b->vbegin[ver];
      if (nc == 0) continue;
      const LineChunk* c = b->chunks + b->vbegin[ver];
      const double* A = b->arena[cur];
      double* B = b->arena[cur ^ 1];
      const bool big = b->sched.region == 256;
#define LBM_LAUNCH(V)                                                                              \
  if (big)                                                                                         \
    launch_line<V, 256>(A, B, b->insts, c, nc, b->budget, (int)n0, h, b->flag, stream);            \
  else                                                                                             \
    launch_line<V, 128>(A, B, b->insts, c, nc, b->budget, (int)n0, h, b->flag, stream);
      if (ver == 1) {
        LBM_LAUNCH(1)
      } else if (ver == 2) {
        LBM_LAUNCH(2)
      } else {
        LBM_LAUNCH(3)
      }
#undef LBM_LAUNCH
      hipError_t e = hipGetLastError();
      if (e != hipSuccess) return e;
    }
    cur ^= 1;
  }
  auto one_step_kernel = [](int ver, int w) {
    if (w == 1) return ver == 2 ? k_batch_tiles<2, true, 1> : ver == 3 ? k_batch_tiles<3, true, 1> : k_batch_tiles<1, true, 1>;
    if (w == 2)
      return ver == 2 ? k_batch_tiles<2, false, 2> : ver == 3 ? k_batch_tiles<3, false, 2> : k_batch_tiles<1, false, 2>;
    return ver == 2 ? k_batch_tiles<2, false, 1> : ver == 3 ? k_batch_tiles<3, false, 1> : k_batch_tiles<1, false, 1>;
  };
  auto launch_tiles = [&](int ver, int w, int c, int64_t n, int pairs) -> hipError_t {
    const int entries = b->tend[ver][w] - b->tbegin[ver][w];
    if (entries == 0) return hipSuccess;
    const int per_xcd = entries / 8;
    hipLaunchKernelGGL(one_step_kernel(ver, w), dim3(8 * per_xcd), dim3(64 * WAVES), 0, stream, b->arena[c],
                       b->arena[c ^ 1], b->tinsts, b->tile_inst + b->tbegin[ver][w], per_xcd, b->budget, (int)n,
                       (int)nsteps, pairs, b->flag);
    return hipGetLastError();
  };
  const bool tiled = (what & 2) && b->ntiles > 0;
  // tiled instances with walls or the flux-limited scheme, and the plain ones
  // when not in pair mode: one launch per step and group
  int cur2 = start_cur2, cur3 = start_cur3;
  for (int64_t n = 0; tiled && n < nsteps; ++n) {
    for (int ver = 1; ver <= 3; ++ver)
      for (int w = 0; w < 3; ++w) {
        if (w == 0 && b->pairs) continue;
        hipError_t e = launch_tiles(ver, w, w == 0 ? cur3 : cur2, n, 0);
        if (e != hipSuccess) return e;
      }
    cur2 ^= 1;
    if (!b->pairs) cur3 ^= 1;
  }
  // pair mode: the plain tiled instances two steps per launch. The budgets
  // are known here, so a launch with nothing to do is left out (a change of
  // budgets drops the cached graphs).
  for (int64_t n = 0; tiled && b->pairs && n < nsteps; n += 2) {
    for (int ver = 1; ver <= 3; ++ver) {
      bool two = false, one = false;
      for (const TileInst& T : b->host_tinsts) {
        const lbm_params& p = b->params[T.gidx];
        if (p.eq_version != ver || tile_variant(p) != 0) continue;
        const int64_t m = std::min<int64_t>(b->host_budget[T.gidx], nsteps);
        const int64_t done = (m + 1) / 2, total = (nsteps + 1) / 2;
        if (n + 2 <= m) two = true;
        else if (n + 1 == m || (n == 2 * done && ((total - done) & 1))) one = true;
      }
      const int entries = b->t2end[ver] - b->t2begin[ver];
      if (two && entries > 0) {
        const int per_xcd = entries / 8;
        auto k2 = ver == 2 ? k_batch_tiles2<2> : ver == 3 ? k_batch_tiles2<3> : k_batch_tiles2<1>;
        hipLaunchKernelGGL(k2, dim3(8 * per_xcd), dim3(128), 0, stream, b->arena[cur3], b->arena[cur3 ^ 1], b->tinsts,
                           b->tile_inst2 + b->t2begin[ver], per_xcd, b->budget, (int)n, (int)nsteps, b->flag);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
      }
      if (one) {
        hipError_t e = launch_tiles(ver, 0, cur3, n, 1);
        if (e != hipSuccess) return e;
      }
    }
    cur3 ^= 1;
  }
  return hipSuccess;
}

static int launches_for(const lbm_batch* b, int64_t nsteps) {
  return (int)((nsteps + b->sched.h - 1) / b->sched.h);
}

extern "C" {

size_t lbm_batch_workspace_bytes(const lbm_params* inst, int32_t n) {
  Layout L;
  if (layout_of(inst, n, &L) != LBM_OK) return 0;
  return L.total;
}

lbm_status lbm_batch_create(const lbm_params* inst, int32_t n, void* d_workspace, size_t ws_bytes, void* hip_stream,
                            lbm_batch** out) {
  if (!out) return fail(LBM_EINVAL, "out is NULL");
  *out = nullptr;
  Layout L;
  lbm_status st = layout_of(inst, n, &L);
  if (st != LBM_OK) return st;
  if (!d_workspace || ((uintptr_t)d_workspace) % 256) return fail(LBM_EINVAL, "workspace must be 256-byte aligned");
  if (ws_bytes < L.total) return fail(LBM_ENOMEM, "workspace has %zu bytes, needs %zu", ws_bytes, L.total);
  lbm_batch* b = new (std::nothrow) lbm_batch;
  if (!b) return fail(LBM_ENOMEM, "host allocation failed");
  b->n = n;
  b->params.assign(inst, inst + n);
  b->stream = (hipStream_t)hip_stream;
  char* base = (char*)d_workspace;
  b->arena[0] = (double*)base;
  b->arena[1] = (double*)(base + L.arena_bytes);
  b->insts = (LineInst*)(base + L.insts_off);
  b->chunks = (LineChunk*)(base + L.chunks_off);
  b->epoch = (int*)(base + L.epoch_off);
  b->tinsts = (TileInst*)(base + L.tinsts_off);
  b->tile_inst = (int2*)(base + L.tiles_off);
  b->tile_inst2 = (int2*)(base + L.tiles2_off);
  b->budget = (int*)(base + L.budget_off);
  b->flag = (int*)(base + L.flag_off);
  b->ctr = (unsigned long long*)(base + L.flag_off + 128);
  b->persistent = 0;
  std::memset(b->resident, 0, sizeof(b->resident));
  b->backup = (double*)(base + L.backup_off);
  b->max_chunks = L.max_chunks;
  b->arena_doubles = L.arena_doubles;
  b->ntiles = 0;
  b->max_tiles = L.ntiles + 72;
  b->tile_rows = 0;
  b->ntiles2 = 0;
  b->max_tiles2 = L.ntiles2 + 24;
  b->host_budget.assign(n, INT_MAX);
  b->tile_rows2 = 0;
  b->pairs = 0;
  b->cur = 0;
  b->cur2 = 0;
  b->cur3 = 0;
  b->use_graph = 1;
  for (int k = 0; k < 8; ++k) {
    b->graph[k] = nullptr;
    b->graph_steps[k] = -1;
  }
  b->capture = nullptr;
  {
    int dev = 0, khz = 0;
    if (hipGetDevice(&dev) != hipSuccess || hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev) != hipSuccess ||
        khz < 1) {
      delete b;
      return hip_fail(hipGetLastError(), "reading the wall-clock rate");
    }
    b->timeout_ticks = (long long)(DEFAULT_BARRIER_TIMEOUT_MS * khz);
  }
  if (hipStreamCreateWithFlags(&b->capture, hipStreamNonBlocking) != hipSuccess) {
    delete b;
    return hip_fail(hipGetLastError(), "creating the capture stream");
  }
  b->host_insts.resize(n);
  b->node_off.resize(n);
  b->tiled.assign(n, 0);
  b->tindex.assign(n, -1);
  long long node = 0;
  for (int i = 0; i < n; ++i) {
    const lbm_params& p = inst[i];
    LineInst& I = b->host_insts[i];
    std::memset(&I, 0, sizeof(I));
    b->node_off[i] = node;
    node += line_len(p);
    if (!is_line(p)) {
      b->tiled[i] = 1;
      b->tindex[i] = (int)b->host_tinsts.size();
      TileInst T;
      std::memset(&T, 0, sizeof(T));
      T.off = L.off[i];
      T.pitch = row_pitch(p.nx);
      T.plane = T.pitch * p.ny;
      T.nx = p.nx;
      T.ny = p.ny;
      T.gidx = i;
      make_coef(&p, &T.hot, &T.cold);
      b->host_tinsts.push_back(T);
      continue;
    }
    I.N = (int)line_len(p);
    I.stride = (I.N + 15) / 16 * 16;
    I.off = L.off[i];
    I.axis = (p.ny == 1 && p.nx > 1) ? 0 : 1;
    I.walls = has_walls(&p) ? 1 : 0;
    make_coef(&p, &I.hot, &I.cold);
  }
  b->total_nodes = node;
  std::vector<int> budget(n, INT_MAX);
  hipError_t e = hipMemcpyAsync(b->insts, b->host_insts.data(), n * sizeof(LineInst), hipMemcpyHostToDevice, b->stream);
  if (e == hipSuccess) e = hipMemcpyAsync(b->budget, budget.data(), n * sizeof(int), hipMemcpyHostToDevice, b->stream);
  if (e == hipSuccess) e = hipMemsetAsync(b->flag, 0, STATUS_BYTES, b->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
  if (e != hipSuccess) {
    (void)hipStreamDestroy(b->capture);
    delete b;
    return hip_fail(e, "uploading the batch description");
  }
  st = build_chunks(b, Schedule{256, 16});
  if (st == LBM_OK) st = build_tiles(b, L.rows);
  if (st == LBM_OK) st = build_tiles2(b, batch_tile_rows2(b));
  if (st != LBM_OK) {
    (void)hipStreamDestroy(b->capture);
    delete b;
    return st;
  }
  *out = b;
  clear_error();
  return LBM_OK;
}

int64_t lbm_batch_offset(const lbm_batch* b, int32_t i) {
  if (!b || i < 0 || i > b->n) return -1;
  return i == b->n ? b->total_nodes : b->node_off[i];
}

// Field view of instance i in arena buffer buf.
static Field field_of(const lbm_batch* b, int i, int buf) {
  const lbm_params& p = b->params[i];
  Field F;
  F.nx = p.nx;
  F.ny = p.ny;
  double* base;
  if (b->tiled[i]) {
    const TileInst& T = b->host_tinsts[b->tindex[i]];
    base = b->arena[buf] + T.off;
    F.pitch = T.pitch;
    F.plane = T.plane;
  } else {
    const LineInst& I = b->host_insts[i];
    base = b->arena[buf] + I.off;
    F.pitch = p.nx;
    F.plane = I.stride;
  }
  F.fin = base;
  F.fout = base;
  return F;
}

// Buffer holding the current state of instance i.
static int current_buf(const lbm_batch* b, int i) {
  if (!b->tiled[i]) return b->cur;
  return tile_variant(b->params[i]) == 0 ? b->cur3 : b->cur2;
}

lbm_status lbm_batch_init(lbm_batch* b, const double* d_rho, const double* d_ux, const double* d_uy,
                          const double* d_T) {
  if (!b || !d_rho || !d_ux || !d_uy || !d_T) return fail(LBM_EINVAL, "NULL argument");
  for (int i = 0; i < b->n; ++i) {
    const lbm_params& p = b->params[i];
    const long long k = b->node_off[i];
    for (int buf = 0; buf < 2; ++buf) {
      Field F = field_of(b, i, buf);
      F.fin = nullptr;
      dim3 grid((p.nx + 63) / 64, p.ny);
      auto kern = p.eq_version == 2 ? k_init<2> : p.eq_version == 3 ? k_init<3> : k_init<1>;
      hipLaunchKernelGGL(kern, grid, dim3(64), 0, b->stream, F, d_rho + k, d_ux + k, d_uy + k, d_T + k);
    }
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(e, "k_init launch");
  b->cur = 0;
  b->cur2 = 0;
  b->cur3 = 0;
  return LBM_OK;
}

lbm_status lbm_batch_set_budgets(lbm_batch* b, const int64_t* steps) {
  if (!b) return fail(LBM_EINVAL, "batch is NULL");
  std::vector<int> budget(b->n, INT_MAX);
  if (steps)
    for (int i = 0; i < b->n; ++i) {
      if (steps[i] < 0) return fail(LBM_EINVAL, "budget of instance %d is negative", i);
      budget[i] = (int)std::min<int64_t>(steps[i], INT_MAX);
    }
  hipError_t e = hipMemcpyAsync(b->budget, budget.data(), b->n * sizeof(int), hipMemcpyHostToDevice, b->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
  if (e != hipSuccess) return hip_fail(e, "uploading budgets");
  b->host_budget = budget;
  drop_graphs(b);  // the pair-mode launches depend on the budgets
  return LBM_OK;
}

lbm_status lbm_batch_step(lbm_batch* b, int64_t nsteps) {
  if (!b) return fail(LBM_EINVAL, "batch is NULL");
  if (nsteps < 0 || nsteps > INT_MAX) return fail(LBM_EINVAL, "nsteps out of range");
  if (nsteps == 0) return LBM_OK;
  const int L = launches_for(b, nsteps);
  if (!b->use_graph) {
    hipError_t e = enqueue_steps(b, nsteps, b->cur, b->cur2, b->cur3, b->stream);
    if (e != hipSuccess) return hip_fail(e, "batched step launch");
  } else {
    const int c = b->cur + 2 * b->cur2 + 4 * b->cur3;
    if (b->graph_steps[c] != nsteps) {
      if (b->graph[c]) (void)hipGraphExecDestroy(b->graph[c]);
      b->graph[c] = nullptr;
      if (b->persistent) {  // occupancy queries outside the capture
        int32_t grid = 0;
        lbm_status st = lbm_batch_get_persistent(b, nullptr, &grid);
        if (st != LBM_OK) return st;
      }
      hipGraph_t g = nullptr;
      hipError_t e = hipStreamBeginCapture(b->capture, hipStreamCaptureModeThreadLocal);
      if (e != hipSuccess) return hip_fail(e, "hipStreamBeginCapture");
      e = enqueue_steps(b, nsteps, b->cur, b->cur2, b->cur3, b->capture);
      hipError_t e2 = hipStreamEndCapture(b->capture, &g);
      if ((e != hipSuccess || e2 != hipSuccess) && g) (void)hipGraphDestroy(g);
      if (e != hipSuccess) return hip_fail(e, "capturing the batched steps");
      if (e2 != hipSuccess) return hip_fail(e2, "hipStreamEndCapture");
      e = hipGraphInstantiate(&b->graph[c], g, nullptr, nullptr, 0);
      (void)hipGraphDestroy(g);
      if (e != hipSuccess) {
        b->graph[c] = nullptr;
        return hip_fail(e, "hipGraphInstantiate");
      }
      b->graph_steps[c] = nsteps;
    }
    hipError_t e = hipGraphLaunch(b->graph[c], b->stream);
    if (e != hipSuccess) return hip_fail(e, "hipGraphLaunch");
  }
  if (L & 1) b->cur ^= 1;
  if (nsteps & 1) b->cur2 ^= 1;
  if ((b->pairs ? (nsteps + 1) / 2 : nsteps) & 1) b->cur3 ^= 1;
  return LBM_OK;
}

lbm_status lbm_batch_moments(lbm_batch* b, double* d_rho, double* d_ux, double* d_uy, double* d_T, double* d_p) {
  if (!b) return fail(LBM_EINVAL, "batch is NULL");
  for (int i = 0; i < b->n; ++i) {
    const lbm_params& p = b->params[i];
    const long long k = b->node_off[i];
    Field F = field_of(b, i, current_buf(b, i));
    F.fout = nullptr;
    dim3 grid((p.nx + 63) / 64, p.ny);
    hipLaunchKernelGGL(k_moments<0>, grid, dim3(64), 0, b->stream, F, d_rho ? d_rho + k : nullptr,
                       d_ux ? d_ux + k : nullptr, d_uy ? d_uy + k : nullptr, d_T ? d_T + k : nullptr,
                       d_p ? d_p + k : nullptr);
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(e, "k_moments launch");
  return LBM_OK;
}

lbm_status lbm_batch_get_f(lbm_batch* b, double* d_f) {
  if (!b || !d_f) return fail(LBM_EINVAL, "NULL argument");
  for (int i = 0; i < b->n; ++i) {
    const lbm_params& p = b->params[i];
    const Field F = field_of(b, i, current_buf(b, i));
    // source rows: 16 planes of ny rows (plane = ny * pitch for tiled
    // instances, one row of nx = N nodes per plane for lines)
    const size_t rows = b->tiled[i] ? (size_t)16 * p.ny : 16;
    const size_t width = b->tiled[i] ? (size_t)p.nx : (size_t)line_len(p);
    const size_t spitch = b->tiled[i] ? (size_t)F.pitch : (size_t)F.plane;
    hipError_t e = hipMemcpy2DAsync(d_f + 16 * b->node_off[i], width * sizeof(double), F.fin, spitch * sizeof(double),
                                    width * sizeof(double), rows, hipMemcpyDeviceToDevice, b->stream);
    if (e != hipSuccess) return hip_fail(e, "hipMemcpy2DAsync");
  }
  return LBM_OK;
}

lbm_status lbm_batch_set_schedule(lbm_batch* b, int32_t region, int32_t steps_per_launch, int32_t use_graph) {
  if (!b) return fail(LBM_EINVAL, "batch is NULL");
  Schedule s{region, steps_per_launch};
  if (!schedule_ok(s))
    return fail(LBM_EINVAL, "schedule needs region in {128, 256} and region - 2 h >= %d", MIN_CHUNK);
  b->use_graph = use_graph ? 1 : 0;
  return build_chunks(b, s);
}

lbm_status lbm_batch_get_schedule(const lbm_batch* b, int32_t* region, int32_t* steps_per_launch,
                                  int32_t* nchunks) {
  if (!b) return fail(LBM_EINVAL, "batch is NULL");
  if (region) *region = b->sched.region;
  if (steps_per_launch) *steps_per_launch = b->sched.h;
  if (nchunks) *nchunks = b->vend[3] - b->vbegin[1];
  return LBM_OK;
}

lbm_status lbm_batch_set_persistent(lbm_batch* b, int32_t persistent, double timeout_ms) {
  if (!b) return fail(LBM_EINVAL, "batch is NULL");
  if (persistent != 0 && persistent != 1) return fail(LBM_EINVAL, "persistent must be 0 or 1");
  if (!(timeout_ms >= 0.0) || timeout_ms > 60000.0) return fail(LBM_EINVAL, "timeout_ms must be in [0, 60000]");
  int dev = 0, khz = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e == hipSuccess) e = hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev);
  if (e != hipSuccess) return hip_fail(e, "reading the wall-clock rate");
  b->persistent = persistent;
  b->timeout_ticks = (long long)(timeout_ms * khz);
  drop_graphs(b);
  return LBM_OK;
}

lbm_status lbm_batch_get_persistent(lbm_batch* b, int32_t* persistent, int32_t* grid) {
  if (!b) return fail(LBM_EINVAL, "batch is NULL");
  if (persistent) *persistent = b->persistent;
  if (grid) {
    int g = 0;
    for (int ver = 1; ver <= 3; ++ver) {
      const int nc = b->vend[ver] - b->vbegin[ver];
      if (nc == 0) continue;
      int cap = 0;
      hipError_t e = resident_workgroups(b, ver, b->sched.region, &cap);
      if (e != hipSuccess) return hip_fail(e, "occupancy query");
      g = std::max(g, std::min(nc, cap));
    }
    *grid = g;
  }
  return LBM_OK;
}

lbm_status lbm_batch_tune(lbm_batch* b, int64_t probe_steps, double* best_ms) {
  if (!b) return fail(LBM_EINVAL, "batch is NULL");
  if (probe_steps < 1) return fail(LBM_EINVAL, "probe_steps must be >= 1");
  // an error left by earlier calls is reported (and cleared) as lbm_batch_check
  // does, before the trials, whose own status words are then discarded
  lbm_status pending = lbm_batch_check(b);
  if (pending != LBM_OK) return pending;
  // keep the current state: every trial runs from a backup copy
  const size_t bytes = (size_t)b->arena_doubles * sizeof(double);
  // (the schedule concerns the line instances only; the trials leave the
  // tiled instances alone)
  hipError_t e = hipMemcpyAsync(b->backup, b->arena[b->cur], bytes, hipMemcpyDeviceToDevice, b->stream);
  if (e != hipSuccess) return hip_fail(e, "backing up the state");
  const int saved_cur = b->cur;
  hipEvent_t t0 = nullptr, t1 = nullptr;
  e = hipEventCreate(&t0);
  if (e == hipSuccess) e = hipEventCreate(&t1);
  if (e != hipSuccess) {
    if (t0) (void)hipEventDestroy(t0);
    return hip_fail(e, "hipEventCreate");
  }
  Schedule best{256, 16};
  int best_pers = b->persistent;
  float best_t = 1e30f;
  const int regions[2] = {128, 256};
  const int hs[6] = {4, 8, 12, 16, 24, 32};
  struct Trial {
    Schedule s;
    int pers;
  };
  std::vector<Trial> trials;
  for (int r : regions)
    for (int h : hs)
      for (int pers = 0; pers < 2; ++pers)
        if (schedule_ok(Schedule{r, h})) trials.push_back(Trial{Schedule{r, h}, pers});
  const bool any_line = b->vend[3] > b->vbegin[1];
  for (const Trial& tr : trials) {
    if (!any_line) break;  // no line instances: nothing to choose
    if (build_chunks(b, tr.s) != LBM_OK) continue;
    b->persistent = tr.pers;
    // warm-up + timed trial, both without graphs
    // at least 8 blocks per trial, so that what happens between blocks
    // (launch gaps, or the persistent form's waits) is weighed; the time is
    // scaled back to probe_steps steps
    const int64_t probe = std::max<int64_t>(probe_steps, 8 * (int64_t)tr.s.h);
    e = enqueue_steps(b, std::min<int64_t>(probe, 2 * tr.s.h), b->cur, b->cur2, b->cur3, b->stream, 1);
    if (e == hipSuccess) e = hipEventRecord(t0, b->stream);
    if (e == hipSuccess) e = enqueue_steps(b, probe, b->cur, b->cur2, b->cur3, b->stream, 1);
    if (e == hipSuccess) e = hipEventRecord(t1, b->stream);
    if (e == hipSuccess) e = hipEventSynchronize(t1);
    if (e != hipSuccess) break;
    float ms = 0;
    e = hipEventElapsedTime(&ms, t0, t1);
    if (e != hipSuccess) break;
    ms *= (float)probe_steps / (float)probe;
    if (ms < best_t) {
      best_t = ms;
      best = tr.s;
      best_pers = tr.pers;
    }
    // restore the state for the next trial
    e = hipMemcpyAsync(b->arena[saved_cur], b->backup, bytes, hipMemcpyDeviceToDevice, b->stream);
    if (e != hipSuccess) break;
  }
  (void)hipEventDestroy(t0);
  (void)hipEventDestroy(t1);
  if (!any_line) best_t = 0.0f;
  if (e == hipSuccess) e = hipMemcpyAsync(b->arena[saved_cur], b->backup, bytes, hipMemcpyDeviceToDevice, b->stream);
  int word[17] = {0};  // a timed-out wait in a trial voids the persistent form
  if (e == hipSuccess) e = hipMemcpyAsync(word, b->flag, sizeof(word), hipMemcpyDeviceToHost, b->stream);
  if (e == hipSuccess) e = hipMemsetAsync(b->flag, 0, STATUS_BYTES, b->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
  if (e != hipSuccess) return hip_fail(e, "tuning run");
  if (word[16]) return fail(LBM_ETIMEOUT, "a wait of a persistent trial timed out");
  b->cur = saved_cur;
  b->persistent = best_pers;
  lbm_status st = build_chunks(b, best);
  if (st != LBM_OK) return st;
  if (b->host_tinsts.empty()) {
    if (best_ms) *best_ms = best_t;
    return LBM_OK;
  }
  // tile shapes of the tiled instances, timed the same way on their state:
  // one step per launch at each tile height, then (with plain tiled
  // instances) two steps per launch at each two-step tile height. First the
  // plain instances' state is moved into the others' buffer, so that one
  // arena holds the whole tiled state.
  e = hipSuccess;
  bool any_plain = false;
  for (const TileInst& T : b->host_tinsts) {
    if (tile_variant(b->params[T.gidx]) != 0) continue;
    any_plain = true;
    if (b->cur3 != b->cur2 && e == hipSuccess)
      e = hipMemcpyAsync(b->arena[b->cur2] + T.off, b->arena[b->cur3] + T.off, (size_t)16 * T.plane * sizeof(double),
                         hipMemcpyDeviceToDevice, b->stream);
  }
  if (e != hipSuccess) return hip_fail(e, "aligning the tiled state");
  b->cur3 = b->cur2;
  const int saved_cur2 = b->cur2;
  const int saved_pairs = b->pairs;
  t0 = t1 = nullptr;
  e = hipMemcpyAsync(b->backup, b->arena[saved_cur2], bytes, hipMemcpyDeviceToDevice, b->stream);
  if (e == hipSuccess) e = hipEventCreate(&t0);
  if (e == hipSuccess) e = hipEventCreate(&t1);
  if (e != hipSuccess) {
    if (t0) (void)hipEventDestroy(t0);
    return hip_fail(e, "backing up the state");
  }
  auto trial = [&](float* ms) -> hipError_t {
    hipError_t r = enqueue_steps(b, 2, b->cur, saved_cur2, saved_cur2, b->stream, 2);
    if (r == hipSuccess) r = hipEventRecord(t0, b->stream);
    if (r == hipSuccess) r = enqueue_steps(b, probe_steps, b->cur, saved_cur2, saved_cur2, b->stream, 2);
    if (r == hipSuccess) r = hipEventRecord(t1, b->stream);
    if (r == hipSuccess) r = hipEventSynchronize(t1);
    if (r == hipSuccess) r = hipEventElapsedTime(ms, t0, t1);
    if (r == hipSuccess) r = hipMemcpyAsync(b->arena[saved_cur2], b->backup, bytes, hipMemcpyDeviceToDevice, b->stream);
    return r;
  };
  int best_rows = b->tile_rows, best_rows2 = b->tile_rows2, best_pairs = 0;
  float best_tt = 1e30f;
  const int heights[5] = {8, 16, 32, 64, 128};
  b->pairs = 0;
  for (int rows : heights) {
    if (build_tiles(b, rows) != LBM_OK) continue;
    float ms = 0;
    e = trial(&ms);
    if (e != hipSuccess) break;
    if (ms < best_tt) {
      best_tt = ms;
      best_rows = rows;
    }
  }
  if (e == hipSuccess && any_plain && build_tiles(b, best_rows) == LBM_OK) {
    b->pairs = 1;
    const int heights2[7] = {8, 16, 24, 32, 48, 64, 128};
    for (int rows : heights2) {
      if (build_tiles2(b, rows) != LBM_OK) continue;
      float ms = 0;
      e = trial(&ms);
      if (e != hipSuccess) break;
      if (ms < best_tt) {
        best_tt = ms;
        best_rows2 = rows;
        best_pairs = 1;
      }
    }
  }
  (void)hipEventDestroy(t0);
  (void)hipEventDestroy(t1);
  b->pairs = saved_pairs;
  if (e == hipSuccess) e = hipMemcpyAsync(b->arena[saved_cur2], b->backup, bytes, hipMemcpyDeviceToDevice, b->stream);
  if (e == hipSuccess) e = hipMemsetAsync(b->flag, 0, sizeof(int), b->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
  if (e != hipSuccess) return hip_fail(e, "tuning run");
  b->cur2 = saved_cur2;
  b->cur3 = saved_cur2;
  if (best_ms) *best_ms = best_t + best_tt;
  lbm_status st2 = build_tiles(b, best_rows);
  if (st2 == LBM_OK) st2 = build_tiles2(b, best_rows2);
  if (st2 == LBM_OK) b->pairs = best_pairs;
  return st2;
}

lbm_status lbm_batch_set_tile_rows(lbm_batch* b, int32_t rows) {
  if (!b) return fail(LBM_EINVAL, "batch is NULL");
  if (rows < WAVES || rows > 4096 || rows % WAVES)
    return fail(LBM_EINVAL, "tile rows must be a multiple of %d in [%d, 4096]", WAVES, WAVES);
  return build_tiles(b, rows);
}

lbm_status lbm_batch_set_two_step(lbm_batch* b, int32_t on, int32_t rows) {
  if (!b) return fail(LBM_EINVAL, "batch is NULL");
  if (on != 0 && on != 1) return fail(LBM_EINVAL, "on must be 0 or 1");
  if (rows < 2 || rows > 4096 || rows % 2) return fail(LBM_EINVAL, "two-step tile rows must be even, in [2, 4096]");
  lbm_status st = build_tiles2(b, rows);
  if (st != LBM_OK) return st;
  b->pairs = on;
  return LBM_OK;
}

lbm_status lbm_batch_get_two_step(const lbm_batch* b, int32_t* on, int32_t* rows, int32_t* ntiles) {
  if (!b) return fail(LBM_EINVAL, "batch is NULL");
  if (on) *on = b->pairs;
  if (rows) *rows = b->tile_rows2;
  if (ntiles) *ntiles = b->ntiles2;
  return LBM_OK;
}

lbm_status lbm_batch_get_tile_rows(const lbm_batch* b, int32_t* rows, int32_t* ntiles) {
  if (!b) return fail(LBM_EINVAL, "batch is NULL");
  if (rows) *rows = b->tile_rows;
  if (ntiles) *ntiles = b->ntiles;
  return LBM_OK;
}

lbm_status lbm_batch_check(lbm_batch* b) {
  if (!b) return fail(LBM_EINVAL, "batch is NULL");
  int word[17] = {0};  // flag at 0, err at 16
  hipError_t e = hipMemcpyAsync(word, b->flag, sizeof(word), hipMemcpyDeviceToHost, b->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
  if (e != hipSuccess) return hip_fail(e, "reading the health flag");
  const int flag = word[0];
  if (word[16]) {  // a wait timed out: clear the error word, the counters and the flag
    e = hipMemsetAsync(b->flag, 0, STATUS_BYTES, b->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
    if (e != hipSuccess) return hip_fail(e, "hipMemsetAsync");
    return fail(LBM_ETIMEOUT, "a wait of the persistent launch timed out; the state is invalid");
  }
  if (flag) {
    e = hipMemsetAsync(b->flag, 0, sizeof(int), b->stream);
    if (e != hipSuccess) return hip_fail(e, "hipMemsetAsync");
    return fail(LBM_ENONFINITE, "a batched step produced rho <= 0, T <= 0 or NaN");
  }
  return LBM_OK;
}

void lbm_batch_destroy(lbm_batch* b) {
  if (!b) return;
  drop_graphs(b);
  if (b->capture) (void)hipStreamDestroy(b->capture);
  delete b;
}

}  // extern "C"
