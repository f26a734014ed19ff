// C ABI of libsllbm (declarations and contracts in include/sllbm.h).
//
// Host side: argument validation, the set-up state machine, host tables
// (tables.cpp), device memory for tables and (unless bound) populations, and
// kernel launches (kernels.hip).  Set-up calls never touch the HIP runtime.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <limits>
#include <string>
#include <thread>
#include <vector>

#include "../../include/sllbm.h"
#include "curvilinear.hpp"
#include "launch.hpp"
#include "tables.hpp"

using namespace sllbm;

namespace {

constexpr int kTileRows = 4;          // rows per workgroup of the tiled kernel
constexpr int kTileCols = 64;         // columns per workgroup (one per lane)
constexpr int kMaxWindowCols = 128;   // widest staged source window

struct DeviceBuf {
  void *ptr = nullptr;
  size_t bytes = 0;
};

}  // namespace

struct sllbm_ctx {
  int device = 0;
  int fp32 = 0;
  int bf16x = 0;  // SLLBM_BF16X: float32 populations, bfloat16 matrix-core x-pass
  std::string err;
  hipStream_t stream = nullptr;

  VelocitySet vs = default_velocity_set();
  double cs = 1.0;  // the set's scale (Sec. II.B): physical velocities cs * xi
  int p = 0;
  bool glc = true;
  bool have_grid = false;
  Axis ax, ay;
  // mesh of bilinear cells (sllbm_init_grid_curvilinear); ax / ay then hold
  // the logical axes (unit cells), which give the node counts and periodicity
  bool curvi = false;
  CurviMesh mesh;
  std::vector<double> cX, cY;  // node coordinates [ny][nx]
  bool have_phys = false;
  double dt = 0, nu = 0, gamma = 1.4, Pr = 1.0, tau = 0, omega = 0, omega_pr = 0;
  int model = 0;
  int path = SLLBM_PATH_AUTO;
  int64_t check_interval = 0;

  // host tables (rebuilt when set-up changes)
  bool host_dirty = true;
  AxisTable xt[kQ1], yt[kQ1];
  std::vector<double> mx, my;
  std::vector<double> mnode;  // curvilinear mesh: node masses [ny][nx]
  int win_rows = 0, win_cols = 0;
  bool mfma_blocks_ok = false;
  std::vector<int32_t> ywin, yrel, xwin, xrel;
  int rows_tx = 0;  // row-segment path: segment width (0: unavailable)
  int ident_x = 0, ident_y = 0, ident_xT = 0, ident_yT = 0;  // identity tables, bit per component
  std::vector<int32_t> rows_xwin, rows_xrel;

  // adjoint: transposed tables, windows (built on first use)
  bool adj_dirty = true;
  AxisTable xtT[kQ1], ytT[kQ1];
  int taps_T = 0, win_rowsT = 0, win_colsT = 0, rows_txT = 0;
  std::vector<int32_t> rows_xwinT, rows_xrelT;
  DeviceBuf rows_xrelT_d, rows_xwinT_d;
  std::vector<int32_t> ywinT, yrelT, xwinT, xrelT;
  DeviceBuf xsrcT, xwT, ysrcT, ywT, yrelT_d, ywinT_d, xrelT_d, xwinT_d;

  // device
  bool dev_checked = false;
  bool dev_dirty = true;
  bool rec_dirty = true;
  DeviceBuf rows_xrel_d, rows_xwin_d;
  DeviceBuf mnode_d;
  DeviceBuf xsrc, xw, ysrc, yw, yrel_d, ywin_d, xrel_d, xwin_d, mxd, myd, flag, partial, scalar,
      macro;
  DeviceBuf rec_cell, rec;  // departure records (see DevTables)
  DeviceBuf adj_tmp;  // Pr != 1 adjoint step: S^T mu before the collision transpose
  DeviceBuf csr_ptr, csr_col, csr_w;  // curvilinear mesh: transposed records (DevTables)
  void *pop[2] = {nullptr, nullptr};
  bool own_pop = false;
  size_t pop_bytes = 0;
  int cur = 0;
  int layout = kPlanar;  // storage order (PopLayout) of pop[cur]
  bool initialised = false;
  int64_t steps_done = 0;
};

namespace {

int fail(sllbm_ctx *c, int code, const std::string &msg) {
  if (c) c->err = msg;
  return code;
}

#define HIP_TRY(ctx, expr)                                                        \
  do {                                                                            \
    hipError_t e_ = (expr);                                                       \
    if (e_ != hipSuccess)                                                         \
      return fail(ctx, e_ == hipErrorOutOfMemory ? SLLBM_E_OOM : SLLBM_E_DEVICE,  \
                  std::string(#expr) + ": " + hipGetErrorString(e_));             \
  } while (0)

bool is_finite(double v) { return std::isfinite(v); }

int nsets(const sllbm_ctx *c) { return c->model == SLLBM_POLYATOMIC ? 2 : 1; }
int q1(const sllbm_ctx *c) { return c->vs.q1; }             // 1-D velocities
int nvel(const sllbm_ctx *c) { return c->vs.q1 * c->vs.q1; }  // 2-D velocities
size_t pop_size(const sllbm_ctx *c) { return c->fp32 ? 4 : 8; }
long long nnodes(const sllbm_ctx *c) { return (long long)c->ax.n * c->ay.n; }

int ready_for_tables(sllbm_ctx *c) {
  if (c->p == 0) return fail(c, SLLBM_E_STATE, "interpolation order not set (sllbm_set_order)");
  if (!c->have_grid) return fail(c, SLLBM_E_STATE, "grid not set (sllbm_init_grid_*)");
  if (!c->have_phys) return fail(c, SLLBM_E_STATE, "physics not set (sllbm_set_physics)");
  return SLLBM_OK;
}

// Source windows of the tiled kernel along one axis.  For tile t (nodes
// [t*tile, min((t+1)*tile, n))) and 1-D velocity comp, the window starts at
// the smallest unwrapped source node of the tile's departure stencils; rel
// holds each node's stencil relative to its tile's window ([comp][m][node]).
// Unwrapped indices keep the window contiguous across a periodic seam.
// Returns the widest window.
int build_windows(const AxisTable *t, int nq1, int n, int tile, std::vector<int32_t> &win,
                  std::vector<int32_t> &rel, bool shared_moving = false) {
  const int taps = t[0].taps;
  const int ntiles = (n + tile - 1) / tile;
  win.assign(size_t(nq1) * ntiles, 0);
  rel.assign(size_t(nq1) * taps * n, 0);
  int width = 0;
  for (int a = 0; a < nq1; ++a) {
    // shared_moving: components 1 .. nq1-1 share one window per tile (the
    // union of their stencils)
    const int a0 = shared_moving && a > 0 ? 1 : a, a1 = shared_moving && a > 0 ? nq1 : a + 1;
    for (int k = 0; k < ntiles; ++k) {
      const int j0 = k * tile, j1 = std::min(j0 + tile, n);
      long lo = std::numeric_limits<long>::max(), hi = std::numeric_limits<long>::min();
      for (int b = a0; b < a1; ++b)
        for (int j = j0; j < j1; ++j) {
          lo = std::min(lo, t[b].start[j]);
          hi = std::max(hi, t[b].start[j] + taps - 1);
        }
      win[size_t(a) * ntiles + k] = int32_t(lo);
      width = std::max<int>(width, int(hi - lo + 1));
      for (int j = j0; j < j1; ++j)
        for (int m = 0; m < taps; ++m)
          rel[(size_t(a) * taps + m) * n + j] = int32_t(t[a].start[j] + m - lo);
    }
  }
  return width;
}

// The matrix-core x-pass covers each block of 16 target columns with
// 4 * ks staged columns starting at the stencil of the block's first column,
// ks = (16 + 2p + 3) / 4 (as in the kernel).
bool mfma_blocks_fit(const sllbm_ctx *c) {
  const int P1 = c->p + 1, n = c->ax.n;
  // float32: k-steps of 4 columns; bfloat16: one product of 32 columns
  const int K = c->bf16x ? 32 : 4 * ((16 + 2 * c->p + 3) / 4);
  for (int a = 0; a < q1(c); ++a)
    for (int n0 = 0; n0 < n; n0 += 16) {
      const int32_t base = c->xrel[(size_t(a) * P1) * n + n0];
      for (int j = n0; j < std::min(n0 + 16, n); ++j) {
        const int32_t st = c->xrel[(size_t(a) * P1) * n + j];
        if (st < base || st + c->p - base > K - 1) return false;
      }
    }
  return true;
}

// Widest row segment (at most 64 columns, at least kRowsMinCols) whose
// x-stencils fit 64 consecutive source columns for every segment and 1-D
// velocity; its windows go to win / rel.  0 when none does.
int rows_segment_width(const AxisTable *t, int nq1, int n, std::vector<int32_t> &win,
                       std::vector<int32_t> &rel, bool shared_moving = false) {
  int tx = 64;
  while (tx >= kRowsMinCols) {
    const int width = build_windows(t, nq1, n, tx, win, rel, shared_moving);
    if (width <= 64) return tx;
    tx -= width - 64;
  }
  win.clear();
  rel.clear();
  return 0;
}

// Departure records (cell cx | cy << 16, reference coordinates r, s) of
// velocity i = a + 5 b for every node: from the axis tables, or located on
// the curvilinear mesh.  Returns "" or an error message.
std::string departure_records(const sllbm_ctx *c, int i, int32_t *cell, double *r, double *s) {
  const int a = i % q1(c), b = i / q1(c);
  if (c->curvi)
    return curvi_records(c->mesh, support_points(c->p, c->glc), c->cX, c->cY,
                         -c->dt * c->cs * c->vs.xi[a], -c->dt * c->cs * c->vs.xi[b], cell, r,
                         s);
  for (int iy = 0; iy < c->ay.n; ++iy)
    for (int ix = 0; ix < c->ax.n; ++ix) {
      const size_t k = size_t(iy) * c->ax.n + ix;
      cell[k] = int32_t(uint32_t(c->xt[a].cell[ix]) | (uint32_t(c->yt[b].cell[iy]) << 16));
      r[k] = c->xt[a].rref[ix];
      s[k] = c->yt[b].rref[iy];
    }
  return "";
}

void build_host_tables(sllbm_ctx *c) {
  if (!c->host_dirty) return;
  for (int a = 0; a < q1(c); ++a) {
    // departure x - dt xi with the physical velocity xi = cs xi_hat
    c->xt[a] = build_axis_table(c->ax, -c->dt * c->cs * c->vs.xi[a]);
    c->yt[a] = build_axis_table(c->ay, -c->dt * c->cs * c->vs.xi[a]);
  }
  c->mx = c->ax.node_mass();
  c->my = c->ay.node_mass();
  if (c->curvi) c->mnode = curvi_node_mass(c->mesh, support_points(c->p, c->glc));
  // windows of the tiled kernel: tiles of kTileCols columns by kTileRows rows
  c->win_rows = build_windows(c->yt, q1(c), c->ay.n, kTileRows, c->ywin, c->yrel);
  c->win_cols = build_windows(c->xt, q1(c), c->ax.n, kTileCols, c->xwin, c->xrel);
  c->mfma_blocks_ok = mfma_blocks_fit(c);
  // the forward step reads the moving x-components of a node with one wide
  // load, so they share a window per segment
  c->rows_tx = rows_segment_width(c->xt, q1(c), c->ax.n, c->rows_xwin, c->rows_xrel, true);
  c->ident_x = c->ident_y = 0;
  for (int b = 0; b < q1(c); ++b) {
    if (identity_table(c->xt[b], c->ax.n)) c->ident_x |= 1 << b;
    if (identity_table(c->yt[b], c->ay.n)) c->ident_y |= 1 << b;
  }
  if (!(c->ident_x & c->ident_y & 1)) c->rows_tx = 0;  // the row-segment kernels need xi_0 = 0
  c->host_dirty = false;
  c->dev_dirty = true;
  c->rec_dirty = true;
}

// The tiled kernel stages window rows (up to 3 per wavefront) of
// up to 128 columns; LDS always fits (one x-component per phase if need be).
bool tiled_fits(const sllbm_ctx *c) {
  return q1(c) == kQ1 && c->win_rows <= 3 * kTileRows && c->win_cols <= kMaxWindowCols;
}

// The matrix-core path: tiled windows, float32, at most 16 (set, row) pairs
// per window, every x-stencil block within the product's columns.
bool mfma_fits(const sllbm_ctx *c) {
  return tiled_fits(c) && c->fp32 && nsets(c) * c->win_rows <= 16 && c->mfma_blocks_ok;
}

// AUTO: the row-segment kernel where it measured faster than (or as fast
// as) the tiled one (1025^2-node grids, p = 1..4, every model, Pr = 1 and
// 0.75, FP32 and FP64): segments of at least 48 columns; then tiled, then
// direct.
bool rows_preferred(const sllbm_ctx *c) { return c->rows_tx >= 48; }

// (The 3-velocity set has row-segment, direct and records kernels only:
// tiled_fits is false for it.)
int effective_path(const sllbm_ctx *c) {
  if (c->bf16x && c->path == SLLBM_PATH_AUTO) return kPathMfma;  // the experiment's only kernel
  if (c->path != SLLBM_PATH_AUTO) return c->path;
  if (c->curvi) return kPathRecords;  // the only gather that takes arbitrary cells
  if (rows_preferred(c) || (!tiled_fits(c) && c->rows_tx >= kRowsMinCols)) return kPathRows;
  return tiled_fits(c) ? kPathTiled : kPathDirect;
}

void free_buf(DeviceBuf &b) {
  if (b.ptr) (void)hipFree(b.ptr);
  b.ptr = nullptr;
  b.bytes = 0;
}

int alloc_buf(sllbm_ctx *c, DeviceBuf &b, size_t bytes) {
  if (b.ptr && b.bytes >= bytes) return SLLBM_OK;
  free_buf(b);
  HIP_TRY(c, hipMalloc(&b.ptr, bytes > 0 ? bytes : 8));
  b.bytes = bytes;
  return SLLBM_OK;
}

template <typename V>
int upload(sllbm_ctx *c, DeviceBuf &b, const std::vector<V> &v) {
  int rc = alloc_buf(c, b, v.size() * sizeof(V));
  if (rc) return rc;
  HIP_TRY(c, hipMemcpy(b.ptr, v.data(), v.size() * sizeof(V), hipMemcpyHostToDevice));
  return SLLBM_OK;
}

// Weights in the population type.
int upload_weights(sllbm_ctx *c, DeviceBuf &b, const std::vector<double> &w) {
  if (!c->fp32) return upload(c, b, w);
  std::vector<float> f(w.begin(), w.end());
  return upload(c, b, f);
}

int check_device(sllbm_ctx *c) {
  if (!c->dev_checked) {
    int n = 0;
    hipError_t e = hipGetDeviceCount(&n);
    if (e != hipSuccess || n == 0)
      return fail(c, SLLBM_E_DEVICE, "no HIP device available");
    if (c->device < 0 || c->device >= n)
      return fail(c, SLLBM_E_ARG, "HIP device index out of range");
    c->dev_checked = true;
  }
  HIP_TRY(c, hipSetDevice(c->device));
  return SLLBM_OK;
}

// Per-axis tables in [comp][m][node] order.
template <typename V>
std::vector<V> comp_major(const AxisTable *t, int nq1, int n, int P1, bool weights) {
  std::vector<V> out(size_t(nq1) * P1 * n);
  for (int a = 0; a < nq1; ++a)
    for (int m = 0; m < P1; ++m)
      for (int j = 0; j < n; ++j)
        out[(size_t(a) * P1 + m) * n + j] =
            weights ? V(t[a].w[size_t(j) * P1 + m]) : V(t[a].src[size_t(j) * P1 + m]);
  return out;
}

int prepare_device(sllbm_ctx *c) {
  int rc = ready_for_tables(c);
  if (rc) return rc;
  rc = check_device(c);
  if (rc) return rc;
  build_host_tables(c);
  if (c->dev_dirty) {
    const int P1 = c->p + 1;
    const int nq1 = q1(c);
    rc = upload(c, c->xsrc, comp_major<int32_t>(c->xt, nq1, c->ax.n, P1, false));
    if (!rc) rc = upload_weights(c, c->xw, comp_major<double>(c->xt, nq1, c->ax.n, P1, true));
    if (!rc) rc = upload(c, c->ysrc, comp_major<int32_t>(c->yt, nq1, c->ay.n, P1, false));
    if (!rc) rc = upload_weights(c, c->yw, comp_major<double>(c->yt, nq1, c->ay.n, P1, true));
    if (!rc) rc = upload(c, c->yrel_d, c->yrel);
    if (!rc) rc = upload(c, c->ywin_d, c->ywin);
    if (!rc) rc = upload(c, c->xrel_d, c->xrel);
    if (!rc) rc = upload(c, c->xwin_d, c->xwin);
    if (!rc && c->rows_tx) rc = upload(c, c->rows_xrel_d, c->rows_xrel);
    if (!rc && c->rows_tx) rc = upload(c, c->rows_xwin_d, c->rows_xwin);
    if (!rc) rc = upload(c, c->mxd, c->mx);
    if (!rc) rc = upload(c, c->myd, c->my);
    if (!rc && c->curvi) rc = upload(c, c->mnode_d, c->mnode);
    if (!rc) rc = alloc_buf(c, c->flag, sizeof(int));
    if (!rc) rc = alloc_buf(c, c->scalar, 2 * sizeof(double));
    if (!rc) rc = alloc_buf(c, c->partial, sizeof(double) * (size_t(nnodes(c)) / 256 + 2));
    if (rc) return rc;
    c->dev_dirty = false;
  }
  if (effective_path(c) == kPathRecords && c->rec_dirty) {
    const long long N = nnodes(c);
    const int nq = nvel(c);
    std::vector<int32_t> cell(size_t(nq) * N);
    std::vector<double> r(size_t(nq) * N), s(size_t(nq) * N);
    // one velocity per task, over up to 16 host threads (locating departure
    // points on a curvilinear mesh takes ~0.5 s per velocity at 1e6 nodes)
    std::vector<std::string> errs(nq);
    const int nthreads =
        std::max(1, std::min({nq, 16, int(std::thread::hardware_concurrency())}));
    std::vector<std::thread> pool;
    for (int t = 0; t < nthreads; ++t)
      pool.emplace_back([&, t] {
        for (int i = t; i < nq; i += nthreads) {
          const size_t off = size_t(i) * N;
          errs[i] = departure_records(c, i, cell.data() + off, r.data() + off, s.data() + off);
        }
      });
    for (auto &th : pool) th.join();
    for (const auto &e : errs)
      if (!e.empty()) return fail(c, SLLBM_E_ARG, e);
    // one record per (velocity, node) in one stretch of memory, read with one
    // load (float32: {cell, r, s}, 12 bytes; float64: {r, s} with the cells
    // in a plane of their own): the shock-vortex records step took 1.04
    // against 1.05 ms with three separate planes
    const size_t nrec = size_t(nq) * N;
    if (c->fp32) {
      std::vector<uint32_t> rec(3 * nrec);
      for (size_t k = 0; k < nrec; ++k) {
        const float rf = float(r[k]), sf = float(s[k]);
        rec[3 * k] = uint32_t(cell[k]);
        std::memcpy(&rec[3 * k + 1], &rf, 4);
        std::memcpy(&rec[3 * k + 2], &sf, 4);
      }
      rc = upload(c, c->rec, rec);
    } else {
      std::vector<double> rs(2 * nrec);
      for (size_t k = 0; k < nrec; ++k) {
        rs[2 * k] = r[k];
        rs[2 * k + 1] = s[k];
      }
      rc = upload(c, c->rec_cell, cell);
      if (!rc) rc = upload(c, c->rec, rs);
    }
    if (rc) return rc;
    c->rec_dirty = false;
  }
  return SLLBM_OK;
}

StepConsts make_consts(const sllbm_ctx *c) {
  StepConsts k{};
  k.nx = c->ax.n;
  k.ny = c->ay.n;
  k.n = nnodes(c);
  k.ncx = c->ax.ncells;
  k.ncy = c->ay.ncells;
  k.p = c->p;
  k.omega = c->omega;
  k.omega_pr = c->omega_pr;
  const double D = kDim;
  double cv = D / 2.0;  // monatomic: C_v = D/2 (R = 1)
  if (c->model == SLLBM_POLYATOMIC) cv = 1.0 / (c->gamma - 1.0);
  k.gfac = 2.0 * cv - D;
  k.inv_2cv = 1.0 / (2.0 * cv);
  k.q1 = q1(c);
  k.cs = c->cs;
  k.inv_cs = 1.0 / c->cs;
  k.bf16x = c->bf16x;
  for (int a = 0; a < q1(c); ++a) {
    k.xi[a] = c->vs.xi[a];
    k.w[a] = c->vs.w[a];
    for (int j = 0; j < 5; ++j) {
      k.hk[a][j] = c->vs.hk[a][j];
      k.whk[a][j] = c->vs.w[a] * c->vs.hk[a][j];
    }
  }
  for (int m = 0; m <= c->p; ++m) {
    k.rn[m] = c->ax.r[m];
    double d = 1.0;
    for (int n = 0; n <= c->p; ++n)
      if (n != m) d *= (c->ax.r[m] - c->ax.r[n]);
    k.lden[m] = 1.0 / d;
  }
  k.perx = c->ax.periodic;
  k.pery = c->ay.periodic;
  k.layout = c->layout;
  return k;
}

DevTables make_tables(const sllbm_ctx *c) {
  DevTables t{};
  t.xsrc = static_cast<const int32_t *>(c->xsrc.ptr);
  t.xw = c->xw.ptr;
  t.ysrc = static_cast<const int32_t *>(c->ysrc.ptr);
  t.yw = c->yw.ptr;
  t.rec_cell = static_cast<const int32_t *>(c->rec_cell.ptr);
  t.rec = c->rec.ptr;
  t.mx = static_cast<const double *>(c->mxd.ptr);
  t.my = static_cast<const double *>(c->myd.ptr);
  t.mnode = c->curvi ? static_cast<const double *>(c->mnode_d.ptr) : nullptr;
  t.yrel = static_cast<const int32_t *>(c->yrel_d.ptr);
  t.ywin = static_cast<const int32_t *>(c->ywin_d.ptr);
  t.xrel = static_cast<const int32_t *>(c->xrel_d.ptr);
  t.xwin = static_cast<const int32_t *>(c->xwin_d.ptr);
  t.tile_rows = kTileRows;
  t.win_rows = c->win_rows;
  t.win_cols = c->win_cols;
  t.taps = c->p + 1;
  t.mfma_ok = c->mfma_blocks_ok ? 1 : 0;
  t.rows_tx = c->rows_tx;
  t.rows_xrel = c->rows_tx ? static_cast<const int32_t *>(c->rows_xrel_d.ptr) : nullptr;
  t.rows_xwin = c->rows_tx ? static_cast<const int32_t *>(c->rows_xwin_d.ptr) : nullptr;
  t.ident_x = c->ident_x;
  t.ident_y = c->ident_y;
  return t;
}

// Storage order a path streams: the row-segment step the grouped order
// (PopLayout), every other gather the planar one.
int path_layout(int path) { return path == kPathRows ? kGrouped : kPlanar; }

// Brings the state pop[cur] into `layout`, through the other buffer (which
// holds nothing between steps).
int to_layout(sllbm_ctx *c, int layout) {
  if (c->layout == layout) return SLLBM_OK;
  HIP_TRY(c, launch_relayout(c->fp32, nsets(c), make_consts(c), c->pop[c->cur],
                             c->pop[1 - c->cur], layout == kGrouped, c->stream));
  c->cur ^= 1;
  c->layout = layout;
  return SLLBM_OK;
}

int ensure_populations(sllbm_ctx *c) {
  const size_t bytes = size_t(nsets(c)) * nvel(c) * size_t(nnodes(c)) * pop_size(c);
  if (c->pop[0] && c->pop_bytes == bytes) return SLLBM_OK;
  if (c->pop[0] && !c->own_pop)
    return fail(c, SLLBM_E_STATE, "bound population buffers do not match the current set-up");
  if (c->own_pop) {
    (void)hipFree(c->pop[0]);
    (void)hipFree(c->pop[1]);
    c->pop[0] = c->pop[1] = nullptr;
  }
  HIP_TRY(c, hipMalloc(&c->pop[0], bytes));
  HIP_TRY(c, hipMalloc(&c->pop[1], bytes));
  c->own_pop = true;
  c->pop_bytes = bytes;
  return SLLBM_OK;
}

int clear_flag(sllbm_ctx *c) {
  HIP_TRY(c, launch_clear_flag(static_cast<int *>(c->flag.ptr), c->stream));
  return SLLBM_OK;
}

// tau = nu / (c_s^2 dt) + 1/2 (Sec. II.D) and tau_Pr = (tau - 1/2)/Pr + 1/2
// (omega_pr exactly omega when Pr = 1); nu = +inf: no collision.
void update_relaxation(sllbm_ctx *c) {
  if (!c->have_phys) return;
  const double nu = c->nu;
  c->tau = std::isinf(nu) ? std::numeric_limits<double>::infinity()
                          : nu / (c->cs * c->cs * c->dt) + 0.5;
  c->omega = std::isinf(nu) ? 0.0 : 1.0 / c->tau;
  c->omega_pr = (c->Pr == 1.0 || std::isinf(nu)) ? c->omega
                                                  : 1.0 / ((c->tau - 0.5) / c->Pr + 0.5);
}

int setup_allowed(sllbm_ctx *c) {
  if (!c) return SLLBM_E_ARG;
  if (c->initialised)
    return fail(c, SLLBM_E_STATE, "set-up cannot change after the populations are initialised");
  return SLLBM_OK;
}

void invalidate(sllbm_ctx *c) {
  c->host_dirty = true;
  c->dev_dirty = true;
  c->rec_dirty = true;
  c->adj_dirty = true;
}

// Extends every node of a table to `taps` entries (zero weights).
void pad_taps(AxisTable &t, const Axis &ax, int taps) {
  if (t.taps == taps) return;
  const int old = t.taps;
  std::vector<int32_t> src(size_t(ax.n) * taps);
  std::vector<double> w(size_t(ax.n) * taps, 0.0);
  for (int j = 0; j < ax.n; ++j)
    for (int q = 0; q < taps; ++q) {
      long v = t.start[j] + q;
      if (ax.periodic) {
        v %= ax.n;
        if (v < 0) v += ax.n;
      } else {
        v = std::min<long>(std::max<long>(v, 0), ax.n - 1);
      }
      src[size_t(j) * taps + q] = int32_t(v);
      if (q < old) w[size_t(j) * taps + q] = t.w[size_t(j) * old + q];
    }
  t.src.swap(src);
  t.w.swap(w);
  t.taps = taps;
}

// Transposed records gather of a curvilinear mesh: for every velocity i and
// source node j, the targets v whose departure stencil (the records' cell,
// p+1 x p+1 nodes) holds j, with the Lagrange weight l_m(r_v) l_n(s_v) of
// j in it.  Every target contributes (p+1)^2 entries, so velocity i's entries
// start at i N (p+1)^2; within a source node they are in target order.
int build_records_transpose(sllbm_ctx *c) {
  const long long N = nnodes(c);
  const int nq = nvel(c), P1 = c->p + 1, p = c->p;
  const int nx = c->ax.n, ny = c->ay.n;
  const uint64_t per_vel = uint64_t(N) * uint64_t(P1 * P1);
  if (per_vel * uint64_t(nq) > uint64_t(0xffffffffu))
    return fail(c, SLLBM_E_UNSUPPORTED,
                "curvilinear mesh too large for the adjoint's 32-bit transposed records");
  const std::vector<double> pts = support_points(p, c->glc);
  std::vector<uint32_t> ptr(size_t(nq) * size_t(N + 1));
  std::vector<int32_t> col(size_t(per_vel) * nq);
  std::vector<double> w(size_t(per_vel) * nq);
  std::vector<std::string> errs(nq);
  const int nthreads = std::max(1, std::min({nq, 16, int(std::thread::hardware_concurrency())}));
  std::vector<std::thread> pool;
  for (int t = 0; t < nthreads; ++t)
    pool.emplace_back([&, t] {
      std::vector<int32_t> cell(N);
      std::vector<double> r(N), s(N);
      std::vector<uint32_t> next(N);
      for (int i = t; i < nq; i += nthreads) {
        errs[i] = departure_records(c, i, cell.data(), r.data(), s.data());
        if (!errs[i].empty()) continue;
        auto node = [&](long long v, int m, int n) {  // as the records gather reads it
          const int32_t rec = cell[v];
          int jx = (rec & 0xffff) * p + m, jy = int(uint32_t(rec) >> 16) * p + n;
          if (jx >= nx) jx -= nx;
          if (jy >= ny) jy -= ny;
          return (long long)jy * nx + jx;
        };
        uint32_t *rp = ptr.data() + size_t(i) * size_t(N + 1);
        std::fill(rp, rp + N + 1, 0u);
        for (long long v = 0; v < N; ++v)
          for (int n = 0; n < P1; ++n)
            for (int m = 0; m < P1; ++m) ++rp[node(v, m, n) + 1];
        rp[0] = uint32_t(uint64_t(i) * per_vel);
        for (long long j = 0; j < N; ++j) rp[j + 1] += rp[j];
        for (long long j = 0; j < N; ++j) next[j] = rp[j];
        double lx[kMaxOrder + 1], ly[kMaxOrder + 1];
        for (long long v = 0; v < N; ++v) {
          lagrange_weights(pts, r[v], lx);
          lagrange_weights(pts, s[v], ly);
          for (int n = 0; n < P1; ++n)
            for (int m = 0; m < P1; ++m) {
              const uint32_t e = next[node(v, m, n)]++;
              col[e] = int32_t(v);
              w[e] = lx[m] * ly[n];
            }
        }
      }
    });
  for (auto &th : pool) th.join();
  for (const auto &e : errs)
    if (!e.empty()) return fail(c, SLLBM_E_ARG, e);
  int rc = upload(c, c->csr_ptr, ptr);
  if (!rc) rc = upload(c, c->csr_col, col);
  if (!rc) rc = upload_weights(c, c->csr_w, w);
  return rc;
}

int prepare_adjoint(sllbm_ctx *c) {
  int rc = prepare_device(c);
  if (rc) return rc;
  if (q1(c) != kQ1)
    return fail(c, SLLBM_E_UNSUPPORTED, "the adjoint covers the 5-velocity set (D2Q25) only");
  if (c->bf16x)
    return fail(c, SLLBM_E_UNSUPPORTED, "the adjoint differentiates the float32/float64 step");
  if (c->cs != 1.0)
    return fail(c, SLLBM_E_UNSUPPORTED, "the adjoint covers the unscaled velocity set (c_s = 1)");
  if (!c->adj_dirty) return SLLBM_OK;
  if (c->curvi) {  // the transposed records gather
    rc = build_records_transpose(c);
    if (rc) return rc;
    c->adj_dirty = false;
    return SLLBM_OK;
  }
  int taps = 0;
  for (int a = 0; a < kQ1; ++a) {
    c->xtT[a] = transpose_axis_table(c->ax, c->xt[a]);
    c->ytT[a] = transpose_axis_table(c->ay, c->yt[a]);
    taps = std::max({taps, c->xtT[a].taps, c->ytT[a].taps});
  }
  if (taps > 12) return fail(c, SLLBM_E_UNSUPPORTED, "transposed stencil wider than 12 nodes");
  for (int a = 0; a < kQ1; ++a) {
    pad_taps(c->xtT[a], c->ax, taps);
    pad_taps(c->ytT[a], c->ay, taps);
  }
  c->taps_T = taps;
  c->win_rowsT = build_windows(c->ytT, kQ1, c->ay.n, kTileRows, c->ywinT, c->yrelT);
  c->win_colsT = build_windows(c->xtT, kQ1, c->ax.n, kTileCols, c->xwinT, c->xrelT);
  c->rows_txT = rows_segment_width(c->xtT, kQ1, c->ax.n, c->rows_xwinT, c->rows_xrelT);
  c->ident_xT = c->ident_yT = 0;
  for (int b = 0; b < kQ1; ++b) {
    if (identity_table(c->xtT[b], c->ax.n)) c->ident_xT |= 1 << b;
    if (identity_table(c->ytT[b], c->ay.n)) c->ident_yT |= 1 << b;
  }
  if (!(c->ident_xT & c->ident_yT & 1)) c->rows_txT = 0;
  rc = upload(c, c->xsrcT, comp_major<int32_t>(c->xtT, kQ1, c->ax.n, taps, false));
  if (!rc) rc = upload_weights(c, c->xwT, comp_major<double>(c->xtT, kQ1, c->ax.n, taps, true));
  if (!rc) rc = upload(c, c->ysrcT, comp_major<int32_t>(c->ytT, kQ1, c->ay.n, taps, false));
  if (!rc) rc = upload_weights(c, c->ywT, comp_major<double>(c->ytT, kQ1, c->ay.n, taps, true));
  if (!rc) rc = upload(c, c->yrelT_d, c->yrelT);
  if (!rc) rc = upload(c, c->ywinT_d, c->ywinT);
  if (!rc) rc = upload(c, c->xrelT_d, c->xrelT);
  if (!rc) rc = upload(c, c->xwinT_d, c->xwinT);
  if (!rc && c->rows_txT) rc = upload(c, c->rows_xrelT_d, c->rows_xrelT);
  if (!rc && c->rows_txT) rc = upload(c, c->rows_xwinT_d, c->rows_xwinT);
  if (rc) return rc;
  c->adj_dirty = false;
  return SLLBM_OK;
}

DevTables make_adjoint_tables(const sllbm_ctx *c) {
  DevTables t{};
  t.xsrc = static_cast<const int32_t *>(c->xsrcT.ptr);
  t.xw = c->xwT.ptr;
  t.ysrc = static_cast<const int32_t *>(c->ysrcT.ptr);
  t.yw = c->ywT.ptr;
  t.yrel = static_cast<const int32_t *>(c->yrelT_d.ptr);
  t.ywin = static_cast<const int32_t *>(c->ywinT_d.ptr);
  t.xrel = static_cast<const int32_t *>(c->xrelT_d.ptr);
  t.xwin = static_cast<const int32_t *>(c->xwinT_d.ptr);
  t.tile_rows = kTileRows;
  t.win_rows = c->win_rowsT;
  t.win_cols = c->win_colsT;
  t.taps = c->taps_T;
  t.rows_tx = c->rows_txT;
  t.rows_xrel = c->rows_txT ? static_cast<const int32_t *>(c->rows_xrelT_d.ptr) : nullptr;
  t.rows_xwin = c->rows_txT ? static_cast<const int32_t *>(c->rows_xwinT_d.ptr) : nullptr;
  t.ident_x = c->ident_xT;
  t.ident_y = c->ident_yT;
  t.csr_ptr = static_cast<const uint32_t *>(c->csr_ptr.ptr);
  t.csr_col = static_cast<const int32_t *>(c->csr_col.ptr);
  t.csr_w = c->csr_w.ptr;
  return t;
}

}  // namespace

extern "C" {

int sllbm_create(sllbm_ctx **out, int hip_device, int precision) {
  if (!out) return SLLBM_E_ARG;
  *out = nullptr;
  if (hip_device < 0) return SLLBM_E_ARG;
  if (precision != SLLBM_FP64 && precision != SLLBM_FP32 && precision != SLLBM_BF16X)
    return SLLBM_E_ARG;
  sllbm_ctx *c = new (std::nothrow) sllbm_ctx();
  if (!c) return SLLBM_E_OOM;
  c->device = hip_device;
  c->fp32 = precision != SLLBM_FP64;
  c->bf16x = precision == SLLBM_BF16X;
  *out = c;
  return SLLBM_OK;
}

void sllbm_destroy(sllbm_ctx *c) {
  if (!c) return;
  if (c->dev_checked) {
    (void)hipSetDevice(c->device);
    if (c->stream) (void)hipStreamSynchronize(c->stream);
    DeviceBuf *bufs[] = {&c->xsrc, &c->xw, &c->ysrc, &c->yw, &c->yrel_d, &c->ywin_d,
                         &c->xrel_d, &c->xwin_d, &c->xsrcT, &c->xwT, &c->ysrcT, &c->ywT,
                         &c->yrelT_d, &c->ywinT_d, &c->xrelT_d, &c->xwinT_d, &c->mxd,
                         &c->myd, &c->mnode_d, &c->flag, &c->partial, &c->scalar, &c->macro,
                         &c->rec_cell,
                         &c->rec, &c->rows_xrel_d, &c->rows_xwin_d,
                         &c->rows_xrelT_d, &c->rows_xwinT_d, &c->adj_tmp, &c->csr_ptr,
                         &c->csr_col, &c->csr_w};
    for (DeviceBuf *b : bufs) free_buf(*b);
    if (c->own_pop) {
      (void)hipFree(c->pop[0]);
      (void)hipFree(c->pop[1]);
    }
  }
  delete c;
}

const char *sllbm_last_error(const sllbm_ctx *c) { return c ? c->err.c_str() : "null context"; }

int sllbm_set_stream(sllbm_ctx *c, void *stream) {
  if (!c) return SLLBM_E_ARG;
  c->stream = static_cast<hipStream_t>(stream);
  return SLLBM_OK;
}

int sllbm_set_velocity_set(sllbm_ctx *c, int q1d, const double *xi1d, const double *w1d,
                           double cs) {
  int rc = setup_allowed(c);
  if (rc) return rc;
  if (!is_finite(cs) || !(cs > 0)) return fail(c, SLLBM_E_ARG, "cs must be positive and finite");
  if (q1d != 5 && q1d != 3)
    return fail(c, SLLBM_E_UNSUPPORTED, "5 (D2Q25) or 3 (D2Q9) velocities per axis");
  if (q1d == 3 && c->have_phys && c->model != SLLBM_ISOTHERMAL)
    return fail(c, SLLBM_E_UNSUPPORTED, "the 3-velocity set (D2Q9) runs the isothermal model only");
  VelocitySet vs{};
  if (!xi1d && !w1d) {
    vs = q1d == 3 ? d1q3_velocity_set() : default_velocity_set();
  } else {
    if (!xi1d || !w1d)
      return fail(c, SLLBM_E_ARG, "xi1d and w1d must both be given or both NULL");
    vs.q1 = q1d;
    for (int a = 0; a < q1d; ++a) {
      if (!is_finite(xi1d[a]) || !is_finite(w1d[a]) || !(w1d[a] > 0))
        return fail(c, SLLBM_E_ARG, "velocities must be finite and weights positive");
      vs.xi[a] = xi1d[a];
      vs.w[a] = w1d[a];
    }
    fill_hermite_constants(vs);
  }
  if (c->have_phys && c->Pr != 1.0 && !gaussian_exact_to_degree(vs, 7))
    return fail(c, SLLBM_E_UNSUPPORTED,
                "Pr != 1 needs a velocity set exact to degree 7 (zero equilibrium heat flux)");
  c->vs = vs;
  c->cs = cs;
  update_relaxation(c);
  invalidate(c);
  return SLLBM_OK;
}

int sllbm_set_order(sllbm_ctx *c, int p, int nodes) {
  int rc = setup_allowed(c);
  if (rc) return rc;
  if (p < 1 || p > kMaxOrder) return fail(c, SLLBM_E_ARG, "order p must be in 1..4");
  if (nodes != SLLBM_NODES_GLC && nodes != SLLBM_NODES_EQUIDISTANT)
    return fail(c, SLLBM_E_ARG, "unknown support-point family");
  c->p = p;
  c->glc = nodes == SLLBM_NODES_GLC;
  c->have_grid = false;  // the grid depends on the order
  invalidate(c);
  return SLLBM_OK;
}

static int init_grid(sllbm_ctx *c, int ncx, int ncy, const std::vector<double> &ex,
                     const std::vector<double> &ey, int bcx, int bcy, bool uniform) {
  const std::vector<double> r = support_points(c->p, c->glc);
  c->ax.setup(ex, c->p, bcx == SLLBM_PERIODIC, uniform, r);
  c->ay.setup(ey, c->p, bcy == SLLBM_PERIODIC, uniform, r);
  if ((long long)c->ax.n * c->ay.n > (1LL << 31) / 64)
    return fail(c, SLLBM_E_ARG, "grid too large (nx * ny * 50 must fit in 32 bits)");
  (void)ncx;
  (void)ncy;
  c->curvi = false;
  c->have_grid = true;
  invalidate(c);
  return SLLBM_OK;
}

static int check_grid_args(sllbm_ctx *c, int ncx, int ncy, int bcx, int bcy) {
  if (c->p == 0) return fail(c, SLLBM_E_STATE, "set the order before the grid");
  if (ncx < 1 || ncy < 1 || ncx > 65535 || ncy > 65535)
    return fail(c, SLLBM_E_ARG, "cell counts must be in 1..65535");
  for (int bc : {bcx, bcy})
    if (bc != SLLBM_PERIODIC && bc != SLLBM_ZERO_GRADIENT)
      return fail(c, SLLBM_E_ARG, "unknown boundary kind");
  return SLLBM_OK;
}

int sllbm_init_grid_uniform(sllbm_ctx *c, int ncx, int ncy, double x0, double x1, double y0,
                            double y1, int bcx, int bcy) {
  int rc = setup_allowed(c);
  if (rc) return rc;
  rc = check_grid_args(c, ncx, ncy, bcx, bcy);
  if (rc) return rc;
  if (!is_finite(x0) || !is_finite(x1) || !is_finite(y0) || !is_finite(y1) || !(x1 > x0) || !(y1 > y0))
    return fail(c, SLLBM_E_ARG, "domain bounds must be finite with x1 > x0 and y1 > y0");
  std::vector<double> ex(ncx + 1), ey(ncy + 1);
  for (int k = 0; k <= ncx; ++k) ex[k] = x0 + (x1 - x0) * double(k) / ncx;
  for (int k = 0; k <= ncy; ++k) ey[k] = y0 + (y1 - y0) * double(k) / ncy;
  ex[ncx] = x1;
  ey[ncy] = y1;
  return init_grid(c, ncx, ncy, ex, ey, bcx, bcy, true);
}

int sllbm_init_grid_mapped(sllbm_ctx *c, int ncx, int ncy, const double *edges_x,
                           const double *edges_y, int bcx, int bcy) {
  int rc = setup_allowed(c);
  if (rc) return rc;
  rc = check_grid_args(c, ncx, ncy, bcx, bcy);
  if (rc) return rc;
  if (!edges_x || !edges_y) return fail(c, SLLBM_E_ARG, "null edge array");
  std::vector<double> ex(edges_x, edges_x + ncx + 1), ey(edges_y, edges_y + ncy + 1);
  for (const auto *e : {&ex, &ey})
    for (size_t k = 0; k < e->size(); ++k) {
      if (!is_finite((*e)[k])) return fail(c, SLLBM_E_ARG, "cell edges must be finite");
      if (k > 0 && !((*e)[k] > (*e)[k - 1]))
        return fail(c, SLLBM_E_ARG, "cell edges must be strictly increasing");
    }
  return init_grid(c, ncx, ncy, ex, ey, bcx, bcy, false);
}

int sllbm_init_grid_curvilinear(sllbm_ctx *c, int ncx, int ncy, const double *vx,
                                const double *vy) {
  int rc = setup_allowed(c);
  if (rc) return rc;
  rc = check_grid_args(c, ncx, ncy, SLLBM_PERIODIC, SLLBM_PERIODIC);
  if (rc) return rc;
  if (!vx || !vy) return fail(c, SLLBM_E_ARG, "null vertex array");
  CurviMesh m;
  const std::string e = m.setup(ncx, ncy, vx, vy);
  if (!e.empty()) return fail(c, SLLBM_E_ARG, e);
  std::vector<double> ex(ncx + 1), ey(ncy + 1);
  for (int k = 0; k <= ncx; ++k) ex[k] = k;
  for (int k = 0; k <= ncy; ++k) ey[k] = k;
  rc = init_grid(c, ncx, ncy, ex, ey, SLLBM_PERIODIC, SLLBM_PERIODIC, true);
  if (rc) return rc;
  c->mesh = std::move(m);
  curvi_node_coords(c->mesh, support_points(c->p, c->glc), c->cX, c->cY);
  c->curvi = true;
  return SLLBM_OK;
}

int sllbm_set_physics(sllbm_ctx *c, double dt, double nu, double gamma, double Pr, int model) {
  int rc = setup_allowed(c);
  if (rc) return rc;
  if (!is_finite(dt) || !(dt > 0)) return fail(c, SLLBM_E_ARG, "dt must be positive and finite");
  if (std::isnan(nu) || !(nu > 0))
    return fail(c, SLLBM_E_ARG, "nu must be positive (tau = nu/dt + 1/2 > 1/2) or +inf");
  if (model < SLLBM_ISOTHERMAL || model > SLLBM_POLYATOMIC)
    return fail(c, SLLBM_E_ARG, "unknown model");
  if (model == SLLBM_POLYATOMIC && (!is_finite(gamma) || !(gamma > 1.0)))
    return fail(c, SLLBM_E_ARG, "gamma must be finite and > 1");
  if (!is_finite(Pr) || !(Pr > 0)) return fail(c, SLLBM_E_ARG, "Pr must be positive and finite");
  if (Pr != 1.0 && model == SLLBM_ISOTHERMAL)
    return fail(c, SLLBM_E_ARG, "Pr != 1 needs a thermal model (no energy equation otherwise)");
  if (q1(c) == 3 && model != SLLBM_ISOTHERMAL)
    return fail(c, SLLBM_E_UNSUPPORTED, "the 3-velocity set (D2Q9) runs the isothermal model only");
  if (Pr != 1.0 && !gaussian_exact_to_degree(c->vs, 7))
    return fail(c, SLLBM_E_UNSUPPORTED,
                "Pr != 1 needs a velocity set exact to degree 7 (zero equilibrium heat flux)");
  c->dt = dt;
  c->nu = nu;
  c->gamma = gamma;
  c->Pr = Pr;
  c->model = model;
  c->have_phys = true;
  update_relaxation(c);
  invalidate(c);
  return SLLBM_OK;
}

int sllbm_set_path(sllbm_ctx *c, int path) {
  if (!c) return SLLBM_E_ARG;
  if (path < SLLBM_PATH_AUTO || path > SLLBM_PATH_ROWS)
    return fail(c, SLLBM_E_ARG, "unknown path");
  c->path = path;
  return SLLBM_OK;
}

int sllbm_resolved_path(const sllbm_ctx *cc, int *path) {
  sllbm_ctx *c = const_cast<sllbm_ctx *>(cc);
  if (!c || !path) return SLLBM_E_ARG;
  const int rc = ready_for_tables(c);
  if (rc) return rc;
  build_host_tables(c);
  *path = effective_path(c);
  return SLLBM_OK;
}

int sllbm_num_nodes(const sllbm_ctx *c, int64_t *nx, int64_t *ny) {
  if (!c || !nx || !ny) return SLLBM_E_ARG;
  if (!c->have_grid) return fail(const_cast<sllbm_ctx *>(c), SLLBM_E_STATE, "grid not set");
  *nx = c->ax.n;
  *ny = c->ay.n;
  return SLLBM_OK;
}

int sllbm_population_layout(const sllbm_ctx *c, int *ns, int *q, int *bytes) {
  if (!c || !ns || !q || !bytes) return SLLBM_E_ARG;
  if (!c->have_phys) return fail(const_cast<sllbm_ctx *>(c), SLLBM_E_STATE, "physics not set");
  *ns = nsets(c);
  *q = nvel(c);
  *bytes = int(pop_size(c));
  return SLLBM_OK;
}

int sllbm_node_coords(const sllbm_ctx *c, double *x, double *y) {
  if (!c || !x || !y) return SLLBM_E_ARG;
  if (!c->have_grid) return fail(const_cast<sllbm_ctx *>(c), SLLBM_E_STATE, "grid not set");
  if (c->curvi)
    return fail(const_cast<sllbm_ctx *>(c), SLLBM_E_UNSUPPORTED,
                "a curvilinear mesh has no axis coordinates (sllbm_node_coords_2d)");
  for (int j = 0; j < c->ax.n; ++j) x[j] = c->ax.coord(j);
  for (int j = 0; j < c->ay.n; ++j) y[j] = c->ay.coord(j);
  return SLLBM_OK;
}

int sllbm_node_coords_2d(const sllbm_ctx *c, double *x, double *y) {
  if (!c || !x || !y) return SLLBM_E_ARG;
  if (!c->have_grid) return fail(const_cast<sllbm_ctx *>(c), SLLBM_E_STATE, "grid not set");
  if (c->curvi) {
    std::memcpy(x, c->cX.data(), c->cX.size() * sizeof(double));
    std::memcpy(y, c->cY.data(), c->cY.size() * sizeof(double));
    return SLLBM_OK;
  }
  for (int iy = 0; iy < c->ay.n; ++iy)
    for (int ix = 0; ix < c->ax.n; ++ix) {
      x[size_t(iy) * c->ax.n + ix] = c->ax.coord(ix);
      y[size_t(iy) * c->ax.n + ix] = c->ay.coord(iy);
    }
  return SLLBM_OK;
}

int sllbm_departure_table(const sllbm_ctx *cc, int axis, int comp, int32_t *src, double *w) {
  sllbm_ctx *c = const_cast<sllbm_ctx *>(cc);
  if (!c || !src || !w) return SLLBM_E_ARG;
  if (c->curvi)
    return fail(c, SLLBM_E_UNSUPPORTED, "a curvilinear mesh has no per-axis departure tables");
  if (axis != 0 && axis != 1) return fail(c, SLLBM_E_ARG, "axis must be 0 or 1");
  if (comp < 0 || comp >= q1(c)) return fail(c, SLLBM_E_ARG, "velocity component out of range");
  int rc = ready_for_tables(c);
  if (rc) return rc;
  build_host_tables(c);
  const AxisTable &t = axis == 0 ? c->xt[comp] : c->yt[comp];
  std::memcpy(src, t.src.data(), t.src.size() * sizeof(int32_t));
  std::memcpy(w, t.w.data(), t.w.size() * sizeof(double));
  return SLLBM_OK;
}

int sllbm_departure_records(const sllbm_ctx *cc, int i, int32_t *cell, double *r, double *s) {
  sllbm_ctx *c = const_cast<sllbm_ctx *>(cc);
  if (!c || !cell || !r || !s) return SLLBM_E_ARG;
  if (i < 0 || i >= nvel(c)) return fail(c, SLLBM_E_ARG, "velocity index out of range");
  int rc = ready_for_tables(c);
  if (rc) return rc;
  build_host_tables(c);
  const std::string e = departure_records(c, i, cell, r, s);
  return e.empty() ? SLLBM_OK : fail(c, SLLBM_E_ARG, e);
}

int sllbm_mass_weights(const sllbm_ctx *c, double *mx, double *my) {
  if (!c || !mx || !my) return SLLBM_E_ARG;
  if (!c->have_grid) return fail(const_cast<sllbm_ctx *>(c), SLLBM_E_STATE, "grid not set");
  if (c->curvi)
    return fail(const_cast<sllbm_ctx *>(c), SLLBM_E_UNSUPPORTED,
                "node masses of a curvilinear mesh are not a product of axis weights");
  const std::vector<double> a = c->ax.node_mass(), b = c->ay.node_mass();
  std::memcpy(mx, a.data(), a.size() * sizeof(double));
  std::memcpy(my, b.data(), b.size() * sizeof(double));
  return SLLBM_OK;
}

int sllbm_node_masses(const sllbm_ctx *cc, double *m) {
  sllbm_ctx *c = const_cast<sllbm_ctx *>(cc);
  if (!c || !m) return SLLBM_E_ARG;
  if (!c->have_grid) return fail(c, SLLBM_E_STATE, "grid not set");
  if (c->curvi) {
    const std::vector<double> M = curvi_node_mass(c->mesh, support_points(c->p, c->glc));
    std::memcpy(m, M.data(), M.size() * sizeof(double));
    return SLLBM_OK;
  }
  const std::vector<double> a = c->ax.node_mass(), b = c->ay.node_mass();
  for (int iy = 0; iy < c->ay.n; ++iy)
    for (int ix = 0; ix < c->ax.n; ++ix) m[size_t(iy) * c->ax.n + ix] = b[iy] * a[ix];
  return SLLBM_OK;
}

int sllbm_relaxation_time(const sllbm_ctx *c, double *tau) {
  if (!c || !tau) return SLLBM_E_ARG;
  if (!c->have_phys) return fail(const_cast<sllbm_ctx *>(c), SLLBM_E_STATE, "physics not set");
  *tau = c->tau;
  return SLLBM_OK;
}

int sllbm_bind_populations(sllbm_ctx *c, void *a, void *b) {
  if (!c) return SLLBM_E_ARG;
  if (!a || !b || a == b) return fail(c, SLLBM_E_ARG, "need two distinct device buffers");
  int rc = ready_for_tables(c);
  if (rc) return rc;
  if (c->own_pop) {
    (void)hipFree(c->pop[0]);
    (void)hipFree(c->pop[1]);
  }
  c->pop[0] = a;
  c->pop[1] = b;
  c->own_pop = false;
  c->pop_bytes = size_t(nsets(c)) * nvel(c) * size_t(nnodes(c)) * pop_size(c);
  c->cur = 0;
  c->initialised = false;
  return SLLBM_OK;
}

int sllbm_init_macro(sllbm_ctx *c, const double *rho, const double *ux, const double *uy,
                     const double *T, int on_device) {
  if (!c) return SLLBM_E_ARG;
  if (!rho || !ux || !uy || (!T && c->model != SLLBM_ISOTHERMAL))
    return fail(c, SLLBM_E_ARG, "null macroscopic field");
  int rc = ready_for_tables(c);
  if (rc) return rc;
  const long long N = nnodes(c);
  if (!on_device) {
    for (long long v = 0; v < N; ++v) {
      if (!is_finite(rho[v]) || !is_finite(ux[v]) || !is_finite(uy[v]) || !(rho[v] > 0))
        return fail(c, SLLBM_E_ARG, "rho must be positive and all fields finite");
      if (c->model != SLLBM_ISOTHERMAL && (!is_finite(T[v]) || !(T[v] > 0)))
        return fail(c, SLLBM_E_ARG, "T must be positive and finite");
    }
  }
  rc = prepare_device(c);
  if (!rc) rc = ensure_populations(c);
  if (rc) return rc;
  const double *d[4] = {rho, ux, uy, T};
  if (!on_device) {
    rc = alloc_buf(c, c->macro, sizeof(double) * 4 * size_t(N));
    if (rc) return rc;
    double *m = static_cast<double *>(c->macro.ptr);
    for (int k = 0; k < 4; ++k) {
      if (!d[k]) {
        d[k] = nullptr;
        continue;
      }
      HIP_TRY(c, hipMemcpyAsync(m + k * N, d[k], sizeof(double) * N, hipMemcpyHostToDevice,
                                c->stream));
      d[k] = m + k * N;
    }
  }
  c->cur = 0;
  c->layout = path_layout(effective_path(c));  // written in the order the next step reads
  HIP_TRY(c, launch_init_eq(c->fp32, c->model, make_consts(c), d[0], d[1], d[2], d[3],
                            c->pop[0], c->stream));
  rc = clear_flag(c);
  if (rc) return rc;
  if (!on_device) HIP_TRY(c, hipStreamSynchronize(c->stream));
  c->steps_done = 0;
  c->initialised = true;
  return SLLBM_OK;
}

int sllbm_set_check_interval(sllbm_ctx *c, int64_t k) {
  if (!c) return SLLBM_E_ARG;
  if (k < 0) return fail(c, SLLBM_E_ARG, "interval must be >= 0");
  c->check_interval = k;
  return SLLBM_OK;
}

static int read_flag(sllbm_ctx *c, int *flag) {
  HIP_TRY(c, hipMemcpyAsync(flag, c->flag.ptr, sizeof(int), hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  return SLLBM_OK;
}

// Moments per node recorded by sllbm_step_record: rho, u_x, u_y and, unless
// isothermal, theta; with Pr != 1 also the centred second moments of each set
// (what the transposed quasi-equilibrium term needs).
static int recorded_moments(const sllbm_ctx *c) {
  if (c->model == SLLBM_ISOTHERMAL) return 3;
  return c->omega_pr != c->omega ? 4 + 3 * nsets(c) : 4;
}

static int run_steps(sllbm_ctx *c, int64_t n, double *moments) {
  if (!c) return SLLBM_E_ARG;
  if (n < 0) return fail(c, SLLBM_E_ARG, "n must be >= 0");
  if (!c->initialised) return fail(c, SLLBM_E_STATE, "populations not initialised");
  int rc = prepare_device(c);
  if (rc) return rc;
  const int path = effective_path(c);
  if (c->curvi && path != kPathRecords)
    return fail(c, SLLBM_E_UNSUPPORTED, "a curvilinear mesh runs on the records path only");
  if ((path == kPathTiled || path == kPathMfma) && q1(c) != kQ1)
    return fail(c, SLLBM_E_UNSUPPORTED,
                "the 3-velocity set (D2Q9) runs on the row-segment, direct and records kernels");
  if (path == kPathTiled && !tiled_fits(c))
    return fail(c, SLLBM_E_UNSUPPORTED, "departures span too many rows for the tiled kernel");
  if (path == kPathRows && c->rows_tx == 0)
    return fail(c, SLLBM_E_UNSUPPORTED,
                "row segments need a first 1-D velocity of 0 and a segment of at least 32 "
                "columns whose x-stencils fit 64 columns");
  if (c->bf16x && path != kPathMfma)
    return fail(c, SLLBM_E_UNSUPPORTED,
                "the bfloat16 experiment runs on the matrix-core path (SLLBM_PATH_MFMA) only");
  if (path == kPathMfma && !mfma_fits(c))
    return fail(c, SLLBM_E_UNSUPPORTED,
                "matrix-core path needs float32, at most 16 set x window rows and departures "
                "within one node spacing of their cell");
  rc = to_layout(c, path_layout(path));  // after a change of path
  if (rc) return rc;
  StepConsts k = make_consts(c);
  const DevTables t = make_tables(c);
  int *flag = static_cast<int *>(c->flag.ptr);
  // bytes each step streams: both population arrays, plus the records the
  // records gather re-reads every step
  const double state_bytes =
      2.0 * double(nsets(c)) * nvel(c) * double(nnodes(c)) * double(pop_size(c)) +
      (path == kPathRecords ? double(nvel(c)) * double(nnodes(c)) * double(4 + 2 * pop_size(c))
                            : 0.0);
  const bool big_state = state_bytes > 256.0 * (1 << 20);
  // Pr != 1 records also carry each set's centred second moments, recovered
  // after the step from the post-collision state (needs omega != 1)
  const bool rec_m2 = moments && c->model != SLLBM_ISOTHERMAL && c->omega_pr != c->omega;
  if (rec_m2 && (c->omega == 1.0 || q1(c) != kQ1))
    return fail(c, SLLBM_E_UNSUPPORTED,
                "a Pr != 1 moment record needs tau != 1 and the 5-velocity set");
  for (int64_t s = 0; s < n; ++s) {
    k.mom_out = moments ? moments + s * recorded_moments(c) * k.n : nullptr;
    // when what a step streams exceeds the 256 MB last-level cache (MALL)
    // of the MI355X, every other step walks the grid backwards, so
    // that it starts on the tiles the previous step wrote last, which are
    // still cached (Riemann 1025^2 f + g: +7 % float32, +1-4 % float64); a
    // state that fits keeps one order (backwards cost 3 % there)
    k.reverse = big_state ? int(c->steps_done & 1) : 0;
    HIP_TRY(c, launch_step(c->fp32, c->model, path, k, t, c->pop[c->cur], c->pop[1 - c->cur],
                           flag, c->stream));
    c->cur ^= 1;
    if (rec_m2)
      HIP_TRY(c, launch_record_m2(c->fp32, c->model, k, c->pop[c->cur], k.mom_out, c->stream));
    ++c->steps_done;
    if (c->check_interval > 0 && c->steps_done % c->check_interval == 0) {
      int f = 0;
      rc = read_flag(c, &f);
      if (rc) return rc;
      if (f) return fail(c, SLLBM_E_UNSTABLE, "stability flag raised (rho, theta or moments)");
    }
  }
  return SLLBM_OK;
}

int sllbm_step(sllbm_ctx *c, int64_t n) { return run_steps(c, n, nullptr); }

int sllbm_recorded_moments(const sllbm_ctx *c, int *k) {
  if (!c || !k) return SLLBM_E_ARG;
  if (!c->have_phys) return fail(const_cast<sllbm_ctx *>(c), SLLBM_E_STATE, "physics not set");
  *k = recorded_moments(c);
  return SLLBM_OK;
}

int sllbm_step_record(sllbm_ctx *c, int64_t n, double *moments) {
  if (!c) return SLLBM_E_ARG;
  if (!moments) return fail(c, SLLBM_E_ARG, "null moments buffer");
  return run_steps(c, n, moments);
}

int sllbm_adjoint_seed(sllbm_ctx *c, const double *g_rho, const double *g_ux, const double *g_uy,
                       const double *g_T, void *lam) {
  if (!c) return SLLBM_E_ARG;
  if (!g_rho || !g_ux || !g_uy || !lam) return fail(c, SLLBM_E_ARG, "null device pointer");
  if (!c->initialised) return fail(c, SLLBM_E_STATE, "populations not initialised");
  int rc = prepare_adjoint(c);
  if (rc) return rc;
  HIP_TRY(c, launch_adjoint_seed(c->fp32, c->model, make_consts(c), c->pop[c->cur], g_rho, g_ux,
                                 g_uy, g_T, lam, c->stream));
  return SLLBM_OK;
}

int sllbm_adjoint_collide(sllbm_ctx *c, const void *lam, const double *moments, void *mu) {
  if (!c) return SLLBM_E_ARG;
  if (!lam || !moments || !mu) return fail(c, SLLBM_E_ARG, "null device pointer");
  int rc = prepare_adjoint(c);
  if (rc) return rc;
  HIP_TRY(c, launch_adjoint_collide(c->fp32, c->model, make_consts(c), lam, moments, mu,
                                    c->stream));
  return SLLBM_OK;
}

int sllbm_adjoint_nu_term(sllbm_ctx *c, const void *lam, const void *pop, const double *moments,
                          double *acc) {
  if (!c) return SLLBM_E_ARG;
  if (!lam || !pop || !moments || !acc) return fail(c, SLLBM_E_ARG, "null device pointer");
  int rc = prepare_adjoint(c);
  if (rc) return rc;
  if (c->omega == 1.0)
    return fail(c, SLLBM_E_UNSUPPORTED,
                "tau = 1: post-collision populations are at equilibrium and do not give the "
                "pre-collision non-equilibrium part");
  if (c->omega_pr != c->omega)
    return fail(c, SLLBM_E_UNSUPPORTED, "the viscosity term covers Pr = 1 (BGK) only");
  // f - f_eq before the collision is (f+ - f_eq) / (1 - omega) (the moments
  // are collision invariants), d(omega)/d(nu) = -1 / (tau^2 dt), and
  // dC/d(omega) = -(f - f_eq)
  const double scale = std::isinf(c->tau) ? 0.0 : 1.0 / ((1.0 - c->omega) * c->tau * c->tau * c->dt);
  HIP_TRY(c, launch_nu_term(c->fp32, c->model, make_consts(c), lam, pop, moments,
                            static_cast<double *>(c->partial.ptr),
                            static_cast<double *>(c->scalar.ptr), scale, acc, c->stream));
  return SLLBM_OK;
}

int sllbm_adjoint_step(sllbm_ctx *c, const void *mu, const double *moments_prev, void *out) {
  if (!c) return SLLBM_E_ARG;
  if (!mu || !out) return fail(c, SLLBM_E_ARG, "null device pointer");
  if (mu == out) return fail(c, SLLBM_E_ARG, "input and output must differ");
  int rc = prepare_adjoint(c);
  if (rc) return rc;
  // the forward's path choice carries over: DIRECT and TILED as set (TILED
  // falling back to DIRECT when its windows do not fit), ROWS when its
  // segments exist, otherwise row segments of >= 48 nodes, then TILED
  const bool tiled_ok = c->win_rowsT <= 3 * kTileRows && c->win_colsT <= kMaxWindowCols;
  const bool rows_ok = c->rows_txT >= kRowsMinCols;
  int kind = kAdjointDirect;
  if (c->curvi) {
    kind = kAdjointCsr;
  } else if (c->path == SLLBM_PATH_TILED) {
    kind = tiled_ok ? kAdjointTiled : kAdjointDirect;
  } else if (c->path == SLLBM_PATH_ROWS && rows_ok) {
    kind = kAdjointRows;
  } else if (c->path != SLLBM_PATH_DIRECT) {
    kind = c->rows_txT >= 48 ? kAdjointRows
           : tiled_ok        ? kAdjointTiled
           : rows_ok         ? kAdjointRows
                             : kAdjointDirect;
  }
  if (moments_prev && c->omega_pr != c->omega) {
    // Pr != 1: S^T into scratch, then the quasi-equilibrium-aware J_C^T
    rc = alloc_buf(c, c->adj_tmp, c->pop_bytes ? c->pop_bytes
                                                : size_t(nsets(c)) * nvel(c) * nnodes(c) *
                                                      pop_size(c));
    if (rc) return rc;
    const StepConsts k = make_consts(c);
    HIP_TRY(c, launch_adjoint_step(c->fp32, c->model, kind, k, make_adjoint_tables(c), mu,
                                   nullptr, c->adj_tmp.ptr, c->stream));
    HIP_TRY(c, launch_adjoint_collide(c->fp32, c->model, k, c->adj_tmp.ptr, moments_prev, out,
                                      c->stream));
    return SLLBM_OK;
  }
  HIP_TRY(c, launch_adjoint_step(c->fp32, c->model, kind, make_consts(c),
                                 make_adjoint_tables(c), mu, moments_prev, out, c->stream));
  return SLLBM_OK;
}

int sllbm_eq_init_vjp(sllbm_ctx *c, const void *lam0, const double *rho0, const double *ux0,
                      const double *uy0, const double *T0, double *g_rho0, double *g_ux0,
                      double *g_uy0, double *g_T0) {
  if (!c) return SLLBM_E_ARG;
  if (!lam0 || !rho0 || !ux0 || !uy0 || !g_rho0 || !g_ux0 || !g_uy0)
    return fail(c, SLLBM_E_ARG, "null device pointer");
  if (c->model != SLLBM_ISOTHERMAL && !T0)
    return fail(c, SLLBM_E_ARG, "the initial temperature is needed unless isothermal");
  int rc = prepare_adjoint(c);
  if (rc) return rc;
  HIP_TRY(c, launch_eq_init_vjp(c->fp32, c->model, make_consts(c), lam0, rho0, ux0, uy0, T0,
                                g_rho0, g_ux0, g_uy0, g_T0, c->stream));
  return SLLBM_OK;
}

int sllbm_status_flags(sllbm_ctx *c, int *unstable, int64_t *steps_done) {
  if (!c || !unstable || !steps_done) return SLLBM_E_ARG;
  if (!c->initialised) return fail(c, SLLBM_E_STATE, "populations not initialised");
  int rc = read_flag(c, unstable);
  if (rc) return rc;
  *steps_done = c->steps_done;
  return SLLBM_OK;
}

int sllbm_moments(sllbm_ctx *c, double *rho, double *ux, double *uy, double *T, int on_device) {
  if (!c) return SLLBM_E_ARG;
  if (!rho || !ux || !uy || !T) return fail(c, SLLBM_E_ARG, "null output array");
  if (!c->initialised) return fail(c, SLLBM_E_STATE, "populations not initialised");
  int rc = prepare_device(c);
  if (rc) return rc;
  const long long N = nnodes(c);
  double *d[4] = {rho, ux, uy, T};
  if (!on_device) {
    rc = alloc_buf(c, c->macro, sizeof(double) * 4 * size_t(N));
    if (rc) return rc;
    for (int k = 0; k < 4; ++k) d[k] = static_cast<double *>(c->macro.ptr) + k * N;
  }
  HIP_TRY(c, launch_moments(c->fp32, c->model, make_consts(c), make_tables(c), c->pop[c->cur],
                            d[0], d[1], d[2], d[3], static_cast<double *>(c->partial.ptr),
                            c->stream));
  if (!on_device) {
    double *h[4] = {rho, ux, uy, T};
    for (int k = 0; k < 4; ++k)
      HIP_TRY(c, hipMemcpyAsync(h[k], d[k], sizeof(double) * N, hipMemcpyDeviceToHost,
                                c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
  }
  return SLLBM_OK;
}

int sllbm_mass(sllbm_ctx *c, double *mass) {
  if (!c || !mass) return SLLBM_E_ARG;
  if (!c->initialised) return fail(c, SLLBM_E_STATE, "populations not initialised");
  int rc = prepare_device(c);
  if (rc) return rc;
  const StepConsts k = make_consts(c);
  double *part = static_cast<double *>(c->partial.ptr);
  HIP_TRY(c, launch_moments(c->fp32, c->model, k, make_tables(c), c->pop[c->cur], nullptr,
                            nullptr, nullptr, nullptr, part, c->stream));
  double *out = static_cast<double *>(c->scalar.ptr);
  HIP_TRY(c, launch_sum(part, mass_blocks(k), out, c->stream));
  HIP_TRY(c, hipMemcpyAsync(mass, out, sizeof(double), hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  return SLLBM_OK;
}

int sllbm_mass_noalloc(sllbm_ctx *c, double *mass_dev) {
  if (!c || !mass_dev) return SLLBM_E_ARG;
  // no set-up work here: the device tables must already exist (they are
  // built by init_macro / set_populations and stay valid until the set-up
  // changes, which is refused once initialised)
  if (!c->initialised || c->dev_dirty || !c->mxd.ptr || !c->myd.ptr ||
      (c->curvi && !c->mnode_d.ptr))
    return fail(c, SLLBM_E_STATE,
                "populations not initialised (sllbm_init_macro or sllbm_set_populations first)");
  const StepConsts k = make_consts(c);
  if (mass_blocks(k) > kScratchDoubles)
    return fail(c, SLLBM_E_ARG, "grid larger than the fixed scratch (" +
                                    std::to_string(int64_t(kScratchDoubles) * 256) + " nodes)");
  HIP_TRY(c, hipSetDevice(c->device));
  double *part = nullptr;
  HIP_TRY(c, scratch_buffer(c->device, &part));
  HIP_TRY(c, launch_moments(c->fp32, c->model, k, make_tables(c), c->pop[c->cur], nullptr,
                            nullptr, nullptr, nullptr, part, c->stream));
  HIP_TRY(c, launch_sum(part, mass_blocks(k), mass_dev, c->stream));
  return SLLBM_OK;
}

int sllbm_get_populations(sllbm_ctx *c, void *dst, int on_device) {
  if (!c || !dst) return SLLBM_E_ARG;
  if (!c->initialised) return fail(c, SLLBM_E_STATE, "populations not initialised");
  if (on_device && (dst == c->pop[0] || dst == c->pop[1]))
    return fail(c, SLLBM_E_ARG, "destination is one of the context's population buffers");
  HIP_TRY(c, hipSetDevice(c->device));
  const void *src = c->pop[c->cur];
  if (c->layout != kPlanar) {  // to the planar order of the ABI
    void *planar = on_device ? dst : c->pop[1 - c->cur];
    HIP_TRY(c, launch_relayout(c->fp32, nsets(c), make_consts(c), src, planar, 0, c->stream));
    if (on_device) return SLLBM_OK;
    src = planar;
  }
  HIP_TRY(c, hipMemcpyAsync(dst, src, c->pop_bytes,
                            on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost,
                            c->stream));
  if (!on_device) HIP_TRY(c, hipStreamSynchronize(c->stream));
  return SLLBM_OK;
}

int sllbm_set_populations(sllbm_ctx *c, const void *src, int on_device) {
  if (!c || !src) return SLLBM_E_ARG;
  int rc = ready_for_tables(c);
  if (rc) return rc;
  rc = prepare_device(c);
  if (!rc) rc = ensure_populations(c);
  if (rc) return rc;
  if (on_device && (src == c->pop[0] || src == c->pop[1]))
    return fail(c, SLLBM_E_ARG, "source is one of the context's population buffers");
  // stored in the order the next step reads
  const int layout = path_layout(effective_path(c));
  c->cur = 0;
  c->layout = layout;
  if (layout == kPlanar) {
    HIP_TRY(c, hipMemcpyAsync(c->pop[0], src, c->pop_bytes,
                              on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice,
                              c->stream));
  } else {
    const void *planar = src;
    if (!on_device) {
      HIP_TRY(c, hipMemcpyAsync(c->pop[1], src, c->pop_bytes, hipMemcpyHostToDevice, c->stream));
      planar = c->pop[1];
    }
    HIP_TRY(c, launch_relayout(c->fp32, nsets(c), make_consts(c), planar, c->pop[0], 1,
                               c->stream));
  }
  rc = clear_flag(c);
  if (rc) return rc;
  if (!on_device) HIP_TRY(c, hipStreamSynchronize(c->stream));
  c->initialised = true;
  return SLLBM_OK;
}

}  // extern "C"
