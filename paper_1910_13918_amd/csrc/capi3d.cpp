// C ABI of the three-dimensional step (declarations and contracts in
// include/sllbm3d.h): set-up state, per-axis departure tables (tables.cpp,
// the same 1-D tables as the two-dimensional grids), device memory and
// kernel launches (step3d.hip).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <limits>
#include <string>
#include <vector>

#include "../../include/sllbm3d.h"
#include "launch.hpp"
#include "launch3d.hpp"
#include "tables.hpp"

using namespace sllbm;

namespace {

struct Buf3 {
  void *ptr = nullptr;
  size_t bytes = 0;
};

}  // namespace

struct sllbm3d_ctx {
  int device = 0;
  int fp32 = 0;
  std::string err;
  hipStream_t stream = nullptr;
  VelocitySet vs = default_velocity_set();
  int p = 0;
  bool glc = true;
  bool have_grid = false;
  Axis ax, ay, az;
  bool have_phys = false;
  double dt = 0, nu = 0, omega = 0;
  bool dev_checked = false;
  bool dev_dirty = true;
  Buf3 xsrc, xw, ysrc, yw, zsrc, zw, mx, my, mz, flag, partial, scalar, macro;
  // row segments (Rows3): segment width (0: unavailable) and windows
  int rows_tx = 0, rows_ntx = 0;
  bool rows_ok = false;  // the row kernels apply (identity zero components)
  Buf3 xwin, xrel;
  void *pop[2] = {nullptr, nullptr};
  bool own_pop = false;
  int cur = 0;
  bool initialised = false;
  int64_t steps_done = 0;
};

namespace {

int fail(sllbm3d_ctx *c, int code, const std::string &msg) {
  if (c) c->err = msg;
  return code;
}

#define HIP_TRY3(ctx, expr)                                                       \
  do {                                                                            \
    hipError_t e_ = (expr);                                                       \
    if (e_ != hipSuccess)                                                         \
      return fail(ctx, e_ == hipErrorOutOfMemory ? SLLBM_E_OOM : SLLBM_E_DEVICE,  \
                  std::string(#expr) + ": " + hipGetErrorString(e_));             \
  } while (0)

long long nnodes(const sllbm3d_ctx *c) { return (long long)c->ax.n * c->ay.n * c->az.n; }
size_t value_bytes(const sllbm3d_ctx *c) { return c->fp32 ? 4 : 8; }
size_t pop_bytes(const sllbm3d_ctx *c) { return size_t(kQ3) * size_t(nnodes(c)) * value_bytes(c); }

int setup_allowed(sllbm3d_ctx *c) {
  if (!c) return SLLBM_E_ARG;
  if (c->initialised)
    return fail(c, SLLBM_E_STATE, "set-up cannot change after the populations are initialised");
  return SLLBM_OK;
}

int ready(sllbm3d_ctx *c) {
  if (c->p == 0) return fail(c, SLLBM_E_STATE, "interpolation order not set (sllbm3d_set_order)");
  if (!c->have_grid) return fail(c, SLLBM_E_STATE, "grid not set (sllbm3d_init_grid)");
  if (!c->have_phys) return fail(c, SLLBM_E_STATE, "physics not set (sllbm3d_set_physics)");
  return SLLBM_OK;
}

// Forgets the population buffers (freeing those the context owns): after a
// change of order or grid they no longer have the right size.
void drop_populations(sllbm3d_ctx *c) {
  if (c->own_pop) {
    (void)hipFree(c->pop[0]);
    (void)hipFree(c->pop[1]);
  }
  c->pop[0] = c->pop[1] = nullptr;
  c->own_pop = false;
}

void free_buf(Buf3 &b) {
  if (b.ptr) (void)hipFree(b.ptr);
  b.ptr = nullptr;
  b.bytes = 0;
}

int alloc_buf(sllbm3d_ctx *c, Buf3 &b, size_t bytes) {
  if (b.ptr && b.bytes >= bytes) return SLLBM_OK;
  free_buf(b);
  HIP_TRY3(c, hipMalloc(&b.ptr, bytes > 0 ? bytes : 8));
  b.bytes = bytes;
  return SLLBM_OK;
}

template <typename V>
int upload(sllbm3d_ctx *c, Buf3 &b, const std::vector<V> &v) {
  int rc = alloc_buf(c, b, v.size() * sizeof(V));
  if (rc) return rc;
  HIP_TRY3(c, hipMemcpy(b.ptr, v.data(), v.size() * sizeof(V), hipMemcpyHostToDevice));
  return SLLBM_OK;
}

// Row segments of the step along x: the widest segment (at most 64
// nodes, at least 32) whose x-stencils fit 64 consecutive source columns for
// every segment and 1-D velocity; fills the windows (first unwrapped column
// per component and segment) and each node's first tap within its window.
int rows3_windows(const AxisTable *t, int n, int P1, std::vector<int32_t> &win,
                  std::vector<int32_t> &rel) {
  int tx = 64;
  while (tx >= 32) {
    const int ntx = (n + tx - 1) / tx;
    win.assign(size_t(5) * ntx, 0);
    rel.assign(size_t(5) * n, 0);
    long width = 0;
    for (int a = 0; a < 5; ++a)
      for (int k = 0; k < ntx; ++k) {
        const int j0 = k * tx, j1 = std::min(j0 + tx, n);
        long lo = std::numeric_limits<long>::max(), hi = std::numeric_limits<long>::min();
        for (int j = j0; j < j1; ++j) {
          lo = std::min(lo, t[a].start[j]);
          hi = std::max(hi, t[a].start[j] + P1 - 1);
        }
        win[size_t(a) * ntx + k] = int32_t(lo);
        width = std::max(width, hi - lo + 1);
        for (int j = j0; j < j1; ++j) rel[size_t(a) * n + j] = int32_t(t[a].start[j] - lo);
      }
    if (width <= 64) return tx;
    tx -= int(width) - 64;
  }
  win.clear();
  rel.clear();
  return 0;
}

// [comp][tap][node] order of five 1-D tables: node indices, or the weights
// in the population type.  `tables` (optional) receives the host tables.
int upload_axis(sllbm3d_ctx *c, const Axis &ax, Buf3 &src, Buf3 &w,
                std::vector<AxisTable> *tables = nullptr) {
  const int P1 = c->p + 1, n = ax.n;
  std::vector<int32_t> s(size_t(5) * P1 * n);
  std::vector<double> wd(s.size());
  for (int a = 0; a < 5; ++a) {
    // departure x - dt xi_a along this axis
    const AxisTable t = build_axis_table(ax, -c->dt * c->vs.xi[a]);
    if (tables) tables->push_back(t);
    for (int m = 0; m < P1; ++m)
      for (int j = 0; j < n; ++j) {
        s[(size_t(a) * P1 + m) * n + j] = t.src[size_t(j) * P1 + m];
        wd[(size_t(a) * P1 + m) * n + j] = t.w[size_t(j) * P1 + m];
      }
  }
  int rc = upload(c, src, s);
  if (rc) return rc;
  if (!c->fp32) return upload(c, w, wd);
  return upload(c, w, std::vector<float>(wd.begin(), wd.end()));
}

int prepare_device(sllbm3d_ctx *c) {
  int rc = ready(c);
  if (rc) return rc;
  if (!c->dev_checked) {
    int n = 0;
    hipError_t e = hipGetDeviceCount(&n);
    if (e != hipSuccess || n == 0) return fail(c, SLLBM_E_DEVICE, "no HIP device available");
    if (c->device >= n) return fail(c, SLLBM_E_ARG, "HIP device index out of range");
    c->dev_checked = true;
  }
  HIP_TRY3(c, hipSetDevice(c->device));
  if (c->dev_dirty) {
    std::vector<AxisTable> xt, yt, zt;
    rc = upload_axis(c, c->ax, c->xsrc, c->xw, &xt);
    if (!rc) rc = upload_axis(c, c->ay, c->ysrc, c->yw, &yt);
    if (!rc) rc = upload_axis(c, c->az, c->zsrc, c->zw, &zt);
    // row kernels: the zero component must depart from the node itself on
    // every axis (identity tables); the segments also need the 125 planes
    // within one 32-bit buffer range (whole rows take a resource per plane)
    c->rows_tx = 0;
    c->rows_ok = !rc && identity_table(xt[0], c->ax.n) && identity_table(yt[0], c->ay.n) &&
                 identity_table(zt[0], c->az.n);
    if (c->rows_ok && double(kQ3) * double(nnodes(c)) * double(value_bytes(c)) < 4294967296.0) {
      std::vector<int32_t> win, rel;
      c->rows_tx = rows3_windows(xt.data(), c->ax.n, c->p + 1, win, rel);
      if (c->rows_tx) {
        c->rows_ntx = (c->ax.n + c->rows_tx - 1) / c->rows_tx;
        rc = upload(c, c->xwin, win);
        if (!rc) rc = upload(c, c->xrel, rel);
      }
    }
    if (!rc) rc = upload(c, c->mx, c->ax.node_mass());
    if (!rc) rc = upload(c, c->my, c->ay.node_mass());
    if (!rc) rc = upload(c, c->mz, c->az.node_mass());
    if (!rc) rc = alloc_buf(c, c->flag, sizeof(int));
    if (!rc) rc = alloc_buf(c, c->partial, sizeof(double) * size_t((nnodes(c) + 255) / 256 + 1));
    if (!rc) rc = alloc_buf(c, c->scalar, sizeof(double));
    if (rc) return rc;
    c->dev_dirty = false;
  }
  if (!c->pop[0]) {
    HIP_TRY3(c, hipMalloc(&c->pop[0], pop_bytes(c)));
    HIP_TRY3(c, hipMalloc(&c->pop[1], pop_bytes(c)));
    c->own_pop = true;
  }
  return SLLBM_OK;
}

Consts3 make_consts(const sllbm3d_ctx *c) {
  Consts3 k{};
  k.nx = c->ax.n;
  k.ny = c->ay.n;
  k.nz = c->az.n;
  k.p = c->p;
  k.n = nnodes(c);
  k.omega = c->omega;
  for (int a = 0; a < 5; ++a) {
    k.xi[a] = c->vs.xi[a];
    k.w[a] = c->vs.w[a];
    for (int m = 0; m < 5; ++m) k.hk[a][m] = c->vs.hk[a][m];
  }
  return k;
}

Rows3 make_rows(const sllbm3d_ctx *c) {
  Rows3 r{};
  r.tx = c->rows_tx;
  r.ntx = c->rows_ntx;
  r.perx = c->ax.periodic ? 1 : 0;
  if (c->rows_ok && c->ax.n <= 64 * kRows3MaxX) r.full = (c->ax.n + 63) / 64;
  r.xwin = static_cast<const int32_t *>(c->xwin.ptr);
  r.xrel = static_cast<const int32_t *>(c->xrel.ptr);
  return r;
}

Tables3 make_tables(const sllbm3d_ctx *c) {
  Tables3 t{};
  t.xsrc = static_cast<const int32_t *>(c->xsrc.ptr);
  t.ysrc = static_cast<const int32_t *>(c->ysrc.ptr);
  t.zsrc = static_cast<const int32_t *>(c->zsrc.ptr);
  t.xw = c->xw.ptr;
  t.yw = c->yw.ptr;
  t.zw = c->zw.ptr;
  t.mx = static_cast<const double *>(c->mx.ptr);
  t.my = static_cast<const double *>(c->my.ptr);
  t.mz = static_cast<const double *>(c->mz.ptr);
  return t;
}

}  // namespace

extern "C" {

int sllbm3d_create(sllbm3d_ctx **out, int hip_device, int precision) {
  if (!out) return SLLBM_E_ARG;
  *out = nullptr;
  if (hip_device < 0) return SLLBM_E_ARG;
  if (precision != SLLBM_FP64 && precision != SLLBM_FP32) return SLLBM_E_ARG;
  sllbm3d_ctx *c = new (std::nothrow) sllbm3d_ctx();
  if (!c) return SLLBM_E_OOM;
  c->device = hip_device;
  c->fp32 = precision == SLLBM_FP32;
  *out = c;
  return SLLBM_OK;
}

void sllbm3d_destroy(sllbm3d_ctx *c) {
  if (!c) return;
  if (c->dev_checked) {
    (void)hipSetDevice(c->device);
    if (c->stream) (void)hipStreamSynchronize(c->stream);
    Buf3 *bufs[] = {&c->xsrc, &c->xw,   &c->ysrc,    &c->yw,     &c->zsrc, &c->zw,   &c->mx,
                    &c->my,   &c->mz,   &c->flag,    &c->partial, &c->scalar, &c->macro,
                    &c->xwin, &c->xrel};
    for (Buf3 *b : bufs) free_buf(*b);
    if (c->own_pop) {
      (void)hipFree(c->pop[0]);
      (void)hipFree(c->pop[1]);
    }
  }
  delete c;
}

const char *sllbm3d_last_error(const sllbm3d_ctx *c) { return c ? c->err.c_str() : "null context"; }

int sllbm3d_set_stream(sllbm3d_ctx *c, void *stream) {
  if (!c) return SLLBM_E_ARG;
  c->stream = static_cast<hipStream_t>(stream);
  return SLLBM_OK;
}

int sllbm3d_set_order(sllbm3d_ctx *c, int p, int nodes) {
  int rc = setup_allowed(c);
  if (rc) return rc;
  if (p < 1 || p > kMaxOrder) return fail(c, SLLBM_E_ARG, "order p must be in 1..4");
  if (nodes != SLLBM_NODES_GLC && nodes != SLLBM_NODES_EQUIDISTANT)
    return fail(c, SLLBM_E_ARG, "unknown support-point family");
  c->p = p;
  c->glc = nodes == SLLBM_NODES_GLC;
  c->have_grid = false;
  c->dev_dirty = true;
  drop_populations(c);
  return SLLBM_OK;
}

int sllbm3d_init_grid(sllbm3d_ctx *c, int ncx, int ncy, int ncz, const double *edges_x,
                      const double *edges_y, const double *edges_z, int bcx, int bcy, int bcz) {
  int rc = setup_allowed(c);
  if (rc) return rc;
  if (c->p == 0) return fail(c, SLLBM_E_STATE, "set the order before the grid");
  if (!edges_x || !edges_y || !edges_z) return fail(c, SLLBM_E_ARG, "null edge array");
  const int nc[3] = {ncx, ncy, ncz};
  const double *e[3] = {edges_x, edges_y, edges_z};
  const int bc[3] = {bcx, bcy, bcz};
  std::vector<double> edges[3];
  for (int d = 0; d < 3; ++d) {
    if (nc[d] < 1 || nc[d] > 65535) return fail(c, SLLBM_E_ARG, "cell counts must be in 1..65535");
    if (bc[d] != SLLBM_PERIODIC && bc[d] != SLLBM_ZERO_GRADIENT)
      return fail(c, SLLBM_E_ARG, "unknown boundary kind");
    edges[d].assign(e[d], e[d] + nc[d] + 1);
    for (size_t k = 0; k < edges[d].size(); ++k) {
      if (!std::isfinite(edges[d][k])) return fail(c, SLLBM_E_ARG, "cell edges must be finite");
      if (k > 0 && !(edges[d][k] > edges[d][k - 1]))
        return fail(c, SLLBM_E_ARG, "cell edges must be strictly increasing");
    }
  }
  const std::vector<double> r = support_points(c->p, c->glc);
  Axis ax, ay, az;
  ax.setup(edges[0], c->p, bcx == SLLBM_PERIODIC, false, r);
  ay.setup(edges[1], c->p, bcy == SLLBM_PERIODIC, false, r);
  az.setup(edges[2], c->p, bcz == SLLBM_PERIODIC, false, r);
  const long long n = (long long)ax.n * ay.n * az.n;
  // one population plane (and every byte offset into it) fits in 32 bits,
  // the z extent in the launch grid
  if (n * 8 >= (1LL << 32) || az.n > 65535)
    return fail(c, SLLBM_E_ARG, "grid too large (one float64 plane must stay below 4 GiB)");
  c->ax = ax;
  c->ay = ay;
  c->az = az;
  c->have_grid = true;
  c->dev_dirty = true;
  drop_populations(c);
  return SLLBM_OK;
}

int sllbm3d_set_physics(sllbm3d_ctx *c, double dt, double nu) {
  int rc = setup_allowed(c);
  if (rc) return rc;
  if (!std::isfinite(dt) || !(dt > 0)) return fail(c, SLLBM_E_ARG, "dt must be positive and finite");
  if (std::isnan(nu) || !(nu > 0))
    return fail(c, SLLBM_E_ARG, "nu must be positive (tau = nu/dt + 1/2 > 1/2) or +inf");
  c->dt = dt;
  c->nu = nu;
  // tau = nu / dt + 1/2 (Sec. II.D, c_s = 1); nu = +inf: no collision
  c->omega = std::isinf(nu) ? 0.0 : 1.0 / (nu / dt + 0.5);
  c->have_phys = true;
  c->dev_dirty = true;
  return SLLBM_OK;
}

int sllbm3d_num_nodes(const sllbm3d_ctx *c, int64_t *nx, int64_t *ny, int64_t *nz) {
  if (!c || !nx || !ny || !nz) return SLLBM_E_ARG;
  if (!c->have_grid) return fail(const_cast<sllbm3d_ctx *>(c), SLLBM_E_STATE, "grid not set");
  *nx = c->ax.n;
  *ny = c->ay.n;
  *nz = c->az.n;
  return SLLBM_OK;
}

int sllbm3d_node_coords(const sllbm3d_ctx *c, double *x, double *y, double *z) {
  if (!c || !x || !y || !z) return SLLBM_E_ARG;
  if (!c->have_grid) return fail(const_cast<sllbm3d_ctx *>(c), SLLBM_E_STATE, "grid not set");
  for (int j = 0; j < c->ax.n; ++j) x[j] = c->ax.coord(j);
  for (int j = 0; j < c->ay.n; ++j) y[j] = c->ay.coord(j);
  for (int j = 0; j < c->az.n; ++j) z[j] = c->az.coord(j);
  return SLLBM_OK;
}

int sllbm3d_bind_populations(sllbm3d_ctx *c, void *a, void *b) {
  if (!c) return SLLBM_E_ARG;
  if (!a || !b || a == b) return fail(c, SLLBM_E_ARG, "need two distinct device buffers");
  int rc = ready(c);
  if (rc) return rc;
  drop_populations(c);
  c->pop[0] = a;
  c->pop[1] = b;
  c->own_pop = false;
  c->cur = 0;
  c->initialised = false;
  return SLLBM_OK;
}

int sllbm3d_init_macro(sllbm3d_ctx *c, const double *rho, const double *ux, const double *uy,
                       const double *uz, int on_device) {
  if (!c) return SLLBM_E_ARG;
  if (!rho || !ux || !uy || !uz) return fail(c, SLLBM_E_ARG, "null macroscopic field");
  int rc = ready(c);
  if (rc) return rc;
  const long long N = nnodes(c);
  if (!on_device)
    for (long long v = 0; v < N; ++v)
      if (!std::isfinite(rho[v]) || !std::isfinite(ux[v]) || !std::isfinite(uy[v]) ||
          !std::isfinite(uz[v]) || !(rho[v] > 0))
        return fail(c, SLLBM_E_ARG, "rho must be positive and all fields finite");
  rc = prepare_device(c);
  if (rc) return rc;
  const double *d[4] = {rho, ux, uy, uz};
  if (!on_device) {
    rc = alloc_buf(c, c->macro, sizeof(double) * 4 * size_t(N));
    if (rc) return rc;
    double *m = static_cast<double *>(c->macro.ptr);
    for (int k = 0; k < 4; ++k) {
      HIP_TRY3(c, hipMemcpyAsync(m + k * N, d[k], sizeof(double) * N, hipMemcpyHostToDevice,
                                 c->stream));
      d[k] = m + k * N;
    }
  }
  c->cur = 0;
  HIP_TRY3(c, launch_init3d(c->fp32, make_consts(c), d[0], d[1], d[2], d[3], c->pop[0], c->stream));
  HIP_TRY3(c, launch_clear_flag(static_cast<int *>(c->flag.ptr), c->stream));
  if (!on_device) HIP_TRY3(c, hipStreamSynchronize(c->stream));
  c->steps_done = 0;
  c->initialised = true;
  return SLLBM_OK;
}

int sllbm3d_step(sllbm3d_ctx *c, int64_t n) {
  if (!c) return SLLBM_E_ARG;
  if (n < 0) return fail(c, SLLBM_E_ARG, "n must be >= 0");
  if (!c->initialised) return fail(c, SLLBM_E_STATE, "populations not initialised");
  int rc = prepare_device(c);
  if (rc) return rc;
  const Consts3 k = make_consts(c);
  const Tables3 t = make_tables(c);
  const Rows3 r = make_rows(c);
  for (int64_t s = 0; s < n; ++s) {
    HIP_TRY3(c, launch_step3d(c->fp32, k, t, r, c->pop[c->cur], c->pop[1 - c->cur],
                              static_cast<int *>(c->flag.ptr), c->stream));
    c->cur ^= 1;
    ++c->steps_done;
  }
  return SLLBM_OK;
}

int sllbm3d_status_flags(sllbm3d_ctx *c, int *unstable, int64_t *steps_done) {
  if (!c || !unstable || !steps_done) return SLLBM_E_ARG;
  if (!c->initialised) return fail(c, SLLBM_E_STATE, "populations not initialised");
  HIP_TRY3(c, hipSetDevice(c->device));
  HIP_TRY3(c, hipMemcpyAsync(unstable, c->flag.ptr, sizeof(int), hipMemcpyDeviceToHost,
                             c->stream));
  HIP_TRY3(c, hipStreamSynchronize(c->stream));
  *steps_done = c->steps_done;
  return SLLBM_OK;
}

int sllbm3d_moments(sllbm3d_ctx *c, double *rho, double *ux, double *uy, double *uz,
                    int on_device) {
  if (!c) return SLLBM_E_ARG;
  if (!rho || !ux || !uy || !uz) return fail(c, SLLBM_E_ARG, "null output array");
  if (!c->initialised) return fail(c, SLLBM_E_STATE, "populations not initialised");
  int rc = prepare_device(c);
  if (rc) return rc;
  const long long N = nnodes(c);
  double *d[4] = {rho, ux, uy, uz};
  if (!on_device) {
    rc = alloc_buf(c, c->macro, sizeof(double) * 4 * size_t(N));
    if (rc) return rc;
    for (int k = 0; k < 4; ++k) d[k] = static_cast<double *>(c->macro.ptr) + k * N;
  }
  HIP_TRY3(c, launch_moments3d(c->fp32, make_consts(c), c->pop[c->cur], d[0], d[1], d[2], d[3],
                               c->stream));
  if (!on_device) {
    double *h[4] = {rho, ux, uy, uz};
    for (int k = 0; k < 4; ++k)
      HIP_TRY3(c, hipMemcpyAsync(h[k], d[k], sizeof(double) * N, hipMemcpyDeviceToHost,
                                 c->stream));
    HIP_TRY3(c, hipStreamSynchronize(c->stream));
  }
  return SLLBM_OK;
}

int sllbm3d_mass(sllbm3d_ctx *c, double *mass) {
  if (!c || !mass) return SLLBM_E_ARG;
  if (!c->initialised) return fail(c, SLLBM_E_STATE, "populations not initialised");
  int rc = prepare_device(c);
  if (rc) return rc;
  double *out = static_cast<double *>(c->scalar.ptr);
  HIP_TRY3(c, launch_mass3d(c->fp32, make_consts(c), make_tables(c), c->pop[c->cur],
                            static_cast<double *>(c->partial.ptr), out, c->stream));
  HIP_TRY3(c, hipMemcpyAsync(mass, out, sizeof(double), hipMemcpyDeviceToHost, c->stream));
  HIP_TRY3(c, hipStreamSynchronize(c->stream));
  return SLLBM_OK;
}

int sllbm3d_get_populations(sllbm3d_ctx *c, void *dst, int on_device) {
  if (!c || !dst) return SLLBM_E_ARG;
  if (!c->initialised) return fail(c, SLLBM_E_STATE, "populations not initialised");
  if (on_device && (dst == c->pop[0] || dst == c->pop[1]))
    return fail(c, SLLBM_E_ARG, "destination is one of the context's population buffers");
  HIP_TRY3(c, hipSetDevice(c->device));
  HIP_TRY3(c, hipMemcpyAsync(dst, c->pop[c->cur], pop_bytes(c),
                             on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost,
                             c->stream));
  if (!on_device) HIP_TRY3(c, hipStreamSynchronize(c->stream));
  return SLLBM_OK;
}

int sllbm3d_set_populations(sllbm3d_ctx *c, const void *src, int on_device) {
  if (!c || !src) return SLLBM_E_ARG;
  int rc = prepare_device(c);
  if (rc) return rc;
  if (on_device && (src == c->pop[0] || src == c->pop[1]))
    return fail(c, SLLBM_E_ARG, "source is one of the context's population buffers");
  c->cur = 0;
  HIP_TRY3(c, hipMemcpyAsync(c->pop[0], src, pop_bytes(c),
                             on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice,
                             c->stream));
  HIP_TRY3(c, launch_clear_flag(static_cast<int *>(c->flag.ptr), c->stream));
  if (!on_device) HIP_TRY3(c, hipStreamSynchronize(c->stream));
  c->initialised = true;
  return SLLBM_OK;
}

}  // extern "C"
