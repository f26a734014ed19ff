// Stream + collide with the departure gather served from LDS.
//
// A workgroup owns a tile of 64 x-nodes (one per lane) by TY rows (one
// wavefront per row).  For the departure points of velocity i = a + 5b, the
// tile needs a window of source rows that depends only on b and a window of
// source columns that depends only on a (both precomputed per tile: the
// departure geometry is static).  Per phase (one b and a group of G
// x-components, for every population set) the workgroup
//   1. stages the raw source windows (W rows by WX columns, WX = 72 or 128)
//      into LDS with row-contiguous buffer loads -- one or two loads per lane
//      per window row, instead of (p+1)^2 scattered gathers per node;
//   2. evaluates each node's cell-local tensor Lagrange interpolant (eq. (17))
//      from LDS: an x-pass over p+1 columns on each of the node's p+1 rows,
//      then the y-combination, keeping all 25 (or 50) streamed values of the
//      node in registers.
// The collision then runs in float64 and the post-collision populations are
// stored with coalesced writes.
//
// Workgroups are numbered so that each of the 8 XCDs (which receive
// workgroups round-robin) sweeps a contiguous band of tiles; vertically
// neighbouring tiles, which share halo rows, then meet in the same L2.
#include <hip/hip_runtime.h>

#include "launch.hpp"
#include "step_common.hpp"
#include "tiled_common.hpp"

namespace sllbm {

template <typename T, int P, int MODEL, int TY, int WX, int G, int R>
__global__ __launch_bounds__(64 * TY) void k_step_tiled(
    const T *__restrict__ fin, T *__restrict__ fout, const int32_t *__restrict__ xrel,
    const T *__restrict__ xw, const int32_t *__restrict__ xwin, const int32_t *__restrict__ yrel,
    const T *__restrict__ yw, const int32_t *__restrict__ ywin, int W, int ntx, int nty,
    StepConsts c, int *__restrict__ flag) {
  constexpr int S = Sets<MODEL>::S;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T *lds = reinterpret_cast<T *>(smem_raw);
  const int tile = xcd_tile(blockIdx.x, ntx * nty);
  if (tile >= ntx * nty) return;  // whole workgroup leaves together
  const int tx = tile % ntx, ty = tile / ntx;
  const int lane = threadIdx.x;
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.y);
  const int ix = tx * 64 + lane;
  const int iy = ty * TY + wv;
  const int ixc = ix < c.nx ? ix : c.nx - 1;
  const int iyc = iy < c.ny ? iy : c.ny - 1;
  T fs[S][25];
  tiled_stream<T, P + 1, S, TY, WX, G, R>(fin, xrel, xw, xwin, yrel, yw, ywin, W, ntx, nty, tx,
                                          ty, ixc, iyc, lane, wv, c, lds, fs);
  if (ix < c.nx && iy < c.ny) collide_store<T, MODEL>(fs, c, fout, (long long)iy * c.nx + ix, flag);
}

template <typename T, int P, int MODEL, int WX, int R>
hipError_t launch_tiled(const StepConsts &c, const DevTables &t, const T *in, T *out, int *flag,
                        hipStream_t s) {
  constexpr int TY = kTileRowsTY;
  constexpr int S = Sets<MODEL>::S;
  const int ntx = (c.nx + 63) / 64, nty = (c.ny + TY - 1) / TY;
  const int grid = ((ntx * nty + 7) / 8) * 8;
  const dim3 block(64, TY);
  // all five x-components per phase when both LDS buffers fit, else one
  if (tiled_lds_bytes<T, S>(5, R, WX) <= kTiledLdsBudget) {
    k_step_tiled<T, P, MODEL, TY, WX, 5, R><<<grid, block, tiled_lds_bytes<T, S>(5, R, WX), s>>>(
        in, out, t.xrel, static_cast<const T *>(t.xw), t.xwin, t.yrel,
        static_cast<const T *>(t.yw), t.ywin, t.win_rows, ntx, nty, c, flag);
  } else {
    k_step_tiled<T, P, MODEL, TY, WX, 1, R><<<grid, block, tiled_lds_bytes<T, S>(1, R, WX), s>>>(
        in, out, t.xrel, static_cast<const T *>(t.xw), t.xwin, t.yrel,
        static_cast<const T *>(t.yw), t.ywin, t.win_rows, ntx, nty, c, flag);
  }
  return hipGetLastError();
}

// Largest window the tiled kernel stages: 3 rows per wavefront and 128
// columns.
bool tiled_window_ok(int win_rows, int win_cols) {
  return win_rows <= 3 * kTileRowsTY && win_cols <= 128;
}

hipError_t launch_step_tiled(int fp32, int model, const StepConsts &c, const DevTables &t,
                             const void *fin, void *fout, int *flag, hipStream_t s) {
  if (t.tile_rows != kTileRowsTY || t.yrel == nullptr || t.xrel == nullptr)
    return hipErrorInvalidValue;
  if (!tiled_window_ok(t.win_rows, t.win_cols)) return hipErrorInvalidValue;
  return dispatch_step(fp32, c.p, model, [&]<typename T, int P, int MODEL>() {
    const T *in = static_cast<const T *>(fin);
    T *out = static_cast<T *>(fout);
    const bool narrow = t.win_cols <= 72;
    if (t.win_rows <= 2 * kTileRowsTY)
      return narrow ? launch_tiled<T, P, MODEL, 72, 2>(c, t, in, out, flag, s)
                    : launch_tiled<T, P, MODEL, 128, 2>(c, t, in, out, flag, s);
    return narrow ? launch_tiled<T, P, MODEL, 72, 3>(c, t, in, out, flag, s)
                  : launch_tiled<T, P, MODEL, 128, 3>(c, t, in, out, flag, s);
  });
}

}  // namespace sllbm
