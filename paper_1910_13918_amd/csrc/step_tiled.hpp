// Stream + collide with the departure gather served from LDS: the windows
// of source rows and columns each tile of 64 x 4 nodes needs are staged per
// velocity group (tiled_common.hpp), interpolated from LDS, and the node's
// streamed populations are collided and stored in the same kernel.
#pragma once

#include <hip/hip_runtime.h>

#include "launch.hpp"
#include "step_common.hpp"
#include "tiled_common.hpp"

namespace sllbm {

template <typename T, int P, int MODEL, int TY, int HALO, int G, int R, bool PR>
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
  // wave priority 2 while staging and interpolating, 0 for the float64
  // collision (as the row-segment step; Riemann 1025^2 134.8 -> 133.0 us
  // float32, 269 -> 266 us float64)
  __builtin_amdgcn_s_setprio(2);
  tiled_stream<T, P + 1, S, TY, HALO, G, R,
               (P + 1 >= kSeparableTaps ? kInterpSep : kInterp2D)>(
      fin, xrel, xw, xwin, yrel, yw, ywin, W, ntx, nty, tx, ty, ixc, iyc, lane, wv, c, lds, fs);
  __builtin_amdgcn_s_setprio(0);
  if (ix < c.nx && iy < c.ny)
    collide_store<T, MODEL, PR>(fs, c, fout, (long long)iy * c.nx + ix, flag);
}

template <typename T, int P, int MODEL, int HALO, int R, bool PR>
hipError_t launch_tiled(const StepConsts &c, const DevTables &t, const T *in, T *out, int *flag,
                        hipStream_t s) {
  constexpr int TY = kTileRowsTY;
  constexpr int S = Sets<MODEL>::S;
  constexpr bool SEP = P + 1 >= kSeparableTaps;
  // all five x-components per phase when the LDS buffers of the tallest
  // window this instantiation serves (R TY rows) fit, else one
  constexpr int G = tiled_lds_bytes(sizeof(T), S, 5, R * TY, 64 + HALO, SEP) <= kTiledLdsBudget
                        ? 5 : 1;
  const int ntx = (c.nx + 63) / 64, nty = (c.ny + TY - 1) / TY;
  const int grid = ((ntx * nty + 7) / 8) * 8;
  const size_t lds = tiled_lds_bytes(sizeof(T), S, G, t.win_rows, 64 + HALO, SEP);
  k_step_tiled<T, P, MODEL, TY, HALO, G, R, PR><<<grid, dim3(64, TY), lds, s>>>(
      in, out, t.xrel, static_cast<const T *>(t.xw), t.xwin, t.yrel, static_cast<const T *>(t.yw),
      t.ywin, t.win_rows, ntx, nty, c, flag);
  return hipGetLastError();
}

// Largest window the tiled kernel stages: 3 rows per wavefront and 128
// columns.
inline bool tiled_window_ok(int win_rows, int win_cols) {
  return win_rows <= 3 * kTileRowsTY && win_cols <= 128;
}

// PR: the Pr != 1 collision (thermal models only)
template <bool PR>
hipError_t launch_tiled_family(int fp32, int model, const StepConsts &c, const DevTables &t,
                               const void *fin, void *fout, int *flag, hipStream_t s) {
  if (t.tile_rows != kTileRowsTY || t.yrel == nullptr || t.xrel == nullptr)
    return hipErrorInvalidValue;
  if (!tiled_window_ok(t.win_rows, t.win_cols)) return hipErrorInvalidValue;
  if (c.q1 != 5) return hipErrorInvalidValue;  // D2Q25 only
  return dispatch_step<PR>(fp32, c.p, model, [&]<typename T, int P, int MODEL>() {
    const T *in = static_cast<const T *>(fin);
    T *out = static_cast<T *>(fout);
    const int halo = tiled_halo(t.win_cols, c.nx, c.ny);
    auto go = [&]<int R>() {
      if (halo == 4) return launch_tiled<T, P, MODEL, 4, R, PR>(c, t, in, out, flag, s);
      if (halo == 8) return launch_tiled<T, P, MODEL, 8, R, PR>(c, t, in, out, flag, s);
      return launch_tiled<T, P, MODEL, 64, R, PR>(c, t, in, out, flag, s);
    };
    return t.win_rows <= 2 * kTileRowsTY ? go.template operator()<2>()
                                          : go.template operator()<3>();
  });
}

}  // namespace sllbm
