// The adjoint step's transposed gather through LDS-staged windows (the
// staging of the forward tiled kernel, fed the transposed tables), fused with
// the transposed collision Jacobian of the previous step.  Instantiated per
// population type in adjoint_tiled_f32.hip and adjoint_tiled_f64.hip (the
// tap-count x halo x window-height variants make this the largest unit).
#pragma once

#include <hip/hip_runtime.h>

#include <type_traits>

#include "adjoint_common.hpp"
#include "launch.hpp"
#include "step_common.hpp"
#include "tiled_common.hpp"

namespace sllbm {

// S^T with the LDS-staged gather of the forward step.
template <typename T, int MODEL, int TAPS, int HALO, int G, int R>
__global__ __launch_bounds__(64 * kTileRowsTY) void k_adjoint_step_tiled(
    const T *__restrict__ mu, const int32_t *__restrict__ xrel, const T *__restrict__ xw,
    const int32_t *__restrict__ xwin, const int32_t *__restrict__ yrel, const T *__restrict__ yw,
    const int32_t *__restrict__ ywin, int W, int ntx, int nty, const double *__restrict__ mom,
    T *__restrict__ out, StepConsts c) {
  constexpr int TY = kTileRowsTY;
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
  T lam[S][25];
  tiled_stream<T, TAPS, S, TY, HALO, G, R, (TAPS >= kSeparableTaps ? kInterpSep : kInterp2D)>(
      mu, xrel, xw, xwin, yrel, yw, ywin, W, ntx, nty, tx, ty, ixc, iyc, lane, wv, c, lds, lam);
  if (ix < c.nx && iy < c.ny) {
    const long long v = (long long)iy * c.nx + ix;
    if (mom)
      collision_adjoint_store<T, MODEL>(lam, mom, c, out, v);
    else
      store_sets<T, S>(lam, c, out, v);
  }
}

template <typename T>
hipError_t launch_adjoint_step_tiled_t(int model, const StepConsts &c, const DevTables &t,
                                       const void *mu, const double *mom_prev, void *out,
                                       hipStream_t s) {
  if (t.taps < 2 || t.taps > kMaxTaps) return hipErrorInvalidValue;
  return dispatch_taps(sizeof(T) == 4, model, t.taps,
                       [&]<typename U, int MODEL, int TAPS>() -> hipError_t {
    if constexpr (!std::is_same_v<U, T>) {
      return hipErrorInvalidValue;
    } else {
      const T *in = static_cast<const T *>(mu);
      T *o = static_cast<T *>(out);
      constexpr int S = Sets<MODEL>::S;
      constexpr int TY = kTileRowsTY;
      const int ntx = (c.nx + 63) / 64, nty = (c.ny + TY - 1) / TY;
      const int grid = ((ntx * nty + 7) / 8) * 8;
      const int W = t.win_rows;
      const int halo = tiled_halo(t.win_cols, c.nx, c.ny);
      if (W > 3 * TY || halo == 0) return hipErrorInvalidValue;
      constexpr bool SEP = TAPS >= kSeparableTaps;
      auto go = [&]<int HALO, int R>() {
        // all five x-components per phase when the LDS buffers of the
        // tallest window this instantiation serves fit, else one
        constexpr int G =
            tiled_lds_bytes(sizeof(T), S, 5, R * TY, 64 + HALO, SEP) <= kTiledLdsBudget ? 5 : 1;
        const size_t lds = tiled_lds_bytes(sizeof(T), S, G, W, 64 + HALO, SEP);
        k_adjoint_step_tiled<T, MODEL, TAPS, HALO, G, R><<<grid, dim3(64, TY), lds, s>>>(
            in, t.xrel, static_cast<const T *>(t.xw), t.xwin, t.yrel,
            static_cast<const T *>(t.yw), t.ywin, W, ntx, nty, mom_prev, o, c);
      };
      auto by_rows = [&]<int HALO>() {
        if (W <= 2 * TY) go.template operator()<HALO, 2>();
        else go.template operator()<HALO, 3>();
      };
      if (halo == 4) by_rows.template operator()<4>();
      else if (halo == 8) by_rows.template operator()<8>();
      else by_rows.template operator()<64>();
      return hipGetLastError();
    }
  });
}

}  // namespace sllbm
