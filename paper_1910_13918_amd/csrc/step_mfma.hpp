// Stream + collide with the x-pass of the interpolation on the matrix cores.
//
// On an axis-product grid the x-pass of velocity component a maps the staged
// source columns of a window row to the tile's 64 target columns through a
// banded matrix: row n holds target column n's p+1 Lagrange weights
// (eq. (17)) at its stencil columns.  For a block of 16 target columns the
// band spans at most 16 + 2p staged columns, so the x-pass of all (set, row)
// pairs of the window is a product of a 16 x 4k weight block with a 4k x 16
// block of staged values: v_mfma_f32_16x16x4f32, float32 in and out.  The
// bfloat16 experiment (StepConsts::bf16x) rounds the weights and the staged
// values to bfloat16 and takes the whole band in one 16 x 16 x 32 product
// (v_mfma_f32_16x16x32_bf16, float32 accumulation).  The y-pass (p+1 FMAs
// per value) and the collision stay on the vector units, in float32/float64.
// Requires float32 populations, at most 16 (set, row) pairs per window and
// departures within one node spacing of their cell (checked on the host).
#pragma once

#include <hip/hip_runtime.h>

#include <type_traits>

#include "launch.hpp"
#include "step_common.hpp"
#include "tiled_common.hpp"

namespace sllbm {

template <int P, int MODEL, int HALO, int G, int R, bool PR, int IM>
__global__ __launch_bounds__(64 * kTileRowsTY) void k_step_mfma(
    const float *__restrict__ fin, float *__restrict__ fout, const int32_t *__restrict__ xrel,
    const float *__restrict__ xw, const int32_t *__restrict__ xwin,
    const int32_t *__restrict__ yrel, const float *__restrict__ yw,
    const int32_t *__restrict__ ywin, int W, int ntx, int nty, StepConsts c,
    int *__restrict__ flag) {
  constexpr int TY = kTileRowsTY;
  constexpr int S = Sets<MODEL>::S;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  float *lds = reinterpret_cast<float *>(smem_raw);
  const int tile = xcd_tile(blockIdx.x, ntx * nty);
  if (tile >= ntx * nty) return;  // whole workgroup leaves together
  const int tx = tile % ntx, ty = tile / ntx;
  const int lane = threadIdx.x;
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.y);
  const int ix = tx * 64 + lane;
  const int iy = ty * TY + wv;
  const int ixc = ix < c.nx ? ix : c.nx - 1;
  const int iyc = iy < c.ny ? iy : c.ny - 1;
  float fs[S][25];
  tiled_stream<float, P + 1, S, TY, HALO, G, R, IM>(fin, xrel, xw, xwin, yrel, yw, ywin, W, ntx,
                                                   nty, tx, ty, ixc, iyc, lane, wv, c, lds, fs);
  if (ix < c.nx && iy < c.ny)
    collide_store<float, MODEL, PR>(fs, c, fout, (long long)iy * c.nx + ix, flag);
}

template <int P, int MODEL, int HALO, int R, bool PR, int IM>
hipError_t launch_mfma(const StepConsts &c, const DevTables &t, const float *in, float *out,
                       int *flag, hipStream_t s) {
  constexpr int TY = kTileRowsTY;
  constexpr int S = Sets<MODEL>::S;
  constexpr int PITCH = tiled_pitch<P + 1, HALO, IM>();
  const int ntx = (c.nx + 63) / 64, nty = (c.ny + TY - 1) / TY;
  const int grid = ((ntx * nty + 7) / 8) * 8;
  const dim3 block(64, TY);
  constexpr int G =
      tiled_lds_bytes(sizeof(float), S, 5, R * TY, PITCH, true) <= kTiledLdsBudget ? 5 : 1;
  const size_t lds = tiled_lds_bytes(sizeof(float), S, G, t.win_rows, PITCH, true);
  k_step_mfma<P, MODEL, HALO, G, R, PR, IM><<<grid, block, lds, s>>>(
      in, out, t.xrel, static_cast<const float *>(t.xw), t.xwin, t.yrel,
      static_cast<const float *>(t.yw), t.ywin, t.win_rows, ntx, nty, c, flag);
  return hipGetLastError();
}

// PR: the Pr != 1 collision (thermal models only)
template <bool PR>
hipError_t launch_mfma_family(int fp32, int model, const StepConsts &c, const DevTables &t,
                              const void *fin, void *fout, int *flag, hipStream_t s) {
  if (!fp32 || !t.mfma_ok || t.tile_rows != kTileRowsTY || t.xrel == nullptr ||
      t.yrel == nullptr || t.win_rows > 3 * kTileRowsTY)
    return hipErrorInvalidValue;
  const int halo = tiled_halo(t.win_cols, c.nx, c.ny);
  if (halo == 0) return hipErrorInvalidValue;
  if (c.q1 != 5) return hipErrorInvalidValue;  // D2Q25 only
  return dispatch_step<PR>(1, c.p, model, [&]<typename T, int P, int MODEL>() -> hipError_t {
    if constexpr (!std::is_same_v<T, float>) {
      return hipErrorInvalidValue;
    } else {
      const float *in = static_cast<const float *>(fin);
      float *out = static_cast<float *>(fout);
      auto go = [&]<int R, int IM>() {
        if (halo == 4) return launch_mfma<P, MODEL, 4, R, PR, IM>(c, t, in, out, flag, s);
        if (halo == 8) return launch_mfma<P, MODEL, 8, R, PR, IM>(c, t, in, out, flag, s);
        return launch_mfma<P, MODEL, 64, R, PR, IM>(c, t, in, out, flag, s);
      };
      // the bfloat16 experiment: bfloat16 weights and staged values
      if (c.bf16x)
        return t.win_rows <= 2 * kTileRowsTY ? go.template operator()<2, kInterpMfmaBf16>()
                                              : go.template operator()<3, kInterpMfmaBf16>();
      return t.win_rows <= 2 * kTileRowsTY ? go.template operator()<2, kInterpMfma>()
                                            : go.template operator()<3, kInterpMfma>();
    }
  });
}

}  // namespace sllbm
