// The adjoint step's transposed gather through row segments (the
// streaming of the forward row-segment kernel, fed the transposed tables),
// fused with the transposed collision Jacobian of the previous step.
#include <hip/hip_runtime.h>

#include "adjoint_common.hpp"
#include "launch.hpp"
#include "step_common.hpp"
#include "step_rows.hpp"
#include "tiled_common.hpp"

namespace sllbm {

// S^T with the row-segment gather of the forward step (transposed tables).
template <typename T, int MODEL, int TAPS>
__global__ __launch_bounds__(64 * kRowsTileRows) void k_adjoint_step_rows(
    const T *__restrict__ mu, const int32_t *__restrict__ xrel, const T *__restrict__ xw,
    const int32_t *__restrict__ xwin, const int32_t *__restrict__ ysrc, const T *__restrict__ yw,
    int TX, int ntx, int nty, const double *__restrict__ mom, T *__restrict__ out, StepConsts c) {
  constexpr int S = Sets<MODEL>::S;
  __shared__ T rows_lds[kRowsTileRows][2][64];
  const int tile = xcd_tile(blockIdx.x, ntx * nty);
  if (tile >= ntx * nty) return;
  const int tx = tile % ntx, ty = tile / ntx;
  const int lane = threadIdx.x;
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.y);
  const int iy = ty * kRowsTileRows + wv;
  if (iy >= c.ny) return;  // whole wavefront; nothing below waits for others
  T lam[S][25];
  rows_stream<T, TAPS, S, sizeof(T) == 4 ? 2 : 4>(mu, xrel, xw, xwin, ysrc, yw, TX, ntx, tx, iy,
                                                  lane, c, &rows_lds[wv][0][0], lam);
  const int ix = tx * TX + lane;
  if (ix < c.nx && lane < TX) {
    const long long v = (long long)iy * c.nx + ix;
    if (mom)
      collision_adjoint_store<T, MODEL>(lam, mom, c, out, v);
    else
      store_sets<T, S>(lam, c, out, v);
  }
}

hipError_t launch_adjoint_step_rows(int fp32, int model, const StepConsts &c, const DevTables &t,
                                    const void *mu, const double *mom_prev, void *out,
                                    hipStream_t s) {
  if (t.taps < 2 || t.taps > kMaxTaps) return hipErrorInvalidValue;
  return dispatch_taps(fp32, model, t.taps, [&]<typename T, int MODEL, int TAPS>() -> hipError_t {
    const T *in = static_cast<const T *>(mu);
    T *o = static_cast<T *>(out);
    if (t.rows_tx < kRowsMinCols || t.rows_tx > 64 || !t.rows_xrel || !t.rows_xwin ||
        !(t.ident_y & t.ident_x & 1))
      return hipErrorInvalidValue;
    const int ntx = (c.nx + t.rows_tx - 1) / t.rows_tx;
    const int nty = (c.ny + kRowsTileRows - 1) / kRowsTileRows;
    const int grid = ((ntx * nty + 7) / 8) * 8;
    k_adjoint_step_rows<T, MODEL, TAPS><<<grid, dim3(64, kRowsTileRows), 0, s>>>(
        in, t.rows_xrel, static_cast<const T *>(t.xw), t.rows_xwin, t.ysrc,
        static_cast<const T *>(t.yw), t.rows_tx, ntx, nty, mom_prev, o, c);
    return hipGetLastError();
  });
}

}  // namespace sllbm
