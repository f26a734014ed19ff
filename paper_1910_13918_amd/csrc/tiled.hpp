// Stream + collide with the separable interpolation staged through LDS.
//
// A workgroup owns a tile of 64 x-nodes (one per lane) by TY rows (one
// wavefront per row).  For each velocity i = a + 5b the interpolation at the
// departure point factorises into an x-pass and a y-pass (the 2-D Lagrange
// basis of a cell is the product of the 1-D bases, eq. (17)):
//   x-pass: every source row r of the tile's row window (the rows that the
//           tile's departure points need for velocity component b) is
//           interpolated in x at the 64 departure abscissae of component a,
//           gathering p+1 values per lane from global memory, and the row is
//           written to LDS;
//   y-pass: each lane combines p+1 LDS rows with the y-weights of its own
//           target row.
// The streamed values of all 25 (or 50) populations of the node stay in
// registers; the collision then runs in float64 and the post-collision values
// are stored with coalesced writes.  LDS is double-buffered so one barrier per
// velocity suffices.
#pragma once

#include "step_common.hpp"

namespace sllbm {

template <typename T, int P, int MODEL, int TY>
__global__ __launch_bounds__(64 * TY) void k_step_tiled(
    const T *__restrict__ fin, T *__restrict__ fout, const int32_t *__restrict__ xsrc,
    const T *__restrict__ xw, const int32_t *__restrict__ yrel, const T *__restrict__ yw,
    const int32_t *__restrict__ ywin, int W, StepConsts c, int *__restrict__ flag) {
  constexpr int S = Sets<MODEL>::S;
  constexpr int P1 = P + 1;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T *H = reinterpret_cast<T *>(smem_raw);  // [2][S][W][64]
  const int lane = threadIdx.x;
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.y);
  const int ix = blockIdx.x * 64 + lane;
  const int ixc = ix < c.nx ? ix : c.nx - 1;
  const int tile = blockIdx.y;
  const int iy = tile * TY + wv;
  const int iyc = iy < c.ny ? iy : c.ny - 1;
  const int ntiles = gridDim.y;
  const long long N = c.n;
  T fs[S][25];
  int buf = 0;
#pragma unroll
  for (int b = 0; b < 5; ++b) {
    const int w0 = ywin[b * ntiles + tile];
    int yr[P1];
    T wy[P1];
#pragma unroll
    for (int n = 0; n < P1; ++n) {
      yr[n] = yrel[(b * P1 + n) * c.ny + iyc];
      wy[n] = yw[(b * P1 + n) * c.ny + iyc];
    }
#pragma unroll
    for (int a = 0; a < 5; ++a) {
      const int i = a + 5 * b;
      int xo[P1];
      T wx[P1];
#pragma unroll
      for (int m = 0; m < P1; ++m) {
        xo[m] = xsrc[(a * P1 + m) * c.nx + ixc];
        wx[m] = xw[(a * P1 + m) * c.nx + ixc];
      }
      T *Hb = H + buf * (S * W * 64);
      for (int k = wv; k < W; k += TY) {
        int r = w0 + k;
        if (c.pery) {
          r %= c.ny;
          if (r < 0) r += c.ny;
        } else if (r > c.ny - 1) {
          r = c.ny - 1;  // window rows past the edge are never weighted
        }
#pragma unroll
        for (int s = 0; s < S; ++s) {
          const T *src = fin + (long long)(s * 25 + i) * N + (long long)r * c.nx;
          T acc = T(0);
#pragma unroll
          for (int m = 0; m < P1; ++m) acc = fma(wx[m], src[xo[m]], acc);
          Hb[(s * W + k) * 64 + lane] = acc;
        }
      }
      __syncthreads();
#pragma unroll
      for (int s = 0; s < S; ++s) {
        T acc = T(0);
#pragma unroll
        for (int n = 0; n < P1; ++n) acc = fma(wy[n], Hb[(s * W + yr[n]) * 64 + lane], acc);
        fs[s][i] = acc;
      }
      buf ^= 1;
    }
  }
  if (ix < c.nx && iy < c.ny) collide_store<T, MODEL>(fs, c, fout, (long long)iy * c.nx + ix, flag);
}

template <typename T, int P, int MODEL>
hipError_t launch_step_tiled(const StepConsts &c, const DevTables &t, const T *in, T *out,
                             int *flag, hipStream_t s) {
  constexpr int TY = 8;
  if (t.tile_rows != TY || t.yrel == nullptr) return hipErrorInvalidValue;
  const int W = t.win_rows;
  const size_t lds = size_t(2) * Sets<MODEL>::S * W * 64 * sizeof(T);
  dim3 grid((c.nx + 63) / 64, (c.ny + TY - 1) / TY);
  k_step_tiled<T, P, MODEL, TY><<<grid, dim3(64, TY), lds, s>>>(
      in, out, t.xsrc, static_cast<const T *>(t.xw), t.yrel, static_cast<const T *>(t.yw), t.ywin,
      W, c, flag);
  return hipGetLastError();
}

}  // namespace sllbm
