// LDS-staged gather shared by the tiled stream + collide kernel and the
// tiled adjoint step.
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
#pragma once

#include <hip/hip_runtime.h>

#include "launch.hpp"
#include "step_common.hpp"

namespace sllbm {

// P1 = taps per axis: p+1 for the forward step, the transposed table width
// for the adjoint.
template <typename T, int P1, int S, int TY, int WX, int G, int R>
__device__ __forceinline__ void tiled_stream(const T *__restrict__ fin,
                                             const int32_t *__restrict__ xrel,
                                             const T *__restrict__ xw,
                                             const int32_t *__restrict__ xwin,
                                             const int32_t *__restrict__ yrel,
                                             const T *__restrict__ yw,
                                             const int32_t *__restrict__ ywin, int W, int ntx,
                                             int nty, int tx, int ty, int ixc, int iyc, int lane,
                                             int wv, const StepConsts &c, T *lds,
                                             T (&fs)[S][25]) {
  constexpr int ROWS = R * TY;            // staged rows per plane (>= window rows)
  constexpr int PLANE = ROWS * WX;
  constexpr int BUF = S * G * PLANE;      // one of two LDS buffers
  constexpr int NPH = 5 * (5 / G);        // phases: (b, group of G x-components)
  T *const dummy = lds + 2 * BUF;         // 64 slots for the unused half-row lanes
  const long long N = c.n;
  const unsigned plane_bytes = unsigned(N * (long long)sizeof(T));
  // this lane's x-stencils for the 5 x-components: p+1 consecutive
  // window-relative columns starting at xr0[a], with weights wx[a][m]
  int xr0[5];
  T wx[5][P1];
  // staged columns in bytes: x0 + lane, and the halo x0 + 64 + lane for
  // WX = 128 or x0 + 64 + (lane % 8) for WX = 72 (lanes 8..63 then repeat
  // lanes 0..7, so the halo load moves only the 8 columns it needs)
  unsigned col_off[5][2];
#pragma unroll
  for (int a = 0; a < 5; ++a) {
    xr0[a] = xrel[(a * P1) * c.nx + ixc];
#pragma unroll
    for (int m = 0; m < P1; ++m) wx[a][m] = xw[(a * P1 + m) * c.nx + ixc];
    const int x0 = xwin[a * ntx + tx];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int col = x0 + 64 * h + (h == 0 || WX == 128 ? lane : (lane & (WX - 65)));
      int wrapped = col % c.nx;
      wrapped += wrapped < 0 ? c.nx : 0;
      const int clamped = col < c.nx - 1 ? col : c.nx - 1;
      col_off[a][h] = unsigned(c.perx ? wrapped : clamped) * unsigned(sizeof(T));
    }
  }
  // prefetch registers: R rows x G planes x S sets x 2 half-rows
  T pre[R][G][S][2];
  auto load = [&](int ph) {
    const int b = ph / (5 / G), a0 = (ph % (5 / G)) * G;
    const int w0 = ywin[b * nty + ty];
#pragma unroll
    for (int rr = 0; rr < R; ++rr) {
      if (rr > 0 && wv + rr * TY >= W) break;  // wave-uniform: rows past the window
      int r = w0 + wv + rr * TY;
      int rw = r % c.ny;
      rw += rw < 0 ? c.ny : 0;
      r = c.pery ? rw : (r < c.ny - 1 ? r : c.ny - 1);  // rows past the window: never weighted
      const unsigned rowoff = unsigned(r) * unsigned(c.nx) * unsigned(sizeof(T));
#pragma unroll
      for (int g = 0; g < G; ++g)
#pragma unroll
        for (int s = 0; s < S; ++s) {
          const auto rs = make_rsrc(fin + (long long)(s * 25 + a0 + g + 5 * b) * N, plane_bytes);
          pre[rr][g][s][0] = buffer_load<T>(rs, col_off[a0 + g][0], rowoff);
          pre[rr][g][s][1] = buffer_load<T>(rs, col_off[a0 + g][1], rowoff);
        }
    }
  };
  auto store = [&](T *buf) {
#pragma unroll
    for (int rr = 0; rr < R; ++rr) {
      if (rr > 0 && wv + rr * TY >= W) break;
#pragma unroll
      for (int g = 0; g < G; ++g)
#pragma unroll
        for (int s = 0; s < S; ++s) {
          T *dst = buf + ((s * G + g) * ROWS + wv + rr * TY) * WX;
          dst[lane] = pre[rr][g][s][0];
          T *slot = (WX == 128 || lane < WX - 64) ? dst + 64 + lane : dummy + lane;
          *slot = pre[rr][g][s][1];
        }
    }
  };
  load(0);
  store(lds);
  lds_barrier();
#pragma unroll
  for (int ph = 0; ph < NPH; ++ph) {
    const int b = ph / (5 / G), a0 = (ph % (5 / G)) * G;
    T *cur = lds + (ph & 1) * BUF;
    if (ph + 1 < NPH) load(ph + 1);  // in flight during this phase's interpolation
    const int yr0 = yrel[(b * P1) * c.ny + iyc];  // wave-uniform target row
    T wy[P1];
#pragma unroll
    for (int n = 0; n < P1; ++n) wy[n] = yw[(b * P1 + n) * c.ny + iyc];
#pragma unroll
    for (int g = 0; g < G; ++g) {
      const int a = a0 + g;
      const T *corner = cur + (yr0 * WX + xr0[a]);
#pragma unroll
      for (int s = 0; s < S; ++s) {
        const T *src = corner + (s * G + g) * PLANE;
        T acc = T(0);
#pragma unroll
        for (int n = 0; n < P1; ++n) {
          T rv = T(0);
#pragma unroll
          for (int m = 0; m < P1; ++m) rv = fma(wx[a][m], src[n * WX + m], rv);
          acc = fma(wy[n], rv, acc);
        }
        // keep the FMAs in this phase: otherwise the compiler sinks them all
        // to the collision and keeps every LDS value of every phase alive
        asm volatile("" : "+v"(acc));
        fs[s][a + 5 * b] = acc;
      }
    }
    if (ph + 1 < NPH) store(lds + ((ph + 1) & 1) * BUF);
    lds_barrier();
  }
}

// Maps the linear workgroup id to a tile so that XCD x (workgroups
// x, x + 8, x + 16, ...) gets the contiguous tile range [x * per, (x+1) * per).
__device__ __forceinline__ int xcd_tile(int bid, int nblk) {
  const int per = (nblk + 7) >> 3;
  return (bid & 7) * per + (bid >> 3);
}

constexpr size_t kTiledLdsBudget = 163840;  // gfx950: 160 KiB of LDS per workgroup
constexpr int kTileRowsTY = 4;

template <typename T, int S>
size_t tiled_lds_bytes(int G, int R, int WX) {
  return (size_t(2) * S * G * R * kTileRowsTY * WX + 64) * sizeof(T);
}

}  // namespace sllbm
