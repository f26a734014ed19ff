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

namespace sllbm {

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

constexpr size_t kTiledLdsBudget = 163840;  // gfx950: 160 KiB of LDS per workgroup
constexpr int kTileRowsTY = 4;

template <typename T, int S>
size_t tiled_lds_bytes(int G, int R, int WX) {
  return (size_t(2) * S * G * R * kTileRowsTY * WX + 64) * sizeof(T);
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
