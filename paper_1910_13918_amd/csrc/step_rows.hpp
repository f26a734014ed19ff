// Stream + collide with one independent wavefront per target row segment.
//
// On an axis-product grid the departure rows of velocity i = a + 5b depend
// only on (b, target row) and are therefore the same for every lane of a
// wavefront that owns one row segment of TX nodes.  For each population
// plane the wavefront
//   1. loads its p+1 source rows over a window of 64 consecutive source
//      columns (one element per lane; the host picks TX so that every
//      tile's x-stencils fit the 64 columns, so there is no halo);
//   2. combines them with the uniform y-weights in registers (eq. (17),
//      y-factor first), writes the one y-interpolated row to its own LDS
//      row, and
//   3. evaluates the x-factor from LDS with each lane's p+1 x-weights.
// No LDS row is shared between wavefronts; loads run a fixed number of planes
// ahead of the arithmetic.  A workgroup barrier every few planes only keeps
// the wavefronts of neighbouring rows, which read overlapping source rows,
// close enough together for those reads to hit in the L1 cache.
// The streamed values stay in registers and the collision is the one of the
// other paths (collide_store).  The forward step reads and writes the grouped
// storage order (PopLayout), in which the four moving x-components of one
// velocity row lie next to each other for every node: the planes of one row
// then come from one stretch of memory instead of four planes 4 MB apart
// (Riemann 1025^2 nodes, float32 f + g: 99.7 against 108.8 us per step on
// one box); the adjoint's transposed gather keeps the planar order of its
// own arrays.
#pragma once

#include <hip/hip_runtime.h>

#include "launch.hpp"
#include "step_common.hpp"
#include "tiled_common.hpp"

namespace sllbm {

constexpr int kRowsTileRows = 4;  // wavefronts (rows) per workgroup: adjoint, float32 step

// Rows per workgroup of the forward step: float64 f + g takes 8 (+1-3 % over
// 4 on 1025^2-node grids, Pr = 0.75 alike), and so does float32 f + g at p = 2
// since the wave priorities (Riemann 1025^2 102.4 -> 101.7 us over three
// same-box pairs; at p = 3 the shock-vortex rows lost 25 % with 8); a single
// float64 set (-3 %) and the other float32 cases keep 4.
template <typename T, int S, int P1 = 0>
constexpr int rows_tile_rows() {
  return S == 2 && (sizeof(T) == 8 || P1 == 3) ? 8 : kRowsTileRows;
}

// Orders this wavefront's LDS accesses: what its lanes wrote before is
// visible to its lanes after (LDS instructions of one wavefront complete in
// order; the fences keep the compiler from moving accesses across).
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront", "local");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront", "local");
}

// Planes whose loads are in flight ahead of the one being interpolated,
// measured on 1025^2-node grids (float32):
//   a single population set: 4 at p = 1, else 3 (one plane more or less
//   costs 1-10 %);
//   f + g, with the barrier of rows_sync_planes: 9 - p (8 ... 5; one plane
//   more or less is within 1 %; without the barrier the best depths were
//   4, 3, 2, 1 and 5-16 % slower).
// float64: a single set 10 at p <= 2 and 6 above (within 5 % from 8 to 20);
//   f + g 14 and 9 (+0-3 % over 10 and 6; 18 and 12 are no better).
template <typename T, int P1, int S, bool PR>
constexpr int rows_lookahead() {
  if (sizeof(T) == 8) return S == 2 ? (P1 <= 3 ? 14 : 9) : (P1 <= 3 ? 10 : 6);
  if (S == 2) return 10 - P1;
  return P1 == 2 ? 4 : 3;
}

// Streams the 25 S planes of `fin` into fs for the node (iy, tx TX + lane):
// P1 taps per axis (p+1 forward, the transposed width for the adjoint),
// D planes of loads in flight; lrow = this wavefront's two LDS rows.
// SYNC > 0: a workgroup barrier after every SYNC planes, so every wavefront
// of the workgroup must call this (none may have returned).  The
// first 1-D velocity is 0 (Table I; the host checks that its x- and y-tables
// are the identity), so the phase b = 0 departs from the node itself and
// loads the target row alone, the x-component a = 0 reads the node's own
// column, and the rest velocity (0, 0) is the node's own value.
template <typename T, int P1, int S, int D, int SYNC = 0, int Q1 = 5>
__device__ __forceinline__ void rows_stream(const T *__restrict__ fin,
                                            const int32_t *__restrict__ xrel,
                                            const T *__restrict__ xw,
                                            const int32_t *__restrict__ xwin,
                                            const int32_t *__restrict__ ysrc,
                                            const T *__restrict__ yw, int TX, int ntx, int tx,
                                            int iy, int lane, const StepConsts &c, T *lrow,
                                            T (&fs)[S][Q1 * Q1]) {
  constexpr int Q = Q1 * Q1;
  constexpr int NQ = Q * S;  // planes, in the order (b, s, a)
  // lanes past the segment take the stencil of its last node (in the window)
  const int ixc = min(tx * TX + min(lane, TX - 1), c.nx - 1);
  const long long N = c.n;
  const unsigned plane_bytes = unsigned(N * (long long)sizeof(T));
  const unsigned row_bytes = unsigned(c.nx) * unsigned(sizeof(T));
  int xr0[Q1];
  T wx[Q1][P1];
  unsigned col_off[Q1];
  const int own0 = ixc - xwin[tx];  // the node's column in the a = 0 window
  const unsigned own_off = unsigned(ixc) * unsigned(sizeof(T));
#pragma unroll
  for (int a = 0; a < Q1; ++a) {
    xr0[a] = xrel[(a * P1) * c.nx + ixc];
#pragma unroll
    for (int m = 0; m < P1; ++m) wx[a][m] = xw[(a * P1 + m) * c.nx + ixc];
    col_off[a] =
        unsigned(wrap_or_clamp(xwin[a * ntx + tx] + lane, c.nx, c.perx)) * unsigned(sizeof(T));
  }
  // source rows (byte offsets) and weights of the y-factor: wave-uniform,
  // fetched one phase (b) at a time, shortly before its first load, so that
  // only two phases' worth occupy scalar registers
  unsigned yoff[Q1][P1];
  T wy[Q1][P1];
  auto fetch_phase = [&](int b) {
    int z = 0;
    asm volatile("" : "+s"(z));  // keeps the scalar loads here
#pragma unroll
    for (int m = 0; m < P1; ++m) {
      yoff[b][m] = unsigned(ysrc[(b * P1 + m) * c.ny + iy + z]) * row_bytes;
      wy[b][m] = yw[(b * P1 + m) * c.ny + iy + z];
    }
  };
  auto plane_of = [](int q) {  // q -> (b, s, a)
    const int b = q / (Q1 * S), r = q % (Q1 * S);
    return int3{b, r / Q1, r % Q1};
  };
  T pre[D + 1][P1];
  auto load = [&](int q, T (&dst)[P1]) {
    const int3 p = plane_of(q);
    const auto rs = make_rsrc(fin + (long long)(p.y * Q + p.z + Q1 * p.x) * N, plane_bytes);
    if (p.x == 0) {  // identity y-factor (resolved at compile time)
      dst[0] = buffer_load<T>(rs, p.z == 0 ? own_off : col_off[p.z], unsigned(iy) * row_bytes);
#pragma unroll
      for (int m = 1; m < P1; ++m) dst[m] = T(0);
    } else {
#pragma unroll
      for (int m = 0; m < P1; ++m) dst[m] = buffer_load<T>(rs, col_off[p.z], yoff[p.x][m]);
    }
  };
  constexpr int PH = Q1 * S;  // planes per phase
#pragma unroll
  for (int b = 1; b <= (D + 1) / PH && b < Q1; ++b) fetch_phase(b);
#pragma unroll
  for (int q = 0; q < D && q < NQ; ++q) load(q, pre[q % (D + 1)]);
#pragma unroll
  for (int q = 0; q < NQ; ++q) {
    if (SYNC > 0 && q > 0 && q % SYNC == 0) __builtin_amdgcn_s_barrier();
    // the phase whose first load comes two iterations from now
    if ((q + D + 2) % PH == 0 && (q + D + 2) / PH < Q1 && (q + D + 2) / PH > (D + 1) / PH)
      fetch_phase((q + D + 2) / PH);
    if (q + D < NQ) load(q + D, pre[(q + D) % (D + 1)]);
    const int3 p = plane_of(q);
    const T(&v)[P1] = pre[q % (D + 1)];
    T y = v[0];
    if (p.x != 0) {
      y = wy[p.x][0] * v[0];
#pragma unroll
      for (int m = 1; m < P1; ++m) y = fma(wy[p.x][m], v[m], y);
    }
    T acc = y;  // the rest velocity: loaded at the node's own column
    if (p.x != 0 || p.z != 0) {
      T *row = lrow + (q & 1) * 64;
      row[lane] = y;
      wave_lds_sync();
      if (p.z == 0) {  // identity x-factor
        acc = row[own0];
      } else {
        acc = wx[p.z][0] * row[xr0[p.z]];
#pragma unroll
        for (int m = 1; m < P1; ++m) acc = fma(wx[p.z][m], row[xr0[p.z] + m], acc);
      }
    }
    asm volatile("" : "+v"(acc));  // keep the plane's arithmetic in its place
    fs[p.y][p.z + Q1 * p.x] = acc;
  }
}

// The forward step's gather over the grouped storage order (PopLayout): the
// same interpolation as rows_stream, velocity row by velocity row.  For each
// group (b, s) the wavefront issues the loads of all Q1 x-components of each
// source row together (the Q1 - 1 moving ones lie in one stretch of memory,
// so the loads share cache lines while in flight), y-combines them, writes
// the Q1 - 1 moving rows to its own LDS rows and x-combines them after one
// LDS sync; the component a = 0 (identity x-factor) is read at the node's own
// column and needs no LDS.  The moving components of a segment share one
// source window (xwin of component 1), so each lane reads the Q1 - 1 values
// of its window column in one wide load: separate 4-byte loads at the
// 16-byte node stride each touched four times the cache lines (L1 accesses
// 81 M against 18 M per step on the planar order).  DG groups of loads run ahead of the arithmetic;
// SYNC: a workgroup barrier before every group (every wavefront of the
// workgroup must call this).  Measured on the Riemann 1025^2-node step
// (float32 f + g, p = 2): the plane-by-plane loop of rows_stream on this
// order took 155 us (four strided 4-byte loads per row, each touching four
// times the cache lines), this one 99.7 against 108.8 us for the planar
// order on the same box.
template <typename T, int P1, int S, int DG, bool SYNC, int Q1>
__device__ __forceinline__ void rows_stream_grouped(
    const T *__restrict__ fin, const int32_t *__restrict__ xrel, const T *__restrict__ xw,
    const int32_t *__restrict__ xwin, const int32_t *__restrict__ ysrc, const T *__restrict__ yw,
    int TX, int ntx, int tx, int iy, int lane, const StepConsts &c, T *lrow,
    T (&fs)[S][Q1 * Q1]) {
  constexpr int NG = Q1 * S;  // groups, in the order (b, s)
  constexpr int K = Q1 - 1;   // moving x-components per group
  const int ixc = min(tx * TX + min(lane, TX - 1), c.nx - 1);
  const long long N = c.n;
  const unsigned plane_bytes = unsigned(N * (long long)sizeof(T));
  const unsigned row_bytes = unsigned(c.nx) * unsigned(sizeof(T));
  int xr0[Q1];
  T wx[Q1][P1];
#pragma unroll
  for (int a = 1; a < Q1; ++a) {
    xr0[a] = xrel[(a * P1) * c.nx + ixc];
#pragma unroll
    for (int m = 0; m < P1; ++m) wx[a][m] = xw[(a * P1 + m) * c.nx + ixc];
  }
  // the moving components share one window per segment (the host builds it
  // so), and this lane reads the K values of its window column with one
  // wide load; a = 0 is read at the node's own column
  const unsigned colq =
      unsigned(wrap_or_clamp(xwin[1 * ntx + tx] + lane, c.nx, c.perx)) * unsigned(sizeof(T) * K);
  const unsigned own_off = unsigned(ixc) * unsigned(sizeof(T));
  unsigned yoff[Q1][P1];
  T wy[Q1][P1];
  auto fetch_phase = [&](int b) {
    int z = 0;
    asm volatile("" : "+s"(z));  // keeps the scalar loads here
#pragma unroll
    for (int m = 0; m < P1; ++m) {
      yoff[b][m] = unsigned(ysrc[(b * P1 + m) * c.ny + iy + z]) * row_bytes;
      wy[b][m] = yw[(b * P1 + m) * c.ny + iy + z];
    }
  };
  T pre[DG + 1][P1][Q1];
  auto load = [&](int g, T (&d)[P1][Q1]) {
    const int b = g / S, s = g % S;
    if (b > 0 && s == 0) fetch_phase(b);
    const int rows = b == 0 ? 1 : P1;  // b = 0: identity y-factor, the target row alone
#pragma unroll
    for (int m = 0; m < P1; ++m) {
      if (m >= rows) {
#pragma unroll
        for (int a = 0; a < Q1; ++a) d[m][a] = T(0);
        continue;
      }
      const unsigned ro = b == 0 ? unsigned(iy) * row_bytes : yoff[b][m];
      T q[K];
      buffer_load_run<T, K>(make_rsrc(fin + pop_base(kGrouped, Q1, s, 1, b, N), plane_bytes * K),
                            colq, ro * K, q);
#pragma unroll
      for (int a = 1; a < Q1; ++a) d[m][a] = q[a - 1];
      d[m][0] = buffer_load<T>(make_rsrc(fin + pop_base(kGrouped, Q1, s, 0, b, N), plane_bytes),
                               own_off, ro);
    }
  };
#pragma unroll
  for (int g = 0; g < DG && g < NG; ++g) load(g, pre[g % (DG + 1)]);
#pragma unroll
  for (int g = 0; g < NG; ++g) {
    if (SYNC && g > 0) __builtin_amdgcn_s_barrier();
    // the group's loads issue at priority 3, the arithmetic at the kernel's 2
    // (float32 Riemann 1025^2 104.4 -> 102.6 us, shock-vortex within the
    // spread; float64 with the kernel's priority below: Riemann 208.5 ->
    // 206.6 us, shock-vortex 1101 -> 1077 us)
    __builtin_amdgcn_s_setprio(3);
    if (g + DG < NG) load(g + DG, pre[(g + DG) % (DG + 1)]);
    __builtin_amdgcn_s_setprio(2);
    const int b = g / S, s = g % S;
    const T(&v)[P1][Q1] = pre[g % (DG + 1)];
    T *rows = lrow + (g & 1) * K * 64;
#pragma unroll
    for (int a = 0; a < Q1; ++a) {
      T y = v[0][a];
      if (b != 0) {
        y = wy[b][0] * v[0][a];
#pragma unroll
        for (int m = 1; m < P1; ++m) y = fma(wy[b][m], v[m][a], y);
      }
      if (a == 0) {
        asm volatile("" : "+v"(y));
        fs[s][Q1 * b] = y;  // identity x-factor
      } else {
        rows[(a - 1) * 64 + lane] = y;
      }
    }
    wave_lds_sync();
#pragma unroll
    for (int a = 1; a < Q1; ++a) {
      const T *row = rows + (a - 1) * 64;
      T acc = wx[a][0] * row[xr0[a]];
#pragma unroll
      for (int m = 1; m < P1; ++m) acc = fma(wx[a][m], row[xr0[a] + m], acc);
      asm volatile("" : "+v"(acc));  // keep the plane's arithmetic in its place
      fs[s][a + Q1 * b] = acc;
    }
  }
}

// Groups of loads in flight ahead of the one being interpolated (grouped
// order), measured with the float32 wave priorities: float32 f + g at p = 3
// takes two (shock-vortex rows 538-543 -> 529 us), at p = 2 two were 0.8 %
// slower (Riemann 1025^2); float64 f + g lost 2 % with two.  Elsewhere one.
template <typename T, int P1, int S>
constexpr int rows_group_lookahead() { return sizeof(T) == 4 && S == 2 && P1 == 4 ? 2 : 1; }

// Planes between workgroup barriers (0: none), measured on 1025^2-node
// grids: for f + g, every 5 planes (with the deeper lookahead it allows)
// gives float32 +5-6 % at p = 1-3 and +16 % at p = 4, float64 +-1 %; every
// 3 or 10 planes is no better.  A single set shows no effect above the
// run-to-run spread.
template <int P1, int S>
constexpr int rows_sync_planes() { return S == 2 ? 5 : 0; }

// Minimum waves per SIMD the compiler is asked to fit: a single float32
// population set gets 6 (70-73 VGPRs instead of ~97; Taylor-Green p = 2:
// +14 %), 5 from p = 3 on (the row-by-row gather of the grouped order spills
// at 6 there), f + g keeps the default (the same request spills and costs
// 3-18 %).
template <typename T, int S, int P1>
constexpr int rows_min_waves() { return sizeof(T) == 4 && S == 1 ? (P1 >= 4 ? 5 : 6) : 1; }

template <typename T, int P, int MODEL, bool PR, int Q1 = 5>
__global__ __launch_bounds__((64 * rows_tile_rows<T, Sets<MODEL>::S, P + 1>()),
                             (rows_min_waves<T, Sets<MODEL>::S, P + 1>())) void k_step_rows(
    const T *__restrict__ fin, T *__restrict__ fout, const int32_t *__restrict__ xrel,
    const T *__restrict__ xw, const int32_t *__restrict__ xwin, const int32_t *__restrict__ ysrc,
    const T *__restrict__ yw, int TX, int ntx, int nty, int strip, StepConsts c,
    int *__restrict__ flag) {
  constexpr int S = Sets<MODEL>::S;
  constexpr int R = rows_tile_rows<T, Sets<MODEL>::S, P + 1>();
  __shared__ T rows_lds[R][2 * (Q1 - 1)][64];
  int tile = xcd_tile(blockIdx.x, ntx * nty);
  if (tile >= ntx * nty) return;
  if (c.reverse) tile = ntx * nty - 1 - tile;
  int tx, ty;
  strip_tile(tile, ntx, nty, strip, tx, ty);
  const int lane = threadIdx.x;
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.y);
  // rows past the grid stream the last row (every wavefront must reach the
  // barriers) and store nothing
  const int iy_t = ty * R + wv;
  const int iy = min(iy_t, c.ny - 1);
  T fs[S][Q1 * Q1];
  // a wavefront that streams issues before one that collides (wave priority
  // 2, back to 0 for the float64 collision), so the other wavefronts' loads
  // are not held behind its float64 arithmetic.  Same-box A/B: float32
  // Riemann 1025^2 105.05 -> 103.95 us, shock-vortex rows (Pr = 0.75) 550 ->
  // 532 us (float64 alone was within the spread; with the load-issue
  // priority of the gather it gains, see there)
  __builtin_amdgcn_s_setprio(2);
  rows_stream_grouped<T, P + 1, S, rows_group_lookahead<T, P + 1, S>(), S == 2, Q1>(
      fin, xrel, xw, xwin, ysrc, yw, TX, ntx, tx, iy, lane, c, &rows_lds[wv][0][0], fs);
  __builtin_amdgcn_s_setprio(0);
  const int ix = tx * TX + lane;
  if (ix < c.nx && lane < TX && iy_t < c.ny)
    collide_store<T, MODEL, PR, Q1, kGrouped>(fs, c, fout, (long long)iy * c.nx + ix, flag);
}

// Segments per strip of the strip-major tile order (strip_tile): rows of up
// to 24 segments keep the row-major order; wider ones (the 3073-node rows of
// the shock-vortex grid: 68 segments) go in strips of 16, so that a tile's
// vertical neighbours, which re-read its source rows, run 16 tiles later on
// the same XCD rather than a whole row later, when those rows have left its
// L2 cache.  Measured on the shock-vortex grid (float32, Pr = 0.75): HBM
// traffic 1.34x -> 1.06x the algorithmic bytes, step time -2 %.
inline int rows_strip(int ntx) { return ntx <= 24 ? ntx : 16; }

// PR: the Pr != 1 collision (thermal models only)
template <bool PR>
hipError_t launch_rows_family(int fp32, int model, const StepConsts &c, const DevTables &t,
                              const void *fin, void *fout, int *flag, hipStream_t s) {
  if (t.rows_tx < kRowsMinCols || t.rows_tx > 64 || t.rows_xrel == nullptr ||
      t.rows_xwin == nullptr || !(t.ident_y & t.ident_x & 1))
    return hipErrorInvalidValue;
  if (c.q1 == 3) {  // D2Q9: isothermal BGK
    if constexpr (PR) {
      return hipErrorInvalidValue;
    } else {
      return dispatch_q3(fp32, c.p, model, [&]<typename T, int P>() {
        constexpr int R = rows_tile_rows<T, 1>();
        const int ntx = (c.nx + t.rows_tx - 1) / t.rows_tx;
        const int nty = (c.ny + R - 1) / R;
        const int grid = ((ntx * nty + 7) / 8) * 8;
        k_step_rows<T, P, kIsothermal, false, 3><<<grid, dim3(64, R), 0, s>>>(
            static_cast<const T *>(fin), static_cast<T *>(fout), t.rows_xrel,
            static_cast<const T *>(t.xw), t.rows_xwin, t.ysrc, static_cast<const T *>(t.yw),
            t.rows_tx, ntx, nty, rows_strip(ntx), c, flag);
        return hipGetLastError();
      });
    }
  }
  if (c.q1 != 5) return hipErrorInvalidValue;
  return dispatch_step<PR>(fp32, c.p, model, [&]<typename T, int P, int MODEL>() {
    constexpr int R = rows_tile_rows<T, Sets<MODEL>::S, P + 1>();
    const int ntx = (c.nx + t.rows_tx - 1) / t.rows_tx;
    const int nty = (c.ny + R - 1) / R;
    const int grid = ((ntx * nty + 7) / 8) * 8;
    k_step_rows<T, P, MODEL, PR><<<grid, dim3(64, R), 0, s>>>(
        static_cast<const T *>(fin), static_cast<T *>(fout), t.rows_xrel,
        static_cast<const T *>(t.xw), t.rows_xwin, t.ysrc, static_cast<const T *>(t.yw),
        t.rows_tx, ntx, nty, rows_strip(ntx), c, flag);
    return hipGetLastError();
  });
}

}  // namespace sllbm
