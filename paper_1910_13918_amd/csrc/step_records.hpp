// Stream + collide: general gather through per-(node, velocity) departure
// records (HIP, gfx950).
#pragma once

#include <hip/hip_runtime.h>

#include "launch.hpp"
#include "step_common.hpp"
#include "tiled_common.hpp"

namespace sllbm {

// ---------------------------------------------------------------------------
// stream + collide, general gather through per-(node, velocity) records
// (departure cell and reference coordinates; weights evaluated here)
// ---------------------------------------------------------------------------
// The p+1 stencil columns of a departure cell are consecutive nodes except
// when the cell is the last one before a periodic seam (its right vertex is
// node 0): rows are then read one value at a time, in a wave-uniform branch.
template <typename T, int P1, bool SEAM>
__device__ __forceinline__ T records_interp(__amdgpu_buffer_rsrc_t rs, const unsigned (&xo)[P1],
                                            const unsigned (&yo)[P1], const T (&wx)[P1],
                                            const T (&wy)[P1]) {
  T acc = T(0);
#pragma unroll
  for (int n = 0; n < P1; ++n) {
    T v[P1];
    if constexpr (SEAM) {
#pragma unroll
      for (int m = 0; m < P1; ++m) v[m] = buffer_load<T>(rs, yo[n] + xo[m], 0);
    } else {
      buffer_load_run<T, P1>(rs, yo[n] + xo[0], 0, v);
    }
    T row = T(0);
#pragma unroll
    for (int m = 0; m < P1; ++m) row = fma(wx[m], v[m], row);
    acc = fma(wy[n], row, acc);
  }
  return acc;
}

// Three 32-bit words (one float32 departure record).
typedef unsigned rec_words3 __attribute__((ext_vector_type(3)));

// Departure record of velocity i at node v (the layout of DevTables::rec):
// float32 one 12-byte {cell, r, s} load, float64 the cell plane and one
// 16-byte {r, s} load.  Each velocity's records get their own buffer
// resource, so offsets stay 32-bit on the largest grids.
template <typename T>
__device__ __forceinline__ void load_record(const int32_t *__restrict__ cell,
                                            const void *__restrict__ rec, int i, long long v,
                                            long long N, int &cellv, T &r, T &s) {
  if constexpr (sizeof(T) == 4) {
    const auto rs = make_rsrc(static_cast<const uint32_t *>(rec) + (long long)i * N * 3,
                              unsigned(N) * 12u);
    const rec_words3 q = __builtin_amdgcn_raw_buffer_load_b96(rs, unsigned(v) * 12u, 0, 0);
    // the words go through scalars: a bit cast of a vector element itself
    // was compiled as a read of the vector's first element
    const unsigned w0 = q[0], w1 = q[1], w2 = q[2];
    cellv = int(w0);
    r = __builtin_bit_cast(T, w1);
    s = __builtin_bit_cast(T, w2);
  } else {
    using u4 = __attribute__((ext_vector_type(4))) unsigned;
    using u2 = __attribute__((ext_vector_type(2))) unsigned;
    const auto rc = make_rsrc(cell + (long long)i * N, unsigned(N) * 4u);
    cellv = int(__builtin_amdgcn_raw_buffer_load_b32(rc, unsigned(v) * 4u, 0, 0));
    const auto rs = make_rsrc(static_cast<const double *>(rec) + (long long)i * N * 2,
                              unsigned(N) * 16u);
    const u4 q = __builtin_amdgcn_raw_buffer_load_b128(rs, unsigned(v) * 16u, 0, 0);
    r = __builtin_bit_cast(T, u2{q.x, q.y});
    s = __builtin_bit_cast(T, u2{q.z, q.w});
  }
}

// Whether the gather of the next velocity is issued before this velocity's
// interpolation: float32 f + g, where it measured +13 % on the shock-vortex
// grid (p = 3) and +3 % at p = 2; a single set and float64 lose 1-3 % to the
// doubled registers.
template <typename T, int S>
constexpr bool records_gather_ahead() { return sizeof(T) == 4 && S == 2; }

// Nodes per workgroup: tiles of 64 x 4 nodes (one wavefront per row), so
// that the stencils a workgroup reads from neighbouring rows overlap.
constexpr int kRecTileRows = 4;

template <typename T, int P, int MODEL, bool PR, int Q1 = 5>
__global__ __launch_bounds__(64 * kRecTileRows) void k_step_records(
    const T *__restrict__ fin, T *__restrict__ fout, const int32_t *__restrict__ cell,
    const void *__restrict__ rec, int ntx, int nty, int strip, StepConsts c,
    int *__restrict__ flag) {
  constexpr int S = Sets<MODEL>::S;
  constexpr int P1 = P + 1;
  constexpr int Q = Q1 * Q1;
  // XCD-aware, strip-major tile order; every other step may visit the tiles
  // backwards (see StepConsts::reverse)
  int tile = xcd_tile(blockIdx.x, ntx * nty);
  if (tile >= ntx * nty) return;
  if (c.reverse) tile = ntx * nty - 1 - tile;
  int tx, ty;
  strip_tile(tile, ntx, nty, strip, tx, ty);
  const int ix = tx * 64 + (threadIdx.x & 63);
  const int iy = ty * kRecTileRows + (threadIdx.x >> 6);
  if (ix >= c.nx || iy >= c.ny) return;
  const long long v = (long long)iy * c.nx + ix;
  const long long N = c.n;
  const unsigned plane_bytes = unsigned(N * (long long)sizeof(T));
  T rn[P1], den[P1];
#pragma unroll
  for (int m = 0; m < P1; ++m) {
    rn[m] = T(c.rn[m]);
    den[m] = T(c.lden[m]);
  }
  T fs[S][Q];
  // float32: wave priority 2 while gathering, 0 for the float64 collision
  // (as the row-segment step; shock-vortex records 1047 -> 1035 us, curved
  // cells 199 -> 196 us)
  if constexpr (sizeof(T) == 4) __builtin_amdgcn_s_setprio(2);
  if constexpr (records_gather_ahead<T, S>()) {
    // f + g in float32: the next velocity's stencil values are loaded
    // before this one is interpolated (two values in flight per lane and
    // tap), its record two velocities ahead
    constexpr int RD = 2;
    int recq[RD + 1];
    T rq[RD + 1], sq[RD + 1];
    auto load_rec = [&](int i) {
      load_record<T>(cell, rec, i, v, N, recq[i % (RD + 1)], rq[i % (RD + 1)], sq[i % (RD + 1)]);
    };
    T vals[2][S][P1][P1];
    T wxq[2][P1], wyq[2][P1];
    auto issue = [&](int i) {
      const int b = i & 1;
      const int rec = recq[i % (RD + 1)];
      // unsigned shift: cell rows up to 65535 (an arithmetic shift would make
      // rows >= 32768 negative)
      const int cx = rec & 0xffff, cy = int(unsigned(rec) >> 16);
      lagrange_eval<T, P1>(rq[i % (RD + 1)], rn, den, wxq[b]);
      lagrange_eval<T, P1>(sq[i % (RD + 1)], rn, den, wyq[b]);
      unsigned xo[P1], yo[P1];
      bool seam = false;
  #pragma unroll
      for (int m = 0; m < P1; ++m) {
        int jx = cx * P + m;
        seam |= jx >= c.nx;
        if (jx >= c.nx) jx -= c.nx;  // periodic seam: last vertex is node 0
        xo[m] = unsigned(jx) * unsigned(sizeof(T));
        int jy = cy * P + m;
        if (jy >= c.ny) jy -= c.ny;
        yo[m] = unsigned(jy) * unsigned(c.nx) * unsigned(sizeof(T));
      }
      const bool any_seam = __builtin_amdgcn_ballot_w64(seam) != 0;
  #pragma unroll
      for (int s = 0; s < S; ++s) {
        const auto rs = make_rsrc(fin + (long long)(s * Q + i) * N, plane_bytes);
  #pragma unroll
        for (int n = 0; n < P1; ++n) {
          if (any_seam) {
  #pragma unroll
            for (int m = 0; m < P1; ++m) vals[b][s][n][m] = buffer_load<T>(rs, yo[n] + xo[m], 0);
          } else {
            buffer_load_run<T, P1>(rs, yo[n] + xo[0], 0, vals[b][s][n]);
          }
        }
      }
    };
  #pragma unroll
    for (int i = 0; i < RD; ++i) load_rec(i);
    issue(0);
  #pragma unroll
    for (int i = 0; i < Q; ++i) {
      if (i + RD < Q) load_rec(i + RD);
      if (i + 1 < Q) issue(i + 1);
      const int b = i & 1;
  #pragma unroll
      for (int s = 0; s < S; ++s) {
        T acc = T(0);
  #pragma unroll
        for (int n = 0; n < P1; ++n) {
          T row = T(0);
  #pragma unroll
          for (int m = 0; m < P1; ++m) row = fma(wxq[b][m], vals[b][s][n][m], row);
          acc = fma(wyq[b][n], row, acc);
        }
        asm volatile("" : "+v"(acc));
        fs[s][i] = acc;
      }
    }
  } else {
    // the next velocity's record is loaded before this one's gather (each
    // velocity is a separate scheduling region; loading ahead overlaps the
    // record's latency with the gather: shock-vortex records +18 %, curved
    // cells p = 2 +9 %, p = 4 +5 %; two or four ahead are no better)
    constexpr int RD = 1;
    int recq[RD + 1];
    T rq[RD + 1], sq[RD + 1];
    auto load_rec = [&](int i) {
      load_record<T>(cell, rec, i, v, N, recq[i % (RD + 1)], rq[i % (RD + 1)], sq[i % (RD + 1)]);
    };
  #pragma unroll
    for (int i = 0; i < RD; ++i) load_rec(i);
  #pragma unroll
    for (int i = 0; i < Q; ++i) {
      if (i + RD < Q) load_rec(i + RD);
      const int rec = recq[i % (RD + 1)];
      // unsigned shift: cell rows up to 65535 (an arithmetic shift would make
      // rows >= 32768 negative)
      const int cx = rec & 0xffff, cy = int(unsigned(rec) >> 16);
      T wx[P1], wy[P1];
      lagrange_eval<T, P1>(rq[i % (RD + 1)], rn, den, wx);
      lagrange_eval<T, P1>(sq[i % (RD + 1)], rn, den, wy);
      unsigned xo[P1], yo[P1];
      bool seam = false;
  #pragma unroll
      for (int m = 0; m < P1; ++m) {
        int jx = cx * P + m;
        seam |= jx >= c.nx;
        if (jx >= c.nx) jx -= c.nx;  // periodic seam: last vertex is node 0
        xo[m] = unsigned(jx) * unsigned(sizeof(T));
        int jy = cy * P + m;
        if (jy >= c.ny) jy -= c.ny;
        yo[m] = unsigned(jy) * unsigned(c.nx) * unsigned(sizeof(T));
      }
      const bool any_seam = __builtin_amdgcn_ballot_w64(seam) != 0;
  #pragma unroll
      for (int s = 0; s < S; ++s) {
        const auto rs = make_rsrc(fin + (long long)(s * Q + i) * N, plane_bytes);
        T acc = any_seam ? records_interp<T, P1, true>(rs, xo, yo, wx, wy)
                         : records_interp<T, P1, false>(rs, xo, yo, wx, wy);
        // keep the interpolation next to its loads
        asm volatile("" : "+v"(acc));
        fs[s][i] = acc;
      }
    }
  }
  if constexpr (sizeof(T) == 4) __builtin_amdgcn_s_setprio(0);
  collide_store<T, MODEL, PR, Q1>(fs, c, fout, v, flag);
}

// PR: the Pr != 1 collision (thermal models only)
template <bool PR>
hipError_t launch_records_family(int fp32, int model, const StepConsts &c, const DevTables &t,
                                 const void *fin, void *fout, int *flag, hipStream_t s) {
  const int ntx = (c.nx + 63) / 64, nty = (c.ny + kRecTileRows - 1) / kRecTileRows;
  const int grid = ((ntx * nty + 7) / 8) * 8;
  // strip-major order on wide grids (strip_tile); with the 64 x 4 tiles it
  // took the shock-vortex records gather from 1.45x to 1.10x the algorithmic
  // HBM bytes (the one-dimensional order of 256-node blocks put vertical
  // neighbours on other XCDs), step time -3 %
  const int strip = ntx <= 24 ? ntx : 16;
  if (c.q1 == 3) {  // D2Q9: isothermal BGK
    if constexpr (PR) {
      return hipErrorInvalidValue;
    } else {
      return dispatch_q3(fp32, c.p, model, [&]<typename T, int P>() {
        k_step_records<T, P, kIsothermal, false, 3><<<grid, 64 * kRecTileRows, 0, s>>>(
            static_cast<const T *>(fin), static_cast<T *>(fout), t.rec_cell, t.rec, ntx, nty,
            strip, c, flag);
        return hipGetLastError();
      });
    }
  }
  if (c.q1 != 5) return hipErrorInvalidValue;
  return dispatch_step<PR>(fp32, c.p, model, [&]<typename T, int P, int MODEL>() {
    k_step_records<T, P, MODEL, PR><<<grid, 64 * kRecTileRows, 0, s>>>(
        static_cast<const T *>(fin), static_cast<T *>(fout), t.rec_cell, t.rec, ntx, nty, strip,
        c, flag);
    return hipGetLastError();
  });
}

}  // namespace sllbm
