// LDS-staged gather shared by the tiled stream + collide kernel and the
// tiled adjoint step.
//
// A workgroup owns a tile of 64 x-nodes (one per lane) by TY rows (one
// wavefront per row).  For the departure points of velocity i = a + 5b, the
// tile needs a window of source rows that depends only on b and a window of
// source columns that depends only on a (both precomputed per tile: the
// departure geometry is static).  Per phase (one b and a group of G
// x-components, for every population set) the workgroup
//   1. stages the raw source windows (W rows by WX = 64 + HALO columns) into
//      LDS with row-contiguous buffer loads: one load per lane per window
//      row for the 64 main columns, and for the HALO extra columns either a
//      second load per row (float32, and any 64-column halo) or, for a
//      narrow halo of float64 values, one load carrying the halo columns of
//      64 / HALO rows;
//   2. evaluates each node's cell-local tensor Lagrange interpolant (eq. (17))
//      from LDS: an x-pass over p+1 columns on each of the node's p+1 rows,
//      then the y-combination, keeping all 25 (or 50) streamed values of the
//      node in registers.  From 6 taps per axis on, the x-pass runs once per
//      staged row and column (shared by the tile's rows) into a second LDS
//      buffer before the y-combination.
// Loads for the next phase are issued before this phase's interpolation and
// written to the other LDS buffer after it, so they stay in flight meanwhile.
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

constexpr size_t kTiledLdsBudget = 163840;  // gfx950: 160 KiB of LDS per workgroup
constexpr int kTileRowsTY = 4;

// Separable evaluation from this many taps per axis on (the transposed
// tables of the adjoint); below it the direct 2-D form measured faster.
constexpr int kSeparableTaps = 6;

// Index j wrapped into a periodic axis of n nodes or clamped into [0, n-1]
// (staged nodes past the window are never weighted).
__device__ __forceinline__ int wrap_or_clamp(int j, int n, int periodic) {
  int w = j % n;
  w += w < 0 ? n : 0;
  const int cl = j < 0 ? 0 : (j < n - 1 ? j : n - 1);
  return periodic ? w : cl;
}

// The same for j within one period of [0, n) (the packed halo loads, which
// the host enables only on axes much longer than a window).
__device__ __forceinline__ int wrap_or_clamp_near(int j, int n, int periodic) {
  const int w = j < 0 ? j + n : (j >= n ? j - n : j);
  const int cl = j < 0 ? 0 : (j < n - 1 ? j : n - 1);
  return periodic ? w : cl;
}


// Interpolation from the staged windows: the direct 2-D form; the separable
// form (x-pass per staged row into LDS, then y); or the separable form with
// the x-pass on the matrix cores, in float32 or (the bfloat16 experiment)
// with bfloat16 weights and staged values and float32 accumulation.
enum InterpMode { kInterp2D = 0, kInterpSep = 1, kInterpMfma = 2, kInterpMfmaBf16 = 3 };

constexpr bool is_mfma_mode(int im) { return im == kInterpMfma || im == kInterpMfmaBf16; }

// Staged columns one bfloat16 x-pass product spans (v_mfma_f32_16x16x32_bf16:
// K = 32 >= the 16 + 2p columns of a 16-column block).
constexpr int kMfmaBf16Cols = 32;

// k-steps of 4 of the matrix-core x-pass: 16 target columns need at most
// 16 + 2 (P1 - 1) staged columns (departures within one node spacing of the
// cell; the host checks every block).
template <int P1>
constexpr int mfma_ksteps() { return (16 + 2 * (P1 - 1) + 3) / 4; }

// Row pitch of the staged windows: 64 + halo columns, plus (for the
// matrix-core x-pass) zero columns that the last k-steps may read.
template <int P1, int HALO, int IM>
constexpr int tiled_pitch() {
  return 64 + HALO + (IM == kInterpMfma ? 4 * mfma_ksteps<P1>()
                                        : (IM == kInterpMfmaBf16 ? kMfmaBf16Cols : 0));
}

// P1 = taps per axis: p+1 for the forward step, the transposed table width
// for the adjoint.  R = staged rows per wavefront (W <= R * TY).  The
// separable forms cost (R + 1) P1 FMAs per value instead of P1 (P1 + 1),
// paid for with a second barrier per phase.
template <typename T, int P1, int S, int TY, int HALO, int G, int R, int IM>
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
  static_assert(HALO == 4 || HALO == 8 || HALO == 64, "halo of 4, 8 or 64 columns");
  static_assert(!is_mfma_mode(IM) || sizeof(T) == 4, "matrix-core x-pass on float32 populations");
  constexpr bool SEP = IM != kInterp2D;
  constexpr int WX = tiled_pitch<P1, HALO, IM>();        // staged row pitch
  constexpr int NQ = S * G;                              // planes staged per phase
  // packed halo loads measured faster for float64 values, slower for float32
  // (their address arithmetic outweighs the loads they save)
  constexpr bool PACKED = HALO < 64 && sizeof(T) == 8;
  constexpr int HROWS = PACKED ? 64 / HALO : 1;          // rows per packed halo load
  constexpr int HPARTS = PACKED ? (R * TY + HROWS - 1) / HROWS : 0;  // loads per plane
  constexpr int NH = PACKED ? (NQ * HPARTS + TY - 1) / TY : 0;       // per wavefront
  constexpr int MAINH = PACKED ? 1 : 2;                  // loads per staged row
  constexpr int NPH = 5 * (5 / G);                       // phases: (b, group of G a's)
  const int PLANE = W * WX;                              // exact window rows per plane
  const int BUF = NQ * PLANE;                            // one of two raw buffers
  T *const dummy = lds + 2 * BUF;                        // 64 slots for unused lanes
  const long long N = c.n;
  const unsigned plane_bytes = unsigned(N * (long long)sizeof(T));
  const unsigned row_bytes = unsigned(c.nx) * unsigned(sizeof(T));
  // this lane's x-stencils for the 5 x-components: P1 consecutive
  // window-relative columns starting at xr0[a], with weights wx[a][m];
  // col_off = byte offset of the staged main column x0 + lane (and, for a
  // 64-column halo, of x0 + 64 + lane)
  int xr0[5];
  T wx[5][P1];
  unsigned col_off[5][MAINH];
#pragma unroll
  for (int a = 0; a < 5; ++a) {
    xr0[a] = xrel[(a * P1) * c.nx + ixc];
#pragma unroll
    for (int m = 0; m < P1; ++m) wx[a][m] = xw[(a * P1 + m) * c.nx + ixc];
    const int x0 = xwin[a * ntx + tx];
#pragma unroll
    for (int h = 0; h < MAINH; ++h) {
      // unpacked narrow halo: lanes 8.. repeat the first HALO columns
      const int off = h == 0 || HALO == 64 ? lane : lane % HALO;
      col_off[a][h] =
          unsigned(wrap_or_clamp(x0 + 64 * h + off, c.nx, c.perx)) * unsigned(sizeof(T));
    }
  }
  // packed halo: this lane's row within a halo load and its halo column
  const int hrow = lane / HALO, hcol = lane % HALO;
  auto row_off = [&](int r) { return unsigned(wrap_or_clamp(r, c.ny, c.pery)) * row_bytes; };
  // prefetch registers: main rows (R x G x S) and this wavefront's share of
  // the packed halo loads
  T pre[R][G][S][MAINH];
  T preh[NH > 0 ? NH : 1];
  auto load = [&](int ph) {
    const int b = ph / (5 / G), a0 = (ph % (5 / G)) * G;
    const int w0 = ywin[b * nty + ty];
#pragma unroll
    for (int rr = 0; rr < R; ++rr) {
      if (wv + rr * TY >= W) break;  // wave-uniform: rows past the window
      const unsigned ro = row_off(w0 + wv + rr * TY);
#pragma unroll
      for (int g = 0; g < G; ++g)
#pragma unroll
        for (int s = 0; s < S; ++s) {
          const auto rs = make_rsrc(fin + (long long)(s * 25 + a0 + g + 5 * b) * N, plane_bytes);
#pragma unroll
          for (int h = 0; h < MAINH; ++h)
            pre[rr][g][s][h] = buffer_load<T>(rs, col_off[a0 + g][h], ro);
        }
    }
    if constexpr (PACKED) {
#pragma unroll
      for (int t = 0; t < NH; ++t) {
        const int j = wv + TY * t;  // halo job: plane q, part k (wave-uniform)
        if (j >= NQ * HPARTS) break;
        const int q = j / HPARTS, k = j % HPARTS;
        const int g = q % G, s = q / G;
        const int x0 = xwin[(a0 + g) * ntx + tx];
        const int r = wrap_or_clamp_near(w0 + k * HROWS + hrow, c.ny, c.pery);
        const unsigned off =
            unsigned(wrap_or_clamp_near(x0 + 64 + hcol, c.nx, c.perx)) * unsigned(sizeof(T)) +
            unsigned(r) * row_bytes;
        const auto rs = make_rsrc(fin + (long long)(s * 25 + a0 + g + 5 * b) * N, plane_bytes);
        preh[t] = buffer_load<T>(rs, off, 0);
      }
    }
  };
  auto store = [&](T *buf) {
#pragma unroll
    for (int rr = 0; rr < R; ++rr) {
      if (wv + rr * TY >= W) break;
#pragma unroll
      for (int g = 0; g < G; ++g)
#pragma unroll
        for (int s = 0; s < S; ++s) {
          T *dst = buf + (s * G + g) * PLANE + (wv + rr * TY) * WX;
          dst[lane] = pre[rr][g][s][0];
          if constexpr (MAINH == 2) {
            T *slot = HALO == 64 || lane < HALO ? dst + 64 + lane : dummy + lane;
            *slot = pre[rr][g][s][MAINH - 1];
          }
        }
    }
    if constexpr (PACKED) {
#pragma unroll
      for (int t = 0; t < NH; ++t) {
        const int j = wv + TY * t;
        if (j >= NQ * HPARTS) break;
        const int q = j / HPARTS, k = j % HPARTS;
        const int row = k * HROWS + hrow;
        T *slot = row < W ? buf + q * PLANE + row * WX + 64 + hcol : dummy + lane;
        *slot = preh[t];
      }
    }
  };
  // matrix-core x-pass: this lane's A-operand entries (banded Lagrange
  // weights of target column 16 wv + lane % 16 against staged column
  // base_a + 4 k + lane / 16, base_a = stencil start of the block's first
  // column), and zeros in the pad columns of both raw buffers
  typedef __bf16 bf8 __attribute__((ext_vector_type(8)));
  constexpr int KS = IM == kInterpMfma ? mfma_ksteps<P1>() : 1;
  float amat[IM == kInterpMfma ? 5 : 1][KS];
  bf8 amat16[IM == kInterpMfmaBf16 ? 5 : 1];  // bfloat16: A[n][8 (l / 16) + e], e = 0..7
  int xbase[5];
  if constexpr (IM == kInterpMfmaBf16) {
    const int n = 16 * wv + (lane & 15), kq = lane >> 4;
#pragma unroll
    for (int a = 0; a < 5; ++a) {
      xbase[a] = __shfl(xr0[a], 16 * wv);
      const int d0 = xbase[a] + 8 * kq - __shfl(xr0[a], n);
      float wn[P1];
#pragma unroll
      for (int m = 0; m < P1; ++m) wn[m] = __shfl(float(wx[a][m]), n);
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        const int d = d0 + e;
        float v = 0.0f;
#pragma unroll
        for (int m = 0; m < P1; ++m) v = d == m ? wn[m] : v;
        amat16[a][e] = __bf16(v);  // round to nearest even
      }
    }
    constexpr int PADC = WX - 64 - HALO;  // pad columns of every staged row
    for (int e = wv * 64 + lane; e < 2 * NQ * W * PADC; e += TY * 64)
      lds[(e / PADC) * WX + 64 + HALO + e % PADC] = T(0);  // rows of both buffers in turn
  }
  if constexpr (IM == kInterpMfma) {
    const int n = 16 * wv + (lane & 15), kq = lane >> 4;
#pragma unroll
    for (int a = 0; a < 5; ++a) {
      xbase[a] = __shfl(xr0[a], 16 * wv);
      const int d0 = xbase[a] + kq - __shfl(xr0[a], n);
      float wn[P1];
#pragma unroll
      for (int m = 0; m < P1; ++m) wn[m] = __shfl(float(wx[a][m]), n);
#pragma unroll
      for (int k = 0; k < KS; ++k) {
        const int d = d0 + 4 * k;
        float v = 0.0f;
#pragma unroll
        for (int m = 0; m < P1; ++m) v = d == m ? wn[m] : v;
        amat[a][k] = v;
      }
    }
    constexpr int PADC = WX - 64 - HALO;  // pad columns of every staged row
    for (int e = wv * 64 + lane; e < 2 * NQ * W * PADC; e += TY * 64)
      lds[(e / PADC) * WX + 64 + HALO + e % PADC] = T(0);  // rows of both buffers in turn
  }
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
    if constexpr (SEP) {
      T *const xb = lds + 2 * BUF + 64;  // [S][G][W][64] x-interpolated rows
      if constexpr (IM == kInterpSep) {
#pragma unroll
        for (int rr = 0; rr < R; ++rr) {
          const int row = wv + rr * TY;
          if (row >= W) break;  // wave-uniform
#pragma unroll
          for (int g = 0; g < G; ++g) {
            const int a = a0 + g;
#pragma unroll
            for (int s = 0; s < S; ++s) {
              const T *src = cur + (s * G + g) * PLANE + row * WX + xr0[a];
              T xv = T(0);
#pragma unroll
              for (int m = 0; m < P1; ++m) xv = fma(wx[a][m], src[m], xv);
              xb[((s * G + g) * W + row) * 64 + lane] = xv;
            }
          }
        }
      } else if constexpr (IM == kInterpMfmaBf16) {
        // X[16 columns of block wv][(set, row) pairs] = A_a (16 x 32) x
        // staged columns (32 x pairs) in one bfloat16 product: lane l
        // supplies A[l % 16][8 (l / 16) + e] and B[8 (l / 16) + e][l % 16]
        // (e = 0..7) and receives X[4 (l / 16) + t][l % 16]
        typedef float f4 __attribute__((ext_vector_type(4)));
        const int j = lane & 15, kq = lane >> 4;
        const bool jok = j < S * W;
        const int jc = jok ? j : 0, js = jc / W, jr = jc % W;
#pragma unroll
        for (int g = 0; g < G; ++g) {
          const int a = a0 + g;
          const float *src = cur + (js * G + g) * PLANE + jr * WX + xbase[a] + 8 * kq;
          bf8 bv;
#pragma unroll
          for (int e = 0; e < 8; ++e) bv[e] = __bf16(jok ? src[e] : 0.0f);
          const f4 zero = {0.0f, 0.0f, 0.0f, 0.0f};
          const f4 acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(amat16[a], bv, zero, 0, 0, 0);
          if (jok)
            *reinterpret_cast<f4 *>(xb + ((js * G + g) * W + jr) * 64 + 16 * wv + 4 * kq) = acc;
        }
      } else {
        // X[16 columns of block wv][(set, row) pairs] = A_a (16 x 4 KS) x
        // staged columns (4 KS x pairs): lane l supplies A[l % 16][l / 16]
        // and B[l / 16][l % 16] and receives X[4 (l / 16) + t][l % 16]
        typedef float f4 __attribute__((ext_vector_type(4)));
        const int j = lane & 15, kq = lane >> 4;
        const bool jok = j < S * W;
        const int jc = jok ? j : 0, js = jc / W, jr = jc % W;
#pragma unroll
        for (int g = 0; g < G; ++g) {
          const int a = a0 + g;
          const float *src = cur + (js * G + g) * PLANE + jr * WX + xbase[a] + kq;
          f4 acc = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
          for (int k = 0; k < KS; ++k)
            acc = __builtin_amdgcn_mfma_f32_16x16x4f32(amat[a][k], jok ? src[4 * k] : 0.0f, acc,
                                                       0, 0, 0);
          if (jok)
            *reinterpret_cast<f4 *>(xb + ((js * G + g) * W + jr) * 64 + 16 * wv + 4 * kq) = acc;
        }
      }
      lds_barrier();
      T acc[G][S];
#pragma unroll
      for (int g = 0; g < G; ++g) {
#pragma unroll
        for (int s = 0; s < S; ++s) {
          const T *col = xb + ((s * G + g) * W + yr0) * 64 + lane;
          T v = T(0);
#pragma unroll
          for (int n = 0; n < P1; ++n) v = fma(wy[n], col[n * 64], v);
          acc[g][s] = v;
        }
      }
#pragma unroll
      for (int g = 0; g < G; ++g)
#pragma unroll
        for (int s = 0; s < S; ++s) {
          asm volatile("" : "+v"(acc[g][s]));
          fs[s][a0 + g + 5 * b] = acc[g][s];
        }
    } else {
      T acc[G][S];
#pragma unroll
      for (int g = 0; g < G; ++g) {
        const int a = a0 + g;
        const T *corner = cur + (yr0 * WX + xr0[a]);
#pragma unroll
        for (int s = 0; s < S; ++s) {
          const T *src = corner + (s * G + g) * PLANE;
          T v = T(0);
#pragma unroll
          for (int n = 0; n < P1; ++n) {
            T rv = T(0);
#pragma unroll
            for (int m = 0; m < P1; ++m) rv = fma(wx[a][m], src[n * WX + m], rv);
            v = fma(wy[n], rv, v);
          }
          acc[g][s] = v;
        }
      }
      // keep the FMAs in this phase (otherwise the compiler sinks them all to
      // the collision and keeps every LDS value of every phase alive), but
      // pin the phase as a whole so that its LDS reads overlap
#pragma unroll
      for (int g = 0; g < G; ++g)
#pragma unroll
        for (int s = 0; s < S; ++s) {
          asm volatile("" : "+v"(acc[g][s]));
          fs[s][a0 + g + 5 * b] = acc[g][s];
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

// Tile (tx, ty) of position t of the strip-major order: the columns of tiles
// are grouped in strips of `strip` columns (the last one may be narrower),
// each strip is walked row by row, and the strips follow each other.  Tiles
// that read the same source rows (vertical neighbours) then run `strip`
// positions apart instead of ntx; strip >= ntx is the row-major order.
__device__ __forceinline__ void strip_tile(int t, int ntx, int nty, int strip, int &tx, int &ty) {
  const int full = ntx / strip;               // strips of full width
  const int per_strip = strip * nty;
  const int s = t / per_strip;
  if (s < full) {
    const int r = t - s * per_strip;
    ty = r / strip;
    tx = s * strip + r % strip;
  } else {                                    // the narrower last strip
    const int w = ntx - full * strip;
    const int r = t - full * per_strip;
    ty = r / w;
    tx = full * strip + r % w;
  }
}

// LDS bytes of a tiled launch: two raw window buffers (S G planes of W rows
// of `pitch` columns), 64 spare slots, and for the separable forms the
// x-pass buffer.
constexpr size_t tiled_lds_bytes(size_t tsize, int S, int G, int W, int pitch, bool sep) {
  const size_t planes = size_t(S) * G;
  return (2 * planes * W * pitch + 64 + (sep ? planes * W * 64 : 0)) * tsize;
}

// Narrowest halo (4, 8 or 64 extra columns) that covers a window of
// win_cols columns; 0 when none does.  Narrow halos need axes of at least
// 256 columns and 32 rows (their loads wrap indices by one period at most).
inline int tiled_halo(int win_cols, int nx, int ny) {
  if (win_cols > 128) return 0;
  if (nx < 256 || ny < 32 || win_cols > 72) return 64;
  return win_cols <= 68 ? 4 : 8;
}

}  // namespace sllbm
