// Stream + collide: direct gather through per-axis departure tables (HIP, gfx950).
#pragma once

#include <hip/hip_runtime.h>

#include "launch.hpp"
#include "step_common.hpp"

namespace sllbm {

// ---------------------------------------------------------------------------
// stream + collide, direct gather through per-axis departure tables
//
// One thread per node (a wavefront is 64 consecutive x-nodes of one row).
// The x-stencil of a departure point is p+1 consecutive nodes of a row, so
// each of the p+1 source rows is read with one wide buffer load per lane
// (dwordx2..x4 runs); only lanes whose stencil wraps around a periodic seam
// re-read their values one by one.
// ---------------------------------------------------------------------------
template <typename T, int P1, int S, bool SEAM, int Q1>
__device__ __forceinline__ void direct_stream(const T *__restrict__ fin,
                                              const int32_t *__restrict__ xsrc,
                                              const T *__restrict__ ysrc_w,
                                              const int32_t *__restrict__ ysrc,
                                              const unsigned (&x0)[Q1], const T (&wx)[Q1][P1],
                                              int ix, int iy, const StepConsts &c,
                                              T (&fs)[S][Q1 * Q1]) {
  constexpr int Q = Q1 * Q1;
  const long long N = c.n;
  const unsigned plane_bytes = unsigned(N * (long long)sizeof(T));
  const unsigned row_bytes = unsigned(c.nx) * unsigned(sizeof(T));
#pragma unroll
  for (int b = 0; b < Q1; ++b) {
    unsigned yo[P1];
    T wy[P1];
#pragma unroll
    for (int n = 0; n < P1; ++n) {
      yo[n] = unsigned(ysrc[(b * P1 + n) * c.ny + iy]) * row_bytes;
      wy[n] = ysrc_w[(b * P1 + n) * c.ny + iy];
    }
#pragma unroll
    for (int a = 0; a < Q1; ++a) {
      const int i = a + Q1 * b;
      unsigned xs[P1];
      if constexpr (SEAM) {
#pragma unroll
        for (int m = 0; m < P1; ++m)
          xs[m] = unsigned(xsrc[(a * P1 + m) * c.nx + ix]) * unsigned(sizeof(T));
      }
#pragma unroll
      for (int s = 0; s < S; ++s) {
        const auto rs = make_rsrc(fin + (long long)(s * Q + i) * N, plane_bytes);
        T acc = T(0);
#pragma unroll
        for (int n = 0; n < P1; ++n) {
          T v[P1];
          if constexpr (SEAM) {
#pragma unroll
            for (int m = 0; m < P1; ++m) v[m] = buffer_load<T>(rs, xs[m], yo[n]);
          } else {
            buffer_load_run<T, P1>(rs, x0[a], yo[n], v);
          }
          T row = T(0);
#pragma unroll
          for (int m = 0; m < P1; ++m) row = fma(wx[a][m], v[m], row);
          acc = fma(wy[n], row, acc);
        }
        // keep the interpolation next to its loads (otherwise the compiler may
        // sink every FMA to the collision and keep all loaded values alive)
        asm volatile("" : "+v"(acc));
        fs[s][i] = acc;
      }
    }
  }
}

template <typename T, int P, int MODEL, bool PR, int Q1 = 5>
__global__ __launch_bounds__(256) void k_step_direct(const T *__restrict__ fin,
                                                     T *__restrict__ fout,
                                                     const int32_t *__restrict__ xsrc,
                                                     const T *__restrict__ xw,
                                                     const int32_t *__restrict__ ysrc,
                                                     const T *__restrict__ yw, StepConsts c,
                                                     int *__restrict__ flag) {
  constexpr int S = Sets<MODEL>::S;
  constexpr int P1 = P + 1;
  const int ix = blockIdx.x * 64 + threadIdx.x;
  const int iy = blockIdx.y * 4 + threadIdx.y;
  if (ix >= c.nx || iy >= c.ny) return;
  unsigned x0[Q1];  // byte offset of the first stencil column
  bool seam = false;
  T wx[Q1][P1];
#pragma unroll
  for (int a = 0; a < Q1; ++a) {
    const int first = xsrc[(a * P1) * c.nx + ix];
    const int last = xsrc[(a * P1 + P) * c.nx + ix];
    x0[a] = unsigned(first) * unsigned(sizeof(T));
    seam |= last != first + P;  // stencil wraps around a periodic seam
#pragma unroll
    for (int m = 0; m < P1; ++m) wx[a][m] = xw[(a * P1 + m) * c.nx + ix];
  }
  T fs[S][Q1 * Q1];
  // one uniform branch: wavefronts touching a seam gather element by element
  if (__builtin_amdgcn_ballot_w64(seam))
    direct_stream<T, P1, S, true, Q1>(fin, xsrc, yw, ysrc, x0, wx, ix, iy, c, fs);
  else
    direct_stream<T, P1, S, false, Q1>(fin, xsrc, yw, ysrc, x0, wx, ix, iy, c, fs);
  collide_store<T, MODEL, PR, Q1>(fs, c, fout, (long long)iy * c.nx + ix, flag);
}

// PR: the Pr != 1 collision (thermal models only)
template <bool PR>
hipError_t launch_direct_family(int fp32, int model, const StepConsts &c, const DevTables &t,
                                const void *fin, void *fout, int *flag, hipStream_t s) {
  if (c.q1 == 3) {  // D2Q9: isothermal BGK
    if constexpr (PR) {
      return hipErrorInvalidValue;
    } else {
      return dispatch_q3(fp32, c.p, model, [&]<typename T, int P>() {
        dim3 grid((c.nx + 63) / 64, (c.ny + 3) / 4);
        k_step_direct<T, P, kIsothermal, false, 3><<<grid, dim3(64, 4), 0, s>>>(
            static_cast<const T *>(fin), static_cast<T *>(fout), t.xsrc,
            static_cast<const T *>(t.xw), t.ysrc, static_cast<const T *>(t.yw), c, flag);
        return hipGetLastError();
      });
    }
  }
  if (c.q1 != 5) return hipErrorInvalidValue;
  return dispatch_step<PR>(fp32, c.p, model, [&]<typename T, int P, int MODEL>() {
    dim3 grid((c.nx + 63) / 64, (c.ny + 3) / 4);
    k_step_direct<T, P, MODEL, PR><<<grid, dim3(64, 4), 0, s>>>(
        static_cast<const T *>(fin), static_cast<T *>(fout), t.xsrc, static_cast<const T *>(t.xw),
        t.ysrc, static_cast<const T *>(t.yw), c, flag);
    return hipGetLastError();
  });
}

}  // namespace sllbm
