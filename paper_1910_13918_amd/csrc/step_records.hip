// Stream + collide: general gather through per-(node, velocity) departure
// records (HIP, gfx950).
#include <hip/hip_runtime.h>

#include "launch.hpp"
#include "step_common.hpp"

namespace sllbm {

// ---------------------------------------------------------------------------
// stream + collide, general gather through per-(node, velocity) records
// (departure cell and reference coordinates; weights evaluated here)
// ---------------------------------------------------------------------------
template <typename T, int P, int MODEL>
__global__ __launch_bounds__(256) void k_step_records(const T *__restrict__ fin,
                                                      T *__restrict__ fout,
                                                      const int32_t *__restrict__ cell,
                                                      const T *__restrict__ rr,
                                                      const T *__restrict__ ss, StepConsts c,
                                                      int *__restrict__ flag) {
  constexpr int S = Sets<MODEL>::S;
  constexpr int P1 = P + 1;
  const long long v = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= c.n) return;
  const long long N = c.n;
  T rn[P1], den[P1];
#pragma unroll
  for (int m = 0; m < P1; ++m) {
    rn[m] = T(c.rn[m]);
    den[m] = T(c.lden[m]);
  }
  T fs[S][25];
#pragma unroll
  for (int i = 0; i < 25; ++i) {
    const int rec = cell[i * N + v];
    const int cx = rec & 0xffff, cy = rec >> 16;
    T wx[P1], wy[P1];
    lagrange_eval<T, P1>(rr[i * N + v], rn, den, wx);
    lagrange_eval<T, P1>(ss[i * N + v], rn, den, wy);
    int xo[P1];
    long long yo[P1];
#pragma unroll
    for (int m = 0; m < P1; ++m) {
      int jx = cx * P + m;
      if (jx >= c.nx) jx -= c.nx;  // periodic seam: last vertex is node 0
      xo[m] = jx;
      int jy = cy * P + m;
      if (jy >= c.ny) jy -= c.ny;
      yo[m] = (long long)jy * c.nx;
    }
#pragma unroll
    for (int s = 0; s < S; ++s) {
      const T *src = fin + (long long)(s * 25 + i) * N;
      T acc = T(0);
#pragma unroll
      for (int n = 0; n < P1; ++n) {
        T row = T(0);
#pragma unroll
        for (int m = 0; m < P1; ++m) row = fma(wx[m], src[yo[n] + xo[m]], row);
        acc = fma(wy[n], row, acc);
      }
      fs[s][i] = acc;
    }
  }
  collide_store<T, MODEL>(fs, c, fout, v, flag);
}

hipError_t launch_step_records(int fp32, int model, const StepConsts &c, const DevTables &t,
                               const void *fin, void *fout, int *flag, hipStream_t s) {
  return dispatch_step(fp32, c.p, model, [&]<typename T, int P, int MODEL>() {
    const unsigned blocks = unsigned((c.n + 255) / 256);
    k_step_records<T, P, MODEL><<<blocks, 256, 0, s>>>(
        static_cast<const T *>(fin), static_cast<T *>(fout), t.rec_cell,
        static_cast<const T *>(t.rec_r), static_cast<const T *>(t.rec_s), c, flag);
    return hipGetLastError();
  });
}

}  // namespace sllbm
