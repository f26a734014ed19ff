// Device building blocks shared by the stream + collide kernels:
// moments, temperature, the factorised 4th-order Hermite equilibrium, BGK
// relaxation with the store, and block reductions.
#pragma once

#include <hip/hip_runtime.h>

#include "launch.hpp"

namespace sllbm {

enum Model { kIsothermal = 0, kMonatomic = 1, kPolyatomic = 2 };

template <int MODEL>
struct Sets {
  static constexpr int S = (MODEL == kPolyatomic) ? 2 : 1;
};

// Lagrange weights l_m(r) = den_m * prod_{n != m} (r - r_n).
template <typename T, int P1>
__device__ __forceinline__ void lagrange_eval(T r, const T (&rn)[P1], const T (&den)[P1],
                                              T (&out)[P1]) {
  T d[P1];
#pragma unroll
  for (int n = 0; n < P1; ++n) d[n] = r - rn[n];
#pragma unroll
  for (int m = 0; m < P1; ++m) {
    T v = den[m];
#pragma unroll
    for (int n = 0; n < P1; ++n)
      if (n != m) v *= d[n];
    out[m] = v;
  }
}

// rho, u_x, u_y, theta of one node's populations (Sec. II, eqs. (3)-(5)):
// rho = sum f, rho u = sum xi f, 2 rho E = sum |xi|^2 f + sum g, and
// theta = (2 rho E - rho |u|^2) / (2 C_v rho) (theta = 1 when isothermal).
template <typename T, int MODEL>
__device__ __forceinline__ void node_moments(const T (&fs)[Sets<MODEL>::S][25],
                                             const StepConsts &c, double (&m)[4]) {
  double rho = 0.0, jx = 0.0, jy = 0.0, e = 0.0;
#pragma unroll
  for (int b = 0; b < 5; ++b) {
    double r_b = 0.0, jx_b = 0.0, e_b = 0.0;
#pragma unroll
    for (int a = 0; a < 5; ++a) {
      const double v = double(fs[0][a + 5 * b]);
      r_b += v;
      jx_b = fma(c.xi[a], v, jx_b);
      if (MODEL != kIsothermal) e_b = fma(c.xi[a] * c.xi[a], v, e_b);
    }
    rho += r_b;
    jx += jx_b;
    jy = fma(c.xi[b], r_b, jy);
    if (MODEL != kIsothermal) e += e_b + c.xi[b] * c.xi[b] * r_b;
  }
  if (MODEL == kPolyatomic) {
#pragma unroll
    for (int i = 0; i < 25; ++i) e += double(fs[Sets<MODEL>::S - 1][i]);
  }
  const double ux = jx / rho, uy = jy / rho;
  double theta = 1.0;
  if (MODEL != kIsothermal) theta = (e - rho * (ux * ux + uy * uy)) * c.inv_2cv / rho;
  m[0] = rho;
  m[1] = ux;
  m[2] = uy;
  m[3] = theta;
}

// Calls fn(i, f_eq_i) for the 25 velocities.  Factorised form of the
// 4th-order Hermite equilibrium (Sec. II.A): with t = theta - 1 and
// A_0 = 1, A_1 = u, A_2 = u^2 + t, A_3 = u^3 + 3ut, A_4 = u^4 + 6u^2 t + 3t^2
// (the Hermite moments of a Gaussian of mean u and variance theta),
// f_eq_{a+5b} = rho w_a w_b sum_{k+m<=4} A_k(u_x) He_k(xi_a)/k! A_m(u_y) He_m(xi_b)/m!,
// which equals the full tensor contraction of eqs. (9)-(10).
template <class Fn>
__device__ __forceinline__ void for_each_equilibrium(double rho, double ux, double uy,
                                                     double theta, const StepConsts &c, Fn &&fn) {
  const double t = theta - 1.0;
  const double ux2 = ux * ux, uy2 = uy * uy;
  const double Ax[5] = {1.0, ux, ux2 + t, ux * (ux2 + 3.0 * t),
                        ux2 * ux2 + 6.0 * ux2 * t + 3.0 * t * t};
  const double Ay[5] = {1.0, uy, uy2 + t, uy * (uy2 + 3.0 * t),
                        uy2 * uy2 + 6.0 * uy2 * t + 3.0 * t * t};
  // partial sums over the y-order: Yc[b][j] = sum_{m <= j} A_m(u_y) He_m(xi_b)/m!
  double Yc[5][5];
#pragma unroll
  for (int b = 0; b < 5; ++b) {
    double acc = 0.0;
#pragma unroll
    for (int j = 0; j < 5; ++j) {
      acc = fma(Ay[j], c.hk[b][j], acc);
      Yc[b][j] = acc;
    }
  }
#pragma unroll
  for (int a = 0; a < 5; ++a) {
    double X[5];
#pragma unroll
    for (int k = 0; k < 5; ++k) X[k] = Ax[k] * c.hk[a][k];
    const double rw = rho * c.w[a];
#pragma unroll
    for (int b = 0; b < 5; ++b) {
      double s = X[0] * Yc[b][4];
      s = fma(X[1], Yc[b][3], s);
      s = fma(X[2], Yc[b][2], s);
      s = fma(X[3], Yc[b][1], s);
      s = fma(X[4], Yc[b][0], s);
      fn(a + 5 * b, rw * c.w[b] * s);
    }
  }
}

// Moments, stability flag, equilibrium and BGK relaxation of one node's
// streamed populations; stores the post-collision values at node v
// (Sec. II.D, eq. (16) with Pr = 1):  f+ = f + (f_eq - f)/tau,
// g+ = g + (g_eq - g)/tau, g_eq = (2 C_v - D) theta f_eq.
template <typename T, int MODEL>
__device__ __forceinline__ void collide_store(const T (&fs)[Sets<MODEL>::S][25],
                                              const StepConsts &c, T *__restrict__ fout,
                                              long long v, int *__restrict__ flag) {
  double m[4];
  node_moments<T, MODEL>(fs, c, m);
  const bool ok = (m[0] > 0.0) && (m[3] > 0.0) && isfinite(m[0]) && isfinite(m[1]) &&
                  isfinite(m[2]) && isfinite(m[3]);
  if (!ok) atomicOr(flag, 1);
  const long long N = c.n;
  const double om = c.omega;
  const double gf = c.gfac * m[3];
  for_each_equilibrium(m[0], m[1], m[2], m[3], c, [&](int i, double feq) {
    const double f = double(fs[0][i]);
    fout[i * N + v] = T(fma(om, feq - f, f));
    if (Sets<MODEL>::S == 2) {
      const double g = double(fs[1][i]);
      fout[(25 + i) * N + v] = T(fma(om, gf * feq - g, g));
    }
  });
}

// Sum over a block of 256 threads (4 wavefronts of 64) in a fixed order;
// the result is valid in thread 0.
__device__ __forceinline__ double block_sum_256(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  __shared__ double part[4];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  if (lane == 0) part[wv] = v;
  __syncthreads();
  double t = 0.0;
  if (threadIdx.x == 0) t = ((part[0] + part[1]) + part[2]) + part[3];
  return t;
}

template <typename T, int P, int MODEL>
hipError_t launch_step_tiled(const StepConsts &c, const DevTables &t, const T *in, T *out,
                             int *flag, hipStream_t s);

}  // namespace sllbm
