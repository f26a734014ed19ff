// Adjoint of the SLLBM step (HIP, gfx950), every model.
//
// One forward step is F' = C(S F): S is the linear semi-Lagrangian
// interpolation of every population plane (eq. (17)) and C the node-local BGK
// collision toward the 4th-order equilibrium (eq. (16)).  For a loss L of the
// final state the reverse sweep is
//     mu^n     = J_C(M^n)^T lambda^{n+1}      (node-local)
//     lambda^n = S^T mu^n                     (transposed interpolation)
// where M^n = (rho, u, theta) of the streamed state S F^n (recorded by the
// forward recomputation).  With f_eq_i = rho Phi_i(u, theta),
// g_eq_i = c theta rho Phi_i (c = 2 C_v - D, Sec. II.D), u = j / rho and
// 2 C_v rho theta = sum |xi|^2 f + sum g - rho |u|^2 (theta = 1 isothermal):
//     d rho / d f_k = 1,  d u / d f_k = (xi_k - u) / rho,
//     d theta / d f_k = (|xi_k - u|^2 - 2 C_v theta) / (2 C_v rho),
//     d theta / d g_k = 1 / (2 C_v rho),
// and with the contractions (lt_i = lam_f_i + c theta lam_g_i)
//     P = sum lt_i Phi_i,  P_u = sum lt_i dPhi_i/du,
//     P_t = sum lt_i dPhi_i/dtheta + c sum lam_g_i Phi_i,
// the transposed collision Jacobian is
//     mu_f_k = (1 - w) lam_f_k + w (P + P_u . (xi_k - u)
//                                   + P_t (|xi_k - u|^2 - 2 C_v theta) / (2 C_v)),
//     mu_g_k = (1 - w) lam_g_k + w P_t / (2 C_v),
// w = 1/tau.  Phi_{a+5b} = w_a w_b sum_{k+m<=4} A_k(u_x) h_{a,k} A_m(u_y) h_{b,m}
// with A_k the Hermite moments of a Gaussian of mean u and variance theta and
// h_{a,k} = He_k(xi_a)/k!, so every contraction factorises through the 5 x 5
// matrix G[k][m] = sum_{a,b} lt_{a+5b} w_a h_{a,k} w_b h_{b,m}.
//
// S^T is a gather through transposed per-axis tables (for source node j, the
// consecutive targets whose departure stencil contains j, with their
// weights), run by the same gathers as the forward step: direct here,
// tiled windows in adjoint_tiled.hpp, row segments in adjoint_rows.hip; the device helpers below the
// kernels live in adjoint_common.hpp.
#include <hip/hip_runtime.h>

#include "launch.hpp"
#include "adjoint_common.hpp"
#include "step_common.hpp"
#include "tiled_common.hpp"

namespace sllbm {


// ---------------------------------------------------------------------------
// lambda^N = dL/dF from dL/d(rho, u, theta) of the current populations (f in
// the storage order c.layout; lambda, like every adjoint array, planar):
//   lam_f_k = g_rho + g_u . (xi_k - u) / rho
//             + g_theta (|xi_k - u|^2 - 2 C_v theta) / (2 C_v rho),
//   lam_g_k = g_theta / (2 C_v rho)                 (g_theta = 0 if absent)
// ---------------------------------------------------------------------------
template <typename T, int MODEL>
__global__ __launch_bounds__(256) void k_adjoint_seed(const T *__restrict__ f,
                                                      const double *__restrict__ g_rho,
                                                      const double *__restrict__ g_ux,
                                                      const double *__restrict__ g_uy,
                                                      const double *__restrict__ g_th,
                                                      T *__restrict__ lam, StepConsts c) {
  constexpr int S = Sets<MODEL>::S;
  const long long v = (long long)blockIdx.x * 256 + threadIdx.x;
  if (v >= c.n) return;
  T fs[S][25];
#pragma unroll
  for (int s = 0; s < S; ++s)
#pragma unroll
    for (int i = 0; i < 25; ++i) fs[s][i] = f[pop_elem(c.layout, 5, s, i % 5, i / 5, v, c.n)];
  double m[4];
  node_moments<T, MODEL>(fs, c, m);
  const double inv_rho = 1.0 / m[0];
  const double gr = g_rho[v], gx = g_ux[v] * inv_rho, gy = g_uy[v] * inv_rho;
  const double gt = (MODEL != kIsothermal && g_th) ? g_th[v] * c.inv_2cv * inv_rho : 0.0;
  const double two_cv_theta = m[3] / c.inv_2cv;
#pragma unroll
  for (int b = 0; b < 5; ++b)
#pragma unroll
    for (int a = 0; a < 5; ++a) {
      const double dx = c.xi[a] - m[1], dy = c.xi[b] - m[2];
      double l = gr + gx * dx + gy * dy;
      if constexpr (MODEL != kIsothermal) l = fma(gt, dx * dx + dy * dy - two_cv_theta, l);
      lam[(a + 5 * b) * c.n + v] = T(l);
      if constexpr (S == 2) lam[(25 + a + 5 * b) * c.n + v] = T(gt);
    }
}

template <typename T, int MODEL, bool PR = false>
__global__ __launch_bounds__(256) void k_adjoint_collide(const T *__restrict__ lam,
                                                         const double *__restrict__ mom,
                                                         T *__restrict__ mu, StepConsts c) {
  constexpr int S = Sets<MODEL>::S;
  const long long v = (long long)blockIdx.x * 256 + threadIdx.x;
  if (v >= c.n) return;
  T l[S][25];
#pragma unroll
  for (int s = 0; s < S; ++s)
#pragma unroll
    for (int i = 0; i < 25; ++i) l[s][i] = lam[(s * 25 + i) * c.n + v];
  collision_adjoint_store<T, MODEL, PR>(l, mom, c, mu, v);
}

// S^T on a curvilinear mesh: for source node j and velocity i, the sum over
// the targets whose departure stencil holds j (their records' Lagrange
// weights, built on the host) of weight x mu_i(target); then J_C^T of the
// previous step when mom_prev is given (Pr = 1).  One thread per source node.
template <typename T, int MODEL>
__global__ __launch_bounds__(256) void k_adjoint_step_csr(const T *__restrict__ mu,
                                                          const uint32_t *__restrict__ ptr,
                                                          const int32_t *__restrict__ col,
                                                          const T *__restrict__ w,
                                                          const double *__restrict__ mom_prev,
                                                          T *__restrict__ out, StepConsts c) {
  constexpr int S = Sets<MODEL>::S;
  const long long j = (long long)blockIdx.x * 256 + threadIdx.x;
  if (j >= c.n) return;
  const long long N = c.n;
  T lam[S][25];
#pragma unroll
  for (int i = 0; i < 25; ++i) {
    const uint32_t e0 = ptr[i * (N + 1) + j], e1 = ptr[i * (N + 1) + j + 1];
    T acc[S];
#pragma unroll
    for (int s = 0; s < S; ++s) acc[s] = T(0);
    for (uint32_t e = e0; e < e1; ++e) {
      const long long v = col[e];
      const T we = w[e];
#pragma unroll
      for (int s = 0; s < S; ++s) acc[s] = fma(we, mu[(s * 25 + i) * N + v], acc[s]);
    }
#pragma unroll
    for (int s = 0; s < S; ++s) lam[s][i] = acc[s];
  }
  if (mom_prev)
    collision_adjoint_store<T, MODEL>(lam, mom_prev, c, out, j);
  else
    store_sets<T, S>(lam, c, out, j);
}

// S^T by direct gathers through the transposed tables (no LDS).
template <typename T, int MODEL, int TAPS>
__global__ __launch_bounds__(256) void k_adjoint_step_direct(
    const T *__restrict__ mu, const int32_t *__restrict__ xsrc, const T *__restrict__ xw,
    const int32_t *__restrict__ ysrc, const T *__restrict__ yw, const double *__restrict__ mom,
    T *__restrict__ out, StepConsts c) {
  constexpr int S = Sets<MODEL>::S;
  const int ix = blockIdx.x * 64 + threadIdx.x;
  const int iy = blockIdx.y * 4 + threadIdx.y;
  if (ix >= c.nx || iy >= c.ny) return;
  const long long N = c.n;
  T lam[S][25];
#pragma unroll
  for (int b = 0; b < 5; ++b)
#pragma unroll
    for (int a = 0; a < 5; ++a)
#pragma unroll
      for (int s = 0; s < S; ++s) {
        const T *src = mu + (s * 25 + a + 5 * b) * N;
        T acc = T(0);
        for (int n = 0; n < TAPS; ++n) {
          const T wyn = yw[(b * TAPS + n) * c.ny + iy];
          const long long row = (long long)ysrc[(b * TAPS + n) * c.ny + iy] * c.nx;
          T r = T(0);
          for (int m = 0; m < TAPS; ++m)
            r = fma(xw[(a * TAPS + m) * c.nx + ix], src[row + xsrc[(a * TAPS + m) * c.nx + ix]],
                    r);
          acc = fma(wyn, r, acc);
        }
        asm volatile("" : "+v"(acc));
        lam[s][a + 5 * b] = acc;
      }
  const long long v = (long long)iy * c.nx + ix;
  if (mom)
    collision_adjoint_store<T, MODEL>(lam, mom, c, out, v);
  else
    store_sets<T, S>(lam, c, out, v);
}

// Gradients through f = f_eq(rho0, u0, theta0) (and g = g_eq):
//   g_rho0 = P,  g_u0 = rho0 P_u,  g_theta0 = rho0 P_t.
template <typename T, int MODEL>
__global__ __launch_bounds__(256) void k_eq_init_vjp(const T *__restrict__ lam,
                                                     const double *__restrict__ rho0,
                                                     const double *__restrict__ ux0,
                                                     const double *__restrict__ uy0,
                                                     const double *__restrict__ th0,
                                                     double *__restrict__ g_rho,
                                                     double *__restrict__ g_ux,
                                                     double *__restrict__ g_uy,
                                                     double *__restrict__ g_th, StepConsts c) {
  constexpr int S = Sets<MODEL>::S;
  const long long v = (long long)blockIdx.x * 256 + threadIdx.x;
  if (v >= c.n) return;
  T l[S][25];
#pragma unroll
  for (int s = 0; s < S; ++s)
#pragma unroll
    for (int i = 0; i < 25; ++i) l[s][i] = lam[(s * 25 + i) * c.n + v];
  const double theta = (MODEL == kIsothermal || !th0) ? 1.0 : th0[v];
  double P, Px, Py, Pt;
  equilibrium_adjoint<T, MODEL>(l, ux0[v], uy0[v], theta, c, P, Px, Py, Pt);
  g_rho[v] = P;
  g_ux[v] = rho0[v] * Px;
  g_uy[v] = rho0[v] * Py;
  if (g_th) g_th[v] = MODEL == kIsothermal ? 0.0 : rho0[v] * Pt;
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------

hipError_t launch_adjoint_seed(int fp32, int model, const StepConsts &c, const void *f,
                               const double *g_rho, const double *g_ux, const double *g_uy,
                               const double *g_th, void *lam, hipStream_t s) {
  const unsigned blocks = unsigned((c.n + 255) / 256);
  return dispatch_model(fp32, model, [&]<typename T, int MODEL>() -> hipError_t {
    k_adjoint_seed<T, MODEL><<<blocks, 256, 0, s>>>(static_cast<const T *>(f), g_rho, g_ux, g_uy,
                                                    g_th, static_cast<T *>(lam), c);
    return hipGetLastError();
  });
}

hipError_t launch_adjoint_collide(int fp32, int model, const StepConsts &c, const void *lam,
                                  const double *mom, void *mu, hipStream_t s) {
  const unsigned blocks = unsigned((c.n + 255) / 256);
  const bool pr = c.omega_pr != c.omega;  // the quasi-equilibrium term (thermal models)
  return dispatch_model(fp32, model, [&]<typename T, int MODEL>() -> hipError_t {
    if constexpr (MODEL != kIsothermal) {
      if (pr) {
        k_adjoint_collide<T, MODEL, true><<<blocks, 256, 0, s>>>(static_cast<const T *>(lam), mom,
                                                                 static_cast<T *>(mu), c);
        return hipGetLastError();
      }
    } else if (pr) {
      return hipErrorInvalidValue;
    }
    k_adjoint_collide<T, MODEL><<<blocks, 256, 0, s>>>(static_cast<const T *>(lam), mom,
                                                       static_cast<T *>(mu), c);
    return hipGetLastError();
  });
}

hipError_t launch_adjoint_step(int fp32, int model, int kind, const StepConsts &c,
                               const DevTables &t, const void *mu, const double *mom_prev,
                               void *out, hipStream_t s) {
  // the fused J_C^T is the Pr = 1 one; the host splits the Pr != 1 step
  if (mom_prev && c.omega_pr != c.omega) return hipErrorInvalidValue;
  if (kind == kAdjointCsr) {
    if (!t.csr_ptr || !t.csr_col || !t.csr_w || c.q1 != 5) return hipErrorInvalidValue;
    const unsigned blocks = unsigned((c.n + 255) / 256);
    return dispatch_model(fp32, model, [&]<typename T, int MODEL>() -> hipError_t {
      k_adjoint_step_csr<T, MODEL><<<blocks, 256, 0, s>>>(
          static_cast<const T *>(mu), t.csr_ptr, t.csr_col, static_cast<const T *>(t.csr_w),
          mom_prev, static_cast<T *>(out), c);
      return hipGetLastError();
    });
  }
  if (t.taps < 2 || t.taps > kMaxTaps) return hipErrorInvalidValue;
  if (kind == kAdjointRows) return launch_adjoint_step_rows(fp32, model, c, t, mu, mom_prev, out, s);
  if (kind == kAdjointTiled)
    return fp32 ? launch_adjoint_step_tiled_t<float>(model, c, t, mu, mom_prev, out, s)
                : launch_adjoint_step_tiled_t<double>(model, c, t, mu, mom_prev, out, s);
  return dispatch_taps(fp32, model, t.taps, [&]<typename T, int MODEL, int TAPS>() -> hipError_t {
    dim3 grid((c.nx + 63) / 64, (c.ny + 3) / 4);
    k_adjoint_step_direct<T, MODEL, TAPS><<<grid, dim3(64, 4), 0, s>>>(
        static_cast<const T *>(mu), t.xsrc, static_cast<const T *>(t.xw), t.ysrc,
        static_cast<const T *>(t.yw), mom_prev, static_cast<T *>(out), c);
    return hipGetLastError();
  });
}

hipError_t launch_eq_init_vjp(int fp32, int model, const StepConsts &c, const void *lam,
                              const double *rho0, const double *ux0, const double *uy0,
                              const double *th0, double *g_rho, double *g_ux, double *g_uy,
                              double *g_th, hipStream_t s) {
  const unsigned blocks = unsigned((c.n + 255) / 256);
  return dispatch_model(fp32, model, [&]<typename T, int MODEL>() -> hipError_t {
    k_eq_init_vjp<T, MODEL><<<blocks, 256, 0, s>>>(static_cast<const T *>(lam), rho0, ux0, uy0,
                                                   th0, g_rho, g_ux, g_uy, g_th, c);
    return hipGetLastError();
  });
}

}  // namespace sllbm
