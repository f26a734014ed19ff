// Adjoint of the isothermal SLLBM step (HIP, gfx950).
//
// One forward step is F' = C(S F): S is the linear semi-Lagrangian
// interpolation of every population plane (eq. (17)) and C the node-local BGK
// collision toward the 4th-order equilibrium (eq. (16), theta = 1).  For a
// loss L of the final state the reverse sweep is
//     mu^n     = J_C(M^n)^T lambda^{n+1}      (node-local)
//     lambda^n = S^T mu^n                     (transposed interpolation)
// where M^n = (rho, u) of the streamed state S F^n (recorded by the forward
// recomputation).  With f_eq_i = rho Phi_i(u), u = j / rho and the moments
// rho = sum f, j = sum xi f:
//     (J_C^T lambda)_k = (1 - w) lambda_k
//                        + w (c_Phi - u . c_u + xi_k . c_u),
//     c_Phi = sum_i lambda_i Phi_i,   c_u = sum_i lambda_i dPhi_i/du,
// w = 1/tau.  Phi_{a+5b} = w_a w_b sum_{k+m<=4} A_k(u_x) h_{a,k} A_m(u_y) h_{b,m}
// with A_k the Hermite moments of a unit-variance Gaussian (theta = 1) and
// h_{a,k} = He_k(xi_a)/k!, so every contraction factorises through the 5 x 5
// matrix G[k][m] = sum_{a,b} lambda_{a+5b} w_a h_{a,k} w_b h_{b,m}.
//
// S^T is a gather through transposed per-axis tables (for source node j, the
// consecutive targets whose departure stencil contains j, with their
// weights), run by the same LDS-staged gather as the forward step.
#include <hip/hip_runtime.h>

#include "launch.hpp"
#include "step_common.hpp"
#include "tiled_common.hpp"

namespace sllbm {

namespace {

// A_k(u) and dA_k/du for theta = 1 (Hermite moments of N(u, 1)).
__device__ __forceinline__ void hermite_moments(double u, double (&A)[5], double (&dA)[5]) {
  const double u2 = u * u;
  A[0] = 1.0;
  A[1] = u;
  A[2] = u2;
  A[3] = u2 * u;
  A[4] = u2 * u2;
  dA[0] = 0.0;
  dA[1] = 1.0;
  dA[2] = 2.0 * u;
  dA[3] = 3.0 * u2;
  dA[4] = 4.0 * u2 * u;
}

// G[k][m] = sum_{a,b} lam_{a+5b} w_a h_{a,k} w_b h_{b,m}
template <typename T>
__device__ __forceinline__ void hermite_projection(const T (&lam)[25], const StepConsts &c,
                                                   double (&G)[5][5]) {
  double H[5][5];  // H[k][b] = sum_a lam_{a+5b} w_a h_{a,k}
#pragma unroll
  for (int b = 0; b < 5; ++b)
#pragma unroll
    for (int k = 0; k < 5; ++k) {
      double s = 0.0;
#pragma unroll
      for (int a = 0; a < 5; ++a) s = fma(double(lam[a + 5 * b]) * c.w[a], c.hk[a][k], s);
      H[k][b] = s;
    }
#pragma unroll
  for (int k = 0; k < 5; ++k)
#pragma unroll
    for (int m = 0; m < 5; ++m) {
      double s = 0.0;
#pragma unroll
      for (int b = 0; b < 5; ++b) s = fma(H[k][b] * c.w[b], c.hk[b][m], s);
      G[k][m] = s;
    }
}

// c_Phi, c_ux, c_uy of lam at velocity u (theta = 1).
template <typename T>
__device__ __forceinline__ void equilibrium_adjoint(const T (&lam)[25], double ux, double uy,
                                                    const StepConsts &c, double &cphi,
                                                    double &cx, double &cy) {
  double G[5][5];
  hermite_projection<T>(lam, c, G);
  double Ax[5], dAx[5], Ay[5], dAy[5];
  hermite_moments(ux, Ax, dAx);
  hermite_moments(uy, Ay, dAy);
  cphi = 0.0;
  cx = 0.0;
  cy = 0.0;
#pragma unroll
  for (int k = 0; k < 5; ++k)
#pragma unroll
    for (int m = 0; m + k <= 4; ++m) {
      cphi = fma(Ax[k] * Ay[m], G[k][m], cphi);
      cx = fma(dAx[k] * Ay[m], G[k][m], cx);
      cy = fma(Ax[k] * dAy[m], G[k][m], cy);
    }
}

// mu = J_C(rho, u)^T lam, stored at node v of a [25][n] array.
template <typename T>
__device__ __forceinline__ void collision_adjoint_store(const T (&lam)[25], double ux, double uy,
                                                        const StepConsts &c, T *__restrict__ out,
                                                        long long v) {
  double cphi, cx, cy;
  equilibrium_adjoint<T>(lam, ux, uy, c, cphi, cx, cy);
  const double om = c.omega;
  const double cr = cphi - ux * cx - uy * cy;
  const unsigned voff = unsigned(v) * unsigned(sizeof(T));
  const unsigned plane_bytes = unsigned(c.n * (long long)sizeof(T));
#pragma unroll
  for (int b = 0; b < 5; ++b)
#pragma unroll
    for (int a = 0; a < 5; ++a) {
      const int i = a + 5 * b;
      const double r = cr + c.xi[a] * cx + c.xi[b] * cy;
      const double mu = fma(1.0 - om, double(lam[i]), om * r);
      buffer_store<T>(T(mu), make_rsrc(out + i * c.n, plane_bytes), voff, 0);
    }
}

template <typename T>
__device__ __forceinline__ void store25(const T (&lam)[25], const StepConsts &c,
                                        T *__restrict__ out, long long v) {
  const unsigned voff = unsigned(v) * unsigned(sizeof(T));
  const unsigned plane_bytes = unsigned(c.n * (long long)sizeof(T));
#pragma unroll
  for (int i = 0; i < 25; ++i) buffer_store<T>(lam[i], make_rsrc(out + i * c.n, plane_bytes), voff, 0);
}

}  // namespace

// ---------------------------------------------------------------------------
// lambda^N_i = dL/dF_i = g_rho + (g_ux (xi_ix - u_x) + g_uy (xi_iy - u_y)) / rho
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(256) void k_adjoint_seed(const T *__restrict__ f,
                                                      const double *__restrict__ g_rho,
                                                      const double *__restrict__ g_ux,
                                                      const double *__restrict__ g_uy,
                                                      T *__restrict__ lam, StepConsts c) {
  const long long v = (long long)blockIdx.x * 256 + threadIdx.x;
  if (v >= c.n) return;
  T fs[1][25];
#pragma unroll
  for (int i = 0; i < 25; ++i) fs[0][i] = f[i * c.n + v];
  double m[4];
  node_moments<T, kIsothermal>(fs, c, m);
  const double gr = g_rho[v], gx = g_ux[v] / m[0], gy = g_uy[v] / m[0];
#pragma unroll
  for (int b = 0; b < 5; ++b)
#pragma unroll
    for (int a = 0; a < 5; ++a)
      lam[(a + 5 * b) * c.n + v] = T(gr + gx * (c.xi[a] - m[1]) + gy * (c.xi[b] - m[2]));
}

template <typename T>
__global__ __launch_bounds__(256) void k_adjoint_collide(const T *__restrict__ lam,
                                                         const double *__restrict__ mom,
                                                         T *__restrict__ mu, StepConsts c) {
  const long long v = (long long)blockIdx.x * 256 + threadIdx.x;
  if (v >= c.n) return;
  T l[25];
#pragma unroll
  for (int i = 0; i < 25; ++i) l[i] = lam[i * c.n + v];
  collision_adjoint_store<T>(l, mom[c.n + v], mom[2 * c.n + v], c, mu, v);
}

// S^T by direct gathers through the transposed tables (no LDS).
template <typename T, int TAPS>
__global__ __launch_bounds__(256) void k_adjoint_step_direct(
    const T *__restrict__ mu, const int32_t *__restrict__ xsrc, const T *__restrict__ xw,
    const int32_t *__restrict__ ysrc, const T *__restrict__ yw, const double *__restrict__ mom,
    T *__restrict__ out, StepConsts c) {
  const int ix = blockIdx.x * 64 + threadIdx.x;
  const int iy = blockIdx.y * 4 + threadIdx.y;
  if (ix >= c.nx || iy >= c.ny) return;
  const long long N = c.n;
  T lam[1][25];
#pragma unroll
  for (int b = 0; b < 5; ++b)
#pragma unroll
    for (int a = 0; a < 5; ++a) {
      const T *src = mu + (a + 5 * b) * N;
      T acc = T(0);
      for (int n = 0; n < TAPS; ++n) {
        const T wyn = yw[(b * TAPS + n) * c.ny + iy];
        const long long row = (long long)ysrc[(b * TAPS + n) * c.ny + iy] * c.nx;
        T r = T(0);
        for (int m = 0; m < TAPS; ++m)
          r = fma(xw[(a * TAPS + m) * c.nx + ix], src[row + xsrc[(a * TAPS + m) * c.nx + ix]], r);
        acc = fma(wyn, r, acc);
      }
      asm volatile("" : "+v"(acc));
      lam[0][a + 5 * b] = acc;
    }
  const long long v = (long long)iy * c.nx + ix;
  if (mom)
    collision_adjoint_store<T>(lam[0], mom[N + v], mom[2 * N + v], c, out, v);
  else
    store25<T>(lam[0], c, out, v);
}

// S^T with the LDS-staged gather of the forward step.
template <typename T, int TAPS, int HALO, int R>
__global__ __launch_bounds__(64 * kTileRowsTY) void k_adjoint_step_tiled(
    const T *__restrict__ mu, const int32_t *__restrict__ xrel, const T *__restrict__ xw,
    const int32_t *__restrict__ xwin, const int32_t *__restrict__ yrel, const T *__restrict__ yw,
    const int32_t *__restrict__ ywin, int W, int ntx, int nty, const double *__restrict__ mom,
    T *__restrict__ out, StepConsts c) {
  constexpr int TY = kTileRowsTY;
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
  T lam[1][25];
  tiled_stream<T, TAPS, 1, TY, HALO, 5, R, (TAPS >= kSeparableTaps ? kInterpSep : kInterp2D)>(
      mu, xrel, xw, xwin, yrel, yw, ywin, W, ntx, nty, tx, ty, ixc, iyc, lane, wv, c, lds, lam);
  if (ix < c.nx && iy < c.ny) {
    const long long v = (long long)iy * c.nx + ix;
    if (mom)
      collision_adjoint_store<T>(lam[0], mom[c.n + v], mom[2 * c.n + v], c, out, v);
    else
      store25<T>(lam[0], c, out, v);
  }
}

// g_rho0 = sum_i lam_i Phi_i(u0),  g_u0 = rho0 sum_i lam_i dPhi_i/du (f = f_eq(rho0, u0)).
template <typename T>
__global__ __launch_bounds__(256) void k_eq_init_vjp(const T *__restrict__ lam,
                                                     const double *__restrict__ rho0,
                                                     const double *__restrict__ ux0,
                                                     const double *__restrict__ uy0,
                                                     double *__restrict__ g_rho,
                                                     double *__restrict__ g_ux,
                                                     double *__restrict__ g_uy, StepConsts c) {
  const long long v = (long long)blockIdx.x * 256 + threadIdx.x;
  if (v >= c.n) return;
  T l[25];
#pragma unroll
  for (int i = 0; i < 25; ++i) l[i] = lam[i * c.n + v];
  double cphi, cx, cy;
  equilibrium_adjoint<T>(l, ux0[v], uy0[v], c, cphi, cx, cy);
  g_rho[v] = cphi;
  g_ux[v] = rho0[v] * cx;
  g_uy[v] = rho0[v] * cy;
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
namespace {

constexpr int kMaxTaps = 12;

template <class F>
hipError_t dispatch_taps(int fp32, int taps, F &&f) {
  auto by_taps = [&]<typename T>() -> hipError_t {
    switch (taps) {
      case 2: return f.template operator()<T, 2>();
      case 3: return f.template operator()<T, 3>();
      case 4: return f.template operator()<T, 4>();
      case 5: return f.template operator()<T, 5>();
      case 6: return f.template operator()<T, 6>();
      case 7: return f.template operator()<T, 7>();
      case 8: return f.template operator()<T, 8>();
      case 9: return f.template operator()<T, 9>();
      case 10: return f.template operator()<T, 10>();
      case 11: return f.template operator()<T, 11>();
      case 12: return f.template operator()<T, 12>();
    }
    return hipErrorInvalidValue;
  };
  return fp32 ? by_taps.template operator()<float>() : by_taps.template operator()<double>();
}

}  // namespace

hipError_t launch_adjoint_seed(int fp32, const StepConsts &c, const void *f, const double *g_rho,
                               const double *g_ux, const double *g_uy, void *lam, hipStream_t s) {
  const unsigned blocks = unsigned((c.n + 255) / 256);
  if (fp32)
    k_adjoint_seed<float><<<blocks, 256, 0, s>>>(static_cast<const float *>(f), g_rho, g_ux, g_uy,
                                                 static_cast<float *>(lam), c);
  else
    k_adjoint_seed<double><<<blocks, 256, 0, s>>>(static_cast<const double *>(f), g_rho, g_ux,
                                                  g_uy, static_cast<double *>(lam), c);
  return hipGetLastError();
}

hipError_t launch_adjoint_collide(int fp32, const StepConsts &c, const void *lam,
                                  const double *mom, void *mu, hipStream_t s) {
  const unsigned blocks = unsigned((c.n + 255) / 256);
  if (fp32)
    k_adjoint_collide<float><<<blocks, 256, 0, s>>>(static_cast<const float *>(lam), mom,
                                                    static_cast<float *>(mu), c);
  else
    k_adjoint_collide<double><<<blocks, 256, 0, s>>>(static_cast<const double *>(lam), mom,
                                                     static_cast<double *>(mu), c);
  return hipGetLastError();
}

hipError_t launch_adjoint_step(int fp32, bool tiled, const StepConsts &c, const DevTables &t,
                               const void *mu, const double *mom_prev, void *out, hipStream_t s) {
  if (t.taps < 2 || t.taps > kMaxTaps) return hipErrorInvalidValue;
  return dispatch_taps(fp32, t.taps, [&]<typename T, int TAPS>() -> hipError_t {
    const T *in = static_cast<const T *>(mu);
    T *o = static_cast<T *>(out);
    if (tiled) {
      constexpr int TY = kTileRowsTY;
      const int ntx = (c.nx + 63) / 64, nty = (c.ny + TY - 1) / TY;
      const int grid = ((ntx * nty + 7) / 8) * 8;
      const int W = t.win_rows;
      const int halo = tiled_halo(t.win_cols, c.nx, c.ny);
      if (W > 3 * TY || halo == 0) return hipErrorInvalidValue;
      constexpr bool SEP = TAPS >= kSeparableTaps;
      const size_t lds = tiled_lds_bytes(sizeof(T), 1, 5, W, 64 + halo, SEP);
      if (lds > kTiledLdsBudget) return hipErrorInvalidValue;
      auto go = [&]<int HALO, int R>() {
        k_adjoint_step_tiled<T, TAPS, HALO, R><<<grid, dim3(64, TY), lds, s>>>(
            in, t.xrel, static_cast<const T *>(t.xw), t.xwin, t.yrel,
            static_cast<const T *>(t.yw), t.ywin, W, ntx, nty, mom_prev, o, c);
      };
      auto by_rows = [&]<int HALO>() {
        if (W <= 2 * TY) go.template operator()<HALO, 2>();
        else go.template operator()<HALO, 3>();
      };
      if (halo == 4) by_rows.template operator()<4>();
      else if (halo == 8) by_rows.template operator()<8>();
      else by_rows.template operator()<64>();
      return hipGetLastError();
    }
    dim3 grid((c.nx + 63) / 64, (c.ny + 3) / 4);
    k_adjoint_step_direct<T, TAPS><<<grid, dim3(64, 4), 0, s>>>(
        in, t.xsrc, static_cast<const T *>(t.xw), t.ysrc, static_cast<const T *>(t.yw), mom_prev,
        o, c);
    return hipGetLastError();
  });
}

hipError_t launch_eq_init_vjp(int fp32, const StepConsts &c, const void *lam, const double *rho0,
                              const double *ux0, const double *uy0, double *g_rho,
                              double *g_ux, double *g_uy, hipStream_t s) {
  const unsigned blocks = unsigned((c.n + 255) / 256);
  if (fp32)
    k_eq_init_vjp<float><<<blocks, 256, 0, s>>>(static_cast<const float *>(lam), rho0, ux0, uy0,
                                                g_rho, g_ux, g_uy, c);
  else
    k_eq_init_vjp<double><<<blocks, 256, 0, s>>>(static_cast<const double *>(lam), rho0, ux0, uy0,
                                                 g_rho, g_ux, g_uy, c);
  return hipGetLastError();
}

}  // namespace sllbm
