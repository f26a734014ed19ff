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
// weights), run by the same LDS-staged gather as the forward step.
#include <hip/hip_runtime.h>

#include "launch.hpp"
#include "step_common.hpp"
#include "step_rows.hpp"
#include "tiled_common.hpp"

namespace sllbm {

namespace {

// A_k(u, t) and their u- and t-derivatives, t = theta - 1 (Hermite moments
// of N(u, theta)).
__device__ __forceinline__ void hermite_moments(double u, double t, double (&A)[5],
                                                double (&dA)[5], double (&tA)[5]) {
  const double u2 = u * u;
  A[0] = 1.0;
  A[1] = u;
  A[2] = u2 + t;
  A[3] = u * (u2 + 3.0 * t);
  A[4] = u2 * u2 + 6.0 * u2 * t + 3.0 * t * t;
  dA[0] = 0.0;
  dA[1] = 1.0;
  dA[2] = 2.0 * u;
  dA[3] = 3.0 * u2 + 3.0 * t;
  dA[4] = 4.0 * u2 * u + 12.0 * u * t;
  tA[0] = 0.0;
  tA[1] = 0.0;
  tA[2] = 1.0;
  tA[3] = 3.0 * u;
  tA[4] = 6.0 * u2 + 6.0 * t;
}

// G[k][m] = sum_{a,b} lam_{a+5b} w_a h_{a,k} w_b h_{b,m}
__device__ __forceinline__ void hermite_projection(const double (&lam)[25], const StepConsts &c,
                                                   double (&G)[5][5]) {
  double H[5][5];  // H[k][b] = sum_a lam_{a+5b} w_a h_{a,k}
#pragma unroll
  for (int b = 0; b < 5; ++b)
#pragma unroll
    for (int k = 0; k < 5; ++k) {
      double s = 0.0;
#pragma unroll
      for (int a = 0; a < 5; ++a) s = fma(lam[a + 5 * b], c.whk[a][k], s);
      H[k][b] = s;
    }
#pragma unroll
  for (int k = 0; k < 5; ++k)
#pragma unroll
    for (int m = 0; m < 5; ++m) {
      double s = 0.0;
#pragma unroll
      for (int b = 0; b < 5; ++b) s = fma(H[k][b], c.whk[b][m], s);
      G[k][m] = s;
    }
}

// P, P_u and (thermal models) P_t of lam at (u, theta).
template <typename T, int MODEL>
__device__ __forceinline__ void equilibrium_adjoint(const T (&lam)[Sets<MODEL>::S][25], double ux,
                                                    double uy, double theta,
                                                    const StepConsts &c, double &P, double &Px,
                                                    double &Py, double &Pt) {
  constexpr int S = Sets<MODEL>::S;
  const double ct = c.gfac * theta;
  double lt[25];
#pragma unroll
  for (int i = 0; i < 25; ++i) {
    lt[i] = double(lam[0][i]);
    if constexpr (S == 2) lt[i] = fma(ct, double(lam[S - 1][i]), lt[i]);
  }
  double G[5][5];
  hermite_projection(lt, c, G);
  const double t = MODEL == kIsothermal ? 0.0 : theta - 1.0;
  double Ax[5], dAx[5], tAx[5], Ay[5], dAy[5], tAy[5];
  hermite_moments(ux, t, Ax, dAx, tAx);
  hermite_moments(uy, t, Ay, dAy, tAy);
  P = 0.0;
  Px = 0.0;
  Py = 0.0;
  Pt = 0.0;
#pragma unroll
  for (int k = 0; k < 5; ++k)
#pragma unroll
    for (int m = 0; m + k <= 4; ++m) {
      P = fma(Ax[k] * Ay[m], G[k][m], P);
      Px = fma(dAx[k] * Ay[m], G[k][m], Px);
      Py = fma(Ax[k] * dAy[m], G[k][m], Py);
      if constexpr (MODEL != kIsothermal)
        Pt = fma(tAx[k] * Ay[m] + Ax[k] * tAy[m], G[k][m], Pt);
    }
  if constexpr (S == 2) {
    double lg[25];
#pragma unroll
    for (int i = 0; i < 25; ++i) lg[i] = double(lam[S - 1][i]);
    double Gg[5][5];
    hermite_projection(lg, c, Gg);
    double Pg = 0.0;
#pragma unroll
    for (int k = 0; k < 5; ++k)
#pragma unroll
      for (int m = 0; m + k <= 4; ++m) Pg = fma(Ax[k] * Ay[m], Gg[k][m], Pg);
    Pt = fma(c.gfac, Pg, Pt);
  }
}

// mu = J_C(rho, u, theta)^T lam, stored at node v of an [S][25][n] array.
template <typename T, int MODEL>
__device__ __forceinline__ void collision_adjoint_store(const T (&lam)[Sets<MODEL>::S][25],
                                                        const double *__restrict__ mom,
                                                        const StepConsts &c, T *__restrict__ out,
                                                        long long v) {
  constexpr int S = Sets<MODEL>::S;
  const double ux = mom[c.n + v], uy = mom[2 * c.n + v];
  const double theta = MODEL == kIsothermal ? 1.0 : mom[3 * c.n + v];
  double P, Px, Py, Pt;
  equilibrium_adjoint<T, MODEL>(lam, ux, uy, theta, c, P, Px, Py, Pt);
  const double om = c.omega;
  const double two_cv_theta = theta / c.inv_2cv;
  const unsigned voff = unsigned(v) * unsigned(sizeof(T));
  const unsigned plane_bytes = unsigned(c.n * (long long)sizeof(T));
#pragma unroll
  for (int b = 0; b < 5; ++b)
#pragma unroll
    for (int a = 0; a < 5; ++a) {
      const int i = a + 5 * b;
      const double dx = c.xi[a] - ux, dy = c.xi[b] - uy;
      double r = fma(Px, dx, fma(Py, dy, P));
      if constexpr (MODEL != kIsothermal)
        r = fma(Pt * c.inv_2cv, dx * dx + dy * dy - two_cv_theta, r);
      const double mu = fma(1.0 - om, double(lam[0][i]), om * r);
      buffer_store<T>(T(mu), make_rsrc(out + i * c.n, plane_bytes), voff, 0);
      if constexpr (S == 2) {
        const double mg = fma(1.0 - om, double(lam[S - 1][i]), om * Pt * c.inv_2cv);
        buffer_store<T>(T(mg), make_rsrc(out + (25 + i) * c.n, plane_bytes), voff, 0);
      }
    }
}

template <typename T, int S>
__device__ __forceinline__ void store_sets(const T (&lam)[S][25], const StepConsts &c,
                                           T *__restrict__ out, long long v) {
  const unsigned voff = unsigned(v) * unsigned(sizeof(T));
  const unsigned plane_bytes = unsigned(c.n * (long long)sizeof(T));
#pragma unroll
  for (int s = 0; s < S; ++s)
#pragma unroll
    for (int i = 0; i < 25; ++i)
      buffer_store<T>(lam[s][i], make_rsrc(out + (s * 25 + i) * c.n, plane_bytes), voff, 0);
}

}  // namespace

// ---------------------------------------------------------------------------
// lambda^N = dL/dF from dL/d(rho, u, theta) of the current populations:
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
    for (int i = 0; i < 25; ++i) fs[s][i] = f[(s * 25 + i) * c.n + v];
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

template <typename T, int MODEL>
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
  collision_adjoint_store<T, MODEL>(l, mom, c, mu, v);
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

// S^T with the LDS-staged gather of the forward step.
template <typename T, int MODEL, int TAPS, int HALO, int G, int R>
__global__ __launch_bounds__(64 * kTileRowsTY) void k_adjoint_step_tiled(
    const T *__restrict__ mu, const int32_t *__restrict__ xrel, const T *__restrict__ xw,
    const int32_t *__restrict__ xwin, const int32_t *__restrict__ yrel, const T *__restrict__ yw,
    const int32_t *__restrict__ ywin, int W, int ntx, int nty, const double *__restrict__ mom,
    T *__restrict__ out, StepConsts c) {
  constexpr int TY = kTileRowsTY;
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
  T lam[S][25];
  tiled_stream<T, TAPS, S, TY, HALO, G, R, (TAPS >= kSeparableTaps ? kInterpSep : kInterp2D)>(
      mu, xrel, xw, xwin, yrel, yw, ywin, W, ntx, nty, tx, ty, ixc, iyc, lane, wv, c, lds, lam);
  if (ix < c.nx && iy < c.ny) {
    const long long v = (long long)iy * c.nx + ix;
    if (mom)
      collision_adjoint_store<T, MODEL>(lam, mom, c, out, v);
    else
      store_sets<T, S>(lam, c, out, v);
  }
}

// S^T with the row-segment gather of the forward step (transposed tables).
template <typename T, int MODEL, int TAPS>
__global__ __launch_bounds__(64 * kRowsTileRows) void k_adjoint_step_rows(
    const T *__restrict__ mu, const int32_t *__restrict__ xrel, const T *__restrict__ xw,
    const int32_t *__restrict__ xwin, const int32_t *__restrict__ ysrc, const T *__restrict__ yw,
    int TX, int ntx, int nty, const double *__restrict__ mom, T *__restrict__ out, StepConsts c) {
  constexpr int S = Sets<MODEL>::S;
  __shared__ T rows_lds[kRowsTileRows][2][64];
  const int tile = xcd_tile(blockIdx.x, ntx * nty);
  if (tile >= ntx * nty) return;
  const int tx = tile % ntx, ty = tile / ntx;
  const int lane = threadIdx.x;
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.y);
  const int iy = ty * kRowsTileRows + wv;
  if (iy >= c.ny) return;  // whole wavefront; nothing below waits for others
  T lam[S][25];
  rows_stream<T, TAPS, S, sizeof(T) == 4 ? 2 : 4>(mu, xrel, xw, xwin, ysrc, yw, TX, ntx, tx, iy,
                                                  lane, c, &rows_lds[wv][0][0], lam);
  const int ix = tx * TX + lane;
  if (ix < c.nx && lane < TX) {
    const long long v = (long long)iy * c.nx + ix;
    if (mom)
      collision_adjoint_store<T, MODEL>(lam, mom, c, out, v);
    else
      store_sets<T, S>(lam, c, out, v);
  }
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
namespace {

constexpr int kMaxTaps = 12;

// f.template operator()<T, MODEL>() for the runtime population type and model.
template <class F>
hipError_t dispatch_model(int fp32, int model, F &&f) {
  auto by_model = [&]<typename T>() -> hipError_t {
    switch (model) {
      case kIsothermal: return f.template operator()<T, kIsothermal>();
      case kMonatomic: return f.template operator()<T, kMonatomic>();
      case kPolyatomic: return f.template operator()<T, kPolyatomic>();
    }
    return hipErrorInvalidValue;
  };
  return fp32 ? by_model.template operator()<float>() : by_model.template operator()<double>();
}

// f.template operator()<T, MODEL, TAPS>() for 2 <= taps <= kMaxTaps.
template <class F>
hipError_t dispatch_taps(int fp32, int model, int taps, F &&f) {
  return dispatch_model(fp32, model, [&]<typename T, int MODEL>() -> hipError_t {
    switch (taps) {
      case 2: return f.template operator()<T, MODEL, 2>();
      case 3: return f.template operator()<T, MODEL, 3>();
      case 4: return f.template operator()<T, MODEL, 4>();
      case 5: return f.template operator()<T, MODEL, 5>();
      case 6: return f.template operator()<T, MODEL, 6>();
      case 7: return f.template operator()<T, MODEL, 7>();
      case 8: return f.template operator()<T, MODEL, 8>();
      case 9: return f.template operator()<T, MODEL, 9>();
      case 10: return f.template operator()<T, MODEL, 10>();
      case 11: return f.template operator()<T, MODEL, 11>();
      case 12: return f.template operator()<T, MODEL, 12>();
    }
    return hipErrorInvalidValue;
  });
}

}  // namespace

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
  return dispatch_model(fp32, model, [&]<typename T, int MODEL>() -> hipError_t {
    k_adjoint_collide<T, MODEL><<<blocks, 256, 0, s>>>(static_cast<const T *>(lam), mom,
                                                       static_cast<T *>(mu), c);
    return hipGetLastError();
  });
}

hipError_t launch_adjoint_step(int fp32, int model, int kind, const StepConsts &c,
                               const DevTables &t, const void *mu, const double *mom_prev,
                               void *out, hipStream_t s) {
  if (t.taps < 2 || t.taps > kMaxTaps) return hipErrorInvalidValue;
  return dispatch_taps(fp32, model, t.taps, [&]<typename T, int MODEL, int TAPS>() -> hipError_t {
    const T *in = static_cast<const T *>(mu);
    T *o = static_cast<T *>(out);
    constexpr int S = Sets<MODEL>::S;
    if (kind == kAdjointRows) {
      if (t.rows_tx < kRowsMinCols || t.rows_tx > 64 || !t.rows_xrel || !t.rows_xwin ||
          !(t.ident_y & t.ident_x & 1))
        return hipErrorInvalidValue;
      const int ntx = (c.nx + t.rows_tx - 1) / t.rows_tx;
      const int nty = (c.ny + kRowsTileRows - 1) / kRowsTileRows;
      const int grid = ((ntx * nty + 7) / 8) * 8;
      k_adjoint_step_rows<T, MODEL, TAPS><<<grid, dim3(64, kRowsTileRows), 0, s>>>(
          in, t.rows_xrel, static_cast<const T *>(t.xw), t.rows_xwin, t.ysrc,
          static_cast<const T *>(t.yw), t.rows_tx, ntx, nty, mom_prev, o, c);
      return hipGetLastError();
    }
    if (kind == kAdjointTiled) {
      constexpr int TY = kTileRowsTY;
      const int ntx = (c.nx + 63) / 64, nty = (c.ny + TY - 1) / TY;
      const int grid = ((ntx * nty + 7) / 8) * 8;
      const int W = t.win_rows;
      const int halo = tiled_halo(t.win_cols, c.nx, c.ny);
      if (W > 3 * TY || halo == 0) return hipErrorInvalidValue;
      constexpr bool SEP = TAPS >= kSeparableTaps;
      auto go = [&]<int HALO, int R>() {
        // all five x-components per phase when the LDS buffers of the
        // tallest window this instantiation serves fit, else one
        constexpr int G =
            tiled_lds_bytes(sizeof(T), S, 5, R * TY, 64 + HALO, SEP) <= kTiledLdsBudget ? 5 : 1;
        const size_t lds = tiled_lds_bytes(sizeof(T), S, G, W, 64 + HALO, SEP);
        k_adjoint_step_tiled<T, MODEL, TAPS, HALO, G, R><<<grid, dim3(64, TY), lds, s>>>(
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
    k_adjoint_step_direct<T, MODEL, TAPS><<<grid, dim3(64, 4), 0, s>>>(
        in, t.xsrc, static_cast<const T *>(t.xw), t.ysrc, static_cast<const T *>(t.yw), mom_prev,
        o, c);
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
