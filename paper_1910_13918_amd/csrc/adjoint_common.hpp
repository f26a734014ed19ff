// Device helpers of the adjoint step (the transposed collision Jacobian and
// its Hermite projections) and the model / tap-count dispatchers, shared by
// adjoint.hip and adjoint_rows.hip.
#pragma once

#include <hip/hip_runtime.h>

#include "launch.hpp"
#include "step_common.hpp"

namespace sllbm {

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

// Transpose of the quasi-equilibrium term of the Pr != 1 collision.  The
// term added to set s is kappa f*_i(Q^s) with kappa = 1/tau - 1/tau_Pr,
// f*_i = sum_k C_ik Q^s_k, C_ik = w_a w_b He_k(xi_a)/k! He_(3-k)(xi_b)/(3-k)!
// (the form relax_each evaluates) and Q^s_k = sum_j s_j c_x^k c_y^(3-k) the
// centred third moments of set s about u = u(f) (c = xi - u).  With
// L^s_k = sum_i lam^s_i C_ik:
//   d/ds_j (direct):  kappa sum_k L^s_k c_x,j^k c_y,j^(3-k)          (every set);
//   through u (f only, du/df_j = c_j / rho):
//     kappa / rho (c_x,j sum_s,k L^s_k dQ^s_k/du_x + c_y,j sum_s,k L^s_k dQ^s_k/du_y),
//   dQ_k/du_x = -k M_(k-1,3-k), dQ_k/du_y = -(3-k) M_(k,2-k), M the centred
//   second moments the forward step recorded (mom slots 4 + 3 s ...).
// Returns L (per set) and the two u-coefficients ax, ay.
template <typename T, int S>
__device__ __forceinline__ void quasi_equilibrium_adjoint(const T (&lam)[S][25],
                                                          const double *__restrict__ mom,
                                                          const StepConsts &c, long long v,
                                                          double (&L)[S][4], double &ax,
                                                          double &ay) {
  const double kq = c.omega - c.omega_pr;
  const double rho = mom[v];
  ax = 0.0;
  ay = 0.0;
#pragma unroll
  for (int s = 0; s < S; ++s) {
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      // sum_b w_b He_(3-k)(xi_b)/(3-k)! sum_a w_a He_k(xi_a)/k! lam_(a+5b)
      double t = 0.0;
#pragma unroll
      for (int b = 0; b < 5; ++b) {
        double r = 0.0;
#pragma unroll
        for (int a = 0; a < 5; ++a) r = fma(c.whk[a][k], double(lam[s][a + 5 * b]), r);
        t = fma(c.w[b] * c.hk[b][3 - k], r, t);
      }
      L[s][k] = t;
    }
    const double mxx = mom[(4 + 3 * s) * c.n + v], mxy = mom[(5 + 3 * s) * c.n + v],
                 myy = mom[(6 + 3 * s) * c.n + v];
    // sum_k L_k dQ_k/du_x and sum_k L_k dQ_k/du_y
    ax -= L[s][1] * myy + 2.0 * L[s][2] * mxy + 3.0 * L[s][3] * mxx;
    ay -= 3.0 * L[s][0] * myy + 2.0 * L[s][1] * mxy + L[s][2] * mxx;
  }
  ax *= kq / rho;
  ay *= kq / rho;
#pragma unroll
  for (int s = 0; s < S; ++s)
#pragma unroll
    for (int k = 0; k < 4; ++k) L[s][k] *= kq;
}

// mu = J_C(rho, u, theta)^T lam, stored at node v of an [S][25][n] array;
// PR: the Pr != 1 collision, whose quasi-equilibrium term also needs the
// recorded centred second moments.
template <typename T, int MODEL, bool PR = false>
__device__ __forceinline__ void collision_adjoint_store(const T (&lam)[Sets<MODEL>::S][25],
                                                        const double *__restrict__ mom,
                                                        const StepConsts &c, T *__restrict__ out,
                                                        long long v) {
  constexpr int S = Sets<MODEL>::S;
  const double ux = mom[c.n + v], uy = mom[2 * c.n + v];
  const double theta = MODEL == kIsothermal ? 1.0 : mom[3 * c.n + v];
  double P, Px, Py, Pt;
  equilibrium_adjoint<T, MODEL>(lam, ux, uy, theta, c, P, Px, Py, Pt);
  double L[S][4], ax = 0.0, ay = 0.0;
  if constexpr (PR) quasi_equilibrium_adjoint<T, S>(lam, mom, c, v, L, ax, ay);
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
      double mu = fma(1.0 - om, double(lam[0][i]), om * r);
      // c_x^k c_y^(3-k), k = 0..3
      double cq[4];
      if constexpr (PR) {
        cq[0] = dy * dy * dy;
        cq[1] = dx * dy * dy;
        cq[2] = dx * dx * dy;
        cq[3] = dx * dx * dx;
        double q = 0.0;
#pragma unroll
        for (int k = 0; k < 4; ++k) q = fma(L[0][k], cq[k], q);
        mu += q + fma(ax, dx, ay * dy);
      }
      buffer_store<T>(T(mu), make_rsrc(out + i * c.n, plane_bytes), voff, 0);
      if constexpr (S == 2) {
        double mg = fma(1.0 - om, double(lam[S - 1][i]), om * Pt * c.inv_2cv);
        if constexpr (PR) {
          double q = 0.0;
#pragma unroll
          for (int k = 0; k < 4; ++k) q = fma(L[S - 1][k], cq[k], q);
          mg += q;
        }
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


// ---------------------------------------------------------------------------
// dispatch
// ---------------------------------------------------------------------------

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


// S^T through LDS-staged windows (adjoint_tiled.hpp; T = float or double).
template <typename T>
hipError_t launch_adjoint_step_tiled_t(int model, const StepConsts &c, const DevTables &t,
                                       const void *mu, const double *mom_prev, void *out,
                                       hipStream_t s);

// S^T through row segments (adjoint_rows.hip).
hipError_t launch_adjoint_step_rows(int fp32, int model, const StepConsts &c, const DevTables &t,
                                    const void *mu, const double *mom_prev, void *out,
                                    hipStream_t s);

}  // namespace sllbm
