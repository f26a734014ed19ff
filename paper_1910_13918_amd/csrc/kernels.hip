// HIP kernels (gfx950) around the SLLBM step: initialisation, moments, the
// mass reduction, and the dispatch to the stream + collide kernels.
//
// Memory layout: populations are structure-of-arrays, S sets (S = 2: f then
// g) of 25 values per node, in one of the two storage orders of PopLayout
// (launch.hpp): planar [S][25][ny][nx], the order of the C ABI, or grouped,
// the order of the row-segment step.  The per-node kernels here take the
// order from StepConsts::layout.  Moments, temperature, equilibrium and
// relaxation are evaluated in float64 for both population types.
#include <hip/hip_runtime.h>

#include <mutex>

#include "launch.hpp"
#include "step_common.hpp"

namespace sllbm {

// ---------------------------------------------------------------------------
// fixed device scratch for callers that cannot allocate: per-block partial
// sums of the mass reduction (one float64 per 256 nodes, so 2^17 entries
// cover the library's largest grid of 2^25 nodes).  Every GPU the library
// runs on holds one copy for the life of the process.  In host code the
// array's name is not a device address: its address on each device comes
// from hipGetSymbolAddress, taken once per device with that device current.
// ---------------------------------------------------------------------------
static __device__ __align__(256) double scratch[kScratchDoubles];

hipError_t scratch_buffer(int device, double **ptr) {
  static std::mutex mu;
  static double *addr[kMaxDevices] = {};
  if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(mu);
  if (!addr[device]) {
    // the caller has made `device` current
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    addr[device] = static_cast<double *>(p);
  }
  *ptr = addr[device];
  return hipSuccess;
}

// ---------------------------------------------------------------------------
// initialisation: f = f_eq(rho, u, theta), g = g_eq
// ---------------------------------------------------------------------------
template <typename T, int MODEL, int Q1 = 5>
__global__ __launch_bounds__(256) void k_init_eq(const double *__restrict__ rho,
                                                 const double *__restrict__ ux,
                                                 const double *__restrict__ uy,
                                                 const double *__restrict__ temp,
                                                 T *__restrict__ f, StepConsts c) {
  const long long v = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= c.n) return;
  // normalised by the velocity-set scale: u / c_s, theta = T / c_s^2
  const double r = rho[v], u = ux[v] * c.inv_cs, w = uy[v] * c.inv_cs;
  const double th = (MODEL == kIsothermal) ? 1.0 : temp[v] * (c.inv_cs * c.inv_cs);
  const long long N = c.n;
  if (c.layout == kPlanar) {
    for_each_equilibrium<Q1>(r, u, w, th, c, [&](int i, double feq) {
      f[i * N + v] = T(feq);
      if (Sets<MODEL>::S == 2) f[(Q1 * Q1 + i) * N + v] = T(c.gfac * th * feq);
    });
    return;
  }
  // grouped order: each velocity row's moving components in one wide store
  constexpr int K = Q1 - 1, S = Sets<MODEL>::S;
  constexpr unsigned E = sizeof(T);
  const unsigned voff = unsigned(v) * E;
  T row[S][Q1];
  for_each_equilibrium<Q1>(r, u, w, th, c, [&](int i, double feq) {
    const int a = i % Q1, b = i / Q1;
    row[0][a] = T(feq);
    if (S == 2) row[S - 1][a] = T(c.gfac * th * feq);
    if (a == Q1 - 1) {
#pragma unroll
      for (int s = 0; s < S; ++s) {
        buffer_store_run<T, K>(
            &row[s][1], make_rsrc(f + pop_base(kGrouped, Q1, s, 1, b, N), unsigned(N) * K * E),
            voff * K, 0);
        buffer_store<T>(row[s][0],
                        make_rsrc(f + pop_base(kGrouped, Q1, s, 0, b, N), unsigned(N) * E), voff,
                        0);
      }
    }
  });
}

// ---------------------------------------------------------------------------
// storage order change (PopLayout), one thread per node and set
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(256) void k_relayout(const T *__restrict__ src, T *__restrict__ dst,
                                                  int sets, int q1, int from, int to,
                                                  long long N) {
  const long long v = (long long)blockIdx.x * 256 + threadIdx.x;
  if (v >= N) return;
  const int s = blockIdx.y;
  if (s >= sets) return;
  for (int b = 0; b < q1; ++b)
    for (int a = 0; a < q1; ++a)
      dst[pop_elem(to, q1, s, a, b, v, N)] = src[pop_elem(from, q1, s, a, b, v, N)];
}

// ---------------------------------------------------------------------------
// moments and mass
// ---------------------------------------------------------------------------
template <typename T, int MODEL, int Q1 = 5>
__global__ __launch_bounds__(256) void k_moments(const T *__restrict__ f, const double *__restrict__ mx,
                                                 const double *__restrict__ my,
                                                 const double *__restrict__ mnode,
                                                 double *__restrict__ rho_o, double *__restrict__ ux_o,
                                                 double *__restrict__ uy_o, double *__restrict__ T_o,
                                                 double *__restrict__ partial, StepConsts c) {
  constexpr int S = Sets<MODEL>::S;
  constexpr int Q = Q1 * Q1;
  const long long v = (long long)blockIdx.x * 256 + threadIdx.x;
  double mass = 0.0;
  if (v < c.n) {
    const long long N = c.n;
    double m[4];
    T fs[S][Q];
#pragma unroll
    for (int s = 0; s < S; ++s)
#pragma unroll
      for (int i = 0; i < Q; ++i) fs[s][i] = f[pop_elem(c.layout, Q1, s, i % Q1, i / Q1, v, N)];
    node_moments<T, MODEL, Q1>(fs, c, m);
    // physical units: u = c_s u_hat, T = c_s^2 theta
    if (rho_o) rho_o[v] = m[0];
    if (ux_o) ux_o[v] = m[1] * c.cs;
    if (uy_o) uy_o[v] = m[2] * c.cs;
    if (T_o) T_o[v] = m[3] * (c.cs * c.cs);
    // 32-bit division (nodes < 2^31): the 64-bit form dominated these kernels
    const unsigned vv = unsigned(v), nx = unsigned(c.nx);
    const int ix = int(vv % nx), iy = int(vv / nx);
    mass = (mnode ? mnode[v] : mx[ix] * my[iy]) * m[0];
  }
  const double tot = block_sum_256(mass);
  if (threadIdx.x == 0) partial[blockIdx.x] = tot;
}

// Mass only: per-block partial sums of M_v rho_v, reading the f planes alone
// (rho = sum f; the same summation order as node_moments).
template <typename T, int Q1 = 5>
__global__ __launch_bounds__(256) void k_mass(const T *__restrict__ f,
                                              const double *__restrict__ mx,
                                              const double *__restrict__ my,
                                              const double *__restrict__ mnode,
                                              double *__restrict__ partial, StepConsts c) {
  const long long v = (long long)blockIdx.x * 256 + threadIdx.x;
  double mass = 0.0;
  if (v < c.n) {
    const long long N = c.n;
    T fs[Q1 * Q1];
#pragma unroll
    for (int i = 0; i < Q1 * Q1; ++i) fs[i] = f[pop_elem(c.layout, Q1, 0, i % Q1, i / Q1, v, N)];
    double rho = 0.0;
#pragma unroll
    for (int b = 0; b < Q1; ++b) {
      double r_b = 0.0;
#pragma unroll
      for (int a = 0; a < Q1; ++a) r_b += double(fs[a + Q1 * b]);
      rho += r_b;
    }
    // 32-bit division (nodes < 2^31): the 64-bit form dominated these kernels
    const unsigned vv = unsigned(v), nx = unsigned(c.nx);
    const int ix = int(vv % nx), iy = int(vv / nx);
    mass = (mnode ? mnode[v] : mx[ix] * my[iy]) * rho;
  }
  const double tot = block_sum_256(mass);
  if (threadIdx.x == 0) partial[blockIdx.x] = tot;
}

// ---------------------------------------------------------------------------
// centred second moments of a step's streamed state, for the record of a
// Pr != 1 step, from its post-collision state F+ (storage order c.layout)
// and the step's recorded rho, u, theta.  Per set, the collision moves the
// centred second moment M (about u) as M+ = (1 - omega) M + omega M_eq:
// f* is built from third-order Hermite terms, whose moments of degree <= 2
// vanish under the D1Q5 rule (exact to degree 9), and the equilibrium's
// centred second moment is rho theta I for f and (2 C_v - D) rho theta^2 I
// for g.  Hence M = (M+ - omega M_eq) / (1 - omega) (omega != 1, checked by
// the host); written to record slots 4 + 3 s .. 6 + 3 s: xx, xy, yy.
// ---------------------------------------------------------------------------
template <typename T, int MODEL>
__global__ __launch_bounds__(256) void k_record_m2(const T *__restrict__ f,
                                                   double *__restrict__ mom, StepConsts c) {
  constexpr int S = Sets<MODEL>::S;
  const long long v = (long long)blockIdx.x * 256 + threadIdx.x;
  if (v >= c.n) return;
  const long long N = c.n;
  const double rho = mom[v], ux = mom[N + v], uy = mom[2 * N + v], th = mom[3 * N + v];
  const double om = c.omega, inv = 1.0 / (1.0 - om);
#pragma unroll
  for (int s = 0; s < S; ++s) {
    double sxx = 0.0, sxy = 0.0, syy = 0.0;
#pragma unroll
    for (int b = 0; b < 5; ++b) {
      const double cy = c.xi[b] - uy;
      double s0 = 0.0, s1 = 0.0, s2 = 0.0;
#pragma unroll
      for (int a = 0; a < 5; ++a) {
        const double val = double(f[pop_elem(c.layout, 5, s, a, b, v, N)]);
        const double cx = c.xi[a] - ux;
        s0 += val;
        s1 = fma(cx, val, s1);
        s2 = fma(cx * cx, val, s2);
      }
      sxx += s2;
      sxy = fma(s1, cy, sxy);
      syy = fma(s0, cy * cy, syy);
    }
    const double iso = om * rho * th * (s == 0 ? 1.0 : c.gfac * th);
    mom[(4 + 3 * s) * N + v] = (sxx - iso) * inv;
    mom[(5 + 3 * s) * N + v] = sxy * inv;
    mom[(6 + 3 * s) * N + v] = (syy - iso) * inv;
  }
}

__global__ void k_clear_int(int *__restrict__ p) {
  if (threadIdx.x == 0) p[0] = 0;
}

__global__ __launch_bounds__(256) void k_sum(const double *__restrict__ partial, int n,
                                             double *__restrict__ out) {
  double s = 0.0;
  for (int k = threadIdx.x; k < n; k += 256) s += partial[k];
  const double tot = block_sum_256(s);
  if (threadIdx.x == 0) out[0] = tot;
}

// ---------------------------------------------------------------------------
// viscosity term of the adjoint: per block, sum over nodes, sets and
// velocities of lambda (F - F_eq(M)), F a post-collision state and M its
// moments [K][n] (rho, u_x, u_y, theta); scaled and added on the host's
// behalf by k_add_scaled.  lambda and F are caller arrays in the planar order.
// ---------------------------------------------------------------------------
template <typename T, int MODEL>
__global__ __launch_bounds__(256) void k_nu_term(const T *__restrict__ lam,
                                                 const T *__restrict__ f,
                                                 const double *__restrict__ mom,
                                                 double *__restrict__ partial, StepConsts c) {
  const long long v = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const long long N = c.n;
  double acc = 0.0;
  if (v < N) {  // no early return: every thread takes part in the block sum
    const double th = MODEL == kIsothermal ? 1.0 : mom[3 * N + v];
    for_each_equilibrium(mom[v], mom[N + v], mom[2 * N + v], th, c, [&](int i, double feq) {
      acc += double(lam[i * N + v]) * (double(f[i * N + v]) - feq);
      if (Sets<MODEL>::S == 2)
        acc += double(lam[(25 + i) * N + v]) * (double(f[(25 + i) * N + v]) - c.gfac * th * feq);
    });
  }
  const double tot = block_sum_256(acc);
  if (threadIdx.x == 0) partial[blockIdx.x] = tot;
}

__global__ void k_add_scaled(const double *__restrict__ s, double a, double *__restrict__ acc) {
  if (threadIdx.x == 0) acc[0] += a * s[0];
}

// ---------------------------------------------------------------------------
// dispatch
// ---------------------------------------------------------------------------
namespace {

template <typename T, int MODEL>
hipError_t nu_term_t(const StepConsts &c, const void *lam, const void *f, const double *mom,
                     double *partial, hipStream_t s) {
  k_nu_term<T, MODEL><<<mass_blocks(c), 256, 0, s>>>(
      static_cast<const T *>(lam), static_cast<const T *>(f), mom, partial, c);
  return hipGetLastError();
}

template <typename T, int MODEL>
hipError_t init_t(const StepConsts &c, const double *rho, const double *ux, const double *uy,
                  const double *temp, void *f, hipStream_t s) {
  const unsigned blocks = unsigned((c.n + 255) / 256);
  if (c.q1 == 3) {  // D2Q9 (isothermal only; the host refuses the rest)
    if constexpr (MODEL != kIsothermal) return hipErrorInvalidValue;
    else k_init_eq<T, MODEL, 3><<<blocks, 256, 0, s>>>(rho, ux, uy, temp, static_cast<T *>(f), c);
  } else {
    k_init_eq<T, MODEL><<<blocks, 256, 0, s>>>(rho, ux, uy, temp, static_cast<T *>(f), c);
  }
  return hipGetLastError();
}

template <typename T, int MODEL>
hipError_t moments_t(const StepConsts &c, const DevTables &t, const void *f, double *rho,
                     double *ux, double *uy, double *temp, double *partial, hipStream_t s) {
  if (!rho && !ux && !uy && !temp) {  // the mass alone needs the f planes only
    if (c.q1 == 3)
      k_mass<T, 3><<<mass_blocks(c), 256, 0, s>>>(static_cast<const T *>(f), t.mx, t.my, t.mnode,
                                                  partial, c);
    else
      k_mass<T><<<mass_blocks(c), 256, 0, s>>>(static_cast<const T *>(f), t.mx, t.my, t.mnode,
                                               partial, c);
    return hipGetLastError();
  }
  if (c.q1 == 3) {
    if constexpr (MODEL != kIsothermal) return hipErrorInvalidValue;
    else k_moments<T, MODEL, 3><<<mass_blocks(c), 256, 0, s>>>(
        static_cast<const T *>(f), t.mx, t.my, t.mnode, rho, ux, uy, temp, partial, c);
    return hipGetLastError();
  }
  k_moments<T, MODEL><<<mass_blocks(c), 256, 0, s>>>(static_cast<const T *>(f), t.mx, t.my,
                                                     t.mnode, rho, ux, uy, temp, partial, c);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_init_eq(int fp32, int model, const StepConsts &c, const double *rho,
                          const double *ux, const double *uy, const double *T, void *f,
                          hipStream_t s) {
  if (fp32) {
    if (model == kIsothermal) return init_t<float, kIsothermal>(c, rho, ux, uy, T, f, s);
    if (model == kMonatomic) return init_t<float, kMonatomic>(c, rho, ux, uy, T, f, s);
    return init_t<float, kPolyatomic>(c, rho, ux, uy, T, f, s);
  }
  if (model == kIsothermal) return init_t<double, kIsothermal>(c, rho, ux, uy, T, f, s);
  if (model == kMonatomic) return init_t<double, kMonatomic>(c, rho, ux, uy, T, f, s);
  return init_t<double, kPolyatomic>(c, rho, ux, uy, T, f, s);
}

hipError_t launch_relayout(int fp32, int sets, const StepConsts &c, const void *src, void *dst,
                          int to_grouped, hipStream_t s) {
  if (src == dst || sets < 1 || sets > 2) return hipErrorInvalidValue;
  const dim3 grid(unsigned((c.n + 255) / 256), unsigned(sets));
  const int from = to_grouped ? kPlanar : kGrouped, to = to_grouped ? kGrouped : kPlanar;
  if (fp32)
    k_relayout<float><<<grid, 256, 0, s>>>(static_cast<const float *>(src),
                                           static_cast<float *>(dst), sets, c.q1, from, to, c.n);
  else
    k_relayout<double><<<grid, 256, 0, s>>>(static_cast<const double *>(src),
                                            static_cast<double *>(dst), sets, c.q1, from, to, c.n);
  return hipGetLastError();
}

hipError_t launch_step(int fp32, int model, int path, const StepConsts &c, const DevTables &t,
                       const void *fin, void *fout, int *flag, hipStream_t s) {
  if (c.omega_pr != c.omega) {  // Pr != 1: quasi-equilibrium collision
    switch (path) {
      case kPathDirect: return launch_step_direct_pr(fp32, model, c, t, fin, fout, flag, s);
      case kPathTiled: return launch_step_tiled_pr(fp32, model, c, t, fin, fout, flag, s);
      case kPathRecords: return launch_step_records_pr(fp32, model, c, t, fin, fout, flag, s);
      case kPathMfma: return launch_step_mfma_pr(fp32, model, c, t, fin, fout, flag, s);
      case kPathRows: return launch_step_rows_pr(fp32, model, c, t, fin, fout, flag, s);
    }
    return hipErrorInvalidValue;
  }
  switch (path) {
    case kPathDirect: return launch_step_direct(fp32, model, c, t, fin, fout, flag, s);
    case kPathTiled: return launch_step_tiled(fp32, model, c, t, fin, fout, flag, s);
    case kPathRecords: return launch_step_records(fp32, model, c, t, fin, fout, flag, s);
    case kPathMfma: return launch_step_mfma(fp32, model, c, t, fin, fout, flag, s);
    case kPathRows: return launch_step_rows(fp32, model, c, t, fin, fout, flag, s);
  }
  return hipErrorInvalidValue;
}

int mass_blocks(const StepConsts &c) { return int((c.n + 255) / 256); }

hipError_t launch_moments(int fp32, int model, const StepConsts &c, const DevTables &t,
                          const void *f, double *rho, double *ux, double *uy, double *T,
                          double *partial, hipStream_t s) {
  if (fp32) {
    if (model == kIsothermal) return moments_t<float, kIsothermal>(c, t, f, rho, ux, uy, T, partial, s);
    if (model == kMonatomic) return moments_t<float, kMonatomic>(c, t, f, rho, ux, uy, T, partial, s);
    return moments_t<float, kPolyatomic>(c, t, f, rho, ux, uy, T, partial, s);
  }
  if (model == kIsothermal) return moments_t<double, kIsothermal>(c, t, f, rho, ux, uy, T, partial, s);
  if (model == kMonatomic) return moments_t<double, kMonatomic>(c, t, f, rho, ux, uy, T, partial, s);
  return moments_t<double, kPolyatomic>(c, t, f, rho, ux, uy, T, partial, s);
}

hipError_t launch_nu_term(int fp32, int model, const StepConsts &c, const void *lam,
                          const void *f, const double *mom, double *partial, double *scalar,
                          double scale, double *acc, hipStream_t s) {
  hipError_t e;
  if (fp32) {
    if (model == kIsothermal) e = nu_term_t<float, kIsothermal>(c, lam, f, mom, partial, s);
    else if (model == kMonatomic) e = nu_term_t<float, kMonatomic>(c, lam, f, mom, partial, s);
    else e = nu_term_t<float, kPolyatomic>(c, lam, f, mom, partial, s);
  } else {
    if (model == kIsothermal) e = nu_term_t<double, kIsothermal>(c, lam, f, mom, partial, s);
    else if (model == kMonatomic) e = nu_term_t<double, kMonatomic>(c, lam, f, mom, partial, s);
    else e = nu_term_t<double, kPolyatomic>(c, lam, f, mom, partial, s);
  }
  if (e != hipSuccess) return e;
  k_sum<<<1, 256, 0, s>>>(partial, mass_blocks(c), scalar);
  k_add_scaled<<<1, 64, 0, s>>>(scalar, scale, acc);
  return hipGetLastError();
}

hipError_t launch_record_m2(int fp32, int model, const StepConsts &c, const void *f, double *mom,
                            hipStream_t s) {
  const unsigned blocks = unsigned((c.n + 255) / 256);
  if (c.q1 != 5 || c.omega == 1.0) return hipErrorInvalidValue;
  auto go = [&]<typename T, int MODEL>() {
    k_record_m2<T, MODEL><<<blocks, 256, 0, s>>>(static_cast<const T *>(f), mom, c);
    return hipGetLastError();
  };
  if (model == kMonatomic)
    return fp32 ? go.template operator()<float, kMonatomic>()
                : go.template operator()<double, kMonatomic>();
  if (model == kPolyatomic)
    return fp32 ? go.template operator()<float, kPolyatomic>()
                : go.template operator()<double, kPolyatomic>();
  return hipErrorInvalidValue;
}

hipError_t launch_clear_flag(int *flag, hipStream_t s) {
  k_clear_int<<<1, 64, 0, s>>>(flag);
  return hipGetLastError();
}

hipError_t launch_sum(const double *partial, int n, double *out, hipStream_t s) {
  k_sum<<<1, 256, 0, s>>>(partial, n, out);
  return hipGetLastError();
}

}  // namespace sllbm
