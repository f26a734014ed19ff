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

// Raw buffer loads: a 128-bit resource (base, size in bytes) in scalar
// registers plus a 32-bit per-lane byte offset and a uniform byte offset.
// Offsets past the size read 0 instead of faulting.
constexpr int kBufferRsrcWord3 = 0x00020000;

__device__ __forceinline__ __amdgpu_buffer_rsrc_t make_rsrc(const void *base, unsigned bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(base), (short)0, (int)bytes,
                                           kBufferRsrcWord3);
}

template <typename T>
__device__ __forceinline__ T buffer_load(__amdgpu_buffer_rsrc_t r, unsigned voff, unsigned soff);

template <>
__device__ __forceinline__ float buffer_load<float>(__amdgpu_buffer_rsrc_t r, unsigned voff,
                                                    unsigned soff) {
  return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, voff, soff, 0));
}

template <>
__device__ __forceinline__ double buffer_load<double>(__amdgpu_buffer_rsrc_t r, unsigned voff,
                                                      unsigned soff) {
  return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, voff, soff, 0));
}

template <typename T>
__device__ __forceinline__ void buffer_store(T v, __amdgpu_buffer_rsrc_t r, unsigned voff,
                                             unsigned soff);

template <>
__device__ __forceinline__ void buffer_store<float>(float v, __amdgpu_buffer_rsrc_t r,
                                                    unsigned voff, unsigned soff) {
  __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, v), r, voff, soff, 0);
}

template <>
__device__ __forceinline__ void buffer_store<double>(double v, __amdgpu_buffer_rsrc_t r,
                                                     unsigned voff, unsigned soff) {
  using u2 = __attribute__((ext_vector_type(2))) unsigned;
  __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u2, v), r, voff, soff, 0);
}

// P1 consecutive values starting at byte offset voff + soff, with the widest
// buffer loads (up to 16 bytes per lane per instruction).
template <typename T, int P1>
__device__ __forceinline__ void buffer_load_run(__amdgpu_buffer_rsrc_t r, unsigned voff,
                                                unsigned soff, T (&v)[P1]) {
  using u4 = __attribute__((ext_vector_type(4))) unsigned;
  using u3 = __attribute__((ext_vector_type(3))) unsigned;
  using u2 = __attribute__((ext_vector_type(2))) unsigned;
  constexpr int W32 = P1 * int(sizeof(T)) / 4;  // 32-bit words to read
  unsigned w[W32];
  int k = 0;
#pragma unroll
  for (; k + 4 <= W32; k += 4) {
    const u4 q = __builtin_amdgcn_raw_buffer_load_b128(r, voff + 4 * k, soff, 0);
    w[k] = q[0]; w[k + 1] = q[1]; w[k + 2] = q[2]; w[k + 3] = q[3];
  }
  if constexpr (W32 % 4 == 3) {
    const u3 q = __builtin_amdgcn_raw_buffer_load_b96(r, voff + 4 * k, soff, 0);
    w[k] = q[0]; w[k + 1] = q[1]; w[k + 2] = q[2];
  } else if constexpr (W32 % 4 == 2) {
    const u2 q = __builtin_amdgcn_raw_buffer_load_b64(r, voff + 4 * k, soff, 0);
    w[k] = q[0]; w[k + 1] = q[1];
  } else if constexpr (W32 % 4 == 1) {
    w[k] = __builtin_amdgcn_raw_buffer_load_b32(r, voff + 4 * k, soff, 0);
  }
#pragma unroll
  for (int m = 0; m < P1; ++m) {
    if constexpr (sizeof(T) == 4) {
      v[m] = __builtin_bit_cast(T, w[m]);
    } else {
      const unsigned long long lo = w[2 * m], hi = w[2 * m + 1];
      v[m] = __builtin_bit_cast(T, lo | (hi << 32));
    }
  }
}

// Stores K consecutive values at byte offset voff + soff with the widest
// buffer stores (up to 16 bytes per lane per instruction).
template <typename T, int K>
__device__ __forceinline__ void buffer_store_run(const T *v, __amdgpu_buffer_rsrc_t r,
                                                 unsigned voff, unsigned soff) {
  using u4 = __attribute__((ext_vector_type(4))) unsigned;
  using u2 = __attribute__((ext_vector_type(2))) unsigned;
  constexpr int W32 = K * int(sizeof(T)) / 4;  // 32-bit words to write
  unsigned w[W32];
#pragma unroll
  for (int m = 0; m < K; ++m) {
    if constexpr (sizeof(T) == 4) {
      w[m] = __builtin_bit_cast(unsigned, v[m]);
    } else {
      const unsigned long long b = __builtin_bit_cast(unsigned long long, v[m]);
      w[2 * m] = unsigned(b);
      w[2 * m + 1] = unsigned(b >> 32);
    }
  }
  int k = 0;
#pragma unroll
  for (; k + 4 <= W32; k += 4)
    __builtin_amdgcn_raw_buffer_store_b128(u4{w[k], w[k + 1], w[k + 2], w[k + 3]}, r,
                                           voff + 4 * k, soff, 0);
  if constexpr (W32 % 4 == 2) {
    __builtin_amdgcn_raw_buffer_store_b64(u2{w[k], w[k + 1]}, r, voff + 4 * k, soff, 0);
  } else if constexpr (W32 % 4 == 1) {
    __builtin_amdgcn_raw_buffer_store_b32(w[k], r, voff + 4 * k, soff, 0);
  } else if constexpr (W32 % 4 == 3) {
    __builtin_amdgcn_raw_buffer_store_b64(u2{w[k], w[k + 1]}, r, voff + 4 * k, soff, 0);
    __builtin_amdgcn_raw_buffer_store_b32(w[k + 2], r, voff + 4 * k + 8, soff, 0);
  }
}

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
// Q1: velocities per axis of the tensor-product set (5: D2Q25; 3: D2Q9).
template <typename T, int MODEL, int Q1 = 5>
__device__ __forceinline__ void node_moments(const T (&fs)[Sets<MODEL>::S][Q1 * Q1],
                                             const StepConsts &c, double (&m)[4]) {
  double rho = 0.0, jx = 0.0, jy = 0.0, e = 0.0;
#pragma unroll
  for (int b = 0; b < Q1; ++b) {
    double r_b = 0.0, jx_b = 0.0, e_b = 0.0;
#pragma unroll
    for (int a = 0; a < Q1; ++a) {
      const double v = double(fs[0][a + Q1 * b]);
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
    for (int i = 0; i < Q1 * Q1; ++i) e += double(fs[Sets<MODEL>::S - 1][i]);
  }
  const double ux = jx / rho, uy = jy / rho;
  double theta = 1.0;
  if (MODEL != kIsothermal) theta = (e - rho * (ux * ux + uy * uy)) * c.inv_2cv / rho;
  m[0] = rho;
  m[1] = ux;
  m[2] = uy;
  m[3] = theta;
}

// Calls fn(i, f_eq_i) for the Q1^2 velocities (i = a + Q1 b).  Factorised form of the
// 4th-order Hermite equilibrium (Sec. II.A): with t = theta - 1 and
// A_0 = 1, A_1 = u, A_2 = u^2 + t, A_3 = u^3 + 3ut, A_4 = u^4 + 6u^2 t + 3t^2
// (the Hermite moments of a Gaussian of mean u and variance theta),
// f_eq_{a+5b} = rho w_a w_b sum_{k+m<=4} A_k(u_x) He_k(xi_a)/k! A_m(u_y) He_m(xi_b)/m!,
// which equals the full tensor contraction of eqs. (9)-(10).
// Evaluated per b as Z_k = A_k(u_x) sum_{m<=4-k} A_m(u_y) He_m(xi_b)/m! and
// f_eq_{a+5b} = rho w_b sum_k (w_a He_k(xi_a)/k!) Z_k, the bracket a kernel
// constant: five live values per b instead of 25 hoisted products.
template <int Q1 = 5, class Fn>
__device__ __forceinline__ void for_each_equilibrium(double rho, double ux, double uy,
                                                     double theta, const StepConsts &c, Fn &&fn) {
  const double t = theta - 1.0;
  const double ux2 = ux * ux, uy2 = uy * uy;
  const double Ax[5] = {1.0, ux, ux2 + t, ux * (ux2 + 3.0 * t),
                        ux2 * ux2 + 6.0 * ux2 * t + 3.0 * t * t};
  const double Ay[5] = {1.0, uy, uy2 + t, uy * (uy2 + 3.0 * t),
                        uy2 * uy2 + 6.0 * uy2 * t + 3.0 * t * t};
#pragma unroll
  for (int b = 0; b < Q1; ++b) {
    // Z[k] = A_k(u_x) sum_{m <= 4-k} A_m(u_y) He_m(xi_b)/m!
    double Z[5];
    double acc = 0.0;
#pragma unroll
    for (int j = 0; j < 5; ++j) {
      acc = fma(Ay[j], c.hk[b][j], acc);
      Z[4 - j] = Ax[4 - j] * acc;
    }
    const double rw = rho * c.w[b];
#pragma unroll
    for (int a = 0; a < Q1; ++a) {
      double s = c.whk[a][0] * Z[0];
#pragma unroll
      for (int k = 1; k < 5; ++k) s = fma(c.whk[a][k], Z[k], s);
      fn(a + Q1 * b, rw * s);
    }
  }
}

// Centred third moments of one population set about u (Sec. II.C):
// q[k] = sum_i f_i (xi_a - u_x)^k (xi_b - u_y)^(3-k), k = 0..3
// (Q_yyy, Q_xyy, Q_xxy, Q_xxx).
template <typename T>
__device__ __forceinline__ void centred_third_moments(const T (&f)[25], double ux, double uy,
                                                      const StepConsts &c, double (&q)[4]) {
  q[0] = q[1] = q[2] = q[3] = 0.0;
#pragma unroll
  for (int b = 0; b < 5; ++b) {
    double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
#pragma unroll
    for (int a = 0; a < 5; ++a) {
      T fr = f[a + 5 * b];
      asm volatile("" : "+v"(fr));  // convert again: the moments' doubles are not kept alive
      const double v = double(fr);
      const double cx = c.xi[a] - ux;
      s0 += v;
      s1 = fma(cx, v, s1);
      s2 = fma(cx * cx, v, s2);
      s3 = fma(cx * cx * cx, v, s3);
    }
    const double cy = c.xi[b] - uy;
    q[3] += s3;
    q[2] = fma(s2, cy, q[2]);
    q[1] = fma(s1, cy * cy, q[1]);
    q[0] = fma(s0, cy * cy * cy, q[0]);
  }
}

// Quasi-equilibrium population of velocity i = a + 5b from the row factors
// y[k] = kappa Q_{k,3-k} He_{3-k}(xi_b)/(3-k)!:  kappa f*_i with
// f*_i = (w_i / 3!) Q : H^(3)(xi_i).  Grouping the 8 index triples by their
// number k of x indices, H^(3) = He_k(xi_a) He_{3-k}(xi_b) with multiplicity
// 3!/(k!(3-k)!), so
// f*_i = w_b sum_k (w_a He_k(xi_a)/k!) (He_{3-k}(xi_b)/(3-k)!) Q_{k,3-k}.
__device__ __forceinline__ double quasi_equilibrium(const double (&y)[4], int i,
                                                    const StepConsts &c) {
  const int a = i % 5, b = i / 5;
  double s = c.whk[a][0] * y[0];
#pragma unroll
  for (int k = 1; k < 4; ++k) s = fma(c.whk[a][k], y[k], s);
  return c.w[b] * s;
}

// Relaxation of one node (m: its moments): calls sink(s, i, value) with the
// post-collision value of set s and velocity i.  With PR the heat flux
// relaxes at 1/tau_Pr instead of 1/tau (Sec. II.C-D, eq. (16)):
// f+ = f + (f_eq - f)/tau + (1/tau - 1/tau_Pr) f*, f* built from the
// non-equilibrium centred third moment of the set.  The equilibrium itself
// has none (the D1Q5 rule integrates degree 7 exactly and the 4th-order
// expansion carries the Gaussian's moments to order 4; the host refuses
// Pr != 1 with a rule that does not), so Q^neq is the moment of f.
// fs[s][i] is read before sink(s, i, .) is called and not after, so a sink
// may overwrite fs in place.
template <typename T, int MODEL, bool PR, int Q1 = 5, class Sink>
__device__ __forceinline__ void relax_each(const T (&fs)[Sets<MODEL>::S][Q1 * Q1],
                                           const double (&m)[4], const StepConsts &c,
                                           Sink &&sink) {
  static_assert(!PR || Q1 == 5, "the quasi-equilibrium term needs a set exact to degree 7");
  constexpr int S = Sets<MODEL>::S;
  const double om = c.omega;
  const double gf = c.gfac * m[3];
  double qf[4], qg[4];
  if constexpr (PR) {
    const double kq = c.omega - c.omega_pr;
    centred_third_moments<T>(fs[0], m[1], m[2], c, qf);
#pragma unroll
    for (int k = 0; k < 4; ++k) qf[k] *= kq;
    if (S == 2) {
      centred_third_moments<T>(fs[S - 1], m[1], m[2], c, qg);
#pragma unroll
      for (int k = 0; k < 4; ++k) qg[k] *= kq;
    }
  }
  double yf[4], yg[4];
  for_each_equilibrium<Q1>(m[0], m[1], m[2], m[3], c, [&](int i, double feq) {
    if (PR && i % 5 == 0) {  // row factors of velocity row b, made when the row starts
      const int b = i / 5;
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        yf[k] = qf[k] * c.hk[b][3 - k];
        asm volatile("" : "+v"(yf[k]));
        if (S == 2) {
          yg[k] = qg[k] * c.hk[b][3 - k];
          asm volatile("" : "+v"(yg[k]));
        }
      }
    }
    // convert again rather than keep the moments' 25 (50) doubles alive
    T fr = fs[0][i];
    asm volatile("" : "+v"(fr));
    const double f = double(fr);
    double fo = fma(om, feq - f, f);
    if (PR) fo += quasi_equilibrium(yf, i, c);
    sink(0, i, T(fo));
    if (S == 2) {
      T gr = fs[S - 1][i];
      asm volatile("" : "+v"(gr));
      const double g = double(gr);
      double go = fma(om, gf * feq - g, g);
      if (PR) go += quasi_equilibrium(yg, i, c);
      sink(1, i, T(go));
    }
  });
}

// Relaxation and store of one node at node index v, in storage order LAYOUT.
template <typename T, int MODEL, bool PR, int Q1 = 5, int LAYOUT = kPlanar>
__device__ __forceinline__ void relax_store(const T (&fs)[Sets<MODEL>::S][Q1 * Q1],
                                            const double (&m)[4], const StepConsts &c,
                                            T *__restrict__ fout, long long v) {
  const long long N = c.n;
  constexpr unsigned E = sizeof(T);
  // 32-bit lane offsets; the base of each velocity's values lives in the
  // (scalar) buffer resource
  const unsigned voff = unsigned(v) * E;
  if constexpr (LAYOUT == kPlanar) {
    relax_each<T, MODEL, PR, Q1>(fs, m, c, [&](int s, int i, T val) {
      const auto rs = make_rsrc(fout + pop_base(kPlanar, Q1, s, i % Q1, i / Q1, N), unsigned(N) * E);
      buffer_store<T>(val, rs, voff, 0);
    });
  } else {
    // a velocity row of each set is held until its last value is known, then
    // its Q1 - 1 moving components go out in one wide store per lane, so each
    // cache line is written whole by one instruction
    constexpr int K = Q1 - 1;
    T row[Sets<MODEL>::S][Q1];
    relax_each<T, MODEL, PR, Q1>(fs, m, c, [&](int s, int i, T val) {
      const int a = i % Q1, b = i / Q1;
      row[s][a] = val;
      if (a == Q1 - 1) {
        const auto rg = make_rsrc(fout + pop_base(kGrouped, Q1, s, 1, b, N), unsigned(N) * K * E);
        buffer_store_run<T, K>(&row[s][1], rg, voff * K, 0);
        const auto r0 = make_rsrc(fout + pop_base(kGrouped, Q1, s, 0, b, N), unsigned(N) * E);
        buffer_store<T>(row[s][0], r0, voff, 0);
      }
    });
  }
}

// Moments of one node's streamed populations; when `valid`, records them for
// the adjoint (if asked) and raises the stability flag on rho <= 0,
// theta <= 0 or a non-finite moment.
template <typename T, int MODEL, int Q1 = 5>
__device__ __forceinline__ void collide_moments(const T (&fs)[Sets<MODEL>::S][Q1 * Q1],
                                                const StepConsts &c, long long v, bool valid,
                                                int *__restrict__ flag, double (&m)[4]) {
  node_moments<T, MODEL, Q1>(fs, c, m);
  if (!valid) return;
  if (c.mom_out) {  // recorded for the adjoint (uniform branch)
    c.mom_out[v] = m[0];
    c.mom_out[c.n + v] = m[1];
    c.mom_out[2 * c.n + v] = m[2];
    if (MODEL != kIsothermal) c.mom_out[3 * c.n + v] = m[3];
  }
  const bool ok = (m[0] > 0.0) && (m[3] > 0.0) && isfinite(m[0]) && isfinite(m[1]) &&
                  isfinite(m[2]) && isfinite(m[3]);
  if (!ok) atomicOr(flag, 1);
}

// Moments, stability flag, equilibrium and relaxation of one node's
// streamed populations; stores the post-collision values at node v
// (Sec. II.D, eq. (16)):  f+ = f + (f_eq - f)/tau, g+ = g + (g_eq - g)/tau,
// g_eq = (2 C_v - D) theta f_eq, plus the quasi-equilibrium term when PR
// (Pr != 1).  PR is a kernel template parameter rather than a runtime
// branch: holding both variants in one kernel costs the Pr = 1 kernels
// registers and occupancy.
template <typename T, int MODEL, bool PR = false, int Q1 = 5, int LAYOUT = kPlanar>
__device__ __forceinline__ void collide_store(const T (&fs)[Sets<MODEL>::S][Q1 * Q1],
                                              const StepConsts &c, T *__restrict__ fout,
                                              long long v, int *__restrict__ flag) {
  double m[4];
  collide_moments<T, MODEL, Q1>(fs, c, v, true, flag, m);
  relax_store<T, MODEL, PR, Q1, LAYOUT>(fs, m, c, fout, v);
}

// Workgroup barrier that orders LDS only: unlike __syncthreads() it does not
// wait for outstanding global loads, so prefetches stay in flight across it.
__device__ __forceinline__ void lds_barrier() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
  __builtin_amdgcn_s_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
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

// Calls f.template operator()<T, P, MODEL>() for the runtime population type
// (float / double), order p and model; THERMAL_ONLY instantiates nothing for
// the isothermal model (which then gets hipErrorInvalidValue).
template <bool THERMAL_ONLY = false, class F>
hipError_t dispatch_step(int fp32, int p, int model, F &&f) {
  auto by_p = [&]<typename T, int MODEL>() -> hipError_t {
    switch (p) {
      case 1: return f.template operator()<T, 1, MODEL>();
      case 2: return f.template operator()<T, 2, MODEL>();
      case 3: return f.template operator()<T, 3, MODEL>();
      case 4: return f.template operator()<T, 4, MODEL>();
    }
    return hipErrorInvalidValue;
  };
  auto by_model = [&]<typename T>() -> hipError_t {
    switch (model) {
      case kIsothermal:
        if constexpr (THERMAL_ONLY) return hipErrorInvalidValue;
        else return by_p.template operator()<T, kIsothermal>();
      case kMonatomic: return by_p.template operator()<T, kMonatomic>();
      case kPolyatomic: return by_p.template operator()<T, kPolyatomic>();
    }
    return hipErrorInvalidValue;
  };
  return fp32 ? by_model.template operator()<float>() : by_model.template operator()<double>();
}

// The D2Q9 (three velocities per axis) variants: isothermal, Pr = 1 only
// (the set carries the Gaussian's moments to degree 5, too few for the
// energy equation); calls f.template operator()<T, P>().
template <class F>
hipError_t dispatch_q3(int fp32, int p, int model, F &&f) {
  if (model != kIsothermal) return hipErrorInvalidValue;
  auto by_p = [&]<typename T>() -> hipError_t {
    switch (p) {
      case 1: return f.template operator()<T, 1>();
      case 2: return f.template operator()<T, 2>();
      case 3: return f.template operator()<T, 3>();
      case 4: return f.template operator()<T, 4>();
    }
    return hipErrorInvalidValue;
  };
  return fp32 ? by_p.template operator()<float>() : by_p.template operator()<double>();
}

}  // namespace sllbm
