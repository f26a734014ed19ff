// Isothermal D3Q125 stream + collide on a tensor product of three axes
// (HIP, gfx950): the two-dimensional step with a third axis (the paper's
// outlook, Sec. IV-V).  Velocity i = a + 5 b + 25 c has the 1-D components
// xi_a, xi_b, xi_c of the D1Q5 rule (Table I); its departure point
// x - dt xi_i is separable, so each axis has its own gather table and the
// interpolant of eq. (17) is the triple product of 1-D Lagrange weights.
#include "launch3d.hpp"
#include "step_common.hpp"
#include "tiled_common.hpp"

#include <utility>

namespace sllbm {
namespace {

// f.template operator()<k>() for k = 0 .. N-1 as straight-line code: every
// index is a compile-time constant, so arrays indexed by it stay in
// registers (a 125-iteration #pragma unroll loop with a large body exceeds
// the compiler's full-unroll threshold and leaves the index dynamic).
template <int N, class F>
__device__ __forceinline__ void static_for(F &&f) {
  [&]<int... K>(std::integer_sequence<int, K...>) {
    (f.template operator()<K>(), ...);
  }(std::make_integer_sequence<int, N>{});
}

// Calls fn(i, f_eq_i) for the 125 velocities: the 4th-order Hermite
// equilibrium at theta = 1 (Sec. II.A, eqs. (9)-(10) in three components),
// whose coefficients are the powers of u, factorised per axis:
//   f_eq_{a+5b+25c} = rho w_a w_b w_c sum_{k+l+m<=4} X_k[a] Y_l[b] Z_m[c],
//   X_k[a] = u_x^k He_k(xi_a)/k!  (Y, Z with u_y, u_z).
// Evaluated per (b, c) as sum_j YZ_j Xc_{4-j}[a] with YZ_j = sum_{l+m=j}
// Y_l Z_m and the running sums Xc_n[a] = sum_{k<=n} X_k[a].  The (b, c)
// loops stay rolled: unrolled, the relaxation's 125 independent loads were
// all hoisted (255 registers, one wavefront per SIMD); ROLLED = false for
// values held in registers, which need compile-time velocity indices.
// The contribution of one (b, c) row: fn(a + 5 b + 25 c, f_eq) for a = 0..4.
template <class Fn>
__device__ __forceinline__ void eq3_row(int b, int cc, double rho, const double (&py)[5],
                                        const double (&pz)[5], const double (&xc)[5][5],
                                        const Consts3 &c, Fn &&fn) {
  double yz[5];
#pragma unroll
  for (int j = 0; j < 5; ++j) {
    double s = 0.0;
#pragma unroll
    for (int l = 0; l <= j; ++l) s = fma(c.hk[b][l] * py[l], c.hk[cc][j - l] * pz[j - l], s);
    yz[j] = s;
  }
  const double rbc = rho * c.w[b] * c.w[cc];
#pragma unroll
  for (int a = 0; a < 5; ++a) {
    double s = 0.0;
#pragma unroll
    for (int j = 0; j < 5; ++j) s = fma(yz[j], xc[a][4 - j], s);
    fn(a + 5 * b + 25 * cc, rbc * c.w[a] * s);
  }
}

template <bool ROLLED = true, class Fn>
__device__ __forceinline__ void for_each_eq3(double rho, double ux, double uy, double uz,
                                             const Consts3 &c, Fn &&fn) {
  const double px[5] = {1.0, ux, ux * ux, ux * ux * ux, (ux * ux) * (ux * ux)};
  const double py[5] = {1.0, uy, uy * uy, uy * uy * uy, (uy * uy) * (uy * uy)};
  const double pz[5] = {1.0, uz, uz * uz, uz * uz * uz, (uz * uz) * (uz * uz)};
  double xc[5][5];
#pragma unroll
  for (int a = 0; a < 5; ++a) {
    double s = 0.0;
#pragma unroll
    for (int k = 0; k < 5; ++k) {
      s = fma(c.hk[a][k], px[k], s);
      xc[a][k] = s;
    }
  }
  if constexpr (ROLLED) {
#pragma unroll 1
    for (int cc = 0; cc < 5; ++cc)
#pragma unroll 1
      for (int b = 0; b < 5; ++b) eq3_row(b, cc, rho, py, pz, xc, c, fn);
  } else {
    // one (b, c) row at a time: its inputs pass through an empty asm, so its
    // arithmetic is not hoisted above the previous row (all 25 rows' float64
    // terms evaluated up front took more registers than the 125 values)
    static_for<25>([&]<int g>() {
      double r = rho, vy = uy, vz = uz;
      asm volatile("" : "+v"(r), "+v"(vy), "+v"(vz));
      const double qy[5] = {1.0, vy, vy * vy, vy * vy * vy, (vy * vy) * (vy * vy)};
      const double qz[5] = {1.0, vz, vz * vz, vz * vz * vz, (vz * vz) * (vz * vz)};
      eq3_row(g % 5, g / 5, r, qy, qz, xc, c, fn);
      __builtin_amdgcn_sched_barrier(0);
    });
  }
}

// The unrolled (register) form of for_each_eq3 over rows G0 .. G0 + NG - 1
// (row g = b + 5 c), each row's inputs pinned by an empty asm (see there).
template <int G0, int NG, class Fn>
__device__ __forceinline__ void for_each_eq3_rows(double rho, double ux, double uy, double uz,
                                                  const Consts3 &c, Fn &&fn) {
  static_for<NG>([&]<int k>() {
    constexpr int g = G0 + k;
    double r = rho, vx = ux, vy = uy, vz = uz;
    asm volatile("" : "+v"(r), "+v"(vx), "+v"(vy), "+v"(vz));
    const double qx[5] = {1.0, vx, vx * vx, vx * vx * vx, (vx * vx) * (vx * vx)};
    const double qy[5] = {1.0, vy, vy * vy, vy * vy * vy, (vy * vy) * (vy * vy)};
    const double qz[5] = {1.0, vz, vz * vz, vz * vz * vz, (vz * vz) * (vz * vz)};
    double xr[5][5];
#pragma unroll
    for (int a = 0; a < 5; ++a) {
      double t = 0.0;
#pragma unroll
      for (int m = 0; m < 5; ++m) {
        t = fma(c.hk[a][m], qx[m], t);
        xr[a][m] = t;
      }
    }
    eq3_row(g % 5, g / 5, r, qy, qz, xr, c, fn);
    __builtin_amdgcn_sched_barrier(0);
  });
}

// Interpolated value of one plane at a lane's departure point: the (p+1)^2
// source rows (z tap l, y tap n; byte offsets so[l][n], wave-uniform) are
// each read as p+1 consecutive values from x0 (one wide load per row), or
// value by value at xs[m] where the x-stencil wraps around a periodic seam.
template <typename T, int P1, bool SEAM>
__device__ __forceinline__ T gather3(__amdgpu_buffer_rsrc_t rs, unsigned x0,
                                     const unsigned (&xs)[P1], const T (&wx)[P1],
                                     const unsigned (&so)[P1][P1], const T (&wy)[P1],
                                     const T (&wz)[P1]) {
  T acc = T(0);
#pragma unroll
  for (int l = 0; l < P1; ++l) {
    T accl = T(0);
#pragma unroll
    for (int n = 0; n < P1; ++n) {
      T v[P1];
      if constexpr (SEAM) {
#pragma unroll
        for (int m = 0; m < P1; ++m) v[m] = buffer_load<T>(rs, xs[m], so[l][n]);
      } else {
        buffer_load_run<T, P1>(rs, x0, so[l][n], v);
      }
      T row = T(0);
#pragma unroll
      for (int m = 0; m < P1; ++m) row = fma(wx[m], v[m], row);
      accl = fma(wy[n], row, accl);
    }
    acc = fma(wz[l], accl, acc);
  }
  return acc;
}

// Pass 1 of the step: stream every velocity into the node's own slots of
// fout and accumulate rho and j (float64) on the way.
template <typename T, int P, bool SEAM>
__device__ __forceinline__ void stream3(const T *__restrict__ fin, T *__restrict__ fout,
                                        const int32_t *__restrict__ ysrc,
                                        const T *__restrict__ yw,
                                        const int32_t *__restrict__ zsrc,
                                        const T *__restrict__ zw, const Tables3 &t,
                                        const Consts3 &c, int ix, int iy, int iz, long long v,
                                        const unsigned (&x0)[5], const T (&wx)[5][P + 1],
                                        double (&mom)[4]) {
  constexpr int P1 = P + 1;
  const long long N = c.n;
  const unsigned plane_bytes = unsigned(N * (long long)sizeof(T));
  const unsigned row_bytes = unsigned(c.nx) * unsigned(sizeof(T));
  const unsigned vo = unsigned(v) * unsigned(sizeof(T));
  double rho = 0.0, jx = 0.0, jy = 0.0, jz = 0.0;
#pragma unroll 1
  for (int cc = 0; cc < 5; ++cc) {
    int zs[P1];
    T wz[P1];
#pragma unroll
    for (int l = 0; l < P1; ++l) {
      zs[l] = zsrc[(cc * P1 + l) * c.nz + iz];
      wz[l] = zw[(cc * P1 + l) * c.nz + iz];
    }
#pragma unroll 1
    for (int b = 0; b < 5; ++b) {
      unsigned so[P1][P1];
      T wy[P1];
#pragma unroll
      for (int n = 0; n < P1; ++n) {
        const int ys = ysrc[(b * P1 + n) * c.ny + iy];
        wy[n] = yw[(b * P1 + n) * c.ny + iy];
#pragma unroll
        for (int l = 0; l < P1; ++l)
          so[l][n] = (unsigned(zs[l]) * unsigned(c.ny) + unsigned(ys)) * row_bytes;
      }
      double r_b = 0.0, jx_b = 0.0;
#pragma unroll
      for (int a = 0; a < 5; ++a) {
        const int i = a + 5 * b + 25 * cc;
        unsigned xs[P1] = {};
        if constexpr (SEAM) {
#pragma unroll
          for (int m = 0; m < P1; ++m)
            xs[m] = unsigned(t.xsrc[(a * P1 + m) * c.nx + ix]) * unsigned(sizeof(T));
        }
        const auto rs = make_rsrc(fin + (long long)i * N, plane_bytes);
        T val = gather3<T, P1, SEAM>(rs, x0[a], xs, wx[a], so, wy, wz);
        // keep the interpolation next to its loads
        asm volatile("" : "+v"(val));
        buffer_store<T>(val, make_rsrc(fout + (long long)i * N, plane_bytes), vo, 0);
        const double d = double(val);
        r_b += d;
        jx_b = fma(c.xi[a], d, jx_b);
      }
      rho += r_b;
      jx += jx_b;
      jy = fma(c.xi[b], r_b, jy);
      jz = fma(c.xi[cc], r_b, jz);
    }
  }
  mom[0] = rho;
  mom[1] = jx;
  mom[2] = jy;
  mom[3] = jz;
}

// The direct step, for grids the row kernels do not serve: rows longer than
// the whole-row mode takes (in float64 at p >= 3 fewer, at p = 4 none) with
// no segment of 32 or more x-nodes whose stencils fit 64 source columns, or
// whose 125 planes exceed 4 GiB.  One thread per node; a workgroup is 64 consecutive
// x-nodes of 4 rows (one wavefront per row), so each wavefront's y and z
// taps are uniform.  Pass 1 streams all 125 velocities into the node's own
// slots of fout (the values are not held in registers), pass 2 reads them
// back, relaxes toward f_eq of the streamed moments and overwrites them
// (the same thread, the same addresses).
// The y- and z-tables are restrict-qualified parameters, so their
// wave-uniform entries are scalar loads (through the Tables3 pointers they
// were vector loads, and every gather became a waterfall loop).
template <typename T, int P>
__global__ __launch_bounds__(256) void k_step3d(const T *__restrict__ fin, T *__restrict__ fout,
                                                const int32_t *__restrict__ ysrc,
                                                const T *__restrict__ yw,
                                                const int32_t *__restrict__ zsrc,
                                                const T *__restrict__ zw, Tables3 t, Consts3 c,
                                                int *__restrict__ flag) {
  constexpr int P1 = P + 1;
  const int ix = blockIdx.x * 64 + (threadIdx.x & 63);
  const int iy = __builtin_amdgcn_readfirstlane(int(blockIdx.y) * 4 + int(threadIdx.x >> 6));
  const int iz = blockIdx.z;
  if (iy >= c.ny || ix >= c.nx) return;
  const long long N = c.n;
  const long long v = ((long long)iz * c.ny + iy) * c.nx + ix;
  const T *xw = static_cast<const T *>(t.xw);
  unsigned x0[5];
  T wx[5][P1];
  bool seam = false;
#pragma unroll
  for (int a = 0; a < 5; ++a) {
    const int first = t.xsrc[(a * P1) * c.nx + ix];
    const int last = t.xsrc[(a * P1 + P) * c.nx + ix];
    x0[a] = unsigned(first) * unsigned(sizeof(T));
    seam |= last != first + P;  // the x-stencil wraps around a periodic seam
#pragma unroll
    for (int m = 0; m < P1; ++m) wx[a][m] = xw[(a * P1 + m) * c.nx + ix];
  }
  double mom[4];
  if (__builtin_amdgcn_ballot_w64(seam))
    stream3<T, P, true>(fin, fout, ysrc, yw, zsrc, zw, t, c, ix, iy, iz, v, x0, wx, mom);
  else
    stream3<T, P, false>(fin, fout, ysrc, yw, zsrc, zw, t, c, ix, iy, iz, v, x0, wx, mom);
  const double rho = mom[0], ux = mom[1] / rho, uy = mom[2] / rho, uz = mom[3] / rho;
  const bool ok = (rho > 0.0) && isfinite(rho) && isfinite(ux) && isfinite(uy) && isfinite(uz);
  if (!ok) atomicOr(flag, 1);
  const unsigned plane_bytes = unsigned(N * (long long)sizeof(T));
  const unsigned vo = unsigned(v) * unsigned(sizeof(T));
  const double om = c.omega;
  for_each_eq3(rho, ux, uy, uz, c, [&](int i, double feq) {
    const auto rs = make_rsrc(fout + (long long)i * N, plane_bytes);
    const double f = double(buffer_load<T>(rs, vo, 0));
    buffer_store<T>(T(f - om * (f - feq)), rs, vo, 0);
  });
}

// ---------------------------------------------------------------------------
// The step on row segments.  A wavefront owns TX consecutive x-nodes of
// one (y, z) row, so the y- and z-taps of every velocity are uniform over its
// lanes.  Per velocity i = a + 5 b + 25 c it loads the (p+1)^2 source rows
// (one value per lane: column xwin + lane of the window of component a),
// combines them with the z- and y-weights in registers, writes the one
// interpolated row to its LDS row and evaluates the x-factor from LDS with
// the lane's p+1 x-weights (eq. (17), z and y factors first).  The zero
// component of each axis departs from the node itself (the host checks that
// its tables are the identity): b = 0 or c = 0 loads one row along that
// axis, a = 0 loads the node's own column and needs no LDS.  The values
// stay in registers for the collision (float32: all 125 in one wavefront;
// float64: split over H wavefronts, below); loads run D velocities ahead.
// Float64 on the 128^3-node grid: 2.54 ms against 5.83 ms of the direct
// two-pass kernel, which rereads its own output for the collision.  Tiles
// (64 x RY x RZ nodes) go to the XCDs in contiguous ranges of the (x, y, z)
// order, so neighbouring rows share an L2.  Measured and not kept on the
// 128^3-node Taylor-Green grid (float32): a workgroup barrier every five
// velocities (+7 %), 4 x 2 or 2 x 2 rows per workgroup and a z-first tile
// order (+1 to +7 %).
// ---------------------------------------------------------------------------
__device__ __forceinline__ void wave_lds_sync3() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront", "local");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront", "local");
}

// A wave-uniform value of lane k (32-bit lanes; a double takes two reads).
template <typename T>
__device__ __forceinline__ T lane_value(T v, int k) {
  if constexpr (sizeof(T) == 4) {
    return __builtin_bit_cast(T, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v), k));
  } else {
    const unsigned long long u = __builtin_bit_cast(unsigned long long, v);
    const unsigned lo = unsigned(__builtin_amdgcn_readlane(int(unsigned(u)), k));
    const unsigned hi = unsigned(__builtin_amdgcn_readlane(int(unsigned(u >> 32)), k));
    return __builtin_bit_cast(T, (static_cast<unsigned long long>(hi) << 32) | lo);
  }
}

// First (b, c) row of part k of H: the 25 rows of five velocities split
// into H consecutive parts (H = 2: 13 + 12, H = 3: 9 + 8 + 8, H = 5: 5 each).
constexpr int rows3_part(int H, int k) { return (25 * k + H - 1) / H; }

// The y- and z-tables come as restrict-qualified parameters: read-only and
// unaliased, their wave-uniform entries are fetched with scalar loads (read
// through the Tables3 pointers, they were vector loads, and every buffer
// load whose row offset depended on them became a waterfall loop).
// Whole rows (FR; rows of at most 64 kRows3MaxX nodes): the RX wavefronts of
// a workgroup cover one (y, z) row, 64 x-nodes each, and load only their
// own nodes' columns; the interpolated rows go to one LDS row of the whole
// x-extent (a periodic row followed by a copy of its first columns) and
// each lane reads its x-taps there, from its first tap's column on, after
// a workgroup barrier.  No source column is loaded twice, and a row needs
// RX wavefronts instead of one per segment of at most 64 - p - 1 nodes
// (three for the 128 nodes of the 64^3-cell grid at p = 2, the last with 6
// nodes): float32 1.258 -> 0.888 ms, float64 2.515 -> 1.847 ms there (0.86
// and 1.70 ms with the block order of the rows).  Any
// x-stencil fits, so graded axes whose stencils spread beyond the segment
// windows run here too.
// H > 1 (float64, whose 125 values do not fit the registers of one
// wavefront): the velocities of a row segment are split over H wavefronts,
// each holding its part's values; the parts add their moment sums through
// LDS in a fixed order (every part gets the same totals) and relax their
// own velocities.
template <typename T, int P, int RY, int RZ, int D, int H, bool FR = false, int XM = kRows3MaxX,
          bool BIG = false>
__global__ __launch_bounds__(64 * (FR ? XM : RZ) * RY * H) void k_step3d_rows(
    const T *__restrict__ fin, T *__restrict__ fout, const int32_t *__restrict__ ysrc,
    const T *__restrict__ yw, const int32_t *__restrict__ zsrc, const T *__restrict__ zw,
    Tables3 t, Rows3 r, Consts3 c, int *__restrict__ flag) {
  static_assert(!FR || RZ == 1, "whole rows: rows along y");
  constexpr int P1 = P + 1;
  constexpr int NV = P1 * P1;  // most loads of one velocity
  constexpr unsigned E = sizeof(T);
  constexpr int ROW = FR ? 64 * XM + 8 : 64;  // LDS row length (XM: most wavefronts along x)
  __shared__ T lds[RY * RZ * H][2][ROW];
  const int ntx = FR ? 1 : r.ntx;
  const int ntiles = ntx * r.nty * r.ntz;
  const int tile = xcd_tile(int(blockIdx.x), ntiles);
  if (tile >= ntiles) return;  // the whole workgroup
  const int tx = tile % ntx, rest = tile / ntx;
  int ty = rest % r.nty, tz = rest / r.nty;
  if constexpr (FR) {
    // whole rows go to the XCDs in blocks of kRows3BlockY x kRows3BlockZ
    // rows (bands of kRows3BlockZ planes, blocks along y inside a band; the
    // last band and block of each band may be smaller), so the z-neighbours
    // that read the same source rows run at the same time on one L2
    constexpr int BY = kRows3BlockY, BZ = kRows3BlockZ;
    const int band = tile / (r.nty * BZ);
    const int t1 = tile - band * r.nty * BZ;
    const int hz = min(BZ, r.ntz - band * BZ);
    const int by = t1 / (BY * hz);
    const int w = t1 - by * BY * hz;
    const int wy = min(BY, r.nty - by * BY);
    ty = by * BY + w % wy;
    tz = band * BZ + w / wy;
  }
  const int lane = threadIdx.x & 63;
  const int wv = __builtin_amdgcn_readfirstlane(int(threadIdx.x >> 6));
  // whole rows: wavefront seg of RX covers x-nodes [64 seg, 64 seg + 64)
  const int RX = FR ? r.full : 1;
  const int h = wv % H;                      // part of the velocities
  const int seg = FR ? (wv / H) % RX : tx;   // segment along x
  const int rw = FR ? wv / (H * RX) : wv / H;  // row of the workgroup
  const int iy0 = ty * RY + rw % RY, iz0 = tz * RZ + rw / RY;
  // rows past the grid stream its last row and store nothing
  const bool row_ok = iy0 < c.ny && iz0 < c.nz;
  const int iy = min(iy0, c.ny - 1), iz = min(iz0, c.nz - 1);
  const int TX = FR ? 64 : r.tx;
  const int ix = seg * TX + lane;
  const bool store = row_ok && lane < TX && ix < c.nx;
  const int ixc = min(seg * TX + min(lane, TX - 1), c.nx - 1);
  const long long N = c.n;
  const unsigned plane_bytes = unsigned(N * E);
  const unsigned row_bytes = unsigned(c.nx) * E;
  const T *xw = static_cast<const T *>(t.xw);
  int xr0[5];
  T wx[5][P1];
  unsigned col_off[5];
#pragma unroll
  for (int a = 0; a < 5; ++a) {
#pragma unroll
    for (int m = 0; m < P1; ++m) wx[a][m] = xw[(a * P1 + m) * c.nx + ixc];
    if constexpr (FR) {
      // the first x-tap's column; the others follow it (the last one of a
      // periodic row wraps into the copy of its first columns)
      xr0[a] = t.xsrc[a * P1 * c.nx + ixc];
      col_off[a] = unsigned(ixc) * E;
    } else {
      xr0[a] = r.xrel[a * c.nx + ixc];
      col_off[a] = unsigned(wrap_or_clamp(r.xwin[a * r.ntx + tx] + lane, c.nx, r.perx)) * E;
    }
  }
  col_off[0] = unsigned(ixc) * E;  // a = 0: the node's own column
  // this row's y- and z-taps, one table entry per lane (lane k = comp (p+1)
  // + tap): each velocity takes its uniform entries with v_readlane, so no
  // scalar memory load is in flight when a wavefront waits for its LDS row
  // (one wait counter covers both)
  const int kk = lane < 5 * P1 ? lane : 0;
  const int ys_v = ysrc[kk * c.ny + iy];
  const T wy_v = yw[kk * c.ny + iy];
  const int zs_v = zsrc[kk * c.nz + iz];
  const T wz_v = zw[kk * c.nz + iz];
  auto ys_of = [&](int k) { return __builtin_amdgcn_readlane(ys_v, k); };
  auto zs_of = [&](int k) { return __builtin_amdgcn_readlane(zs_v, k); };
  auto wy_of = [&](int k) { return lane_value<T>(wy_v, k); };
  auto wz_of = [&](int k) { return lane_value<T>(wz_v, k); };
  T *lrow = &lds[rw * H + h][0][0];
  auto row_of = [&](int zs, int ys) { return (unsigned(zs) * unsigned(c.ny) + unsigned(ys)) * row_bytes; };
  T pre[D + 1][NV];
  // one resource per array, the plane a uniform offset (125 planes below
  // 4 GiB); BIG: one resource per plane (each plane stays below 4 GiB), for
  // grids beyond that (a few more scalar registers, which at p = 1 spill)
  const auto rin_all = make_rsrc(fin, BIG ? 0u : unsigned(kQ3) * plane_bytes);
  auto load = [&]<int q>(T(&dst)[NV]) {
    constexpr int a = q % 5, b = (q / 5) % 5, cc = q / 25;
    const auto rin = BIG ? make_rsrc(fin + (long long)q * N, plane_bytes) : rin_all;
    const unsigned po = BIG ? 0u : unsigned(q) * plane_bytes;
    if constexpr (b == 0 && cc == 0) {
      dst[0] = buffer_load<T>(rin, col_off[a], po + row_of(iz, iy));
    } else if constexpr (cc == 0) {
#pragma unroll
      for (int n = 0; n < P1; ++n)
        dst[n] = buffer_load<T>(rin, col_off[a], po + row_of(iz, ys_of(b * P1 + n)));
    } else if constexpr (b == 0) {
#pragma unroll
      for (int l = 0; l < P1; ++l)
        dst[l] = buffer_load<T>(rin, col_off[a], po + row_of(zs_of(cc * P1 + l), iy));
    } else {
#pragma unroll
      for (int l = 0; l < P1; ++l)
#pragma unroll
        for (int n = 0; n < P1; ++n)
          dst[l * P1 + n] = buffer_load<T>(rin, col_off[a],
                                           po + row_of(zs_of(cc * P1 + l), ys_of(b * P1 + n)));
    }
  };
  constexpr int QH = 5 * (H == 1 ? 25 : rows3_part(H, 1));  // values one wavefront holds
  T fs[QH];
  double rho = 0.0, jx = 0.0, jy = 0.0, jz = 0.0;
  // velocities [Q0, Q0 + NQ) of this wavefront
  auto stream = [&]<int Q0, int NQ>() {
    static_assert(Q0 % 5 == 0 && NQ % 5 == 0, "whole (b, c) rows of five velocities");
    static_for<(D < NQ ? D : NQ)>([&]<int k>() { load.template operator()<Q0 + k>(pre[k]); });
    static_for<NQ>([&]<int k>() {
      constexpr int q = Q0 + k;
      if constexpr (k + D < NQ) load.template operator()<q + D>(pre[(k + D) % (D + 1)]);
      constexpr int a = q % 5, b = (q / 5) % 5, cc = q / 25;
      const T(&v)[NV] = pre[k % (D + 1)];
      T y;
      if constexpr (b == 0 && cc == 0) {
        y = v[0];
      } else if constexpr (cc == 0) {
        y = T(0);
#pragma unroll
        for (int n = 0; n < P1; ++n) y = fma(wy_of(b * P1 + n), v[n], y);
      } else if constexpr (b == 0) {
        y = T(0);
#pragma unroll
        for (int l = 0; l < P1; ++l) y = fma(wz_of(cc * P1 + l), v[l], y);
      } else {
        y = T(0);
#pragma unroll
        for (int l = 0; l < P1; ++l) {
          T yl = T(0);
#pragma unroll
          for (int n = 0; n < P1; ++n) yl = fma(wy_of(b * P1 + n), v[l * P1 + n], yl);
          y = fma(wz_of(cc * P1 + l), yl, y);
        }
      }
      T acc = y;  // a = 0: loaded at the node's own column
      if constexpr (a != 0) {
        // the two LDS rows alternate over the velocities that use them (the
        // a = 0 ones do not): with whole rows a wavefront may write the next
        // row before the others have read the last, never the one before it
        // (they read that before the barrier it waited for)
        constexpr int slot = (4 * (k / 5) + a - 1) & 1;
        T *row = lrow + slot * ROW;
        if constexpr (FR) {
          if (ix < c.nx) row[ix] = y;
          if (r.perx && ix < P) row[c.nx + ix] = y;
          __syncthreads();
        } else {
          row[lane] = y;
          wave_lds_sync3();
        }
        acc = T(0);
#pragma unroll
        for (int m = 0; m < P1; ++m) acc = fma(wx[a][m], row[xr0[a] + m], acc);
      }
      asm volatile("" : "+v"(acc));  // keep the velocity's arithmetic in its place
      fs[k] = acc;
      // moments as the values arrive: each float64 conversion is used at
      // once (summed after the loop, the scheduler kept all of them live)
      const double d = double(acc);
      rho += d;
      jx = fma(c.xi[a], d, jx);
      jy = fma(c.xi[b], d, jy);
      jz = fma(c.xi[cc], d, jz);
      // one scheduling region per velocity: in a single region of all 125
      // the scheduler moved the moment sums behind the last load and kept
      // every value's float64 conversion live
      __builtin_amdgcn_sched_barrier(0);
    });
    if constexpr (FR) {
      // every wavefront of the workgroup passes the same number of barriers:
      // one per velocity with a != 0, as many as the largest part has
      constexpr int most = 4 * (H == 1 ? 25 : rows3_part(H, 1));
      static_for<most - 4 * (NQ / 5)>([&]<int>() { __syncthreads(); });
    }
  };
  // wave priority 2 while streaming, 0 for the float64 collision (as the 2-D
  // row step; float32 segments 1.284 -> 1.260 ms; whole rows without it 3 %
  // slower, with the loads issued at priority 3 unchanged)
  __builtin_amdgcn_s_setprio(2);
  static_for<H>([&]<int k>() {
    if (h == k)
      stream.template operator()<5 * rows3_part(H, k),
                                 5 * (rows3_part(H, k + 1) - rows3_part(H, k))>();
  });
  __builtin_amdgcn_s_setprio(0);
  if constexpr (H > 1) {
    // the parts' moment sums, added in a fixed order
    __shared__ double mom_part[RY * (FR ? XM : RZ)][H][4][64];
    const int mi = wv / H;  // the row segment
    mom_part[mi][h][0][lane] = rho;
    mom_part[mi][h][1][lane] = jx;
    mom_part[mi][h][2][lane] = jy;
    mom_part[mi][h][3][lane] = jz;
    __syncthreads();
    rho = jx = jy = jz = 0.0;
#pragma unroll
    for (int k = 0; k < H; ++k) {
      rho += mom_part[mi][k][0][lane];
      jx += mom_part[mi][k][1][lane];
      jy += mom_part[mi][k][2][lane];
      jz += mom_part[mi][k][3][lane];
    }
  }
  // stability flag, BGK toward the 4th-order equilibrium
  if (!store) return;
  const double ux = jx / rho, uy = jy / rho, uz = jz / rho;
  const bool ok = (rho > 0.0) && isfinite(rho) && isfinite(ux) && isfinite(uy) && isfinite(uz);
  if (!ok && h == 0) atomicOr(flag, 1);
  const unsigned vo = unsigned(((long long)iz * c.ny + iy) * c.nx + ix) * E;
  const double om = c.omega;
  const auto rout_all = make_rsrc(fout, BIG ? 0u : unsigned(kQ3) * plane_bytes);
  auto put = [&](int i, T v) {
    if constexpr (BIG)
      buffer_store<T>(v, make_rsrc(fout + (long long)i * N, plane_bytes), vo, 0);
    else
      buffer_store<T>(v, rout_all, vo, unsigned(i) * plane_bytes);
  };
  if constexpr (H == 1) {
    for_each_eq3<false>(rho, ux, uy, uz, c, [&](int i, double feq) {
      T x = fs[i];
      asm volatile("" : "+v"(x));  // not the conversion of the moment sums
      const double f = double(x);
      put(i, T(f - om * (f - feq)));
    });
    return;
  }
  static_for<H>([&]<int k>() {
    if (h == k) {
      constexpr int G0 = rows3_part(H, k);
      for_each_eq3_rows<G0, rows3_part(H, k + 1) - G0>(
          rho, ux, uy, uz, c, [&](int i, double feq) {
            T x = fs[i - 5 * G0];
            asm volatile("" : "+v"(x));  // not the conversion of the moment sums
            const double f = double(x);
            put(i, T(f - om * (f - feq)));
          });
    }
  });
}

template <typename T>
__global__ __launch_bounds__(256) void k_init3d(const double *__restrict__ rho,
                                                const double *__restrict__ ux,
                                                const double *__restrict__ uy,
                                                const double *__restrict__ uz, T *__restrict__ f,
                                                Consts3 c) {
  const long long v = (long long)blockIdx.x * 256 + threadIdx.x;
  if (v >= c.n) return;
  const long long N = c.n;
  for_each_eq3(rho[v], ux[v], uy[v], uz[v], c,
               [&](int i, double feq) { f[(long long)i * N + v] = T(feq); });
}

template <typename T>
__device__ __forceinline__ void node_moments3(const T *__restrict__ f, long long v,
                                              const Consts3 &c, double (&m)[4]) {
  const long long N = c.n;
  double rho = 0.0, jx = 0.0, jy = 0.0, jz = 0.0;
#pragma unroll 1
  for (int cc = 0; cc < 5; ++cc) {
#pragma unroll
    for (int b = 0; b < 5; ++b) {
      double r_b = 0.0, jx_b = 0.0;
#pragma unroll
      for (int a = 0; a < 5; ++a) {
        const double d = double(f[(long long)(a + 5 * b + 25 * cc) * N + v]);
        r_b += d;
        jx_b = fma(c.xi[a], d, jx_b);
      }
      rho += r_b;
      jx += jx_b;
      jy = fma(c.xi[b], r_b, jy);
      jz = fma(c.xi[cc], r_b, jz);
    }
  }
  m[0] = rho;
  m[1] = jx / rho;
  m[2] = jy / rho;
  m[3] = jz / rho;
}

template <typename T>
__global__ __launch_bounds__(256) void k_moments3d(const T *__restrict__ f,
                                                   double *__restrict__ rho,
                                                   double *__restrict__ ux,
                                                   double *__restrict__ uy,
                                                   double *__restrict__ uz, Consts3 c) {
  const long long v = (long long)blockIdx.x * 256 + threadIdx.x;
  if (v >= c.n) return;
  double m[4];
  node_moments3<T>(f, v, c, m);
  rho[v] = m[0];
  ux[v] = m[1];
  uy[v] = m[2];
  uz[v] = m[3];
}

// Per-block partial sums of M_v rho_v, M_v = mx[ix] my[iy] mz[iz].
template <typename T>
__global__ __launch_bounds__(256) void k_mass3d(const T *__restrict__ f, Tables3 t,
                                                double *__restrict__ partial, Consts3 c) {
  const long long v = (long long)blockIdx.x * 256 + threadIdx.x;
  double mass = 0.0;
  if (v < c.n) {
    const long long N = c.n;
    double rho = 0.0;
#pragma unroll 5
    for (int i = 0; i < kQ3; ++i) rho += double(f[(long long)i * N + v]);
    const long long row = v / c.nx;
    const int ix = int(v - row * c.nx);
    const int iy = int(row % c.ny), iz = int(row / c.ny);
    mass = t.mx[ix] * t.my[iy] * t.mz[iz] * rho;
  }
  const double tot = block_sum_256(mass);
  if (threadIdx.x == 0) partial[blockIdx.x] = tot;
}

// Sum of the partials in a fixed order (one block).
__global__ __launch_bounds__(256) void k_sum3d(const double *__restrict__ partial, long long n,
                                               double *__restrict__ out) {
  double s = 0.0;
  for (long long k = threadIdx.x; k < n; k += 256) s += partial[k];
  const double tot = block_sum_256(s);
  if (threadIdx.x == 0) out[0] = tot;
}

template <class F>
hipError_t dispatch3(int fp32, int p, F &&f) {
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

}  // namespace

// Row-segment shape of the step: workgroups of RY rows (of H wavefronts
// each), loads D velocities ahead.
constexpr int kRows3Y = 4;  // rows of a float32 workgroup
// rows of a whole-row workgroup (two: float32 0.895 against 0.888 ms)
constexpr int kRows3FullY = 1;
// velocities of loads in flight ahead: about 45 registers of prefetch
constexpr int rows3_lookahead(int p) { return p == 1 ? 6 : p == 2 ? 4 : p == 3 ? 2 : 1; }
// float64: two parts of the velocities for p <= 2 (two rows a workgroup),
// three for p = 3 and five for p = 4 (one row).  Measured at p = 2 on the
// 128^3-node grid: loads one velocity ahead 2.514 ms, two 2.540, three
// 2.555; one row a workgroup 2.550; five parts (three wavefronts per SIMD)
// 2.808.
constexpr int rows3_parts64(int p) { return p <= 2 ? 2 : p == 3 ? 3 : 5; }
constexpr int rows3_lookahead64(int p) { return p == 1 ? 4 : 1; }
// whole rows at p = 2, 128-node rows (the same box): float32 six velocities
// ahead 0.897 ms, five 0.901, four 0.907, three 0.908; float64 two 1.812,
// three 1.808, one 1.854, none 2.327
constexpr int rows3_lookahead_whole(int p) { return p == 2 ? 6 : rows3_lookahead(p); }
constexpr int rows3_lookahead64_whole(int p) { return p == 2 ? 2 : rows3_lookahead64(p); }

hipError_t launch_step3d(int fp32, const Consts3 &c, const Tables3 &t, const Rows3 &r,
                         const void *fin, void *fout, int *flag, hipStream_t s) {
  auto launch = [&]<typename T, int P, int RY, int D, int H, bool FR, int XM = kRows3MaxX,
                    bool BIG = false>(Rows3 rr) -> hipError_t {
    rr.nty = (c.ny + RY - 1) / RY;
    rr.ntz = c.nz;
    const long long ntiles = (long long)(FR ? 1 : rr.ntx) * rr.nty * rr.ntz;
    if (ntiles >= (1LL << 31) - 8) return hipErrorInvalidValue;
    const unsigned grid = unsigned((ntiles + 7) / 8 * 8);  // whole rounds of the 8 XCDs
    k_step3d_rows<T, P, RY, 1, D, H, FR, XM, BIG>
        <<<grid, 64 * RY * H * (FR ? rr.full : 1), 0, s>>>(
            static_cast<const T *>(fin), static_cast<T *>(fout), t.ysrc,
            static_cast<const T *>(t.yw), t.zsrc, static_cast<const T *>(t.zw), t, rr, c, flag);
    return hipGetLastError();
  };
  // the 125 planes beyond one 32-bit buffer range: whole rows only, with a
  // resource per plane
  const bool big = double(kQ3) * double(c.n) * (fp32 ? 4.0 : 8.0) >= 4294967296.0;
  // whole rows: float32, and float64 where a workgroup of its parts has at
  // most 8 wavefronts (256 registers per lane): two parts up to 256 nodes
  // (p <= 2), three up to 128 (p = 3)
  const bool whole = r.full > 0 && r.full <= kRows3MaxX &&
                     (fp32 || c.p <= 2 || (c.p == 3 && r.full <= 2));
  const bool segments = r.tx > 0 && !big;
  if (whole || segments) {
    auto pick = [&]<int P>() -> hipError_t {
      constexpr int H = rows3_parts64(P);
      if (whole) {
        auto rows = [&]<bool BIG>() -> hipError_t {
          if (fp32)
            return launch.template operator()<float, P, kRows3FullY, rows3_lookahead_whole(P), 1,
                                              true, kRows3MaxX, BIG>(r);
          if constexpr (H == 2)
            return launch.template operator()<double, P, kRows3FullY, rows3_lookahead64_whole(P), 2,
                                              true, kRows3MaxX, BIG>(r);
          if constexpr (H == 3)
            return launch.template operator()<double, P, kRows3FullY, rows3_lookahead64_whole(P), 3,
                                              true, 2, BIG>(r);
          return hipErrorInvalidValue;
        };
        return big ? rows.template operator()<true>() : rows.template operator()<false>();
      }
      if (fp32) return launch.template operator()<float, P, kRows3Y, rows3_lookahead(P), 1, false>(r);
      return launch.template operator()<double, P, H == 2 ? 2 : 1, rows3_lookahead64(P), H, false>(r);
    };
    switch (c.p) {
      case 1: return pick.template operator()<1>();
      case 2: return pick.template operator()<2>();
      case 3: return pick.template operator()<3>();
      case 4: return pick.template operator()<4>();
    }
    return hipErrorInvalidValue;
  }
  if (c.nz > 65535 || c.ny > 4 * 65535) return hipErrorInvalidValue;
  return dispatch3(fp32, c.p, [&]<typename T, int P>() -> hipError_t {
    const dim3 grid(unsigned((c.nx + 63) / 64), unsigned((c.ny + 3) / 4), unsigned(c.nz));
    k_step3d<T, P><<<grid, 256, 0, s>>>(static_cast<const T *>(fin), static_cast<T *>(fout), t.ysrc,
                                        static_cast<const T *>(t.yw), t.zsrc,
                                        static_cast<const T *>(t.zw), t, c, flag);
    return hipGetLastError();
  });
}

hipError_t launch_init3d(int fp32, const Consts3 &c, const double *rho, const double *ux,
                         const double *uy, const double *uz, void *f, hipStream_t s) {
  const unsigned blocks = unsigned((c.n + 255) / 256);
  if (fp32)
    k_init3d<float><<<blocks, 256, 0, s>>>(rho, ux, uy, uz, static_cast<float *>(f), c);
  else
    k_init3d<double><<<blocks, 256, 0, s>>>(rho, ux, uy, uz, static_cast<double *>(f), c);
  return hipGetLastError();
}

hipError_t launch_moments3d(int fp32, const Consts3 &c, const void *f, double *rho, double *ux,
                            double *uy, double *uz, hipStream_t s) {
  const unsigned blocks = unsigned((c.n + 255) / 256);
  if (fp32)
    k_moments3d<float><<<blocks, 256, 0, s>>>(static_cast<const float *>(f), rho, ux, uy, uz, c);
  else
    k_moments3d<double><<<blocks, 256, 0, s>>>(static_cast<const double *>(f), rho, ux, uy, uz,
                                               c);
  return hipGetLastError();
}

hipError_t launch_mass3d(int fp32, const Consts3 &c, const Tables3 &t, const void *f,
                         double *partial, double *out, hipStream_t s) {
  const long long blocks = (c.n + 255) / 256;
  if (fp32)
    k_mass3d<float><<<unsigned(blocks), 256, 0, s>>>(static_cast<const float *>(f), t, partial, c);
  else
    k_mass3d<double><<<unsigned(blocks), 256, 0, s>>>(static_cast<const double *>(f), t, partial,
                                                      c);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  k_sum3d<<<1, 256, 0, s>>>(partial, blocks, out);
  return hipGetLastError();
}

}  // namespace sllbm
