// Interface between the three-dimensional C ABI (capi3d.cpp) and its HIP
// kernels (step3d.hip): isothermal D3Q125 on a tensor product of three axes.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace sllbm {

// Populations: 125 planes of N values, plane i = a + 5 b + 25 c (the 1-D
// components along x, y, z), node v = (iz ny + iy) nx + ix.
constexpr int kQ3 = 125;

struct Consts3 {
  int nx, ny, nz, p;
  long long n;       // nx ny nz
  double omega;      // 1 / tau
  double xi[5];      // 1-D abscissae
  double w[5];       // 1-D weights
  double hk[5][5];   // He_k(xi_a) / k!
};

// Per-axis departure tables, component-major: entry (comp, tap, j) at
// (comp * (p + 1) + tap) * n_axis + j; src holds node indices on that axis,
// w the Lagrange weights (float or double as the populations).
struct Tables3 {
  const int32_t *xsrc, *ysrc, *zsrc;
  const void *xw, *yw, *zw;
  const double *mx, *my, *mz;  // per-axis node masses (float64)
};

// Row segments of the step: the wavefronts of one (y, z) row own TX
// consecutive x-nodes (float64 splits the velocities over two to five
// wavefronts) and load, per 1-D x-component a, the 64 source columns
// starting at xwin[a * ntx + tx] (unwrapped; the kernel wraps or clamps);
// xrel[a * nx + ix] is node ix's first x-tap within that window.  tx == 0:
// unavailable.  Whole rows (full > 0) need no windows; with neither, the
// direct kernel runs.
// Whole-row mode: at most this many wavefronts along x (rows of up to 256
// nodes).
constexpr int kRows3MaxX = 4;
// ... and their tile order: blocks of this many rows along y and z.  On the
// 128^3-node grid (same box) against the plain (y, z) order, float32 /
// float64 ms per step: 16 x 8 0.862 / 1.686, 8 x 16 0.859 / 1.692, 32 x 4
// 0.866 / 1.750, plain 0.875 / 1.801; on another box 16 x 8 0.866 / 1.693,
// 8 x 8 0.871 / 1.689, 16 x 16 0.862 / 1.700, 4 x 16 0.881 / 1.696.
constexpr int kRows3BlockY = 16, kRows3BlockZ = 8;

struct Rows3 {
  int tx, ntx, nty, ntz;
  int perx;
  int full;  // > 0: wavefronts along x of the whole-row mode (rows of at most 64 kRows3MaxX nodes)
  const int32_t *xwin, *xrel;
};

// One step fin -> fout (both planar, 125 N values); flag |= 1 when a node's
// rho is not positive or a moment is not finite.  The step runs on row
// segments when r.tx > 0.
hipError_t launch_step3d(int fp32, const Consts3 &c, const Tables3 &t, const Rows3 &r,
                         const void *fin, void *fout, int *flag, hipStream_t s);
// f = f_eq(rho, u) from float64 device fields.
hipError_t launch_init3d(int fp32, const Consts3 &c, const double *rho, const double *ux,
                         const double *uy, const double *uz, void *f, hipStream_t s);
// rho, u per node (float64).
hipError_t launch_moments3d(int fp32, const Consts3 &c, const void *f, double *rho, double *ux,
                            double *uy, double *uz, hipStream_t s);
// sum_v M_v rho_v into out[0]; partial holds (n + 255) / 256 doubles.
hipError_t launch_mass3d(int fp32, const Consts3 &c, const Tables3 &t, const void *f,
                         double *partial, double *out, hipStream_t s);

}  // namespace sllbm
