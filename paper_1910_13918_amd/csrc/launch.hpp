// Interface between the C-ABI host code and the HIP kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace sllbm {

// Storage orders of a population array of S sets of Q1^2 velocities over N
// nodes; value (s, i = a + Q1 b, v), v = iy nx + ix.  Each set occupies
// Q1^2 N consecutive values in both.
//   kPlanar (the order of the C ABI): plane s Q1^2 + i, i.e. s Q1^2 N + i N + v.
//   kGrouped (the order the row-segment kernel streams): the Q1 - 1 moving
//     x-components a = 1 .. Q1-1 of velocity row b sit together for each
//     node, followed by the Q1 planes of a = 0:
//       a >= 1:  s Q1^2 N + (b N + v)(Q1 - 1) + a - 1
//       a == 0:  s Q1^2 N + Q1 (Q1 - 1) N + b N + v
//     The values a row segment streams for one velocity row b then lie in
//     one contiguous stretch per source row instead of Q1 - 1 planes apart.
enum PopLayout { kPlanar = 0, kGrouped = 1 };

// Element index of (s, a, b, v) in `layout` (q1 velocities per axis).
__host__ __device__ inline long long pop_elem(int layout, int q1, int s, int a, int b,
                                              long long v, long long N) {
  const long long set = (long long)s * q1 * q1 * N;
  if (layout == kPlanar) return set + (long long)(a + q1 * b) * N + v;
  const int k = q1 - 1;
  return a == 0 ? set + (long long)q1 * k * N + (long long)b * N + v
                : set + ((long long)b * N + v) * k + (a - 1);
}

// First element and node stride of the values of (s, a, b): value at node v
// is base + v * stride.
__host__ __device__ inline long long pop_base(int layout, int q1, int s, int a, int b,
                                              long long N) {
  return pop_elem(layout, q1, s, a, b, 0, N);
}
__host__ __device__ constexpr int pop_stride(int layout, int q1, int a) {
  return layout == kGrouped && a != 0 ? q1 - 1 : 1;
}

// Per-step scalar constants, passed by value as kernel arguments.
struct StepConsts {
  int nx, ny;
  long long n;        // nx * ny
  int ncx, ncy, p;
  double omega;       // 1 / tau
  double omega_pr;    // 1 / tau_Pr, tau_Pr = (tau - 1/2)/Pr + 1/2 (= omega when Pr = 1)
  double gfac;        // 2 C_v - D  (g_eq = gfac * theta * f_eq)
  double inv_2cv;     // 1 / (2 C_v)  (theta from the energy moment)
  double xi[5];       // 1-D abscissae (the first q1 entries are used)
  double w[5];        // 1-D weights
  double hk[5][5];    // He_k(xi_a) / k!
  double whk[5][5];   // w_a He_k(xi_a) / k!
  double rn[5];       // reference support points r_0..r_p
  double lden[5];     // 1 / prod_{n != m} (r_m - r_n)
  int q1;             // 1-D velocities (5: D2Q25; 3: D2Q9, isothermal only)
  int bf16x;          // matrix-core x-pass with bfloat16 operands (the experiment)
  double cs, inv_cs;  // velocity-set scale: the kernels work in xi / cs, u / cs and T / cs^2
  int perx, pery;     // periodic axes
  int reverse;        // row-segment and records steps: visit the tiles / blocks in reverse order
  int layout;         // PopLayout of the populations the per-node kernels (init, moments,
                      // mass, adjoint seed, nu term) read or write
  double *mom_out;    // optional [K][n]: rho, u_x, u_y (and theta unless isothermal) of
                      // the streamed state
};

// Device-side departure data.  Per-axis tables are laid out [comp][m][node]
// so that neighbouring threads read neighbouring words.
struct DevTables {
  const int32_t *xsrc;  // [5][p+1][nx]
  const void *xw;       // [5][p+1][nx], population type
  const int32_t *ysrc;  // [5][p+1][ny]
  const void *yw;       // [5][p+1][ny]
  // departure records per (velocity, node), velocity-major: float32: {cell,
  // r, s} triples of 32-bit words in `rec`; float64: {r, s} pairs in `rec`
  // and the cells in `rec_cell`; cell = cx | cy << 16
  const int32_t *rec_cell;  // [25][n] (float64 populations)
  const void *rec;          // [25][n] triples (float32) or pairs (float64)
  const double *rnodes;     // p + 1 reference support points (records path)
  const double *mx;     // [nx] mass weights
  const double *my;     // [ny]
  const double *mnode;  // [n] node mass weights of a curvilinear mesh (else null)
  // tiled path: per-tile source windows (tiles of 64 columns by tile_rows rows)
  const int32_t *yrel;  // [5][p+1][ny]: source row relative to the tile's window
  const int32_t *ywin;  // [5][ntiles_y]: first (unwrapped) source row of the window
  const int32_t *xrel;  // [5][p+1][nx]: source column relative to the tile's window
  const int32_t *xwin;  // [5][ntiles_x]: first (unwrapped) source column of the window
  int tile_rows;        // target rows per tile
  int win_rows;         // source rows staged per tile (max over tiles)
  int win_cols;         // source columns staged per tile (max over tiles)
  int taps;             // table entries per node (p+1 forward, more when transposed)
  int mfma_ok;          // every 16-column block's x-stencils fit the matrix-core x-pass
  // row-segment path: segments of rows_tx columns whose x-stencils fit 64
  // consecutive source columns starting at rows_xwin[comp][segment]
  int rows_tx;                 // 0: no such segment width (path unavailable)
  const int32_t *rows_xrel;    // [5][p+1][nx], relative to the segment's window
  const int32_t *rows_xwin;    // [5][nsegments]
  int ident_x, ident_y;        // bit a (b): the x- (y-) table of component a (b) is the
                               // identity (the row-segment kernels need bit 0: xi_0 = 0)
  // adjoint on a curvilinear mesh: the transposed records gather, per
  // velocity i and source node j the entries csr_ptr[i (n+1) + j] ..
  // csr_ptr[i (n+1) + j + 1] - 1 of (target node csr_col, weight csr_w)
  const uint32_t *csr_ptr;     // [25][n + 1], offsets into csr_col / csr_w
  const int32_t *csr_col;
  const void *csr_w;           // population type
};

// Narrowest row segment of the row-segment path (narrower ones leave most
// lanes idle).
constexpr int kRowsMinCols = 32;

enum Path { kPathDirect = 1, kPathTiled = 2, kPathRecords = 3, kPathMfma = 4, kPathRows = 5 };

// dst = src in the other storage order (to_grouped: kPlanar -> kGrouped, else
// back); S sets, c.q1 velocities per axis, c.n nodes; dst != src.
hipError_t launch_relayout(int fp32, int sets, const StepConsts &c, const void *src, void *dst,
                          int to_grouped, hipStream_t s);

hipError_t launch_init_eq(int fp32, int model, const StepConsts &c, const double *rho,
                          const double *ux, const double *uy, const double *T, void *f,
                          hipStream_t s);

hipError_t launch_step(int fp32, int model, int path, const StepConsts &c, const DevTables &t,
                       const void *fin, void *fout, int *flag, hipStream_t s);
hipError_t launch_step_direct(int fp32, int model, const StepConsts &c, const DevTables &t,
                              const void *fin, void *fout, int *flag, hipStream_t s);
hipError_t launch_step_tiled(int fp32, int model, const StepConsts &c, const DevTables &t,
                             const void *fin, void *fout, int *flag, hipStream_t s);
hipError_t launch_step_records(int fp32, int model, const StepConsts &c, const DevTables &t,
                               const void *fin, void *fout, int *flag, hipStream_t s);
hipError_t launch_step_mfma(int fp32, int model, const StepConsts &c, const DevTables &t,
                            const void *fin, void *fout, int *flag, hipStream_t s);
hipError_t launch_step_rows(int fp32, int model, const StepConsts &c, const DevTables &t,
                            const void *fin, void *fout, int *flag, hipStream_t s);
// the same with the quasi-equilibrium (Pr != 1) collision; thermal models only
hipError_t launch_step_direct_pr(int fp32, int model, const StepConsts &c, const DevTables &t,
                                 const void *fin, void *fout, int *flag, hipStream_t s);
hipError_t launch_step_tiled_pr(int fp32, int model, const StepConsts &c, const DevTables &t,
                                const void *fin, void *fout, int *flag, hipStream_t s);
hipError_t launch_step_records_pr(int fp32, int model, const StepConsts &c, const DevTables &t,
                                  const void *fin, void *fout, int *flag, hipStream_t s);
hipError_t launch_step_mfma_pr(int fp32, int model, const StepConsts &c, const DevTables &t,
                               const void *fin, void *fout, int *flag, hipStream_t s);
hipError_t launch_step_rows_pr(int fp32, int model, const StepConsts &c, const DevTables &t,
                               const void *fin, void *fout, int *flag, hipStream_t s);

// Moments per node (any output pointer may be null) and per-block partial
// sums of M_v rho_v into `partial` (mass_blocks(c) entries).
int mass_blocks(const StepConsts &c);
hipError_t launch_moments(int fp32, int model, const StepConsts &c, const DevTables &t,
                          const void *f, double *rho, double *ux, double *uy, double *T,
                          double *partial, hipStream_t s);
hipError_t launch_sum(const double *partial, int n, double *out, hipStream_t s);
// acc += scale * sum lambda (F - F_eq(M)) (partial: mass_blocks doubles,
// scalar: one double of scratch)
hipError_t launch_nu_term(int fp32, int model, const StepConsts &c, const void *lam,
                          const void *f, const double *mom, double *partial, double *scalar,
                          double scale, double *acc, hipStream_t s);

// Fixed per-device scratch of kScratchDoubles float64 (kernels.hip) for the
// entry points that allocate nothing; *ptr receives its address on `device`,
// which must be the current device.  Shared by every call on that device.
constexpr int kScratchDoubles = 1 << 17;  // mass partials of up to 2^25 nodes
constexpr int kMaxDevices = 64;
hipError_t scratch_buffer(int device, double **ptr);

// Record slots 4 + 3 s .. 6 + 3 s of a Pr != 1 step (thermal models, D2Q25,
// omega != 1): each set's centred second moments of the streamed state,
// recovered from the post-collision state f (order c.layout) and the step's
// recorded rho, u, theta in mom ([K][n]).
hipError_t launch_record_m2(int fp32, int model, const StepConsts &c, const void *f, double *mom,
                            hipStream_t s);

// flag = 0 (a kernel, not a memset, so the call can live inside a captured graph)
hipError_t launch_clear_flag(int *flag, hipStream_t s);

// ---- adjoint of the step (adjoint.hip), every model ----
// lam = d L / d F from d L / d (rho, u_x, u_y, theta) of the current populations
// (g_th may be null: no temperature term)
hipError_t launch_adjoint_seed(int fp32, int model, const StepConsts &c, const void *f,
                               const double *g_rho, const double *g_ux, const double *g_uy,
                               const double *g_th, void *lam, hipStream_t s);
// mu = J_C(M)^T lam, node by node (M: [K][n] moments of the streamed state,
// K = 3 isothermal, 4 with theta, and with Pr != 1 another 3 per set: the
// centred second moments of f (and g))
hipError_t launch_adjoint_collide(int fp32, int model, const StepConsts &c, const void *lam,
                                  const double *mom, void *mu, hipStream_t s);
// out = S^T mu (transposed tables t), then J_C(M_prev)^T when mom_prev is given
// (Pr = 1 only: with Pr != 1 the host applies J_C^T through launch_adjoint_collide);
// kind: the gather (direct, tiled windows, row segments, or the transposed
// records of a curvilinear mesh)
enum AdjointKind { kAdjointDirect = 0, kAdjointTiled = 1, kAdjointRows = 2, kAdjointCsr = 3 };
hipError_t launch_adjoint_step(int fp32, int model, int kind, const StepConsts &c,
                               const DevTables &t, const void *mu, const double *mom_prev,
                               void *out, hipStream_t s);
// gradients of sum_i lam_i f_eq_i (+ g_eq_i) with respect to rho0, u0 and theta0
hipError_t launch_eq_init_vjp(int fp32, int model, const StepConsts &c, const void *lam,
                              const double *rho0, const double *ux0, const double *uy0,
                              const double *th0, double *g_rho, double *g_ux, double *g_uy,
                              double *g_th, hipStream_t s);

}  // namespace sllbm
