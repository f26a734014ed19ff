/*
 * sllbm.h -- C ABI of libsllbm, the MI355X (gfx950) semi-Lagrangian lattice
 * Boltzmann step of Wilde, Kraemer, Reith, Foysi, "Semi-Lagrangian lattice
 * Boltzmann method for compressible flows" (arXiv:1910.13918).
 *
 * One time step (sllbm_step) does, for every grid node x and each of the Q
 * discrete velocities xi_i:
 *   1. trace the characteristic back to x - dt xi_i, find the departure cell
 *      and evaluate the cell-local Lagrange interpolant of order p on
 *      Gauss-Lobatto-Chebyshev support points of the previous post-collision
 *      populations (Sec. II.E, eq. (17));
 *   2. moments rho, rho u, 2 rho E of the streamed populations (Sec. II,
 *      eqs. (3)-(5)) and the temperature theta;
 *   3. BGK relaxation toward the 4th-order Hermite equilibrium (Sec. II.A,
 *      eqs. (9)-(10)) with tau = nu/(c_s^2 dt) + 1/2 (Sec. II.D, eq. (16));
 *      the second population g relaxes toward g_eq = (2 C_v - D) theta f_eq
 *      (Sec. II.D, eq. (15)).
 * The collision acts on node values and the interpolant of the post-collision
 * field is what is streamed.  For Pr != 1 the collision adds the
 * quasi-equilibrium term of eq. (16), (1/tau - 1/tau_Pr) f*, with
 * f*_i = (w_i/3!) Q^neq : H^(3)(xi_i) built from the centred third moment
 * Q^neq = sum_i (f_i - f_eq_i)(xi_i - u)^3 of each population set and
 * tau_Pr = (tau - 1/2)/Pr + 1/2 (Sec. II.C-D), so that the heat flux relaxes
 * at 1/tau_Pr.  Code units: c_s = R = T0 = 1, D = 2.
 *
 * Conventions
 *   - Every function returns an sllbm_status; nothing throws or aborts across
 *     the ABI.  sllbm_last_error() returns the message of the last failure on
 *     that context (valid until the next call on it).
 *   - Set-up calls (velocity set, order, grid, physics, precision, path) only
 *     touch host memory and validate their arguments before anything else;
 *     they work without a GPU.  Device memory is allocated on first need
 *     (bind / init / set_populations / step).
 *   - Call order: create -> [set_velocity_set] -> set_order -> init_grid_* ->
 *     set_physics -> [bind_populations] -> init_macro | set_populations ->
 *     step / moments / mass / get_populations.  Changing the order, grid or
 *     physics after initialisation returns SLLBM_E_STATE.
 *   - Node arrays are node-major: element (iy, ix) at iy * nx + ix, float64.
 *   - Populations cross the boundary (get / set_populations, the adjoint's
 *     arrays) as structure-of-arrays [S][Q][ny][nx] of the population type
 *     (float64 for SLLBM_FP64, float32 for SLLBM_FP32), with S = 2 for the
 *     polyatomic model (f then g) and 1 otherwise, and i = a + q1 * b for
 *     the velocity (xi_a, xi_b) (g divided by cs^2 for a scaled velocity
 *     set, sllbm_set_velocity_set).  Inside the two state buffers (bound or
 *     the library's own) the order depends on the kernel family that runs:
 *     the row-segment step keeps the q1 - 1 values a = 1 .. q1-1 of each
 *     velocity row b together per node (then the planes of a = 0), the
 *     other gathers the order above; the library converts on a change of
 *     path.  Read and write the state through get / set_populations only.
 *   - Device pointers are HIP device addresses on the context's device.
 *     Kernels run asynchronously on the bound stream (default: the null
 *     stream); calls that return host data synchronise that stream.
 *   - One context per thread; contexts are independent.
 *   - The library never takes ownership of caller memory.
 *
 * The same step in three dimensions (D3Q125, isothermal) has a context of its
 * own, declared in sllbm3d.h; it shares these status codes and enums.
 */
#ifndef SLLBM_H
#define SLLBM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct sllbm_ctx sllbm_ctx;

typedef enum {
  SLLBM_OK = 0,
  SLLBM_E_ARG = -1,         /* invalid argument (range, NaN, null pointer, size) */
  SLLBM_E_STATE = -2,       /* call out of order */
  SLLBM_E_DEVICE = -3,      /* HIP runtime error (no device, launch failure, ...) */
  SLLBM_E_OOM = -4,         /* device allocation failed */
  SLLBM_E_UNSTABLE = -5,    /* stability flag raised: rho <= 0, theta <= 0 or non-finite */
  SLLBM_E_UNSUPPORTED = -6  /* valid but not implemented combination */
} sllbm_status;

typedef enum {
  SLLBM_FP64 = 0,  /* float64 populations, interpolation, moments, equilibrium */
  SLLBM_FP32 = 1,  /* float32 populations and interpolation; float64 moments,
                      temperature, equilibrium and relaxation */
  SLLBM_BF16X = 3  /* experiment: as SLLBM_FP32 (float32 populations in
                      memory, same layout), with the x-pass of the
                      interpolation (eq. (17)) on the matrix cores taking
                      bfloat16 Lagrange weights and bfloat16 staged values
                      (round to nearest even) with float32 accumulation
                      (v_mfma_f32_16x16x32_bf16); runs on SLLBM_PATH_MFMA
                      only (AUTO resolves to it; other paths and the adjoint
                      return SLLBM_E_UNSUPPORTED).  Its error is a measured
                      result, not a bound. */
} sllbm_precision;

typedef enum { SLLBM_PERIODIC = 0, SLLBM_ZERO_GRADIENT = 1 } sllbm_bc;

typedef enum { SLLBM_NODES_GLC = 0, SLLBM_NODES_EQUIDISTANT = 1 } sllbm_nodes;

typedef enum {
  SLLBM_ISOTHERMAL = 0, /* f only, theta = 1 (Sec. III.A) */
  SLLBM_MONATOMIC = 1,  /* f only, theta from the energy moment, gamma = (D+2)/D */
  SLLBM_POLYATOMIC = 2  /* f and g, gamma given (Sec. II.D) */
} sllbm_model;

typedef enum {
  SLLBM_PATH_AUTO = 0,    /* library choice (sllbm_resolved_path): ROWS for
                             row segments of >= 48 nodes (measured at least as
                             fast as TILED everywhere), else whichever of the
                             two fits, else DIRECT */
  SLLBM_PATH_DIRECT = 1,  /* one thread per node, (p+1)^2 gathers per velocity
                             through per-axis departure tables */
  SLLBM_PATH_TILED = 2,   /* raw source windows of each velocity staged in LDS
                             per tile of 64 x 4 nodes, interpolated from LDS */
  SLLBM_PATH_RECORDS = 3, /* per-(node, velocity) departure records (cell, r, s)
                             with weights evaluated in the kernel: the general
                             gather for grids that are not axis products */
  SLLBM_PATH_MFMA = 4,    /* as TILED, with the x-pass of the interpolation as
                             16 x 16 x 4 float32 matrix-core products (float32
                             populations, at most 16 population-set x window
                             rows, departures within one node spacing of their
                             cell; SLLBM_E_UNSUPPORTED otherwise); chosen by
                             AUTO only for SLLBM_BF16X, whose x-pass is one
                             16 x 16 x 32 bfloat16 product per block */
  SLLBM_PATH_ROWS = 5     /* one wavefront per row segment of up to 64 nodes:
                             the p+1 source rows of each velocity combined in
                             registers (y-factor), the x-factor from a per-
                             wavefront LDS row, no workgroup barrier (needs a
                             segment of >= 32 columns whose x-stencils fit 64
                             source columns and a first 1-D velocity of 0, as
                             in Table I; SLLBM_E_UNSUPPORTED otherwise) */
} sllbm_path;

/* ---- lifetime ------------------------------------------------------------ */

/* Create a context for HIP device `hip_device` (checked lazily, at the first
 * device call).  *out receives the context; on failure *out is NULL. */
int sllbm_create(sllbm_ctx **out, int hip_device, int precision);

/* Free the context's device tables and any buffers the library allocated.
 * Bound (caller-owned) buffers are not freed.  NULL is accepted. */
void sllbm_destroy(sllbm_ctx *ctx);

/* Message of the last failed call on ctx ("" if none).  Never NULL. */
const char *sllbm_last_error(const sllbm_ctx *ctx);

/* Run all later kernels on `hip_stream` (a hipStream_t; NULL = null stream). */
int sllbm_set_stream(sllbm_ctx *ctx, void *hip_stream);

/* ---- set-up (host only) -------------------------------------------------- */

/* 1-D velocity set of the tensor-product 2-D set (Sec. II.B).  xi1d/w1d hold
 * q1d abscissae and weights of the unscaled set (c_s = 1); NULL/NULL selects
 * the set of that size: for q1d = 5 the D1Q5 Gauss-Hermite set of Table I
 * (0, +sqrt(5-sqrt(10)), +sqrt(5+sqrt(10)), -sqrt(5-sqrt(10)),
 * -sqrt(5+sqrt(10))), for q1d = 3 the D1Q3 one (0, +sqrt(3), -sqrt(3);
 * 2/3, 1/6, 1/6), whose product D2Q9 is the comparison set of Sec. III.A
 * (isothermal model only, on the row-segment, direct and records kernels).
 * Other sizes: SLLBM_E_UNSUPPORTED.  Weights must be positive and finite.
 * cs > 0 scales the set (Sec. II.B: "unless scaled", c_s = 1): the
 * physical velocities are cs * xi1d, the reference temperature is
 * T0 = cs^2 (c_s^2 = R T0, R = 1), tau = nu / (cs^2 dt) + 1/2, and the
 * equilibrium is the Hermite expansion in xi / cs, u / cs and T / T0.  All
 * node fields in and out (init_macro, moments) are physical; inside, the
 * second population is held as g / cs^2.  The adjoint calls need cs = 1. */
int sllbm_set_velocity_set(sllbm_ctx *ctx, int q1d, const double *xi1d, const double *w1d,
                           double cs);

/* Interpolation order p in 1..4 and support-point family (Sec. II.E:
 * Gauss-Lobatto-Chebyshev points; equidistant points as the unstable
 * comparison of Sec. III.D). */
int sllbm_set_order(sllbm_ctx *ctx, int p, int nodes);

/* Uniform grid of ncx x ncy cells on [x0, x1] x [y0, y1].  Periodic axes
 * carry nc * p unique nodes, zero-gradient axes nc * p + 1 (outer support
 * points are shared between neighbouring cells).  Zero-gradient boundaries
 * clamp departure points to the boundary (the paper's "d f = 0"). */
int sllbm_init_grid_uniform(sllbm_ctx *ctx, int ncx, int ncy, double x0, double x1, double y0,
                            double y1, int bcx, int bcy);

/* Tensor-product grid from strictly increasing cell edges (ncx + 1 and
 * ncy + 1 values, copied), cells affine per axis -- e.g. the transformed grid
 * of Sec. III.E.  Same node numbering and boundaries as the uniform grid. */
int sllbm_init_grid_mapped(sllbm_ctx *ctx, int ncx, int ncy, const double *edges_x,
                           const double *edges_y, int bcx, int bcy);

/* Curvilinear mesh of ncx x ncy bilinear cells, periodic in x and y: the
 * cell interpolation of Sec. II.E, eq. (17), on cells that are bilinear
 * images of the reference square (curved cells are the generalisation the
 * paper leaves to future work).  vx, vy: host float64 arrays
 * [ncy + 1][ncx + 1] (copied) of vertex coordinates; vertex column ncx must
 * be column 0 moved by (Lx, 0) and row ncy row 0 moved by (0, Ly), the
 * periods, and every cell's Jacobian must be positive at its four corners
 * (counter-clockwise, not folded), else SLLBM_E_ARG.  Nodes: nx = ncx p,
 * ny = ncy p; node (ix, iy) is support point (ix mod p, iy mod p) of cell
 * (ix / p, iy / p) (sllbm_node_coords_2d gives their coordinates).
 * Departure points are located on the host (Newton's method on the cell
 * map and a walk across neighbouring cells, at the first step after set-up;
 * a departure point that is not found fails that step with SLLBM_E_ARG) and
 * streamed with the records gather: AUTO resolves to SLLBM_PATH_RECORDS and
 * every other path is refused (SLLBM_E_UNSUPPORTED), as are the per-axis
 * queries (sllbm_node_coords, sllbm_departure_table, sllbm_mass_weights).
 * sllbm_mass integrates the interpolated density with the node masses of the
 * bilinear cells (sllbm_node_masses).  The adjoint's S^T is the transposed
 * records gather (built on the host at the first adjoint call: per velocity,
 * N (p+1)^2 entries of a target index and a weight). */
int sllbm_init_grid_curvilinear(sllbm_ctx *ctx, int ncx, int ncy, const double *vx,
                                const double *vy);

/* Time step dt > 0, kinematic viscosity nu > 0 (nu = +inf: no collision,
 * pure streaming), heat-capacity ratio gamma > 1 (used by SLLBM_POLYATOMIC
 * only), Prandtl number Pr > 0, model (sllbm_model).  Pr != 1 needs a
 * thermal model (SLLBM_E_ARG for SLLBM_ISOTHERMAL) and a 1-D
 * velocity set that integrates the Gaussian's moments exactly up to degree 7
 * (the default set does), so that the equilibrium has no centred third
 * moment; SLLBM_E_UNSUPPORTED otherwise (also from a later
 * sllbm_set_velocity_set that breaks it).  The adjoint calls below cover
 * Pr != 1 except the viscosity term (SLLBM_E_UNSUPPORTED there). */
int sllbm_set_physics(sllbm_ctx *ctx, double dt, double nu, double gamma, double Pr, int model);

/* Streaming kernel family (sllbm_path).  SLLBM_PATH_TILED needs departures
 * that stay within a bounded row window, SLLBM_PATH_ROWS segments of >= 32
 * nodes whose x-stencils fit 64 columns and a first 1-D velocity of 0,
 * SLLBM_PATH_MFMA float32 and narrow stencils (checked at sllbm_step;
 * SLLBM_E_UNSUPPORTED otherwise).  The adjoint calls use the same family
 * for their transposed gather (AUTO: row segments, else tiled, else
 * direct). */
int sllbm_set_path(sllbm_ctx *ctx, int path);

/* The kernel family the next step runs (sllbm_path, never AUTO), after grid,
 * order and physics are set.  Host only. */
int sllbm_resolved_path(const sllbm_ctx *ctx, int *path);

/* ---- queries (host only, after init_grid; tables after set_physics) -------- */

int sllbm_num_nodes(const sllbm_ctx *ctx, int64_t *nx, int64_t *ny);

/* Number of population sets S (1 or 2) and bytes per population value. */
int sllbm_population_layout(const sllbm_ctx *ctx, int *nsets, int *q, int *bytes_per_value);

/* Node coordinates per axis: x[nx], y[ny] (host arrays); axis-product
 * grids only. */
int sllbm_node_coords(const sllbm_ctx *ctx, double *x, double *y);

/* Coordinates of every node, x[ny][nx] and y[ny][nx] (host arrays), on any
 * grid. */
int sllbm_node_coords_2d(const sllbm_ctx *ctx, double *x, double *y);

/* Departure table of one axis (0 = x, 1 = y) and 1-D velocity index comp:
 * for each node j of that axis, src[j * (p+1) + m] is the source node along
 * the axis and w[j * (p+1) + m] the Lagrange weight, so that the 1-D value
 * at the departure point is sum_m w * value[src].  Host arrays. */
int sllbm_departure_table(const sllbm_ctx *ctx, int axis, int comp, int32_t *src, double *w);

/* Departure records of velocity i = a + 5 b (0..24) for every node, as the
 * records gather reads them: cell[v] = cx | cy << 16 (the departure cell),
 * r[v], s[v] in [0, 1] its reference coordinates (Sec. II.E, eq. (17)).
 * Host arrays of nx*ny; any grid.  SLLBM_E_ARG if a departure point of a
 * curvilinear mesh is not found. */
int sllbm_departure_records(const sllbm_ctx *ctx, int i, int32_t *cell, double *r, double *s);

/* Integral of each node's shape function per axis (mass weights): the 2-D
 * weight of node (iy, ix) is my[iy] * mx[ix]. */
int sllbm_mass_weights(const sllbm_ctx *ctx, double *mx, double *my);

/* Mass weight of every node, m[ny][nx] (host array), on any grid: the
 * integral of the node's shape function, i.e. the sum over the cells sharing
 * the node of the integral of its local basis l_a(r) l_b(s) times the cell
 * map's Jacobian (Sec. II.E; the weights of the mass monitor of Sec. III.E).
 * On axis-product grids the product my[iy] mx[ix] of sllbm_mass_weights; on
 * a curvilinear mesh of bilinear cells from the Jacobian, which is linear in
 * (r, s) there. */
int sllbm_node_masses(const sllbm_ctx *ctx, double *m);

/* Relaxation time tau = nu/(c_s^2 dt) + 1/2 (Sec. II.D); +inf for nu = +inf. */
int sllbm_relaxation_time(const sllbm_ctx *ctx, double *tau);

/* ---- state ----------------------------------------------------------------- */

/* Use two caller-owned device buffers of S*Q*nx*ny population values each
 * as the ping-pong pair.  The caller keeps ownership and must keep them
 * alive while the context uses them; their contents are the library's (in
 * its internal order, see the header comment), to be read and written
 * through sllbm_get_populations / sllbm_set_populations.  Without this call
 * the library allocates the pair itself. */
int sllbm_bind_populations(sllbm_ctx *ctx, void *dev_a, void *dev_b);

/* Initialise populations at equilibrium: f = f_eq(rho, u, theta) and, for
 * the polyatomic model, g = g_eq (the paper does not state its
 * initialisation; this is the reading used).  rho, ux, uy, T are node arrays
 * (host if on_device = 0, device otherwise).  rho and T must be positive
 * and every value finite (checked for host arrays; SLLBM_E_ARG).  The
 * isothermal model ignores T.  Resets the step counter and stability flag. */
int sllbm_init_macro(sllbm_ctx *ctx, const double *rho, const double *ux, const double *uy,
                     const double *T, int on_device);

/* ---- time stepping ----------------------------------------------------------- */

/* Advance n >= 0 steps, asynchronously on the bound stream.  The stability
 * flag (set when any node has rho <= 0, theta <= 0 or a non-finite moment,
 * the paper's "bounded" criterion of Sec. III.C) is read back every
 * check_interval steps if that interval is > 0 (sllbm_set_check_interval),
 * in which case SLLBM_E_UNSTABLE is returned at the first raised flag. */
int sllbm_step(sllbm_ctx *ctx, int64_t n);

/* Interval for the flag read-back inside sllbm_step (0 = never; default 0). */
int sllbm_set_check_interval(sllbm_ctx *ctx, int64_t k);

/* sllbm_step that also records, for each of the n steps, the moments of the
 * streamed (pre-collision) state: moments[s][0..K-1][ny][nx] = rho, u_x, u_y
 * and, unless isothermal, theta, and with Pr != 1 the centred second moments
 * sum f (xi_x - u_x)^2, sum f (xi_x - u_x)(xi_y - u_y), sum f (xi_y - u_y)^2
 * of f and then of g (float64, device pointer, K * nx * ny values per step,
 * K from sllbm_recorded_moments).  These are what the collision Jacobian of
 * step s depends on; the adjoint sweep replays a checkpointed segment with
 * this call.  The second moments are recovered after each step from its
 * post-collision state (the collision moves them by the factor 1 - 1/tau),
 * so a Pr != 1 record needs tau != 1 (SLLBM_E_UNSUPPORTED otherwise). */
int sllbm_step_record(sllbm_ctx *ctx, int64_t n, double *moments);

/* K, the moments sllbm_step_record keeps per node and step: 3 isothermal,
 * 4 for the thermal models at Pr = 1, 4 + 3 S at Pr != 1 (S population
 * sets).  Needs the physics (SLLBM_E_STATE otherwise). */
int sllbm_recorded_moments(const sllbm_ctx *ctx, int *k);

/* Synchronise and report the stability flag (1 = raised) and step count. */
int sllbm_status_flags(sllbm_ctx *ctx, int *unstable, int64_t *steps_done);

/* ---- outputs ----------------------------------------------------------------- */

/* rho, ux, uy, T per node (physical units: T = theta T0 with T0 = cs^2, so
 * T = theta for the unscaled set) from the current populations.
 * rho, ux, uy, T and the collision invariants they derive from are equal
 * before and after the collision, so these are the post-streaming moments.
 * Arrays of nx*ny float64, host (synchronises) or device (async). */
int sllbm_moments(sllbm_ctx *ctx, double *rho, double *ux, double *uy, double *T, int on_device);

/* Total mass sum_v M_v rho_v with M_v the integral of node v's shape function
 * (sllbm_node_masses; relative mass m/m0 is the monitor of Sec. III.E), on
 * every grid.  Deterministic FP64 reduction; synchronises. */
int sllbm_mass(sllbm_ctx *ctx, double *mass);

/* sllbm_mass for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc): the
 * same reduction, written to mass_dev (a caller-owned float64 on the
 * context's device), asynchronously on the bound stream; nothing is
 * allocated and nothing synchronises.  The per-block partial sums go to a
 * fixed device array of 2^17 float64 (1 MiB) that the library holds on each
 * GPU it runs on until the process ends; it covers every grid the library
 * accepts (up to 2^25 nodes; SLLBM_E_ARG beyond).  Every context on a GPU
 * shares that array: calls that overlap on one GPU (other streams, other
 * threads) race on it, and each call overwrites what the last one left.
 * Needs initialised populations (SLLBM_E_STATE otherwise, as the device
 * tables are built by sllbm_init_macro / sllbm_set_populations);
 * on every grid, as sllbm_mass. */
int sllbm_mass_noalloc(sllbm_ctx *ctx, double *mass_dev);

/* Copy the current populations out / in ([S][Q][ny][nx], population type,
 * whatever order the state buffers hold).  set_populations makes the given
 * state current (step counter unchanged, stability flag cleared).  A device
 * pointer must not be one of the context's two state buffers (SLLBM_E_ARG);
 * both calls may use the buffer that does not hold the state as staging. */
int sllbm_get_populations(sllbm_ctx *ctx, void *dst, int on_device);
int sllbm_set_populations(sllbm_ctx *ctx, const void *src, int on_device);

/* ---- adjoint of the step (every model and Prandtl number) ----
 * The paper has no adjoint; these calls differentiate exactly the step above.
 * One step is F' = C(S F) with S the interpolation of every population plane
 * (Sec. II.E, eq. (17)) and C the collision of Sec. II.D, eq. (16): BGK, plus
 * with Pr != 1 the quasi-equilibrium term (1/tau - 1/tau_Pr) f*(Q) built from
 * the centred third moments Q of each set (Sec. II.C), whose transpose needs
 * the centred second moments the record then holds.
 * Reverse sweep:  mu^n = J_C(M^n)^T lambda^{n+1},  lambda^n = S^T mu^n,
 * where M^n are the moments recorded by sllbm_step_record for step n.
 * All arrays are device pointers on the context's device; lambda / mu arrays
 * are [S][25][ny][nx] in the population type (S = 2 for the polyatomic
 * model); node fields are float64 [ny][nx]; a moments record is [K][ny][nx]
 * as sllbm_step_record writes it (K from sllbm_recorded_moments).  Calls
 * are asynchronous on the bound stream. */

/* lambda = dL/dF of the current populations F for a loss with gradients
 * g_rho, g_ux, g_uy, g_T with respect to the node moments rho, u_x, u_y and
 * temperature of F (g_T may be NULL: no temperature term; ignored when
 * isothermal). */
int sllbm_adjoint_seed(sllbm_ctx *ctx, const double *g_rho, const double *g_ux, const double *g_uy,
                       const double *g_T, void *lambda);

/* mu = J_C(M)^T lambda node by node; moments = one step's [K][ny][nx] record. */
int sllbm_adjoint_collide(sllbm_ctx *ctx, const void *lambda, const double *moments, void *mu);

/* Viscosity term of the gradient (Pr = 1): acc[0] += <lambda, dC/d(nu)> for
 * one step, lambda = dL/dF+ of that step's post-collision populations
 * `populations` (device, the population layout) and `moments` their
 * [K][ny][nx] record.  The BGK collision of Sec. II.D depends on nu through
 * 1/tau with tau = nu/dt + 1/2; because the moments are collision
 * invariants, F - F_eq before the collision is (F+ - F_eq)/(1 - 1/tau), so
 * the term is sum lambda (F+ - F_eq) / ((1 - 1/tau) tau^2 dt).  Summed over
 * the steps it is dL/d(nu).  acc: one float64 on the device, accumulated in
 * stream order.  SLLBM_E_UNSUPPORTED when tau = 1 (F+ = F_eq carries no
 * non-equilibrium part) or with Pr != 1. */
int sllbm_adjoint_nu_term(sllbm_ctx *ctx, const void *lambda, const void *populations,
                          const double *moments, double *acc);

/* out = S^T mu (the transposed interpolation, a gather through transposed
 * departure tables, or on a curvilinear mesh through the transposed
 * records), followed by J_C(M_prev)^T when moments_prev (the record
 * of the previous step) is not NULL (fused into one kernel at Pr = 1; at
 * Pr != 1 two kernels through a library-owned scratch array of one state).
 * mu and out must differ. */
int sllbm_adjoint_step(sllbm_ctx *ctx, const void *mu, const double *moments_prev, void *out);

/* Gradient through the initialisation f = f_eq(rho0, u0, T0), g = g_eq:
 * g_rho0 = sum_i lambda_i dF_eq_i/drho0, likewise for u0 and T0.  T0 is
 * required unless isothermal (where it and g_T0 may be NULL); g_T0 may be
 * NULL. */
int sllbm_eq_init_vjp(sllbm_ctx *ctx, const void *lambda0, const double *rho0, const double *ux0,
                      const double *uy0, const double *T0, double *g_rho0, double *g_ux0,
                      double *g_uy0, double *g_T0);

#ifdef __cplusplus
}
#endif

#endif /* SLLBM_H */
