/* libsllbm, three dimensions: the semi-Lagrangian lattice Boltzmann step of
 * Wilde, Kraemer, Reith, Foysi (arXiv:1910.13918) on D3Q125, the tensor
 * product of three D1Q5 rules (Sec. II.B, Table I), which the paper names as
 * its extension to three dimensions (Sec. IV and V).
 *
 * What one step computes (isothermal, theta = 1, c_s = 1): for every node x
 * and velocity xi_i = (xi_a, xi_b, xi_c), i = a + 5 b + 25 c, the value at
 * the departure point x - dt xi_i of the cell-local Lagrange interpolant of
 * order p (Sec. II.E, eq. (17) with a third factor; GLC or equidistant
 * support points), with periodic wrap or zero-gradient clamp per axis; then
 * the BGK relaxation toward the 4th-order Hermite equilibrium of Sec. II.A
 * (eqs. (9)-(10) in three components) with tau = nu / dt + 1/2 (Sec. II.D).
 * Moments (rho, u) and the equilibrium are evaluated in float64 in both
 * precisions.
 *
 * Grid: the tensor product of three axes of cells (per-axis edges, so
 * uniform and per-axis mapped grids), nodes shared between neighbouring
 * cells; nx = ncx p (periodic) or ncx p + 1, likewise y and z; node index
 * v = (iz ny + iy) nx + ix.
 *
 * Populations cross the boundary as 125 planes of N = nx ny nz values:
 * value (i, v) at i N + v, float64 or float32 as the precision.
 *
 * Status codes, precisions, boundary kinds and support-point families are
 * those of sllbm.h.  Every call returns SLLBM_OK or a negative code; the
 * context's sllbm3d_last_error() then holds a message.  Calls on one context
 * are not thread-safe.  Set-up (order, grid, physics) is refused once the
 * populations are initialised (SLLBM_E_STATE); create a new context instead.
 */
#ifndef SLLBM3D_H
#define SLLBM3D_H

#include <stdint.h>

#include "sllbm.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct sllbm3d_ctx sllbm3d_ctx;

/* New context on HIP device hip_device; precision SLLBM_FP64 or SLLBM_FP32
 * (SLLBM_E_ARG otherwise).  No device work until the first populations. */
int sllbm3d_create(sllbm3d_ctx **out, int hip_device, int precision);
/* Frees the context, its device tables and the population buffers it owns
 * (bound buffers stay the caller's).  NULL is accepted. */
void sllbm3d_destroy(sllbm3d_ctx *ctx);
/* Message of the last failed call ("" if none); owned by the context. */
const char *sllbm3d_last_error(const sllbm3d_ctx *ctx);
/* HIP stream for every launch and copy (default: the null stream). */
int sllbm3d_set_stream(sllbm3d_ctx *ctx, void *hip_stream);

/* Interpolation order p in 1..4 and the support points (Sec. II.E):
 * SLLBM_NODES_GLC or SLLBM_NODES_EQUIDISTANT.  Resets the grid. */
int sllbm3d_set_order(sllbm3d_ctx *ctx, int p, int nodes);
/* Cells: ncx + 1, ncy + 1, ncz + 1 strictly increasing finite edges per
 * axis (host arrays, copied); bc_* SLLBM_PERIODIC or SLLBM_ZERO_GRADIENT.
 * SLLBM_E_ARG when a cell count is outside 1..65535 or one population plane
 * would exceed 2^32 bytes; SLLBM_E_STATE before sllbm3d_set_order. */
int sllbm3d_init_grid(sllbm3d_ctx *ctx, int ncx, int ncy, int ncz, const double *edges_x,
                      const double *edges_y, const double *edges_z, int bc_x, int bc_y, int bc_z);
/* Time step dt > 0 and kinematic viscosity nu > 0 (+inf: no collision,
 * 1/tau = 0), tau = nu / dt + 1/2 (Sec. II.D, c_s = 1). */
int sllbm3d_set_physics(sllbm3d_ctx *ctx, double dt, double nu);
int sllbm3d_num_nodes(const sllbm3d_ctx *ctx, int64_t *nx, int64_t *ny, int64_t *nz);
/* Node coordinates per axis into host arrays of nx, ny and nz doubles. */
int sllbm3d_node_coords(const sllbm3d_ctx *ctx, double *x, double *y, double *z);

/* Two distinct device buffers of 125 N values each (the library otherwise
 * allocates its own at the first initialisation); the caller keeps
 * ownership and must keep them alive.  Needs order, grid and physics; a
 * later change of order or grid forgets the binding. */
int sllbm3d_bind_populations(sllbm3d_ctx *ctx, void *dev_a, void *dev_b);
/* f = f_eq(rho, u) at every node from N-value float64 arrays (host arrays,
 * checked: rho > 0 and all finite; or device arrays with on_device != 0,
 * unchecked).  Clears the stability flag and the step counter. */
int sllbm3d_init_macro(sllbm3d_ctx *ctx, const double *rho, const double *ux, const double *uy,
                       const double *uz, int on_device);
/* n >= 0 steps, enqueued on the stream (no synchronisation).  SLLBM_E_STATE
 * before the populations are initialised. */
int sllbm3d_step(sllbm3d_ctx *ctx, int64_t n);
/* Synchronises; unstable = 1 once any step met a node with rho <= 0 or a
 * non-finite moment (Sec. III.C's bounded-values criterion), and the number
 * of steps taken since the last initialisation. */
int sllbm3d_status_flags(sllbm3d_ctx *ctx, int *unstable, int64_t *steps_done);
/* rho, u_x, u_y, u_z per node (float64, N values each) of the current
 * populations: host arrays (synchronises) or device arrays (on_device). */
int sllbm3d_moments(sllbm3d_ctx *ctx, double *rho, double *ux, double *uy, double *uz,
                    int on_device);
/* Mass sum_v M_v rho_v with M_v the integral of node v's shape function
 * (the product of the three axes' integrals; the mass monitor of Sec. III.E),
 * a fixed-order float64 reduction on the device.  Synchronises. */
int sllbm3d_mass(sllbm3d_ctx *ctx, double *mass);
/* Copy of the current populations (125 N values, planar as above) to host
 * memory (synchronises) or device memory (on_device); set replaces them and
 * clears the stability flag.  The context's own buffers are refused as
 * source or destination (SLLBM_E_ARG). */
int sllbm3d_get_populations(sllbm3d_ctx *ctx, void *dst, int on_device);
int sllbm3d_set_populations(sllbm3d_ctx *ctx, const void *src, int on_device);

#ifdef __cplusplus
}
#endif

#endif /* SLLBM3D_H */
