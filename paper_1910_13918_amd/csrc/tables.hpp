// Host-side precomputation for the SLLBM step: velocity set constants,
// support points, Lagrange weights, departure tables, mass weights.
//
// All tables are built once per (grid, dt, velocity set) in float64 on the
// host; the kernels only read them.
#pragma once

#include <cstdint>
#include <string>
#include <vector>

namespace sllbm {

constexpr int kMaxOrder = 4;
constexpr int kQ1 = 5;           // most 1-D velocities of a tensor-product set
constexpr int kQ = kQ1 * kQ1;    // most 2-D velocities
constexpr int kDim = 2;

// 1-D velocity set (Sec. II.B, Table I) and per-velocity Hermite constants;
// q1 = 5 (D1Q5, whose product is D2Q25) or 3 (D1Q3: D2Q9, Sec. III.A).
struct VelocitySet {
  int q1 = kQ1;
  double xi[kQ1];
  double w[kQ1];
  // hk[a][k] = He_k(xi_a) / k!  (probabilists' Hermite polynomials, k <= 4)
  double hk[kQ1][5];
};

VelocitySet default_velocity_set();
// Three-point Gauss-Hermite rule: 0, +sqrt(3), -sqrt(3); 2/3, 1/6, 1/6.
VelocitySet d1q3_velocity_set();
void fill_hermite_constants(VelocitySet &vs);

// True when the 1-D rule reproduces the moments of the unit Gaussian,
// sum_a w_a xi_a^n = (n-1)!! (n even) or 0 (n odd), for every n <= degree
// (relative tolerance 1e-12).
bool gaussian_exact_to_degree(const VelocitySet &vs, int degree);

// Reference support points on [0, 1] for order p (Sec. II.E).
std::vector<double> support_points(int p, bool glc);

// Lagrange weights l_m(r), m = 0..p, product formula on the given points.
void lagrange_weights(const std::vector<double> &pts, double r, double *out);

// Integrals over [0, 1] of each Lagrange polynomial, by exact integration of
// the monomial expansion.
std::vector<double> lagrange_integrals(const std::vector<double> &pts);
// Moments int_0^1 r^k l_m(r) dr of each Lagrange polynomial (k = 0: the
// integrals above).
std::vector<double> lagrange_moments(const std::vector<double> &pts, int k);

// One grid direction.
struct Axis {
  std::vector<double> edges;  // ncells + 1, strictly increasing
  int ncells = 0;
  int p = 0;
  bool periodic = true;
  bool uniform = true;
  int n = 0;                  // unique nodes
  std::vector<double> r;      // reference support points (p + 1)

  void setup(const std::vector<double> &e, int order, bool per, bool unif,
             const std::vector<double> &pts);
  double coord(int j) const;
  // Cell and local support-point index of node j (the last node of a
  // non-periodic axis is the right vertex of the last cell).
  void cell_of(int j, int &cell, int &local) const;
  int node(int cell, int m) const { int j = cell * p + m; return periodic ? j % n : j; }
  // Departure point of node j displaced by `disp`: cell and reference
  // coordinate after the boundary treatment (periodic wrap / clamp).
  // `unwrapped` (optional) receives the cell index before the periodic wrap
  // (it may be negative or >= ncells), which keeps neighbouring departures
  // contiguous across the seam.
  void departure(int j, double disp, int &cell, double &r, long *unwrapped = nullptr) const;
  std::vector<double> node_mass() const;
};

// Per-axis gather table for one 1-D velocity: node j combines `taps`
// consecutive nodes starting at the unwrapped index start[j]:
// value(j) = sum_t w[j * taps + t] * f[src[j * taps + t]], with src the
// start + t wrapped onto the axis.  For the forward step the taps are the
// p+1 nodes of the departure cell; for the transposed step (adjoint) they are
// the targets whose departure stencil contains j.
struct AxisTable {
  int taps = 0;
  std::vector<int32_t> src;
  std::vector<double> w;
  std::vector<long> start;     // unwrapped first tap (contiguous across a periodic seam)
  std::vector<int32_t> cell;   // forward only: departure cell per node
  std::vector<double> rref;    // forward only: reference coordinate per node
};

AxisTable build_axis_table(const Axis &ax, double disp);

// True when every node's stencil in t is the node itself with weight 1 (all
// other weights exactly 0): the table of a zero velocity component.
bool identity_table(const AxisTable &t, int n);

// Transpose of a forward table: entry (j, t) holds the weight with which
// node j's value enters target start[j] + t.  Targets of one source node are
// consecutive because departures are monotone along the axis.
AxisTable transpose_axis_table(const Axis &ax, const AxisTable &fwd);

}  // namespace sllbm
