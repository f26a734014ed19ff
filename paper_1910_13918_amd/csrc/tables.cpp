// Host-side precomputation (see tables.hpp).
#include "tables.hpp"

#include <algorithm>
#include <cmath>
#include <limits>
#include <utility>

namespace sllbm {

VelocitySet default_velocity_set() {
  // Table I: 0, +sqrt(5 - sqrt(10)), +sqrt(5 + sqrt(10)), and the negatives;
  // weights 8/15, (7 + 2 sqrt(10))/60, (7 - 2 sqrt(10))/60.
  VelocitySet vs{};
  const double r10 = std::sqrt(10.0);
  const double c1 = std::sqrt(5.0 - r10), c2 = std::sqrt(5.0 + r10);
  const double w1 = (7.0 + 2.0 * r10) / 60.0, w2 = (7.0 - 2.0 * r10) / 60.0;
  const double xi[kQ1] = {0.0, c1, c2, -c1, -c2};
  const double w[kQ1] = {8.0 / 15.0, w1, w2, w1, w2};
  for (int a = 0; a < kQ1; ++a) { vs.xi[a] = xi[a]; vs.w[a] = w[a]; }
  vs.q1 = kQ1;
  fill_hermite_constants(vs);
  return vs;
}

VelocitySet d1q3_velocity_set() {
  // roots of He_3 = x^3 - 3x and their Gauss-Hermite weights
  VelocitySet vs{};
  vs.q1 = 3;
  const double r3 = std::sqrt(3.0);
  const double xi[3] = {0.0, r3, -r3};
  const double w[3] = {2.0 / 3.0, 1.0 / 6.0, 1.0 / 6.0};
  for (int a = 0; a < 3; ++a) { vs.xi[a] = xi[a]; vs.w[a] = w[a]; }
  fill_hermite_constants(vs);
  return vs;
}

void fill_hermite_constants(VelocitySet &vs) {
  for (int a = 0; a < vs.q1; ++a) {
    const double x = vs.xi[a], x2 = x * x;
    vs.hk[a][0] = 1.0;
    vs.hk[a][1] = x;
    vs.hk[a][2] = (x2 - 1.0) / 2.0;
    vs.hk[a][3] = (x2 * x - 3.0 * x) / 6.0;
    vs.hk[a][4] = (x2 * x2 - 6.0 * x2 + 3.0) / 24.0;
  }
}

bool gaussian_exact_to_degree(const VelocitySet &vs, int degree) {
  double exact = 1.0;  // (n-1)!! for even n
  for (int n = 0; n <= degree; ++n) {
    double sum = 0.0, mag = 0.0;
    for (int a = 0; a < vs.q1; ++a) {
      const double t = vs.w[a] * std::pow(vs.xi[a], n);
      sum += t;
      mag += std::fabs(t);
    }
    const double want = (n % 2) ? 0.0 : exact;
    if (!(std::fabs(sum - want) <= 1e-12 * std::max(1.0, mag))) return false;
    if (n % 2 == 0) exact *= double(n + 1);
  }
  return true;
}

std::vector<double> support_points(int p, bool glc) {
  std::vector<double> r(p + 1);
  const double pi = 3.14159265358979323846;
  for (int k = 0; k <= p; ++k) {
    if (glc) {
      // (1 - cos(k pi / p)) / 2 written as sin^2(k pi / (2p)); ends exact
      const double s = std::sin(0.5 * pi * k / p);
      r[k] = s * s;
    } else {
      r[k] = double(k) / p;
    }
  }
  r[0] = 0.0;
  r[p] = 1.0;
  return r;
}

void lagrange_weights(const std::vector<double> &pts, double r, double *out) {
  const int n = int(pts.size());
  for (int m = 0; m < n; ++m) {
    double v = 1.0;
    for (int k = 0; k < n; ++k)
      if (k != m) v *= (r - pts[k]) / (pts[m] - pts[k]);
    out[m] = v;
  }
}

std::vector<double> lagrange_integrals(const std::vector<double> &pts) {
  return lagrange_moments(pts, 0);
}

std::vector<double> lagrange_moments(const std::vector<double> &pts, int k) {
  const int n = int(pts.size());
  std::vector<double> out(n);
  for (int m = 0; m < n; ++m) {
    // monomial coefficients of prod_{k != m} (r - r_k) / (r_m - r_k)
    std::vector<double> c(1, 1.0);
    for (int k = 0; k < n; ++k) {
      if (k == m) continue;
      const double d = pts[m] - pts[k];
      std::vector<double> nc(c.size() + 1, 0.0);
      for (size_t t = 0; t < c.size(); ++t) {
        nc[t + 1] += c[t] / d;
        nc[t] -= c[t] * pts[k] / d;
      }
      c.swap(nc);
    }
    // int_0^1 r^k r^t dr = 1 / (t + k + 1)
    double s = 0.0;
    for (size_t t = 0; t < c.size(); ++t) s += c[t] / double(t + k + 1);
    out[m] = s;
  }
  return out;
}

void Axis::setup(const std::vector<double> &e, int order, bool per, bool unif,
                 const std::vector<double> &pts) {
  edges = e;
  ncells = int(e.size()) - 1;
  p = order;
  periodic = per;
  uniform = unif;
  n = periodic ? ncells * p : ncells * p + 1;
  r = pts;
}

void Axis::cell_of(int j, int &cell, int &local) const {
  cell = j / p;
  local = j % p;
  if (cell == ncells) {  // right vertex of a non-periodic axis
    cell = ncells - 1;
    local = p;
  }
}

double Axis::coord(int j) const {
  int c, a;
  cell_of(j, c, a);
  return edges[c] + r[a] * (edges[c + 1] - edges[c]);
}

void Axis::departure(int j, double disp, int &cell, double &rr, long *unwrapped) const {
  int c, a;
  cell_of(j, c, a);
  if (uniform) {
    // cell units: offset from the node's own cell, exact for disp = 0
    const double h = (edges[ncells] - edges[0]) / ncells;
    const double d = r[a] + disp / h;
    const double fl = std::floor(d);
    long cc = long(c) + long(fl);
    rr = d - fl;
    if (unwrapped) *unwrapped = cc;
    if (periodic) {
      cc %= ncells;
      if (cc < 0) cc += ncells;
    } else if (cc < 0) {
      cc = 0;
      rr = 0.0;
    } else if (cc > ncells - 1) {
      cc = ncells - 1;
      rr = 1.0;
    }
    if (unwrapped && !periodic) *unwrapped = cc;
    cell = int(cc);
    return;
  }
  // mapped axis: stay in the node's cell when possible (exact for disp = 0)
  const double h = edges[c + 1] - edges[c];
  const double loc = r[a] + disp / h;
  if (loc >= 0.0 && loc <= 1.0) {
    cell = c;
    rr = loc;
    if (unwrapped) *unwrapped = c;
    return;
  }
  double x = coord(j) + disp;
  const double lo = edges[0], hi = edges[ncells], L = hi - lo;
  long shift = 0;
  if (periodic) {
    shift = long(std::floor((x - lo) / L));
    x -= double(shift) * L;
    if (x < lo) { x += L; --shift; }
    if (x >= hi) { x -= L; ++shift; }
    if (x < lo) x = lo;
  } else {
    x = std::min(std::max(x, lo), hi);
  }
  // binary search: number of interior edges <= x
  const auto it = std::upper_bound(edges.begin() + 1, edges.begin() + ncells, x);
  cell = int(it - (edges.begin() + 1));
  rr = (x - edges[cell]) / (edges[cell + 1] - edges[cell]);
  rr = std::min(std::max(rr, 0.0), 1.0);
  if (unwrapped) *unwrapped = long(cell) + shift * long(ncells);
}

std::vector<double> Axis::node_mass() const {
  const std::vector<double> W = lagrange_integrals(r);
  std::vector<double> m(n, 0.0);
  for (int c = 0; c < ncells; ++c) {
    const double h = edges[c + 1] - edges[c];
    for (int a = 0; a <= p; ++a) m[node(c, a)] += W[a] * h;
  }
  return m;
}

AxisTable build_axis_table(const Axis &ax, double disp) {
  AxisTable t;
  const int P1 = ax.p + 1;
  t.taps = P1;
  t.src.resize(size_t(ax.n) * P1);
  t.w.resize(size_t(ax.n) * P1);
  t.cell.resize(ax.n);
  t.rref.resize(ax.n);
  t.start.resize(ax.n);
  double lw[kMaxOrder + 1];
  for (int j = 0; j < ax.n; ++j) {
    int c;
    double rr;
    long uc;
    ax.departure(j, disp, c, rr, &uc);
    lagrange_weights(ax.r, rr, lw);
    t.cell[j] = c;
    t.start[j] = uc * ax.p;
    t.rref[j] = rr;
    for (int m = 0; m < P1; ++m) {
      t.src[size_t(j) * P1 + m] = ax.node(c, m);
      t.w[size_t(j) * P1 + m] = lw[m];
    }
  }
  return t;
}

bool identity_table(const AxisTable &t, int n) {
  for (int j = 0; j < n; ++j) {
    int ones = 0;
    for (int m = 0; m < t.taps; ++m) {
      const double w = t.w[size_t(j) * t.taps + m];
      if (w == 0.0) continue;
      if (w != 1.0 || t.src[size_t(j) * t.taps + m] != j) return false;
      ++ones;
    }
    if (ones != 1) return false;
  }
  return true;
}

AxisTable transpose_axis_table(const Axis &ax, const AxisTable &fwd) {
  const int n = ax.n, P1 = fwd.taps;
  // (virtual target, weight) pairs per source node
  std::vector<std::vector<std::pair<long, double>>> in(n);
  for (int v = 0; v < n; ++v)
    for (int m = 0; m < P1; ++m) {
      const long su = fwd.start[v] + m;  // unwrapped source index
      long j = su % n;
      if (j < 0) j += n;
      const long k = (su - j) / n;       // periodic image of the source
      in[j].push_back({long(v) - k * n, fwd.w[size_t(v) * P1 + m]});
    }
  AxisTable t;
  int taps = 1;
  std::vector<long> lo(n, 0);
  for (int j = 0; j < n; ++j) {
    long a = std::numeric_limits<long>::max(), b = std::numeric_limits<long>::min();
    for (const auto &e : in[j]) {
      a = std::min(a, e.first);
      b = std::max(b, e.first);
    }
    if (in[j].empty()) a = b = j;
    lo[j] = a;
    taps = std::max<int>(taps, int(b - a + 1));
  }
  t.taps = taps;
  t.start = lo;
  t.src.assign(size_t(n) * taps, 0);
  t.w.assign(size_t(n) * taps, 0.0);
  for (int j = 0; j < n; ++j) {
    for (int q = 0; q < taps; ++q) {
      long v = lo[j] + q;
      if (ax.periodic) {
        v %= n;
        if (v < 0) v += n;
      } else {
        v = std::min<long>(std::max<long>(v, 0), n - 1);
      }
      t.src[size_t(j) * taps + q] = int32_t(v);
    }
    for (const auto &e : in[j]) t.w[size_t(j) * taps + (e.first - lo[j])] += e.second;
  }
  return t;
}

}  // namespace sllbm
