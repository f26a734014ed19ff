#include "curvilinear.hpp"
#include "tables.hpp"

#include <algorithm>
#include <cmath>

namespace sllbm {

namespace {

long floor_div(long a, long b) { return a >= 0 ? a / b : -((-a + b - 1) / b); }

// Partial derivatives of the bilinear map at (r, s).
void jacobian(const double (&x)[4], const double (&y)[4], double r, double s, double &xr,
              double &xs, double &yr, double &ys) {
  xr = (1 - s) * (x[1] - x[0]) + s * (x[3] - x[2]);
  xs = (1 - r) * (x[2] - x[0]) + r * (x[3] - x[1]);
  yr = (1 - s) * (y[1] - y[0]) + s * (y[3] - y[2]);
  ys = (1 - r) * (y[2] - y[0]) + r * (y[3] - y[1]);
}

// Newton's method for x(r, s) = (px, py) from the cell centre, for a point
// inside the cell (where the Jacobian is positive); iterates are kept near
// the unit square.
bool newton(const double (&x)[4], const double (&y)[4], double px, double py, double &r,
            double &s) {
  r = s = 0.5;
  for (int it = 0; it < 60; ++it) {
    double fx, fy, xr, xs, yr, ys;
    bilinear_map(x, y, r, s, fx, fy);
    fx -= px;
    fy -= py;
    jacobian(x, y, r, s, xr, xs, yr, ys);
    const double det = xr * ys - xs * yr;
    if (!(std::fabs(det) > 0)) return false;
    const double dr = (ys * fx - xs * fy) / det, ds = (xr * fy - yr * fx) / det;
    r = std::clamp(r - dr, -0.5, 1.5);
    s = std::clamp(s - ds, -0.5, 1.5);
    if (std::fabs(dr) + std::fabs(ds) < 1e-15) break;
  }
  return std::isfinite(r) && std::isfinite(s);
}

// Which side of the cell the point lies beyond: the cell edges are straight
// (the map is affine along each), and a cell with a positive Jacobian at its
// corners is a convex counter-clockwise quadrilateral, so the point is inside
// exactly when it is not to the right of any edge.  mx, my in {-1, 0, 1}.
void outside(const double (&x)[4], const double (&y)[4], double px, double py, int &mx, int &my) {
  // edges in counter-clockwise order: bottom 0->1, right 1->3, top 3->2, left 2->0
  static const int from[4] = {0, 1, 3, 2}, to[4] = {1, 3, 2, 0};
  static const int dxs[4] = {0, 1, 0, -1}, dys[4] = {-1, 0, 1, 0};
  mx = my = 0;
  for (int e = 0; e < 4; ++e) {
    const double ex = x[to[e]] - x[from[e]], ey = y[to[e]] - y[from[e]];
    const double cr = ex * (py - y[from[e]]) - ey * (px - x[from[e]]);
    if (cr < -1e-12 * (ex * ex + ey * ey)) {
      mx += dxs[e];
      my += dys[e];
    }
  }
}

}  // namespace

void bilinear_map(const double (&x)[4], const double (&y)[4], double r, double s, double &px,
                  double &py) {
  const double w0 = (1 - r) * (1 - s), w1 = r * (1 - s), w2 = (1 - r) * s, w3 = r * s;
  px = w0 * x[0] + w1 * x[1] + w2 * x[2] + w3 * x[3];
  py = w0 * y[0] + w1 * y[1] + w2 * y[2] + w3 * y[3];
}

std::string CurviMesh::setup(int nx_cells, int ny_cells, const double *px, const double *py) {
  ncx = nx_cells;
  ncy = ny_cells;
  const size_t nv = size_t(ncx + 1) * (ncy + 1);
  vx.assign(px, px + nv);
  vy.assign(py, py + nv);
  for (size_t k = 0; k < nv; ++k)
    if (!std::isfinite(vx[k]) || !std::isfinite(vy[k])) return "vertex coordinates must be finite";
  auto X = [&](int i, int j) { return vx[size_t(j) * (ncx + 1) + i]; };
  auto Y = [&](int i, int j) { return vy[size_t(j) * (ncx + 1) + i]; };
  Lx = X(ncx, 0) - X(0, 0);
  Ly = Y(0, ncy) - Y(0, 0);
  if (!(Lx > 0) || !(Ly > 0)) return "the mesh must span positive periods in x and y";
  const double tol = 1e-12 * std::max(Lx, Ly);
  for (int j = 0; j <= ncy; ++j)
    if (std::fabs(X(ncx, j) - X(0, j) - Lx) > tol || std::fabs(Y(ncx, j) - Y(0, j)) > tol)
      return "vertex column ncx must be column 0 moved by (Lx, 0) (periodic in x)";
  for (int i = 0; i <= ncx; ++i)
    if (std::fabs(Y(i, ncy) - Y(i, 0) - Ly) > tol || std::fabs(X(i, ncy) - X(i, 0)) > tol)
      return "vertex row ncy must be row 0 moved by (0, Ly) (periodic in y)";
  // the Jacobian determinant of a bilinear map is affine in r and in s, so
  // positive corners make it positive everywhere
  for (int j = 0; j < ncy; ++j)
    for (int i = 0; i < ncx; ++i) {
      double x[4], y[4];
      corners(i, j, x, y);
      for (int k = 0; k < 4; ++k) {
        double xr, xs, yr, ys;
        jacobian(x, y, double(k & 1), double(k >> 1), xr, xs, yr, ys);
        if (!(xr * ys - xs * yr > 0))
          return "cell (" + std::to_string(i) + ", " + std::to_string(j) +
                 ") is folded or not counter-clockwise (Jacobian <= 0 at a corner)";
      }
    }
  return "";
}

void CurviMesh::corners(long ux, long uy, double (&x)[4], double (&y)[4]) const {
  const long kx = floor_div(ux, ncx), ky = floor_div(uy, ncy);
  const int i = int(ux - kx * ncx), j = int(uy - ky * ncy);
  const double sx = double(kx) * Lx, sy = double(ky) * Ly;
  for (int k = 0; k < 4; ++k) {
    const size_t v = size_t(j + (k >> 1)) * (ncx + 1) + (i + (k & 1));
    x[k] = vx[v] + sx;
    y[k] = vy[v] + sy;
  }
}

void curvi_node_coords(const CurviMesh &m, const std::vector<double> &pts, std::vector<double> &X,
                       std::vector<double> &Y) {
  const int p = int(pts.size()) - 1;
  const int nx = m.ncx * p, ny = m.ncy * p;
  X.assign(size_t(nx) * ny, 0.0);
  Y.assign(size_t(nx) * ny, 0.0);
  for (int iy = 0; iy < ny; ++iy)
    for (int ix = 0; ix < nx; ++ix) {
      double x[4], y[4];
      m.corners(ix / p, iy / p, x, y);
      const size_t v = size_t(iy) * nx + ix;
      bilinear_map(x, y, pts[ix % p], pts[iy % p], X[v], Y[v]);
    }
}

std::string curvi_records(const CurviMesh &m, const std::vector<double> &pts,
                          const std::vector<double> &X, const std::vector<double> &Y, double dx,
                          double dy, int32_t *cell, double *r, double *s) {
  const int p = int(pts.size()) - 1;
  const int nx = m.ncx * p, ny = m.ncy * p;
  const double tol = 1e-9;  // Newton's answer for a point found inside
  const int max_moves = 2 * (m.ncx + m.ncy) + 16;
  for (int iy = 0; iy < ny; ++iy)
    for (int ix = 0; ix < nx; ++ix) {
      const size_t v = size_t(iy) * nx + ix;
      const double px = X[v] + dx, py = Y[v] + dy;
      long ux = ix / p, uy = iy / p;
      bool found = false;
      double rr = 0, ss = 0;
      for (int k = 0; k <= max_moves && !found; ++k) {
        double x[4], y[4];
        m.corners(ux, uy, x, y);
        int mx, my;
        outside(x, y, px, py, mx, my);
        if (mx != 0 || my != 0) {
          ux += mx;
          uy += my;
          continue;
        }
        if (!newton(x, y, px, py, rr, ss)) break;
        found = rr >= -tol && rr <= 1 + tol && ss >= -tol && ss <= 1 + tol;
        break;
      }
      if (!found)
        return "departure point of node (" + std::to_string(ix) + ", " + std::to_string(iy) +
               ") not found in the mesh";
      const long cx = ux - floor_div(ux, m.ncx) * m.ncx, cy = uy - floor_div(uy, m.ncy) * m.ncy;
      cell[v] = int32_t(uint32_t(cx) | (uint32_t(cy) << 16));
      r[v] = std::clamp(rr, 0.0, 1.0);
      s[v] = std::clamp(ss, 0.0, 1.0);
    }
  return "";
}

std::vector<double> curvi_node_mass(const CurviMesh &m, const std::vector<double> &pts) {
  const int p = int(pts.size()) - 1;
  const int nx = m.ncx * p, ny = m.ncy * p;
  const std::vector<double> W0 = lagrange_moments(pts, 0), W1 = lagrange_moments(pts, 1);
  std::vector<double> M(size_t(nx) * ny, 0.0);
  for (int cy = 0; cy < m.ncy; ++cy)
    for (int cx = 0; cx < m.ncx; ++cx) {
      double x[4], y[4];  // corners 00, 10, 01, 11
      m.corners(cx, cy, x, y);
      // x(r, s) = A0 + A1 r + A2 s + A3 r s; det of [x_r x_s] is
      // A1 x A2 + (A1 x A3) r + (A3 x A2) s (the r s terms cancel)
      const double a1x = x[1] - x[0], a1y = y[1] - y[0];
      const double a2x = x[2] - x[0], a2y = y[2] - y[0];
      const double a3x = x[0] - x[1] - x[2] + x[3], a3y = y[0] - y[1] - y[2] + y[3];
      const double J0 = a1x * a2y - a1y * a2x;
      const double Jr = a1x * a3y - a1y * a3x;
      const double Js = a3x * a2y - a3y * a2x;
      for (int b = 0; b <= p; ++b)
        for (int a = 0; a <= p; ++a) {
          const int ix = (cx * p + a) % nx, iy = (cy * p + b) % ny;
          M[size_t(iy) * nx + ix] += J0 * W0[a] * W0[b] + Jr * W1[a] * W0[b] + Js * W0[a] * W1[b];
        }
    }
  return M;
}

}  // namespace sllbm
