// Host-side geometry of meshes of bilinear cells (the curvilinear
// generalisation of the cell interpolation of Sec. II.E, eq. (17)).
//
// Each cell is the bilinear image of the reference square [0, 1]^2 spanned
// by its four vertices; its support points are the images of the
// tensor-product support points.  The mesh is periodic in x and y: vertex
// column ncx is column 0 moved by (Lx, 0), vertex row ncy is row 0 moved by
// (0, Ly), and nodes are numbered v = iy * nx + ix with nx = ncx p,
// ny = ncy p, node (ix, iy) being support point (ix mod p, iy mod p) of cell
// (ix / p, iy / p).  The departure records it produces are the ones of the
// records gather: cell (cx | cy << 16) and reference coordinates (r, s).
#pragma once

#include <cstdint>
#include <string>
#include <vector>

namespace sllbm {

struct CurviMesh {
  int ncx = 0, ncy = 0;
  std::vector<double> vx, vy;  // (ncy + 1) x (ncx + 1), row-major
  double Lx = 0, Ly = 0;       // periods

  // Copies and validates the vertices; returns "" or what is wrong
  // (non-finite values, vertex row / column ncy / ncx not the periodic image
  // of 0, a cell whose Jacobian is not positive at every corner).
  std::string setup(int ncx, int ncy, const double *vx, const double *vy);

  // Vertices (00, 10, 01, 11) of the cell with unwrapped index (ux, uy):
  // the cell (ux mod ncx, uy mod ncy) moved by whole periods.
  void corners(long ux, long uy, double (&x)[4], double (&y)[4]) const;
};

// Image of (r, s) under the bilinear map of the given corners.
void bilinear_map(const double (&x)[4], const double (&y)[4], double r, double s, double &px,
                  double &py);

// Node coordinates [ny][nx] for support points pts (p + 1 on [0, 1]).
void curvi_node_coords(const CurviMesh &m, const std::vector<double> &pts, std::vector<double> &X,
                       std::vector<double> &Y);

// Integral of each node's shape function over the mesh, [ny][nx]: on a cell
// the local basis l_a(r) l_b(s) times the Jacobian determinant of the
// bilinear map, which is linear in (r, s) (J = J0 + Jr r + Js s), so the
// integral is J0 W_a W_b + Jr W1_a W_b + Js W_a W1_b with W = int l and
// W1 = int r l over [0, 1]; summed over the cells sharing the node.
std::vector<double> curvi_node_mass(const CurviMesh &m, const std::vector<double> &pts);

// Departure records of every node for the displacement (dx, dy) (the
// departure point is x + (dx, dy)): cell[v] = cx | cy << 16, r[v], s[v] in
// [0, 1].  The point is found by a walk from the node's own cell to the
// neighbour beyond whichever straight edge the point lies outside of, then
// Newton's method on that cell's bilinear map.  Returns "" or an error
// message.
std::string curvi_records(const CurviMesh &m, const std::vector<double> &pts,
                          const std::vector<double> &X, const std::vector<double> &Y, double dx,
                          double dy, int32_t *cell, double *r, double *s);

}  // namespace sllbm
