"""Cells, support points, Lagrange shape functions (oracle; test infrastructure only).

Sec. II.E: the domain is split into cells; inside each cell the distribution is
represented by Lagrange polynomials of order p on support points, eq. (17).
The support points are Gauss-Lobatto-Chebyshev points,

    x_k = (1 - cos((k - 1) pi / (n - 1))) / 2,   k = 1..n,  n = p + 1,

on the unit reference interval (equidistant points are kept as a switch, the
paper's unstable comparison case).  The outer support points are shared with
the neighbouring cell (caption of the shock-vortex grid figure, Sec. III.E), so
an axis with N_c cells carries N_c p unique nodes if periodic and N_c p + 1
otherwise.

The 2-D grid is the tensor product of two 1-D axes; each axis is a list of cell
edges, so uniform grids and the transformed grid of Sec. III.E (a map applied
per axis) are both covered.  Inside a cell the map from the reference interval
is affine.

Everything here works with absolute coordinates and brute-force searches; it
is meant to be checked by eye, not to be fast.
"""
import numpy as np


def support_points(p, kind="glc"):
    """Reference-cell support points for order p (Sec. II.E)."""
    n = p + 1
    k = np.arange(1, n + 1)
    if kind == "glc":
        return 0.5 * (1.0 - np.cos((k - 1) * np.pi / (n - 1)))
    if kind == "equidistant":
        return (k - 1) / (n - 1)
    raise ValueError(kind)


def lagrange_basis(r_nodes, r):
    """Values of all Lagrange polynomials l_m(r) = prod_{n != m} (r - r_n)/(r_m - r_n).

    r may be an array; returns shape (p+1,) + r.shape.
    """
    r = np.asarray(r)
    out = []
    for m in range(len(r_nodes)):
        val = np.ones_like(r, dtype=np.result_type(r, float))
        for n in range(len(r_nodes)):
            if n != m:
                val = val * (r - r_nodes[n]) / (r_nodes[m] - r_nodes[n])
        out.append(val)
    return np.array(out)


def basis_integrals(r_nodes):
    """Exact integrals over [0, 1] of each Lagrange polynomial (Gauss-Legendre, 8 points)."""
    g, gw = np.polynomial.legendre.leggauss(8)
    s = 0.5 * (g + 1.0)
    return (lagrange_basis(r_nodes, s) * (0.5 * gw)).sum(axis=1)


class Axis:
    """One grid direction: cell edges, order, boundary kind."""

    def __init__(self, edges, p, periodic, kind="glc"):
        self.edges = np.asarray(edges, dtype=float)
        self.ncells = len(self.edges) - 1
        self.p = p
        self.periodic = bool(periodic)
        self.r = support_points(p, kind)
        self.n = self.ncells * p if self.periodic else self.ncells * p + 1
        self.lo = self.edges[0]
        self.hi = self.edges[-1]
        self.length = self.hi - self.lo

    def node_coords(self):
        x = np.zeros(self.n)
        for c in range(self.ncells):
            h = self.edges[c + 1] - self.edges[c]
            for a in range(self.p + 1):
                j = c * self.p + a
                if j < self.n:
                    x[j] = self.edges[c] + self.r[a] * h
        return x

    def node_of(self, cell, a):
        j = cell * self.p + a
        return np.mod(j, self.n) if self.periodic else j

    def apply_boundary(self, x):
        """Periodic wrap into [lo, hi) or zero-gradient clamp into [lo, hi]."""
        if self.periodic:
            return self.lo + np.mod(x - self.lo, self.length)
        return np.clip(x, self.lo, self.hi)

    def locate(self, x):
        """Brute-force cell search: the cell index is the number of interior
        edges at or left of x (so x == hi falls in the last cell with r = 1);
        returns (cell, reference coordinate r in [0, 1])."""
        x = np.asarray(x, dtype=float)
        cell = np.zeros(x.shape, dtype=np.int64)
        for k in range(1, self.ncells):
            cell += (x >= self.edges[k]).astype(np.int64)
        left = self.edges[cell]
        right = self.edges[cell + 1]
        r = (x - left) / (right - left)
        return cell, r

    def node_mass(self):
        """Integral of each global shape function along this axis."""
        W = basis_integrals(self.r)
        m = np.zeros(self.n)
        for c in range(self.ncells):
            h = self.edges[c + 1] - self.edges[c]
            for a in range(self.p + 1):
                m[self.node_of(c, a)] += W[a] * h
        return m


class Grid:
    """Tensor-product grid; nodes are numbered v = iy * nx + ix."""

    def __init__(self, edges_x, edges_y, p, periodic_x, periodic_y, kind="glc"):
        self.ax = Axis(edges_x, p, periodic_x, kind)
        self.ay = Axis(edges_y, p, periodic_y, kind)
        self.p = p
        self.nx = self.ax.n
        self.ny = self.ay.n
        self.nnodes = self.nx * self.ny

    def coords(self):
        x = self.ax.node_coords()
        y = self.ay.node_coords()
        X = np.tile(x, self.ny)
        Y = np.repeat(y, self.nx)
        return X, Y

    def node_mass(self):
        return np.outer(self.ay.node_mass(), self.ax.node_mass()).reshape(-1)


def uniform_edges(ncells, lo, hi):
    return lo + (hi - lo) * np.arange(ncells + 1) / ncells
