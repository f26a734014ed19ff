"""Curvilinear 2-D cells for the semi-Lagrangian step (oracle; test
infrastructure only).

The paper's interpolation (Sec. II.E, eq. (17)) is written for cells that are
images of a reference square under a map; its grids are axis products, and
curved cells are the generalisation it names as future work.  Here each cell
is the bilinear image of the unit reference square [0, 1]^2 spanned by its four
vertices,

    x(r, s) = (1-r)(1-s) v00 + r(1-s) v10 + (1-r) s v01 + r s v11,

and the support points inside it are the images of the tensor-product support
points (r_a, s_b).  Cells share edges, so the outer support points are shared
as on the axis-product grids.  The domain is periodic in both directions with
periods Lx, Ly: vertex column ncx is vertex column 0 moved by (Lx, 0) and
vertex row ncy is row 0 moved by (0, Ly).

Streaming evaluates, for each node x and velocity xi_i, the cell interpolant
of the post-collision populations at the departure point x - dt xi_i.  The
departure point is located by brute force: for every cell and every periodic
image the bilinear map is inverted in closed form (a quadratic in s, below),
and the first cell whose reference coordinates fall in [0, 1]^2 is taken.  On
a shared edge every containing cell gives the same value (the interpolant is
continuous there), so the choice does not matter beyond rounding.

Inversion.  With A0 = v00, A1 = v10 - v00, A2 = v01 - v00,
A3 = v00 - v10 - v01 + v11 the map is x = A0 + A1 r + A2 s + A3 r s.  For a
point P put Q = P - A0; the 2-D cross product of Q - A2 s with A1 + A3 s must
vanish, which is the quadratic
    -(A2 x A3) s^2 + (Q x A3 - A2 x A1) s + Q x A1 = 0,
and r follows by projecting Q - A2 s onto A1 + A3 s.

Nothing here is fast; it is written to be checked by eye.
"""
import numpy as np

from .grid import lagrange_basis, support_points
from .sllbm import Sim


def _cross(ax, ay, bx, by):
    return ax * by - ay * bx


def bilinear(v, r, s):
    """Image of (r, s) under the cell map; v = ((x00, y00), (x10, y10), (x01, y01), (x11, y11))."""
    (x00, y00), (x10, y10), (x01, y01), (x11, y11) = v
    x = (1 - r) * (1 - s) * x00 + r * (1 - s) * x10 + (1 - r) * s * x01 + r * s * x11
    y = (1 - r) * (1 - s) * y00 + r * (1 - s) * y10 + (1 - r) * s * y01 + r * s * y11
    return x, y


def invert_bilinear(v, px, py):
    """Reference coordinates (r, s) of the points (px, py) under the cell map,
    in closed form; of the two roots of the quadratic the one nearer the unit
    interval is returned (NaN where the quadratic has no real root)."""
    (x00, y00), (x10, y10), (x01, y01), (x11, y11) = v
    a1x, a1y = x10 - x00, y10 - y00
    a2x, a2y = x01 - x00, y01 - y00
    a3x, a3y = x00 - x10 - x01 + x11, y00 - y10 - y01 + y11
    qx, qy = px - x00, py - y00
    alpha = -_cross(a2x, a2y, a3x, a3y)
    beta = _cross(qx, qy, a3x, a3y) - _cross(a2x, a2y, a1x, a1y)
    gamma = _cross(qx, qy, a1x, a1y)
    scale = abs(_cross(a1x, a1y, a2x, a2y))
    if abs(alpha) <= 1e-14 * scale:  # parallelogram: the equation is linear
        s = -gamma / beta
    else:
        disc = beta * beta - 4 * alpha * gamma
        root = np.sqrt(np.where(disc >= 0, disc, np.nan))
        q = -0.5 * (beta + np.where(beta >= 0, 1.0, -1.0) * root)
        s1 = q / alpha
        with np.errstate(divide="ignore", invalid="ignore"):
            s2 = np.where(q != 0, gamma / q, s1)
        d1 = np.maximum(0, np.maximum(-s1, s1 - 1))
        d2 = np.maximum(0, np.maximum(-s2, s2 - 1))
        s = np.where(d2 < d1, s2, s1)
    dx, dy = a1x + a3x * s, a1y + a3y * s
    r = ((qx - a2x * s) * dx + (qy - a2y * s) * dy) / (dx * dx + dy * dy)
    return r, s


class CurviGrid:
    """Bilinear cells from vertex arrays vx, vy of shape (ncy + 1, ncx + 1),
    periodic in x and y; nodes numbered v = iy * nx + ix with nx = ncx p and
    ny = ncy p (the vertex column / row ncx, ncy is the periodic image of 0)."""

    def __init__(self, vx, vy, p, kind="glc"):
        self.vx = np.asarray(vx, dtype=float)
        self.vy = np.asarray(vy, dtype=float)
        self.ncy, self.ncx = self.vx.shape[0] - 1, self.vx.shape[1] - 1
        self.p = p
        self.r = support_points(p, kind)
        self.nx = self.ncx * p
        self.ny = self.ncy * p
        self.nnodes = self.nx * self.ny
        self.Lx = self.vx[0, -1] - self.vx[0, 0]
        self.Ly = self.vy[-1, 0] - self.vy[0, 0]

    def cell_vertices(self, cx, cy):
        vx, vy = self.vx, self.vy
        return ((vx[cy, cx], vy[cy, cx]), (vx[cy, cx + 1], vy[cy, cx + 1]),
                (vx[cy + 1, cx], vy[cy + 1, cx]), (vx[cy + 1, cx + 1], vy[cy + 1, cx + 1]))

    def coords(self):
        """Node coordinates: node (ix, iy) is support point (ix mod p, iy mod p)
        of cell (ix // p, iy // p)."""
        X = np.zeros(self.nnodes)
        Y = np.zeros(self.nnodes)
        for iy in range(self.ny):
            for ix in range(self.nx):
                v = self.cell_vertices(ix // self.p, iy // self.p)
                X[iy * self.nx + ix], Y[iy * self.nx + ix] = bilinear(
                    v, self.r[ix % self.p], self.r[iy % self.p])
        return X, Y

    def node_of(self, cx, cy, a, b):
        return ((cy * self.p + b) % self.ny) * self.nx + (cx * self.p + a) % self.nx

    def locate(self, px, py, tol=1e-12):
        """Cell (cx, cy) and reference coordinates (r, s) in [0, 1] of each
        point, by brute force over every cell and the periodic images up to
        two periods away."""
        n = len(px)
        cx = np.full(n, -1, dtype=np.int64)
        cy = np.full(n, -1, dtype=np.int64)
        r = np.zeros(n)
        s = np.zeros(n)
        for ky in (0, -1, 1, -2, 2):
            for kx in (0, -1, 1, -2, 2):
                qx, qy = px - kx * self.Lx, py - ky * self.Ly
                for j in range(self.ncy):
                    for i in range(self.ncx):
                        rr, ss = invert_bilinear(self.cell_vertices(i, j), qx, qy)
                        inside = ((rr >= -tol) & (rr <= 1 + tol) & (ss >= -tol) & (ss <= 1 + tol)
                                  & (cx < 0))
                        cx[inside], cy[inside] = i, j
                        r[inside], s[inside] = rr[inside], ss[inside]
        if (cx < 0).any():
            raise ValueError("departure point outside every cell and periodic image")
        return cx, cy, np.clip(r, 0.0, 1.0), np.clip(s, 0.0, 1.0)

    def node_mass(self, nquad=8):
        """Integral of each node's shape function over the mesh (the mass
        weights of the mass monitor, Sec. III.E): on every cell the local
        basis l_a(r) l_b(s) times the Jacobian determinant of the bilinear
        map, integrated over the reference square by tensor Gauss-Legendre
        quadrature (nquad points per axis), summed over the cells that share
        the node."""
        g, gw = np.polynomial.legendre.leggauss(nquad)
        q = 0.5 * (g + 1.0)
        qw = 0.5 * gw
        R, S = np.meshgrid(q, q, indexing="ij")
        Wq = np.outer(qw, qw)
        lr = lagrange_basis(self.r, R)  # (p+1, nquad, nquad)
        ls = lagrange_basis(self.r, S)
        M = np.zeros(self.nnodes)
        for cy in range(self.ncy):
            for cx in range(self.ncx):
                (x00, y00), (x10, y10), (x01, y01), (x11, y11) = self.cell_vertices(cx, cy)
                # partial derivatives of the bilinear map at the quadrature points
                dxdr = (1 - S) * (x10 - x00) + S * (x11 - x01)
                dydr = (1 - S) * (y10 - y00) + S * (y11 - y01)
                dxds = (1 - R) * (x01 - x00) + R * (x11 - x10)
                dyds = (1 - R) * (y01 - y00) + R * (y11 - y10)
                J = np.abs(dxdr * dyds - dxds * dydr)
                for a in range(self.p + 1):
                    for b in range(self.p + 1):
                        M[self.node_of(cx, cy, a, b)] += np.sum(lr[a] * ls[b] * J * Wq)
        return M

    def stencil(self, px, py):
        """Source nodes (p+1, p+1, n) and weights (p+1, p+1, n) of the cell
        interpolant at the points, eq. (17) on the reference square."""
        cx, cy, r, s = self.locate(px, py)
        lr = lagrange_basis(self.r, r)
        ls = lagrange_basis(self.r, s)
        P1 = self.p + 1
        src = np.zeros((P1, P1, len(px)), dtype=np.int64)
        wgt = np.zeros((P1, P1, len(px)))
        for a in range(P1):
            for b in range(P1):
                src[a, b] = self.node_of(cx, cy, a, b)
                wgt[a, b] = lr[a] * ls[b]
        return src, wgt


class CurviSim(Sim):
    """The oracle step of Sim (moments, equilibrium, collision unchanged) with
    the departure points interpolated on curvilinear cells.  The stencils of
    all nodes are located once, for all velocities together (the grid and
    dt do not change)."""

    def departure_stencil(self, i, nodes):
        nodes = np.asarray(nodes)
        if not hasattr(self, "_all"):
            n = self.grid.nnodes
            px = np.concatenate([self.X - self.dt * self.xi[k, 0] for k in range(self.Q)])
            py = np.concatenate([self.Y - self.dt * self.xi[k, 1] for k in range(self.Q)])
            src, wgt = self.grid.stencil(px, py)
            self._all = [(src[:, :, k * n:(k + 1) * n], wgt[:, :, k * n:(k + 1) * n])
                         for k in range(self.Q)]
        src, wgt = self._all[i]
        return src[:, :, nodes], wgt[:, :, nodes]


def wavy_vertices(ncx, ncy, Lx, Ly, amp):
    """Periodic test mesh: the uniform vertex lattice of [0, Lx] x [0, Ly]
    with both coordinates moved by
        d = amp min(Lx, Ly) / (2 pi) sin(2 pi X / Lx) sin(2 pi Y / Ly);
    the Jacobian of the continuous map is 1 + dd/dX + dd/dY >= 1 - 2 amp for
    Lx = Ly, so amp < 1/2 keeps it invertible."""
    X, Y = np.meshgrid(np.linspace(0, Lx, ncx + 1), np.linspace(0, Ly, ncy + 1))
    d = amp * min(Lx, Ly) / (2 * np.pi) * np.sin(2 * np.pi * X / Lx) * np.sin(2 * np.pi * Y / Ly)
    return X + d, Y + d
