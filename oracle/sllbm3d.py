"""The SLLBM step in three dimensions (oracle; test infrastructure only).

The paper works in 2-D and names the 3-D extension (D3Q125, the tensor
product of three D1Q5 rules) as future work (Sec. IV and V).  This module is
the same method with one more axis, taken literally:

* velocity set: xi_i = (xi_a, xi_b, xi_c), w_i = w_a w_b w_c with the D1Q5
  abscissae and weights of Table I, index i = a + 5 b + 25 c (x, y, z);
* equilibrium: f_eq_i = w_i sum_{n<=4} (1/n!) a_eq^(n) : H^(n)(xi_i)
  (Sec. II.A, eq. (9)) with the coefficients of eq. (10) in three
  components (the same reading of the garbled 4th-order line as in 2-D),
  evaluated as the full contraction over all 3^n index tuples;
* grid: the tensor product of three axes of cells with GLC support points
  (Sec. II.E), node index v = (iz ny + iy) nx + ix;
* stream: departure x - dt xi_i, periodic wrap or zero-gradient clamp per
  axis, brute-force cell search per axis, the product of the three 1-D
  Lagrange bases of the departure cell (eq. (17) with a third factor);
* collide: the isothermal BGK relaxation of Sec. II.D at theta = 1
  (Sec. III.A): f+ = f - (f - f_eq(rho, u))/tau, tau = nu/dt + 1/2.

Populations: array (Q, nnodes), Q = 125.
"""
import itertools
import math

import numpy as np

from .grid import Axis, lagrange_basis
from .velocity import d1q5, delta, hermite_tensor

D3 = 3


def d3q125():
    """xi (125, 3) and w (125,), i = a + 5 b + 25 c."""
    x1, w1 = d1q5()
    xi = np.zeros((125, 3))
    w = np.zeros(125)
    for c in range(5):
        for b in range(5):
            for a in range(5):
                i = a + 5 * b + 25 * c
                xi[i] = (x1[a], x1[b], x1[c])
                w[i] = w1[a] * w1[b] * w1[c]
    return xi, w


def index_tuples3(n):
    """All 3^n index tuples (alpha_1, ..., alpha_n) in {0, 1, 2}^n."""
    return list(itertools.product(range(D3), repeat=n))


def eq_coefficient3(n, idx, rho, u, theta):
    """Component ``idx`` of a_eq^(n) (eq. (10)) with u = (ux, uy, uz)."""
    t = theta - 1.0
    if n == 0:
        return rho
    if n == 1:
        (a,) = idx
        return rho * u[a]
    if n == 2:
        a, b = idx
        return rho * (u[a] * u[b] + t * delta(a, b))
    if n == 3:
        a, b, c = idx
        return rho * (u[a] * u[b] * u[c]
                      + t * (delta(a, b) * u[c] + delta(a, c) * u[b] + delta(b, c) * u[a]))
    if n == 4:
        a, b, c, d = idx
        uu = (delta(a, b) * u[c] * u[d] + delta(a, c) * u[b] * u[d]
              + delta(a, d) * u[b] * u[c] + delta(b, c) * u[a] * u[d]
              + delta(b, d) * u[a] * u[c] + delta(c, d) * u[a] * u[b])
        dd = (delta(a, b) * delta(c, d) + delta(a, c) * delta(b, d)
              + delta(a, d) * delta(b, c))
        return rho * (u[a] * u[b] * u[c] * u[d] + t * uu + t * t * dd)
    raise ValueError("the equilibrium is truncated at 4th order")


def f_eq3(xi, w, rho, ux, uy, uz, theta=1.0):
    """Discrete 4th-order Hermite equilibrium for every velocity, shape (Q, n):
    for each order n and each of the 3^n index tuples the product
    a_eq^(n)[idx] H^(n)[idx](xi_i) / n! is added, then the sum is multiplied
    by w_i."""
    rho = np.atleast_1d(np.asarray(rho))
    u = tuple(np.atleast_1d(np.asarray(v)) for v in (ux, uy, uz))
    theta = np.asarray(theta) * np.ones_like(rho)
    dtype = np.result_type(rho, *u, theta, float)
    xT = np.asarray(xi, dtype=float).T  # (3, Q)
    total = np.zeros((len(w),) + rho.shape, dtype=dtype)
    for n in range(5):
        for idx in index_tuples3(n):
            h = hermite_tensor(n, idx, xT)
            a = eq_coefficient3(n, idx, rho, u, theta)
            total = total + np.multiply.outer(h, a) / math.factorial(n)
    return np.asarray(w, dtype=float)[:, None] * total


class Grid3:
    """Tensor product of three axes; nodes v = (iz * ny + iy) * nx + ix."""

    def __init__(self, edges_x, edges_y, edges_z, p, periodic, kind="glc"):
        px, py, pz = periodic
        self.ax = Axis(edges_x, p, px, kind)
        self.ay = Axis(edges_y, p, py, kind)
        self.az = Axis(edges_z, p, pz, kind)
        self.p = p
        self.nx, self.ny, self.nz = self.ax.n, self.ay.n, self.az.n
        self.nnodes = self.nx * self.ny * self.nz

    def coords(self):
        Z, Y, X = np.meshgrid(self.az.node_coords(), self.ay.node_coords(),
                              self.ax.node_coords(), indexing="ij")
        return X.reshape(-1), Y.reshape(-1), Z.reshape(-1)

    def node_mass(self):
        mz, my, mx = self.az.node_mass(), self.ay.node_mass(), self.ax.node_mass()
        return (mz[:, None, None] * my[None, :, None] * mx[None, None, :]).reshape(-1)


class Sim3:
    """Isothermal D3Q125 SLLBM (theta = 1, c_s = 1)."""

    def __init__(self, grid, dt, nu):
        self.grid = grid
        self.dt = float(dt)
        self.nu = float(nu)
        self.xi, self.w = d3q125()
        self.Q = 125
        self.tau = np.inf if np.isinf(self.nu) else self.nu / self.dt + 0.5
        self.omega = 0.0 if np.isinf(self.tau) else 1.0 / self.tau
        self.X, self.Y, self.Z = grid.coords()

    def init(self, rho, ux, uy, uz):
        return f_eq3(self.xi, self.w, rho, ux, uy, uz)

    def departure_stencil(self, i, nodes):
        """Source nodes and weights (p+1, p+1, p+1, n) of the departure points
        of velocity i at the selected nodes ([a][b][c]: x, y, z offsets)."""
        g = self.grid
        xd = g.ax.apply_boundary(self.X[nodes] - self.dt * self.xi[i, 0])
        yd = g.ay.apply_boundary(self.Y[nodes] - self.dt * self.xi[i, 1])
        zd = g.az.apply_boundary(self.Z[nodes] - self.dt * self.xi[i, 2])
        cx, rx = g.ax.locate(xd)
        cy, ry = g.ay.locate(yd)
        cz, rz = g.az.locate(zd)
        lx = lagrange_basis(g.ax.r, rx)
        ly = lagrange_basis(g.ay.r, ry)
        lz = lagrange_basis(g.az.r, rz)
        P1 = g.p + 1
        src = np.zeros((P1, P1, P1, len(nodes)), dtype=np.int64)
        wgt = np.zeros((P1, P1, P1, len(nodes)))
        for a in range(P1):
            for b in range(P1):
                for c in range(P1):
                    src[a, b, c] = ((g.az.node_of(cz, c) * g.ny + g.ay.node_of(cy, b)) * g.nx
                                    + g.ax.node_of(cx, a))
                    wgt[a, b, c] = lx[a] * ly[b] * lz[c]
        return src, wgt

    def stream(self, F, nodes=None):
        """Values of the interpolant of F at the departure points; the stencils
        of all nodes are located once (the grid and dt do not change)."""
        if nodes is None:
            if not hasattr(self, "_all"):
                every = np.arange(self.grid.nnodes)
                self._all = [self.departure_stencil(i, every) for i in range(self.Q)]
            stencils = self._all
        else:
            stencils = [self.departure_stencil(i, np.asarray(nodes)) for i in range(self.Q)]
        out = np.zeros((self.Q, stencils[0][0].shape[-1]), dtype=F.dtype)
        for i, (src, wgt) in enumerate(stencils):
            out[i] = (wgt * F[i, src]).sum(axis=(0, 1, 2))
        return out

    def moments(self, F):
        """rho, u_x, u_y, u_z (eqs. (3)-(4))."""
        rho = F.sum(axis=0)
        u = [(self.xi[:, k, None] * F).sum(axis=0) / rho for k in range(3)]
        return rho, u[0], u[1], u[2]

    def collide(self, F):
        rho, ux, uy, uz = self.moments(F)
        return F - self.omega * (F - f_eq3(self.xi, self.w, rho, ux, uy, uz))

    def step(self, F, nodes=None):
        return self.collide(self.stream(F, nodes))

    def run(self, F, nsteps):
        for _ in range(nsteps):
            F = self.step(F)
        return F

    def mass(self, F):
        return float(np.sum(self.grid.node_mass() * F.sum(axis=0)))
