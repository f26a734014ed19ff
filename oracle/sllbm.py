"""One SLLBM time step, literally (oracle; test infrastructure only).

Order of operations per step (Sec. II.D eq. (16) and Sec. II.E eq. (17)), with
the reading that the collision is applied at the nodes and the post-collision
field is what gets interpolated (so f, f_eq and f* "at x - dt xi_i" in eq. (16)
are values of the interpolant of the nodal post-collision populations):

1. stream: for every node x and velocity xi_i, the departure point
   x - dt xi_i is moved back into the domain (periodic wrap, or zero-gradient
   clamp to the boundary), its cell is found by brute force, and the cell's
   Lagrange interpolant of the post-collision populations f+_i of the previous
   step is evaluated there, eq. (17);
2. moments of the streamed populations, eqs. (3)-(5): rho = sum f,
   rho u = sum xi f, 2 rho E = sum (|xi|^2 f + g);
3. temperature: theta = (2 rho E - rho |u|^2) / (2 C_v rho); for a single
   population (monatomic gas, C_v = D/2) the g sum is absent; isothermal
   models fix theta = 1 (Sec. III.A);
4. BGK relaxation toward the 4th-order equilibrium with
   tau = nu / (c_s^2 dt) + 1/2 (Sec. II.D), plus the quasi-equilibrium term of
   eq. (16) with tau_Pr = (tau - 1/2)/Pr + 1/2 (Sec. II.C):
   f+ = f - (f - f_eq)/tau + (1/tau - 1/tau_Pr) f*, likewise for g; with
   Pr = 1 the term vanishes.  Reading of the garbled f* of Sec. II.C:
   f*_i = (w_i / 3!) Qneq : H^(3)(xi_i) with c_s = 1 (the third-order term of
   the Hermite expansion, whose 1/n! the printed formula drops), and
   Qneq = Q - Q_eq, Q = sum_i f_i (xi_i - u)^(x3) the centred third moment;
   g* the same with g and its own Q.

A scaled velocity set (Sec. II.B, c_s != 1) streams with xi = c_s xi_hat and
expands the equilibrium in xi_hat, u / c_s and theta = T / T0 with T0 = c_s^2
(readings S3/S4); every input and output here is in physical units.

Populations are stored as an array of shape (S, Q, nnodes) with S = 1 (f) or
S = 2 (f, g) and node index v = iy * nx + ix.
"""
import math

import numpy as np

from .equilibrium import cv_of_gamma, f_eq, g_eq
from .grid import lagrange_basis
from .velocity import D, d1q5, hermite_tensor, index_tuples, tensor_product

MODELS = ("isothermal", "monatomic", "polyatomic")


class Sim:
    def __init__(self, grid, dt, nu, model, gamma=1.4, xi1=None, w1=None, Pr=1.0, cs=1.0):
        if model not in MODELS:
            raise ValueError(model)
        self.grid = grid
        self.dt = float(dt)
        self.nu = float(nu)
        self.model = model
        if xi1 is None:
            xi1, w1 = d1q5()
        # Sec. II.B: the abscissae are given for c_s = 1 "unless scaled"; a
        # scaled set has physical velocities xi = c_s xi_hat, and the Hermite
        # expansion of Sec. II.A is in the normalised velocity xi_hat with the
        # reference temperature T0 = c_s^2 (c_s^2 = R T0, R = 1)
        self.cs = float(cs)
        self.T0 = self.cs ** 2
        xi_hat, self.w = tensor_product(np.asarray(xi1, float), np.asarray(w1, float))
        self.xi_hat = xi_hat
        self.xi = self.cs * xi_hat
        self.Q = len(self.w)
        # relaxation time tau = nu/(c_s^2 dt) + 1/2 (Sec. II.D);
        # nu = inf means pure streaming (1/tau = 0)
        self.tau = np.inf if np.isinf(self.nu) else self.nu / (self.cs ** 2 * self.dt) + 0.5
        self.omega = 0.0 if np.isinf(self.tau) else 1.0 / self.tau
        # Sec. II.D: tau_Pr = (tau - 1/2)/Pr + 1/2
        self.Pr = float(Pr)
        self.omega_pr = 0.0 if np.isinf(self.tau) else 1.0 / ((self.tau - 0.5) / self.Pr + 0.5)
        if model == "polyatomic":
            self.gamma = float(gamma)
            self.cv = cv_of_gamma(self.gamma)
            self.S = 2
        elif model == "monatomic":
            self.cv = D / 2.0
            self.gamma = 1.0 + 1.0 / self.cv
            self.S = 1
        else:
            self.cv = None
            self.gamma = None
            self.S = 1
        self.X, self.Y = grid.coords()

    # ---- equilibrium and initialisation -------------------------------------------
    def equilibrium(self, rho, ux, uy, T):
        """f_eq of eq. (9) in the normalised variables xi_hat = xi / c_s,
        u / c_s and theta = T / T0, and g_eq = (2 C_v - D) T f_eq (R = 1)."""
        c = self.cs
        feq = f_eq(self.xi_hat, self.w, rho, ux / c, uy / c, T / self.T0)
        if self.S == 1:
            return feq[None]
        return np.stack([feq, g_eq(feq, T, self.gamma)])

    def init(self, rho, ux, uy, T):
        """Populations at equilibrium with the given node fields (the paper is
        silent on initialisation; f = f_eq and g = g_eq is the reading used).
        The isothermal model sits at the reference temperature T0."""
        T = self.T0 * np.ones_like(rho) if self.model == "isothermal" else T
        return self.equilibrium(rho, ux, uy, T)

    # ---- streaming ------------------------------------------------------------
    def departure_stencil(self, i, nodes):
        """For velocity i and the selected nodes: source node indices (p+1, p+1, n)
        and interpolation weights (p+1, p+1, n) of the departure point."""
        g = self.grid
        xd = g.ax.apply_boundary(self.X[nodes] - self.dt * self.xi[i, 0])
        yd = g.ay.apply_boundary(self.Y[nodes] - self.dt * self.xi[i, 1])
        cx, rx = g.ax.locate(xd)
        cy, ry = g.ay.locate(yd)
        lx = lagrange_basis(g.ax.r, rx)
        ly = lagrange_basis(g.ay.r, ry)
        P1 = g.p + 1
        src = np.zeros((P1, P1, len(nodes)), dtype=np.int64)
        wgt = np.zeros((P1, P1, len(nodes)))
        for a in range(P1):
            for b in range(P1):
                src[a, b] = g.ay.node_of(cy, b) * g.nx + g.ax.node_of(cx, a)
                wgt[a, b] = lx[a] * ly[b]
        return src, wgt

    def stream(self, F, nodes=None):
        """Values of the interpolant of F at the departure points, eq. (17)."""
        if nodes is None:
            nodes = np.arange(self.grid.nnodes)
        nodes = np.asarray(nodes)
        out = np.zeros((F.shape[0], self.Q, len(nodes)), dtype=F.dtype)
        for i in range(self.Q):
            src, wgt = self.departure_stencil(i, nodes)
            acc = np.zeros((F.shape[0], len(nodes)), dtype=F.dtype)
            for a in range(self.grid.p + 1):
                for b in range(self.grid.p + 1):
                    acc = acc + wgt[a, b] * F[:, i, src[a, b]]
            out[:, i] = acc
        return out

    # ---- moments and collision --------------------------------------------------
    def moments(self, F):
        """rho, u_x, u_y, theta of a population array (S, Q, n), eqs. (3)-(5)."""
        f = F[0]
        rho = f.sum(axis=0)
        jx = (self.xi[:, 0, None] * f).sum(axis=0)
        jy = (self.xi[:, 1, None] * f).sum(axis=0)
        ux = jx / rho
        uy = jy / rho
        if self.model == "isothermal":
            theta = self.T0 * np.ones_like(rho)
        else:
            two_rho_e = ((self.xi[:, 0] ** 2 + self.xi[:, 1] ** 2)[:, None] * f).sum(axis=0)
            if self.S == 2:
                two_rho_e = two_rho_e + F[1].sum(axis=0)
            theta = (two_rho_e - rho * (ux * ux + uy * uy)) / (2.0 * self.cv * rho)
        return rho, ux, uy, theta

    def centred_third_moment(self, f, ux, uy):
        """Q[a][b][c] = sum_i f_i (xi_i - u)_a (xi_i - u)_b (xi_i - u)_c for
        every node (Sec. II.C), shape (2, 2, 2, n)."""
        c = np.stack([self.xi[:, 0, None] - ux[None], self.xi[:, 1, None] - uy[None]])  # (2, Q, n)
        Q = np.zeros((2, 2, 2) + f.shape[1:], dtype=np.result_type(f, c))
        for a in range(2):
            for b in range(2):
                for d in range(2):
                    Q[a, b, d] = (f * c[a] * c[b] * c[d]).sum(axis=0)
        return Q

    def quasi_equilibrium(self, Qneq):
        """f*_i = (w_i / 3!) Qneq : H^(3)(xi_i) (reading of Sec. II.C) in the
        normalised velocities (Qneq / c_s^3 against H^(3)(xi_hat)), shape (Q, n)."""
        xT = self.xi_hat.T
        Qh = Qneq / self.cs ** 3
        total = np.zeros((self.Q,) + Qneq.shape[3:], dtype=Qneq.dtype)
        for idx in index_tuples(3):
            total = total + np.multiply.outer(hermite_tensor(3, idx, xT), Qh[idx])
        return self.w[:, None] * total / math.factorial(3)

    def collide(self, F):
        """BGK relaxation at the nodes with the quasi-equilibrium term, eq. (16)."""
        rho, ux, uy, theta = self.moments(F)
        feq = self.equilibrium(rho, ux, uy, theta)
        out = F - self.omega * (F - feq)
        if self.Pr != 1.0:
            for s in range(self.S):
                Qneq = (self.centred_third_moment(F[s], ux, uy)
                        - self.centred_third_moment(feq[s], ux, uy))
                out[s] = out[s] + (self.omega - self.omega_pr) * self.quasi_equilibrium(Qneq)
        return out

    def step(self, F, nodes=None):
        """One full time step; with ``nodes`` only those nodes' new values are returned."""
        return self.collide(self.stream(F, nodes))

    def run(self, F, nsteps):
        for _ in range(nsteps):
            F = self.step(F)
        return F

    # ---- outputs ---------------------------------------------------------------
    def macro(self, F):
        """rho, u_x, u_y, T per node (physical units; R = 1)."""
        return self.moments(F)

    def mass(self, F):
        """Integral of the interpolated density: sum_v M_v rho_v."""
        rho = F[0].sum(axis=0)
        return float(np.sum(self.grid.node_mass() * rho))

    def unstable(self, F):
        """The paper's stability criterion: all macroscopic values bounded."""
        rho, ux, uy, theta = self.moments(F)
        ok = np.all(np.isfinite(rho)) and np.all(np.isfinite(ux)) and np.all(np.isfinite(uy))
        ok = ok and np.all(np.isfinite(theta)) and np.all(rho > 0) and np.all(theta > 0)
        return not ok
