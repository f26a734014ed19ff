"""Seeded, synthetic workloads shaped like the paper's test cases.

This module only describes problems: domains, cell edges, orders, boundary
kinds, physical parameters and initial macroscopic fields evaluated at given
node coordinates.  It holds none of the lattice Boltzmann arithmetic (no
velocity set, no equilibrium, no interpolation), so both the HIP path and the
CPU oracle can draw their inputs from it.

Units are code units with c_s = R = T0 = 1, so the pressure is P = rho T.
Time steps follow a CFL number of 0.5 on the smallest node spacing,
CFL = dt * XI_MAX / dx_min, with XI_MAX the largest D1Q5 speed; when an end
time is given the step count is rounded up and dt shrunk to hit it exactly.

Shapes (Sec. III of arXiv:1910.13918):
* ``tgv``      -- Taylor-Green vortex, periodic [0, 2 pi]^2 (Sec. III.A);
* ``sod``      -- Sod shock tube as a quasi-1-D strip (Sec. III.C, with the
                  standard 1 / 0.125 density and 1 / 0.1 pressure ratios);
* ``riemann``  -- four-quadrant Riemann problem on [0, 1]^2 with zero-gradient
                  boundaries (Sec. III.D) and seeded quadrant states;
* ``svi``      -- stationary normal shock plus an isentropic vortex on a grid
                  stretched in x by the sinusoidal map of Sec. III.E;
* ``smooth_density`` -- density wave advected at constant velocity and
                  pressure (Sec. III.B).
"""
import math
from dataclasses import dataclass, field
from typing import Callable, Optional

import numpy as np

XI_MAX = 2.8569700138728056  # sqrt(5 + sqrt(10)), largest D1Q5 speed (CFL definition)
# smallest gap between neighbouring Gauss-Lobatto-Chebyshev points of a unit cell, per order
GLC_MIN_GAP = {1: 1.0, 2: 0.5, 3: 0.25, 4: 0.14644660940672627}


def cfl_time_step(dx_min, cfl=0.5, t_end=None, steps=None):
    dt = cfl * dx_min / XI_MAX
    if t_end is not None:
        n = int(math.ceil(t_end / dt - 1e-9))
        return t_end / n, n
    return dt, steps


def uniform_edges(ncells, lo, hi):
    return lo + (hi - lo) * np.arange(ncells + 1, dtype=float) / ncells


@dataclass
class Workload:
    name: str
    edges_x: np.ndarray
    edges_y: np.ndarray
    p: int
    periodic_x: bool
    periodic_y: bool
    model: str            # "isothermal" | "monatomic" | "polyatomic"
    gamma: float
    nu: float
    dt: float
    steps: int
    fields: Callable      # (x, y) -> rho, ux, uy, T
    uniform: bool = True
    meta: dict = field(default_factory=dict)
    Pr: float = 1.0       # Prandtl number (Sec. II.C-D)
    vertices: tuple = None  # (vx, vy) [ncy + 1][ncx + 1] of a curvilinear mesh, else None
    q1: int = 5           # velocities per axis of the tensor-product set (5: D2Q25, 3: D2Q9)
    cs: float = 1.0       # scale of the velocity set (Sec. II.B; 1: unscaled)

    @property
    def ncx(self):
        return len(self.edges_x) - 1

    @property
    def ncy(self):
        return len(self.edges_y) - 1

    @property
    def nx(self):
        return self.ncx * self.p + (0 if self.periodic_x else 1)

    @property
    def ny(self):
        return self.ncy * self.p + (0 if self.periodic_y else 1)

    @property
    def nnodes(self):
        return self.nx * self.ny

    @property
    def nsets(self):
        return 2 if self.model == "polyatomic" else 1


# ---------------------------------------------------------------------------- TGV
def tgv(ncells=8, p=2, U0=0.1, Re=100.0, steps=200, cfl=0.5, model="isothermal", name=None):
    """Taylor-Green vortex on [0, 2 pi]^2: u = U0 sin x cos y, v = -U0 cos x sin y,
    rho = 1 + (U0^2 / 4)(cos 2x + cos 2y) (pressure of the closed form with
    P = rho for the isothermal model), nu = U0 * 2 pi / Re."""
    L = 2.0 * np.pi
    h = L / ncells
    dt, n = cfl_time_step(h * GLC_MIN_GAP[p], cfl, steps=steps)
    nu = U0 * L / Re

    def fields(x, y):
        ux = U0 * np.sin(x) * np.cos(y)
        uy = -U0 * np.cos(x) * np.sin(y)
        rho = 1.0 + 0.25 * U0 * U0 * (np.cos(2 * x) + np.cos(2 * y))
        return rho, ux, uy, np.ones_like(x)

    e = uniform_edges(ncells, 0.0, L)
    return Workload(name or f"tgv_{ncells}x{ncells}_p{p}", e, e.copy(), p, True, True, model,
                    1.4, nu, dt, n, fields, True, {"U0": U0, "Re": Re})


# ------------------------------------------ Taylor-Green on a moving frame (Fig. 3)
def tgv_moving(ncells=4, p=4, ma_h=0.0, q1=5, ma_v=0.01, Re=10.0, name=None):
    """The Taylor-Green comparison of Sec. III.A (D2Q9 against D2Q25, Fig. 3):
    vortex Mach number 0.01 (U0 = 0.01 with c_s = 1), Re = U0 2 pi / nu = 10,
    a uniform horizontal velocity u_h = ma_h, and the paper's time step,
    dt = 0.0008 in the paper's time unit (vortex speed 1, length 2 pi) at 4
    cells of order 4 per direction and halved with the cell size, i.e.
    dt = 0.0008 / U0 * 4 / ncells in code units.  The end time is the
    paper's t = 1.83 (vortex speed decayed to 0.1 U0), t = 1.83 / U0 in code
    units, rounded to whole steps.  Isothermal; the exact solution is the
    decaying vortex advected by u_h:
    u = u_h + U0 e^(-2 nu t) sin(x - u_h t) cos y, v = -U0 e^(-2 nu t) cos(x - u_h t) sin y."""
    L = 2.0 * np.pi
    U0 = ma_v
    nu = U0 * L / Re
    dt = 0.0008 / U0 * 4.0 / ncells
    steps = int(round(1.83 / U0 / dt))

    def fields(x, y):
        ux = ma_h + U0 * np.sin(x) * np.cos(y)
        uy = -U0 * np.cos(x) * np.sin(y)
        rho = 1.0 + 0.25 * U0 * U0 * (np.cos(2 * x) + np.cos(2 * y))
        return rho, ux, uy, np.ones_like(x)

    def exact(x, y, t):
        d = U0 * np.exp(-2.0 * nu * t)
        return ma_h + d * np.sin(x - ma_h * t) * np.cos(y), -d * np.cos(x - ma_h * t) * np.sin(y)

    e = uniform_edges(ncells, 0.0, L)
    wl = Workload(name or f"tgv_moving_{ncells}x{ncells}_p{p}_mah{ma_h}_q{q1 * q1}", e, e.copy(),
                  p, True, True, "isothermal", 1.4, nu, dt, steps, fields, True,
                  {"U0": U0, "Re": Re, "ma_h": ma_h, "exact": exact}, q1=q1)
    return wl


# ------------------------------------------------------- Taylor-Green, curved cells
def wavy_vertices(ncx, ncy, Lx, Ly, amp):
    """Vertices [ncy + 1][ncx + 1] of a periodic mesh of bilinear cells: the
    uniform lattice of [0, Lx] x [0, Ly] with both coordinates moved by
    amp min(Lx, Ly) / (2 pi) sin(2 pi X / Lx) sin(2 pi Y / Ly) (for Lx = Ly the
    map's Jacobian is >= 1 - 2 amp, so amp < 1/2 keeps the cells unfolded)."""
    X, Y = np.meshgrid(np.linspace(0.0, Lx, ncx + 1), np.linspace(0.0, Ly, ncy + 1))
    d = amp * min(Lx, Ly) / (2 * np.pi) * np.sin(2 * np.pi * X / Lx) * np.sin(2 * np.pi * Y / Ly)
    return X + d, Y + d


def tgv_wavy(ncells=8, p=2, amp=0.3, U0=0.1, Re=100.0, steps=200, cfl=0.5, model="isothermal",
             name=None):
    """The Taylor-Green vortex of tgv() on a curvilinear periodic mesh of
    ncells^2 bilinear cells (wavy_vertices of [0, 2 pi]^2); dt from the
    uniform spacing shrunk by 1 - amp."""
    wl = tgv(ncells, p, U0=U0, Re=Re, steps=steps, cfl=cfl * (1 - amp), model=model,
             name=name or f"tgv_wavy_{ncells}x{ncells}_p{p}_a{amp}")
    L = 2.0 * np.pi
    wl.vertices = wavy_vertices(ncells, ncells, L, L, amp)
    wl.edges_x = np.arange(ncells + 1, dtype=float)  # logical cells: node counts only
    wl.edges_y = wl.edges_x.copy()
    wl.meta["amp"] = amp
    return wl


# ---------------------------------------------------------------------------- Sod
def sod(ncx=1024, ncy=4, p=3, t_end=0.2, nu=1.2e-4, gamma=1.4, cfl=0.5, name=None):
    """Sod tube on x in [0, 1] (zero-gradient), y periodic with ncy square cells.
    Left (x < 1/2): rho = 1, P = 1; right: rho = 0.125, P = 0.1; u = 0."""
    h = 1.0 / ncx
    dt, n = cfl_time_step(h * GLC_MIN_GAP[p], cfl, t_end=t_end)

    def fields(x, y):
        left = x < 0.5
        rho = np.where(left, 1.0, 0.125)
        P = np.where(left, 1.0, 0.1)
        return rho, np.zeros_like(x), np.zeros_like(x), P / rho

    return Workload(name or f"sod_{ncx}x{ncy}_p{p}", uniform_edges(ncx, 0.0, 1.0),
                    uniform_edges(ncy, 0.0, ncy * h), p, False, True, "polyatomic", gamma,
                    nu, dt, n, fields, True, {"t_end": t_end})


# ------------------------------------------------------------------------- Riemann
# First seed >= 0 whose states survive to t = 0.25 on 64 x 64 cells of order 2
# with the FP64 oracle (search and log: tests/golden/make_riemann_seed.py).
RIEMANN_DEFAULT_SEED = 14

# Quadrant states (NE, NW, SW, SE) of the Lax-Liu configuration printed in
# Table III (Sec. III.D): (rho, u_x, u_y, P).
RIEMANN_TABLE3_STATES = [(0.5313, 0.0, 0.0, 0.4), (1.0, 0.7276, 0.0, 1.0),
                         (0.8, 0.0, 0.0, 1.0), (1.0, 0.0, 0.7276, 1.0)]


def riemann_states(seed):
    """Quadrant states (NE, NW, SW, SE) drawn with numpy's default_rng(seed):
    rho ~ U[0.1, 1.5], P ~ U[0.03, 1.5], |u| ~ U[0, 1.2], angle ~ U[0, 2 pi)."""
    rng = np.random.default_rng(seed)
    states = []
    for _ in range(4):
        rho = rng.uniform(0.1, 1.5)
        P = rng.uniform(0.03, 1.5)
        speed = rng.uniform(0.0, 1.2)
        ang = rng.uniform(0.0, 2.0 * np.pi)
        states.append((rho, speed * np.cos(ang), speed * np.sin(ang), P))
    return states


def riemann(ncells=512, p=2, seed=None, t_end=0.25, nu=1.73e-4, gamma=1.4, cfl=0.5,
            states=None, name=None):
    """Four-quadrant Riemann problem on [0, 1]^2 with zero-gradient boundaries;
    quadrant boundaries at x = 1/2 and y = 1/2 (a node on x = 1/2 or y = 1/2
    takes the state of the upper / right side)."""
    if states is None:
        seed = RIEMANN_DEFAULT_SEED if seed is None else seed
        states = riemann_states(seed)
    h = 1.0 / ncells
    dt, n = cfl_time_step(h * GLC_MIN_GAP[p], cfl, t_end=t_end)

    def fields(x, y):
        east = x >= 0.5
        north = y >= 0.5
        quad = np.where(north, np.where(east, 0, 1), np.where(east, 3, 2))
        tab = np.array(states)
        rho, ux, uy, P = (tab[quad, k] for k in range(4))
        return rho, ux, uy, P / rho

    e = uniform_edges(ncells, 0.0, 1.0)
    return Workload(name or f"riemann_{ncells}x{ncells}_p{p}", e, e.copy(), p, False, False,
                    "polyatomic", gamma, nu, dt, n, fields, True,
                    {"seed": seed, "states": [tuple(map(float, s)) for s in states]})


def riemann_table3_p4(name=None):
    """The four-quadrant configuration of Sec. III.D as printed: Table III
    states, 128 x 128 cells of order 4, t_end = 0.25 in 2091 steps
    (tau = 1.948 with nu = 1.73e-4), zero-gradient boundaries."""
    h = 1.0 / 128
    cfl = 0.25 / 2091 * XI_MAX / (h * GLC_MIN_GAP[4]) * (1.0 + 1e-6)
    wl = riemann(128, 4, states=RIEMANN_TABLE3_STATES, cfl=cfl,
                 name=name or "riemann_table3_128x128_p4")
    assert wl.steps == 2091
    return wl


# ------------------------------------------------------------------ adjoint TGV
def adjoint_tgv(ncells=128, p=4, U0=0.3, Re=100.0, steps=500, cfl=0.5, name=None):
    return tgv(ncells, p, U0, Re, steps, cfl, "isothermal",
               name or f"adjoint_tgv_{ncells}x{ncells}_p{p}")


def fourier_target(x, y, U0, seed=1234, modes=8, kmax=4):
    """Seeded target velocity field: a sum of ``modes`` random Fourier modes with
    integer wave vectors |k| <= kmax and amplitudes below U0."""
    rng = np.random.default_rng(seed)
    ut = np.zeros_like(x)
    vt = np.zeros_like(x)
    for _ in range(modes):
        while True:
            k = rng.integers(-kmax, kmax + 1, size=2)
            if 0 < k[0] ** 2 + k[1] ** 2 <= kmax * kmax:
                break
        amp = rng.uniform(0.0, U0, size=2) / modes
        ph = rng.uniform(0.0, 2.0 * np.pi, size=2)
        arg = k[0] * x + k[1] * y
        ut += amp[0] * np.sin(arg + ph[0])
        vt += amp[1] * np.sin(arg + ph[1])
    return ut, vt


def random_directions(n, count, seed=4321):
    """``count`` seeded unit directions in R^(2n) (for u and v of n nodes)."""
    rng = np.random.default_rng(seed)
    d = rng.standard_normal((count, 2, n))
    d /= np.sqrt((d * d).sum(axis=(1, 2)))[:, None, None]
    return d


# --------------------------------------------------------------------------- SVI
def rankine_hugoniot(mach, gamma=1.4):
    """Downstream/upstream ratios across a normal shock: (rho_B/rho_A, P_B/P_A, Ma_B)."""
    m2 = mach * mach
    rr = (gamma + 1.0) * m2 / ((gamma - 1.0) * m2 + 2.0)
    pr = 1.0 + 2.0 * gamma / (gamma + 1.0) * (m2 - 1.0)
    mb = math.sqrt(((gamma - 1.0) * m2 + 2.0) / (2.0 * gamma * m2 - (gamma - 1.0)))
    return rr, pr, mb


def stretched_edges(ncells, length, lam=0.95):
    """Cell edges of the sinusoidal map of Sec. III.E scaled to [0, length]:
    x_t = (L / 2 pi)(lam sin(2 pi x / L) + 2 pi x / L); cells are finest
    (by the factor 1 - lam) at x = L / 2."""
    x = uniform_edges(ncells, 0.0, length)
    k = 2.0 * np.pi / length
    return (lam * np.sin(k * x) + k * x) / k


def isentropic_vortex(x, y, xc, yc, radius, mach_v, rho_inf, P_inf, u_inf, gamma=1.4):
    """Isentropic vortex of Sec. III.E on a uniform stream (rho_inf, P_inf, u_inf, 0):
    u_theta = c Ma_v r' exp((1 - r'^2)/2), r' = r / radius, c = sqrt(gamma P_inf / rho_inf),
    rho = rho_inf phi^(1/(gamma-1)), P = P_inf phi^(gamma/(gamma-1)),
    phi = 1 - (gamma - 1)/2 Ma_v^2 exp(1 - r'^2)
    (with Ma_v squared, which makes dP/dr = rho u_theta^2 / r hold exactly)."""
    dx = x - xc
    dy = y - yc
    rp = np.sqrt(dx * dx + dy * dy) / radius
    c = math.sqrt(gamma * P_inf / rho_inf)
    ut = c * mach_v * rp * np.exp(0.5 * (1.0 - rp * rp))
    phi = 1.0 - 0.5 * (gamma - 1.0) * mach_v * mach_v * np.exp(1.0 - rp * rp)
    rho = rho_inf * phi ** (1.0 / (gamma - 1.0))
    P = P_inf * phi ** (gamma / (gamma - 1.0))
    r = np.maximum(np.sqrt(dx * dx + dy * dy), 1e-300)
    ux = u_inf - ut * dy / r
    uy = ut * dx / r
    return rho, ux, uy, P


def svi(ncx=1024, ncy=512, p=3, steps=2000, mach_s=1.2, mach_v=0.25, radius=0.075, Re=800.0,
        gamma=1.4, lam=0.8, cfl=0.5, Pr=0.75, name=None):
    """Stationary normal shock at x = 1 on [0, 2] x [0, 1] (x zero-gradient and
    stretched, y periodic), upstream state A (x > 1): rho = 1, T = 1,
    u = -Ma_s sqrt(gamma); downstream state B from Rankine-Hugoniot; an
    isentropic vortex of radius 0.075 centred at (1.15, 0.5) on the upstream
    flow; nu = c_A * radius / Re; Pr = 0.75 as in the paper's shock-vortex
    case.  The x-map uses lam = 0.8 rather than the paper's 0.95: this grid
    is 2-3 times finer per vortex radius than the paper's, and with 0.95 the
    finest cells (0.0013 radii) put the departures of the refined zone five
    node spacings away and the run blows up when the vortex crosses the shock
    (step ~925 of 2000, in FP64 and FP32 alike); with 0.8 (finest cells 0.005
    radii, the paper's 0.012) it runs through."""
    Lx, Ly = 2.0, 1.0
    hx = Lx / ncx
    dt, n = cfl_time_step(hx * GLC_MIN_GAP[p], cfl, steps=steps)
    cA = math.sqrt(gamma)
    uA = -mach_s * cA
    rr, pr, _ = rankine_hugoniot(mach_s, gamma)
    rhoB, PB, uB = rr, pr, uA / rr
    nu = cA * radius / Re

    def fields(x, y):
        rv, uxv, uyv, Pv = isentropic_vortex(x, y, 1.15, 0.5, radius, mach_v, 1.0, 1.0, uA, gamma)
        up = x > 1.0
        rho = np.where(up, rv, rhoB)
        ux = np.where(up, uxv, uB)
        uy = np.where(up, uyv, 0.0)
        P = np.where(up, Pv, PB)
        return rho, ux, uy, P / rho

    return Workload(name or f"svi_{ncx}x{ncy}_p{p}", stretched_edges(ncx, Lx, lam),
                    uniform_edges(ncy, 0.0, Ly), p, False, True, "polyatomic", gamma, nu, dt,
                    n, fields, False, {"mach_s": mach_s, "mach_v": mach_v, "Re": Re}, Pr)


# --------------------------------------------------------------- smooth density
def smooth_density(ncells=4, p=4, t_end=2.0, ux0=1.0, nu=1e-10, gamma=1.4, cfl=0.5,
                   steps: Optional[int] = None, name=None):
    """rho = 1 + 0.2 sin(pi (x - ux0 t)) sin(pi y), u = (ux0, 0), P = 1 on
    [-1, 1]^2 periodic (Sec. III.B); the exact solution is pure advection."""
    h = 2.0 / ncells
    if steps is None:
        dt, n = cfl_time_step(h * GLC_MIN_GAP[p], cfl, t_end=t_end)
    else:
        dt, n = t_end / steps, steps

    def fields(x, y):
        rho = 1.0 + 0.2 * np.sin(np.pi * x) * np.sin(np.pi * y)
        return rho, np.full_like(x, ux0), np.zeros_like(x), 1.0 / rho

    e = uniform_edges(ncells, -1.0, 1.0)
    return Workload(name or f"smooth_density_{ncells}x{ncells}_p{p}", e, e.copy(), p, True, True,
                    "polyatomic", gamma, nu, dt, n, fields, True, {"ux0": ux0, "t_end": t_end})


def population_noise(shape, seed, rel=0.05):
    """Seeded multiplicative perturbation factors 1 + rel * U(-1, 1)."""
    rng = np.random.default_rng(seed)
    return 1.0 + rel * rng.uniform(-1.0, 1.0, size=shape)


# ------------------------------------------------------ three dimensions (D3Q125)
@dataclass
class Workload3:
    name: str
    edges: tuple          # (edges_x, edges_y, edges_z)
    p: int
    periodic: tuple       # (x, y, z)
    nu: float
    dt: float
    steps: int
    fields: Callable      # (x, y, z) -> rho, ux, uy, uz
    meta: dict = field(default_factory=dict)


def tgv3d(ncells=64, p=2, U0=0.1, Re=100.0, steps=100, cfl=0.5, name=None):
    """Three-dimensional Taylor-Green vortex on the periodic box [0, 2 pi]^3
    (isothermal, P = rho): u = U0 sin x cos y cos z, v = -U0 cos x sin y cos z,
    w = 0, rho = 1 + (U0^2 / 16)(cos 2x + cos 2y)(cos 2z + 2), nu = U0 2 pi / Re."""
    L = 2.0 * np.pi
    h = L / ncells
    dt, n = cfl_time_step(h * GLC_MIN_GAP[p], cfl, steps=steps)
    nu = U0 * L / Re

    def fields(x, y, z):
        ux = U0 * np.sin(x) * np.cos(y) * np.cos(z)
        uy = -U0 * np.cos(x) * np.sin(y) * np.cos(z)
        rho = 1.0 + U0 * U0 / 16.0 * (np.cos(2 * x) + np.cos(2 * y)) * (np.cos(2 * z) + 2.0)
        return rho, ux, uy, np.zeros_like(x)

    e = uniform_edges(ncells, 0.0, L)
    return Workload3(name or f"tgv3d_{ncells}^3_p{p}", (e, e.copy(), e.copy()), p,
                     (True, True, True), nu, dt, n, fields, {"U0": U0, "Re": Re})


def sine_stretched_edges(ncells, lo, hi, amp=0.3):
    """Cell edges of [lo, hi] moved by amp h sin(2 pi k / ncells) / (2 pi) (a
    smooth, monotone stretching for amp < 1)."""
    k = np.arange(ncells + 1, dtype=float)
    h = (hi - lo) / ncells
    return lo + h * (k + amp * np.sin(2 * np.pi * k / ncells) / (2 * np.pi))


def box3d(ncells=(5, 4, 3), p=2, periodic=(True, False, True), U0=0.15, cfl=0.6, seed=3,
          name=None):
    """Small mapped (stretched) box of unit-ish extents with seeded smooth
    fields (a few low Fourier modes per velocity component, density 1 +/- 5 %),
    for parity tests: mixed periodic and zero-gradient axes."""
    lengths = (1.0, 0.8, 0.9)
    edges = tuple(sine_stretched_edges(n, 0.0, L) for n, L in zip(ncells, lengths))
    hmin = min(float(np.min(np.diff(e))) for e in edges)
    dt, n = cfl_time_step(hmin * GLC_MIN_GAP[p], cfl, steps=10)
    rng = np.random.default_rng(seed)
    ph = rng.uniform(0, 2 * np.pi, size=(4, 3))
    amp = rng.uniform(0.5, 1.0, size=4)

    def fields(x, y, z):
        k = [2 * np.pi / L for L in lengths]
        s = [amp[j] * np.sin(k[0] * x + ph[j, 0]) * np.cos(k[1] * y + ph[j, 1])
             * np.sin(k[2] * z + ph[j, 2]) for j in range(4)]
        return 1.0 + 0.05 * s[0], U0 * s[1], U0 * s[2], U0 * s[3]

    # tau = nu / dt + 1/2 = 0.8
    return Workload3(name or f"box3d_{ncells}_p{p}", edges, p, tuple(periodic), 0.3 * dt, dt, n,
                     fields, {"U0": U0})
