"""Pins of the curvilinear-cell oracle (oracle/curvilinear.py) against facts
that do not come from the oracle itself:

* cells given by the vertices of an axis-product grid are rectangles, so the
  curvilinear step must equal the axis-product oracle step (itself pinned by
  the tests of oracle/sllbm.py) on the same nodes;
* a bilinear cell map is of degree 1 in each reference coordinate, so a
  polynomial of total degree p in (x, y) is of degree <= p in r and in s and
  the order-p tensor interpolant on any bilinear cell reproduces it exactly
  (Sec. II.E, eq. (17)); degree p + 1 is not reproduced;
* the closed-form inverse maps back: x(r(P), s(P)) = P;
* the stencil weights of every point sum to 1 (partition of unity).
"""
import numpy as np
import pytest

from oracle.curvilinear import CurviGrid, CurviSim, bilinear, invert_bilinear, wavy_vertices
from oracle.grid import Grid
from oracle.sllbm import Sim


def _wavy(p, amp=0.35):
    return CurviGrid(*wavy_vertices(7, 5, 2 * np.pi, 2 * np.pi * 5 / 7, amp), p)


@pytest.mark.parametrize("p", [1, 2, 3, 4])
@pytest.mark.parametrize("model", ["isothermal", "polyatomic"])
def test_rectangular_cells_equal_axis_product_step(p, model):
    ex = np.array([0.0, 0.7, 1.5, 2.0, 3.1, 4.0, 5.2])
    ey = np.array([0.0, 1.1, 1.9, 3.0, 4.2])
    VX, VY = np.meshgrid(ex, ey)
    cg, g = CurviGrid(VX, VY, p), Grid(ex, ey, p, True, True)
    X, Y = g.coords()
    Xc, Yc = cg.coords()
    assert np.abs(Xc - X).max() < 1e-14 and np.abs(Yc - Y).max() < 1e-14
    # dt large enough that departures leave the node's cell and cross the seam
    a, b = CurviSim(cg, 0.15, 0.02, model), Sim(g, 0.15, 0.02, model)
    F = b.init(1 + 0.1 * np.sin(X), 0.1 * np.cos(Y), 0.05 * np.sin(X + Y), 1 + 0.1 * np.cos(X))
    F = F * (1 + 0.05 * np.random.default_rng(p).standard_normal(F.shape))
    ref = b.step(F)
    assert np.abs(a.step(F) - ref).max() <= 1e-13 * np.abs(ref).max()


def _interior_points(cg, n, seed):
    """Points whose cells are not in the last cell column or row, so no
    stencil node is the periodic image of column / row 0."""
    rng = np.random.default_rng(seed)
    px = rng.uniform(0.4, cg.Lx * (cg.ncx - 1) / cg.ncx - 0.4, n)
    py = rng.uniform(0.4, cg.Ly * (cg.ncy - 1) / cg.ncy - 0.4, n)
    cx, cy, _, _ = cg.locate(px, py)
    assert cx.max() < cg.ncx - 1 and cy.max() < cg.ncy - 1
    return px, py


@pytest.mark.parametrize("p", [1, 2, 3, 4])
def test_polynomials_of_degree_p_reproduced_on_bilinear_cells(p):
    cg = _wavy(p)
    X, Y = cg.coords()
    px, py = _interior_points(cg, 1500, p)
    src, wgt = cg.stencil(px, py)
    c = np.random.default_rng(10 + p).standard_normal((p + 1, p + 1))

    def poly(x, y):
        return sum(c[i, j] * x ** i * y ** j for i in range(p + 1) for j in range(p + 1 - i))

    f = poly(X, Y)
    val = (wgt * f[src]).sum(axis=(0, 1))
    assert np.abs(val - poly(px, py)).max() <= 1e-13 * np.abs(f).max()
    g = X ** (p + 1) + Y ** (p + 1)
    assert np.abs((wgt * g[src]).sum(axis=(0, 1)) - (px ** (p + 1) + py ** (p + 1))).max() > 1e-4
    assert np.abs(wgt.sum(axis=(0, 1)) - 1).max() <= 1e-13


def test_inverse_maps_back_and_cells_are_not_affine():
    cg = _wavy(3)
    px, py = _interior_points(cg, 400, 7)
    cx, cy, r, s = cg.locate(px, py)
    for i, j, rr, ss, x, y in zip(cx, cy, r, s, px, py):
        bx, by = bilinear(cg.cell_vertices(i, j), rr, ss)
        assert abs(bx - x) <= 1e-12 and abs(by - y) <= 1e-12
    # the test mesh is genuinely bilinear: some cell has A3 != 0
    a3 = [np.hypot(*np.subtract(np.add(v[0], v[3]), np.add(v[1], v[2])))
          for v in (cg.cell_vertices(i, j) for i in range(cg.ncx) for j in range(cg.ncy))]
    assert max(a3) > 0.05


def test_inverse_of_a_parallelogram_is_linear():
    v = ((0.0, 0.0), (2.0, 0.5), (0.3, 1.0), (2.3, 1.5))
    r, s = invert_bilinear(v, np.array([1.15, 0.0]), np.array([0.75, 0.0]))
    assert np.allclose(r, [0.5, 0.0], atol=1e-15) and np.allclose(s, [0.5, 0.0], atol=1e-15)


def test_departure_outside_every_cell_is_an_error():
    cg = _wavy(2)
    with pytest.raises(ValueError):
        cg.locate(np.array([4 * cg.Lx]), np.array([0.5]))


@pytest.mark.parametrize("p", [1, 2, 3, 4])
def test_node_mass_rectangles_equal_axis_product(p):
    """On rectangular cells the curvilinear node masses are the axis-product
    weights of the grid oracle (Clenshaw-Curtis weights times the cell size,
    pinned in test_oracle_grid_stream.py)."""
    ex = np.array([0.0, 0.7, 1.5, 2.0, 3.1])
    ey = np.array([0.0, 1.1, 1.9, 3.0])
    VX, VY = np.meshgrid(ex, ey)
    M = CurviGrid(VX, VY, p).node_mass()
    np.testing.assert_allclose(M, Grid(ex, ey, p, True, True).node_mass(), rtol=1e-13, atol=0)


@pytest.mark.parametrize("p", [1, 2, 3, 4])
def test_node_mass_wavy_area_and_smooth_integral(p):
    """On a genuinely curved periodic mesh: the masses sum to the area of the
    periodic box (the shape functions sum to one and the cells tile one
    period), and sum_v M_v f(x_v) of a smooth periodic f converges to its
    exact integral (cos^2(2 pi x / Lx) integrates to half the area)."""
    L = 2 * np.pi
    errs = []
    for n in (8, 16):
        cg = CurviGrid(*wavy_vertices(n, n, L, L, 0.3), p)
        M = cg.node_mass()
        assert abs(M.sum() - L * L) <= 1e-12 * L * L
        X, Y = cg.coords()
        errs.append(abs(np.sum(M * np.cos(X) ** 2) - 0.5 * L * L))
    assert errs[1] < errs[0] * 2.0 ** (-p) or errs[1] < 1e-11, errs
