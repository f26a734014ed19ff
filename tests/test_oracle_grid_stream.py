"""Pins of the oracle's grid, interpolation and streaming.

Compared against: the printed GLC formula values, Clenshaw-Curtis weights in
closed form, numpy's floor / searchsorted for the cell search, direct
polynomial evaluation (interpolation reproduces Q_p exactly), and np.roll for
a velocity set whose displacements are whole node spacings.
"""
import json
import os

import numpy as np
import pytest

from oracle.grid import Axis, Grid, basis_integrals, lagrange_basis, support_points, uniform_edges
from oracle.sllbm import Sim
from tests.conftest import GOLDEN


def test_glc_points_printed_formula():
    gold = json.load(open(os.path.join(GOLDEN, "paper_numbers.json")))["glc_formula"]
    for p in (2, 3, 4):
        np.testing.assert_allclose(support_points(p), gold[f"p{p}"], atol=1e-15)
    np.testing.assert_allclose(support_points(1), [0.0, 1.0])


@pytest.mark.parametrize("p", [1, 2, 3, 4])
def test_lagrange_kronecker_and_partition(p):
    r = support_points(p)
    np.testing.assert_array_equal(lagrange_basis(r, r), np.eye(p + 1))
    s = np.linspace(-0.3, 1.3, 41)
    np.testing.assert_allclose(lagrange_basis(r, s).sum(axis=0), 1.0, atol=1e-13)


def test_basis_integrals_clenshaw_curtis():
    cc = {1: [1 / 2, 1 / 2], 2: [1 / 6, 2 / 3, 1 / 6], 3: [1 / 18, 4 / 9, 4 / 9, 1 / 18],
          4: [1 / 30, 4 / 15, 2 / 5, 4 / 15, 1 / 30]}
    for p, ref in cc.items():
        np.testing.assert_allclose(basis_integrals(support_points(p)), ref, atol=1e-15)


def test_cell_search_uniform_vs_floor():
    ax = Axis(uniform_edges(13, -0.5, 2.1), 3, False)
    x = np.random.default_rng(0).uniform(-0.5, 2.1, 2000)
    cell, r = ax.locate(x)
    h = 2.6 / 13
    ref = np.minimum(np.floor((x + 0.5) / h).astype(int), 12)
    np.testing.assert_array_equal(cell, ref)
    assert np.all((r >= 0) & (r <= 1))
    c_hi, r_hi = ax.locate(np.array([ax.hi]))
    assert c_hi[0] == 12 and r_hi[0] == 1.0


def test_cell_search_mapped_vs_searchsorted():
    e = np.sort(np.random.default_rng(1).uniform(0, 1, 30))
    e = np.concatenate([[0.0], e, [1.0]])
    ax = Axis(e, 2, True)
    x = np.random.default_rng(2).uniform(0, 1, 3000)
    cell, _ = ax.locate(x)
    np.testing.assert_array_equal(cell, np.searchsorted(e, x, side="right") - 1)


@pytest.mark.parametrize("periodic", [True, False])
def test_node_count_and_mass(periodic):
    g = Grid(uniform_edges(5, 0.0, 2.0), uniform_edges(3, 1.0, 1.6), 4, periodic, periodic)
    assert g.nx == 20 + (0 if periodic else 1)
    # integral of a constant over the domain
    assert g.node_mass().sum() == pytest.approx(2.0 * 0.6, rel=1e-14)


def _poly_grid_sim(p, kind="glc"):
    ex = np.array([0.0, 0.7, 1.1, 1.9, 2.6, 3.0])       # non-uniform cells
    ey = uniform_edges(4, -1.0, 1.0)
    g = Grid(ex, ey, p, False, False, kind)
    sim = Sim(g, 0.031, np.inf, "isothermal")
    return g, sim


@pytest.mark.parametrize("p", [1, 2, 3, 4])
def test_streaming_reproduces_polynomials(p):
    """Nodal values of a random polynomial of degree <= p per axis, streamed with
    1/tau = 0, equal the polynomial at the departure points (brute force)."""
    g, sim = _poly_grid_sim(p)
    X, Y = g.coords()
    rng = np.random.default_rng(p)
    C = rng.normal(size=(p + 1, p + 1))

    def P(x, y):
        return sum(C[a, b] * x ** a * y ** b for a in range(p + 1) for b in range(p + 1))

    F = np.tile(P(X, Y), (1, 25, 1))
    out = sim.stream(F)
    for i in range(25):
        xd = X - sim.dt * sim.xi[i, 0]
        yd = Y - sim.dt * sim.xi[i, 1]
        inside = (xd >= 0) & (xd <= 3.0) & (yd >= -1) & (yd <= 1)
        np.testing.assert_allclose(out[0, i, inside], P(xd, yd)[inside], rtol=1e-12, atol=1e-12)
        # departures outside are clamped to the boundary (zero gradient)
        xc = np.clip(xd, 0, 3.0)
        yc = np.clip(yd, -1, 1)
        np.testing.assert_allclose(out[0, i], P(xc, yc), rtol=1e-12, atol=1e-12)


def test_streaming_rest_velocity_is_identity():
    g, sim = _poly_grid_sim(3)
    F = np.random.default_rng(5).normal(size=(1, 25, g.nnodes))
    out = sim.stream(F)
    # absolute coordinates put the departure on the node only up to rounding
    np.testing.assert_allclose(out[0, 0], F[0, 0], rtol=0, atol=1e-14)


def test_streaming_whole_node_shifts_is_roll():
    """A velocity set whose displacements dt * xi are whole multiples of the node
    spacing (p = 2: equidistant nodes) turns streaming into a periodic permutation."""
    nc, p, L = 6, 2, 3.0
    h = L / nc / p
    dt = 0.1
    xi1 = np.array([0.0, h / dt, 2 * h / dt, -h / dt, -3 * h / dt])
    w1 = np.full(5, 0.2)
    g = Grid(uniform_edges(nc, 0.0, L), uniform_edges(nc, 0.0, L), p, True, True)
    sim = Sim(g, dt, np.inf, "isothermal", xi1=xi1, w1=w1)
    F = np.random.default_rng(7).normal(size=(1, 25, g.nnodes))
    out = sim.stream(F)
    shifts = [0, 1, 2, -1, -3]
    for b in range(5):
        for a in range(5):
            i = a + 5 * b
            ref = np.roll(F[0, i].reshape(g.ny, g.nx), (shifts[b], shifts[a]), axis=(0, 1))
            np.testing.assert_allclose(out[0, i], ref.reshape(-1), rtol=0, atol=1e-14)


def test_interpolation_error_order():
    """Error of interpolating a smooth function at off-node points decays like
    h^(p+1) (p = 3, periodic)."""
    errs = []
    for nc in (4, 8, 16):
        g = Grid(uniform_edges(nc, 0, 2 * np.pi), uniform_edges(2, 0, 1.0), 3, True, True)
        sim = Sim(g, 0.37 * 2 * np.pi / nc, np.inf, "isothermal")
        X, Y = g.coords()
        F = np.tile(np.sin(X), (1, 25, 1))
        out = sim.stream(F)
        errs.append(np.abs(out[0, 1] - np.sin(X - sim.dt * sim.xi[1, 0])).max())
    orders = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert np.all(orders > 3.5), (errs, orders)


def test_dependency_cone_steps_equal_full_steps():
    """The cone helper (several steps evaluated only on the samples'
    dependency sets) returns the full run's values at the samples, bit for
    bit: a stream sums the same terms in the same order whichever nodes are
    evaluated.  A cone missing a node would leave a NaN instead."""
    from paper_1910_13918_amd import workloads as W
    from tests.oracle_cone import dependencies, steps_at
    wl = W.riemann(10, 2, states=W.RIEMANN_TABLE3_STATES)
    g = Grid(wl.edges_x, wl.edges_y, wl.p, wl.periodic_x, wl.periodic_y)
    sim = Sim(g, wl.dt, wl.nu, wl.model, gamma=wl.gamma, Pr=0.75)
    X, Y = g.coords()
    F0 = sim.init(*wl.fields(X, Y))
    nodes = np.array([0, 37, 200, g.nnodes - 1])
    full = sim.run(F0, 3)[:, :, nodes]
    np.testing.assert_array_equal(steps_at(sim, F0, nodes, 3), full)
    # the cone of a node holds its own departure stencils and stays local
    dep = dependencies(sim, np.array([200]))
    assert 200 in dep and len(dep) <= 25
    iy, ix = np.divmod(dep, g.nx)
    assert np.abs(ix - 200 % g.nx).max() <= 2 and np.abs(iy - 200 // g.nx).max() <= 2
