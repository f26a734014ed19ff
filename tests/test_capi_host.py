"""CPU tests of libsllbm's host path: exported symbols, argument validation and
call-order errors, and the host-side tables (node coordinates, departure
tables, mass weights) against the oracle's brute-force geometry.

No kernel is launched here; set-up calls never touch the HIP runtime.
"""
import ctypes
import os
import re

import numpy as np
import pytest

from oracle.grid import Grid
from oracle.sllbm import Sim
from paper_1910_13918_amd import sllbm as C
from paper_1910_13918_amd import workloads as W
from tests.conftest import ROOT

HEADER = os.path.join(ROOT, "include", "sllbm.h")


def test_every_declared_symbol_is_exported():
    src = open(HEADER).read()
    names = set(re.findall(r"\b(sllbm_[a-z_]+)\s*\(", src))
    assert len(names) >= 20
    for n in sorted(names):
        assert hasattr(C.lib, n), n
        assert n in C.EXPORTED, n


def _ctx(precision=C.FP64):
    return C.sllbm_create(0, precision)


def _code(fn, *args):
    try:
        fn(*args)
        return C.OK
    except C.SllbmError as e:
        return e.code


def _setup(ctx, p=2, nc=4, bc=C.PERIODIC, model=C.POLYATOMIC, dt=0.01, nu=0.01):
    C.sllbm_set_order(ctx, p, C.NODES_GLC)
    C.sllbm_init_grid_uniform(ctx, nc, nc, 0.0, 1.0, 0.0, 1.0, bc, bc)
    C.sllbm_set_physics(ctx, dt, nu, 1.4, 1.0, model)


def test_create_validation():
    h = ctypes.c_void_p()
    assert C.lib.sllbm_create(ctypes.byref(h), 0, 7) == C.E_ARG
    assert C.lib.sllbm_create(ctypes.byref(h), -1, 0) == C.E_ARG
    assert C.lib.sllbm_create(None, 0, 0) == C.E_ARG
    C.sllbm_destroy(None)  # accepted


def test_setup_validation_and_call_order():
    ctx = _ctx()
    try:
        # grid before order
        assert _code(C.sllbm_init_grid_uniform, ctx, 4, 4, 0, 1, 0, 1, 0, 0) == C.E_STATE
        assert "order" in C.sllbm_last_error(ctx)
        assert _code(C.sllbm_set_order, ctx, 0, 0) == C.E_ARG
        assert _code(C.sllbm_set_order, ctx, 5, 0) == C.E_ARG
        assert _code(C.sllbm_set_order, ctx, 2, 9) == C.E_ARG
        C.sllbm_set_order(ctx, 3, C.NODES_GLC)
        assert _code(C.sllbm_init_grid_uniform, ctx, 0, 4, 0, 1, 0, 1, 0, 0) == C.E_ARG
        assert _code(C.sllbm_init_grid_uniform, ctx, 4, 4, 1, 0, 0, 1, 0, 0) == C.E_ARG
        assert _code(C.sllbm_init_grid_uniform, ctx, 4, 4, 0, float("nan"), 0, 1, 0, 0) == C.E_ARG
        assert _code(C.sllbm_init_grid_uniform, ctx, 4, 4, 0, 1, 0, 1, 2, 0) == C.E_ARG
        bad = np.array([0.0, 0.5, 0.4, 1.0])
        good = np.array([0.0, 0.3, 0.6, 1.0])
        assert _code(C.sllbm_init_grid_mapped, ctx, 3, 3, bad.ctypes.data, good.ctypes.data, 0, 0) == C.E_ARG
        assert _code(C.sllbm_init_grid_mapped, ctx, 3, 3, None, good.ctypes.data, 0, 0) == C.E_ARG
        C.sllbm_init_grid_uniform(ctx, 4, 4, 0, 1, 0, 1, 0, 1)
        assert C.sllbm_num_nodes(ctx) == (12, 13)
        # physics
        assert _code(C.sllbm_set_physics, ctx, 0.0, 0.1, 1.4, 1.0, 2) == C.E_ARG
        assert _code(C.sllbm_set_physics, ctx, 0.1, 0.0, 1.4, 1.0, 2) == C.E_ARG   # tau = 1/2
        assert _code(C.sllbm_set_physics, ctx, 0.1, -1.0, 1.4, 1.0, 2) == C.E_ARG
        assert _code(C.sllbm_set_physics, ctx, 0.1, float("nan"), 1.4, 1.0, 2) == C.E_ARG
        assert _code(C.sllbm_set_physics, ctx, 0.1, 0.1, 1.0, 1.0, 2) == C.E_ARG
        assert _code(C.sllbm_set_physics, ctx, 0.1, 0.1, 1.4, 0.0, 2) == C.E_ARG
        assert _code(C.sllbm_set_physics, ctx, 0.1, 0.1, 1.4, float("nan"), 2) == C.E_ARG
        assert _code(C.sllbm_set_physics, ctx, 0.1, 0.1, 1.4, float("inf"), 2) == C.E_ARG
        assert _code(C.sllbm_set_physics, ctx, 0.1, 0.1, 1.4, 1.0, 3) == C.E_ARG
        # queries before physics
        assert _code(C.sllbm_relaxation_time, ctx) == C.E_STATE
        assert _code(C.sllbm_resolved_path, ctx) == C.E_STATE
        C.sllbm_set_physics(ctx, 0.1, 0.2, 1.4, 1.0, C.POLYATOMIC)
        assert C.sllbm_relaxation_time(ctx) == pytest.approx(0.2 / 0.1 + 0.5)
        assert C.sllbm_population_layout(ctx) == (2, 25, 8)
        # stepping before initialisation
        assert _code(C.sllbm_step, ctx, 1) == C.E_STATE
        assert _code(C.sllbm_step, ctx, -1) == C.E_ARG
        assert _code(C.sllbm_mass, ctx) == C.E_STATE
        assert _code(C.sllbm_set_path, ctx, 9) == C.E_ARG
        assert _code(C.sllbm_set_path, ctx, 6) == C.E_ARG
        assert _code(C.sllbm_set_check_interval, ctx, -2) == C.E_ARG
    finally:
        C.sllbm_destroy(ctx)


def test_resolved_path():
    """AUTO resolves to ROWS for row segments of >= 48 nodes, to TILED while
    every tile's source window fits the LDS staging (at most 3 rows per
    wavefront, 128 columns), else to DIRECT."""
    for prec, p, Pr, want in ((C.FP64, 2, 1.0, C.PATH_ROWS), (C.FP32, 2, 1.0, C.PATH_ROWS),
                              (C.FP32, 3, 1.0, C.PATH_ROWS), (C.FP64, 3, 1.0, C.PATH_ROWS),
                              (C.FP64, 2, 0.75, C.PATH_ROWS), (C.FP32, 2, 0.75, C.PATH_ROWS)):
        ctx = _ctx(prec)
        try:
            C.sllbm_set_order(ctx, p, C.NODES_GLC)
            C.sllbm_init_grid_uniform(ctx, 200, 8, 0.0, 1.0, 0.0, 1.0, C.PERIODIC, C.PERIODIC)
            C.sllbm_set_physics(ctx, 1e-3, 0.01, 1.4, Pr, C.POLYATOMIC)
            assert C.sllbm_resolved_path(ctx) == want, (prec, p, Pr)
        finally:
            C.sllbm_destroy(ctx)
    # the row-segment kernels load a single row for the first 1-D velocity,
    # which must be 0: a permuted velocity set resolves to TILED
    r10 = np.sqrt(10.0)
    xi = np.array([np.sqrt(5 - r10), 0.0, np.sqrt(5 + r10), -np.sqrt(5 - r10), -np.sqrt(5 + r10)])
    w = np.array([(7 + 2 * r10) / 60, 8 / 15, (7 - 2 * r10) / 60, (7 + 2 * r10) / 60,
                  (7 - 2 * r10) / 60])
    ctx = _ctx()
    try:
        C.sllbm_set_velocity_set(ctx, 5, xi.ctypes.data, w.ctypes.data)
        _setup(ctx, nc=20, dt=1e-3)
        assert C.sllbm_resolved_path(ctx) == C.PATH_TILED
    finally:
        C.sllbm_destroy(ctx)
    ctx = _ctx()
    try:
        _setup(ctx, nc=20, dt=1e-3)
        assert C.sllbm_resolved_path(ctx) == C.PATH_ROWS
        for p in (C.PATH_DIRECT, C.PATH_TILED, C.PATH_RECORDS, C.PATH_MFMA, C.PATH_ROWS):
            C.sllbm_set_path(ctx, p)
            assert C.sllbm_resolved_path(ctx) == p
        C.sllbm_set_path(ctx, C.PATH_AUTO)
        # 200 cells of width 1e-3 next to 10 cells of width 0.1: departures of
        # 0.05 from the wide cells cross ~100 narrow cells, a window far wider
        # than 128 columns
        ex = np.concatenate([np.linspace(0.0, 0.2, 201), 0.2 + 0.1 * np.arange(1, 11)])
        ey = np.linspace(0.0, 1.0, 11)
        C.sllbm_init_grid_mapped(ctx, len(ex) - 1, len(ey) - 1, ex.ctypes.data, ey.ctypes.data,
                                 C.ZERO_GRADIENT, C.PERIODIC)
        C.sllbm_set_physics(ctx, 0.05 / W.XI_MAX, 0.01, 1.4, 1.0, C.POLYATOMIC)
        assert C.sllbm_resolved_path(ctx) == C.PATH_DIRECT
    finally:
        C.sllbm_destroy(ctx)


def test_prandtl_needs_a_rule_exact_to_degree_seven():
    """Pr != 1 relies on the equilibrium having no centred third moment, which
    holds for a 1-D rule that integrates the Gaussian exactly to degree 7:
    the default D1Q5 set and, e.g., nodes 0, +-1, +-sqrt(6) with weights 1/3,
    3/10, 1/30 (exact to degree 7, not 8); a rule exact only to degree 5 is
    refused whichever of the two calls comes last."""
    xi7 = np.array([0.0, 1.0, np.sqrt(6.0), -1.0, -np.sqrt(6.0)])
    w7 = np.array([1 / 3, 0.3, 1 / 30, 0.3, 1 / 30])
    # nodes 0, +-1, +-2 with weights matching degrees 0, 2, 4 (degree 6 gives 11)
    xi5 = np.array([0.0, 1.0, 2.0, -1.0, -2.0])
    w5 = np.array([1 / 2, 1 / 6, 1 / 12, 1 / 6, 1 / 12])
    ctx = _ctx()
    try:
        C.sllbm_set_order(ctx, 2, C.NODES_GLC)
        C.sllbm_init_grid_uniform(ctx, 4, 4, 0, 1, 0, 1, 1, 1)
        C.sllbm_set_physics(ctx, 0.01, 0.02, 1.4, 0.75, C.POLYATOMIC)
        C.sllbm_set_velocity_set(ctx, 5, xi7.ctypes.data, w7.ctypes.data)
        assert _code(C.sllbm_set_velocity_set, ctx, 5, xi5.ctypes.data, w5.ctypes.data) == C.E_UNSUPPORTED
        assert "degree 7" in C.sllbm_last_error(ctx)
        C.sllbm_set_physics(ctx, 0.01, 0.02, 1.4, 1.0, C.POLYATOMIC)
        C.sllbm_set_velocity_set(ctx, 5, xi5.ctypes.data, w5.ctypes.data)
        assert _code(C.sllbm_set_physics, ctx, 0.01, 0.02, 1.4, 0.75, C.POLYATOMIC) == C.E_UNSUPPORTED
        C.sllbm_set_velocity_set(ctx, 5, None, None)
        C.sllbm_set_physics(ctx, 0.01, 0.02, 1.4, 0.75, C.MONATOMIC)
        # the isothermal model has no heat flux to relax
        assert _code(C.sllbm_set_physics, ctx, 0.01, 0.02, 1.4, 0.75, C.ISOTHERMAL) == C.E_ARG
    finally:
        C.sllbm_destroy(ctx)


def test_velocity_set_validation():
    ctx = _ctx()
    try:
        xi = np.zeros(5)
        w = np.ones(5)
        assert _code(C.sllbm_set_velocity_set, ctx, 4, xi.ctypes.data, w.ctypes.data) == C.E_UNSUPPORTED
        assert _code(C.sllbm_set_velocity_set, ctx, 7, None, None) == C.E_UNSUPPORTED
        w[2] = -1.0
        assert _code(C.sllbm_set_velocity_set, ctx, 5, xi.ctypes.data, w.ctypes.data) == C.E_ARG
        assert _code(C.sllbm_set_velocity_set, ctx, 5, xi.ctypes.data, None) == C.E_ARG
        assert _code(C.sllbm_set_velocity_set, ctx, 5, None, None, 0.0) == C.E_ARG
        assert _code(C.sllbm_set_velocity_set, ctx, 5, None, None, float("nan")) == C.E_ARG
        assert _code(C.sllbm_set_velocity_set, ctx, 5, None, None, -1.0) == C.E_ARG
        C.sllbm_set_velocity_set(ctx, 5, None, None)
    finally:
        C.sllbm_destroy(ctx)


def test_init_macro_validates_host_fields_before_device():
    ctx = _ctx()
    try:
        _setup(ctx, nc=2)
        nx, ny = C.sllbm_num_nodes(ctx)
        n = nx * ny
        rho = np.ones(n)
        u = np.zeros(n)
        T = np.ones(n)
        rho[3] = -1.0
        args = [a.ctypes.data for a in (rho, u, u, T)]
        assert _code(C.sllbm_init_macro, ctx, *args, 0) == C.E_ARG
        rho[3] = 1.0
        T[1] = float("nan")
        args = [a.ctypes.data for a in (rho, u, u, T)]
        assert _code(C.sllbm_init_macro, ctx, *args, 0) == C.E_ARG
        T[1] = 0.0
        args = [a.ctypes.data for a in (rho, u, u, T)]
        assert _code(C.sllbm_init_macro, ctx, *args, 0) == C.E_ARG
        assert _code(C.sllbm_init_macro, ctx, None, args[1], args[2], args[3], 0) == C.E_ARG
    finally:
        C.sllbm_destroy(ctx)


def _oracle_and_lib(wl, kind=C.NODES_GLC):
    g = Grid(wl.edges_x, wl.edges_y, wl.p, wl.periodic_x, wl.periodic_y,
             "glc" if kind == C.NODES_GLC else "equidistant")
    sim = Sim(g, wl.dt, wl.nu, wl.model, gamma=wl.gamma, Pr=wl.Pr)
    ctx = _ctx()
    C.sllbm_set_order(ctx, wl.p, kind)
    bcx = C.PERIODIC if wl.periodic_x else C.ZERO_GRADIENT
    bcy = C.PERIODIC if wl.periodic_y else C.ZERO_GRADIENT
    ex = np.ascontiguousarray(wl.edges_x)
    ey = np.ascontiguousarray(wl.edges_y)
    if wl.uniform:
        C.sllbm_init_grid_uniform(ctx, len(ex) - 1, len(ey) - 1, ex[0], ex[-1], ey[0], ey[-1], bcx, bcy)
    else:
        C.sllbm_init_grid_mapped(ctx, len(ex) - 1, len(ey) - 1, ex.ctypes.data, ey.ctypes.data, bcx, bcy)
    C.sllbm_set_physics(ctx, wl.dt, wl.nu, wl.gamma, wl.Pr,
                        {"isothermal": 0, "monatomic": 1, "polyatomic": 2}[wl.model])
    return g, sim, ctx


CASES = [
    W.tgv(3, 2, name="tgv"),
    W.tgv(2, 4, name="tgv_p4"),
    W.sod(6, 1, 3, name="sod"),
    W.riemann(3, 1, seed=1, name="riemann_p1"),
    W.svi(7, 2, 3, name="svi"),
    W.riemann(2, 4, seed=1, cfl=3.0, name="riemann_bigcfl"),
]


@pytest.mark.parametrize("wl", CASES, ids=lambda w: w.name)
def test_node_coords_and_mass_weights(wl):
    g, sim, ctx = _oracle_and_lib(wl)
    try:
        nx, ny = C.sllbm_num_nodes(ctx)
        assert (nx, ny) == (g.nx, g.ny)
        x = np.zeros(nx)
        y = np.zeros(ny)
        C.sllbm_node_coords(ctx, x.ctypes.data, y.ctypes.data)
        np.testing.assert_allclose(x, g.ax.node_coords(), rtol=0, atol=1e-14)
        np.testing.assert_allclose(y, g.ay.node_coords(), rtol=0, atol=1e-14)
        mx = np.zeros(nx)
        my = np.zeros(ny)
        C.sllbm_mass_weights(ctx, mx.ctypes.data, my.ctypes.data)
        np.testing.assert_allclose(mx, g.ax.node_mass(), rtol=1e-13, atol=1e-16)
        np.testing.assert_allclose(my, g.ay.node_mass(), rtol=1e-13, atol=1e-16)
        assert C.sllbm_relaxation_time(ctx) == pytest.approx(sim.tau, rel=1e-15)
    finally:
        C.sllbm_destroy(ctx)


@pytest.mark.parametrize("wl", CASES, ids=lambda w: w.name)
def test_departure_tables_match_bruteforce(wl):
    """The library's separable (x-table times y-table) departure weights, as a
    dense streaming matrix per velocity, equal the oracle's brute-force
    stencil (absolute coordinates, linear cell scan)."""
    g, sim, ctx = _oracle_and_lib(wl)
    try:
        P1 = wl.p + 1
        N = g.nnodes
        tabs = {}
        for axis, n in ((0, g.nx), (1, g.ny)):
            for comp in range(5):
                src = np.zeros(n * P1, dtype=np.int32)
                w = np.zeros(n * P1)
                C.sllbm_departure_table(ctx, axis, comp, src.ctypes.data, w.ctypes.data)
                tabs[axis, comp] = (src.reshape(n, P1), w.reshape(n, P1))
        nodes = np.arange(N)
        for b in range(5):
            for a in range(5):
                i = a + 5 * b
                osrc, owgt = sim.departure_stencil(i, nodes)
                M_o = np.zeros((N, N))
                for aa in range(P1):
                    for bb in range(P1):
                        np.add.at(M_o, (nodes, osrc[aa, bb]), owgt[aa, bb])
                sx, wx = tabs[0, a]
                sy, wy = tabs[1, b]
                ix = nodes % g.nx
                iy = nodes // g.nx
                M_l = np.zeros((N, N))
                for m in range(P1):
                    for k in range(P1):
                        np.add.at(M_l, (nodes, sy[iy, k] * g.nx + sx[ix, m]), wx[ix, m] * wy[iy, k])
                np.testing.assert_allclose(M_l, M_o, rtol=0, atol=2e-13, err_msg=f"velocity {i}")
    finally:
        C.sllbm_destroy(ctx)


def test_equidistant_nodes_tables():
    wl = W.tgv(3, 4, name="equi")
    g, sim, ctx = _oracle_and_lib(wl, C.NODES_EQUIDISTANT)
    try:
        x = np.zeros(g.nx)
        y = np.zeros(g.ny)
        C.sllbm_node_coords(ctx, x.ctypes.data, y.ctypes.data)
        np.testing.assert_allclose(x, g.ax.node_coords(), atol=1e-14)
    finally:
        C.sllbm_destroy(ctx)


def test_records_pack_cell_rows_above_32767():
    """Departure records of a 4 x 40000-cell strip: the packed cell
    (cx | cy << 16) read as an unsigned 32-bit word gives back the oracle's
    departure cell for rows up to 39999 (a signed read would turn rows of
    32768 and more negative)."""
    h = 1.0 / 4000
    ctx = _ctx()
    try:
        C.sllbm_set_order(ctx, 1, C.NODES_GLC)
        C.sllbm_init_grid_uniform(ctx, 4, 40000, 0.0, 4 * h, 0.0, 40000 * h, C.PERIODIC,
                                  C.ZERO_GRADIENT)
        dt = 0.5 * h / W.XI_MAX
        C.sllbm_set_physics(ctx, dt, 1e-3, 1.4, 1.0, C.MONATOMIC)
        nx, ny = C.sllbm_num_nodes(ctx)
        g = Grid(W.uniform_edges(4, 0.0, 4 * h), W.uniform_edges(40000, 0.0, 40000 * h), 1,
                 True, False)
        sim = Sim(g, dt, 1e-3, "monatomic")
        nodes = np.arange(nx * (ny - 700), nx * ny)  # rows 39301 .. 40000
        n = nx * ny
        for i in (0, 6, 13, 24):  # the rest velocity and three others
            cell = np.zeros(n, dtype=np.int32)
            r = np.zeros(n)
            s = np.zeros(n)
            C.sllbm_departure_records(ctx, i, cell.ctypes.data, r.ctypes.data, s.ctypes.data)
            u = cell.view(np.uint32)[nodes]
            xd = g.ax.apply_boundary(sim.X[nodes] - dt * sim.xi[i, 0])
            yd = g.ay.apply_boundary(sim.Y[nodes] - dt * sim.xi[i, 1])
            cx, _ = g.ax.locate(xd)
            cy, ry = g.ay.locate(yd)
            assert (cell[nodes] < 0).any()  # rows >= 32768 fill the sign bit
            np.testing.assert_array_equal(u >> 16, cy)
            np.testing.assert_array_equal(u & 0xFFFF, cx)
            np.testing.assert_allclose(s[nodes], ry, atol=1e-9)
    finally:
        C.sllbm_destroy(ctx)


def test_scaled_velocity_set_tables_and_tau():
    """A velocity set scaled by c_s = 1.7 (Sec. II.B): departure weights of
    the library's tables against the oracle's brute-force stencils of the
    scaled set, and tau = nu / (c_s^2 dt) + 1/2, whichever of the set-up
    calls comes last."""
    wl = W.riemann(6, 3, states=W.RIEMANN_TABLE3_STATES)
    cs = 1.7
    g = Grid(wl.edges_x, wl.edges_y, wl.p, wl.periodic_x, wl.periodic_y)
    sim = Sim(g, wl.dt, wl.nu, wl.model, gamma=wl.gamma, cs=cs)
    ctx = _ctx()
    try:
        C.sllbm_set_order(ctx, wl.p, C.NODES_GLC)
        C.sllbm_init_grid_uniform(ctx, 6, 6, 0.0, 1.0, 0.0, 1.0, C.ZERO_GRADIENT, C.ZERO_GRADIENT)
        C.sllbm_set_physics(ctx, wl.dt, wl.nu, wl.gamma, 1.0, C.POLYATOMIC)
        C.sllbm_set_velocity_set(ctx, 5, None, None, cs)
        assert C.sllbm_relaxation_time(ctx) == pytest.approx(sim.tau, rel=1e-15)
        P1 = wl.p + 1
        nodes = np.arange(g.nnodes)
        for i in (1, 7, 18, 24):
            a, b = i % 5, i // 5
            sx, wx = np.zeros(g.nx * P1, dtype=np.int32), np.zeros(g.nx * P1)
            sy, wy = np.zeros(g.ny * P1, dtype=np.int32), np.zeros(g.ny * P1)
            C.sllbm_departure_table(ctx, 0, a, sx.ctypes.data, wx.ctypes.data)
            C.sllbm_departure_table(ctx, 1, b, sy.ctypes.data, wy.ctypes.data)
            sx, wx, sy, wy = sx.reshape(-1, P1), wx.reshape(-1, P1), sy.reshape(-1, P1), wy.reshape(-1, P1)
            osrc, owgt = sim.departure_stencil(i, nodes)
            ix, iy = nodes % g.nx, nodes // g.nx
            M_o = np.zeros((g.nnodes, g.nnodes))
            M_l = np.zeros((g.nnodes, g.nnodes))
            for m in range(P1):
                for k in range(P1):
                    np.add.at(M_o, (nodes, osrc[m, k]), owgt[m, k])
                    np.add.at(M_l, (nodes, sy[iy, k] * g.nx + sx[ix, m]), wx[ix, m] * wy[iy, k])
            np.testing.assert_allclose(M_l, M_o, rtol=0, atol=2e-13)
    finally:
        C.sllbm_destroy(ctx)


def test_recorded_moments_per_model_and_prandtl_number():
    """K of sllbm_step_record: rho, u (3); + theta for the thermal models (4);
    + three centred second moments per set when Pr != 1 (what the transposed
    quasi-equilibrium term needs)."""
    cases = [(C.ISOTHERMAL, 1.0, 3), (C.MONATOMIC, 1.0, 4), (C.POLYATOMIC, 1.0, 4),
             (C.MONATOMIC, 0.75, 7), (C.POLYATOMIC, 0.75, 10), (C.POLYATOMIC, 2.0, 10)]
    for model, Pr, k in cases:
        ctx = _ctx()
        try:
            assert _code(C.sllbm_recorded_moments, ctx) == C.E_STATE  # physics not set
            C.sllbm_set_order(ctx, 2, C.NODES_GLC)
            C.sllbm_init_grid_uniform(ctx, 4, 4, 0.0, 1.0, 0.0, 1.0, C.PERIODIC, C.PERIODIC)
            C.sllbm_set_physics(ctx, 0.01, 0.01, 1.4, Pr, model)
            assert C.sllbm_recorded_moments(ctx) == k, (model, Pr)
        finally:
            C.sllbm_destroy(ctx)
