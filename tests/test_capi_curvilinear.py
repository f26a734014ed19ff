"""CPU tests of the curvilinear-mesh host path of libsllbm: argument checks,
node coordinates, and the departure records (Newton's method and a walk
across cells, on the host) against the oracle's closed-form, brute-force
location (oracle/curvilinear.py).  No kernel is launched."""
import numpy as np
import pytest

from oracle.curvilinear import CurviGrid
from oracle.grid import lagrange_basis
from oracle.velocity import d1q5, tensor_product
from paper_1910_13918_amd import sllbm as C
from paper_1910_13918_amd import workloads as W


def _code(fn, *args):
    try:
        fn(*args)
        return C.OK
    except C.SllbmError as e:
        return e.code


def _ctx(vx, vy, p=3, dt=0.1, model=C.POLYATOMIC):
    ctx = C.sllbm_create(0, C.FP64)
    C.sllbm_set_order(ctx, p, C.NODES_GLC)
    vx = np.ascontiguousarray(vx, dtype=np.float64)
    vy = np.ascontiguousarray(vy, dtype=np.float64)
    C.sllbm_init_grid_curvilinear(ctx, vx.shape[1] - 1, vx.shape[0] - 1, vx.ctypes.data,
                                  vy.ctypes.data)
    C.sllbm_set_physics(ctx, dt, 0.01, 1.4, 1.0, model)
    return ctx


def _mesh(ncx=7, ncy=5, amp=0.35):
    return W.wavy_vertices(ncx, ncy, 2 * np.pi, 2 * np.pi * ncy / ncx, amp)


def test_vertex_checks():
    ctx = C.sllbm_create(0, C.FP64)
    try:
        vx, vy = (np.ascontiguousarray(a) for a in _mesh())
        args = (ctx, vx.shape[1] - 1, vx.shape[0] - 1)
        assert _code(C.sllbm_init_grid_curvilinear, *args, vx.ctypes.data,
                     vy.ctypes.data) == C.E_STATE  # order first
        C.sllbm_set_order(ctx, 2, C.NODES_GLC)
        assert _code(C.sllbm_init_grid_curvilinear, *args, 0, vy.ctypes.data) == C.E_ARG
        bad = vx.copy()
        bad[2, -1] += 0.01  # column ncx not the periodic image of column 0
        assert _code(C.sllbm_init_grid_curvilinear, *args, bad.ctypes.data,
                     vy.ctypes.data) == C.E_ARG
        fold = vx.copy()
        fold[2, 3] = fold[2, 4] + 0.5  # vertex moved past its right neighbour
        assert _code(C.sllbm_init_grid_curvilinear, *args, fold.ctypes.data,
                     vy.ctypes.data) == C.E_ARG
        nan = vy.copy()
        nan[1, 1] = np.nan
        assert _code(C.sllbm_init_grid_curvilinear, *args, vx.ctypes.data,
                     nan.ctypes.data) == C.E_ARG
        assert "periodic" in C.sllbm_last_error(ctx) or "finite" in C.sllbm_last_error(ctx)
        C.sllbm_init_grid_curvilinear(ctx, *args[1:], vx.ctypes.data, vy.ctypes.data)
    finally:
        C.sllbm_destroy(ctx)


@pytest.mark.parametrize("p", [1, 2, 3, 4])
def test_node_coordinates_match_the_oracle(p):
    vx, vy = _mesh()
    ctx = _ctx(vx, vy, p)
    try:
        nx, ny = C.sllbm_num_nodes(ctx)
        assert (nx, ny) == (7 * p, 5 * p)
        x = np.zeros(nx * ny)
        y = np.zeros(nx * ny)
        C.sllbm_node_coords_2d(ctx, x.ctypes.data, y.ctypes.data)
        X, Y = CurviGrid(vx, vy, p).coords()
        assert np.abs(x - X).max() <= 1e-13 and np.abs(y - Y).max() <= 1e-13
    finally:
        C.sllbm_destroy(ctx)


def test_axis_queries_refused_and_auto_is_records():
    vx, vy = _mesh()
    ctx = _ctx(vx, vy)
    try:
        nx, ny = C.sllbm_num_nodes(ctx)
        buf = np.zeros(max(nx, ny) * 5)
        ibuf = np.zeros(max(nx, ny) * 5, dtype=np.int32)
        assert _code(C.sllbm_node_coords, ctx, buf.ctypes.data, buf.ctypes.data) == C.E_UNSUPPORTED
        assert _code(C.sllbm_departure_table, ctx, 0, 1, ibuf.ctypes.data,
                     buf.ctypes.data) == C.E_UNSUPPORTED
        assert _code(C.sllbm_mass_weights, ctx, buf.ctypes.data,
                     buf.ctypes.data) == C.E_UNSUPPORTED
        assert C.sllbm_resolved_path(ctx) == C.PATH_RECORDS
    finally:
        C.sllbm_destroy(ctx)


@pytest.mark.parametrize("p,dt", [(1, 0.1), (2, 0.1), (3, 0.1), (4, 0.1), (3, 1.0), (2, 2.5)])
def test_departure_records_locate_the_oracle_points(p, dt):
    """Host records against the oracle: the interpolation weights of each
    departure point agree (a point on a shared edge may sit in either cell;
    the weights of its stencil nodes agree either way).  dt = 1 and 2.5 move
    departures up to about 3 and 7 node spacings, across several cells and
    the periodic seam."""
    vx, vy = _mesh()
    ctx = _ctx(vx, vy, p, dt=dt)
    g = CurviGrid(vx, vy, p)
    xi, _ = tensor_product(*d1q5())
    X, Y = g.coords()
    n = g.nnodes
    try:
        for i in range(25):
            cell = np.zeros(n, dtype=np.int32)
            r = np.zeros(n)
            s = np.zeros(n)
            C.sllbm_departure_records(ctx, i, cell.ctypes.data, r.ctypes.data, s.ctypes.data)
            src, wgt = g.stencil(X - dt * xi[i, 0], Y - dt * xi[i, 1])
            # dense weight matrices over the nodes, host vs oracle
            cx, cy = cell & 0xFFFF, cell >> 16
            assert cx.max() < g.ncx and cy.max() < g.ncy
            assert r.min() >= 0 and r.max() <= 1 and s.min() >= 0 and s.max() <= 1
            lr, ls = lagrange_basis(g.r, r), lagrange_basis(g.r, s)
            host = np.zeros((n, n))
            ref = np.zeros((n, n))
            rows = np.arange(n)
            for a in range(p + 1):
                for b in range(p + 1):
                    np.add.at(host, (rows, g.node_of(cx, cy, a, b)), lr[a] * ls[b])
                    np.add.at(ref, (rows, src[a, b]), wgt[a, b])
            assert np.abs(host - ref).max() <= 1e-11, i
    finally:
        C.sllbm_destroy(ctx)


def test_records_of_an_axis_grid_match_its_tables():
    ctx = C.sllbm_create(0, C.FP64)
    try:
        C.sllbm_set_order(ctx, 2, C.NODES_GLC)
        C.sllbm_init_grid_uniform(ctx, 6, 4, 0.0, 1.0, 0.0, 1.0, C.PERIODIC, C.ZERO_GRADIENT)
        C.sllbm_set_physics(ctx, 0.01, 0.01, 1.4, 1.0, C.ISOTHERMAL)
        nx, ny = C.sllbm_num_nodes(ctx)
        cell = np.zeros(nx * ny, dtype=np.int32)
        r = np.zeros(nx * ny)
        s = np.zeros(nx * ny)
        C.sllbm_departure_records(ctx, 7, cell.ctypes.data, r.ctypes.data, s.ctypes.data)
        # velocity 7 = (a, b) = (2, 1): x-component from table a, y from table b
        srcx = np.zeros(nx * 3, dtype=np.int32)
        wx = np.zeros(nx * 3)
        C.sllbm_departure_table(ctx, 0, 2, srcx.ctypes.data, wx.ctypes.data)
        lr = lagrange_basis(np.array([0.0, 0.5, 1.0]), r.reshape(ny, nx)[0])
        assert np.abs(lr.T - wx.reshape(nx, 3)).max() <= 1e-14
        assert _code(C.sllbm_departure_records, ctx, 25, cell.ctypes.data, r.ctypes.data,
                     s.ctypes.data) == C.E_ARG
    finally:
        C.sllbm_destroy(ctx)


@pytest.mark.parametrize("p", [1, 2, 3, 4])
def test_node_masses_match_the_oracle(p):
    """The library's node masses on wavy bilinear cells (closed form of the
    Jacobian, which is linear in (r, s)) against the oracle's tensor
    Gauss-Legendre quadrature of l_a l_b |J|; on an axis grid the same query
    gives the product of the per-axis weights."""
    vx, vy = _mesh()
    ctx = _ctx(vx, vy, p)
    try:
        nx, ny = C.sllbm_num_nodes(ctx)
        m = np.zeros(nx * ny)
        C.sllbm_node_masses(ctx, m.ctypes.data)
        want = CurviGrid(vx, vy, p).node_mass()
        np.testing.assert_allclose(m, want, rtol=1e-13, atol=1e-15)
    finally:
        C.sllbm_destroy(ctx)
    ctx = C.sllbm_create(0, C.FP64)
    try:
        C.sllbm_set_order(ctx, p, C.NODES_GLC)
        C.sllbm_init_grid_uniform(ctx, 5, 4, 0.0, 1.0, 0.0, 2.0, C.PERIODIC, C.ZERO_GRADIENT)
        nx, ny = C.sllbm_num_nodes(ctx)
        m = np.zeros(nx * ny)
        mx, my = np.zeros(nx), np.zeros(ny)
        C.sllbm_node_masses(ctx, m.ctypes.data)
        C.sllbm_mass_weights(ctx, mx.ctypes.data, my.ctypes.data)
        np.testing.assert_allclose(m, np.outer(my, mx).reshape(-1), rtol=1e-15)
    finally:
        C.sllbm_destroy(ctx)
