"""CPU tests of the three-dimensional C ABI (include/sllbm3d.h): exported
symbols, argument validation and call order, node coordinates against the
oracle's grid, and the refusal of device work without a device.  No kernel is
launched here.
"""
import ctypes
import os
import re

import numpy as np
import pytest

from oracle.sllbm3d import Grid3
from paper_1910_13918_amd import sllbm as C
from paper_1910_13918_amd import workloads as W
from tests.conftest import ROOT

HEADER = os.path.join(ROOT, "include", "sllbm3d.h")


def test_every_declared_symbol_is_exported():
    names = set(re.findall(r"\b(sllbm3d_[a-z_]+)\s*\(", open(HEADER).read()))
    assert len(names) >= 17
    for n in sorted(names):
        assert hasattr(C.lib, n), n
        assert n in C.EXPORTED, n


def _code(fn, *args):
    try:
        fn(*args)
        return C.OK
    except C.SllbmError as e:
        return e.code


def _grid(ctx, wl):
    e = [np.ascontiguousarray(a) for a in wl.edges]
    bc = [C.PERIODIC if p else C.ZERO_GRADIENT for p in wl.periodic]
    C.sllbm3d_init_grid(ctx, *[len(a) - 1 for a in e], *[a.ctypes.data for a in e], *bc)
    return e


def test_create_and_setup_validation():
    h = ctypes.c_void_p()
    assert C.lib.sllbm3d_create(ctypes.byref(h), 0, C.BF16X) == C.E_ARG
    assert C.lib.sllbm3d_create(ctypes.byref(h), -1, C.FP32) == C.E_ARG
    assert C.lib.sllbm3d_create(None, 0, C.FP32) == C.E_ARG
    C.sllbm3d_destroy(None)
    ctx = C.sllbm3d_create(0, C.FP64)
    try:
        e = np.linspace(0, 1, 4)
        # grid before the order
        assert _code(C.sllbm3d_init_grid, ctx, 3, 3, 3, e.ctypes.data, e.ctypes.data,
                     e.ctypes.data, 0, 0, 0) == C.E_STATE
        assert _code(C.sllbm3d_set_order, ctx, 5, C.NODES_GLC) == C.E_ARG
        assert _code(C.sllbm3d_set_order, ctx, 2, 7) == C.E_ARG
        C.sllbm3d_set_order(ctx, 2, C.NODES_GLC)
        bad = np.array([0.0, 0.5, 0.5, 1.0])
        assert _code(C.sllbm3d_init_grid, ctx, 3, 3, 3, e.ctypes.data, bad.ctypes.data,
                     e.ctypes.data, 0, 0, 0) == C.E_ARG
        nan = np.array([0.0, np.nan, 0.7, 1.0])
        assert _code(C.sllbm3d_init_grid, ctx, 3, 3, 3, e.ctypes.data, e.ctypes.data,
                     nan.ctypes.data, 0, 0, 0) == C.E_ARG
        assert _code(C.sllbm3d_init_grid, ctx, 0, 3, 3, e.ctypes.data, e.ctypes.data,
                     e.ctypes.data, 0, 0, 0) == C.E_ARG
        assert _code(C.sllbm3d_init_grid, ctx, 3, 3, 3, e.ctypes.data, e.ctypes.data,
                     e.ctypes.data, 0, 2, 0) == C.E_ARG
        assert _code(C.sllbm3d_init_grid, ctx, 3, 3, 3, None, e.ctypes.data,
                     e.ctypes.data, 0, 0, 0) == C.E_ARG
        # one float64 plane must stay below 4 GiB
        big = np.linspace(0, 1, 1001)
        assert _code(C.sllbm3d_init_grid, ctx, 1000, 1000, 1000, big.ctypes.data,
                     big.ctypes.data, big.ctypes.data, 0, 0, 0) == C.E_ARG
        C.sllbm3d_init_grid(ctx, 3, 3, 3, e.ctypes.data, e.ctypes.data, e.ctypes.data,
                            C.PERIODIC, C.ZERO_GRADIENT, C.PERIODIC)
        assert C.sllbm3d_num_nodes(ctx) == (6, 7, 6)
        for dt, nu in ((0.0, 0.1), (np.inf, 0.1), (0.01, 0.0), (0.01, np.nan), (-1.0, 0.1)):
            assert _code(C.sllbm3d_set_physics, ctx, dt, nu) == C.E_ARG
        C.sllbm3d_set_physics(ctx, 0.01, np.inf)  # pure streaming is allowed
        C.sllbm3d_set_physics(ctx, 0.01, 0.002)
        # nothing initialised yet
        assert _code(C.sllbm3d_step, ctx, 1) == C.E_STATE
        assert _code(C.sllbm3d_status_flags, ctx) == C.E_STATE
        assert _code(C.sllbm3d_mass, ctx) == C.E_STATE
        assert _code(C.sllbm3d_get_populations, ctx, 8, 1) == C.E_STATE
        out = [np.empty(6 * 7 * 6) for _ in range(4)]
        assert _code(C.sllbm3d_moments, ctx, *[a.ctypes.data for a in out], 0) == C.E_STATE
        assert _code(C.sllbm3d_step, ctx, -1) == C.E_ARG
        assert _code(C.sllbm3d_bind_populations, ctx, 16, 16) == C.E_ARG
        # host fields are checked before any device work
        rho = np.ones(6 * 7 * 6)
        rho[5] = -1.0
        z = np.zeros_like(rho)
        assert _code(C.sllbm3d_init_macro, ctx, rho.ctypes.data, z.ctypes.data, z.ctypes.data,
                     z.ctypes.data, 0) == C.E_ARG
        assert _code(C.sllbm3d_init_macro, ctx, rho.ctypes.data, None, z.ctypes.data,
                     z.ctypes.data, 0) == C.E_ARG
    finally:
        C.sllbm3d_destroy(ctx)


def test_call_order_before_physics():
    ctx = C.sllbm3d_create(0, C.FP32)
    try:
        assert _code(C.sllbm3d_num_nodes, ctx) == C.E_STATE
        C.sllbm3d_set_order(ctx, 3, C.NODES_EQUIDISTANT)
        _grid(ctx, W.box3d(p=3))
        assert _code(C.sllbm3d_bind_populations, ctx, 16, 32) == C.E_STATE  # no physics yet
        rho = np.ones(10)
        assert _code(C.sllbm3d_init_macro, ctx, *[rho.ctypes.data] * 4, 0) == C.E_STATE
    finally:
        C.sllbm3d_destroy(ctx)


@pytest.mark.parametrize("p", [1, 2, 3, 4])
def test_node_coords_match_the_oracle(p):
    wl = W.box3d(p=p, periodic=(True, False, True))
    ctx = C.sllbm3d_create(0, C.FP64)
    try:
        C.sllbm3d_set_order(ctx, p, C.NODES_GLC)
        _grid(ctx, wl)
        nx, ny, nz = C.sllbm3d_num_nodes(ctx)
        g = Grid3(*wl.edges, p, wl.periodic)
        assert (nx, ny, nz) == (g.nx, g.ny, g.nz)
        x, y, z = np.zeros(nx), np.zeros(ny), np.zeros(nz)
        C.sllbm3d_node_coords(ctx, x.ctypes.data, y.ctypes.data, z.ctypes.data)
        np.testing.assert_allclose(x, g.ax.node_coords(), rtol=0, atol=1e-15)
        np.testing.assert_allclose(y, g.ay.node_coords(), rtol=0, atol=1e-15)
        np.testing.assert_allclose(z, g.az.node_coords(), rtol=0, atol=1e-15)
    finally:
        C.sllbm3d_destroy(ctx)


def test_device_work_without_a_device_is_refused():
    """In a container without a GPU the first call that needs the device
    fails cleanly with SLLBM_E_DEVICE (and nothing falls back to the host)."""
    import torch
    if torch.cuda.is_available():
        pytest.skip("a HIP device is present")
    wl = W.box3d(p=2)
    ctx = C.sllbm3d_create(0, C.FP32)
    try:
        C.sllbm3d_set_order(ctx, 2, C.NODES_GLC)
        _grid(ctx, wl)
        C.sllbm3d_set_physics(ctx, wl.dt, wl.nu)
        nx, ny, nz = C.sllbm3d_num_nodes(ctx)
        f = [np.ones(nx * ny * nz)] + [np.zeros(nx * ny * nz)] * 3
        assert _code(C.sllbm3d_init_macro, ctx, *[a.ctypes.data for a in f], 0) == C.E_DEVICE
    finally:
        C.sllbm3d_destroy(ctx)
