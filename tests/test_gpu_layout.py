"""The two storage orders of the state buffers (planar for most gathers,
grouped for the row-segment step) never show at the boundary:

* get / set_populations round-trip bit for bit in either order, from host
  and device arrays, for f + g and single sets, D2Q25 and D2Q9;
* a run that changes path between steps (so the library converts the state)
  gives bit for bit what the same sequence of kernels gives on a state
  initialised under the final path, and matches the oracle;
* moments, the mass and the adjoint seed read the grouped order as the
  planar one (identical values: same arithmetic, same summation order);
* a device pointer that is one of the context's own buffers is refused.
"""
import numpy as np
import pytest
import torch

from oracle.grid import Grid
from oracle.sllbm import Sim
from paper_1910_13918_amd import sllbm as C
from paper_1910_13918_amd import workloads as W

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not torch.cuda.is_available(), reason="needs a HIP device")]


def _solver(wl, precision, path):
    from paper_1910_13918_amd.solver import Solver
    return Solver.from_workload(wl, precision=precision, path=path)


def _riemann(p=2, ncx=37, ncy=11):
    wl = W.riemann(ncx, p, seed=14)
    wl.edges_y = wl.edges_y[: ncy + 1]
    return wl


def _d2q9(p=2, ncx=35, ncy=9):
    wl = W.tgv(ncx, p, U0=0.2, model="isothermal", name="tgv_d2q9_layout")
    wl.q1 = 3
    wl.edges_y = wl.edges_y[0] + (wl.edges_x[1] - wl.edges_x[0]) * np.arange(ncy + 1)
    return wl


def _state(s, seed):
    rng = np.random.default_rng(seed)
    dtype = np.float64 if s.precision == "fp64" else np.float32
    return (0.01 + rng.random((s.nsets, s.q, s.n))).astype(dtype)


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("kind", ["riemann", "tgv", "d2q9"])
def test_round_trip_in_either_order(kind, precision):
    wl = {"riemann": _riemann(), "tgv": W.tgv(16, 3, U0=0.1), "d2q9": _d2q9()}[kind]
    for path in ("rows", "direct"):
        s = _solver(wl, precision, path)
        try:
            print(f"[gpu] round trip {kind} {precision} {path}", flush=True)
            F = _state(s, 3)
            s.set_populations(F)
            assert np.array_equal(s.populations(), F)
            t = torch.from_numpy(F).to(s.device)
            s.set_populations(t)
            assert torch.equal(s.populations_device().reshape(-1), t.reshape(-1))
            assert np.array_equal(s.populations(), F)
        finally:
            s.close()


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_path_changes_convert_the_state(precision):
    """rows x3, tiled x2, rows x2 from a state set under the tiled path
    (planar) against the same kernels from a state set under the row path
    (grouped): identical bits; and both against the FP64 oracle."""
    wl = _riemann()
    g = Grid(wl.edges_x, wl.edges_y, wl.p, wl.periodic_x, wl.periodic_y)
    sim = Sim(g, wl.dt, wl.nu, wl.model, gamma=wl.gamma, Pr=wl.Pr)
    X, Y = g.coords()
    F0 = sim.init(*wl.fields(X, Y)) * W.population_noise((2, 25, g.nnodes), 5, 0.03)
    want = sim.run(F0, 7)
    out = []
    for first in ("tiled", "rows"):
        s = _solver(wl, precision, first)
        try:
            print(f"[gpu] path changes {precision} from {first}", flush=True)
            s.set_populations(F0)
            for path, n in ((C.PATH_ROWS, 3), (C.PATH_TILED, 2), (C.PATH_ROWS, 2)):
                C.sllbm_set_path(s.ctx, path)
                s.step(n)
            assert s.flags() == (0, 7)
            out.append(s.populations())
        finally:
            s.close()
    assert np.array_equal(out[0], out[1])
    tol = 1e-12 if precision == "fp64" else 2e-6
    assert np.abs(out[0] - want).max() <= tol * np.abs(want).max()


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_per_node_kernels_read_the_grouped_order(precision):
    """One state set into a row-path context (grouped order) and a direct-path
    context (planar): moments, mass and the adjoint seed agree bit for bit."""
    wl = _riemann()
    s = _solver(wl, precision, "rows")
    t = _solver(wl, precision, "direct")
    try:
        print(f"[gpu] per-node kernels {precision}", flush=True)
        F = _state(s, 8)
        s.set_populations(F)
        t.set_populations(F)
        for a, b in zip(s.moments(), t.moments()):
            assert np.array_equal(a, b)
        assert s.mass() == t.mass()
        g = [torch.linspace(0.5, 1.5, s.n, dtype=torch.float64, device=s.device) * (k + 1)
             for k in range(4)]
        lams = []
        for u in (s, t):
            lam = torch.empty(u.nsets * u.q * u.n, dtype=u.dtype, device=u.device)
            C.sllbm_adjoint_seed(u.ctx, *[x.data_ptr() for x in g], lam.data_ptr())
            torch.cuda.synchronize()
            lams.append(lam.cpu().numpy())
        assert np.array_equal(lams[0], lams[1])
    finally:
        s.close()
        t.close()


def test_own_buffers_refused():
    s = _solver(_riemann(), "fp32", "rows")
    try:
        s.init_from_workload()
        for buf in (s.buf_a, s.buf_b):
            with pytest.raises(C.SllbmError) as e:
                C.sllbm_get_populations(s.ctx, buf.data_ptr(), 1)
            assert e.value.code == C.E_ARG
            with pytest.raises(C.SllbmError) as e:
                C.sllbm_set_populations(s.ctx, buf.data_ptr(), 1)
            assert e.value.code == C.E_ARG
    finally:
        s.close()
