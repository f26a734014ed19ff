"""GPU parity of curvilinear periodic meshes (bilinear cells; the records
gather fed by host-located departure points) against the FP64 oracle of
oracle/curvilinear.py, which locates every departure point by brute force
with a closed-form inverse.

Tolerances are those of the axis-product parity tests: FP64 one step
<= 1e-12 and FP32 one step <= 2e-6 relative to max |F|; a 30-step FP64
trajectory <= 1e-11.
"""
import numpy as np
import pytest
import torch

from oracle.curvilinear import CurviGrid, CurviSim
from paper_1910_13918_amd import sllbm as C
from paper_1910_13918_amd import workloads as W

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not torch.cuda.is_available(), reason="needs a HIP device")]


def _solver(wl, precision, path="auto"):
    from paper_1910_13918_amd.solver import Solver
    return Solver.from_workload(wl, precision=precision, path=path)


def _rel(a, b):
    return float(np.abs(a - b).max() / np.abs(b).max())


def _wl(model, p, ncells=7, amp=0.35, Pr=1.0):
    wl = W.tgv_wavy(ncells, p, amp=amp, U0=0.2, model=model)
    if model != "isothermal":
        base = wl.fields

        def fields(x, y):
            rho, ux, uy, _ = base(x, y)
            return rho, ux, uy, 0.8 + 0.3 * np.cos(x) * np.sin(y)

        wl.fields = fields
    wl.nu = 0.3 * wl.dt
    wl.Pr = Pr
    return wl


def _sim(wl):
    g = CurviGrid(*wl.vertices, wl.p)
    return g, CurviSim(g, wl.dt, wl.nu, wl.model, gamma=wl.gamma, Pr=wl.Pr)


def _state(wl, sim, g, seed, fp32):
    X, Y = g.coords()
    F = sim.init(*wl.fields(X, Y))
    F = F * W.population_noise(F.shape, seed, 0.05)
    return F.astype(np.float32).astype(np.float64) if fp32 else F


CASES = [(m, p) for m in ("isothermal", "monatomic", "polyatomic") for p in (1, 2, 3, 4)]


@pytest.mark.parametrize("case", CASES, ids=lambda c: f"{c[0]}-p{c[1]}")
def test_one_step_fp64(case):
    wl = _wl(*case)
    g, sim = _sim(wl)
    F0 = _state(wl, sim, g, seed=41, fp32=False)
    s = _solver(wl, "fp64")
    try:
        print(f"[gpu] curvilinear fp64 {case} nodes={g.nnodes}", flush=True)
        assert s.resolved_path() == "records"
        X, Y = s.coords()
        Xo, Yo = g.coords()
        assert np.abs(X - Xo).max() <= 1e-13 and np.abs(Y - Yo).max() <= 1e-13
        s.set_populations(F0)
        s.step(1)
        assert _rel(s.populations(), sim.step(F0)) <= 1e-12
        assert s.flags() == (0, 1)
    finally:
        s.close()


@pytest.mark.parametrize("case", CASES, ids=lambda c: f"{c[0]}-p{c[1]}")
def test_one_step_fp32(case):
    wl = _wl(*case)
    g, sim = _sim(wl)
    F0 = _state(wl, sim, g, seed=42, fp32=True)
    s = _solver(wl, "fp32")
    try:
        print(f"[gpu] curvilinear fp32 {case} nodes={g.nnodes}", flush=True)
        s.set_populations(F0)
        s.step(1)
        assert _rel(s.populations(), sim.step(F0)) <= 2e-6
    finally:
        s.close()


@pytest.mark.parametrize("p,dt", [(2, 0.8), (3, 2.0)])
def test_large_cfl_departures_several_cells_away(p, dt):
    """Departures up to 2.3 and 5.7 (cells are about 0.9 wide): the host walk
    crosses several cells and the periodic seam."""
    wl = _wl("polyatomic", p)
    wl.dt, wl.nu = dt, 0.3 * dt
    g, sim = _sim(wl)
    F0 = _state(wl, sim, g, seed=43, fp32=False)
    s = _solver(wl, "fp64")
    try:
        print(f"[gpu] curvilinear large CFL p={p} dt={dt}", flush=True)
        s.set_populations(F0)
        s.step(1)
        assert _rel(s.populations(), sim.step(F0)) <= 1e-12
    finally:
        s.close()


def test_prandtl_one_step_fp64():
    wl = _wl("polyatomic", 3, Pr=0.75)
    g, sim = _sim(wl)
    F0 = _state(wl, sim, g, seed=44, fp32=False)
    s = _solver(wl, "fp64")
    try:
        print("[gpu] curvilinear Pr = 0.75", flush=True)
        s.set_populations(F0)
        s.step(1)
        assert _rel(s.populations(), sim.step(F0)) <= 1e-12
    finally:
        s.close()


def test_trajectory_fp64():
    """30 steps of the Taylor-Green vortex on 16 x 16 wavy cells of order 3."""
    wl = _wl("isothermal", 3, ncells=16)
    g, sim = _sim(wl)
    X, Y = g.coords()
    F0 = sim.init(*wl.fields(X, Y))
    s = _solver(wl, "fp64")
    try:
        print(f"[gpu] curvilinear trajectory nodes={g.nnodes}", flush=True)
        s.init_from_workload()
        assert _rel(s.populations(), F0) <= 1e-14
        s.step(30)
        F = sim.run(F0, 30)
        assert _rel(F, F0) > 1e-4
        assert s.flags()[0] == 0
        assert _rel(s.populations(), F) <= 1e-11
        for a, b in zip(s.moments(), sim.macro(F)):
            assert _rel(a, b) <= 1e-11
    finally:
        s.close()


def test_other_paths_and_adjoint_refused():
    wl = _wl("isothermal", 2)
    s = _solver(wl, "fp64", path="tiled")
    try:
        s.init_from_workload()
        with pytest.raises(C.SllbmError) as e:
            s.step(1)
        assert e.value.code == C.E_UNSUPPORTED
        C.sllbm_set_path(s.ctx, C.PATH_RECORDS)
        s.step(1)
        lam = torch.zeros(s.nsets * s.q * s.n, dtype=torch.float64, device="cuda")
        mom = torch.ones(3 * s.n, dtype=torch.float64, device="cuda")
        with pytest.raises(C.SllbmError) as e:
            C.sllbm_adjoint_collide(s.ctx, lam.data_ptr(), mom.data_ptr(), lam.data_ptr())
        assert e.value.code == C.E_UNSUPPORTED
    finally:
        s.close()


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("p", [2, 4])
def test_mass_monitor_on_curved_cells(p, precision):
    """The mass monitor (Sec. III.E) on 9 x 9 wavy cells: sum_v M_v rho_v with
    the node masses of the bilinear cells, against the oracle's quadrature
    masses and density, initially and after 20 steps; the no-allocation
    variant gives the same value."""
    wl = _wl("isothermal", p, ncells=9)
    g, sim = _sim(wl)
    X, Y = g.coords()
    F0 = sim.init(*wl.fields(X, Y))
    F20 = sim.run(F0, 20)
    s = _solver(wl, precision)
    try:
        print(f"[gpu] curvilinear mass p={p} {precision} nodes={g.nnodes}", flush=True)
        s.init_from_workload()
        m0 = s.mass()
        s.step(20)
        m1 = s.mass()
        out = torch.zeros(1, dtype=torch.float64, device=s.device)
        C.sllbm_mass_noalloc(s.ctx, out.data_ptr())
        torch.cuda.synchronize()
        m1n = float(out.item())
    finally:
        s.close()
    # float32: the records hold the reference coordinates in float32, so the
    # weights (and the mass they carry) are rounded (measured 1.2e-6 after
    # 20 steps at p = 4)
    tol = 1e-12 if precision == "fp64" else 1e-5
    assert abs(m0 - sim.mass(F0)) <= tol * abs(m0)
    assert abs(m1 - sim.mass(F20)) <= tol * abs(m1)
    assert m1n == m1
