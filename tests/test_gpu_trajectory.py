"""Whole runs of two benchmark configurations on the GPU.

* The seeded four-quadrant Riemann problem on 64 x 64 cells of order 2 to
  t = 0.25, against the FP64 oracle's moments at every 4th node per axis
  (tests/golden/riemann64_reference.json, written by the oracle alone):
  FP64 to 1e-10 relative (rounding-order differences grown over the run's
  steps through the shocks), FP32 populations with the error stated.
* The shock-vortex interaction, 1024 x 512 cells of order 3 on the stretched
  grid at Pr = 0.75, for its 2000 steps in FP32 and FP64 (the vortex crosses
  the shock): both stay stable and the FP32 result is stated against the
  FP64 one (measured: rho 3.2e-5 max / 1.0e-5 L2, u 2.5e-5 / 2.5e-6,
  T 1.5e-5 / 2.4e-6; mass change -6.9e-6 vs 2.5e-7); the bounds leave a
  factor 4-6 of room.
"""
import json
import os

import numpy as np
import pytest
import torch

from paper_1910_13918_amd import workloads as W

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not torch.cuda.is_available(), reason="needs a HIP device")]

HERE = os.path.dirname(os.path.abspath(__file__))


def _run(wl, precision, steps):
    from paper_1910_13918_amd.solver import Solver
    s = Solver.from_workload(wl, precision=precision)
    try:
        s.init_from_workload()
        m0 = s.mass()
        s.step(steps)
        return s.moments(), s.flags()[0], s.mass() / m0 - 1.0
    finally:
        s.close()


def _errors(got, ref):
    """max and L2 relative errors of rho, |u| (vector) and T."""
    d_rho = got[0] - ref[0]
    d_u = np.hypot(got[1] - ref[1], got[2] - ref[2])
    u_ref = np.hypot(ref[1], ref[2])
    d_t = got[3] - ref[3]
    return {"rho_max": float(np.abs(d_rho).max() / np.abs(ref[0]).max()),
            "rho_l2": float(np.linalg.norm(d_rho) / np.linalg.norm(ref[0])),
            "u_max": float(d_u.max() / u_ref.max()),
            "u_l2": float(np.linalg.norm(d_u) / np.linalg.norm(u_ref)),
            "T_max": float(np.abs(d_t).max() / np.abs(ref[3]).max()),
            "T_l2": float(np.linalg.norm(d_t) / np.linalg.norm(ref[3]))}


def _reference():
    ref = json.load(open(os.path.join(HERE, "golden", "riemann64_reference.json")))
    nodes = np.array(ref["nodes"])
    return ref, nodes, [np.array(ref[k]) for k in ("rho", "ux", "uy", "T")]


@pytest.mark.parametrize("precision,bound", [("fp64", 1e-10), ("fp32", 2e-5)])
def test_riemann64_to_quarter_time_against_oracle(precision, bound):
    ref, nodes, want = _reference()
    wl = W.riemann(64, 2)
    assert wl.steps == ref["steps"]
    print(f"[gpu] riemann 64^2 to t = 0.25, {precision}, {wl.steps} steps", flush=True)
    m, unstable, _ = _run(wl, precision, wl.steps)
    assert unstable == 0
    err = _errors([a[nodes] for a in m], want)
    print(f"[gpu] {precision} error vs FP64 oracle: {err}", flush=True)
    assert max(err.values()) <= bound, err


def test_shock_vortex_full_run_fp32_vs_fp64():
    wl = W.svi(1024, 512, 3)
    assert wl.steps == 2000 and wl.Pr == 0.75
    print("[gpu] shock-vortex 1024x512 p = 3, 2000 steps, fp32 and fp64", flush=True)
    m32, u32, dm32 = _run(wl, "fp32", wl.steps)
    m64, u64, dm64 = _run(wl, "fp64", wl.steps)
    assert u32 == 0 and u64 == 0
    err = _errors(m32, m64)
    print(f"[gpu] shock-vortex FP32 vs FP64 after 2000 steps: {err}; mass change "
          f"{dm32:.3e} (FP32), {dm64:.3e} (FP64)", flush=True)
    assert max(err["rho_max"], err["u_max"], err["T_max"]) <= 2e-4, err
    assert max(err["rho_l2"], err["u_l2"], err["T_l2"]) <= 5e-5, err
    assert abs(dm32 - dm64) <= 4e-5


def test_sod_full_configuration_against_exact_solution():
    """The Sod tube of the benchmark configurations (1024 x 4 cells, p = 3,
    nu = 1.2e-4) to t = 0.2 in FP64 and FP32 populations, against the exact
    Riemann solution (the oracle's exact solver, pinned on the CPU): the
    L1 density error stays at the viscous-smearing level, the shock lands
    within 3 node spacings, and FP32 tracks FP64 (measured: L1 1.8e-3, shock
    0.5e-3 from the exact position; FP32 vs FP64 L2 3.0e-5 rho, 1.8e-4 u,
    4.5e-5 T, while the pointwise maximum, 4.3e-3 on u, sits at the fronts,
    where a shift of a fraction of a node spacing changes a node's value by
    the jump)."""
    from oracle import riemann
    wl = W.sod(1024, 4, 3)
    out = {}
    for prec in ("fp64", "fp32"):
        print(f"[gpu] Sod 1024x4 p = 3 to t = 0.2, {prec}, {wl.steps} steps", flush=True)
        m, unstable, _ = _run(wl, prec, wl.steps)
        assert unstable == 0
        out[prec] = m
    from paper_1910_13918_amd.solver import Solver
    s = Solver.from_workload(wl, precision="fp64")
    try:
        x, _ = s.axis_coords()
        nx = s.nx
    finally:
        s.close()
    r_ex, u_ex, p_ex = riemann.solution((1.0, 0.0, 1.0), (0.125, 0.0, 0.1), wl.gamma, x, 0.5,
                                        wl.dt * wl.steps)
    rho = out["fp64"][0][:nx]
    l1 = float(np.mean(np.abs(rho - r_ex)))
    thr = 0.5 * (0.125 + 0.26557)
    xs_num = x[np.nonzero(rho > thr)[0].max()]
    xs_ex = x[np.nonzero(r_ex > thr)[0].max()]
    d32 = _errors(out["fp32"], out["fp64"])
    print(f"[gpu] Sod L1 density error vs exact {l1:.3e}, shock at {xs_num:.5f} (exact {xs_ex:.5f}); "
          f"FP32 vs FP64 {d32}", flush=True)
    assert l1 <= 5e-3
    assert abs(xs_num - xs_ex) <= 3 * (1.0 / 1024 / 3) + 1e-12
    assert max(d32["rho_l2"], d32["u_l2"], d32["T_l2"]) <= 1e-3, d32
    assert max(d32["rho_max"], d32["u_max"], d32["T_max"]) <= 2e-2, d32


@pytest.fixture(scope="module")
def smooth_reference():
    """The FP64 oracle's smooth density propagation (Sec. III.B) on 4 x 4
    cells of order 4 with the paper's time step, 276 steps (t = 0.4995)."""
    from oracle.grid import Grid
    from oracle.sllbm import Sim
    dt = 2.0 / 1105
    wl = W.smooth_density(4, 4, t_end=276 * dt, steps=276)
    g = Grid(wl.edges_x, wl.edges_y, wl.p, True, True)
    sim = Sim(g, wl.dt, wl.nu, wl.model, gamma=wl.gamma)
    X, Y = g.coords()
    F = sim.run(sim.init(*wl.fields(X, Y)), wl.steps)
    return wl, sim.macro(F)


@pytest.mark.parametrize("precision,path,bound", [("fp64", "auto", 1e-11), ("fp64", "tiled", 1e-11),
                                                  ("fp64", "direct", 1e-11),
                                                  ("fp64", "records", 1e-11),
                                                  ("fp32", "auto", 1e-5)])
def test_smooth_density_trajectory_against_oracle(smooth_reference, precision, path, bound):
    """The GPU run of the same workload follows the oracle's trajectory at
    every node (polyatomic f + g on a smooth compressible flow)."""
    from paper_1910_13918_amd.solver import Solver
    wl, want = smooth_reference
    s = Solver.from_workload(wl, precision=precision, path=path)
    try:
        print(f"[gpu] smooth density 4x4 p4, {wl.steps} steps, {precision} {path}", flush=True)
        s.init_from_workload()
        s.step(wl.steps)
        got = s.moments()
        assert s.flags()[0] == 0
    finally:
        s.close()
    err = _errors(got, want)
    print(f"[gpu] smooth density {precision} {path} error vs FP64 oracle: {err}", flush=True)
    assert max(err.values()) <= bound, err


@pytest.mark.parametrize("precision,path,bound", [
    ("fp64", "records", 1e-10), ("fp64", "rows", 1e-10), ("fp64", "tiled", 1e-10),
    ("fp64", "direct", 1e-10), ("fp32", "records", 5e-5), ("fp32", "rows", 5e-5),
    ("fp32", "tiled", 5e-5), ("fp32", "direct", 5e-5)])
def test_shock_vortex_reduced_trajectory_against_oracle(precision, path, bound):
    """The shock-vortex configuration (Sec. III.E: stretched x map, Pr = 0.75,
    per-vertex gathers) on 128 x 64 cells of order 3 for 200 steps (Re = 100,
    which keeps the full configuration's tau on the 8 times coarser grid), against
    the FP64 oracle's moments at every 6th node per axis
    (tests/golden/svi128_reference.json, written by the oracle alone), on
    every gather: the departure records and the per-axis tables through row
    segments, LDS windows and direct loads."""
    ref = json.load(open(os.path.join(HERE, "golden", "svi128_reference.json")))
    nodes = np.array(ref["nodes"])
    want = [np.array(ref[k]) for k in ("rho", "ux", "uy", "T")]
    wl = W.svi(128, 64, 3, steps=ref["steps"], Re=ref["Re"])
    assert wl.Pr == 0.75 and abs(wl.dt - ref["dt"]) <= 1e-15 * ref["dt"]
    from paper_1910_13918_amd.solver import Solver
    s = Solver.from_workload(wl, precision=precision, path=path)
    try:
        print(f"[gpu] shock-vortex 128x64 p3, {wl.steps} steps, {precision} {path}", flush=True)
        s.init_from_workload()
        m0 = s.mass()
        s.step(wl.steps)
        got = [a[nodes] for a in s.moments()]
        dm = s.mass() / m0 - 1.0
        assert s.flags()[0] == 0
    finally:
        s.close()
    err = _errors(got, want)
    print(f"[gpu] shock-vortex 128x64 {precision} {path} error vs FP64 oracle: {err}; mass change "
          f"{dm:.3e} (oracle {ref['mass_rel_change']:.3e})", flush=True)
    assert max(err.values()) <= bound, err
    # FP32: the records path rounds its reference coordinates to float32, so
    # its weights (and the mass the interpolation carries) differ from the
    # oracle's by ~1e-7 per step (measured: mass change 6.0e-6 against the
    # oracle's 2.2e-6 after 200 steps; the per-axis tables < 1e-6)
    assert abs(dm - ref["mass_rel_change"]) <= (1e-12 if precision == "fp64" else 2e-5)


def test_shock_vortex_paper_stretching_needs_half_time_step():
    """Reading R29: with the paper's stretching Lambda = 0.95 on this grid
    (2-3 times finer per vortex radius than the paper's), the CFL time step of
    the finest cells is too long once the vortex reaches the shock: the
    stability flag rises before step 2000 (FP32, checked every 50 steps); at
    half that time step the 2000 steps run through."""
    import copy

    from paper_1910_13918_amd import sllbm as C
    from paper_1910_13918_amd.solver import Solver
    wl = W.svi(1024, 512, 3, lam=0.95)
    half = copy.copy(wl)
    half.dt = wl.dt / 2
    print("[gpu] shock-vortex lambda = 0.95 at half the time step, 2000 steps", flush=True)
    s = Solver.from_workload(half, precision="fp32")
    try:
        s.init_from_workload()
        s.step(2000)
        assert s.flags() == (0, 2000)
        assert all(np.isfinite(a).all() for a in s.moments())
    finally:
        s.close()
    print("[gpu] shock-vortex lambda = 0.95 at the CFL time step", flush=True)
    s = Solver.from_workload(wl, precision="fp32")
    try:
        s.init_from_workload()
        C.sllbm_set_check_interval(s.ctx, 50)
        with pytest.raises(C.SllbmError) as e:
            s.step(2000)
        assert e.value.code == C.E_UNSTABLE
        unstable, done = s.flags()
        print(f"[gpu] flag raised by step {done}", flush=True)
        assert unstable == 1 and 400 <= done < 2000
    finally:
        s.close()
