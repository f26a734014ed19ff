"""Parity at the full benchmark sizes.

* Riemann, 512 x 512 cells of order 2 (1025^2 nodes, f + g), in the launch
  configuration the benchmark times (FP32, automatic path) and on every other
  path (the matrix-core x-pass included): one step at 4000 seeded nodes against the FP64 oracle, and two full
  steps at every node on the automatic path.
* Shock-vortex interaction, 1024 x 512 cells of order 3 with the stretched x
  map (3073 x 1536 nodes): one step at 4000 seeded nodes on every path.
* Largest grid the library accepts (nx * ny <= 2^31 / 64): a uniform moving
  state must stay the oracle's equilibrium of that state at every node.

The oracle's expected values come from the workload fields alone (its own
initialisation and step); nothing it reads comes from the GPU.
"""
import numpy as np
import pytest
import torch

from oracle.grid import Grid
from oracle.sllbm import Sim
from paper_1910_13918_amd import workloads as W

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not torch.cuda.is_available(), reason="needs a HIP device")]

# FP32 populations with FP64 moments: a step rounds every stored value once
# (2^-24 relative) after an interpolation whose weights sum to one and a
# collision that contracts by (1 - 1/tau) < 1; inputs were rounded once at
# initialisation.  A few ulps of the largest population bound the error.
FP32_REL = 2e-6
FP64_REL = 1e-12


class _Case:
    def __init__(self, wl, nsample=4000, seed=7):
        self.wl = wl
        g = Grid(wl.edges_x, wl.edges_y, wl.p, wl.periodic_x, wl.periodic_y)
        self.sim = Sim(g, wl.dt, wl.nu, wl.model, gamma=wl.gamma, Pr=wl.Pr)
        X, Y = g.coords()
        self.F0 = self.sim.init(*wl.fields(X, Y))
        rng = np.random.default_rng(seed)
        self.nodes = np.sort(rng.choice(g.nnodes, size=nsample, replace=False))
        self.F1 = self.sim.step(self.F0, self.nodes)
        self.scale = np.abs(self.F1).max()


@pytest.fixture(scope="module")
def riemann_case():
    print("[gpu] full-size oracle: riemann 512x512 p2", flush=True)
    return _Case(W.riemann(512, 2))


@pytest.fixture(scope="module")
def svi_case():
    print("[gpu] full-size oracle: shock-vortex 1024x512 p3 stretched", flush=True)
    return _Case(W.svi(1024, 512, 3))


def _one_step(case, precision, path):
    from paper_1910_13918_amd.solver import Solver
    s = Solver.from_workload(case.wl, precision=precision, path=path)
    try:
        print(f"[gpu] {case.wl.name} {precision} {path} nodes={s.n}", flush=True)
        assert s.n == case.sim.grid.nnodes
        s.init_from_workload()
        s.step(1)
        assert s.flags()[0] == 0
        G = s.populations_device()[:, :, torch.as_tensor(case.nodes, device=s.device)]
        return G.double().cpu().numpy()
    finally:
        s.close()


@pytest.mark.parametrize("precision,path", [("fp32", "auto"), ("fp32", "tiled"),
                                            ("fp32", "direct"), ("fp32", "records"),
                                            ("fp32", "mfma"), ("fp32", "rows"), ("fp64", "auto"),
                                            ("fp64", "records"), ("fp64", "rows")])
def test_riemann_512_one_step_sampled(riemann_case, precision, path):
    G = _one_step(riemann_case, precision, path)
    err = np.abs(G - riemann_case.F1).max() / riemann_case.scale
    assert err <= (FP32_REL if precision == "fp32" else FP64_REL), err


def test_riemann_512_two_steps_every_node(riemann_case):
    """Two steps of the benchmark configuration against two full oracle steps."""
    from paper_1910_13918_amd.solver import Solver
    sim = riemann_case.sim
    F2 = sim.step(sim.step(riemann_case.F0))
    s = Solver.from_workload(riemann_case.wl, precision="fp32", path="auto")
    try:
        s.init_from_workload()
        s.step(2)
        G = s.populations().astype(np.float64)
    finally:
        s.close()
    err = np.abs(G - F2).max() / np.abs(F2).max()
    assert err <= FP32_REL, err


@pytest.mark.parametrize("precision,path", [("fp32", "auto"), ("fp32", "direct"),
                                            ("fp32", "records"), ("fp32", "mfma"),
                                            ("fp32", "rows"), ("fp64", "auto")])
def test_svi_one_step_sampled(svi_case, precision, path):
    G = _one_step(svi_case, precision, path)
    err = np.abs(G - svi_case.F1).max() / svi_case.scale
    assert err <= (FP32_REL if precision == "fp32" else FP64_REL), err


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_largest_grid_uniform_state(precision):
    """2895^2 cells of order 2 = 5791^2 nodes (the largest square grid under
    the 2^31 / 64 node limit), zero-gradient, polyatomic: a uniform state with
    rho = 1.2, u = (0.3, -0.2), theta = 0.8 is a fixed point of the scheme."""
    from paper_1910_13918_amd.solver import Solver
    ncells = 2895
    wl = W.riemann(ncells, 2, states=[(1.2, 0.3, -0.2, 0.96)] * 4)
    g = Grid(np.array([0.0, 1.0]), np.array([0.0, 1.0]), 2, False, False)
    sim = Sim(g, wl.dt, wl.nu, wl.model, gamma=wl.gamma, Pr=wl.Pr)
    one = np.ones(1)
    ref = sim.init(1.2 * one, 0.3 * one, -0.2 * one, 0.8 * one)[:, :, 0]  # (S, 25)
    s = Solver.from_workload(wl, precision=precision)
    try:
        print(f"[gpu] largest grid {precision} nodes={s.n}", flush=True)
        assert s.n == (2 * ncells + 1) ** 2 and s.n <= (1 << 31) // 64
        n = s.n
        s.init_macro(torch.full((n,), 1.2, dtype=torch.float64, device=s.device),
                     torch.full((n,), 0.3, dtype=torch.float64, device=s.device),
                     torch.full((n,), -0.2, dtype=torch.float64, device=s.device),
                     torch.full((n,), 0.8, dtype=torch.float64, device=s.device))
        s.step(2)
        assert s.flags()[0] == 0
        F = s.populations_device()
        err = 0.0
        for k in range(F.shape[0]):
            for i in range(25):
                d = (F[k, i].double() - float(ref[k, i])).abs().max()
                err = max(err, float(d) / np.abs(ref).max())
        del F
    finally:
        s.close()
    assert err <= (FP32_REL if precision == "fp32" else FP64_REL), err
