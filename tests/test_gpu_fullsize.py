"""Parity at the full benchmark sizes.

* Riemann, 512 x 512 cells of order 2 (1025^2 nodes, f + g), in the launch
  configuration the benchmark times (FP32, automatic path) and on every other
  path (the matrix-core x-pass included): one step at 4000 seeded nodes against the FP64 oracle, and two full
  steps at every node on the automatic path.
* Shock-vortex interaction, 1024 x 512 cells of order 3 with the stretched x
  map (3073 x 1536 nodes): one step at 4000 seeded nodes on every path.
* Largest grid the library accepts (nx * ny <= 2^31 / 64): a uniform moving
  state must stay the oracle's equilibrium of that state at every node.
* The alternating traversal: when the two population arrays (plus, on the
  records path, the departure records) exceed 256 MB, every other step visits
  the tiles or blocks backwards.  Two full steps at every node, and four steps
  at sampled nodes (the oracle evaluated on the samples' dependency cones),
  compare the forward and the backward orders with the oracle on the row-
  segment kernels (float32, and float64 with its 8-row workgroups) and the
  records kernel (float32 and float64), on the Riemann grid and (two steps,
  sampled) on the shock-vortex grid.
* A tall strip of 4 x 40000 cells, whose departure cells have row indices
  above 32767, through the records gather (the cell row is the upper half of
  the packed 32-bit record).

The oracle's expected values come from the workload fields alone (its own
initialisation and step); nothing it reads comes from the GPU.
"""
import numpy as np
import pytest
import torch

from oracle.grid import Grid
from oracle.sllbm import Sim
from paper_1910_13918_amd import workloads as W
from tests.oracle_cone import steps_at

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


MALL_BYTES = 256 * 2 ** 20


def _streamed_bytes(wl, precision, path):
    """Bytes a step streams: both population arrays, plus the records."""
    size = 4 if precision == "fp32" else 8
    b = 2 * wl.nsets * 25 * wl.nnodes * size
    if path == "records":
        b += 25 * wl.nnodes * (4 + 2 * size)
    return b


@pytest.fixture(scope="module")
def riemann_f2(riemann_case):
    print("[gpu] full-size oracle: riemann 512x512 p2, two steps at every node", flush=True)
    sim = riemann_case.sim
    return sim.step(sim.step(riemann_case.F0))


@pytest.mark.parametrize("precision,path", [("fp32", "auto"), ("fp32", "records"),
                                            ("fp64", "rows"), ("fp64", "records")])
def test_riemann_512_two_steps_every_node(riemann_case, riemann_f2, precision, path):
    """Two steps against two full oracle steps at every node; the second step
    runs in the reversed order (the state exceeds the 256 MB cache)."""
    from paper_1910_13918_amd.solver import Solver
    assert _streamed_bytes(riemann_case.wl, precision, path) > MALL_BYTES
    s = Solver.from_workload(riemann_case.wl, precision=precision, path=path)
    try:
        print(f"[gpu] riemann 512 two steps {precision} {path} ({s.resolved_path()})", flush=True)
        s.init_from_workload()
        s.step(2)
        assert s.flags() == (0, 2)
        G = s.populations().astype(np.float64)
    finally:
        s.close()
    err = np.abs(G - riemann_f2).max() / np.abs(riemann_f2).max()
    assert err <= (FP32_REL if precision == "fp32" else FP64_REL), err


@pytest.fixture(scope="module")
def riemann_f4_sampled(riemann_case):
    print("[gpu] full-size oracle: riemann 512x512 p2, four steps at sampled nodes", flush=True)
    return steps_at(riemann_case.sim, riemann_case.F0, riemann_case.nodes, 4)


@pytest.mark.parametrize("precision,path", [("fp32", "auto"), ("fp32", "records"),
                                            ("fp64", "auto")])
def test_riemann_512_four_steps_sampled(riemann_case, riemann_f4_sampled, precision, path):
    """Four steps (forward, backward, forward, backward order) at 4000 nodes."""
    from paper_1910_13918_amd.solver import Solver
    s = Solver.from_workload(riemann_case.wl, precision=precision, path=path)
    try:
        print(f"[gpu] riemann 512 four steps {precision} {path}", flush=True)
        s.init_from_workload()
        s.step(4)
        assert s.flags() == (0, 4)
        G = s.populations_device()[:, :, torch.as_tensor(riemann_case.nodes, device=s.device)]
        G = G.double().cpu().numpy()
    finally:
        s.close()
    ref = riemann_f4_sampled
    err = np.abs(G - ref).max() / np.abs(ref).max()
    assert err <= (FP32_REL if precision == "fp32" else FP64_REL), err


@pytest.fixture(scope="module")
def svi_f2_sampled(svi_case):
    print("[gpu] full-size oracle: shock-vortex, two steps at sampled nodes", flush=True)
    return steps_at(svi_case.sim, svi_case.F0, svi_case.nodes, 2)


@pytest.mark.parametrize("precision,path", [("fp32", "auto"), ("fp32", "records"),
                                            ("fp64", "auto")])
def test_svi_two_steps_sampled(svi_case, svi_f2_sampled, precision, path):
    """Shock-vortex grid (Pr = 0.75): the second step runs backwards."""
    from paper_1910_13918_amd.solver import Solver
    assert _streamed_bytes(svi_case.wl, precision, path) > MALL_BYTES
    s = Solver.from_workload(svi_case.wl, precision=precision, path=path)
    try:
        print(f"[gpu] shock-vortex two steps {precision} {path} ({s.resolved_path()})", flush=True)
        s.init_from_workload()
        s.step(2)
        assert s.flags() == (0, 2)
        G = s.populations_device()[:, :, torch.as_tensor(svi_case.nodes, device=s.device)]
        G = G.double().cpu().numpy()
    finally:
        s.close()
    err = np.abs(G - svi_f2_sampled).max() / np.abs(svi_f2_sampled).max()
    assert err <= (FP32_REL if precision == "fp32" else FP64_REL), err


def _tall_strip():
    """4 x 40000 cells of order 1, x periodic, y zero-gradient, monatomic,
    smooth fields varying along y."""
    h = 1.0 / 4000
    ex = W.uniform_edges(4, 0.0, 4 * h)
    ey = W.uniform_edges(40000, 0.0, 40000 * h)
    dt = 0.5 * h / W.XI_MAX

    def fields(x, y):
        rho = 1.0 + 0.1 * np.sin(2 * np.pi * y / (37 * h))
        ux = 0.2 * np.cos(2 * np.pi * y / (53 * h))
        uy = 0.1 * np.sin(2 * np.pi * y / (41 * h))
        return rho, ux, uy, 1.0 + 0.05 * np.cos(2 * np.pi * y / (29 * h))

    return W.Workload("tall_strip_4x40000_p1", ex, ey, 1, True, False, "monatomic", 1.4, 1e-3,
                      dt, 1, fields)


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_records_tall_strip_cell_rows_above_32767(precision):
    from paper_1910_13918_amd.solver import Solver
    wl = _tall_strip()
    g = Grid(wl.edges_x, wl.edges_y, wl.p, wl.periodic_x, wl.periodic_y)
    sim = Sim(g, wl.dt, wl.nu, wl.model, gamma=wl.gamma)
    X, Y = g.coords()
    F0 = sim.init(*wl.fields(X, Y))
    rng = np.random.default_rng(3)
    top = np.nonzero(Y >= 32768 * (wl.edges_y[1] - wl.edges_y[0]))[0]
    nodes = np.sort(np.concatenate([rng.choice(top, 400, replace=False),
                                    rng.choice(g.nnodes, 100, replace=False)]))
    F1 = sim.step(F0, nodes)
    s = Solver.from_workload(wl, precision=precision, path="records")
    try:
        print(f"[gpu] tall strip records {precision} nodes={s.n}", flush=True)
        s.init_from_workload()
        s.step(1)
        assert s.flags()[0] == 0
        G = s.populations_device()[:, :, torch.as_tensor(nodes, device=s.device)]
        G = G.double().cpu().numpy()
    finally:
        s.close()
    err = np.abs(G - F1).max() / np.abs(F1).max()
    assert err <= (FP32_REL if precision == "fp32" else FP64_REL), err


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
