"""GPU tests of the adjoint step and the checkpointed rollout gradient.

* transposed streaming: <mu, S v> = <S^T mu, v> (dot-product test, FP64);
* one full step: <S^T J_C^T lam, v> against central differences of
  <lam, step(F + eps v)> (FP64);
* rollout gradient (checkpointed) against the oracle's complex-step
  derivative (exact to rounding) on a reduced Taylor-Green instance;
* FP32 rollout gradient against the FP64 one;
* the 128 x 128-cell, p = 4 adjoint workload against central differences on
  the FP64 path.
"""
import numpy as np
import pytest
import torch

from oracle.adjoint import complex_step_directional, kinetic_misfit_loss
from oracle.grid import Grid
from oracle.sllbm import Sim
from paper_1910_13918_amd import workloads as W

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not torch.cuda.is_available(), reason="needs a HIP device")]


def _solver(wl, precision="fp64", path="auto"):
    from paper_1910_13918_amd.solver import Solver
    return Solver.from_workload(wl, precision=precision, path=path)


def _rand(shape, seed, dtype=torch.float64):
    g = torch.Generator().manual_seed(seed)
    return torch.randn(shape, generator=g, dtype=torch.float64).to(dtype=dtype, device="cuda")


GRIDS = [
    ("tgv_per", lambda: W.tgv(9, 4, U0=0.3)),
    ("tgv_p2", lambda: W.tgv(37, 2, U0=0.3)),
    ("zero_gradient", lambda: _iso(W.riemann(23, 3, states=W.RIEMANN_TABLE3_STATES))),
    ("stretched", lambda: _iso(W.svi(40, 6, 3))),
]


def _iso(wl):
    wl.model = "isothermal"
    wl.Pr = 1.0
    return wl


@pytest.mark.parametrize("path", ["tiled", "direct", "rows"])
@pytest.mark.parametrize("name,make", GRIDS, ids=[g[0] for g in GRIDS])
def test_transposed_streaming_dot_product(name, make, path):
    from paper_1910_13918_amd import sllbm as C
    wl = make()
    wl.nu = np.inf  # 1/tau = 0: the step is the interpolation alone
    s = _solver(wl, "fp64", path)
    try:
        print(f"[gpu] adjoint dot product {name} {path} nodes={s.n}", flush=True)
        v = _rand((25, s.n), 1)
        mu = _rand((25, s.n), 2)
        s.set_populations(v)
        s.step(1)
        Sv = s.populations_device()[0]
        StMu = torch.empty_like(mu)
        C.sllbm_adjoint_step(s.ctx, mu.data_ptr(), None, StMu.data_ptr())
        torch.cuda.synchronize()
        lhs = float((mu * Sv).sum())
        rhs = float((StMu * v).sum())
        assert lhs == pytest.approx(rhs, rel=1e-12)
    finally:
        s.close()


@pytest.mark.parametrize("name,make", GRIDS[:3], ids=[g[0] for g in GRIDS[:3]])
def test_one_step_adjoint_against_central_differences(name, make):
    from paper_1910_13918_amd import sllbm as C
    wl = make()
    s = _solver(wl, "fp64")
    try:
        s.init_from_workload()
        s.step(3)
        F = s.populations_device()[0].clone()
        lam = _rand((25, s.n), 3)
        v = _rand((25, s.n), 4) * F.abs().mean()
        # adjoint: S^T J_C(M)^T lam with M of this step
        s.set_populations(F)
        mom = s.step_record(1)
        mu = torch.empty_like(lam)
        out = torch.empty_like(lam)
        C.sllbm_adjoint_collide(s.ctx, lam.data_ptr(), mom[0].data_ptr(), mu.data_ptr())
        C.sllbm_adjoint_step(s.ctx, mu.data_ptr(), None, out.data_ptr())
        torch.cuda.synchronize()
        adj = float((out * v).sum())
        eps = 1e-6

        def g(e):
            s.set_populations(F + e * v)
            s.step(1)
            return float((lam * s.populations_device()[0]).sum())

        fd = (g(eps) - g(-eps)) / (2 * eps)
        assert adj == pytest.approx(fd, rel=1e-6)
    finally:
        s.close()


def _loss_torch(rho, ux, uy, M, ut, vt):
    return 0.5 * (M * rho * (ux * ux + uy * uy)).sum() + (M * ((ux - ut) ** 2 + (uy - vt) ** 2)).sum()


def _mass_weights(s):
    from paper_1910_13918_amd import sllbm as C
    mx = np.zeros(s.nx)
    my = np.zeros(s.ny)
    C.sllbm_mass_weights(s.ctx, mx.ctypes.data, my.ctypes.data)
    return torch.tensor(np.outer(my, mx).reshape(-1), device="cuda")


def _rollout_grad(wl, precision, nsteps, every, seed_target=1234):
    from paper_1910_13918_amd.adjoint import rollout
    s = _solver(wl, precision)
    X, Y = s.coords()
    rho0, ux0, uy0, _ = wl.fields(X, Y)
    ut, vt = W.fourier_target(X, Y, wl.meta["U0"], seed=seed_target)
    t = lambda a: torch.tensor(a, device="cuda")
    u0 = t(ux0).requires_grad_(True)
    v0 = t(uy0).requires_grad_(True)
    r0 = t(rho0).requires_grad_(True)
    rho, ux, uy = rollout(r0, u0, v0, s, nsteps, every)
    L = _loss_torch(rho, ux, uy, _mass_weights(s), t(ut), t(vt))
    L.backward()
    out = (float(L.detach()), u0.grad.detach().cpu().numpy(), v0.grad.detach().cpu().numpy(),
           r0.grad.detach().cpu().numpy(), s)
    return out


def test_rollout_gradient_matches_complex_step():
    """8 x 8 cells p = 4, 20 steps, checkpoints every 7 steps (uneven last
    segment): directional derivatives of the GPU gradient against the oracle's
    complex-step derivative."""
    wl = W.tgv(8, 4, U0=0.3, steps=20)
    L, gu, gv, gr, s = _rollout_grad(wl, "fp64", 20, 7)
    s.close()
    g = Grid(wl.edges_x, wl.edges_y, wl.p, True, True)
    sim = Sim(g, wl.dt, wl.nu, wl.model)
    X, Y = g.coords()
    rho0, ux0, uy0, T0 = wl.fields(X, Y)
    ut, vt = W.fourier_target(X, Y, 0.3)
    loss = lambda sm, F: kinetic_misfit_loss(sm, F, ut, vt)
    for d in W.random_directions(g.nnodes, 3, seed=4321):
        ref = complex_step_directional(sim, rho0, ux0, uy0, T0, d[0], d[1], 20, loss)
        got = float(np.dot(gu, d[0]) + np.dot(gv, d[1]))
        assert got == pytest.approx(ref, rel=1e-9, abs=1e-14)


def test_recorded_rollout_equals_checkpointed():
    """every = 0 (moments of every step recorded in the forward, no replay)
    gives the checkpointed gradient: the replay recomputes the same moments."""
    wl = W.tgv(16, 4, U0=0.3, steps=30)
    _, gu_c, gv_c, gr_c, s = _rollout_grad(wl, "fp64", 30, 7)
    s.close()
    _, gu_r, gv_r, gr_r, s = _rollout_grad(wl, "fp64", 30, 0)
    s.close()
    for a, b in ((gu_c, gu_r), (gv_c, gv_r), (gr_c, gr_r)):
        np.testing.assert_allclose(b, a, rtol=0, atol=1e-14 * np.abs(a).max())


def test_fp32_rollout_gradient_close_to_fp64():
    wl = W.tgv(16, 4, U0=0.3, steps=60)
    _, gu64, gv64, _, s = _rollout_grad(wl, "fp64", 60, 25)
    s.close()
    _, gu32, gv32, _, s = _rollout_grad(wl, "fp32", 60, 25)
    s.close()
    g64 = np.concatenate([gu64, gv64])
    g32 = np.concatenate([gu32, gv32])
    assert np.linalg.norm(g32 - g64) <= 1e-3 * np.linalg.norm(g64)


def test_adjoint_workload_against_central_differences():
    """The 128 x 128-cell, p = 4 Taylor-Green adjoint workload (500 steps,
    checkpoints every 50), FP64 path: the gradient's directional derivatives
    against central differences with eps = 1e-4 along 32 seeded directions;
    the FP32 rollout's gradient against the FP64 one (relative L2)."""
    from paper_1910_13918_amd.solver import Solver
    wl = W.adjoint_tgv()
    L, gu, gv, _, s = _rollout_grad(wl, "fp64", wl.steps, 50)
    M = _mass_weights(s)
    X, Y = s.coords()
    rho0, ux0, uy0, _ = wl.fields(X, Y)
    ut, vt = (torch.tensor(a, device="cuda") for a in W.fourier_target(X, Y, 0.3))

    def loss(dx, dy, e):
        s.init_macro(rho0, ux0 + e * dx, uy0 + e * dy, np.ones_like(rho0))
        s.step(wl.steps)
        rho, ux, uy, _ = s.moments_device()
        return float(_loss_torch(rho, ux, uy, M, ut, vt))

    try:
        print("[gpu] adjoint workload: 32 central differences (FP64)", flush=True)
        for d in W.random_directions(s.n, 32, seed=4321):
            fd = (loss(d[0], d[1], 1e-4) - loss(d[0], d[1], -1e-4)) / 2e-4
            got = float(np.dot(gu, d[0]) + np.dot(gv, d[1]))
            assert got == pytest.approx(fd, rel=1e-5)
    finally:
        s.close()
    _, gu32, gv32, _, s32 = _rollout_grad(wl, "fp32", wl.steps, 50)
    s32.close()
    g64, g32 = np.concatenate([gu, gv]), np.concatenate([gu32, gv32])
    rel = float(np.linalg.norm(g32 - g64) / np.linalg.norm(g64))
    print(f"[gpu] adjoint workload FP32 vs FP64 gradient: {rel:.2e} relative L2", flush=True)
    assert rel <= 1e-4  # measured 8.4e-6
    assert isinstance(Solver, type)


# ---------------------------------------------------------------- thermal models
def _thermal(wl, model, periodic=None):
    wl.model = model
    if periodic is not None:
        wl.periodic_x = wl.periodic_y = periodic
    base = wl.fields

    def fields(x, y):
        rho, ux, uy, _ = base(x, y)
        return rho, ux, uy, 1.0 + 0.1 * np.cos(2.0 * x) * np.sin(y)

    wl.fields = fields
    return wl


THERMAL = [
    ("monatomic", lambda: _thermal(W.tgv(9, 3, U0=0.3), "monatomic")),
    ("polyatomic", lambda: _thermal(W.riemann(14, 2, states=W.RIEMANN_TABLE3_STATES),
                                    "polyatomic")),
]


@pytest.mark.parametrize("path", ["tiled", "direct", "rows"])
@pytest.mark.parametrize("name,make", THERMAL, ids=[t[0] for t in THERMAL])
def test_thermal_transposed_streaming_dot_product(name, make, path):
    from paper_1910_13918_amd import sllbm as C
    wl = make()
    wl.nu = np.inf
    s = _solver(wl, "fp64", path)
    try:
        print(f"[gpu] thermal dot product {name} {path} nodes={s.n}", flush=True)
        shape = (s.nsets * 25, s.n)
        v, mu = _rand(shape, 5), _rand(shape, 6)
        s.set_populations(v)
        s.step(1)
        Sv = s.populations_device().reshape(shape)
        StMu = torch.empty_like(mu)
        C.sllbm_adjoint_step(s.ctx, mu.data_ptr(), None, StMu.data_ptr())
        torch.cuda.synchronize()
        assert float((mu * Sv).sum()) == pytest.approx(float((StMu * v).sum()), rel=1e-12)
    finally:
        s.close()


@pytest.mark.parametrize("name,make", THERMAL, ids=[t[0] for t in THERMAL])
def test_thermal_one_step_adjoint_against_central_differences(name, make):
    from paper_1910_13918_amd import sllbm as C
    wl = make()
    s = _solver(wl, "fp64")
    try:
        s.init_from_workload()
        s.step(3)
        F = s.populations_device().clone()
        shape = tuple(F.shape)
        lam = _rand(shape, 7)
        v = _rand(shape, 8) * F.abs().mean()
        s.set_populations(F)
        mom = s.step_record(1)
        assert mom.shape[1] == 4
        mu, out = torch.empty_like(lam), torch.empty_like(lam)
        C.sllbm_adjoint_collide(s.ctx, lam.data_ptr(), mom[0].data_ptr(), mu.data_ptr())
        C.sllbm_adjoint_step(s.ctx, mu.data_ptr(), None, out.data_ptr())
        torch.cuda.synchronize()
        adj = float((out * v).sum())

        def g(e):
            s.set_populations(F + e * v)
            s.step(1)
            return float((lam * s.populations_device()).sum())

        fd = (g(1e-6) - g(-1e-6)) / 2e-6
        assert adj == pytest.approx(fd, rel=1e-6)
    finally:
        s.close()


@pytest.mark.parametrize("model", ["monatomic", "polyatomic"])
def test_thermal_rollout_gradient_matches_complex_step(model):
    """8 x 8 cells p = 2, periodic, 12 steps with checkpoints every 5: the
    gradient with respect to (rho0, u0, v0, T0) of the kinetic energy + velocity
    and temperature misfit, along seeded directions, against the oracle's
    complex-step derivative."""
    from oracle.adjoint import complex_step_fields, thermal_misfit_loss
    from paper_1910_13918_amd.adjoint import rollout
    wl = _thermal(W.tgv(8, 2, U0=0.3, steps=12), model, periodic=True)
    s = _solver(wl, "fp64")
    try:
        X, Y = s.coords()
        f0 = wl.fields(X, Y)
        ut, vt = W.fourier_target(X, Y, 0.3, seed=1234)
        Tt = 1.0 + 0.05 * np.sin(X)
        t = lambda a: torch.tensor(a, device="cuda")
        leaves = [t(a).requires_grad_(True) for a in f0]
        rho, ux, uy, T = rollout(leaves[0], leaves[1], leaves[2], s, 12, 5, T0=leaves[3])
        M = _mass_weights(s)
        L = _loss_torch(rho, ux, uy, M, t(ut), t(vt)) + (M * (T - t(Tt)) ** 2).sum()
        L.backward()
        grads = [a.grad.detach().cpu().numpy() for a in leaves]
    finally:
        s.close()
    g = Grid(wl.edges_x, wl.edges_y, wl.p, True, True)
    sim = Sim(g, wl.dt, wl.nu, model, gamma=wl.gamma)
    loss = lambda sm, F: thermal_misfit_loss(sm, F, ut, vt, Tt)
    rng = np.random.default_rng(77)
    for _ in range(3):
        d = [rng.standard_normal(g.nnodes) for _ in range(4)]
        ref = complex_step_fields(sim, f0, d, 12, loss)
        got = sum(float(np.dot(gr, di)) for gr, di in zip(grads, d))
        assert got == pytest.approx(ref, rel=1e-9, abs=1e-13)


# ------------------------------------------------------------ viscosity gradient
@pytest.mark.parametrize("model", ["isothermal", "monatomic", "polyatomic"])
def test_nu_gradient_matches_complex_step(model):
    """dL/d(nu) through 10 steps (8 x 8 cells p = 3, periodic; Pr = 1) against
    the oracle's complex-step derivative in nu, and against central
    differences of the GPU loss itself."""
    from oracle.adjoint import complex_step_nu, thermal_misfit_loss
    from paper_1910_13918_amd.adjoint import nu_gradient
    wl = W.tgv(8, 3, U0=0.3, steps=10)
    if model != "isothermal":
        wl = _thermal(wl, model, periodic=True)
    wl.nu = 0.3 * wl.dt  # tau = 0.8
    s = _solver(wl, "fp64")
    try:
        X, Y = s.coords()
        f0 = wl.fields(X, Y)
        ut, vt = W.fourier_target(X, Y, 0.3, seed=99)
        Tt = 1.0 + 0.05 * np.sin(X)
        M = _mass_weights(s)
        t = lambda a: torch.tensor(a, device="cuda")

        def torch_loss(rho, ux, uy, T=None):
            L = _loss_torch(rho, ux, uy, M, t(ut), t(vt))
            return L if T is None else L + (M * (T - t(Tt)) ** 2).sum()

        def loss_grad(*m):
            leaves = [a.detach().clone().requires_grad_(True) for a in m]
            torch_loss(*leaves).backward()
            return [a.grad for a in leaves]

        T0 = f0[3] if model != "isothermal" else None
        got = nu_gradient(s, f0[0], f0[1], f0[2], 10, loss_grad, T0=T0)
        print(f"[gpu] nu gradient {model}: {got}", flush=True)
    finally:
        s.close()
    g = Grid(wl.edges_x, wl.edges_y, wl.p, True, True)
    sim = Sim(g, wl.dt, wl.nu, model, gamma=wl.gamma)
    if model == "isothermal":
        loss = lambda sm, F: kinetic_misfit_loss(sm, F, ut, vt)
    else:
        loss = lambda sm, F: thermal_misfit_loss(sm, F, ut, vt, Tt)
    ref = complex_step_nu(sim, f0, 10, loss)
    assert abs(ref) > 1e-3
    assert got == pytest.approx(ref, rel=1e-9)


@pytest.mark.parametrize("model,tau", [("isothermal", 0.8), ("polyatomic", 0.8),
                                       ("monatomic", 1.5)])
def test_nu_gradient_fp32_against_fp64(model, tau):
    """dL/d(nu) with float32 populations against the float64 path (10 steps,
    8 x 8 cells p = 3).  The term rebuilds f - f_eq before the collision as
    (f+ - f_eq) / (1 - 1/tau) from stored post-collision values: float32
    rounding of f+ (2^-24 relative) divided by the non-equilibrium part
    (about 1e-3 of f here) and amplified by 1 / |1 - 1/tau| (4 at tau = 0.8,
    3 at tau = 1.5; unbounded as tau -> 1, where the library refuses the
    exact value tau = 1).  Measured: 8.7e-7 (isothermal, tau = 0.8), 8.3e-7
    (polyatomic, 0.8), 1.2e-7 (monatomic, 1.5); bound 1e-5 relative."""
    from paper_1910_13918_amd.adjoint import nu_gradient
    wl = W.tgv(8, 3, U0=0.3, steps=10)
    if model != "isothermal":
        wl = _thermal(wl, model, periodic=True)
    wl.nu = (tau - 0.5) * wl.dt
    out = {}
    for prec in ("fp64", "fp32"):
        s = _solver(wl, prec)
        try:
            X, Y = s.coords()
            f0 = wl.fields(X, Y)
            ut, vt = W.fourier_target(X, Y, 0.3, seed=99)
            Tt = 1.0 + 0.05 * np.sin(X)
            M = _mass_weights(s)
            t = lambda a: torch.tensor(a, device="cuda")

            def loss_grad(*m):
                leaves = [a.detach().clone().requires_grad_(True) for a in m]
                L = _loss_torch(leaves[0], leaves[1], leaves[2], M, t(ut), t(vt))
                if len(leaves) == 4:
                    L = L + (M * (leaves[3] - t(Tt)) ** 2).sum()
                L.backward()
                return [a.grad for a in leaves]

            T0 = f0[3] if model != "isothermal" else None
            out[prec] = nu_gradient(s, f0[0], f0[1], f0[2], 10, loss_grad, T0=T0)
        finally:
            s.close()
    rel = abs(out["fp32"] - out["fp64"]) / abs(out["fp64"])
    print(f"[gpu] nu gradient {model} tau={tau}: fp32 {out['fp32']:.9e} fp64 {out['fp64']:.9e} "
          f"rel {rel:.3e}", flush=True)
    assert rel <= 1e-5


def test_nu_term_refused_at_tau_one():
    from paper_1910_13918_amd import sllbm as C
    wl = W.tgv(4, 2, U0=0.1)
    wl.nu = 0.5 * wl.dt  # tau = 1
    s = _solver(wl, "fp64")
    try:
        s.init_from_workload()
        lam = torch.zeros(s.nsets * s.q * s.n, dtype=torch.float64, device="cuda")
        mom = torch.ones(3 * s.n, dtype=torch.float64, device="cuda")
        acc = torch.zeros(1, dtype=torch.float64, device="cuda")
        with pytest.raises(C.SllbmError) as e:
            C.sllbm_adjoint_nu_term(s.ctx, lam.data_ptr(), lam.data_ptr(), mom.data_ptr(),
                                    acc.data_ptr())
        assert e.value.code == C.E_UNSUPPORTED
    finally:
        s.close()


@pytest.mark.parametrize("model", ["isothermal", "polyatomic"])
def test_checkpointed_rollout_nu_gradient(model):
    """rollout(..., nu=tensor) with checkpoints every 4 of 10 steps (uneven
    last segment) gives the same dL/d(nu) as the oracle's complex step, and
    the same field gradients as without the viscosity input."""
    from oracle.adjoint import complex_step_nu, thermal_misfit_loss
    from paper_1910_13918_amd.adjoint import rollout
    wl = W.tgv(8, 3, U0=0.3, steps=10)
    if model != "isothermal":
        wl = _thermal(wl, model, periodic=True)
    wl.nu = 0.3 * wl.dt
    s = _solver(wl, "fp64")
    try:
        X, Y = s.coords()
        f0 = wl.fields(X, Y)
        ut, vt = W.fourier_target(X, Y, 0.3, seed=99)
        Tt = 1.0 + 0.05 * np.sin(X)
        M = _mass_weights(s)
        t = lambda a: torch.tensor(a, device="cuda")

        def run(with_nu):
            leaves = [t(a).requires_grad_(True) for a in f0[:3]]
            T0 = t(f0[3]) if model != "isothermal" else None
            nu = torch.tensor(wl.nu, dtype=torch.float64, requires_grad=True) if with_nu else None
            out = rollout(*leaves, s, 10, 4, T0=T0, nu=nu)
            L = _loss_torch(*out[:3], M, t(ut), t(vt))
            if model != "isothermal":
                L = L + (M * (out[3] - t(Tt)) ** 2).sum()
            L.backward()
            return [a.grad.cpu().numpy() for a in leaves], (float(nu.grad) if with_nu else None)

        g_plain, _ = run(False)
        g_nu, dnu = run(True)
        print(f"[gpu] checkpointed nu gradient {model}: {dnu}", flush=True)
    finally:
        s.close()
    for a, b in zip(g_plain, g_nu):
        assert np.abs(a - b).max() <= 1e-12 * np.abs(a).max()
    g = Grid(wl.edges_x, wl.edges_y, wl.p, True, True)
    sim = Sim(g, wl.dt, wl.nu, model, gamma=wl.gamma)
    if model == "isothermal":
        loss = lambda sm, F: kinetic_misfit_loss(sm, F, ut, vt)
    else:
        loss = lambda sm, F: thermal_misfit_loss(sm, F, ut, vt, Tt)
    assert dnu == pytest.approx(complex_step_nu(sim, f0, 10, loss), rel=1e-9)


# ------------------------------------------------------------ Pr != 1
PRANDTL = [(m, Pr) for m in ("monatomic", "polyatomic") for Pr in (0.75, 2.0)]


def _prandtl(model, Pr):
    wl = dict(THERMAL)[model]()
    wl.Pr = Pr
    return wl


@pytest.mark.parametrize("model,Pr", PRANDTL)
def test_prandtl_one_step_adjoint_against_central_differences(model, Pr):
    """J^T of one step with the quasi-equilibrium collision (Sec. II.C-D):
    <J^T lam, v> against central differences of <lam, step(F + e v)>; the
    record carries the centred second moments of each set; the library's
    combined S^T + J_C^T call equals the two separate calls."""
    from paper_1910_13918_amd import sllbm as C
    wl = _prandtl(model, Pr)
    s = _solver(wl, "fp64")
    try:
        print(f"[gpu] Pr adjoint one step {model} Pr={Pr} nodes={s.n}", flush=True)
        s.init_from_workload()
        s.step(3)
        F = s.populations_device().clone()
        shape = tuple(F.shape)
        lam = _rand(shape, 7)
        v = _rand(shape, 8) * F.abs().mean()
        s.set_populations(F)
        mom = s.step_record(1)
        assert mom.shape[1] == 4 + 3 * s.nsets
        mu, out = torch.empty_like(lam), torch.empty_like(lam)
        C.sllbm_adjoint_collide(s.ctx, lam.data_ptr(), mom[0].data_ptr(), mu.data_ptr())
        C.sllbm_adjoint_step(s.ctx, mu.data_ptr(), None, out.data_ptr())
        torch.cuda.synchronize()
        adj = float((out * v).sum())

        def g(e):
            s.set_populations(F + e * v)
            s.step(1)
            return float((lam * s.populations_device()).sum())

        fd = (g(1e-6) - g(-1e-6)) / 2e-6
        assert adj == pytest.approx(fd, rel=1e-6)
        x = _rand(shape, 9)
        a1, a2, b = torch.empty_like(lam), torch.empty_like(lam), torch.empty_like(lam)
        C.sllbm_adjoint_step(s.ctx, x.data_ptr(), mom[0].data_ptr(), a1.data_ptr())
        C.sllbm_adjoint_step(s.ctx, x.data_ptr(), None, b.data_ptr())
        C.sllbm_adjoint_collide(s.ctx, b.data_ptr(), mom[0].data_ptr(), a2.data_ptr())
        torch.cuda.synchronize()
        assert torch.equal(a1, a2)
    finally:
        s.close()


@pytest.mark.parametrize("model", ["monatomic", "polyatomic"])
def test_prandtl_rollout_gradient_matches_complex_step(model):
    """12 steps at Pr = 0.75 (8 x 8 cells p = 2, periodic, checkpoints every
    5): the gradient in (rho0, u0, v0, T0) of the kinetic energy + velocity
    and temperature misfit, along seeded directions, against the oracle's
    complex-step derivative of the same Pr = 0.75 rollout."""
    from oracle.adjoint import complex_step_fields, thermal_misfit_loss
    from paper_1910_13918_amd.adjoint import rollout
    wl = _thermal(W.tgv(8, 2, U0=0.3, steps=12), model, periodic=True)
    wl.Pr = 0.75
    s = _solver(wl, "fp64")
    try:
        print(f"[gpu] Pr adjoint rollout {model}", flush=True)
        X, Y = s.coords()
        f0 = wl.fields(X, Y)
        ut, vt = W.fourier_target(X, Y, 0.3, seed=1234)
        Tt = 1.0 + 0.05 * np.sin(X)
        t = lambda a: torch.tensor(a, device="cuda")
        leaves = [t(a).requires_grad_(True) for a in f0]
        rho, ux, uy, T = rollout(leaves[0], leaves[1], leaves[2], s, 12, 5, T0=leaves[3])
        M = _mass_weights(s)
        L = _loss_torch(rho, ux, uy, M, t(ut), t(vt)) + (M * (T - t(Tt)) ** 2).sum()
        L.backward()
        grads = [a.grad.detach().cpu().numpy() for a in leaves]
    finally:
        s.close()
    g = Grid(wl.edges_x, wl.edges_y, wl.p, True, True)
    sim = Sim(g, wl.dt, wl.nu, model, gamma=wl.gamma, Pr=0.75)
    loss = lambda sm, F: thermal_misfit_loss(sm, F, ut, vt, Tt)
    rng = np.random.default_rng(78)
    for _ in range(3):
        d = [rng.standard_normal(g.nnodes) for _ in range(4)]
        ref = complex_step_fields(sim, f0, d, 12, loss)
        got = sum(float(np.dot(gr, di)) for gr, di in zip(grads, d))
        assert got == pytest.approx(ref, rel=1e-9, abs=1e-13)


def test_viscosity_term_refused_at_prandtl():
    from paper_1910_13918_amd import sllbm as C
    from paper_1910_13918_amd.adjoint import rollout
    wl = _prandtl("monatomic", 0.75)
    s = _solver(wl, "fp64")
    try:
        s.init_from_workload()
        mom = s.step_record(1)
        F = s.populations_device()
        lam = torch.zeros_like(F)
        acc = torch.zeros(1, dtype=torch.float64, device="cuda")
        with pytest.raises(C.SllbmError) as e:
            C.sllbm_adjoint_nu_term(s.ctx, lam.data_ptr(), F.data_ptr(), mom[0].data_ptr(),
                                    acc.data_ptr())
        assert e.value.code == C.E_UNSUPPORTED
        X, Y = s.coords()
        f0 = [torch.tensor(a, device="cuda") for a in wl.fields(X, Y)]
        nu = torch.tensor(wl.nu, dtype=torch.float64, requires_grad=True)
        with pytest.raises(ValueError):
            rollout(f0[0], f0[1], f0[2], s, 3, 2, T0=f0[3], nu=nu)
    finally:
        s.close()
