"""Reference derivatives of the oracle (test infrastructure only).

The paper has no adjoint; the gradient of a loss of the final state with
respect to the initial velocity field is checked against the complex-step
derivative of the oracle itself:

    d L / d eps (u0 + eps d) = Im L(u0 + i h d) / h,   h = 1e-30,

which is exact to rounding because every operation of the step (interpolation
with geometry-only weights, moments, division by rho, the polynomial
equilibrium, the relaxation) is analytic in the populations and the cell
search depends only on the geometry.

The derivative with respect to the viscosity is taken the same way: the BGK
relaxation rate 1/tau, tau = nu/dt + 1/2 (Sec. II.D), is evaluated at
nu + i h (Pr = 1, so tau_Pr = tau); the interpolation weights do not depend
on nu.

``kinetic_misfit_loss`` is the loss used for the adjoint workload:
L = 1/2 sum_v M_v rho |u|^2 + sum_v M_v |u - u_target|^2 at the final step,
with M_v the exact integral of node v's shape function; ``thermal_misfit_loss``
adds sum_v M_v (T - T_target)^2 for the models with a temperature.
"""
import numpy as np


def kinetic_misfit_loss(sim, F, u_target, v_target):
    rho, ux, uy, _ = sim.moments(F)
    M = sim.grid.node_mass()
    ke = 0.5 * np.sum(M * rho * (ux * ux + uy * uy))
    mis = np.sum(M * ((ux - u_target) ** 2 + (uy - v_target) ** 2))
    return ke + mis


def complex_step_directional(sim, rho0, ux0, uy0, T0, dux, duy, nsteps, loss, h=1e-30):
    """Directional derivative of loss(run(init(rho0, ux0 + eps dux, uy0 + eps duy, T0)))."""
    ux = ux0 + 1j * h * dux
    uy = uy0 + 1j * h * duy
    F = sim.init(rho0.astype(complex), ux, uy, T0.astype(complex))
    F = sim.run(F, nsteps)
    return float(np.imag(loss(sim, F)) / h)


def thermal_misfit_loss(sim, F, u_target, v_target, T_target):
    rho, ux, uy, T = sim.moments(F)
    M = sim.grid.node_mass()
    return (0.5 * np.sum(M * rho * (ux * ux + uy * uy))
            + np.sum(M * ((ux - u_target) ** 2 + (uy - v_target) ** 2))
            + np.sum(M * (T - T_target) ** 2))


def complex_step_fields(sim, fields0, dfields, nsteps, loss, h=1e-30):
    """Directional derivative of loss(run(init(fields0 + eps dfields))) for the
    node fields (rho, u_x, u_y, T)."""
    rho, ux, uy, T = (np.asarray(f, dtype=complex) + 1j * h * np.asarray(d)
                      for f, d in zip(fields0, dfields))
    F = sim.run(sim.init(rho, ux, uy, T), nsteps)
    return float(np.imag(loss(sim, F)) / h)


def complex_step_nu(sim, fields0, nsteps, loss, h=1e-30):
    """d loss(run(init(fields0))) / d nu by complex step (Pr = 1)."""
    if sim.Pr != 1.0:
        raise ValueError("complex_step_nu covers Pr = 1")
    saved = sim.omega, sim.omega_pr
    sim.omega = sim.omega_pr = 1.0 / ((sim.nu + 1j * h) / sim.dt + 0.5)
    try:
        F = sim.run(sim.init(*[np.asarray(f, dtype=complex) for f in fields0]), nsteps)
        return float(np.imag(loss(sim, F)) / h)
    finally:
        sim.omega, sim.omega_pr = saved
