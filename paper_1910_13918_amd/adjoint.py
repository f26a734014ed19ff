"""Gradients through an SLLBM rollout for torch autograd (every model).

``rollout(rho0, ux0, uy0, solver, nsteps, every, T0)`` initialises the solver
at equilibrium with the given node fields, advances ``nsteps`` steps and
returns the final node moments (rho, u_x, u_y, and T unless isothermal).  Its
backward pass runs the adjoint of every step in the library:

* forward: a copy of the populations is kept every ``every`` steps;
* backward: for each segment, newest first, the checkpoint is restored and the
  segment replayed with ``sllbm_step_record`` (which keeps only the moments
  per node and step that the collision Jacobian needs: rho, u and, unless
  isothermal, theta; with Pr != 1 also each set's centred second moments),
  then ``mu = J_C^T lambda`` and ``lambda = S^T mu`` are applied step by
  step, and finally the gradient is carried through the initialisation
  F = F_eq.

Memory: one population copy per checkpoint plus K float64 per node and step
of one segment (K = 3 isothermal, 4 thermal, 4 + 3 S at Pr != 1).  With ``every=0`` the forward records the moments of
every step instead (24 or 32 bytes per node and step: 3.1 GB for 500
isothermal steps of 512^2 nodes) and the backward replays nothing.  Every
arithmetic step runs in the HIP kernels; this module only sequences the calls
and owns the torch buffers.
"""
import torch

from . import sllbm as C


class SLLBMRollout(torch.autograd.Function):
    @staticmethod
    def forward(ctx, rho0, ux0, uy0, T0, nu, solver, nsteps, every):
        dev = solver.device
        thermal = solver.model != "isothermal"
        rho0 = rho0.detach().to(device=dev, dtype=torch.float64).contiguous()
        ux0 = ux0.detach().to(device=dev, dtype=torch.float64).contiguous()
        uy0 = uy0.detach().to(device=dev, dtype=torch.float64).contiguous()
        T0 = (T0.detach().to(device=dev, dtype=torch.float64).contiguous() if T0 is not None
              else torch.ones_like(rho0))
        solver.init_macro(rho0, ux0, uy0, T0)
        checkpoints, lengths, record = [], [], None
        if every == 0:
            record = solver.step_record(nsteps) if nsteps > 0 else None
        else:
            done = 0
            while done < nsteps:
                k = min(every, nsteps - done)
                checkpoints.append(solver.populations_device())
                lengths.append(k)
                solver.step(k)
                done += k
        final = solver.populations_device()
        rho, ux, uy, T = solver.moments_device()
        ctx.save_for_backward(rho0, ux0, uy0, T0)
        ctx.solver = solver
        ctx.checkpoints = checkpoints
        ctx.lengths = lengths
        ctx.record = record
        ctx.final = final
        ctx.thermal = thermal
        ctx.nu_dtype = nu.dtype if nu is not None else None
        ctx.nu_device = nu.device if nu is not None else None
        return rho, ux, uy, T

    @staticmethod
    def backward(ctx, g_rho, g_ux, g_uy, g_T):
        rho0, ux0, uy0, T0 = ctx.saved_tensors
        s = ctx.solver
        dev = s.device
        zeros = torch.zeros(s.n, dtype=torch.float64, device=dev)
        g = [t.to(dtype=torch.float64).contiguous() if t is not None else zeros
             for t in (g_rho, g_ux, g_uy, g_T)]
        lam = torch.empty((s.nsets, s.q, s.n), dtype=s.dtype, device=dev)
        mu = torch.empty_like(lam)
        mu2 = torch.empty_like(lam)
        s.set_populations(ctx.final)
        C.sllbm_adjoint_seed(s.ctx, g[0].data_ptr(), g[1].data_ptr(), g[2].data_ptr(),
                             g[3].data_ptr() if ctx.thermal else None, lam.data_ptr())

        want_nu = ctx.needs_input_grad[4]
        acc = torch.zeros(1, dtype=torch.float64, device=dev)

        def reverse_segment(mom, L, states=None):
            # states (dL/d(nu) wanted): the post-collision populations of the
            # segment's steps; lambda is then formed at every step (S^T and
            # J_C^T as two calls) so that each step's viscosity term can use it
            nonlocal mu, mu2
            if states is not None:
                C.sllbm_adjoint_nu_term(s.ctx, lam.data_ptr(), states[L - 1].data_ptr(),
                                        mom[L - 1].data_ptr(), acc.data_ptr())
            C.sllbm_adjoint_collide(s.ctx, lam.data_ptr(), mom[L - 1].data_ptr(), mu.data_ptr())
            for t in range(L - 1, 0, -1):
                if states is None:
                    C.sllbm_adjoint_step(s.ctx, mu.data_ptr(), mom[t - 1].data_ptr(),
                                         mu2.data_ptr())
                    mu, mu2 = mu2, mu
                else:
                    C.sllbm_adjoint_step(s.ctx, mu.data_ptr(), None, lam.data_ptr())
                    C.sllbm_adjoint_nu_term(s.ctx, lam.data_ptr(), states[t - 1].data_ptr(),
                                            mom[t - 1].data_ptr(), acc.data_ptr())
                    C.sllbm_adjoint_collide(s.ctx, lam.data_ptr(), mom[t - 1].data_ptr(),
                                            mu.data_ptr())
            C.sllbm_adjoint_step(s.ctx, mu.data_ptr(), None, lam.data_ptr())

        if ctx.record is not None:
            reverse_segment(ctx.record, ctx.record.shape[0])
        for ck, L in zip(reversed(ctx.checkpoints), reversed(ctx.lengths)):
            s.set_populations(ck)
            if want_nu:
                mom, states = [], []
                for _ in range(L):
                    mom.append(s.step_record(1)[0])
                    states.append(s.populations_device())
                reverse_segment(mom, L, states)
            else:
                reverse_segment(s.step_record(L), L)
        out = [torch.empty(s.n, dtype=torch.float64, device=dev) for _ in range(4)]
        C.sllbm_eq_init_vjp(s.ctx, lam.data_ptr(), rho0.data_ptr(), ux0.data_ptr(), uy0.data_ptr(),
                            T0.data_ptr(), *[o.data_ptr() for o in out])
        gT = out[3] if ctx.thermal else None
        gnu = acc.reshape(()).to(device=ctx.nu_device, dtype=ctx.nu_dtype) if want_nu else None
        return out[0], out[1], out[2], gT, gnu, None, None, None


def rollout(rho0, ux0, uy0, solver, nsteps, every=50, T0=None, nu=None):
    """Final (rho, u_x, u_y) -- and T for the monatomic and polyatomic models --
    after nsteps from F = F_eq(rho0, u0, T0); differentiable in rho0, ux0, uy0
    (and T0).  every > 0: checkpoint interval (the backward replays each
    segment); every = 0: record every step's moments in the forward.

    nu: optional 0-dim tensor holding the solver's viscosity; when it requires
    grad, the backward also gives dL/d(nu) (Pr = 1, tau != 1, every > 0; each
    replayed segment then keeps its steps' populations).  The gradients in the
    initial fields cover every Prandtl number."""
    if every < 0:
        raise ValueError("every must be >= 0")
    if solver.model != "isothermal" and T0 is None:
        raise ValueError("the initial temperature T0 is needed unless isothermal")
    if nu is not None:
        if every == 0 and nu.requires_grad:
            raise ValueError("the viscosity gradient needs checkpoints (every > 0)")
        if abs(float(nu) - solver.nu) > 1e-12 * abs(solver.nu):
            raise ValueError("nu must hold the solver's viscosity")
        if nu.requires_grad and solver.Pr != 1.0:
            raise ValueError("the viscosity gradient covers Pr = 1")
    rho, ux, uy, T = SLLBMRollout.apply(rho0, ux0, uy0, T0, nu, solver, nsteps, every)
    return (rho, ux, uy) if solver.model == "isothermal" else (rho, ux, uy, T)


def nu_gradient(solver, rho0, ux0, uy0, nsteps, loss_grad, T0=None):
    """dL/d(nu) of a loss L of the final node moments after nsteps from
    F = F_eq(rho0, u0, T0) (Pr = 1, tau != 1).  loss_grad(rho, ux, uy[, T])
    receives the final moments (float64 device tensors; T unless isothermal)
    and returns dL/d of each, in the same order.

    The forward keeps every step's post-collision populations and moments
    (one population copy per step: for short rollouts); the backward runs the
    adjoint step by step and adds each step's viscosity term
    (sllbm_adjoint_nu_term) on the device.  Returns (L-independent) dL/d(nu)
    as a Python float."""
    dev = solver.device
    thermal = solver.model != "isothermal"
    if thermal and T0 is None:
        raise ValueError("the initial temperature T0 is needed unless isothermal")
    f64 = dict(device=dev, dtype=torch.float64)
    fields = [torch.as_tensor(a, **f64).contiguous() for a in (rho0, ux0, uy0)]
    fields.append(torch.as_tensor(T0, **f64).contiguous() if thermal
                  else torch.ones_like(fields[0]))
    solver.init_macro(*fields)
    states, moments = [], []
    for _ in range(nsteps):
        moments.append(solver.step_record(1)[0])
        states.append(solver.populations_device())
    rho, ux, uy, T = solver.moments_device()
    g = loss_grad(rho, ux, uy, T) if thermal else loss_grad(rho, ux, uy)
    g = [t.to(**f64).contiguous() for t in g]
    lam = torch.empty((solver.nsets, solver.q, solver.n), dtype=solver.dtype, device=dev)
    mu = torch.empty_like(lam)
    acc = torch.zeros(1, **f64)
    C.sllbm_adjoint_seed(solver.ctx, g[0].data_ptr(), g[1].data_ptr(), g[2].data_ptr(),
                         g[3].data_ptr() if thermal else None, lam.data_ptr())
    for n in range(nsteps - 1, -1, -1):
        C.sllbm_adjoint_nu_term(solver.ctx, lam.data_ptr(), states[n].data_ptr(),
                                moments[n].data_ptr(), acc.data_ptr())
        C.sllbm_adjoint_collide(solver.ctx, lam.data_ptr(), moments[n].data_ptr(), mu.data_ptr())
        C.sllbm_adjoint_step(solver.ctx, mu.data_ptr(), None, lam.data_ptr())
    torch.cuda.synchronize(dev)
    return float(acc.item())
