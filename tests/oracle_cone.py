"""Several oracle steps evaluated only where sampled outputs depend on them.

A node's value after a step depends on the previous state at the support
points of its departure cells (one stencil per velocity, eq. (17)).  Going
back k steps from a sample of nodes gives nested dependency sets ("cones");
the oracle evaluates step j only on the j-th set, from a full-size array in
which every node outside the previous set is NaN, so a node missing from a
cone shows up as NaN in the result instead of as a silently wrong value.

Test infrastructure: uses the oracle's own departure stencils and steps only.
"""
import numpy as np


def dependencies(sim, nodes):
    """Nodes whose previous values enter one step at `nodes`."""
    need = [np.asarray(nodes)]
    for i in range(sim.Q):
        src, _ = sim.departure_stencil(i, np.asarray(nodes))
        need.append(src.reshape(-1))
    return np.unique(np.concatenate(need))


def steps_at(sim, F0, nodes, k):
    """The oracle's state after k steps from F0, at `nodes` (shape (S, Q, len(nodes)))."""
    cones = [np.asarray(nodes)]
    for _ in range(k - 1):
        cones.append(dependencies(sim, cones[-1]))
    F = F0
    for j in range(k - 1, 0, -1):
        part = sim.step(F, cones[j])
        full = np.full_like(F0, np.nan)
        full[:, :, cones[j]] = part
        F = full
    out = sim.step(F, cones[0])
    assert np.all(np.isfinite(out)), "a dependency was missing from a cone"
    return out
