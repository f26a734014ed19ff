"""Pick the seed of the seeded four-quadrant Riemann workload.

Rule: starting from seed 0, accept the first seed whose quadrant states,
run with the FP64 oracle on 64 x 64 cells of order 2 (same CFL, viscosity and
end time t = 0.25 as the full workload), reach the end time with every node's
density and temperature positive and finite.  Writes riemann_seed.json next
to this script.  Calls only the oracle and the workload generator.

    python tests/golden/make_riemann_seed.py
"""
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle.grid import Grid  # noqa: E402
from oracle.sllbm import Sim  # noqa: E402
from paper_1910_13918_amd import workloads as W  # noqa: E402


def survives(seed, ncells=64):
    wl = W.riemann(ncells, 2, seed=seed)
    g = Grid(wl.edges_x, wl.edges_y, wl.p, wl.periodic_x, wl.periodic_y)
    sim = Sim(g, wl.dt, wl.nu, wl.model, gamma=wl.gamma, Pr=wl.Pr)
    X, Y = g.coords()
    F = sim.init(*wl.fields(X, Y))
    for n in range(wl.steps):
        F = sim.step(F)
        if n % 20 == 19 and sim.unstable(F):
            return False, n + 1
    return (not sim.unstable(F)), wl.steps


def main():
    log = []
    for seed in range(0, 50):
        t0 = time.time()
        ok, n = survives(seed)
        log.append({"seed": seed, "stable": bool(ok), "steps": n})
        print(f"seed {seed}: {'stable' if ok else 'unstable'} ({n} steps, {time.time() - t0:.0f} s)",
              flush=True)
        if ok:
            out = {"seed": seed, "rule": "first seed >= 0 stable to t = 0.25 on 64x64 cells, p = 2, "
                   "FP64 oracle", "states": W.riemann_states(seed), "tried": log}
            json.dump(out, open(os.path.join(HERE, "riemann_seed.json"), "w"), indent=1)
            return
    raise SystemExit("no stable seed in 0..49")


if __name__ == "__main__":
    main()
