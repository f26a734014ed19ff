"""sllbm_mass_noalloc: the mass reduction into a caller-owned device double
with the partial sums in the library's fixed per-device scratch (no device
allocation).  Checked through the C ABI against sllbm_mass on two calls in a
row, the second on a smaller grid (so it reuses the scratch that the larger
call left behind), and against its refusals.
"""
import numpy as np
import pytest
import torch

from paper_1910_13918_amd import sllbm as C
from paper_1910_13918_amd import workloads as W

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not torch.cuda.is_available(), reason="needs a HIP device")]


def _solver(ncells, p, precision):
    from paper_1910_13918_amd.solver import Solver
    s = Solver.from_workload(W.riemann(ncells, p), precision=precision)
    s.init_from_workload()
    s.step(3)  # a state that is not the initial one
    return s


def _noalloc(s):
    out = torch.full((1,), float("nan"), dtype=torch.float64, device=s.device)
    C.sllbm_mass_noalloc(s.ctx, out.data_ptr())
    torch.cuda.synchronize(s.device)
    return float(out.item())


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_mass_noalloc_matches_mass_on_two_calls(precision):
    big = _solver(160, 2, precision)     # 321^2 nodes: 403 partial sums
    small = _solver(12, 3, precision)    # 37^2 nodes: 6 partial sums
    try:
        for s in (big, small):
            print(f"[gpu] mass_noalloc {precision} nodes={s.n}", flush=True)
            ref = s.mass()
            got = _noalloc(s)
            # the same kernels in the same order: identical up to (here: no) rounding
            assert abs(got - ref) <= 1e-12 * abs(ref), (got, ref)
        # and again on the larger grid after the smaller call
        assert abs(_noalloc(big) - big.mass()) <= 1e-12 * abs(big.mass())
    finally:
        big.close()
        small.close()


def test_mass_noalloc_refusals():
    from paper_1910_13918_amd.solver import Solver
    s = Solver.from_workload(W.riemann(8, 2), precision="fp64")
    out = torch.zeros(1, dtype=torch.float64, device=s.device)
    try:
        with pytest.raises(C.SllbmError) as e:  # not initialised: no tables to use
            C.sllbm_mass_noalloc(s.ctx, out.data_ptr())
        assert e.value.code == C.E_STATE
        with pytest.raises(C.SllbmError) as e:
            C.sllbm_mass_noalloc(s.ctx, None)
        assert e.value.code == C.E_ARG
        s.init_from_workload()
        assert np.isclose(_noalloc(s), s.mass(), rtol=1e-14, atol=0.0)
    finally:
        s.close()
