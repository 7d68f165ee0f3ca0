"""The allocation-free preconditioner apply (precond_apply_noalloc), called
through the C ABI, against precond_apply on the same handle: two calls in a
row, the second on a smaller system, for the block preconditioner (FP64 and
FP32 hierarchies) and for CPR.  The two entry points launch the same kernels
in the same order, so their outputs are compared bit for bit."""
import sys

import numpy as np
import pytest

from paper_1902_00095_amd import solver, synth
from paper_1902_00095_amd import tpsolve as tps

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module", autouse=True)
def _init():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    tps.init(0)
    yield


GRIDS = [synth.Grid(24, 20, 12, 1, 1, 1), synth.Grid(13, 9, 7, 1, 1, 1)]   # second: smaller, odd n


@pytest.mark.parametrize("cfg", [solver.SolveConfig(), solver.SolveConfig(storage=1),
                                 solver.SolveConfig(variant="full"), solver.SolveConfig(method="cpr")],
                         ids=["lower-fp64", "lower-fp32", "full-fp64", "cpr"])
def test_noalloc_apply_equals_apply(cfg):
    import torch
    for k, g in enumerate(GRIDS):
        say("noalloc", cfg.method, cfg.variant, cfg.storage, g.nx, g.ny, g.nz)
        p = synth.make_problem("W2", grid=g)
        d = solver.to_device(p)
        J, G = solver.assemble(p, d)
        a_pp, a_S, M = solver.setup(J, cfg)
        r = -G.clone()
        r[1::2] *= 1e-3
        z_ref = M.apply(r)
        z = torch.full_like(r, float("nan"))
        M.apply_noalloc(r, z)
        torch.cuda.synchronize()
        assert torch.isfinite(z).all()
        assert torch.equal(z, z_ref), f"grid {k}"
        # a second call on the same handle with another right-hand side
        r2 = torch.roll(r, 7)
        z_ref2 = M.apply(r2)
        M.apply_noalloc(r2, z)
        assert torch.equal(z, z_ref2), f"grid {k}, second rhs"
        M.close(); a_pp.close(); a_S.close()
