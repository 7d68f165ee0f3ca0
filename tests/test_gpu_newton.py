"""GPU Newton time stepping (assembly, both AMG setups and FGMRES per Newton
iteration) against the oracle's exact-Newton reference (sparse direct linear
steps) on a small grid of the 256x256x64 workload's recipe."""
import numpy as np
import pytest

import oracle
from paper_1902_00095_amd import solver, synth
from paper_1902_00095_amd import tpsolve as tps

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)


@pytest.fixture(scope="module", autouse=True)
def _init():
    import torch
    assert torch.cuda.is_available()
    tps.init(0)
    yield


@pytest.mark.parametrize("storage", [0, 1])
def test_newton_time_steps_match_oracle(storage):
    say("newton", storage)
    p = synth.make_problem("W5", grid=synth.Grid(16, 16, 8, 1.0, 1.0, 1.0))
    steps = 2
    xo, its_o, _ = oracle.newton_simulate(p, steps)
    x, st = solver.simulate(p, solver.SolveConfig(storage=storage), solver.NewtonConfig(steps=steps))
    xg = x.cpu().numpy()
    say(f"  newton per step gpu {st['newton_per_step']} oracle {its_o}, linear/newton {st['linear_per_newton']:.1f}")
    assert st["unconverged_steps"] == 0
    assert all(abs(a - b) <= 1 for a, b in zip(st["newton_per_step"], its_o))
    for blk in (0, 1):
        ref = xo[-1][blk::2]
        err = np.linalg.norm(xg[blk::2] - ref) / np.linalg.norm(ref)
        chg = np.linalg.norm(ref - p.x_prev[blk::2]) / np.linalg.norm(ref)
        say(f"  block {blk}: rel err {err:.2e} (state change over the run {chg:.2e})")
        assert err <= 1e-9
