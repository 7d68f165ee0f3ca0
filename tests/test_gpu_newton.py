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


@pytest.mark.parametrize("storage,reuse,method,interp_pp", [
    (0, False, "block", None), (1, False, "block", None), (0, True, "block", None), (1, True, "block", None),
    (0, False, "cpr", None), (0, True, "cpr", None), (1, False, "block", 1), (1, True, "block", 1),
    (0, "numeric", "block", None), (1, "numeric", "block", None), (1, "numeric_run", "block", None),
    (0, "numeric", "cpr", None), (0, "numeric", "block", 1)])
def test_newton_time_steps_match_oracle(storage, reuse, method, interp_pp):
    """With hierarchy reuse the later Newton iterations of a step run on
    refreshed hierarchies: the finest level only ("fine"), or every level
    recomputed on the kept splits and patterns ("numeric"; "numeric_run" keeps
    them for the whole run; an extended+i pressure hierarchy is rebuilt
    instead); the Newton root, and so the states, must not change.  CPR keeps one ILU(0) handle for the run and refactorises it for
    every Jacobian."""
    say("newton", storage, reuse, method, interp_pp)
    p = synth.make_problem("W5", grid=synth.Grid(16, 16, 8, 1.0, 1.0, 1.0))
    steps = 2
    xo, its_o, _ = oracle.newton_simulate(p, steps)
    x, st = solver.simulate(p, solver.SolveConfig(storage=storage, amg=tps.AmgParams(coarse_max=200),
                                                  method=method, interp_pp=interp_pp),
                            solver.NewtonConfig(steps=steps, reuse=reuse))
    assert st["hierarchy_builds"] + st["hierarchy_refreshes"] == st["solves"]
    if reuse in (True, "numeric"):
        assert st["hierarchy_builds"] == steps < st["solves"]
    elif reuse == "numeric_run":
        assert 1 <= st["hierarchy_builds"] < st["solves"]
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


def test_refresh_fine_in_place():
    """Refreshing the finest level with the values it was built on leaves the
    V-cycle bit for bit unchanged; with another state's values the level-0
    operator reads back as the new values and the V-cycle changes; refreshing
    back restores the original V-cycle exactly.  Both the pressure hierarchy
    (Galerkin) and the Schur one (Petrov-Galerkin), FP64 and FP32."""
    import torch
    say("refresh fine")
    p = synth.make_problem("W2", grid=synth.Grid(20, 18, 10, 1.0, 1.0, 1.0))
    d = solver.to_device(p)
    J1, _ = solver.assemble(p, d)
    d2 = dict(d)
    d2["x_k"] = d["x_k"] + 0.01 * torch.abs(d["x_k"]) * torch.randn(d["x_k"].shape, dtype=torch.float64,
                                                                      device="cuda", generator=torch.Generator(device="cuda").manual_seed(3))
    J2, _ = solver.assemble(p, d2)
    b = torch.as_tensor(synth.random_rhs(5, J1.n), device="cuda")
    for storage in (0, 1):
        for which, restr in (("pp", 0), ("S", 1)):
            v1, v2 = getattr(J1, which), getattr(J2, which).clone()
            a = tps.AMG(J1.rowptr, J1.col, v1.clone(), tps.AmgParams(restriction=restr, storage=storage, coarse_max=64))
            assert a.nlev >= 2
            y0 = a.vcycle(b).cpu().numpy()
            a.refresh_fine(v1.clone())
            assert np.array_equal(a.vcycle(b).cpu().numpy(), y0)
            a.refresh_fine(v2)
            assert np.array_equal(a.level(0)["A_val"].cpu().numpy(), v2.cpu().numpy())
            assert not np.array_equal(a.vcycle(b).cpu().numpy(), y0)
            a.refresh_fine(v1.clone())
            assert np.array_equal(a.vcycle(b).cpu().numpy(), y0), (storage, which)
            a.close()


def test_newton_line_search_matches_oracle():
    """Newton with line search (Section 4, opening) on high-rate wells, where the first
    increment of the step is damped: the GPU takes the oracle's step lengths
    and reaches its state."""
    import dataclasses
    say("newton line search")
    p = synth.make_problem("W5", grid=synth.Grid(10, 10, 2, 2.0, 2.0, 1.0))
    p.wells = [dataclasses.replace(w, rate=1e-4) for w in p.wells]
    xo, its_o, _, lams_o = oracle.newton_simulate(p, 1, max_newton=12, line_search=True)
    x, st = solver.simulate(p, solver.SolveConfig(amg=tps.AmgParams(coarse_max=100)),
                            solver.NewtonConfig(steps=1, max_newton=12, line_search=True))
    say(f"  step lengths gpu {st['step_lengths']} oracle {lams_o[0]}")
    assert st["unconverged_steps"] == 0 and st["backtracks"] >= 1
    assert abs(st["newton_per_step"][0] - its_o[0]) <= 1
    n = min(len(lams_o[0]), len(st["step_lengths"]))
    # the increments are FGMRES solutions to rtol 1e-8 (the oracle solves directly), and the
    # rejected full step lies far from the root, where G magnifies that difference
    assert np.allclose(st["step_lengths"][:n], lams_o[0][:n], rtol=1e-4, atol=0)
    # both stop on the step-norm test |dx| <= 1e-8 |x|, which the pressure (1e7 Pa)
    # dominates; from the damped start the two iterations end 1e-7 apart
    xg = x.cpu().numpy()
    for blk in (0, 1):
        ref = xo[-1][blk::2]
        err = np.linalg.norm(xg[blk::2] - ref) / np.linalg.norm(ref)
        say(f"  block {blk}: rel err {err:.2e}")
        assert err <= 1e-6


@pytest.mark.parametrize("case", ["CaseV", "CaseI"])
def test_newton_paper_physics_matches_oracle(case):
    """The paper's physics together: Bennison heavy oil, the anisotropic well case
    (V) with its constant-rate wells replaced by Peaceman wells, or the heater
    case (I); Newton with line search, no iteration cap of 4.  States as the
    oracle's exact-Newton reference."""
    import dataclasses
    say("newton paper physics", case)
    g = synth.Grid(16, 16, 1, 20.0 / 16, 20.0 / 16, 1.0)
    p = synth.make_problem(case, grid=g, props=synth.Props(api=10.0))
    if case == "CaseV":
        wi = synth.peaceman_wi(3e-11, 3e-13)
        p0 = p.props.p0
        p.wells = [dataclasses.replace(w, kind=3 + w.kind, rate=5e-6, p_bh=p0 + (2e5 if w.kind == 0 else -2e5), wi=wi)
                   for w in p.wells]
    xo, its_o, hists, lams_o = oracle.newton_simulate(p, 2, max_newton=20, line_search=True)
    x, st = solver.simulate(p, solver.SolveConfig(interp_pp=1), solver.NewtonConfig(steps=2, max_newton=20, line_search=True))
    say(f"  newton per step gpu {st['newton_per_step']} oracle {its_o}, backtracks {st['backtracks']}")
    assert st["unconverged_steps"] == 0
    assert all(abs(a - b) <= 1 for a, b in zip(st["newton_per_step"], its_o))
    xg = x.cpu().numpy()
    for blk in (0, 1):
        ref = xo[-1][blk::2]
        err = np.linalg.norm(xg[blk::2] - ref) / np.linalg.norm(ref)
        say(f"  block {blk}: rel err {err:.2e}")
        assert err <= 1e-6
