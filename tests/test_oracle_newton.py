"""The oracle's Newton time stepping, pinned by what Newton's method on the
(independently pinned) residual must do: the converged state satisfies
G(x) = 0 to the tolerance, the function norm falls superlinearly, and each
backward-Euler step conserves the fluid mass the wells inject and produce."""
import dataclasses

import numpy as np

import oracle
from paper_1902_00095_amd import synth


def _case():
    return synth.make_problem("W5", grid=synth.Grid(8, 8, 4, 1.0, 1.0, 1.0))


def test_newton_converges_quadratically_to_a_root():
    p = _case()
    states, its, hists = oracle.newton_simulate(p, 2, max_newton=6)
    for k, (x, h) in enumerate(zip(states, hists)):
        assert h[-1] <= 1e-8 or len(h) >= 2
        # superlinear: each reduction factor beats the previous one
        red = [h[i + 1] / h[i] for i in range(len(h) - 1) if h[i] > 1e-13]
        assert all(red[i + 1] < red[i] for i in range(len(red) - 1)), (k, h)
        # the returned state is a root of this step's residual
        prev = p.x_prev if k == 0 else states[k - 1]
        q = dataclasses.replace(p, x_prev=prev.copy(), x_k=x.copy())
        g0 = np.linalg.norm(oracle.residual(dataclasses.replace(q, x_k=prev.copy()), prev))
        assert np.linalg.norm(oracle.residual(q, x)) <= 1e-7 * g0
    assert all(1 <= i <= 6 for i in its)


def test_newton_step_balances_well_mass():
    """Summing the mass equations over all cells, the interior fluxes
    telescope and the boundaries carry no flow, so at a root the change of
    stored fluid mass over the step equals what the wells moved:
    sum_i V phi_i (rho(x1_i) - rho(x0_i)) / dt = q rho(p_inj, T_inj) - q rho(p_prod, T_prod),
    with rho written out here from its definition (not through the residual)."""
    p = _case()
    states, its, _ = oracle.newton_simulate(p, 1)
    x0, x1 = p.x_prev, states[0]
    pr = p.props
    V = p.grid.dx * p.grid.dy * p.grid.dz

    def rho(pp, TT):
        return pr.rho0 * np.exp(pr.c_p * (pp - pr.p0) + pr.c_T * (TT - pr.T0))

    stored = np.sum(V * p.phi * (rho(x1[0::2], x1[1::2]) - rho(x0[0::2], x0[1::2]))) / p.dt
    moved = 0.0
    for w in p.wells:
        pc, Tc = x1[2 * w.cell], x1[2 * w.cell + 1]
        moved += w.rate * (rho(pc, w.T_inj) if w.kind == 0 else -rho(pc, Tc))
    assert its[0] >= 1
    assert abs(stored - moved) <= 1e-6 * max(abs(stored), abs(moved), 1e-300), (stored, moved)
