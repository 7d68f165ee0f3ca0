"""The oracle's Newton time stepping, pinned by what Newton's method on the
(independently pinned) residual must do: the converged state satisfies
G(x) = 0 to the tolerance, the function norm falls superlinearly, and each
backward-Euler step conserves the fluid mass the wells inject and produce."""
import dataclasses

import numpy as np
import pytest

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


def test_line_search_affine_takes_the_full_step():
    """For affine G the Newton step is exact: lam = 1 with no backtracking."""
    A = np.array([[3.0, 1.0], [1.0, 2.0]])
    b = np.array([1.0, -2.0])
    x = np.array([5.0, 7.0])
    G = A @ x - b
    dx = np.linalg.solve(A, -G)
    lam, xt, Gt, rej = oracle.line_search_step(lambda y: A @ y - b, x, dx, float(G @ G))
    assert lam == 1.0 and rej == 0 and np.abs(Gt).max() < 1e-12


def test_line_search_rescues_newton_on_arctan():
    """Textbook case: Newton on arctan(x) = 0 diverges from x0 = 3 (any start
    with |x0| beyond about 1.39); the damped iteration converges to 0.  Every
    rejected trial violates the sufficient-decrease test and every accepted
    one satisfies it."""
    G = lambda y: np.arctan(y)
    x = np.array([3.0])
    xf = x.copy()
    for _ in range(4):
        xf = xf - np.arctan(xf) * (1.0 + xf * xf)
    assert abs(xf[0]) > 1e3
    for _ in range(30):
        g = G(x)
        g2 = float(g @ g)
        if g2 < 1e-28:
            break
        dx = -g * (1.0 + x * x)
        lam, xn, gn, rej = oracle.line_search_step(G, x, dx, g2)
        assert 0.5 * float(gn @ gn) <= 0.5 * g2 - 1e-4 * lam * g2
        if rej:
            assert 0.5 * float(G(x + dx) @ G(x + dx)) > 0.5 * g2 - 1e-4 * g2
            assert lam <= 0.5
        x = xn
    assert abs(x[0]) < 1e-14


def test_line_search_newton_reaches_the_same_root():
    """With high-rate wells the first Newton step of a step is damped (lam < 1);
    the damped iteration still converges, to the root the full-step iteration
    finds."""
    import dataclasses
    p = synth.make_problem("W5", grid=synth.Grid(10, 10, 2, 2.0, 2.0, 1.0))
    p.wells = [dataclasses.replace(w, rate=1e-4) for w in p.wells]
    xs, its, _ = oracle.newton_simulate(p, 1, max_newton=12)
    xl, itl, hl, lams = oracle.newton_simulate(p, 1, max_newton=12, line_search=True)
    assert min(lams[0]) < 1.0 and hl[0][-1] <= 1e-8
    for blk in (0, 1):
        assert np.linalg.norm(xl[0][blk::2] - xs[0][blk::2]) <= 1e-9 * np.linalg.norm(xs[0][blk::2])


def test_line_search_rejects_non_finite_trials():
    """A trial whose residual is not finite (as a state outside the fluid
    laws' range gives) is rejected and halves the step, whatever the
    quadratic model would say.  On G(y) = y - 1 with G NaN for y > 2, a
    wild step of 4 from 0 first lands on a NaN (lam = 1), the halving gives
    lam = 0.5 (y = 2, finite but no decrease), and the quadratic model then
    takes over; the accepted lam passes the sufficient-decrease test.  A
    NaN compared with a bound is False, so a rule without the finiteness
    test would keep the NaN in lam for every later trial."""
    def G_at(y):
        return np.array([np.nan if y[0] > 2.0 else y[0] - 1.0])

    x = np.zeros(1)
    dx = np.array([4.0])
    g2 = 1.0
    lam, xt, Gt, rej = oracle.line_search_step(G_at, x, dx, g2)
    assert np.isfinite(Gt).all()
    assert rej >= 1 and lam <= 0.5
    # f(lam) = (4 lam - 1)^2 / 2 must satisfy the sufficient-decrease test
    assert 0.5 * (4 * lam - 1) ** 2 <= 0.5 - 1e-4 * lam * g2
    # the first trial (lam = 1) was NaN: a halving, not a quadratic-model step,
    # took lam to 0.5 -- replaying the rule by hand gives the same lam
    seq, l = [], 1.0
    while True:
        f1 = 0.5 * float(G_at(x + l * dx) @ G_at(x + l * dx))
        if np.isfinite(f1) and f1 <= 0.5 * g2 - 1e-4 * l * g2:
            break
        if np.isfinite(f1):
            l = min(max(g2 * l * l / (2.0 * (f1 - 0.5 * g2 + g2 * l)), 0.1 * l), 0.5 * l)
        else:
            l = 0.5 * l
        seq.append(l)
    assert seq[0] == 0.5 and lam == l


def test_line_search_raises_when_every_trial_is_non_finite():
    with pytest.raises(FloatingPointError):
        oracle.line_search_step(lambda y: np.array([np.inf]), np.zeros(1), np.ones(1), 1.0)
