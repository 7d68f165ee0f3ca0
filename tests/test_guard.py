"""The learned smoother's guard across solves (host logic, no GPU): when a
solve runs with the network, the contraction bound it passes, and when the
network is switched off for the rest of a run."""
import math

from paper_1902_00095_amd.solver import LearnedGuard


def st(rel, iters, fallback=-1, converged=True):
    return {"rel_true": rel, "iters": iters, "fallback_iter": fallback, "converged": converged}


def test_first_solve_is_plain_and_sets_the_reference():
    g = LearnedGuard()
    assert not g.use_net()
    g.record(st(1e-9, 6), 0.030, learned=False)
    assert g.use_net()
    # rho_p = rel^(1/iters); no learned solve timed yet: the bound is rho_p itself
    assert math.isclose(g.ref_rate(), 1e-9 ** (1 / 6), rel_tol=1e-12)


def test_bound_relaxed_by_the_cost_ratio():
    g = LearnedGuard()
    g.record(st(1e-9, 6), 0.030, learned=False)          # 5 ms per iteration
    g.record(st(1e-10, 6), 0.036, learned=True)          # 6 ms per iteration, 3.6 ms per decade
    rho = 1e-9 ** (1 / 6)
    assert math.isclose(g.ref_rate(), rho ** (6.0 / 5.0), rel_tol=1e-12)


def test_two_learned_solves_behind_in_a_row_switch_it_off_for_the_run():
    g = LearnedGuard()
    g.record(st(1e-9, 6), 0.030, learned=False)           # 3.33 ms per decade
    g.record(st(5e-9, 7), 0.040, learned=True)            # 4.8 ms per decade: slower
    assert g.use_net() and g.slower == 1
    g.record(st(2e-9, 8), 0.045, learned=True)            # 5.2 ms per decade: slower again
    assert not g.use_net()
    assert g.stats()["network_off_for_rest"]


def test_a_faster_learned_solve_resets_the_streak():
    g = LearnedGuard()
    g.record(st(1e-9, 6), 0.030, learned=False)
    g.record(st(1e-9, 10, fallback=7), 0.060, learned=True)   # switched off inside the solve
    assert g.use_net() and g.switched_off == 1
    g.record(st(1e-10, 5), 0.025, learned=True)               # 2.5 ms per decade: faster
    g.record(st(1e-9, 10, fallback=6), 0.060, learned=True)   # behind once more: streak 1 again
    assert g.use_net()
    assert g.stats() == {"learned_solves": 3, "plain_solves": 1, "network_switched_off": 2,
                         "slower_per_decade": 0, "network_off_for_rest": False}
