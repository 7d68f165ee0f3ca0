"""The seeded input generator: determinism and the stated field statistics."""
import numpy as np

from paper_1902_00095_amd import synth


def test_deterministic():
    a = synth.make_problem("W2", grid=synth.Grid(16, 16, 8, 1, 1, 1))
    b = synth.make_problem("W2", grid=synth.Grid(16, 16, 8, 1, 1, 1))
    for k in ("K", "phi", "x_k"):
        assert np.array_equal(getattr(a, k), getattr(b, k))
    c = synth.make_problem("W2", seed=99, grid=synth.Grid(16, 16, 8, 1, 1, 1))
    assert not np.array_equal(a.K, c.K)


def test_layered_field_statistics():
    p = synth.make_problem("W2")
    logk = np.log10(p.K).reshape(p.grid.nz, -1)
    assert logk.min() >= -15 - 1e-12 and logk.max() <= -11 + 1e-12
    spread = logk.max(axis=1) - logk.min(axis=1)
    assert np.all(spread <= 0.4 + 1e-9)          # +-0.2 jitter within a layer
    assert np.std(logk.mean(axis=1)) > 0.5       # layer means ~ N(-13, 1)
    assert p.phi.min() >= 0.1 and p.phi.max() <= 0.3
    assert np.corrcoef(np.log10(p.K), p.phi)[0, 1] > 0.9


def test_channel_field():
    p = synth.make_problem("W4", grid=synth.Grid(48, 48, 48, 1, 1, 1))
    frac = np.mean(p.K > 1e-12)
    assert 0.005 < frac < 0.3
    assert set(np.unique(p.K)) <= {1e-15, 1e-11}
    assert p.wells[0].T_inj == 550.0


def test_perturbation_statistics():
    p = synth.make_problem("W2")
    dp = p.x_k[0::2] - p.x_prev[0::2]
    dT = p.x_k[1::2] - p.x_prev[1::2]
    assert abs(np.std(dp) / 1e5 - 1) < 0.02 and abs(np.std(dT) / 5 - 1) < 0.02


def test_refinement_recipe_uniform_start_and_corner_wells():
    for N in (20, 40):
        g = synth.Grid(N, N, 1, 20.0 / N, 20.0 / N, 1.0)
        p = synth.make_problem("R2", grid=g)
        assert p.grid.n == N * N and np.all(p.K == 1e-13) and np.all(p.phi == 0.2)
        assert np.array_equal(p.x_prev, p.x_k)
        assert np.all(p.x_k[0::2] == p.props.p0) and np.all(p.x_k[1::2] == p.props.T0)
        assert [(w.cell, w.kind) for w in p.wells] == [(0, 0), (N * N - 1, 1)]


def test_paper_heater_case():
    for N in (20, 80):
        g = synth.Grid(N, N, 1, 20.0 / N, 20.0 / N, 1.0)
        p = synth.make_problem("CaseI", grid=g)
        assert [w.kind for w in p.wells] == [2] * 6 and len({w.cell for w in p.wells}) == 6
        assert all(w.rate == 5.44409e-6 and w.T_inj == 422.039 for w in p.wells)
        assert np.all(p.x_k[1::2] == 288.706) and p.dt == 10 * 86400.0


def test_paper_anisotropic_cases():
    """Cases IV and V: K_x raised to 3e-11 m^2, K_y = K_z = 3e-13 m^2; Case IV
    heats as Case I, Case V runs the wells of Case III at 12-hour steps from
    288.706 K."""
    g = synth.Grid(40, 40, 1, 0.5, 0.5, 1.0)
    a, b = synth.make_problem("CaseIV", grid=g), synth.make_problem("CaseI", grid=g)
    assert a.K.shape == (3, g.n) and np.all(a.K[0] == 3e-11) and np.all(a.K[1:] == 3e-13)
    assert a.wells == b.wells and a.dt == b.dt
    v, w = synth.make_problem("CaseV", grid=g), synth.make_problem("CaseIII", grid=g)
    assert np.array_equal(v.K, a.K) and v.wells == w.wells and v.dt == 43200.0
    assert np.all(v.x_k[1::2] == 288.706)


def test_paper_well_cases():
    for name, T0, q in (("CaseII", 288.706, 5e-8), ("CaseIII", 320.0, 1e-6)):
        for N in (20, 80):
            g = synth.Grid(N, N, 1, 20.0 / N, 20.0 / N, 1.0)
            p = synth.make_problem(name, grid=g)
            assert np.all(p.K == 3e-13) and np.all(p.x_k[1::2] == T0) and p.dt == 10 * 86400.0
            assert [w.kind for w in p.wells] == [0, 0, 0, 1, 1, 1]
            assert all(w.rate == q for w in p.wells) and all(w.T_inj == 422.039 for w in p.wells)
            cells = {w.cell for w in p.wells}
            assert len(cells) == 6 and all(0 <= c < N * N for c in cells)
