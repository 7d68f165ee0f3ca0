"""GPU parity of ILU(0) and the CPR comparator against the CPU oracle.

Bars: level counts, patterns and ILU(0) factors bit-exact (both sides
eliminate in the same order, without contraction, with correctly rounded
FP64 division); triangular solves within a backward error of 1e-12 (|b - L U x|
against |L| |U| |x| + |b|: the lanes of a row sum in another order); the CPR
apply within 1e-10 relative per block (the V-cycle's bar); FGMRES with CPR to
a true relative residual <= rtol in the oracle's iteration count +-1.
"""
import sys

import numpy as np
import pytest
import scipy.sparse as sp

import oracle
from paper_1902_00095_amd import solver, synth
from paper_1902_00095_amd import tpsolve as tps
from parity_bars import history_bound

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


def np_(t):
    return t.detach().cpu().numpy()


def dev(a, dtype=None):
    import torch
    return torch.as_tensor(np.ascontiguousarray(a), device="cuda", dtype=dtype)


CASES = {
    "W1": lambda: synth.make_problem("W1"),
    "W2s": lambda: synth.make_problem("W2", grid=synth.Grid(20, 18, 10, 1, 1, 1)),
    "W2g": lambda: synth.make_problem("W2", grid=synth.Grid(9, 7, 11, 1, 1, 2.0),
                                      props=synth.Props(g=9.80665)),
    "W2": lambda: synth.make_problem("W2"),
}


def _oracle_J_on_device(p):
    Jo = oracle.jacobian(p)
    return Jo, tps.Jacobian.from_host(Jo.n, Jo.rowptr, Jo.col, Jo.pp, Jo.pT, Jo.Tp, Jo.TT, Jo.S)


def _row_rel(a, b, rowptr):
    """max over rows of max |a - b| / max |b| within the row"""
    rows = np.repeat(np.arange(len(rowptr) - 1), np.diff(rowptr))
    scale = np.maximum.reduceat(np.abs(b), rowptr[:-1])
    return float((np.abs(a - b) / scale[rows]).max())


def _levels(rowptr, col):
    """Level counts of the forward and backward dependency graphs."""
    N = len(rowptr) - 1
    lev = np.zeros(N, np.int64)
    for i in range(N):
        c = col[rowptr[i]:rowptr[i + 1]]
        lo = c[c < i]
        lev[i] = lev[lo].max() + 1 if len(lo) else 0
    nl = int(lev.max()) + 1
    lev[:] = 0
    for i in range(N - 1, -1, -1):
        c = col[rowptr[i]:rowptr[i + 1]]
        hi = c[c > i]
        lev[i] = lev[hi].max() + 1 if len(hi) else 0
    return nl, int(lev.max()) + 1


@pytest.mark.parametrize("case", ["W1", "W2s", "W2g", "W2"])
def test_ilu0_factors_match_oracle(case):
    say("ilu0 factors", case)
    p = CASES[case]()
    Jo, Jd = _oracle_J_on_device(p)
    F = tps.ILU0.jacobian(Jd)
    rp, ci, lu = (np_(t) for t in F.factors())
    orp, oci, oval = oracle.jac_fieldwise(Jo)
    Fo = oracle.ILU0(orp, oci, oval)
    assert Fo.status == 0
    assert np.array_equal(rp, orp) and np.array_equal(ci, oci)
    err = _row_rel(lu, Fo.lu, rp)
    inf = F.info()
    say(f"  N {inf['N']} levels {inf['levels_lower']}/{inf['levels_upper']} "
        f"max row-relative factor difference {err:.2e} (bit-identical: {np.array_equal(lu, Fo.lu)})")
    assert np.array_equal(lu, Fo.lu), err
    if case != "W2":
        assert (inf["levels_lower"], inf["levels_upper"]) == _levels(orp, oci)


@pytest.mark.parametrize("case", ["W1", "W2s", "W2"])
def test_ilu0_solve_backward_error(case):
    say("ilu0 solve", case)
    p = CASES[case]()
    Jo, Jd = _oracle_J_on_device(p)
    F = tps.ILU0.jacobian(Jd)
    rp, ci, lu = (np_(t) for t in F.factors())
    N = len(rp) - 1
    A = sp.csr_matrix((lu, ci, rp), shape=(N, N))
    L = sp.tril(A, -1, format="csr") + sp.identity(N, format="csr")
    U = sp.triu(A, 0, format="csr")
    b = synth.random_rhs(4, N)
    b[N // 2:] *= 1e5                  # energy rows carry larger residuals
    x = np_(F.solve(dev(b)))
    res = np.abs(b - L @ (U @ x))
    bound = abs(L) @ (abs(U) @ np.abs(x)) + np.abs(b)
    worst = float((res / bound).max())
    say(f"  componentwise backward error {worst:.2e}")
    assert worst <= 1e-12
    if case != "W2":
        xo = oracle.ILU0(*oracle.jac_fieldwise(Jo)).solve(b)
        say(f"  relative difference to the oracle's solve {np.linalg.norm(x - xo) / np.linalg.norm(xo):.2e}")
    # in place (b and x the same array) gives the same result
    bd = dev(b)
    F.solve(bd, bd)
    assert np.array_equal(np_(bd), x)


def test_ilu0_exact_on_a_closed_pattern():
    """ilu0_create on a general CSR matrix: the cell-interleaved Jacobian of
    a 1-D grid is block tridiagonal with full 2 x 2 blocks, so ILU(0) is the
    exact factorisation and the solve inverts A."""
    say("ilu0 closed pattern")
    p = synth.make_problem("W2", grid=synth.Grid(40, 1, 1, 1, 1, 1))
    A = oracle.sparse_interleaved(oracle.jacobian(p))
    A.sort_indices()
    F = tps.ILU0(dev(A.indptr.astype(np.int32)), dev(A.indices.astype(np.int32)), dev(A.data))
    b = synth.random_rhs(2, A.shape[0])
    x = np_(F.solve(dev(b)))
    Ad = A.toarray()
    assert np.all(np.abs(Ad @ x - b) <= 1e-12 * (np.abs(Ad) @ np.abs(x) + np.abs(b)))


def test_ilu0_rejects_malformed_patterns():
    """Host checks before any factorisation kernel: a missing diagonal, an
    unsorted row, a column out of range."""
    say("ilu0 malformed")
    bad = [
        (np.array([0, 2, 3]), np.array([0, 1, 0]), "diagonal"),         # row 1 lacks (1, 1)
        (np.array([0, 2, 4]), np.array([1, 0, 0, 1]), "sorted"),         # row 0 unsorted
        (np.array([0, 2, 4]), np.array([0, 5, 0, 1]), "out of range"),
    ]
    for rp, ci, what in bad:
        with pytest.raises(tps.TpError) as e:
            tps.ILU0(dev(rp.astype(np.int32)), dev(ci.astype(np.int32)), dev(np.ones(len(ci))))
        assert e.value.code == tps.TP_ERR_ARG and what in str(e.value), (what, str(e.value))
    # a zero pivot is a numeric error
    with pytest.raises(tps.TpError) as e:
        tps.ILU0(dev(np.array([0, 2, 4], np.int32)), dev(np.array([0, 1, 0, 1], np.int32)),
                 dev(np.array([1.0, 1.0, 1.0, 1.0])))
    assert e.value.code == tps.TP_ERR_NUMERIC


def test_ilu0_refactor_equals_a_fresh_factorisation():
    say("ilu0 refactor")
    p = CASES["W2s"]()
    d = solver.to_device(p)
    J, G = solver.assemble(p, d)
    F = tps.ILU0.jacobian(J)
    d["x_k"] = d["x_k"].clone()
    d["x_k"][0::2] += 1e5              # another state: every pressure 1 bar higher
    J, G = solver.assemble(p, d, J, G)
    F.refactor(J)
    F2 = tps.ILU0.jacobian(J)
    a, b = np_(F.factors()[2]), np_(F2.factors()[2])
    assert np.array_equal(a, b)


def _cpr_pair(case, coarse_max):
    p = CASES[case]()
    Jo, Jd = _oracle_J_on_device(p)
    prm = tps.AmgParams(restriction=0, coarse_max=coarse_max)
    ao = oracle.AMG(Jo.n, Jo.rowptr, Jo.col, Jo.pp, **prm.oracle_kwargs())
    ag = tps.AMG(Jd.rowptr, Jd.col, Jd.pp, prm)
    Fo = oracle.cpr_ilu(Jo)
    Fg = tps.ILU0.jacobian(Jd)
    return p, Jo, Jd, ao, ag, Fo, Fg


@pytest.mark.parametrize("case,cm", [("W1", 64), ("W2s", 64), ("W2s", tps.AmgParams().coarse_max)])
def test_cpr_apply_matches_oracle(case, cm):
    say("cpr apply", case, cm)
    p, Jo, Jd, ao, ag, Fo, Fg = _cpr_pair(case, cm)
    M = tps.Precond.cpr(Jd, ag, Fg)
    r = synth.random_rhs(3, 2 * Jo.n)
    r[1::2] *= 1e5
    zo = oracle.cpr_apply(Jo, ao, Fo, r)
    zg = np_(M.apply(dev(r)))
    for blk in (0, 1):
        e = np.abs(zg[blk::2] - zo[blk::2]).max() / np.abs(zo[blk::2]).max()
        say(f"  block {blk}: {e:.2e}")
        assert e <= 1e-10, blk


@pytest.mark.parametrize("case", ["W1", "W2s", "W2g"])
def test_fgmres_cpr_matches_oracle(case):
    say("fgmres cpr", case)
    rtol = 1e-8
    p = CASES[case]()
    d = solver.to_device(p)
    J, G = solver.assemble(p, d)
    cfg = solver.SolveConfig(rtol=rtol, method="cpr")
    dx, st, hand = solver.solve(J, G, cfg, history=True)
    Jo = oracle.jacobian(p)
    bo = -oracle.residual(p)
    ao = oracle.AMG(Jo.n, Jo.rowptr, Jo.col, Jo.pp, **solver.amg_params(cfg, "pp").oracle_kwargs())
    xo, io = oracle.gmres_cpr(Jo, ao, oracle.cpr_ilu(Jo), bo, rtol=rtol)
    say(f"  gpu its {st['iters']} rel {st['rel_true']:.2e}; oracle its {io['iters']} rel {io['rel_true']:.2e}")
    assert st["converged"] and st["rel_true"] <= rtol
    assert io["converged"]
    assert abs(st["iters"] - io["iters"]) <= 1
    # the ILU(0) factors are bit-identical; the pressure V-cycle is the one
    # rounding difference: estimates within 1e-8 relative, or (one-level
    # A_pp hierarchy, the whole block solved by the dense inverse) within
    # u kappa(A_pp) h_0 (derivation in test_gpu_parity.history_bound)
    h_g, h_o = st["history"], io["history"]
    k = min(11, len(h_g), len(h_o))
    bound = history_bound(Jo, (hand[0].nlev,), h_o[:k], blocks=("pp",))
    say(f"  history max |d|/bound {np.max(np.abs(h_g[:k] - h_o[:k]) / bound):.2e}")
    assert np.all(np.abs(h_g[:k] - h_o[:k]) <= bound)
    x = np_(dx)
    for blk in (0, 1):
        d_go = np.linalg.norm(x[blk::2] - xo[blk::2]) / np.linalg.norm(xo[blk::2])
        say(f"  block {blk}: |gpu-oracle|/|oracle| {d_go:.2e}")
        assert d_go <= 1e-8
    for h in reversed(hand):
        h.close()


def test_cpr_graph_replay_matches_eager():
    """CPR's apply (a V-cycle, two small kernels and a few hundred
    level-scheduled solve launches) replayed from the captured graph gives
    bit-identical iterates to launching its kernels one by one."""
    import torch
    say("cpr graph replay")
    p = CASES["W2s"]()
    d = solver.to_device(p)
    J, G = solver.assemble(p, d)
    a_pp, F, M = solver.setup(J, solver.SolveConfig(method="cpr"))
    runs = []
    for graph in (False, True, True, False):
        x = torch.zeros_like(G)
        torch.cuda.synchronize()
        x, st = tps.fgmres_solve(J, M, -G, x=x, rtol=1e-10, history=True, graph=graph)
        torch.cuda.synchronize()
        runs.append((np_(x), st))
    x0, s0 = runs[0]
    say(f"  its {s0['iters']} rel {s0['rel_true']:.2e}")
    assert s0["converged"]
    for x, st in runs[1:]:
        assert st["iters"] == s0["iters"]
        assert np.array_equal(st["history"], s0["history"])
        assert np.array_equal(x, x0)
    M.close(); F.close(); a_pp.close()


def test_cpr_full_size_solve():
    """At the 64 x 64 x 32 workload the CPR solve converges to 1e-8 (true
    residual); its iteration count is reported beside the block
    preconditioner's."""
    say("cpr W2")
    p = CASES["W2"]()
    d = solver.to_device(p)
    J, G = solver.assemble(p, d)
    _, sc, hc = solver.solve(J, G, solver.SolveConfig(method="cpr"))
    _, sb, hb = solver.solve(J, G, solver.SolveConfig())
    say(f"  cpr its {sc['iters']} rel {sc['rel_true']:.2e}; block its {sb['iters']}")
    assert sc["converged"] and sc["rel_true"] <= 1e-8
    assert sb["converged"]
    for h in list(reversed(hc)) + list(reversed(hb)):
        h.close()
