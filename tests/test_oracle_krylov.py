"""Pins of the oracle's block preconditioner and restarted GMRES(30)+CGS2."""
import numpy as np
import pytest
import scipy.sparse as sp

import oracle
from paper_1902_00095_amd import synth


def _dense_csr(M):
    n, m = M.shape
    rp = np.arange(0, n * m + 1, m).astype(np.int32)
    c = np.tile(np.arange(m), n).astype(np.int32)
    return rp, c, M.reshape(-1).copy()


def _setup(dims=(5, 4, 3), seed=3, props=None):
    p = synth.make_problem("W2", seed=seed, grid=synth.Grid(*dims, 1.0, 1.0, 1.0),
                           props=props or synth.Props())
    J = oracle.jacobian(p)
    b = -oracle.residual(p)
    return p, J, b


def _exact_hierarchies(J, schur="exact"):
    App, ApT, ATp, ATT = (J.block(k).toarray() for k in ["pp", "pT", "Tp", "TT"])
    S = ATT - ATp @ np.linalg.solve(App, ApT) if schur == "exact" else J.block("S").toarray()
    a_pp = oracle.AMG(J.n, J.rowptr, J.col, J.pp, coarse_max=4096)
    a_S = oracle.AMG(J.n, *_dense_csr(S), coarse_max=4096)
    assert a_pp.nlev == 1 and a_S.nlev == 1
    return a_pp, a_S


@pytest.mark.parametrize("variant,maxits", [("lower", 2), ("upper", 2), ("full", 1)])
def test_exact_blocks_iteration_count(variant, maxits):
    """With exact A_pp and exact S, (M P_L^{-1} - I)^2 = 0 for the triangular
    forms, so GMRES stops in two steps; the full factorisation (eq. Ainv) is
    the exact inverse and stops in one."""
    _, J, b = _setup()
    a_pp, a_S = _exact_hierarchies(J)
    x, info = oracle.gmres(J, a_pp, a_S, b, variant=variant, rtol=1e-10)
    assert info["converged"] and info["iters"] <= maxits, info


def test_constant_properties_lower_is_exact():
    """Constant rho, mu: A_pT = 0 and S~ = S, so the lower form with exact
    blocks is the exact inverse: one iteration."""
    pr = synth.Props(c_p=0.0, c_T=0.0, mu_B=0.0)
    _, J, b = _setup(props=pr)
    a_pp, a_S = _exact_hierarchies(J, schur="approx")
    x, info = oracle.gmres(J, a_pp, a_S, b, variant="lower", rtol=1e-10)
    assert info["iters"] == 1


@pytest.mark.parametrize("k", [1, 2, 3, 5])
def test_gmres_minimises_over_krylov_space(k):
    """Identity preconditioner: after k steps the residual equals the least
    squares minimum of ||b - A K_k c|| over the explicit Krylov basis."""
    _, J, b = _setup(dims=(4, 3, 2))
    A = J.dense()
    x, info = oracle.gmres(J, None, None, b, variant="identity", rtol=0.0, maxit=k)
    K = np.column_stack([np.linalg.matrix_power(A, i) @ b for i in range(k)])
    Q, _ = np.linalg.qr(K)
    c, *_ = np.linalg.lstsq(A @ Q, b, rcond=None)
    rmin = np.linalg.norm(b - A @ Q @ c)
    r = np.linalg.norm(b - A @ x)
    assert abs(r - rmin) <= 1e-6 * rmin + 1e-14 * np.linalg.norm(b)


def test_gmres_restart_semantics():
    """GMRES(m) = successive m-step minimisations from the previous iterate."""
    _, J, b = _setup(dims=(4, 3, 2))
    A = J.dense()
    m = 3
    x, info = oracle.gmres(J, None, None, b, variant="identity", rtol=0.0, maxit=2 * m,
                           restart=m)
    xb = np.zeros_like(b)
    for _ in range(2):
        r = b - A @ xb
        K = np.column_stack([np.linalg.matrix_power(A, i) @ r for i in range(m)])
        Q, _ = np.linalg.qr(K)
        c, *_ = np.linalg.lstsq(A @ Q, r, rcond=None)
        xb = xb + Q @ c
    assert abs(np.linalg.norm(b - A @ x) - np.linalg.norm(b - A @ xb)) <= 1e-6 * np.linalg.norm(b - A @ xb)


def test_w1_solve_converges_and_matches_dense():
    p = synth.make_problem("W1")
    J = oracle.jacobian(p)
    b = -oracle.residual(p)
    a_pp = oracle.AMG(J.n, J.rowptr, J.col, J.pp)
    a_S = oracle.AMG(J.n, J.rowptr, J.col, J.S, restriction=1)
    x, info = oracle.gmres(J, a_pp, a_S, b, rtol=1e-10)
    assert info["converged"] and info["rel_true"] <= 1e-10
    # estimated and true residual agree in FP64
    assert abs(info["history"][-1] - info["rel_true"]) <= 1e-3 * info["rel_true"]
    xd = np.linalg.solve(J.dense(), b)
    for blk in (0, 1):
        err = np.linalg.norm(x[blk::2] - xd[blk::2]) / np.linalg.norm(xd[blk::2])
        assert err <= 1e-6, (blk, err)
