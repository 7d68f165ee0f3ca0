"""Pins of the oracle's ILU(0) and of the two-stage CPR preconditioner.

ILU(0) (Section 3; Saad 2003, Section 10.3) is fixed by a hand-worked
example, by the special case of a pattern closed under elimination (where it
is the exact LU factorisation), and by its defining property: L U equals A
at every position of A's pattern.  The two-stage preconditioner (Section 3.1)
is pinned against its closed form M^{-1} = M2^{-1}(I - A M1^{-1}) + M1^{-1}
assembled from dense matrices, and by the case of an exact second stage."""
from fractions import Fraction

import numpy as np
import pytest
import scipy.linalg as sla
import scipy.sparse as sp

import oracle
from paper_1902_00095_amd import synth


def _csr(M):
    A = sp.csr_matrix(M)
    A.sort_indices()
    return A.indptr.astype(np.int32), A.indices.astype(np.int32), A.data.copy()


def _problem(dims, seed=3):
    return synth.make_problem("W2", seed=seed, grid=synth.Grid(*dims, 1.0, 1.0, 1.0))


def test_ilu0_hand_worked_laplacian():
    A = np.array([[4, -1, -1, 0], [-1, 4, 0, -1], [-1, 0, 4, -1], [0, -1, -1, 4]], float)
    F = oracle.ILU0(*_csr(A))
    assert F.status == 0
    got = {}
    for i in range(4):
        for q in range(F.rowptr[i], F.rowptr[i + 1]):
            got[(i, int(F.col[q]))] = F.lu[q]
    want = {}
    for line in open("tests/golden/ilu0_laplace_2x2.txt"):
        if line.startswith("#") or not line.strip():
            continue
        i, j, v = line.split()
        want[(int(i), int(j))] = float(Fraction(v))
    assert set(got) == set(want)
    for k, v in want.items():
        assert got[k] == pytest.approx(v, rel=1e-15, abs=0.0), k
    # the dropped fill-in makes it differ from the exact factorisation
    L, U = F.factors()
    assert not np.allclose((L @ U).toarray(), A)


def test_ilu0_is_exact_lu_on_a_closed_pattern():
    """A 1-D grid in the cell-interleaved ordering is block tridiagonal with
    full 2 x 2 blocks; elimination creates no entry outside that pattern, so
    ILU(0) is the exact factorisation and its solve inverts A."""
    p = _problem((24, 1, 1))
    A = oracle.sparse_interleaved(oracle.jacobian(p))
    A.sort_indices()
    F = oracle.ILU0(A.indptr, A.indices, A.data)
    assert F.status == 0
    L, U = F.factors()
    Ad = A.toarray()
    scale = np.abs(Ad).max(axis=1, keepdims=True)
    assert np.abs(((L @ U).toarray() - Ad) / scale).max() < 1e-13
    b = synth.random_rhs(5, A.shape[0])
    x = F.solve(b)
    xr = np.linalg.solve(Ad, b)
    assert np.linalg.norm(x - xr) <= 1e-9 * np.linalg.norm(xr)


def test_ilu0_matches_lapack_lu_on_a_dense_pattern():
    """With a full pattern nothing is dropped: the factors are those of LU
    without pivoting (LAPACK's partial pivoting never swaps rows of a
    column diagonally dominant matrix)."""
    rng = np.random.default_rng(7)
    n = 9
    A = rng.standard_normal((n, n))
    A += np.diag(np.abs(A).sum(axis=0) + 1.0)
    P, Lr, Ur = sla.lu(A)
    assert np.array_equal(P, np.eye(n))
    F = oracle.ILU0(*_csr(A))
    L, U = F.factors()
    assert np.allclose(L.toarray(), Lr, rtol=0, atol=1e-14)
    assert np.allclose(U.toarray(), Ur, rtol=1e-14, atol=1e-13)


@pytest.mark.parametrize("dims", [(6, 5, 1), (5, 4, 3)])
def test_ilu0_product_equals_A_on_its_pattern(dims):
    """The defining property: (L U)_ij = a_ij wherever A stores an entry, L
    unit lower and U upper triangular on A's pattern; off the pattern L U
    keeps the dropped fill (nonzero somewhere)."""
    J = oracle.jacobian(_problem(dims))
    rp, ci, v = oracle.jac_fieldwise(J)
    F = oracle.ILU0(rp, ci, v)
    assert F.status == 0
    N = 2 * J.n
    A = sp.csr_matrix((v, ci, rp), shape=(N, N)).toarray()
    L, U = F.factors()
    P = (L @ U).toarray()
    mask = sp.csr_matrix((np.ones_like(v), ci, rp), shape=(N, N)).toarray() > 0
    scale = np.abs(A).max(axis=1, keepdims=True)
    assert np.abs((P - A) / scale)[mask].max() < 1e-13
    assert np.abs(P[~mask]).max() > 1e-6 * np.abs(A).max()
    assert np.all(np.diag(L.toarray()) == 1.0)
    b = synth.random_rhs(9, N)
    x = F.solve(b)
    # backward error of the two triangular solves (the rows span ~9 decades)
    assert np.all(np.abs(P @ x - b) <= 1e-12 * (np.abs(P) @ np.abs(x) + np.abs(b)))


def test_fieldwise_is_a_symmetric_permutation_of_the_interleaved_jacobian():
    J = oracle.jacobian(_problem((4, 3, 2)))
    n = J.n
    rp, ci, v = oracle.jac_fieldwise(J)
    Af = sp.csr_matrix((v, ci, rp), shape=(2 * n, 2 * n)).toarray()
    Ai = oracle.sparse_interleaved(J).toarray()
    perm = np.concatenate([2 * np.arange(n), 2 * np.arange(n) + 1])  # field row -> interleaved row
    assert np.array_equal(Af, Ai[np.ix_(perm, perm)])
    assert len(ci) == 4 * len(J.col) and np.all(np.diff(ci[rp[0]:rp[1]]) > 0)


def _dense_operator(apply, m):
    return np.column_stack([apply(e) for e in np.eye(m)])


@pytest.mark.parametrize("coarse_max", [4096, 8])
def test_cpr_apply_is_the_two_stage_formula(coarse_max):
    """x = M2^{-1}(r - A M1^{-1} r) + M1^{-1} r with M1^{-1} = [V_pp 0; 0 0]
    (V_pp the V-cycle as a matrix: exact A_pp^{-1} on one level, a multilevel
    cycle otherwise) and M2^{-1} = (L U)^{-1} in field order."""
    p = _problem((4, 3, 2))
    J = oracle.jacobian(p)
    n = J.n
    a_pp = oracle.AMG(n, J.rowptr, J.col, J.pp, coarse_max=coarse_max)
    F = oracle.cpr_ilu(J)
    Vpp = _dense_operator(a_pp.vcycle, n)
    if coarse_max > n:
        App = J.block("pp").toarray()
        res = np.abs(App @ Vpp - np.eye(n))
        assert np.all(res <= 1e-10 * (np.abs(App) @ np.abs(Vpp)))
    else:
        assert a_pp.nlev > 1
    A = oracle.sparse_interleaved(J).toarray()
    perm = np.concatenate([2 * np.arange(n), 2 * np.arange(n) + 1])
    M1 = np.zeros((2 * n, 2 * n))
    M1[np.ix_(2 * np.arange(n), 2 * np.arange(n))] = Vpp
    L, U = F.factors()
    M2f = np.linalg.inv((L @ U).toarray())
    M2 = np.zeros_like(M2f)
    M2[np.ix_(perm, perm)] = M2f
    Minv = M2 @ (np.eye(2 * n) - A @ M1) + M1
    for seed in (1, 2):
        r = synth.random_rhs(seed, 2 * n)
        z = oracle.cpr_apply(J, a_pp, F, r)
        want = Minv @ r
        assert np.linalg.norm(z - want) <= 1e-10 * np.linalg.norm(want)


def test_cpr_with_an_exact_second_stage_is_the_inverse():
    """On two cells the field-ordered Jacobian is a dense 4 x 4 matrix, so
    ILU(0) is exact; then M^{-1} = A^{-1} whatever the first stage is, and
    GMRES stops after one iteration.  The physical two-cell Jacobian has a
    condition number near 1e15, so the blocks here are random and well
    conditioned instead (the oracle's routines take any values)."""
    rng = np.random.default_rng(11)
    rowptr = np.array([0, 2, 4], np.int32)
    col = np.array([0, 1, 0, 1], np.int32)
    blocks = [rng.uniform(-1, 1, 4) for _ in range(4)]
    for b in (blocks[0], blocks[3]):
        b[[0, 3]] += 4.0  # diagonally dominant pressure and temperature blocks
    J = oracle.Jacobian(2, rowptr, col, *blocks, np.zeros(4))
    a_pp = oracle.AMG(J.n, J.rowptr, J.col, J.pp)
    F = oracle.cpr_ilu(J)
    A = oracle.sparse_interleaved(J).toarray()
    assert np.linalg.cond(A) < 1e3
    r = synth.random_rhs(3, 4)
    z = oracle.cpr_apply(J, a_pp, F, r)
    xr = np.linalg.solve(A, r)
    assert np.linalg.norm(z - xr) <= 1e-13 * np.linalg.norm(xr)
    x, st = oracle.gmres_cpr(J, a_pp, F, r, rtol=1e-12)
    assert st["converged"] and st["iters"] == 1


def test_gmres_cpr_converges_on_a_heterogeneous_grid():
    p = _problem((12, 10, 6))
    J = oracle.jacobian(p)
    b = -oracle.residual(p)
    a_pp = oracle.AMG(J.n, J.rowptr, J.col, J.pp, coarse_max=64)
    F = oracle.cpr_ilu(J)
    x, st = oracle.gmres_cpr(J, a_pp, F, b, rtol=1e-8)
    assert st["converged"] and st["rel_true"] <= 1e-8
    A = oracle.sparse_interleaved(J)
    assert np.linalg.norm(b - A @ x) <= 1.01e-8 * np.linalg.norm(b)
