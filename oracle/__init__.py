"""CPU FP64 oracle for the coupled pressure-temperature solve.

TEST INFRASTRUCTURE ONLY.  Plain, slow, single-threaded C (built with gcc,
``-O2 -ffp-contract=off``, no fast-math) behind the ctypes wrappers below;
the dense brute-force checks live in the tests.  Only the test-suite, the smoke check and the CPU
baseline leg of the benchmark may import this package; the product library
never does, and it shares no source with the HIP path.

What it computes, and the passage each part follows:
  residual / Jacobian / Schur approximation  Section 2.2, eq. (Fm), (Fe),
      (AXR)-(rhouT), (Se)                    -> physics.c
  AMG setup and V-cycle                      Section 3 (AMG background),
      components named in amg.c             -> amg.c
  block preconditioner and GMRES             Section 3.2 (five-step list),
      Section 4 (right-preconditioned GMRES, restart 30) -> krylov.c
  ILU(0) and the two-stage CPR preconditioner  Section 3 (ILU), Section 3.1,
      Section 4 (ILU(0) as the second stage) -> ilu.c
  3-D convolution smoother network           cnn.c
  Newton time stepping (sparse direct linear steps)  Section 2.2, Section 4 (its opening: Newton settings)
                                             -> newton_simulate
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB = os.path.join(_HERE, "liboracle.so")
_SRC = ["physics.c", "amg.c", "krylov.c", "cnn.c", "ilu.c"]


def build(force: bool = True) -> str:
    """Compile the oracle shared library with gcc (no GPU, no HIP)."""
    srcs = [os.path.join(_HERE, s) for s in _SRC if os.path.exists(os.path.join(_HERE, s))]
    if not force and os.path.exists(_LIB):
        newest = max(os.path.getmtime(s) for s in srcs + [os.path.join(_HERE, "tp_oracle.h")])
        if os.path.getmtime(_LIB) >= newest:
            return _LIB
    tmp = _LIB + f".tmp{os.getpid()}"
    cmd = ["gcc", "-std=gnu99", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fPIC",
           "-shared", "-Wall", "-Wno-unused-function", "-Wno-maybe-uninitialized", "-o", tmp] + srcs + ["-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, _LIB)
    return _LIB


class _Grid(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32),
                ("dx", C.c_double), ("dy", C.c_double), ("dz", C.c_double)]


class _Props(C.Structure):
    _fields_ = [(k, C.c_double) for k in
                ("rho0", "p0", "T0", "c_p", "c_T", "mu0", "mu_B", "cv", "rho_r", "c_r", "g",
                 "api")]


class _Well(C.Structure):
    _fields_ = [("cell", C.c_int32), ("kind", C.c_int32), ("rate", C.c_double),
                ("T_inj", C.c_double), ("p_bh", C.c_double), ("wi", C.c_double)]


class _AmgParams(C.Structure):
    _fields_ = [("theta", C.c_double), ("seed", C.c_uint64), ("max_levels", C.c_int32),
                ("coarse_max", C.c_int32), ("omega", C.c_double), ("nu_pre", C.c_int32),
                ("nu_post", C.c_int32), ("skip_lu", C.c_int32), ("smoother", C.c_int32),
                ("cheb_degree", C.c_int32), ("cheb_lo", C.c_double), ("restriction", C.c_int32),
                ("cheb_degree_coarse", C.c_int32), ("interp", C.c_int32), ("interp_pmax", C.c_int32)]


class _Ilu(C.Structure):
    _fields_ = [("N", C.c_int32), ("rowptr", C.c_void_p), ("col", C.c_void_p), ("lu", C.c_void_p)]


class _Jac(C.Structure):
    _fields_ = [("n", C.c_int32), ("rowptr", C.c_void_p), ("col", C.c_void_p),
                ("pp", C.c_void_p), ("pT", C.c_void_p), ("Tp", C.c_void_p), ("TT", C.c_void_p)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        _lib = C.CDLL(_LIB)
        _lib.or_amg_setup.restype = C.c_int
        _lib.or_amg_nlev.restype = C.c_int32
        _lib.or_stencil_nnz.restype = C.c_int32
        _lib.or_stencil_pattern.restype = C.c_int32
        _lib.or_splitmix64.restype = C.c_uint64
        _lib.or_splitmix64.argtypes = [C.c_uint64]
        _lib.or_gmres.restype = C.c_int
        _lib.or_amg_free.argtypes = [C.c_void_p]
        _lib.or_amg_nlev.argtypes = [C.c_void_p]
        _lib.or_amg_level_R_nnz.restype = C.c_int32
        _lib.or_ilu0.restype = C.c_int
        _lib.or_gmres_cpr.restype = C.c_int
        _lib.or_amg_refresh.restype = C.c_int
    return _lib


def _p(a):
    return a.ctypes.data_as(C.c_void_p) if a is not None else None


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _i32(a):
    return np.ascontiguousarray(a, dtype=np.int32)


def _grid(g):
    return _Grid(g.nx, g.ny, g.nz, g.dx, g.dy, g.dz)


def _props(pr):
    return _Props(*pr.as_tuple())


def _wells(ws):
    arr = (_Well * max(1, len(ws)))()
    for k, w in enumerate(ws):
        arr[k] = _Well(w.cell, w.kind, w.rate, w.T_inj, w.p_bh, w.wi)
    return arr


def splitmix64(x: int) -> int:
    return int(lib().or_splitmix64(C.c_uint64(x & (2 ** 64 - 1))))


def stencil_pattern(grid):
    g = _grid(grid)
    nnz = lib().or_stencil_nnz(C.byref(g))
    rowptr = np.zeros(grid.n + 1, np.int32)
    col = np.zeros(nnz, np.int32)
    lib().or_stencil_pattern(C.byref(g), _p(rowptr), _p(col))
    return rowptr, col


def _perm(K):
    """Pointer and stride of the permeability: a scalar per cell (shape (n,))
    or the diagonal tensor (shape (3, n): K_x, K_y, K_z)."""
    K = _f64(K)
    if K.ndim == 1:
        return _p(K), C.c_int32(0)
    if K.ndim != 2 or K.shape[0] != 3:
        raise ValueError("K must have shape (n,) or (3, n)")
    return _p(K), C.c_int32(K.shape[1])


def residual(prob, x=None):
    x = prob.x_k if x is None else x
    G = np.zeros(2 * prob.grid.n)
    ws = _wells(prob.wells)
    lib().or_residual(C.byref(_grid(prob.grid)), C.byref(_props(prob.props)),
                      *_perm(prob.K), _p(_f64(prob.phi)), _p(_f64(prob.kappa)),
                      C.c_int32(len(prob.wells)), ws, C.c_double(prob.dt),
                      _p(_f64(prob.x_prev)), _p(_f64(x)), _p(G))
    return G


def residual_complex(prob, xc):
    """G on a complex state (for complex-step differentiation)."""
    xc = np.ascontiguousarray(xc, dtype=np.complex128)
    G = np.zeros(2 * prob.grid.n, dtype=np.complex128)
    ws = _wells(prob.wells)
    lib().or_residual_c(C.byref(_grid(prob.grid)), C.byref(_props(prob.props)),
                        *_perm(prob.K), _p(_f64(prob.phi)), _p(_f64(prob.kappa)),
                        C.c_int32(len(prob.wells)), ws, C.c_double(prob.dt),
                        _p(_f64(prob.x_prev)), _p(xc), _p(G))
    return G


class Jacobian:
    """The four blocks of eq. AXR plus the Schur approximation, CSR on the stencil."""

    def __init__(self, n, rowptr, col, pp, pT, Tp, TT, S):
        self.n, self.rowptr, self.col = n, rowptr, col
        self.pp, self.pT, self.Tp, self.TT, self.S = pp, pT, Tp, TT, S

    def block(self, name):
        import scipy.sparse as sp
        return sp.csr_matrix((getattr(self, name), self.col, self.rowptr), shape=(self.n, self.n))

    def dense(self):
        """Full 2n x 2n interleaved Jacobian (dense; tiny grids only)."""
        n = self.n
        A = np.zeros((2 * n, 2 * n))
        for i in range(n):
            for k in range(self.rowptr[i], self.rowptr[i + 1]):
                j = self.col[k]
                A[2 * i, 2 * j] = self.pp[k]
                A[2 * i, 2 * j + 1] = self.pT[k]
                A[2 * i + 1, 2 * j] = self.Tp[k]
                A[2 * i + 1, 2 * j + 1] = self.TT[k]
        return A

    def _cstruct(self):
        self._keep = [_i32(self.rowptr), _i32(self.col), _f64(self.pp), _f64(self.pT),
                      _f64(self.Tp), _f64(self.TT)]
        k = self._keep
        return _Jac(self.n, _p(k[0]), _p(k[1]), _p(k[2]), _p(k[3]), _p(k[4]), _p(k[5]))


def jacobian(prob, x=None):
    x = prob.x_k if x is None else x
    rowptr, col = stencil_pattern(prob.grid)
    nnz = len(col)
    arrs = [np.zeros(nnz) for _ in range(5)]
    ws = _wells(prob.wells)
    lib().or_jacobian(C.byref(_grid(prob.grid)), C.byref(_props(prob.props)),
                      *_perm(prob.K), _p(_f64(prob.phi)), _p(_f64(prob.kappa)),
                      C.c_int32(len(prob.wells)), ws, C.c_double(prob.dt),
                      _p(_f64(prob.x_prev)), _p(_f64(x)), _p(rowptr), _p(col),
                      *[_p(a) for a in arrs])
    return Jacobian(prob.grid.n, rowptr, col, *arrs)


def sparse_interleaved(J):
    """The full 2n x 2n Jacobian of eq. AXR, interleaved [p_i, T_i], as a
    SciPy CSR matrix (from the four stencil blocks)."""
    import scipy.sparse as sp
    n = J.n
    rows = np.repeat(np.arange(n), np.diff(J.rowptr))
    cols = np.asarray(J.col, dtype=np.int64)
    r = np.concatenate([2 * rows, 2 * rows, 2 * rows + 1, 2 * rows + 1])
    c = np.concatenate([2 * cols, 2 * cols + 1, 2 * cols, 2 * cols + 1])
    v = np.concatenate([J.pp, J.pT, J.Tp, J.TT])
    return sp.csr_matrix((v, (r, c)), shape=(2 * n, 2 * n))


def schur_diag(J):
    """The diagonal Schur approximation A_TT - A_Tp diag(A_pp)^{-1} A_pT
    (Section 3.2), by SciPy sparse products: (rowptr, col, val), sorted rows."""
    import scipy.sparse as sp
    Dinv = sp.diags(1.0 / J.block("pp").diagonal())
    S = (J.block("TT") - J.block("Tp") @ (Dinv @ J.block("pT"))).tocsr()
    S.sort_indices()
    return S.indptr.astype(np.int32), S.indices.astype(np.int32), S.data.copy()


def line_search_step(G_at, x, dx, g2, alpha=1e-4, max_backtracks=10):
    """Backtracking line search on f(lam) = |G(x + lam dx)|^2 / 2 along a
    Newton direction (Section 4, the Newton settings: Newton's method with
    line search; the backtracking rule of Dennis and Schnabel, "Numerical
    Methods for Unconstrained Optimization and Nonlinear Equations", 1983,
    Section 6.3).  For the Newton direction the slope of f at lam = 0 is
    -|G(x)|^2 = -g2.  lam = 1 is tried first; a trial is accepted when
    f(lam) <= f(0) - alpha lam g2, else the next lam minimises the quadratic
    through f(0), f'(0) and f(lam), kept within [lam/10, lam/2].  A trial
    whose |G| is not finite (a state outside the fluid laws' range) is
    rejected and halves lam without the quadratic model.  After
    `max_backtracks` rejections the last trial is taken if its |G| is
    finite; if it is not, FloatingPointError is raised.  Returns (lam, the
    accepted point, its G, the number of rejected trials)."""
    f0 = 0.5 * g2
    lam, rejected = 1.0, 0
    while True:
        xt = x + lam * dx
        Gt = G_at(xt)
        f1 = 0.5 * float(Gt @ Gt)
        finite = np.isfinite(f1)
        if finite and (f1 <= f0 - alpha * lam * g2 or rejected == max_backtracks):
            return lam, xt, Gt, rejected
        if rejected == max_backtracks:
            raise FloatingPointError(f"line search: |G| not finite at the last trial step {lam:g}")
        if finite:
            lq = g2 * lam * lam / (2.0 * (f1 - f0 + g2 * lam))
            lam = min(max(lq, 0.1 * lam), 0.5 * lam)
        else:
            lam = 0.5 * lam
        rejected += 1


def newton_simulate(prob, steps, max_newton=4, rtol_f=1e-8, rtol_dx=1e-8, line_search=False):
    """Backward-Euler time stepping from prob.x_prev with Newton's method on
    G(x) = 0 (Section 2.2: each Newton iteration solves eq. AXR for the
    increment; Section 4, the Newton settings: a step has converged when |G| relative to the
    step's first |G|, or |dx| relative to |x|, is below 1e-8).  The linear
    step is a sparse direct solve (SuperLU through SciPy), so the result is
    the exact-Newton reference.  With `line_search` each increment is scaled
    by `line_search_step` (the step-norm test then uses the scaled
    increment).  Returns (states after each step, Newton iterations per step,
    relative |G| histories per step); with `line_search` also the step
    lengths taken, per step."""
    import dataclasses

    import scipy.sparse.linalg as spla
    x = np.array(prob.x_prev, dtype=np.float64)
    states, its, hists, lams = [], [], [], []
    for _ in range(steps):
        p = dataclasses.replace(prob, x_prev=x.copy(), x_k=x.copy())
        g0, done, k_its, hist, lam_s = None, False, 0, [], []
        G = residual(p, x)
        for k in range(max_newton + 1):
            gn = float(np.linalg.norm(G))
            if g0 is None:
                g0 = gn
            hist.append(gn / g0 if g0 > 0 else 0.0)
            if gn <= rtol_f * g0 or done or k == max_newton:
                break
            A = sparse_interleaved(jacobian(p, x))
            dx = spla.spsolve(A.tocsc(), -G)
            if line_search:
                lam, x, G, _ = line_search_step(lambda xt: residual(p, xt), x, dx, gn * gn)
                dx = lam * dx
                lam_s.append(lam)
            else:
                x = x + dx
                G = residual(p, x)
            k_its += 1
            done = float(np.linalg.norm(dx)) <= rtol_dx * float(np.linalg.norm(x))
        states.append(x.copy())
        its.append(k_its)
        hists.append(hist)
        lams.append(lam_s)
    if line_search:
        return states, its, hists, lams
    return states, its, hists


class AMG:
    """Oracle AMG hierarchy (owns a C handle)."""

    def __init__(self, n, rowptr, col, val, theta=0.25, seed=12345, max_levels=25,
                 coarse_max=256, omega=1.0, nu_pre=1, nu_post=1, skip_lu=False,
                 smoother=1, cheb_degree=3, cheb_lo=0.3, restriction=0, cheb_degree_coarse=0, interp=0, interp_pmax=0):
        self._rowptr, self._col, self._val = _i32(rowptr), _i32(col), _f64(val)
        prm = _AmgParams(theta, seed, max_levels, coarse_max, omega, nu_pre, nu_post,
                         1 if skip_lu else 0, smoother, cheb_degree, cheb_lo, restriction,
                         cheb_degree_coarse, interp, interp_pmax)
        h = C.c_void_p()
        self.status = lib().or_amg_setup(C.c_int32(n), _p(self._rowptr), _p(self._col),
                                         _p(self._val), C.byref(prm), C.byref(h))
        self.h = h
        self.n = n

    def __del__(self):
        if getattr(self, "h", None) and _lib is not None:
            _lib.or_amg_free(self.h)
            self.h = None

    @property
    def nlev(self):
        return int(lib().or_amg_nlev(self.h))

    def level(self, l):
        n, nnzA, nnzP = C.c_int32(), C.c_int32(), C.c_int32()
        lib().or_amg_level_sizes(self.h, C.c_int32(l), C.byref(n), C.byref(nnzA), C.byref(nnzP))
        n, nnzA, nnzP = n.value, nnzA.value, nnzP.value
        out = dict(n=n, A_rowptr=np.zeros(n + 1, np.int32), A_col=np.zeros(nnzA, np.int32),
                   A_val=np.zeros(nnzA), dinv=np.zeros(n))
        coarsest = l == self.nlev - 1
        if not coarsest:
            out.update(cf=np.zeros(n, np.int32), P_rowptr=np.zeros(n + 1, np.int32),
                       P_col=np.zeros(nnzP, np.int32), P_val=np.zeros(nnzP))
        lib().or_amg_level_copy(self.h, C.c_int32(l), _p(out["A_rowptr"]), _p(out["A_col"]),
                                _p(out["A_val"]), _p(out.get("cf")), _p(out.get("P_rowptr")),
                                _p(out.get("P_col")), _p(out.get("P_val")), _p(out["dinv"]))
        if not coarsest:
            nr = lib().or_amg_level_R_nnz(self.h, C.c_int32(l))
            nc = self.level_n(l + 1)
            out.update(R_rowptr=np.zeros(nc + 1, np.int32), R_col=np.zeros(nr, np.int32),
                       R_val=np.zeros(nr))
            lib().or_amg_level_R_copy(self.h, C.c_int32(l), _p(out["R_rowptr"]),
                                      _p(out["R_col"]), _p(out["R_val"]))
        return out

    def level_n(self, l):
        n, a, b = C.c_int32(), C.c_int32(), C.c_int32()
        lib().or_amg_level_sizes(self.h, C.c_int32(l), C.byref(n), C.byref(a), C.byref(b))
        return n.value

    def refresh(self, val):
        """New level-0 values on the same pattern: C/F splits, strength
        patterns and every sparsity pattern kept, values recomputed
        (or_amg_refresh).  Returns the status (0, -4 zero pivot)."""
        self._val = _f64(val).copy()
        return int(lib().or_amg_refresh(self.h, _p(self._val)))

    def vcycle(self, b):
        b = _f64(b)
        x = np.zeros_like(b)
        lib().or_vcycle(self.h, _p(b), _p(x))
        return x


def spmv(rowptr, col, val, x):
    x = _f64(x)
    y = np.zeros(len(rowptr) - 1)
    lib().or_spmv(C.c_int32(len(rowptr) - 1), _p(_i32(rowptr)), _p(_i32(col)), _p(_f64(val)),
                  _p(x), _p(y))
    return y


VARIANTS = {"identity": -1, "lower": 0, "upper": 1, "full": 2}


def precond_apply(J: Jacobian, amg_pp, amg_S, r, variant="lower"):
    js = J._cstruct()
    r = _f64(r)
    z = np.zeros_like(r)
    lib().or_precond_apply(C.byref(js), amg_pp.h if amg_pp else None,
                           amg_S.h if amg_S else None, C.c_int32(VARIANTS[variant]),
                           _p(r), _p(z))
    return z


def gmres(J: Jacobian, amg_pp, amg_S, b, x0=None, variant="lower", rtol=1e-8,
          restart=30, maxit=1000):
    js = J._cstruct()
    b = _f64(b)
    x = np.zeros_like(b) if x0 is None else _f64(x0).copy()
    it, rel = C.c_int32(), C.c_double()
    hist = np.zeros(maxit + 1)
    st = lib().or_gmres(C.byref(js), amg_pp.h if amg_pp else None,
                        amg_S.h if amg_S else None, C.c_int32(VARIANTS[variant]),
                        _p(b), _p(x), C.c_double(rtol), C.c_int32(restart),
                        C.c_int32(maxit), C.byref(it), C.byref(rel), _p(hist))
    return x, dict(converged=(st == 0), iters=it.value, rel_true=rel.value,
                   history=hist[: it.value + 1])


# ---- ILU(0) and CPR -----------------------------------------------------------------
def jac_fieldwise(J: Jacobian):
    """(rowptr, col, val) of the 2n x 2n Jacobian in field-by-field order
    [p_0..p_{n-1}, T_0..T_{n-1}] (every stored entry of the blocks kept)."""
    js = J._cstruct()
    n, nnz = J.n, len(J.col)
    rowptr = np.zeros(2 * n + 1, np.int32)
    col = np.zeros(4 * nnz, np.int32)
    val = np.zeros(4 * nnz)
    lib().or_jac_fieldwise(C.byref(js), _p(rowptr), _p(col), _p(val))
    return rowptr, col, val


class ILU0:
    """ILU(0) factors of an N x N CSR matrix with sorted rows: `lu` holds L
    below the diagonal (unit diagonal implied) and U on and above it."""

    def __init__(self, rowptr, col, val):
        self.rowptr, self.col = _i32(rowptr), _i32(col)
        self.N = len(self.rowptr) - 1
        self.lu = np.zeros(len(self.col))
        self.status = lib().or_ilu0(C.c_int32(self.N), _p(self.rowptr), _p(self.col),
                                    _p(_f64(val)), _p(self.lu))

    def solve(self, b):
        b = _f64(b)
        x = np.zeros(self.N)
        lib().or_ilu0_solve(C.c_int32(self.N), _p(self.rowptr), _p(self.col), _p(self.lu), _p(b), _p(x))
        return x

    def factors(self):
        """(L, U) as SciPy CSR matrices (L with its unit diagonal)."""
        import scipy.sparse as sp
        A = sp.csr_matrix((self.lu, self.col, self.rowptr), shape=(self.N, self.N))
        L = sp.tril(A, -1, format="csr") + sp.identity(self.N, format="csr")
        U = sp.triu(A, 0, format="csr")
        return L.tocsr(), U.tocsr()

    def _cstruct(self):
        return _Ilu(self.N, _p(self.rowptr), _p(self.col), _p(self.lu))


def cpr_ilu(J: Jacobian):
    """ILU(0) of the field-by-field Jacobian (the second stage of CPR)."""
    return ILU0(*jac_fieldwise(J))


def cpr_apply(J: Jacobian, amg_pp, F: ILU0, r):
    js, fs = J._cstruct(), F._cstruct()
    r = _f64(r)
    z = np.zeros_like(r)
    lib().or_cpr_apply(C.byref(js), amg_pp.h, C.byref(fs), _p(r), _p(z))
    return z


def gmres_cpr(J: Jacobian, amg_pp, F: ILU0, b, x0=None, rtol=1e-8, restart=30, maxit=1000):
    js, fs = J._cstruct(), F._cstruct()
    b = _f64(b)
    x = np.zeros_like(b) if x0 is None else _f64(x0).copy()
    it, rel = C.c_int32(), C.c_double()
    hist = np.zeros(maxit + 1)
    st = lib().or_gmres_cpr(C.byref(js), amg_pp.h, C.byref(fs), _p(b), _p(x), C.c_double(rtol),
                            C.c_int32(restart), C.c_int32(maxit), C.byref(it), C.byref(rel), _p(hist))
    return x, dict(converged=(st == 0), iters=it.value, rel_true=rel.value,
                   history=hist[: it.value + 1])


# ---- learned post-smoother network -------------------------------------------------
CNN_SIZES = dict(W1=16 * 8 * 27, b1=16, W2=16 * 27, b2=1)
CNN_NPARAM = sum(CNN_SIZES.values())


def cnn_unpack(theta):
    theta = np.asarray(theta, dtype=np.float64)
    o = 0
    out = {}
    for k, m in CNN_SIZES.items():
        out[k] = theta[o:o + m]
        o += m
    return out


def cnn_forward(grid, theta, f):
    """out (n,) and pre-activations h (16, n) for features f (8, n)."""
    p = cnn_unpack(theta)
    n = grid.n
    f = _f64(f).reshape(8, n)
    h = np.zeros((16, n))
    out = np.zeros(n)
    lib().or_cnn_forward(C.byref(_grid(grid)), _p(_f64(p["W1"])), _p(_f64(p["b1"])),
                         _p(_f64(p["W2"])), C.c_double(float(p["b2"][0])), _p(f), _p(h), _p(out))
    return out, h


def cnn_backward(grid, theta, f, y):
    """(loss, gradient with the layout of theta) for target y."""
    p = cnn_unpack(theta)
    n = grid.n
    g = np.zeros(CNN_NPARAM)
    lib().or_cnn_backward.restype = C.c_double
    loss = lib().or_cnn_backward(C.byref(_grid(grid)), _p(_f64(p["W1"])), _p(_f64(p["b1"])),
                                 _p(_f64(p["W2"])), C.c_double(float(p["b2"][0])),
                                 _p(_f64(f).reshape(8, n)), _p(_f64(y)), _p(g))
    return float(loss), g


def cnn_features(grid, rowptr, col, val, r):
    """features (8, n) and the scale s of the learned smoother's input."""
    n = grid.n
    f = np.zeros((8, n))
    lib().or_cnn_features.restype = C.c_double
    s = lib().or_cnn_features(C.byref(_grid(grid)), _p(_i32(rowptr)), _p(_i32(col)), _p(_f64(val)),
                              _p(_f64(r)), _p(f))
    return f, float(s)
