"""Python binding of the tpsolve C ABI (include/tpsolve.h).

Argument marshalling only: every step runs in the HIP library
``libtpsolve.so``.  PyTorch provides device memory (tensors passed by
pointer) and the current HIP stream.  Importing this module does not need a
GPU; loading the library does need the built shared object and fails loudly
when it is missing -- there is no fallback path.
"""
from __future__ import annotations

import ctypes as C
import dataclasses
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libtpsolve.so")

TP_OK, TP_ERR_ARG, TP_ERR_HIP, TP_ERR_OOM, TP_ERR_NUMERIC, TP_ERR_CAPACITY = 0, -1, -2, -3, -4, -5
TP_NOT_CONVERGED = 1


class TpError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"tpsolve status {code}: {msg}")
        self.code = code


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


class _Jac(C.Structure):
    _fields_ = [("n", C.c_int32), ("nnz", C.c_int32), ("rowptr", C.c_void_p), ("col", C.c_void_p),
                ("pp", C.c_void_p), ("pT", C.c_void_p), ("Tp", C.c_void_p), ("TT", C.c_void_p),
                ("S", C.c_void_p)]


class _AmgParams(C.Structure):
    _fields_ = [("theta", C.c_double), ("seed", C.c_uint64), ("max_levels", C.c_int32),
                ("coarse_max", C.c_int32), ("smoother", C.c_int32), ("cheb_degree", C.c_int32),
                ("cheb_lo", C.c_double), ("omega", C.c_double), ("nu_pre", C.c_int32),
                ("nu_post", C.c_int32), ("restriction", C.c_int32), ("storage", C.c_int32),
                ("cheb_degree_coarse", C.c_int32), ("interp", C.c_int32), ("interp_pmax", C.c_int32)]


class _KParams(C.Structure):
    _fields_ = [("rtol", C.c_double), ("restart", C.c_int32), ("maxit", C.c_int32),
                ("stag_ratio", C.c_double), ("graph", C.c_int32), ("atol", C.c_double),
                ("stag_window", C.c_int32), ("ref_rate", C.c_double)]


class _KStats(C.Structure):
    _fields_ = [("iters", C.c_int32), ("restarts", C.c_int32), ("rel_true", C.c_double),
                ("rel_est", C.c_double), ("fallback_iter", C.c_int32)]


_ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_size_t, C.c_void_p, C.c_void_p)
_FREE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_void_p, C.c_void_p)


class _Allocator(C.Structure):
    _fields_ = [("alloc", _ALLOC_FN), ("free", _FREE_FN), ("ctx", C.c_void_p)]


EXPORTS = ["tp_last_error", "tp_init", "tp_jacobian_sizes", "assemble_tpfa", "assemble_tpfa_aniso", "amg_setup", "amg_setup_schur_diag", "amg_refresh_fine", "amg_refresh",
           "amg_num_levels", "amg_level_info", "amg_level_format", "amg_level_copy", "amg_vcycle", "amg_destroy",
           "precond_create", "precond_apply", "precond_apply_noalloc", "precond_destroy", "fgmres_solve",
           "ilu0_create", "ilu0_create_jacobian", "ilu0_refactor_jacobian", "ilu0_solve", "ilu0_info",
           "ilu0_copy", "ilu0_destroy", "precond_create_cpr",
           "cnn_create", "cnn_get_params", "cnn_get_grad", "cnn_destroy", "cnn_forward", "cnn_loss_grad",
           "cnn_adam_step", "amg_attach_post_smoother", "amg_features", "amg_presmoothed_pair",
           "amg_cnn_loss_grad",
           "amg_time_fine_smoother", "amg_time_fine_smoother_flushed", "tp_timer_enable", "tp_timer_read"]
CNN_NPARAM = 3905

_lib = None


def load(path: str = LIB_PATH):
    """Load libtpsolve.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"tpsolve HIP library not built: {path} is missing "
                           "(run __graft_entry__.build())")
    # torch first: its HIP runtime must be the one the process uses, so the
    # library's libamdhip64 dependency resolves to the copy torch loaded
    import torch  # noqa: F401
    lib = C.CDLL(path)
    lib.tp_last_error.restype = C.c_char_p
    for name in EXPORTS[1:]:
        getattr(lib, name).restype = C.c_int
    _lib = lib
    return lib


def _check(code, ok=(TP_OK,)):
    if code not in ok:
        raise TpError(code, _lib.tp_last_error().decode(errors="replace"))
    return code


@dataclasses.dataclass
class AmgParams:
    theta: float = 0.25
    seed: int = 12345
    max_levels: int = 25
    coarse_max: int = 1200
    smoother: int = 1          # 0 l1-Jacobi, 1 Chebyshev
    cheb_degree: int = 10
    cheb_lo: float = 0.03
    omega: float = 1.0
    nu_pre: int = 1
    nu_post: int = 1
    restriction: int = 0       # 0 Galerkin, 1 Petrov-Galerkin (Schur operator)
    storage: int = 0           # 0 FP64, 1 FP32, 2 FP32 with BF16 off-diagonal operator entries
    cheb_degree_coarse: int = 1  # degree on levels >= 1 (0: cheb_degree)
    interp: int = 0            # 0 direct interpolation, 1 extended+i (distance two)
    interp_pmax: int = 4       # extended+i: at most this many weights per row (0: all)

    def oracle_kwargs(self):
        """The same parameters as keyword arguments of the CPU oracle's AMG
        (for tests and the CPU baseline, which must build the same hierarchy)."""
        return dict(theta=self.theta, seed=self.seed, max_levels=self.max_levels,
                    coarse_max=self.coarse_max, omega=self.omega, nu_pre=self.nu_pre,
                    nu_post=self.nu_post, smoother=self.smoother, cheb_degree=self.cheb_degree,
                    cheb_lo=self.cheb_lo, restriction=self.restriction,
                    cheb_degree_coarse=self.cheb_degree_coarse, interp=self.interp,
                    interp_pmax=self.interp_pmax)

    def c(self):
        return _AmgParams(self.theta, self.seed, self.max_levels, self.coarse_max, self.smoother,
                          self.cheb_degree, self.cheb_lo, self.omega, self.nu_pre, self.nu_post,
                          self.restriction, self.storage, self.cheb_degree_coarse, self.interp,
                          self.interp_pmax)


def _torch():
    import torch
    return torch


def _stream(stream=None):
    torch = _torch()
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


def _ptr(t):
    return C.c_void_p(t.data_ptr()) if t is not None else None


_keep_alloc = None


def init(device: int = 0, torch_allocator: bool = False):
    """Select the device; optionally route library allocations through
    torch's caching allocator (default: the HIP stream-ordered pool)."""
    global _keep_alloc
    lib = load()
    import torch
    torch.cuda.init()
    if torch_allocator:
        torch = _torch()

        def _a(nbytes, stream, ctx):
            return torch.cuda.caching_allocator_alloc(int(nbytes), device,
                                                      torch.cuda.current_stream(device))

        def _f(ptr, stream, ctx):
            torch.cuda.caching_allocator_delete(ptr)

        al = _Allocator(_ALLOC_FN(_a), _FREE_FN(_f), None)
        _keep_alloc = al
        _check(lib.tp_init(C.byref(al), C.c_int(device)))
    else:
        _keep_alloc = None
        _check(lib.tp_init(None, C.c_int(device)))


def grid_c(g):
    return _Grid(g.nx, g.ny, g.nz, g.dx, g.dy, g.dz)


def jacobian_sizes(grid):
    lib = load()
    n, nnz = C.c_int32(), C.c_int32()
    _check(lib.tp_jacobian_sizes(C.byref(grid_c(grid)), C.byref(n), C.byref(nnz)))
    return n.value, nnz.value


class Jacobian:
    """Device Jacobian: shared CSR pattern + pp, pT, Tp, TT, S value tensors."""

    def __init__(self, n, nnz, device="cuda"):
        torch = _torch()
        self.n, self.nnz = n, nnz
        self.rowptr = torch.zeros(n + 1, dtype=torch.int32, device=device)
        self.col = torch.zeros(nnz, dtype=torch.int32, device=device)
        for k in ("pp", "pT", "Tp", "TT", "S"):
            setattr(self, k, torch.zeros(nnz, dtype=torch.float64, device=device))

    @classmethod
    def from_host(cls, n, rowptr, col, pp, pT, Tp, TT, S, device="cuda"):
        torch = _torch()
        J = cls.__new__(cls)
        J.n, J.nnz = n, len(col)
        J.rowptr = torch.as_tensor(np.asarray(rowptr, np.int32), device=device)
        J.col = torch.as_tensor(np.asarray(col, np.int32), device=device)
        for k, v in zip(("pp", "pT", "Tp", "TT", "S"), (pp, pT, Tp, TT, S)):
            setattr(J, k, torch.as_tensor(np.asarray(v, np.float64), device=device))
        return J

    def c(self):
        return _Jac(self.n, self.nnz, self.rowptr.data_ptr(), self.col.data_ptr(),
                    self.pp.data_ptr(), self.pT.data_ptr(), self.Tp.data_ptr(),
                    self.TT.data_ptr(), self.S.data_ptr())


def assemble_tpfa(grid, props, K, phi, kappa, wells, dt, x_prev, x_k, J=None, G=None,
                  stream=None):
    """Assemble G(x_k) and the Jacobian on the device (tensors in, tensors out).
    K is a scalar permeability per cell (n,) or the diagonal tensor (3, n)."""
    torch = _torch()
    lib = load()
    n, nnz = jacobian_sizes(grid)
    if K.dim() == 2:
        if tuple(K.shape) != (3, n) or not K.is_contiguous():
            raise ValueError("anisotropic K must be a contiguous (3, n) tensor")
        entry = lib.assemble_tpfa_aniso
    elif K.dim() == 1 and K.numel() == n:
        entry = lib.assemble_tpfa
    else:
        raise ValueError("K must have shape (n,) or (3, n)")
    if J is None:
        J = Jacobian(n, nnz, device=x_k.device)
    if G is None:
        G = torch.empty(2 * n, dtype=torch.float64, device=x_k.device)
    ws = (_Well * max(1, len(wells)))()
    for i, w in enumerate(wells):
        ws[i] = _Well(w.cell, w.kind, w.rate, w.T_inj, w.p_bh, w.wi)
    pr = _Props(*props.as_tuple())
    jc = J.c()
    _check(entry(C.byref(grid_c(grid)), C.byref(pr), _ptr(K), _ptr(phi), _ptr(kappa),
                             C.c_int32(len(wells)), ws, C.c_double(dt), _ptr(x_prev), _ptr(x_k),
                             C.byref(jc), _ptr(G), _stream(stream)))
    return J, G


class AMG:
    """Device AMG hierarchy of an n x n CSR matrix (tensors)."""

    def __init__(self, rowptr, col, val, params: AmgParams | None = None, stream=None):
        lib = load()
        self.params = params or AmgParams()
        self.n = int(rowptr.numel() - 1)
        self._keep = (rowptr, col, val)
        h = C.c_void_p()
        pc = self.params.c()
        _check(lib.amg_setup(C.c_int32(self.n), _ptr(rowptr), _ptr(col), _ptr(val), C.byref(pc),
                             C.byref(h), _stream(stream)))
        self.h = h

    @classmethod
    def schur_diag(cls, J: "Jacobian", params: AmgParams | None = None, stream=None):
        """Hierarchy of S_diag = A_TT - A_Tp diag(A_pp)^{-1} A_pT (formed on the device)."""
        lib = load()
        self = cls.__new__(cls)
        self.params = params or AmgParams()
        self.n = J.n
        self._keep = (J.rowptr, J.col, J)    # (device of the first: level copies)
        h = C.c_void_p()
        pc = self.params.c()
        jc = J.c()
        _check(lib.amg_setup_schur_diag(C.byref(jc), C.byref(pc), C.byref(h), _stream(stream)))
        self.h = h
        return self

    def refresh_fine(self, val, stream=None):
        """New finest-level values on the same pattern; coarse levels kept."""
        self._keep = self._keep[:2] + (val,)
        _check(_lib.amg_refresh_fine(self.h, _ptr(val), _stream(stream)))

    def refresh(self, val, stream=None):
        """New finest-level values on the same pattern; C/F splits and every
        pattern kept, all values recomputed (numeric-only setup)."""
        self._keep = self._keep[:2] + (val,)
        _check(_lib.amg_refresh(self.h, _ptr(val), _stream(stream)))

    def close(self):
        if getattr(self, "h", None) and self.h.value:
            _check(_lib.amg_destroy(self.h))
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def nlev(self):
        v = C.c_int32()
        _check(_lib.amg_num_levels(self.h, C.byref(v)))
        return v.value

    def level_sizes(self, l):
        n, a, p, r = C.c_int32(), C.c_int32(), C.c_int32(), C.c_int32()
        _check(_lib.amg_level_info(self.h, C.c_int32(l), C.byref(n), C.byref(a), C.byref(p),
                                   C.byref(r)))
        return n.value, a.value, p.value, r.value

    def time_fine_smoother(self, reps=200, stream=None, flush=None):
        """(ms per launch, algorithmic bytes per launch) of the finest-level
        sweep replayed back to back; with `flush` (a float64 device tensor),
        each launch follows a pass over it that evicts the last-level cache
        and is timed alone."""
        ms, b = C.c_double(), C.c_double()
        if flush is None:
            _check(_lib.amg_time_fine_smoother(self.h, C.c_int32(reps), C.byref(ms), C.byref(b),
                                               _stream(stream)))
        else:
            _check(_lib.amg_time_fine_smoother_flushed(self.h, C.c_int32(reps), _ptr(flush),
                                                       C.c_int64(flush.numel()), C.byref(ms), C.byref(b),
                                                       _stream(stream)))
        return ms.value, b.value

    def level_format(self, l):
        nd, g = C.c_int32(), C.c_int32()
        _check(_lib.amg_level_format(self.h, C.c_int32(l), C.byref(nd), C.byref(g)))
        return nd.value, g.value

    def vcycle_bytes(self):
        """Algorithmic bytes of one V-cycle (each array read or written once
        per pass): Chebyshev(3) pre/post sweeps with the zero-guess steps
        fused, residual, restriction, prolongation, coarse dense inverse.
        Storage 2 reads level-operator values as BF16 (2 bytes) plus the FP32
        diagonal (4 bytes a row)."""
        st = self.params.storage
        es = 8 if st == 0 else 4
        vs = 2 if st == 2 else es          # level-operator value bytes
        dgb = 4 if st == 2 else 0          # separate diagonal, bytes per row
        d0, dc = self.params.cheb_degree, self.params.cheb_degree_coarse
        total = 0.0
        L = self.nlev
        for l in range(L):
            n, nnzA, nnzP, nnzR = self.level_sizes(l)
            if l == L - 1:
                total += n * n * 8 + 2 * n * es
                continue
            deg = dc if (l > 0 and dc > 0) else d0
            nc = self.level_sizes(l + 1)[0]
            nd, _ = self.level_format(l)
            mA = (nd * n * vs if nd else nnzA * (vs + 4) + (n + 1) * 4) + dgb * n
            mP = nnzP * (es + 4) + (n + 1) * 4
            mR = nnzR * (es + 4) + (nc + 1) * 4
            if deg >= 2:   # steps 0 and 1 fused, then deg - 2 steps
                pre = (mA + 4 * n * es) + (deg - 2) * (mA + 6 * n * es)
            else:          # the zero-guess step alone reads no matrix
                pre = 4 * n * es
            post = (mA + 5 * n * es) + (deg - 1) * (mA + 6 * n * es)
            total += pre + (mA + 3 * n * es) + (mR + (n + nc) * es) + (mP + (2 * n + nc) * es) + post
        return total

    def level(self, l, stream=None):
        torch = _torch()
        n, nnzA, nnzP, nnzR = self.level_sizes(l)
        dev = self._keep[0].device
        i32 = dict(dtype=torch.int32, device=dev)
        f64 = dict(dtype=torch.float64, device=dev)
        out = dict(n=n, A_rowptr=torch.zeros(n + 1, **i32), A_col=torch.zeros(nnzA, **i32),
                   A_val=torch.zeros(nnzA, **f64))
        coarse = l == self.nlev - 1
        if not coarse:
            nc = self.level_sizes(l + 1)[0]
            out.update(cf=torch.zeros(n, **i32), P_rowptr=torch.zeros(n + 1, **i32),
                       P_col=torch.zeros(nnzP, **i32), P_val=torch.zeros(nnzP, **f64),
                       R_rowptr=torch.zeros(nc + 1, **i32), R_col=torch.zeros(nnzR, **i32),
                       R_val=torch.zeros(nnzR, **f64))
        g = out.get
        _check(_lib.amg_level_copy(self.h, C.c_int32(l), _ptr(g("A_rowptr")), _ptr(g("A_col")),
                                   _ptr(g("A_val")), _ptr(g("cf")), _ptr(g("P_rowptr")),
                                   _ptr(g("P_col")), _ptr(g("P_val")), _ptr(g("R_rowptr")),
                                   _ptr(g("R_col")), _ptr(g("R_val")), _stream(stream)))
        torch.cuda.current_stream().synchronize()
        return out

    def attach(self, net, grid):
        """Use `net` (Net or None) as the finest-level post-smoother."""
        self._net = net
        _check(_lib.amg_attach_post_smoother(self.h, net.h if net is not None else None,
                                             C.byref(grid_c(grid)) if grid is not None else None))

    def features(self, r, feat=None, stream=None):
        torch = _torch()
        if feat is None:
            feat = torch.empty(8 * self.n, dtype=torch.float32, device=r.device)
        s = C.c_float()
        _check(_lib.amg_features(self.h, _ptr(r), _ptr(feat), C.byref(s), _stream(stream)))
        return feat, s.value

    def op_loss_grad(self, feat, target, err_weight=0.0, stream=None):
        """Loss of the attached network in the D^{-1} A norm, plus err_weight
        times the mean squared error (gradient kept for Adam)."""
        loss = C.c_double()
        _check(_lib.amg_cnn_loss_grad(self.h, _ptr(feat), _ptr(target), C.c_float(err_weight), C.byref(loss),
                                      _stream(stream)))
        return loss.value

    def presmoothed_pair(self, y, stream=None):
        torch = _torch()
        r = torch.empty_like(y)
        e = torch.empty_like(y)
        _check(_lib.amg_presmoothed_pair(self.h, _ptr(y), _ptr(r), _ptr(e), _stream(stream)))
        return r, e

    def vcycle(self, b, x=None, stream=None):
        torch = _torch()
        if x is None:
            x = torch.empty_like(b)
        _check(_lib.amg_vcycle(self.h, _ptr(b), _ptr(x), _stream(stream)))
        return x


VARIANTS = {"lower": 0, "upper": 1, "full": 2}


class ILU0:
    """Device ILU(0) factors: of a CSR matrix (tensors), or with
    ``ILU0.jacobian(J)`` of the whole Jacobian in field-by-field order."""

    def __init__(self, rowptr, col, val, stream=None):
        lib = load()
        h = C.c_void_p()
        self._keep = (rowptr,)
        _check(lib.ilu0_create(C.c_int32(int(rowptr.numel() - 1)), _ptr(rowptr), _ptr(col), _ptr(val),
                               _stream(stream), C.byref(h)))
        self.h = h

    @classmethod
    def jacobian(cls, J: "Jacobian", stream=None):
        lib = load()
        self = cls.__new__(cls)
        self._keep = (J.rowptr,)
        h = C.c_void_p()
        jc = J.c()
        _check(lib.ilu0_create_jacobian(C.byref(jc), _stream(stream), C.byref(h)))
        self.h = h
        return self

    def refactor(self, J: "Jacobian", stream=None):
        jc = J.c()
        _check(_lib.ilu0_refactor_jacobian(self.h, C.byref(jc), _stream(stream)))

    def info(self):
        N, nnz, ll, lu = C.c_int32(), C.c_int32(), C.c_int32(), C.c_int32()
        _check(_lib.ilu0_info(self.h, C.byref(N), C.byref(nnz), C.byref(ll), C.byref(lu)))
        return dict(N=N.value, nnz=nnz.value, levels_lower=ll.value, levels_upper=lu.value)

    def factors(self, stream=None):
        """(rowptr, col, lu) device tensors: L strictly below the diagonal, U on and above."""
        torch = _torch()
        inf = self.info()
        dev = self._keep[0].device
        rp = torch.empty(inf["N"] + 1, dtype=torch.int32, device=dev)
        ci = torch.empty(inf["nnz"], dtype=torch.int32, device=dev)
        lu = torch.empty(inf["nnz"], dtype=torch.float64, device=dev)
        _check(_lib.ilu0_copy(self.h, _ptr(rp), _ptr(ci), _ptr(lu), _stream(stream)))
        return rp, ci, lu

    def solve(self, b, x=None, stream=None):
        torch = _torch()
        if x is None:
            x = torch.empty_like(b)
        _check(_lib.ilu0_solve(self.h, _ptr(b), _ptr(x), _stream(stream)))
        return x

    def close(self):
        if getattr(self, "h", None) and self.h.value:
            _check(_lib.ilu0_destroy(self.h))
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Precond:
    def __init__(self, J: Jacobian, amg_pp: AMG, amg_S: AMG, variant="lower"):
        lib = load()
        self._keep = (J, amg_pp, amg_S)
        self._jc = J.c()
        h = C.c_void_p()
        _check(lib.precond_create(C.byref(self._jc), amg_pp.h, amg_S.h,
                                  C.c_int32(VARIANTS[variant]), C.byref(h)))
        self.h = h

    @classmethod
    def cpr(cls, J: Jacobian, amg_pp: AMG, ilu: ILU0):
        """CPR two-stage preconditioner: AMG V-cycle on A_pp, then ILU(0) of J."""
        lib = load()
        self = cls.__new__(cls)
        self._keep = (J, amg_pp, ilu)
        self._jc = J.c()
        h = C.c_void_p()
        _check(lib.precond_create_cpr(C.byref(self._jc), amg_pp.h, ilu.h, C.byref(h)))
        self.h = h
        return self

    def apply(self, r, z=None, stream=None):
        torch = _torch()
        if z is None:
            z = torch.empty_like(r)
        _check(_lib.precond_apply(self.h, _ptr(r), _ptr(z), _stream(stream)))
        return z

    def apply_noalloc(self, r, z, stream=None):
        """The same apply with no device allocation by the library (fixed
        device scratch; see precond_apply_noalloc)."""
        _check(_lib.precond_apply_noalloc(self.h, _ptr(r), _ptr(z), _stream(stream)))
        return z

    def close(self):
        if getattr(self, "h", None) and self.h.value:
            _check(_lib.precond_destroy(self.h))
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Net:
    """Learned post-smoother network (device parameters, FP32 master + BF16 copy)."""

    def __init__(self, params):
        lib = load()
        p = np.ascontiguousarray(params, dtype=np.float32)
        assert p.size == CNN_NPARAM
        h = C.c_void_p()
        _check(lib.cnn_create(p.ctypes.data_as(C.c_void_p), C.byref(h)))
        self.h = h

    def params(self):
        p = np.zeros(CNN_NPARAM, dtype=np.float32)
        _check(_lib.cnn_get_params(self.h, p.ctypes.data_as(C.c_void_p)))
        return p

    def grad(self):
        g = np.zeros(CNN_NPARAM, dtype=np.float32)
        _check(_lib.cnn_get_grad(self.h, g.ctypes.data_as(C.c_void_p)))
        return g

    def forward(self, grid, feat, out=None, stream=None):
        torch = _torch()
        if out is None:
            out = torch.empty(grid.n, dtype=torch.float32, device=feat.device)
        _check(_lib.cnn_forward(self.h, C.byref(grid_c(grid)), _ptr(feat), _ptr(out), _stream(stream)))
        return out

    def loss_grad(self, grid, feat, target, grad=None, stream=None):
        loss = C.c_double()
        _check(_lib.cnn_loss_grad(self.h, C.byref(grid_c(grid)), _ptr(feat), _ptr(target),
                                  C.byref(loss), _ptr(grad), _stream(stream)))
        return loss.value

    def adam_step(self, lr, stream=None):
        _check(_lib.cnn_adam_step(self.h, C.c_float(lr), _stream(stream)))

    def close(self):
        if getattr(self, "h", None) and self.h.value:
            _check(_lib.cnn_destroy(self.h))
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# Below this many cells the preconditioner apply is launch-bound and its
# replay from a captured graph pays for the capture within a solve; above,
# its kernels are long enough that launching them one by one costs nothing,
# and a handle's first capture does not pay back (measured on 256x256x64: a
# solve on a fresh handle, 8 iterations, 24.1 ms with the graph against
# 23.6 ms without).
GRAPH_MAX_CELLS = 1 << 20


def fgmres_solve(J: Jacobian, M: Precond, b, x=None, rtol=1e-8, restart=30, maxit=1000,
                 history=False, stag_ratio=0.95, graph=None, stream=None, atol=0.0, stag_window=2,
                 ref_rate=0.0):
    """Solve J x = b; returns (x, stats dict).  x (tensor) is the initial
    guess when given and is overwritten.  graph: replay the preconditioner
    apply from a captured HIP graph (None: when J has fewer than
    GRAPH_MAX_CELLS cells).  stag_ratio / stag_window / ref_rate: the learned
    smoother's guards (see tp_krylov_params)."""
    torch = _torch()
    lib = load()
    if graph is None:
        graph = J.n < GRAPH_MAX_CELLS
    if x is None:
        x = torch.zeros_like(b)
    kp = _KParams(rtol, restart, maxit, stag_ratio, 1 if graph else 0, atol, stag_window, ref_rate)
    st = _KStats()
    hist = np.zeros(maxit + 1) if history else None
    jc = J.c()
    code = lib.fgmres_solve(C.byref(jc), M.h, _ptr(b), _ptr(x), C.byref(kp), C.byref(st),
                            hist.ctypes.data_as(C.c_void_p) if hist is not None else None,
                            _stream(stream))
    _check(code, ok=(TP_OK, TP_NOT_CONVERGED))
    out = dict(converged=code == TP_OK, iters=st.iters, restarts=st.restarts,
               rel_true=st.rel_true, rel_est=st.rel_est, fallback_iter=st.fallback_iter)
    if hist is not None:
        out["history"] = hist[: st.iters + 1]
    return x, out


def timer_enable(on=True):
    _check(load().tp_timer_enable(C.c_int32(1 if on else 0)))


def timer_read():
    lib = load()
    n, ms, b = C.c_int64(), C.c_double(), C.c_double()
    _check(lib.tp_timer_read(C.byref(n), C.byref(ms), C.byref(b)))
    return n.value, ms.value, b.value
