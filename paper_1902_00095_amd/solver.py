"""One coupled pressure-temperature solve on the GPU, end to end.

assemble_tpfa -> amg_setup(A_pp) and amg_setup(S) -> precond_create ->
fgmres_solve, all through the C ABI (the CPR comparator: amg_setup(A_pp) and
ilu0_create_jacobian -> precond_create_cpr).  The Schur-approximation hierarchy uses
the Petrov-Galerkin restriction (its columns, not its rows, are diagonally
dominant); the pressure hierarchy the Galerkin one.
"""
from __future__ import annotations

import dataclasses
import math

from . import tpsolve as tps


@dataclasses.dataclass
class SolveConfig:
    rtol: float = 1e-8
    restart: int = 30
    maxit: int = 1000
    variant: str = "lower"
    storage: int = 0              # 0 FP64 hierarchy, 1 FP32, 2 FP32 with BF16 off-diagonals
    amg: tps.AmgParams = dataclasses.field(default_factory=tps.AmgParams)
    # Schur approximation the second hierarchy is built on: "T" the paper's
    # S~_T (eq. Se), "ATT" the energy block A_TT alone, "diag"
    # A_TT - A_Tp diag(A_pp)^{-1} A_pT (the simple forms it is compared with)
    schur: str = "T"
    # "block": the block-triangular preconditioner (Section 3.2); "cpr": the
    # two-stage CPR comparator (Section 3.1: AMG on A_pp, then ILU(0) of J)
    method: str = "block"
    # interpolation of the pressure hierarchy alone (None: amg.interp).  1,
    # the default, puts extended+i on A_pp: after PMIS coarsening (which,
    # unlike the Ruge-Stueben coarsening the paper's AMG used, does not give
    # every strong F-F pair a common C point) it restores the quality of
    # classical interpolation -- the V-cycle's stationary factor drops from
    # ~0.45 to ~0.12, and on the 256x256x64 Newton systems FGMRES needs 8
    # iterations instead of 46 for a 2x more expensive pressure setup.  The
    # Schur hierarchy keeps direct interpolation (extended+i built from
    # S~^T diverges on it).  0 gives direct interpolation on both.
    interp_pp: int | None = 1


def to_device(prob, device="cuda"):
    import torch
    t = lambda a: torch.as_tensor(a, dtype=torch.float64, device=device)
    return dict(K=t(prob.K), phi=t(prob.phi), kappa=t(prob.kappa), x_prev=t(prob.x_prev),
                x_k=t(prob.x_k))


def assemble(prob, dev, J=None, G=None):
    """G(x_k) and the Jacobian; into the buffers of J and G when given."""
    return tps.assemble_tpfa(prob.grid, prob.props, dev["K"], dev["phi"], dev["kappa"],
                             prob.wells, prob.dt, dev["x_prev"], dev["x_k"], J=J, G=G)


_side = {}


def _side_streams():
    import torch
    dev = torch.cuda.current_device()
    if dev not in _side:
        _side[dev] = (torch.cuda.Stream(), torch.cuda.Stream())   # default priority
    return _side[dev]


def _schur_amg(J, cfg, prm, stream=None):
    if cfg.schur == "T":
        return tps.AMG(J.rowptr, J.col, J.S, prm, stream=stream)
    if cfg.schur == "ATT":
        return tps.AMG(J.rowptr, J.col, J.TT, prm, stream=stream)
    if cfg.schur == "diag":
        return tps.AMG.schur_diag(J, prm, stream=stream)
    raise ValueError(f"unknown Schur approximation {cfg.schur!r}")


def amg_params(cfg: SolveConfig, which: str) -> tps.AmgParams:
    """The AMG parameters `setup` gives the pressure ("pp") or the Schur
    ("S") hierarchy of `cfg` (for building the oracle's counterpart too)."""
    if which == "pp":
        p = dataclasses.replace(cfg.amg, restriction=0, storage=cfg.storage)
        return p if cfg.interp_pp is None else dataclasses.replace(p, interp=cfg.interp_pp)
    if which == "S":
        return dataclasses.replace(cfg.amg, restriction=1, storage=cfg.storage)
    raise ValueError(f"unknown hierarchy {which!r}")


def setup(J, cfg: SolveConfig, concurrent: bool = True, ilu=None):
    """Both hierarchies; with `concurrent`, built at the same time on two
    streams from two host threads (the two setups are independent; each
    call synchronises its own stream before returning).  CPR: the pressure
    hierarchy and the ILU(0) factors of J; `ilu`, a handle built earlier from
    a Jacobian with J's pattern, is refactorised in place (numeric
    factorisation only, the level analysis kept)."""
    import threading

    import torch
    p_pp, p_S = amg_params(cfg, "pp"), amg_params(cfg, "S")
    if cfg.method == "cpr":
        def second(st):
            if ilu is None:
                return tps.ILU0.jacobian(J, stream=st)
            ilu.refactor(J, stream=st)
            return ilu
        make = lambda a, b: tps.Precond.cpr(J, a, b)
    elif cfg.method == "block":
        second = lambda st: _schur_amg(J, cfg, p_S, st)
        make = lambda a, b: tps.Precond(J, a, b, cfg.variant)
    else:
        raise ValueError(f"unknown method {cfg.method!r}")
    if not concurrent:
        a_pp = tps.AMG(J.rowptr, J.col, J.pp, p_pp)
        a_S = second(None)
        return a_pp, a_S, make(a_pp, a_S)
    s1, s2 = _side_streams()
    ev = torch.cuda.Event()
    ev.record()                       # J is complete on the current stream
    s1.wait_event(ev)
    s2.wait_event(ev)
    out, err = {}, []

    def run(key, build, st):
        try:
            out[key] = build(st)
        except Exception as e:        # re-raised below
            err.append(e)

    th = threading.Thread(target=run, args=("S", second, s2))
    th.start()
    run("pp", lambda st: tps.AMG(J.rowptr, J.col, J.pp, p_pp, stream=st), s1)
    th.join()
    if err:
        raise err[0]
    return out["pp"], out["S"], make(out["pp"], out["S"])


def _refresh_pair(hier, J, cfg, refresh):
    """Both hierarchies (or the pressure hierarchy and the ILU(0) factors)
    refreshed for J at the same time, on two streams from two host threads,
    as `setup` builds them; each refresh synchronises its own stream."""
    import threading

    import torch
    s1, s2 = _side_streams()
    ev = torch.cuda.Event()
    ev.record()                       # J is complete on the current stream
    s1.wait_event(ev)
    s2.wait_event(ev)
    err = []

    def run(f):
        try:
            f()
        except Exception as e:        # re-raised below
            err.append(e)

    if cfg.method == "cpr":
        second = lambda: hier[1].refactor(J, stream=s2)
    else:
        second = lambda: refresh(hier[1], _schur_values(J, cfg), s2)
    th = threading.Thread(target=run, args=(second,))
    th.start()
    run(lambda: refresh(hier[0], J.pp, s1))
    th.join()
    if err:
        raise err[0]


def solve(J, G, cfg: SolveConfig, history=False):
    """Newton step: J dx = -G.  Returns (dx, stats, (a_pp, a_S, M)); a_S is
    the ILU(0) handle for the CPR method."""
    a_pp, a_S, M = setup(J, cfg)
    b = -G
    dx, st = tps.fgmres_solve(J, M, b, rtol=cfg.rtol, restart=cfg.restart, maxit=cfg.maxit,
                              history=history)
    return dx, st, (a_pp, a_S, M)


@dataclasses.dataclass
class NewtonConfig:
    """Backward-Euler time stepping with Newton's method on G(x) = 0 (Section
    2.2: one Jacobian solve per Newton iteration; Section 4, opening: a Newton
    iteration has converged when the function norm relative to the step's
    first one, or the step norm relative to the iterate's, is below 1e-8).
    reuse: hierarchy reuse across Newton iterations.  "fine" (or True):
    build both hierarchies at a step's first Newton iteration only and
    refresh their finest level at the later ones (coarse levels lagged).
    "numeric": build at a step's first iteration, then refresh every level
    numerically on the kept C/F splits and patterns (amg_refresh).
    "numeric_run": build once for the run and refresh numerically at every
    later Newton iteration, rebuilding when a solve takes more than
    `rebuild_ratio` times the FGMRES iterations of the first solve after the
    last build.
    line_search: scale each increment by backtracking on |G|^2 / 2 (Section 4, opening:
    Newton with line search; Dennis and Schnabel's rule: try the full step,
    accept when the sufficient-decrease test with alpha = 1e-4 holds, else
    minimise the quadratic model within [lam/10, lam/2], at most 10 times)."""
    steps: int = 20
    max_newton: int = 4
    rtol_f: float = 1e-8
    rtol_dx: float = 1e-8
    reuse: bool | str = False
    line_search: bool = False
    rebuild_ratio: float = 1.5


def _schur_values(J, cfg):
    return {"T": J.S, "ATT": J.TT}.get(cfg.schur)


def _backtrack(prob, dev, J, G, x, dx, gn, alpha=1e-4, max_backtracks=10):
    """Line search along the Newton increment dx from x (|G(x)| = gn).  For a
    Newton direction f(lam) = |G(x + lam dx)|^2 / 2 has slope -gn^2 at 0.  The
    full step is tried first; a trial passes when f(lam) <= f(0) - alpha lam
    gn^2; otherwise the next trial is the minimiser of the quadratic matching
    f(0), f'(0) and f(lam), clamped to [lam/10, lam/2].  A trial whose |G| is
    not finite (a state outside the fluid laws' range) halves lam without the
    quadratic model.  After max_backtracks failures the last trial stands if
    its |G| is finite; otherwise FloatingPointError is raised.  J and G are
    left assembled at the accepted point, which dev["x_k"] holds.  Returns
    (lam, rejected trials, |G| there)."""
    import math

    import torch
    g2 = gn * gn
    lam, rejected = 1.0, 0
    while True:
        dev["x_k"] = torch.add(x, dx, alpha=lam)
        assemble(prob, dev, J, G)
        gt = float(torch.linalg.vector_norm(G))
        finite = math.isfinite(gt)
        if finite and (0.5 * gt * gt <= 0.5 * g2 - alpha * lam * g2 or rejected == max_backtracks):
            return lam, rejected, gt
        if rejected == max_backtracks:
            raise FloatingPointError(f"line search: |G| not finite at the last trial step {lam:g}")
        if finite:
            lam = min(max(g2 * lam * lam / (2.0 * (0.5 * gt * gt - 0.5 * g2 + g2 * lam)), 0.1 * lam), 0.5 * lam)
        else:
            lam = 0.5 * lam
        rejected += 1


class LearnedGuard:
    """When a solve runs with the learned post-smoother, and the contraction
    it must keep (tp_krylov_params.ref_rate).

    The first solve of a run is plain: its mean contraction per iteration
    rho_p = rel_true^(1/iters) and its FGMRES time per iteration t_p are
    kept, and every later plain solve updates them.  A learned solve passes
    ref_rate = rho_p^(t_l / t_p), t_l the learned solves' own time per
    iteration (t_p until one has been timed): the rate at which it reaches
    the plain solve's residual in the plain solve's time, so the network is
    switched off as soon as it falls behind the plain form in time, not
    only when it stagnates.  A learned solve that ran to the end without
    being switched off is still behind when its time per decade of
    residual reduction, FGMRES time / -log10(rel_true), exceeds the last
    plain solve's (short solves end before the per-iteration check can
    act).  After two learned solves in a row that were behind (switched off
    or slower per decade), the rest of the run is plain."""

    def __init__(self):
        self.rho_p = self.t_p = self.t_l = None
        self.tau_p = None   # plain solve's FGMRES seconds per decade
        self.streak = 0
        self.off = False
        self.learned_solves = self.plain_solves = self.switched_off = self.slower = 0

    def use_net(self):
        return self.rho_p is not None and not self.off

    def ref_rate(self):
        c = self.t_l / self.t_p if (self.t_l and self.t_p) else 1.0
        return min(self.rho_p ** c, 0.999)

    @staticmethod
    def _per_decade(st, fgmres_s):
        d = -math.log10(st["rel_true"]) if st["rel_true"] > 0.0 else 0.0
        return fgmres_s / d if d > 0.0 else math.inf

    def record(self, st, fgmres_s, learned):
        its = max(st["iters"], 1)
        per_it = fgmres_s / its
        if not learned:
            self.plain_solves += 1
            if st["converged"] and st["rel_true"] > 0.0:
                self.rho_p = st["rel_true"] ** (1.0 / its)
                self.t_p = per_it
                self.tau_p = self._per_decade(st, fgmres_s)
            return
        self.learned_solves += 1
        behind = False
        if st["fallback_iter"] >= 0:
            self.switched_off += 1
            behind = True
        else:
            self.t_l = per_it
            if self.tau_p is not None and self._per_decade(st, fgmres_s) > self.tau_p:
                self.slower += 1
                behind = True
        self.streak = self.streak + 1 if behind else 0
        self.off = self.off or self.streak >= 2

    def stats(self):
        return dict(learned_solves=self.learned_solves, plain_solves=self.plain_solves,
                    network_switched_off=self.switched_off, slower_per_decade=self.slower,
                    network_off_for_rest=self.off)


def simulate(prob, cfg: SolveConfig, ncfg: NewtonConfig, net=None, log=None, on_solve=None):
    """Run `ncfg.steps` time steps of `prob` from its x_prev.  Each Newton
    iteration assembles at the current iterate (into the same Jacobian
    buffers), builds both hierarchies (or, with `ncfg.reuse`, refreshes their
    finest level after a step's first iteration; `net` attached to the Schur
    hierarchy when given) and solves J dx = -G to `cfg.rtol`.  `on_solve`,
    when given, is called before each linear solve with (step, Newton
    iteration, x_prev, x_k) (device tensors; copy them to keep them).  With
    `net`, a LearnedGuard decides per solve whether the network is attached
    and passes its contraction bound to FGMRES.  Returns (x, stats): the
    final state (device, interleaved) and per-run counts and times."""
    import time

    import torch
    if net is not None and cfg.method != "block":
        raise ValueError("the learned smoother belongs to the Schur hierarchy of the block preconditioner")
    dev = to_device(prob)
    x = dev["x_prev"].clone()
    dev["x_k"] = x
    newton, lin, solves, unconverged, builds, backtracks = 0, 0, 0, 0, 0, 0
    lin_unconverged = 0   # linear solves that ended above rtol (maxit or the rounding floor)
    step_lengths = []
    solve_s = 0.0
    per_step = []
    lin_per_step = []
    J = G = None
    hier = None

    ilu = None   # CPR: one ILU(0) handle per run, refactorised for every Jacobian

    def close(h, final=False):
        if h is not None:
            a_pp, a_S, M = h
            if net is not None:
                a_S.attach(None, None)     # (a no-op when nothing is attached)
            M.close(); a_pp.close()
            if cfg.method != "cpr" or final:
                a_S.close()

    # S_diag has a pattern of its own; CPR refactorises its ILU(0) in place
    mode = {False: None, None: None, True: "fine"}.get(ncfg.reuse, ncfg.reuse)
    if mode not in (None, "fine", "numeric", "numeric_run"):
        raise ValueError(f"unknown reuse mode {ncfg.reuse!r}")
    reusable = mode is not None and (cfg.method == "cpr" or cfg.schur in ("T", "ATT"))
    refresh = ((lambda h, v, st: h.refresh_fine(v, stream=st)) if mode == "fine"
               else (lambda h, v, st: h.refresh(v, stream=st)))
    refreshes, base_its, rebuild = 0, None, False
    guard = LearnedGuard() if net is not None else None
    attached = False
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    try:
        for step in range(ncfg.steps):
            dev["x_prev"] = x.clone()
            g0 = None
            its = 0
            lin0 = lin
            done = False
            fresh = False   # J and G already assembled at x (by the line search)
            for k in range(ncfg.max_newton + 1):
                if not fresh:
                    J, G = assemble(prob, dev, J, G)
                fresh = False
                gn = float(torch.linalg.vector_norm(G))
                if g0 is None:
                    g0 = gn
                if gn <= ncfg.rtol_f * g0 or done or k == ncfg.max_newton:
                    if not (gn <= ncfg.rtol_f * g0 or done):
                        unconverged += 1
                    break
                if on_solve is not None:
                    on_solve(step, k, dev["x_prev"], dev["x_k"])
                torch.cuda.synchronize()
                ts = time.perf_counter()
                built = False
                if hier is not None and reusable and (k > 0 or mode == "numeric_run") and not rebuild:
                    _refresh_pair(hier, J, cfg, refresh)
                    refreshes += 1
                else:
                    close(hier)
                    hier = None
                    hier = setup(J, cfg, ilu=ilu)
                    if cfg.method == "cpr":
                        ilu = hier[1]
                    builds += 1
                    built, rebuild = True, False
                    attached = False
                learned = guard is not None and guard.use_net()
                if guard is not None and learned != attached:
                    hier[1].attach(net if learned else None, prob.grid if learned else None)
                    attached = learned
                tf = time.perf_counter()
                dx, st = tps.fgmres_solve(J, hier[2], -G, rtol=cfg.rtol, restart=cfg.restart, maxit=cfg.maxit,
                                          ref_rate=guard.ref_rate() if learned else 0.0)
                torch.cuda.synchronize()
                te = time.perf_counter()
                solve_s += te - ts
                if guard is not None:
                    guard.record(st, te - tf, learned)
                if mode == "numeric_run":
                    if built:
                        base_its = st["iters"]
                    elif st["iters"] > ncfg.rebuild_ratio * base_its:
                        rebuild = True
                if not reusable:
                    close(hier)
                    hier = None
                if ncfg.line_search:
                    lam, rej, gn = _backtrack(prob, dev, J, G, x, dx, gn)
                    x.copy_(dev["x_k"])
                    dev["x_k"] = x
                    dx *= lam
                    backtracks += rej
                    step_lengths.append(lam)
                    fresh = True
                else:
                    x += dx
                its += 1
                lin += st["iters"]
                solves += 1
                lin_unconverged += 0 if st["converged"] else 1
                done = float(torch.linalg.vector_norm(dx)) <= ncfg.rtol_dx * float(torch.linalg.vector_norm(x))
            newton += its
            per_step.append(its)
            lin_per_step.append(lin - lin0)
            if log:
                log(f"step {step}: newton {its}, |G|/|G0| {gn / g0 if g0 else 0.0:.2e}")
    finally:
        close(hier, final=True)
        if ilu is not None:
            ilu.close()
    torch.cuda.synchronize()
    total = time.perf_counter() - t0
    extra = guard.stats() if guard is not None else {}
    return x, dict(extra, steps=ncfg.steps, newton_iters=newton, linear_iters=lin, solves=solves,
                   linear_unconverged=lin_unconverged,
                   backtracks=backtracks, step_lengths=step_lengths,
                   hierarchy_builds=builds, hierarchy_refreshes=refreshes, unconverged_steps=unconverged, newton_per_step=per_step,
                   linear_per_step=lin_per_step,
                   linear_per_newton=lin / max(newton, 1), total_s=total,
                   ms_per_solve=1e3 * solve_s / max(solves, 1))
