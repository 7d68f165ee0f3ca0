"""One coupled pressure-temperature solve on the GPU, end to end.

assemble_tpfa -> amg_setup(A_pp) and amg_setup(S) -> precond_create ->
fgmres_solve, all through the C ABI.  The Schur-approximation hierarchy uses
the Petrov-Galerkin restriction (its columns, not its rows, are diagonally
dominant); the pressure hierarchy the Galerkin one.
"""
from __future__ import annotations

import dataclasses

from . import tpsolve as tps


@dataclasses.dataclass
class SolveConfig:
    rtol: float = 1e-8
    restart: int = 30
    maxit: int = 1000
    variant: str = "lower"
    storage: int = 0              # 0 FP64 hierarchy, 1 FP32
    amg: tps.AmgParams = dataclasses.field(default_factory=tps.AmgParams)


def to_device(prob, device="cuda"):
    import torch
    t = lambda a: torch.as_tensor(a, dtype=torch.float64, device=device)
    return dict(K=t(prob.K), phi=t(prob.phi), kappa=t(prob.kappa), x_prev=t(prob.x_prev),
                x_k=t(prob.x_k))


def assemble(prob, dev):
    return tps.assemble_tpfa(prob.grid, prob.props, dev["K"], dev["phi"], dev["kappa"],
                             prob.wells, prob.dt, dev["x_prev"], dev["x_k"])


def setup(J, cfg: SolveConfig):
    p_pp = dataclasses.replace(cfg.amg, restriction=0, storage=cfg.storage)
    p_S = dataclasses.replace(cfg.amg, restriction=1, storage=cfg.storage)
    a_pp = tps.AMG(J.rowptr, J.col, J.pp, p_pp)
    a_S = tps.AMG(J.rowptr, J.col, J.S, p_S)
    return a_pp, a_S, tps.Precond(J, a_pp, a_S, cfg.variant)


def solve(J, G, cfg: SolveConfig, history=False):
    """Newton step: J dx = -G.  Returns (dx, stats, (a_pp, a_S, M))."""
    a_pp, a_S, M = setup(J, cfg)
    b = -G
    dx, st = tps.fgmres_solve(J, M, b, rtol=cfg.rtol, restart=cfg.restart, maxit=cfg.maxit,
                              history=history)
    return dx, st, (a_pp, a_S, M)
