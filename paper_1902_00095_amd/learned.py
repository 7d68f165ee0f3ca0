"""Learned post-smoother for the Schur-approximation V-cycle: training-pair
generation, training and evaluation, all on the GPU through the C ABI.

Pairs come from the plain solver's own V-cycle: for a seeded random y,
b = S y; the V-cycle from a zero guess, stopped just before the finest-level
post-smoothing, leaves x; the post-smoother's input is r = b - S x and the
error it should remove is e = y - x, known exactly (no inner solve).  The
network sees the features of r (scaled by s = RMS(D^{-1} r)) and is trained
to output e / s (mean squared error, Adam).
"""
from __future__ import annotations

import dataclasses
import time

import numpy as np

from . import solver, synth
from . import tpsolve as tps

NPARAM = tps.CNN_NPARAM


def init_params(seed: int = 0) -> np.ndarray:
    """He-scaled first layer, small second layer: the untrained network's
    correction is close to zero."""
    rng = np.random.default_rng(np.random.PCG64(seed))
    w1 = rng.standard_normal(16 * 8 * 27) * np.sqrt(2.0 / (8 * 27))
    b1 = np.zeros(16)
    w2 = rng.standard_normal(16 * 27) * np.sqrt(1.0 / (16 * 27)) * 0.1
    b2 = np.zeros(1)
    return np.concatenate([w1, b1, w2, b2]).astype(np.float32)


@dataclasses.dataclass
class Sample:
    grid: synth.Grid
    feat: object     # torch (8n,) float32
    target: object   # torch (n,) float32
    amg: object = None   # Schur hierarchy of the field (operator-norm loss)


def schur_hierarchy(J, storage=0, coarse_max=None):
    """The Schur-approximation hierarchy the learned smoother attaches to
    (coarse_max None: the library default)."""
    prm = tps.AmgParams(restriction=1, storage=storage)
    if coarse_max is not None:
        prm.coarse_max = coarse_max
    return tps.AMG(J.rowptr, J.col, J.S, prm)


def make_pairs(seeds, grid, net=None, per_field=1, workload="W4", smooth_y=0):
    """Training samples from the plain V-cycle on seeded fields.  With `net`
    the field's Schur hierarchy stays attached to it (operator-norm loss)."""
    import torch
    net0 = net if net is not None else tps.Net(init_params())
    out = []
    for seed in seeds:
        prob = synth.make_problem(workload, seed=seed, grid=grid)
        dev = solver.to_device(prob)
        J, G = solver.assemble(prob, dev)
        a_S = schur_hierarchy(J)
        a_S.attach(net0, grid)
        gen = torch.Generator(device="cuda").manual_seed(int(seed))
        for _ in range(per_field):
            y = torch.randn(grid.n, generator=gen, dtype=torch.float64, device="cuda")
            for _ in range(smooth_y):          # smoother errors: y <- V-cycle(y)
                y = a_S.vcycle(y)
                y = y / torch.linalg.vector_norm(y)
            r, e = a_S.presmoothed_pair(y)
            f, s = a_S.features(r)
            out.append(Sample(grid, f.clone(), (e / s).float(), a_S if net is not None else None))
        if net is None:
            a_S.attach(None, None)
            a_S.close()
    if net is None:
        net0.close()
    return out


def sample_loss(net, smp, loss="op", err_weight=0.0):
    """Operator-norm loss ||D^{-1} S (out - e/s)||^2 / n (the residual the
    correction leaves) plus err_weight ||out - e/s||^2 / n, or the Euclidean
    error loss ||out - e/s||^2 / n alone."""
    if loss == "op":
        return smp.amg.op_loss_grad(smp.feat, smp.target, err_weight)
    return net.loss_grad(smp.grid, smp.feat, smp.target)


def train(net, samples, steps, lr=1e-3, log_every=0, loss="op", err_weight=0.0):
    losses = []
    for it in range(steps):
        smp = samples[it % len(samples)]
        loss_v = sample_loss(net, smp, loss, err_weight)
        net.adam_step(lr)
        losses.append(loss_v)
        if log_every and (it % log_every == 0 or it == steps - 1):
            print(f"  step {it:5d} loss {loss_v:.4e}", flush=True)
    return np.asarray(losses)


def eval_loss(net, samples, loss="op", err_weight=0.0):
    return float(np.mean([sample_loss(net, s, loss, err_weight) for s in samples]))


def compare(net, prob, cfg=None, stag_ratio=0.95):
    """Plain vs learned solve of one problem: iterations, time, residual."""
    import torch
    cfg = cfg or solver.SolveConfig()
    dev = solver.to_device(prob)
    J, G = solver.assemble(prob, dev)
    res = {}
    for mode in ("plain", "learned"):
        a_pp, a_S, M = solver.setup(J, cfg)
        if mode == "learned":
            a_S.attach(net, prob.grid)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        x, st = tps.fgmres_solve(J, M, -G, rtol=cfg.rtol, restart=cfg.restart, maxit=cfg.maxit,
                                 stag_ratio=stag_ratio)
        torch.cuda.synchronize()
        st["solve_ms"] = (time.perf_counter() - t0) * 1e3
        res[mode] = st
        if mode == "learned":
            a_S.attach(None, None)
        M.close(); a_pp.close(); a_S.close()
    return res
