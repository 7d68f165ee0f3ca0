"""Learned post-smoother for the Schur-approximation V-cycle: training-pair
generation, training and evaluation, all on the GPU through the C ABI.

Pairs come from the plain solver's own V-cycle.  `plain_solve_pairs` runs
the first Arnoldi steps of the plain block-preconditioned FGMRES on a
field's Jacobian and records, at every preconditioner apply, the right-hand
side b_V the Schur hierarchy's V-cycle receives (step 2 of the block
list: b_V = r_T - A_Tp z_p); y* = S^{-1} b_V comes from an inner GMRES
solve to 1e-10, preconditioned by the same V-cycle.  The V-cycle from a zero guess on b = S y*, stopped just before the
finest-level post-smoothing, leaves x; the post-smoother's input is
r = b - S x and the error it should remove is e = y* - x.  (`make_pairs`
draws y at random instead.)  The network sees the features of r (scaled by
s = RMS(D^{-1} r)) and is trained to output e / s (Adam).
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


def _interleaved_csr(J):
    """The 2n x 2n Jacobian (interleaved [p_i, T_i]) and the blocks A_Tp and S
    as SciPy CSR matrices on the host (pair generation on small grids)."""
    import scipy.sparse as sp
    n = J.n
    rp, ci = J.rowptr.cpu().numpy(), J.col.cpu().numpy()
    blk = {k: sp.csr_matrix((getattr(J, k).cpu().numpy(), ci, rp), shape=(n, n)) for k in ("pp", "pT", "Tp", "TT", "S")}
    rows = np.repeat(np.arange(n), np.diff(rp))
    r = np.concatenate([2 * rows, 2 * rows, 2 * rows + 1, 2 * rows + 1])
    c = np.concatenate([2 * ci, 2 * ci + 1, 2 * ci, 2 * ci + 1]).astype(np.int64)
    v = np.concatenate([blk["pp"].data, blk["pT"].data, blk["Tp"].data, blk["TT"].data])
    return sp.csr_matrix((v, (r, c)), shape=(2 * n, 2 * n)), blk


def _schur_solve(a_S, S, b, rtol=1e-10, m=40, maxit=400):
    """y = S^{-1} b (host vectors) by right-preconditioned GMRES(m) with the
    field's own Schur V-cycle as the preconditioner (the V-cycle on the GPU,
    the products with S and the Gram-Schmidt passes on the host)."""
    import torch
    bn = np.linalg.norm(b)
    y = np.zeros_like(b)
    if bn == 0.0:
        return y
    it = 0
    while it < maxit:
        r = b - S @ y
        beta = np.linalg.norm(r)
        if beta <= rtol * bn:
            break
        V = [r / beta]
        Z = []
        H = np.zeros((m + 1, m))
        k = 0
        for j in range(m):
            z = a_S.vcycle(torch.as_tensor(V[j], device="cuda")).cpu().numpy()
            Z.append(z)
            w = S @ z
            for _ in range(2):                            # Gram-Schmidt, two passes
                for i, q in enumerate(V):
                    hij = q @ w
                    H[i, j] += hij
                    w = w - hij * q
            H[j + 1, j] = np.linalg.norm(w)
            k = j + 1
            it += 1
            e1 = np.zeros(k + 1)
            e1[0] = beta
            c, res, _, _ = np.linalg.lstsq(H[:k + 1, :k], e1, rcond=None)
            est = np.linalg.norm(H[:k + 1, :k] @ c - e1)
            if est <= rtol * bn or H[j + 1, j] == 0.0 or it >= maxit:
                break
            V.append(w / H[j + 1, j])
        e1 = np.zeros(k + 1)
        e1[0] = beta
        c = np.linalg.lstsq(H[:k + 1, :k], e1, rcond=None)[0]
        y = y + np.column_stack(Z[:k]) @ c
    return y


def plain_solve_pairs(prob, net, arnoldi_steps=3, cfg=None):
    """Training samples at the plain solve's own finest-level post-smoothing
    points of the Schur V-cycle (see the module docstring): the first
    `arnoldi_steps` Arnoldi steps of the right-preconditioned solve of
    J dx = -G on the field `prob`, each preconditioner apply's Schur
    right-hand side b_V, y* = S^{-1} b_V by an inner solve to 1e-10
    (`_schur_solve`), and the pair (r, e) at the point the post-smoother
    would act.  The samples keep
    the field's Schur hierarchy, attached to `net` (operator-norm loss)."""
    import torch
    cfg = cfg or solver.SolveConfig()
    dev = solver.to_device(prob)
    J, G = solver.assemble(prob, dev)
    a_pp, a_S, M = solver.setup(J, cfg, concurrent=False)
    M.close()
    Jh, blk = _interleaved_csr(J)
    n = J.n
    b = -G.cpu().numpy()
    V = [b / np.linalg.norm(b)]
    pairs = []
    for _ in range(arnoldi_steps):
        v = V[-1]
        zp = a_pp.vcycle(torch.as_tensor(np.ascontiguousarray(v[0::2]), device="cuda")).cpu().numpy()
        bV = v[1::2] - blk["Tp"] @ zp                    # the Schur V-cycle's right-hand side
        zT = a_S.vcycle(torch.as_tensor(bV, device="cuda")).cpu().numpy()   # plain cycle (no network yet)
        ystar = _schur_solve(a_S, blk["S"], bV)
        pairs.append(a_S.presmoothed_pair(torch.as_tensor(ystar, device="cuda")))
        z = np.empty(2 * n)
        z[0::2], z[1::2] = zp, zT
        w = Jh @ z
        for _ in range(2):                               # Gram-Schmidt, two passes
            for q in V:
                w = w - (q @ w) * q
        V.append(w / np.linalg.norm(w))
    a_S.attach(net, prob.grid)                           # features need the attachment's diagonal
    out = []
    for r, e in pairs:
        f, sc = a_S.features(r)
        out.append(Sample(prob.grid, f.clone(), (e / sc).float(), a_S))
    a_pp.close()
    return out


# the C4 training set: 200 seeded fields of the channelised recipe; the
# thermal conductivity cycles over the 256x256x64 runs' two values and the
# recipe's own, so the network sees conduction- and advection-dominated
# Schur operators
C4_SEEDS = range(1000, 1200)
C4_KAPPAS = (2.0, 0.5, 20.0)


def train_c4(quick=False, grid=None, steps=None, lr=3e-3, seed=0, loss="op", err_weight=0.0, log=None):
    """Train a network on the GPU on the C4 set: pairs from plain solves
    (`plain_solve_pairs`, three Arnoldi steps per field) of the channelised
    recipe at 24^3 (fields 1000-1199, conductivity C4_KAPPAS[seed % 3]),
    Adam on the operator-norm loss (loss="op", plus err_weight times the
    error loss) or the error loss alone (loss="err").  quick: 12 fields, 300
    steps.  Returns (Net, record)."""
    grid = grid or synth.Grid(24, 24, 24, 1.0, 1.0, 1.0)
    seeds = list(C4_SEEDS)[:12] if quick else list(C4_SEEDS)
    steps = steps or (300 if quick else 3000)
    net = tps.Net(init_params(seed))
    samples = []
    for sd in seeds:
        prob = synth.make_problem("W4", seed=sd, grid=grid, kappa=C4_KAPPAS[sd % len(C4_KAPPAS)])
        samples += plain_solve_pairs(prob, net)
    losses = train(net, samples, steps, lr=lr, loss=loss, err_weight=err_weight)
    hier = {id(smp.amg): smp.amg for smp in samples}
    for h in hier.values():
        h.attach(None, None)
        h.close()
    rec = {"fields": f"channelised recipe {grid.nx}^3, seeds {seeds[0]}-{seeds[-1]} ({len(seeds)} fields), "
                     f"conductivity cycling over {C4_KAPPAS}",
           "pairs": len(samples), "pair_source": "Schur V-cycle inputs of the first 3 Arnoldi steps of plain solves",
           "loss": loss, "err_weight": err_weight, "adam_steps": steps, "lr": lr, "loss_first": float(losses[0]),
           "loss_last_100_mean": float(np.mean(losses[-100:]))}
    if log:
        log(rec)
    return net, rec


C4_EVAL_SEEDS = (4001, 4002, 4003, 4004, 4005)


def evaluate_c4(net, seeds=C4_EVAL_SEEDS, grid=None, storage=0, rtol=1e-8):
    """Held-out evaluation on the channelised recipe (96^3 by default): per
    seed, FGMRES iterations, FGMRES time and true residual of the plain form
    (the hierarchy's Chebyshev post-smoother), of the learned form (the
    network as the Schur hierarchy's finest-level post-smoother, stagnation
    guard on), of the learned form with the contraction guard as well
    (ref_rate = the plain solve's mean contraction per iteration), and of
    the same cycle with no finest-level post-smoothing at all (an all-zero
    network: what the network's slot gives without it)."""
    import torch
    grid = grid or synth.Grid(96, 96, 96, 1.0, 1.0, 1.0)
    cfg = solver.SolveConfig(rtol=rtol, storage=storage)
    zero = tps.Net(np.zeros(NPARAM, dtype=np.float32))
    rows = []
    for sd in seeds:
        prob = synth.make_problem("W4", seed=sd, grid=grid)
        dev = solver.to_device(prob)
        J, G = solver.assemble(prob, dev)
        row = {"seed": sd}
        rho_p = 0.0
        for key, nt in (("plain", None), ("learned", net), ("learned_guarded", net), ("no_post", zero)):
            a_pp, a_S, M = solver.setup(J, cfg)
            if nt is not None:
                a_S.attach(nt, grid)
            ref = rho_p if key == "learned_guarded" else 0.0
            tps.fgmres_solve(J, M, -G, rtol=rtol, ref_rate=ref)          # warm (graph capture)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            x, st = tps.fgmres_solve(J, M, -G, rtol=rtol, stag_ratio=0.0 if key == "no_post" else 0.95,
                                     ref_rate=ref)
            if key == "plain":
                rho_p = st["rel_true"] ** (1.0 / max(st["iters"], 1))
            torch.cuda.synchronize()
            row[key] = {"iters": st["iters"], "fgmres_ms": round((time.perf_counter() - t0) * 1e3, 3),
                        "rel_true": st["rel_true"], "converged": st["converged"],
                        "fallback_iter": st["fallback_iter"]}
            if nt is not None:
                a_S.attach(None, None)
            M.close(); a_pp.close(); a_S.close()
        rows.append(row)
    zero.close()
    return rows


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
