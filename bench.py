"""Benchmark: time-to-rtol 1e-8 of one coupled pressure-temperature solve.

A step is one pass of the whole hot path on the 64x64x32 layered workload
(262,144 unknowns): TPFA assembly of the Jacobian and Schur approximation,
AMG setup of A_pp and of S, block lower-triangular preconditioner, FGMRES(30)
with CGS2 to a true relative residual <= 1e-8.  Inputs (fields and states)
are resident in HBM before the timed region.  One JSON line on stdout.

Extra objects in the line:
  roofline      the fine-level smoother sweep (the V-cycle's dominant
                kernel): algorithmic bytes per launch / mean launch time from
                HIP events recorded on its stream during the timed steps;
  cpu_baseline  the CPU FP64 oracle, single-threaded, on the same workload
                (one full solve), run on rank 0 only.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0

WORKLOADS = {
    "W2": dict(desc="64x64x32 layered log-normal permeability, corner wells 450 K, "
                    "perturbed Newton state, FP64 plain method"),
    "W3": dict(desc="128x128x64 layered log-normal permeability, corner wells 450 K, "
                    "perturbed Newton state"),
    "W4": dict(desc="96^3 channelised permeability, hot injection 550 K, perturbed state"),
}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="W2", choices=list(WORKLOADS))
    ap.add_argument("--storage", type=int, default=0, help="0 FP64 hierarchy, 1 FP32")
    ap.add_argument("--rtol", type=float, default=1e-8)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; --gpus must be 1"}))
        sys.exit(2)

    import numpy as np
    import torch

    from paper_1902_00095_amd import solver, synth
    from paper_1902_00095_amd import tpsolve as tps

    tps.init(0)
    prob = synth.make_problem(args.workload)
    dev = solver.to_device(prob)
    cfg = solver.SolveConfig(rtol=args.rtol, storage=args.storage)

    def step():
        J, G = solver.assemble(prob, dev)
        dx, st, (a_pp, a_S, M) = solver.solve(J, G, cfg)
        info = dict(iters=st["iters"], rel_true=st["rel_true"], converged=st["converged"],
                    levels_pp=a_pp.nlev, levels_S=a_S.nlev)
        M.close(); a_pp.close(); a_S.close()
        return info

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    infos = []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        infos.append(step())
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms_per_step = (t1 - t0) * 1e3 / args.steps
    # roofline pass: the same steps again with the fine-level smoother's
    # launches carrying HIP event pairs (kept out of the metric's region
    # because event recording slows the step)
    tps.timer_enable(True)
    for _ in range(min(args.steps, 3)):
        step()
    torch.cuda.synchronize()
    launches, kms, kbytes = tps.timer_read()
    tps.timer_enable(False)
    achieved = (kbytes / launches) / (kms / launches * 1e-3) / 1e9 if launches else 0.0

    # phase breakdown of one more (untimed) step, synchronised between phases
    def tsync():
        torch.cuda.synchronize()
        return time.perf_counter()
    ph = {}
    t_a = tsync()
    J, G = solver.assemble(prob, dev)
    t_b = tsync()
    import dataclasses as _dc
    a_pp = tps.AMG(J.rowptr, J.col, J.pp, _dc.replace(cfg.amg, restriction=0, storage=cfg.storage))
    t_c = tsync()
    a_S = tps.AMG(J.rowptr, J.col, J.S, _dc.replace(cfg.amg, restriction=1, storage=cfg.storage))
    t_d = tsync()
    M = tps.Precond(J, a_pp, a_S, cfg.variant)
    _, st = tps.fgmres_solve(J, M, -G, rtol=cfg.rtol, restart=cfg.restart, maxit=cfg.maxit)
    t_e = tsync()
    ph = {"assemble_ms": round((t_b - t_a) * 1e3, 3), "setup_pp_ms": round((t_c - t_b) * 1e3, 3),
          "setup_S_ms": round((t_d - t_c) * 1e3, 3), "fgmres_ms": round((t_e - t_d) * 1e3, 3)}
    M.close(); a_pp.close(); a_S.close()

    # V-cycle-only throughput on a fixed right-hand side (warm caches)
    J, G = solver.assemble(prob, dev)
    a_pp, a_S, M = solver.setup(J, cfg)
    b = -G
    z = torch.empty_like(b)
    for _ in range(3):
        M.apply(b, z)
    torch.cuda.synchronize()
    nrep = 50
    ts = time.perf_counter()
    for _ in range(nrep):
        M.apply(b, z)
    torch.cuda.synchronize()
    precond_ms = (time.perf_counter() - ts) * 1e3 / nrep

    line = {
        "metric": "time-to-rtol 1e-8 per coupled P-T solve (assembly + 2 AMG setups + FGMRES)",
        "value": round(ms_per_step, 3),
        "unit": "ms/solve",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 3),
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if args.storage == 0 else "f64-outer/f32-hierarchy",
        "data": "synthetic",
        "config": {"workload": f"{args.workload}: {WORKLOADS[args.workload]['desc']}",
                   "unknowns": 2 * prob.grid.n, "rtol": args.rtol,
                   "fgmres_iters": infos[-1]["iters"], "rel_true": infos[-1]["rel_true"],
                   "amg_levels": [infos[-1]["levels_pp"], infos[-1]["levels_S"]],
                   "precond_apply_ms": round(precond_ms, 4), "phases": ph},
        "roofline": {"bound": "hbm", "kernel": "k_cheb_step (fine level)",
                     "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None,
                     "launches": launches, "mean_us": round(kms / max(launches, 1) * 1e3, 3),
                     "bytes_per_launch": round(kbytes / max(launches, 1))},
    }
    if not all(i["converged"] for i in infos):
        line["error"] = "a timed solve did not converge"

    if not args.no_cpu_baseline:
        import oracle
        oracle.build(force=False)
        tc = time.perf_counter()
        Jo = oracle.jacobian(prob)
        bo = -oracle.residual(prob)
        ao_pp = oracle.AMG(Jo.n, Jo.rowptr, Jo.col, Jo.pp)
        ao_S = oracle.AMG(Jo.n, Jo.rowptr, Jo.col, Jo.S, restriction=1)
        xo, io = oracle.gmres(Jo, ao_pp, ao_S, bo, rtol=args.rtol)
        cpu_ms = (time.perf_counter() - tc) * 1e3
        line["cpu_baseline"] = {"value": round(cpu_ms, 1), "unit": "ms/solve", "cores": 1,
                                "kind": "oracle",
                                "sample": f"one full {args.workload} solve (assembly, 2 AMG setups, "
                                          f"GMRES to rtol {args.rtol}: {io['iters']} iterations), "
                                          "single-threaded FP64 C"}
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
