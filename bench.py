"""Benchmark: time-to-rtol 1e-8 per coupled pressure-temperature solve,
mixed precision + learned post-smoother against plain FP64, and V-cycle GB/s.

Headline workload: the 256x256x64 grid (4,194,304 cells, 8,388,608
unknowns), layered log-normal permeability with channel streaks, corner wells
(450 K injection), thermal conductivity 20 W/m/K, uniform initial state.  Its
Newton systems of the first backward-Euler steps (day 1, 2) are produced by
the GPU time stepper before the timed region and kept in HBM.  A step is one
coupled solve of one of them: TPFA assembly of the Jacobian blocks and of
S~_T, AMG setup of A_pp and of S~_T, the block lower-triangular
preconditioner and FGMRES(30) with CGS2 to a true relative residual <= 1e-8.
`value` times it in the mixed-precision + learned form (FP32 hierarchies and
V-cycles, the trained network as the Schur hierarchy's finest-level
post-smoother, FP64 outer loop, residuals and coarsest inverse); the same
steps in the plain FP64 form are timed next and reported beside it with the
ratio.  One JSON line on stdout; progress on stderr.

Extra objects in the line:
  roofline      the timed form's dominant kernel, the finest-level Chebyshev
                step (FP32 values and vectors, seven diagonals):
                algorithmic bytes per launch / mean launch duration, from HIP
                event pairs carried by every launch of that kernel during two
                more solves of the timed form on the same stream;
  cpu_baseline  the CPU FP64 oracle, single-threaded, on one of the same
                Newton systems: assembly and both AMG setups timed once,
                GMRES iterations timed as the median of three one-iteration
                runs, scaled to a whole solve by the plain GPU path's
                iteration count; the same computations check the GPU's
                assembly, every hierarchy level's C/F split and pattern, and
                the first residual estimate on that system.
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
RTOL = 1e-8

HEADLINE = ("256x256x64 (8,388,608 unknowns) layered log-normal permeability with channel streaks, "
            "corner wells 450 K, thermal conductivity 20 W/m/K, Newton systems of backward-Euler "
            "steps 1-2 (dt 1 day)")


def _progress(msg):
    """One line per finished stage on stderr (the JSON result stays the only stdout line)."""
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def _sync_time():
    import torch
    torch.cuda.synchronize()
    return time.perf_counter()


# ---- the learned post-smoother ------------------------------------------------------------------
def trained_network(quick=False):
    """The network trained on the GPU by the library's own kernels (learned.train_c4),
    with its training record."""
    from paper_1902_00095_amd import learned
    t0 = time.perf_counter()
    net, rec = learned.train_c4(quick=quick)
    rec["seconds"] = round(time.perf_counter() - t0, 2)
    return net, rec


# ---- Newton systems of the headline workload -------------------------------------------------
def newton_systems(prob, steps):
    """(x_prev, x_k) before every linear solve of the first `steps` time steps,
    from the GPU time stepper (FP32 hierarchies); device tensors."""
    from paper_1902_00095_amd import solver
    out = []

    def rec(step, k, xp, xk):
        out.append((step, k, xp.clone(), xk.clone()))
    solver.simulate(prob, solver.SolveConfig(storage=1), solver.NewtonConfig(steps=steps), on_solve=rec)
    return out


class Solves:
    """One coupled solve per call on a workload's device fields."""

    def __init__(self, prob):
        from paper_1902_00095_amd import solver
        self.prob = prob
        self.dev = solver.to_device(prob)
        self.J = self.G = None

    def assemble(self, system):
        from paper_1902_00095_amd import solver
        if system is not None:
            self.dev["x_prev"], self.dev["x_k"] = system[2], system[3]
        self.J, self.G = solver.assemble(self.prob, self.dev, self.J, self.G)

    def run(self, system, cfg, net=None, keep=False, history=False, guard=None):
        """With `net`: the learned post-smoother on the Schur hierarchy; with a
        LearnedGuard as well, the guard decides whether this solve uses it and
        passes its contraction bound (and records the solve)."""
        import torch

        from paper_1902_00095_amd import solver
        from paper_1902_00095_amd import tpsolve as tps
        if system is not None:
            self.dev["x_prev"], self.dev["x_k"] = system[2], system[3]
        self.J, self.G = solver.assemble(self.prob, self.dev, self.J, self.G)
        a_pp, a_S, M = solver.setup(self.J, cfg)
        learned = net is not None and (guard is None or guard.use_net())
        if learned:
            a_S.attach(net, self.prob.grid)
        tf = time.perf_counter()
        x, st = tps.fgmres_solve(self.J, M, -self.G, rtol=cfg.rtol, restart=cfg.restart, maxit=cfg.maxit,
                                 history=history, ref_rate=guard.ref_rate() if (learned and guard) else 0.0)
        if guard is not None:
            torch.cuda.synchronize()
            guard.record(st, time.perf_counter() - tf, learned)
        if learned:
            a_S.attach(None, None)
        if keep:
            return x, st, (a_pp, a_S, M)
        M.close(); a_pp.close(); a_S.close()
        return x, st


def timed_steps(S, systems, cfg, net, steps, warmup):
    """Warm-up steps, then exactly `steps` timed ones between synchronisations.
    With a network, one LearnedGuard follows all of them (the first warm-up
    solve is the plain calibration solve)."""
    from paper_1902_00095_amd import solver
    guard = solver.LearnedGuard() if net is not None else None
    for i in range(warmup):
        S.run(systems[i % len(systems)], cfg, net, guard=guard)
    t0 = _sync_time()
    stats = []
    for i in range(steps):
        _, st = S.run(systems[i % len(systems)], cfg, net, guard=guard)
        stats.append(st)
    t1 = _sync_time()
    if guard is not None:
        stats[-1]["guard"] = guard.stats()
    return (t1 - t0) * 1e3 / steps, stats


def _summ(stats):
    import numpy as np
    its = [s["iters"] for s in stats]
    out = {"fgmres_iters_mean": round(float(np.mean(its)), 2), "fgmres_iters": its,
           "max_rel_true": max(s["rel_true"] for s in stats),
           "all_converged": all(s["converged"] for s in stats),
           "network_switched_off_in": sum(1 for s in stats if s["fallback_iter"] >= 0)}
    if "guard" in stats[-1]:
        out["guard"] = stats[-1]["guard"]
    return out


def _block_err(x, ref):
    import torch
    return [float(torch.linalg.vector_norm(x[b::2] - ref[b::2]) / torch.linalg.vector_norm(ref[b::2]))
            for b in (0, 1)]


# ---- V-cycle throughput -----------------------------------------------------------------------
def apply_numbers(S, system, cfg, net=None):
    """Preconditioner apply time and algorithmic GB/s of its two V-cycles on one
    Newton system (over the apply, and over the two cycles timed alone), and
    the finest-level Chebyshev step replayed back to back."""
    import torch
    _, _, (a_pp, a_S, M) = S.run(system, cfg, net, keep=True)
    if net is not None:
        a_S.attach(net, S.prob.grid)
    b = -S.G
    z = torch.empty_like(b)
    for _ in range(3):
        M.apply(b, z)
    nrep = 20
    t0 = _sync_time()
    for _ in range(nrep):
        M.apply(b, z)
    ms = (_sync_time() - t0) * 1e3 / nrep
    vb = a_pp.vcycle_bytes() + a_S.vcycle_bytes()
    # the two V-cycles alone, back to back, each on its field's right-hand
    # side with its FP64 interface (the apply above adds A_Tp z_p, the split
    # and the join of the interleaved vectors)
    bp, bT = b[0::2].contiguous(), b[1::2].contiguous()
    xp, xT = torch.empty_like(bp), torch.empty_like(bT)
    for _ in range(3):
        a_pp.vcycle(bp, xp)
        a_S.vcycle(bT, xT)
    t0 = _sync_time()
    for _ in range(nrep):
        a_pp.vcycle(bp, xp)
        a_S.vcycle(bT, xT)
    cyc_ms = (_sync_time() - t0) * 1e3 / nrep
    rep_ms, rep_bytes = a_S.time_fine_smoother(100)
    # the same sweep with the 256 MB last-level cache evicted before every
    # launch (a 1 GiB read pass), each launch timed alone
    flush = torch.zeros(1 << 27, dtype=torch.float64, device="cuda")
    fl_ms, _ = a_S.time_fine_smoother(20, flush=flush)
    del flush
    if net is not None:
        a_S.attach(None, None)
    out = {"apply_ms": round(ms, 4), "vcycle_pair_bytes": int(vb),
           "vcycle_pair_GBps": round(vb / (ms * 1e-3) / 1e9, 1),
           "vcycle_pair_frac_of_8TBps": round(vb / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
           "vcycles_alone_ms": round(cyc_ms, 4),
           "vcycles_alone_GBps": round(vb / (cyc_ms * 1e-3) / 1e9, 1),
           "vcycles_alone_frac_of_8TBps": round(vb / (cyc_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
           "fine_sweep_replay_us": round(rep_ms * 1e3, 3),
           "fine_sweep_replay_GBps": round(rep_bytes / (rep_ms * 1e-3) / 1e9, 1),
           "fine_sweep_llc_flushed_us": round(fl_ms * 1e3, 3),
           "fine_sweep_llc_flushed_GBps": round(rep_bytes / (fl_ms * 1e-3) / 1e9, 1),
           "levels": [a_pp.nlev, a_S.nlev]}
    M.close(); a_pp.close(); a_S.close()
    return out


# ---- HBM traffic record of the roofline kernel (rocprofv3 --pmc) ------------------------------
TRAFFIC_JSON = os.path.join(ROOT, "profiles", "traffic_k_cheb_step_dia_f32_256x256x64.json")
TRAFFIC_KERNEL = "k_cheb_step_dia<float, float, 7>"
TRAFFIC_SRC = "paper_1902_00095_amd/csrc/tp_vcycle.hip"
TRAFFIC_START = "// ---- DIA (stencil-level) kernels"
TRAFFIC_END = "// R consecutive rows per thread"
CALIB_BYTES = 32 * 1024 * 1024 * 8   # the calibration copy reads and writes this many bytes


def _kernel_text_hash():
    import hashlib
    text = open(os.path.join(ROOT, TRAFFIC_SRC)).read()
    a, b = text.find(TRAFFIC_START), text.find(TRAFFIC_END)
    return hashlib.sha256(text[a:b].encode()).hexdigest() if a >= 0 and b > a else ""


def write_traffic(fetch_db, write_db):
    """Per-dispatch counter means of the roofline kernel, each scaled by what the
    counter reads for the calibration copy (the run's largest dispatch)."""
    import sqlite3
    import statistics

    def load(path):
        # the calibration copy is the largest device-to-device copy dispatch
        # (the runtime's blit kernel) of the run
        cur = sqlite3.connect(path).cursor()
        vals, top = [], 0.0
        for name, v in cur.execute("select name, counter_value from pmc_events"):
            if "copyBuffer" in name:
                top = max(top, float(v))
            if TRAFFIC_KERNEL in name:
                vals.append(float(v))
        return vals, top
    vf, cf = load(fetch_db)
    vw, cw = load(write_db)
    if not vf or not vw:
        sys.exit(f"no dispatch of {TRAFFIC_KERNEL} in {fetch_db} / {write_db}")
    fs, ws = CALIB_BYTES / (cf * 1024), CALIB_BYTES / (cw * 1024)
    mf, mw = statistics.mean(vf), statistics.mean(vw)
    rec = dict(kernel=TRAFFIC_KERNEL, workload="256x256x64 mixed precision + learned (FP32 finest level)",
               dispatches=len(vf), fetch_kib=mf, write_kib=mw,
               calibration_fetch_kib=cf, calibration_write_kib=cw, fetch_scale=fs, write_scale=ws,
               traffic_bytes_per_launch=mf * 1024 * fs + mw * 1024 * ws, source=TRAFFIC_SRC,
               source_sha256=_kernel_text_hash(), source_start=TRAFFIC_START, source_end=TRAFFIC_END)
    with open(TRAFFIC_JSON, "w") as f:
        json.dump(rec, f, indent=1)
    print(json.dumps(rec))


KERNELS_MD = os.path.join(ROOT, "profiles", "kernels_256x256x64_mixed_learned.md")


def write_kernel_summary(db, bench_line, unprofiled=None):
    """Per-kernel summary of a rocprofv3 --kernel-trace database of
    `bench.py --steps 2 --warmup 1 --no-variants --no-cpu-baseline` (with
    the JSON line that run printed): dispatches, total and mean duration of
    the kernels that take most time, and the roofline kernel's mean beside
    the means measured with HIP events by that run and (`unprofiled`, the
    JSON line of a default run without the profiler) by an unprofiled run."""
    import re
    import sqlite3
    import statistics
    cur = sqlite3.connect(db).cursor()
    agg = {}
    for name, s, e in cur.execute("select name, start, end from kernels"):
        k = re.sub(r"\(.*", "", name).replace("void ", "")
        agg.setdefault(k, []).append((e - s) / 1e3)
    line = json.loads(open(bench_line).read().strip().splitlines()[-1])
    rf = line["roofline"]
    rk = [v for k, v in agg.items() if k.endswith(TRAFFIC_KERNEL)]
    rk = rk[0] if rk else []
    tot = sum(sum(v) for v in agg.values())
    out = ["# Kernel trace: 256x256x64, mixed precision + learned form (short bench run)", "",
           "Commands (repository root, one MI355X):", "", "```",
           "rocprofv3 --kernel-trace --stats -d gpurun_out/prof_bench -o run -- "
           "python3 -u bench.py --steps 2 --warmup 1 --no-variants --no-cpu-baseline > gpurun_out/prof_bench.json",
           "python3 bench.py --write-kernel-summary gpurun_out/prof_bench/run_results.db gpurun_out/prof_bench.json"
           + (f" {unprofiled}" if unprofiled else ""),
           "```", "",
           "The run trains the network, prepares the Newton systems, times the mixed + learned, FP64 and FP32 "
           "forms, stamps every launch of the roofline kernel with HIP events over two solves, and measures the "
           "preconditioner applies.  All kernels of the whole run are counted.", "",
           f"Roofline kernel `{TRAFFIC_KERNEL}`: rocprofv3 {len(rk)} dispatches, mean "
           f"{statistics.mean(rk) if rk else 0:.3f} us, median {statistics.median(rk) if rk else 0:.3f} us; "
           f"the run's HIP events: {rf['launches']} launches, mean {rf['mean_us']} us "
           f"({rf['bytes_per_launch']} algorithmic bytes per launch, {rf['achieved']} GB/s, frac {rf['frac']}).", ""]
    if unprofiled:
        ru = json.loads(open(unprofiled).read().strip().splitlines()[-1])["roofline"]
        out += [f"The default run without the profiler (`python3 bench.py`) measured {ru['launches']} launches "
                f"at a mean of {ru['mean_us']} us ({ru['achieved']} GB/s, frac {ru['frac']}), within "
                f"{100 * abs(ru['mean_us'] / statistics.mean(rk) - 1) if rk else 0:.1f}% of the profiler's "
                "kernel-trace mean; under the profiler the event pairs read longer, since the profiler's own "
                "handling of each dispatch falls between them.", ""]
    out += [f"Total kernel time {tot / 1e3:.1f} ms.", "",
            "| kernel | dispatches | total ms | mean us | share |", "|---|---|---|---|---|"]
    for k, v in sorted(agg.items(), key=lambda x: -sum(x[1]))[:40]:
        out.append(f"| `{k[:90]}` | {len(v)} | {sum(v) / 1e3:.2f} | {statistics.mean(v):.1f} | "
                   f"{100 * sum(v) / tot:.1f}% |")
    with open(KERNELS_MD, "w") as f:
        f.write("\n".join(out) + "\n")
    print(f"wrote {KERNELS_MD}")


def _traffic():
    if not os.path.exists(TRAFFIC_JSON):
        return None
    rec = json.load(open(TRAFFIC_JSON))
    if rec.get("source_sha256") == _kernel_text_hash() and rec.get("kernel") == TRAFFIC_KERNEL:
        return round(rec["traffic_bytes_per_launch"])
    return None


# ---- CPU oracle on one headline system --------------------------------------------------------
def _host_cpu():
    model = "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return model, os.cpu_count()


def cpu_baseline(S, system, plain_iters, cfg64, run20=None):
    """The oracle on one Newton system of the headline workload (see the module
    docstring); returns the cpu_baseline object with its parity checks.  With
    `run20` (the plain FP64 GPU run's stats over 20 time steps), the oracle's
    time per solve is also extrapolated to the systems of steps 1, 10 and 20:
    the measured assembly, setup and per-iteration times with that step's
    mean GPU iteration count per solve."""
    import dataclasses

    import numpy as np
    import torch

    import oracle
    from paper_1902_00095_amd import tpsolve as tps
    oracle.build(force=False)
    p = dataclasses.replace(S.prob, x_prev=system[2].cpu().numpy(), x_k=system[3].cpu().numpy())
    t0 = time.perf_counter()
    Jo = oracle.jacobian(p)
    bo = -oracle.residual(p)
    t_asm = time.perf_counter() - t0
    _progress(f"oracle assembly {t_asm:.1f} s")
    S.assemble(system)              # the GPU's own assembly of the same system
    g_err = float(np.abs(S.G.cpu().numpy() + bo).max() / np.abs(bo).max())
    j_err = max(float(np.abs(getattr(S.J, k).cpu().numpy() - getattr(Jo, k)).max() / np.abs(getattr(Jo, k)).max())
                for k in ("pp", "pT", "Tp", "TT", "S"))
    from paper_1902_00095_amd import solver
    prm = {w: solver.amg_params(cfg64, w) for w in ("pp", "S")}
    t0 = time.perf_counter()
    ao_pp = oracle.AMG(Jo.n, Jo.rowptr, Jo.col, Jo.pp, **prm["pp"].oracle_kwargs())
    ao_S = oracle.AMG(Jo.n, Jo.rowptr, Jo.col, Jo.S, **prm["S"].oracle_kwargs())
    t_setup = time.perf_counter() - t0
    _progress(f"oracle setups {t_setup:.1f} s")
    # the GPU hierarchies of the oracle's operators: every level's split and pattern
    Jd = tps.Jacobian.from_host(Jo.n, Jo.rowptr, Jo.col, Jo.pp, Jo.pT, Jo.Tp, Jo.TT, Jo.S)
    split_ok, levels = True, []
    for val, ho, w in ((Jd.pp, ao_pp, "pp"), (Jd.S, ao_S, "S")):
        hg = tps.AMG(Jd.rowptr, Jd.col, val, prm[w])
        levels.append(hg.nlev)
        split_ok &= hg.nlev == ho.nlev
        for l in range(min(hg.nlev, ho.nlev) - 1):
            Lg, Lo = hg.level(l), ho.level(l)
            split_ok &= bool(np.array_equal(Lg["cf"].cpu().numpy(), Lo["cf"]))
            for k in ("A_col", "P_col", "R_col"):
                split_ok &= bool(np.array_equal(Lg[k].cpu().numpy(), Lo[k]))
        hg.close()
    # GMRES: one-iteration runs (initial residual, one preconditioned Arnoldi
    # step, the closing true residual), the median of three
    t_it = []
    h1 = None
    for _ in range(3):
        t0 = time.perf_counter()
        _, io = oracle.gmres(Jo, ao_pp, ao_S, bo, rtol=RTOL, maxit=1)
        t_it.append(time.perf_counter() - t0)
        h1 = io["history"]
    t_iter = float(np.median(t_it))
    _progress(f"oracle GMRES iteration {t_iter:.1f} s")
    # the GPU's first residual estimate on the same operators
    a_pp, a_S, M = solver.setup(Jd, cfg64)
    _, stg = tps.fgmres_solve(Jd, M, torch.as_tensor(bo, device="cuda"), rtol=RTOL, maxit=1, history=True)
    M.close(); a_pp.close(); a_S.close()
    h_diff = float(abs(stg["history"][1] - h1[1]) / h1[1])
    model, ncpu = _host_cpu()
    per_solve_s = t_asm + t_setup + plain_iters * t_iter
    at_steps = None
    if run20 and run20.get("linear_per_step"):
        lps, nps = run20["linear_per_step"], run20["newton_per_step"]
        at_steps = {}
        for stp in (1, 10, 20):
            if stp <= len(lps) and nps[stp - 1] > 0:
                its = lps[stp - 1] / nps[stp - 1]
                at_steps[str(stp)] = {"gpu_fp64_iters_per_solve": round(its, 2),
                                      "oracle_ms_per_solve": round((t_asm + t_setup + its * t_iter) * 1e3, 1)}
    return {"value": round(per_solve_s * 1e3, 1), "unit": "ms/solve", "cores": 1, "kind": "oracle",
            "sample": (f"one Newton system of the headline workload (step {system[0] + 1}, Newton iteration "
                       f"{system[1]}): assembly {t_asm:.2f} s and both AMG setups {t_setup:.2f} s timed once, "
                       f"GMRES at {t_iter:.2f} s per iteration (median of 3 one-iteration runs) times the "
                       f"plain GPU path's {plain_iters} iterations; single-threaded FP64 C"),
            "assembly_s": round(t_asm, 3), "setup_s": round(t_setup, 3), "gmres_s_per_iteration": round(t_iter, 3),
            "gmres_iteration_runs_s": [round(t, 3) for t in t_it],
            "host_cpu_model": model, "host_cpu_count": ncpu,
            "extrapolated_to_steps_1_10_20_kappa_20": at_steps,
            "parity": {"G_rel_err": g_err, "jacobian_blocks_rel_err": j_err,
                       "hierarchy_splits_and_patterns_bit_exact": bool(split_ok), "levels": levels,
                       "first_residual_estimate_rel_diff": h_diff}}


# ---- the full 256x256x64 runs (20 steps, both conductivities) ---------------------------------
def c5_runs(net, kappa):
    """20 backward-Euler steps x <= 4 Newton iterations, every Newton iteration
    a coupled solve to rtol 1e-8: plain FP64, mixed + learned, and both with
    the numeric hierarchy refresh within each time step."""
    import dataclasses as dc

    from paper_1902_00095_amd import solver, synth
    prob = synth.make_problem("W5", kappa=kappa)
    cfg = solver.SolveConfig(rtol=RTOL)
    forms = [("fp64", cfg, None, solver.NewtonConfig(steps=20)),
             ("mixed_learned", dc.replace(cfg, storage=1), net, solver.NewtonConfig(steps=20)),
             ("fp64_numeric_reuse", cfg, None, solver.NewtonConfig(steps=20, reuse="numeric")),
             ("mixed_learned_numeric_reuse", dc.replace(cfg, storage=1), net,
              solver.NewtonConfig(steps=20, reuse="numeric"))]
    out = {}
    for key, c, nt, nc in forms:
        _, st = solver.simulate(prob, c, nc, net=nt)
        st.pop("step_lengths", None)
        out[key] = {k: (round(v, 3) if isinstance(v, float) else v) for k, v in st.items()}
        _progress(f"256x256x64 kappa {kappa} {key}: {st['solves']} solves, {st['total_s']:.1f} s")
    out["mixed_learned_vs_fp64_time"] = round(out["mixed_learned"]["total_s"] / out["fp64"]["total_s"], 3)
    return out


def smaller_workloads():
    """The 64x64x32 and 128x128x64 layered workloads (perturbed Newton state):
    FP64, FP32 and FP32 + BF16 off-diagonal hierarchies, solve time and V-cycle
    throughput; CPR on 64x64x32."""
    import dataclasses as dc

    from paper_1902_00095_amd import solver, synth
    out = {}
    for name in ("W2", "W3"):
        prob = synth.make_problem(name)
        S = Solves(prob)
        row = {}
        x64 = None
        for key, st_ in (("fp64", 0), ("fp32_hierarchy", 1), ("bf16_offdiag_hierarchy", 2)):
            cfg = solver.SolveConfig(rtol=RTOL, storage=st_)
            ms, stats = timed_steps(S, [None], cfg, None, 3, 1)
            x, st = S.run(None, cfg)
            r = dict(ms_per_solve=round(ms, 3), iters=st["iters"], rel_true=st["rel_true"])
            if x64 is None:
                x64 = x.clone()
            else:
                r["diff_vs_fp64_per_block"] = _block_err(x, x64)
            r.update(apply_numbers(S, None, cfg))
            row[key] = r
        if name == "W2":
            ms, _ = timed_steps(S, [None], solver.SolveConfig(rtol=RTOL, method="cpr"), None, 3, 1)
            row["cpr_ms_per_solve"] = round(ms, 3)
        g = prob.grid
        out[f"{g.nx}x{g.ny}x{g.nz}"] = row
        _progress(f"{name} variants done")
    return out


# ---- the paper's comparison studies (opt-in: --studies) --------------------------------------
def _solve_once(prob, cfg, reps=2):
    """Mean time of `reps` full solves (assembly, both setups, FGMRES) after a warm one."""
    S = Solves(prob)
    ms, stats = timed_steps(S, [None], cfg, None, reps, 1)
    st = stats[-1]
    return {"ms_per_solve": round(ms, 3), "iters": st["iters"], "rel_true": st["rel_true"],
            "converged": st["converged"]}


def _cpr_numbers(prob):
    """CPR's pieces on one assembled system: ILU(0) creation (level analysis
    on the host plus the numeric factorisation), refactorisation (numeric
    only, as a Newton iteration on the same pattern), one ILU solve, one
    preconditioner apply."""
    import torch

    from paper_1902_00095_amd import solver
    from paper_1902_00095_amd import tpsolve as tps
    S = Solves(prob)
    S.assemble(None)
    J, G = S.J, S.G
    t0 = _sync_time()
    F = tps.ILU0.jacobian(J)
    t1 = _sync_time()
    F.refactor(J)
    t2 = _sync_time()
    b = -G[: 2 * J.n].clone()
    x = torch.empty_like(b)
    F.solve(b, x)
    t3 = _sync_time()
    for _ in range(20):
        F.solve(b, x)
    t4 = _sync_time()
    a_pp = tps.AMG(J.rowptr, J.col, J.pp, solver.amg_params(solver.SolveConfig(), "pp"))
    M = tps.Precond.cpr(J, a_pp, F)
    z = torch.empty_like(b)
    for _ in range(3):
        M.apply(b, z)
    t5 = _sync_time()
    for _ in range(20):
        M.apply(b, z)
    t6 = _sync_time()
    inf = F.info()
    out = {"ilu_create_ms": round((t1 - t0) * 1e3, 3), "ilu_refactor_ms": round((t2 - t1) * 1e3, 3),
           "ilu_solve_ms": round((t4 - t3) * 1e3 / 20, 4), "apply_ms": round((t6 - t5) * 1e3 / 20, 4),
           "levels_lower_upper": [inf["levels_lower"], inf["levels_upper"]]}
    M.close(); a_pp.close(); F.close()
    return out


# the paper's figures for its problem-size cases (Section 4, tables isoH, isoW,
# isoHighW, anisoH and anisoW; PETSc with BoomerAMG, serial CPU; "> 200" as None),
# linear iterations per Newton iteration at N = 20, 40, 80, 160, 320
PAPER_CASES = {"CaseI": {"block": [2.57, 3.23, 2.86, 3.44, 3.71], "cpr": [3.4, 5.38, 9.09, 16.3, 30.7]},
               "CaseII": {"block": [2.43, 2.43, 2.86, 3.28, 3.71], "cpr": [3.71, 5.71, 9.86, 19.4, 37.4],
                          "block_S_ATT": [4.57, 5.0, 5.57, 6.29, 6.57],
                          "block_S_diag": [4.14, 4.43, 5.29, 5.86, 6.43]},
               "CaseIII": {"block": [3.67, 4.38, 4.7, 5.10, 5.52], "cpr": [4.71, 7.31, 13.1, 24.7, 50.6]},
               "CaseIV": {"block": [2.31, 2.67, 3.25, 3.67, 3.86], "cpr": [3.11, 4.56, 8.56, 15.8, 30.4]},
               "CaseV": {"block": [2.38, 3.27, 4.52, 4.68, 5.36], "cpr": [2.86, 3.6, 4.76, 7.0, 12.04],
                         "block_S_ATT": [9, 17.1, 24.1, 27.9, 31.6], "block_S_diag": [None] * 5}}


def paper_studies():
    """The paper's comparisons on this build: the three Schur approximations
    (64x64x32 layered), CPR against the block preconditioner (64x64x32 and
    128x128x64), the mesh-refinement study (2-D, N = 20 .. 640) and the
    problem-size Cases I-V (N = 20 .. 320, the paper's heavy oil, Newton with
    line search, FGMRES to the paper's 1e-5), each with the pressure
    hierarchy's extended+i interpolation (the default) and direct
    interpolation ("_direct")."""
    import dataclasses as dc

    from paper_1902_00095_amd import solver, synth
    from paper_1902_00095_amd import tpsolve as tps
    out = {}
    cfg = solver.SolveConfig(rtol=RTOL)
    direct = dict(interp_pp=0)
    w2 = synth.make_problem("W2")
    sch = {}
    for key in ("T", "ATT", "diag"):
        name = {"T": "S_T", "ATT": "A_TT", "diag": "S_diag"}[key]
        sch[name] = _solve_once(w2, dc.replace(cfg, schur=key, maxit=200), 1)
        sch[name + "_direct"] = _solve_once(w2, dc.replace(cfg, schur=key, maxit=200, **direct), 1)
    out["schur_approximations_64x64x32"] = dict(sch, note="FGMRES capped at 200 iterations")
    _progress("Schur approximations done")
    cpr = {}
    for name in ("W2", "W3"):
        pr = synth.make_problem(name)
        g = pr.grid
        row = {"block": _solve_once(pr, cfg), "cpr": _solve_once(pr, dc.replace(cfg, method="cpr")),
               "block_direct": _solve_once(pr, dc.replace(cfg, **direct)),
               "cpr_direct": _solve_once(pr, dc.replace(cfg, method="cpr", **direct))}
        row["cpr_pieces"] = _cpr_numbers(pr)
        cpr[f"{g.nx}x{g.ny}x{g.nz}"] = row
    out["cpr"] = dict(cpr, note="ms_per_solve includes assembly, the setups and a fresh ILU(0) (level analysis "
                                "included); a Newton loop refactorises instead (ilu_refactor_ms)")
    _progress("CPR done")
    ref = {}
    for N in (20, 40, 80, 160, 320, 640):
        g = synth.Grid(N, N, 1, 20.0 / N, 20.0 / N, 1.0)
        pr = synth.make_problem("R2", grid=g)
        row = {}
        for key, cr in (("block", dc.replace(cfg, maxit=400)), ("block_direct", dc.replace(cfg, maxit=400, **direct)),
                        ("cpr", dc.replace(cfg, method="cpr", maxit=400))):
            _, sr = solver.simulate(pr, cr, solver.NewtonConfig(steps=2))
            row[key] = {"linear_per_newton": round(sr["linear_per_newton"], 2), "newton_iters": sr["newton_iters"],
                        "ms_per_solve": round(sr["ms_per_solve"], 3), "unconverged_steps": sr["unconverged_steps"]}
        ref[f"{N}x{N}"] = row
    out["refinement_2d"] = dict(ref, note="N x N cells of a 20 m x 20 m x 1 m slab, k = 1e-13 m^2, injector "
                                "450 K and producer 1e-6 m^3/s at opposite corners, 2 steps of 1 day from a "
                                "uniform state; FGMRES capped at 400")
    _progress("refinement done")
    cases = {}
    for case in ("CaseI", "CaseII", "CaseIII", "CaseIV", "CaseV"):
        rows = {}
        for N in (20, 40, 80, 160, 320):
            g = synth.Grid(N, N, 1, 20.0 / N, 20.0 / N, 1.0)
            pc = synth.make_problem(case, grid=g, props=synth.Props(api=10.0))
            c5 = dc.replace(cfg, rtol=1e-5, maxit=400)
            forms = [("block", c5), ("block_direct", dc.replace(c5, **direct)),
                     ("cpr", dc.replace(c5, method="cpr"))]
            if case in ("CaseII", "CaseV"):
                forms += [("block_S_ATT", dc.replace(c5, schur="ATT")),
                          ("block_S_diag", dc.replace(c5, schur="diag"))]
            row = {}
            for key, cr in forms:
                try:
                    _, sr = solver.simulate(pc, cr, solver.NewtonConfig(steps=2, max_newton=20, line_search=True))
                except tps.TpError as e:
                    # a weak preconditioner can steer Newton out of the fluid laws' range
                    # (T below 0 F has no Bennison viscosity); the setup then reports it
                    row[key] = None
                    row[key + "_failed"] = str(e)[:120]
                    continue
                row[key] = round(sr["linear_per_newton"], 2)
                if sr["unconverged_steps"]:
                    row[key + "_unconverged_steps"] = sr["unconverged_steps"]
            rows[f"{N}x{N}"] = row
        cases[case] = {"this_build": rows, "paper": PAPER_CASES[case]}
        _progress(f"{case} done")
    out["paper_cases_2d"] = dict(cases, note="linear iterations per Newton iteration, 2 steps of 10 days "
                                 "(Case V: 12 hours), Bennison heavy oil (API 10), Newton with line search, "
                                 "FGMRES to rtol 1e-5 capped at 400")
    return out


SETUP_REPS = 4
SETUP_NAMES = {"pp": "pressure (A_pp, extended+i interpolation)", "S": "Schur (S~_T, Petrov-Galerkin)"}


def setup_study(which):
    """One hierarchy's AMG setup ("pp" or "S") on the first Newton system of
    the 256x256x64 workload, with the timed form's parameters (FP32 storage):
    SETUP_REPS setups one after another, the first a warm-up; prints one JSON
    line with their wall times (for a kernel trace of the setup alone)."""
    import dataclasses as dc
    from paper_1902_00095_amd import solver, synth
    from paper_1902_00095_amd import tpsolve as tps
    tps.init(0)
    prob = synth.make_problem("W5")
    J, _ = solver.assemble(prob, solver.to_device(prob))
    prm = solver.amg_params(dc.replace(solver.SolveConfig(rtol=RTOL), storage=1), which)
    val = J.pp if which == "pp" else J.S
    ms, rows = [], []
    for _ in range(SETUP_REPS):
        t0 = _sync_time()
        h = tps.AMG(J.rowptr, J.col, val, prm)
        ms.append(round((_sync_time() - t0) * 1e3, 2))
        rows = [h.level_sizes(l)[0] for l in range(h.nlev)]
        h.close()
    print(json.dumps({"setup_study": which, "setups": SETUP_REPS, "setup_ms": ms, "level_rows": rows}),
          flush=True)


def write_setup_summary(db, study_json, out_md):
    """Per-kernel summary of a rocprofv3 --kernel-trace database of
    `bench.py --setup-study WHICH` (with the JSON line it printed): the
    library's setup kernels (the assembly's left out), per setup, averaged
    over the run's setups."""
    import re
    import sqlite3
    line = json.loads(open(study_json).read().strip().splitlines()[-1])
    which, reps = line["setup_study"], line["setups"]
    agg = {}
    for name, s, e in sqlite3.connect(db).cursor().execute("select name, start, end from kernels"):
        k = re.sub(r"\(.*", "", name).replace("void ", "")
        if k.startswith("tp::") and "assemble" not in k:
            agg.setdefault(k, []).append((e - s) / 1e3)
    tot = sum(sum(v) for v in agg.values()) / reps / 1e3
    tag = "pressure" if which == "pp" else "schur"
    out = [f"# Kernel trace: one {SETUP_NAMES[which]} hierarchy setup, 256x256x64", "",
           "Commands (repository root, one MI355X):", "", "```",
           f"rocprofv3 --kernel-trace --stats -d gpurun_out/prof_setup_{which} -o run -- "
           f"python3 -u bench.py --setup-study {which} > gpurun_out/setup_{which}.json",
           f"python3 bench.py --write-setup-summary gpurun_out/prof_setup_{which}/run_results.db "
           f"gpurun_out/setup_{which}.json profiles/setup_{tag}_256x256x64.md", "```", "",
           f"{reps} setups of the hierarchy on the workload's first Newton system (FP32 storage, the timed "
           "form's parameters), one after another, the first a warm-up; the table averages the library's "
           "kernels over all of them (the assembly's kernels left out).", "",
           f"Wall time per setup under the profiler: {', '.join(f'{v:.1f}' for v in line['setup_ms'])} ms; "
           f"level sizes {line['level_rows']}.", "",
           f"Kernel time per setup {tot:.2f} ms.", "",
           "| kernel | dispatches per setup | ms per setup | mean us | share |", "|---|---|---|---|---|"]
    for k, v in sorted(agg.items(), key=lambda kv: -sum(kv[1]))[:30]:
        t = sum(v) / reps / 1e3
        out.append(f"| `{k}` | {len(v) / reps:g} | {t:.3f} | {sum(v) / len(v):.1f} | {100 * t / tot:.1f}% |")
    open(out_md, "w").write("\n".join(out) + "\n")
    print(f"wrote {out_md}")


APPLY_REPS = 20
APPLY_FORMS = {"fp32": "FP32 hierarchies", "fp32_learned": "FP32 hierarchies with the network as the Schur "
               "finest-level post-smoother", "fp64": "FP64 hierarchies"}
PHASE_GAP_MS = 100  # host pause between the set-up and the timed applies (found again in the trace)


def apply_study(form):
    """The block preconditioner of the timed form on the first Newton system
    of the 256x256x64 workload: set up, then (after a PHASE_GAP_MS host pause
    that marks the phase in a kernel trace) 3 + APPLY_REPS applies through
    precond_apply, the last APPLY_REPS timed; prints one JSON line.  The
    learned form attaches an untrained network of the trained one's shape
    (the kernels' work does not depend on the weights)."""
    import torch
    from paper_1902_00095_amd import learned, solver, synth
    from paper_1902_00095_amd import tpsolve as tps
    tps.init(0)
    prob = synth.make_problem("W5")
    J, G = solver.assemble(prob, solver.to_device(prob))
    a_pp, a_S, M = solver.setup(J, solver.SolveConfig(rtol=RTOL, storage=0 if form == "fp64" else 1))
    net = None
    if form == "fp32_learned":
        net = tps.Net(learned.init_params(3))
        a_S.attach(net, prob.grid)
    b = -G
    z = torch.empty_like(b)
    torch.cuda.synchronize()
    time.sleep(PHASE_GAP_MS / 1e3)
    for _ in range(3):
        M.apply(b, z)
    t0 = _sync_time()
    for _ in range(APPLY_REPS):
        M.apply(b, z)
    ms = (_sync_time() - t0) * 1e3 / APPLY_REPS
    print(json.dumps({"apply_study": form, "applies": 3 + APPLY_REPS, "apply_ms": round(ms, 4),
                      "levels": [a_pp.nlev, a_S.nlev]}), flush=True)
    if net is not None:
        a_S.attach(None, None)
        net.close()
    M.close(); a_pp.close(); a_S.close()


def write_apply_summary(db, study_json, out_md):
    """Per-kernel summary of a rocprofv3 --kernel-trace database of
    `bench.py --apply-study FORM`: the kernels after the run's last pause of
    more than PHASE_GAP_MS / 2 (the applies), per apply."""
    import re
    import sqlite3
    line = json.loads(open(study_json).read().strip().splitlines()[-1])
    form, reps = line["apply_study"], line["applies"]
    ks = sorted(sqlite3.connect(db).cursor().execute("select start, end, name from kernels"))
    cut = 0
    for j in range(1, len(ks)):
        if ks[j][0] - ks[j - 1][1] > PHASE_GAP_MS / 2 * 1e6:
            cut = j
    agg = {}
    for s0, e0, name in ks[cut:]:
        k = re.sub(r"\(.*", "", name).replace("void ", "")
        agg.setdefault(k, []).append((e0 - s0) / 1e3)
    tot = sum(sum(v) for v in agg.values()) / reps
    span = (ks[-1][1] - ks[cut][0]) / 1e3 / reps
    out = [f"# Kernel trace: the preconditioner apply, {APPLY_FORMS[form]}, 256x256x64", "",
           "Commands (repository root, one MI355X):", "", "```",
           f"rocprofv3 --kernel-trace --stats -d gpurun_out/prof_apply_{form} -o run -- "
           f"python3 -u bench.py --apply-study {form} > gpurun_out/apply_{form}.json",
           f"python3 bench.py --write-apply-summary gpurun_out/prof_apply_{form}/run_results.db "
           f"gpurun_out/apply_{form}.json profiles/apply_{form}_256x256x64.md", "```", "",
           f"{reps} applies (`precond_apply`, interleaved vectors, the apply replayed from its HIP graph) of the "
           "block preconditioner on the workload's first Newton system; the kernels after the pause that "
           "follows the set-up, averaged per apply."
           + (" The network is an untrained one of the trained network's shape (the kernels' work does not "
              "depend on its weights)." if form == "fp32_learned" else ""), "",
           f"Apply time measured by the run (host clock over {APPLY_REPS} applies): {line['apply_ms']:.3f} ms; "
           f"under the profiler, kernel time {tot / 1e3:.3f} ms and span {span / 1e3:.3f} ms per apply; "
           f"levels {line['levels']}.", "",
           "| kernel | dispatches per apply | us per apply | mean us | share |", "|---|---|---|---|---|"]
    for k, v in sorted(agg.items(), key=lambda kv: -sum(kv[1]))[:30]:
        t = sum(v) / reps
        out.append(f"| `{k}` | {len(v) / reps:g} | {t:.1f} | {sum(v) / len(v):.1f} | {100 * t / tot:.1f}% |")
    open(out_md, "w").write("\n".join(out) + "\n")
    print(f"wrote {out_md}")


COUNTER_SETS = {  # tag: kernel, the run profiled, what the kernel is, summary file
    "cnn": ("k_cnn_fused<float, 1>", "--apply-study fp32_learned",
            "fused network, the learned post-smoother, in the learned apply", "pmc_k_cnn_fused_256x256x64.md"),
    "spgemm": ("k_spgemm_short<64, 256>", "--setup-study pp",
               "short-row SpGEMM with 256 product slots, in the pressure hierarchy's setup",
               "pmc_k_spgemm_short_256x256x64.md"),
}
COUNTER_PASSES = ("SQ_WAVES SQ_WAVE_CYCLES SQ_BUSY_CYCLES SQ_WAIT_ANY SQ_WAIT_INST_ANY SQ_ACTIVE_INST_ANY "
              "SQ_ACTIVE_INST_LDS SQ_LDS_BANK_CONFLICT GRBM_GUI_ACTIVE",
              "SQ_INSTS_VALU SQ_ACTIVE_INST_VALU SQ_INSTS_MFMA SQ_VALU_MFMA_BUSY_CYCLES SQ_INSTS_LDS "
              "SQ_WAIT_INST_LDS SQ_INSTS_SALU SQ_INSTS_SMEM")


def _pmc_means(db, kernel):
    """Mean per dispatch of every counter a rocprofv3 --pmc database holds
    for the kernels whose name contains `kernel` (a dispatch's rows, one per
    hardware instance, summed first)."""
    import sqlite3
    cur = sqlite3.connect(db).cursor()
    acc = {}
    for d, name, cn, v in cur.execute("select dispatch_id, name, counter_name, counter_value from pmc_events"):
        if kernel in name:
            per = acc.setdefault(cn, {})
            per[d] = per.get(d, 0.0) + float(v)
    return ({k: sum(v.values()) / len(v) for k, v in acc.items()},
            max((len(v) for v in acc.values()), default=0))


def write_counters(tag, db_a, db_b, out_md):
    """Counter summary of one kernel (COUNTER_SETS[tag]) from two rocprofv3
    --pmc passes (COUNTER_PASSES) of the run that COUNTER_SETS names."""
    kernel, run, what, fname = COUNTER_SETS[tag]
    ma, na = _pmc_means(db_a, kernel)
    mb, nb = _pmc_means(db_b, kernel)
    m = {**ma, **mb}
    waves = m["SQ_WAVES"]
    out = [f"# Counters: {kernel} ({what}), 256x256x64", "",
           "Commands (repository root, one MI355X; each counter pass its own run, then the summary):", "", "```"]
    for j, c in enumerate(COUNTER_PASSES):
        out.append(f"timeout -s KILL 120 rocprofv3 --pmc {c} -d gpurun_out/pmc_{tag}_{j} -o run -- "
                   f"python3 -u bench.py {run}")
    out += [f"python3 bench.py --write-counters {tag} gpurun_out/pmc_{tag}_0/run_results.db "
            f"gpurun_out/pmc_{tag}_1/run_results.db profiles/{fname}", "```", "",
            f"Means per dispatch over {na} and {nb} dispatches (a dispatch's rows, one per "
            "hardware instance, summed). SQ cycle counters are summed over the chip's wavefronts "
            "(wave-cycles, in the counters' own units); the shares below divide them by SQ_WAVE_CYCLES.", "",
            "| counter | mean per dispatch |", "|---|---|"]
    out += [f"| {k} | {v:.6g} |" for k, v in sorted(m.items())]
    wc = m["SQ_WAVE_CYCLES"]
    out += ["", "| derived | value |", "|---|---|",
            f"| wavefronts per dispatch | {waves:.0f} |",
            f"| VALU instructions per wavefront | {m['SQ_INSTS_VALU'] / waves:.0f} |",
            f"| MFMA instructions per wavefront | {m['SQ_INSTS_MFMA'] / waves:.0f} |",
            f"| LDS instructions per wavefront | {m['SQ_INSTS_LDS'] / waves:.0f} |",
            f"| scalar instructions per wavefront | {m['SQ_INSTS_SALU'] / waves:.0f} |",
            f"| share of wave-cycles issuing (SQ_ACTIVE_INST_ANY) | {m['SQ_ACTIVE_INST_ANY'] / wc:.2f} |",
            f"| share waiting on memory counters (SQ_WAIT_ANY) | {m['SQ_WAIT_ANY'] / wc:.2f} |",
            f"| share waiting to issue (SQ_WAIT_INST_ANY) | {m['SQ_WAIT_INST_ANY'] / wc:.2f} |",
            f"| LDS bank-conflict cycles / active LDS cycles | "
            f"{m['SQ_LDS_BANK_CONFLICT'] / max(m['SQ_ACTIVE_INST_LDS'], 1):.2f} |"]
    open(out_md, "w").write("\n".join(out) + "\n")
    print(f"wrote {out_md}")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-variants", action="store_true")
    ap.add_argument("--studies", action="store_true",
                    help="also run the paper's comparison studies (Schur approximations, CPR, mesh "
                         "refinement, Cases I-V: several minutes)")
    ap.add_argument("--quick", action="store_true",
                    help="two solves of the timed form plus the calibration copy (for counter runs)")
    ap.add_argument("--write-traffic", nargs=2, metavar=("FETCH_DB", "WRITE_DB"),
                    help="write the roofline kernel's traffic record from two rocprofv3 --pmc databases and exit")
    ap.add_argument("--write-kernel-summary", nargs="+", metavar="PATH",
                    help="TRACE_DB BENCH_JSON [UNPROFILED_JSON]: write the kernel-trace summary of a short "
                         "bench run and exit")
    ap.add_argument("--setup-study", choices=("pp", "S"),
                    help="time one hierarchy's AMG setup on the 256x256x64 workload (for a kernel trace) and exit")
    ap.add_argument("--write-setup-summary", nargs=3, metavar=("TRACE_DB", "STUDY_JSON", "OUT_MD"),
                    help="write the kernel-trace summary of a --setup-study run and exit")
    ap.add_argument("--apply-study", choices=tuple(APPLY_FORMS),
                    help="time the preconditioner apply of one form on the 256x256x64 workload (for a kernel "
                         "trace) and exit")
    ap.add_argument("--write-apply-summary", nargs=3, metavar=("TRACE_DB", "STUDY_JSON", "OUT_MD"),
                    help="write the kernel-trace summary of an --apply-study run and exit")
    ap.add_argument("--write-counters", nargs=4, metavar=("TAG", "PASS0_DB", "PASS1_DB", "OUT_MD"),
                    help="write a kernel's counter summary (TAG: " + ", ".join(COUNTER_SETS)
                         + ") from two --pmc runs and exit")
    args = ap.parse_args()
    if args.write_counters:
        write_counters(*args.write_counters)
        return
    if args.apply_study:
        apply_study(args.apply_study)
        return
    if args.write_apply_summary:
        write_apply_summary(*args.write_apply_summary)
        return
    if args.setup_study:
        setup_study(args.setup_study)
        return
    if args.write_setup_summary:
        write_setup_summary(*args.write_setup_summary)
        return
    if args.write_traffic:
        write_traffic(*args.write_traffic)
        return
    if args.write_kernel_summary:
        write_kernel_summary(*args.write_kernel_summary)
        return
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only: --gpus must be 1 "
                                   "(the multi-GPU sharding is a design, not built)"}))
        sys.exit(2)

    import dataclasses as dc

    import torch

    from paper_1902_00095_amd import solver, synth
    from paper_1902_00095_amd import tpsolve as tps

    tps.init(0)
    prob = synth.make_problem("W5")
    S = Solves(prob)
    net, train_rec = trained_network(quick=args.quick)
    _progress(f"network trained ({train_rec['seconds']} s)")
    systems = newton_systems(prob, 1 if args.quick else 2)
    _progress(f"{len(systems)} Newton systems prepared")
    cfg64 = solver.SolveConfig(rtol=RTOL)
    cfg_ml = dc.replace(cfg64, storage=1)

    if args.quick:
        for s in systems[:2]:
            S.run(s, cfg_ml, net)
        src = torch.ones(32 * 1024 * 1024, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"quick": True, "calibration_copy_bytes": 2 * src.numel() * 8}), flush=True)
        return

    # the metric: mixed precision + learned, then plain FP64 on the same systems
    ms_ml, st_ml = timed_steps(S, systems, cfg_ml, net, args.steps, args.warmup)
    _progress(f"mixed + learned: {ms_ml:.1f} ms/solve")
    ms_64, st_64 = timed_steps(S, systems, cfg64, None, args.steps, args.warmup)
    _progress(f"plain FP64: {ms_64:.1f} ms/solve")
    nsys = min(args.steps, len(systems))
    ms_32, st_32 = timed_steps(S, systems, cfg_ml, None, nsys, 1)
    _progress(f"FP32 hierarchy alone: {ms_32:.1f} ms/solve")
    # equal accuracy: both forms' solutions of the last system, per block
    x_ml, _ = S.run(systems[-1], cfg_ml, net)
    x_ml = x_ml.clone()
    x_64, _ = S.run(systems[-1], cfg64)
    diff = _block_err(x_ml, x_64)

    # phase breakdown of one mixed + learned solve
    S.dev["x_prev"], S.dev["x_k"] = systems[-1][2], systems[-1][3]
    t_a = _sync_time()
    S.J, S.G = solver.assemble(prob, S.dev, S.J, S.G)
    t_b = _sync_time()
    a_pp, a_S, M = solver.setup(S.J, cfg_ml)
    t_c = _sync_time()
    a_S.attach(net, prob.grid)
    _, st = tps.fgmres_solve(S.J, M, -S.G, rtol=RTOL)
    t_d = _sync_time()
    a_S.attach(None, None)
    M.close(); a_pp.close(); a_S.close()
    phases = {"assemble_ms": round((t_b - t_a) * 1e3, 3), "setups_ms": round((t_c - t_b) * 1e3, 3),
              "fgmres_ms": round((t_d - t_c) * 1e3, 3)}

    # roofline: the Chebyshev step kernel's launches carry HIP event pairs
    tps.timer_enable(True)
    for s in systems[:2]:
        S.run(s, cfg_ml, net)
    torch.cuda.synchronize()
    launches, kms, kbytes = tps.timer_read()
    tps.timer_enable(False)
    mean_us = kms / max(launches, 1) * 1e3
    bpl = kbytes / max(launches, 1)
    achieved = bpl / (mean_us * 1e-6) / 1e9 if launches else 0.0

    # V-cycle GB/s (the metric's second half), both forms
    vc = {"mixed_learned": apply_numbers(S, systems[-1], cfg_ml, net),
          "fp32_hierarchy": apply_numbers(S, systems[-1], cfg_ml),
          "fp64": apply_numbers(S, systems[-1], cfg64)}
    _progress("V-cycle throughput measured")

    variants = {}
    if args.studies:
        variants["studies"] = paper_studies()
    if not args.no_variants:
        variants["256x256x64_20_steps_kappa_20"] = c5_runs(net, 20.0)
        variants["256x256x64_20_steps_kappa_0.5"] = c5_runs(net, 0.5)
        variants.update(smaller_workloads())

    # calibration copy of known size (for PMC byte counters): 256 MiB
    src = torch.ones(32 * 1024 * 1024, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    del src, dst

    sm, s64 = _summ(st_ml), _summ(st_64)
    line = {
        "metric": "time-to-rtol 1e-8 per coupled P-T solve, mixed+learned vs FP64; V-cycle GB/s",
        "value": round(ms_ml, 3),
        "unit": "ms/solve",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_ml, 3),
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64 outer / f32 hierarchy / bf16 network",
        "data": "synthetic",
        "config": {"workload": HEADLINE, "form": "mixed precision + learned post-smoother",
                   "unknowns": 2 * prob.grid.n, "rtol": RTOL, "systems": len(systems),
                   "mixed_learned": sm, "phases_ms": phases,
                   "fp64_ms_per_solve": round(ms_64, 3), "fp64": s64,
                   "fp32_hierarchy_ms_per_solve": round(ms_32, 3), "fp32_hierarchy": _summ(st_32),
                   "mixed_learned_over_fp64_time": round(ms_ml / ms_64, 4),
                   "solution_diff_mixed_learned_vs_fp64_per_block": diff,
                   "vcycle": vc, "training": train_rec},
        "variants": variants,
        "roofline": {"bound": "hbm",
                     "kernel": "k_cheb_step_dia<float,float,7> (finest-level Chebyshev step, FP32, 7 diagonals)",
                     "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": _traffic(),
                     "bytes_per_launch": round(bpl), "mean_us": round(mean_us, 3), "launches": launches,
                     "timing": "HIP event pair stamped by every launch of the kernel in two solves of the "
                               "timed form (both hierarchies' finest levels), on the solve stream",
                     # one sweep's working set (~218 MB) fits the 256 MB last-level cache, so
                     # consecutive sweeps of a level are partly served from it; the same kernel
                     # with that cache evicted before each launch:
                     "llc_evicted": {"mean_us": vc["fp32_hierarchy"]["fine_sweep_llc_flushed_us"],
                                     "achieved": vc["fp32_hierarchy"]["fine_sweep_llc_flushed_GBps"],
                                     "frac": round(vc["fp32_hierarchy"]["fine_sweep_llc_flushed_GBps"]
                                                   / HBM_PEAK_GBS, 4)}},
    }
    if not (sm["all_converged"] and s64["all_converged"]):
        line["error"] = "a timed solve did not converge"
    if not args.no_cpu_baseline:
        _progress("CPU oracle sample started")
        run20 = variants.get("256x256x64_20_steps_kappa_20", {}).get("fp64")
        line["cpu_baseline"] = cpu_baseline(S, systems[min(3, len(systems) - 1)],
                                            round(s64["fgmres_iters_mean"]), cfg64, run20)
    net.close()
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
