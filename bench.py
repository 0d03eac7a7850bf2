"""Benchmark of the MI355X HPR-LP solver (one GPU).

Default workload: the batched solve, 256 independent LPs from the tiny-LP generator
(m_i ~ U{1k..50k}, n_i = 2 m_i, 8-30 nonzeros per row; 6.5M rows, 13.1M columns, 124M
nonzeros in all) packed block-diagonally, plain FP64, check_every = 100.  It is the largest
workload that fits one GPU.

One step = one chunk of the hot path: 100 iterations of Algorithm 2 for every instance
(column pass = x-step over A^T, row pass = y-step over A), with the check passes of the
chunk's first and last iteration, the restart / SigmaUpdate / termination decisions of every
instance and the restart copies: one launch of the captured chunk graph through the C ABI
(hprlp_step).  The inputs are resident in HBM: generation, preprocessing, schedule
autotuning and upload happen in create; the power method runs in hprlp_begin, before the
warm-up steps (the paper counts the power method in the solve time and excludes
preprocessing, Section 4.1; the time-to-tolerance fields below follow that convention).

value = instance-iterations per second over the K timed steps (every instance is still
iterating then).  In the same run, after the timed steps:
  * time_to_tol: one solve from the origin capped at --ttt-cap seconds; instances solved to
    relative KKT 1e-8 and the time at which each was solved (power method included);
  * compare: the same solve in FP32 -> FP64 mixed precision, and the single-LP FP64 solver
    run on the instances one after another, under the same cap;
  * roofline: algorithmic bytes of the dominant pass kernel / its mean launch duration, from
    HIP event nodes inside the chunk graphs of the timed steps;
  * cpu_baseline: the oracle (plain FP64 C) on a sample of instances, on all host cores
    (one instance per core) and on one core, in instance-iterations per second.
The optional legs run only while the whole run stays inside --wall-budget seconds; the one
JSON line is printed at the end.

--config selects a single-LP workload instead (then one step = one solve capped at
--time-limit; see run_single): zipf1m, zipf4m, transport10m, qap40, ot4m, tiny.
--ablation runs the four steps of the paper's ablation (Section 4.2, Fig. 1) on the first
64 batch256 instances.
"""
import argparse
import json
import os
import sys
import time

T_PROC0 = time.perf_counter()
ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0
METRIC = "time to rel. KKT 1e-8 + SpMV HBM GB/s; FP32→FP64 & batched vs plain FP64"
BOX_CPU_SHARE = 16  # host threads one GPU's share of the box may use


def log(msg):
    print(f"[bench {time.perf_counter() - T_PROC0:6.1f}s] {msg}", file=sys.stderr, flush=True)


def pass_bytes(m, n, nnz, s_val, s_vec):
    """Algorithmic HBM bytes of one launch of each pass (values + int32 indices + int32 row
    pointers, epilogue vectors read/written once, the gathered vector read once)."""
    col = nnz * (s_val + 4) + 4 * (n + 1) + 6 * n * s_vec + m * s_vec
    row = nnz * (s_val + 4) + 4 * (m + 1) + 4 * m * s_vec + n * s_vec
    return col, row


def read_traffic(kind, workload):
    """HBM traffic per launch from the committed rocprofv3 PMC summary, if it was taken on
    the current kernel source (else None)."""
    import hashlib
    import re
    path = os.path.join(ROOT, "profiles", f"pmc_{workload}.md")
    if not os.path.exists(path):
        return None
    text = open(path).read()
    src = open(os.path.join(ROOT, "paper_2408_12179_amd", "csrc", "kernels.hip"), "rb").read()
    sha = hashlib.sha256(src).hexdigest()[:16]
    msha = re.search(r"kernels\.hip sha256\[:16\]: ([0-9a-f]+)", text)
    if not msha or msha.group(1) != sha:
        return None
    mt = re.search(rf"^{kind}_bytes_per_launch: ([0-9.e+]+)", text, re.M)
    return float(mt.group(1)) if mt else None


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def host_threads():
    return max(1, min(os.cpu_count() or 1, BOX_CPU_SHARE))


# ------------------------------------------------------------------------ CPU baselines

def cpu_baseline_batched(lp, n_sample, sample_iters, deadline):
    """The oracle (one thread per instance) on n_sample instances spread over the batch,
    run concurrently on all host cores, then the smallest few alone on one core.  Each run
    does sample_iters iterations (lambda from a 50-iteration power method; preconditioning
    excluded).  Its cost per nonzero-iteration gives the rate at which it would run
    iterations of the whole batch, in instance-iterations per second."""
    import numpy as np
    from concurrent.futures import ThreadPoolExecutor
    import oracle
    n_inst = len(lp.inst_m1)
    nnz_i = np.diff(lp.rowptr[lp.inst_row_off]).astype(float)
    idx = [int(i) for i in np.linspace(0, n_inst - 1, n_sample).astype(int)]
    insts = {i: lp.instance(i) for i in idx}

    def run(i):
        r = oracle.solve(insts[i], max_iter=sample_iters, power_max_iter=50, power_tol=0.0,
                         check_every=100)
        return i, r.iters, r.t_solve - r.t_power

    threads = host_threads()
    t0 = time.perf_counter()
    with ThreadPoolExecutor(max_workers=threads) as ex:
        res = list(ex.map(run, idx))
    wall = time.perf_counter() - t0
    # aggregate nonzero-iterations per second with all threads busy
    agg = sum(nnz_i[i] * it / t for i, it, t in res)
    rate_all = agg / nnz_i.sum() * n_inst  # instance-iterations/s of the whole batch
    out = {"value": rate_all, "unit": "instance-iterations/s", "cores": threads,
           "kind": "oracle",
           "sample": f"{len(idx)} instances spread over the batch ({list(idx)}), "
                     f"{sample_iters} HPR-LP iterations each, one instance per host thread on "
                     f"{threads} threads concurrently ({wall:.1f} s wall incl. their "
                     f"preconditioning and a 50-iteration power method); iteration cost per "
                     f"nonzero applied to the whole batch",
           "host_cpu": cpu_model(), "os_cpu_count": os.cpu_count()}
    # one core: the 3 smallest sampled instances, one after another
    small = sorted(idx, key=lambda i: nnz_i[i])[:3]
    if time.perf_counter() < deadline:
        res1 = [run(i) for i in small]
        per_nnz = sum(t for _, _, t in res1) / sum(nnz_i[i] * it for i, it, _ in res1)
        out["single_core_value"] = n_inst / (per_nnz * nnz_i.sum())
        out["single_core_sample"] = (f"instances {small}, {sample_iters} iterations each, "
                                     f"one after another on one thread")
    return out


def cpu_baseline_single(lp, gpu_iters, gpu_power_iters, sample_iters=300, sample_power=60):
    """The oracle timed on a bounded sample of the same LP: sample_power power iterations and
    sample_iters HPR-LP iterations, extrapolated to the GPU run's counts; once on one thread
    and once with the OpenMP build on all host threads (bitwise the same arithmetic)."""
    import oracle
    out = None
    for threads in (1, host_threads()):
        t0 = time.perf_counter()
        r = oracle.solve(lp, max_iter=sample_iters, power_max_iter=sample_power, power_tol=0.0,
                         threads=threads)
        wall = time.perf_counter() - t0
        it_rate = r.iters / max(r.t_solve - r.t_power, 1e-9)
        pw_rate = r.power_iters / max(r.t_power, 1e-9)
        est = gpu_power_iters / pw_rate + gpu_iters / it_rate
        d = {"value": est, "unit": "s", "cores": threads, "kind": "oracle",
             "sample": f"{r.power_iters} power iterations + {r.iters} HPR-LP iterations of "
                       f"the same LP on {threads} host thread(s) ({wall:.1f} s wall incl. its "
                       f"preconditioning), extrapolated to the GPU run's {gpu_power_iters} "
                       f"power + {gpu_iters} iterations",
             "oracle_iters_per_s": it_rate}
        if out is None:
            out = d
        else:
            out = dict(d, single_core_value=out["value"],
                       single_core_iters_per_s=out["oracle_iters_per_s"])
    out["host_cpu"] = cpu_model()
    out["os_cpu_count"] = os.cpu_count()
    return out


# ------------------------------------------------------------------------ batched default

def ttt_fields(solver, lp, t_create):
    """Per-instance outcome of the last solve: solved count and times to tolerance."""
    import numpy as np
    n_inst = len(lp.inst_m1)
    per = [solver.stats_instance(i) for i in range(n_inst)]
    ok = [p["status"] == "OPTIMAL" for p in per]
    times = sorted(p["t_solve_ms"] / 1e3 for p, o in zip(per, ok) if o)
    errs = []
    for i, p in enumerate(per):
        if ok[i]:
            inst = lp.instance(i)
            if inst.cert is not None:
                errs.append(abs(p["pobj"] - inst.cert.obj) / (1 + abs(inst.cert.obj)))
    st = solver.stats()
    return {
        "instances": n_inst, "solved": int(sum(ok)),
        "time_to_tol_s_sorted": [round(t, 4) for t in times],
        "time_to_tol_s_p50_of_solved": float(np.median(times)) if times else None,
        "time_all_solved_s": times[-1] if all(ok) else None,
        "batch_iters": int(st["iters"]), "power_iters": int(st["power_iters"]),
        "t_power_s": st["t_power_ms"] / 1e3, "t_solve_s": st["t_solve_ms"] / 1e3,
        "iters_fp32": int(st["iters_fp32"]), "compactions": int(st["n_compactions"]),
        "create_s": t_create,
        "inst_iters": [int(p["iters"]) for p in per],
        "inst_solved": [bool(o) for o in ok],
        "max_obj_rel_err_vs_certificate": max(errs) if errs else None,
    }


def run_batched(args):
    import numpy as np
    import torch
    import lpgen
    from paper_2408_12179_amd import hprlp

    deadline = T_PROC0 + args.wall_budget
    ce = 100
    t0 = time.perf_counter()
    lp = lpgen.make("batch256")
    n_inst = len(lp.inst_m1)
    log(f"batch256: {n_inst} instances, m={lp.m} n={lp.n} nnz={lp.nnz} generated in "
        f"{time.perf_counter() - t0:.1f}s")
    P = {"mixed": hprlp.MIXED, "fp64a32": hprlp.FP64_A32}.get(args.precision, hprlp.FP64)
    opts = dict(check_every=ce, tol=args.tol, time_limit=args.ttt_cap, precision=P,
                profile=args.profile_every, autotune=0 if args.no_autotune else 1,
                tile_order=args.tile_order, bundle_rows=args.bundle_rows)
    t0 = time.perf_counter()
    solver = hprlp.Solver(lp, batched=True, **opts)
    t_create = time.perf_counter() - t0
    sched = {"A": solver.schedule(0), "AT": solver.schedule(1)}
    log(f"create {t_create:.2f}s; A: {sched['A']}; A^T: {sched['AT']}")

    st0 = solver.begin()
    log(f"begin: power method {st0['power_iters']} iterations, {st0['t_power_ms']:.0f} ms")
    for w in range(args.warmup):
        solver.step(ce)
    log(f"{args.warmup} warm-up steps done")

    def inst_iters():
        return np.array([solver.stats_instance(i)["iters"] for i in range(n_inst)])

    it_before = inst_iters()
    sb = solver.stats()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        solver.step(ce)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    sa = solver.stats()
    it_after = inst_iters()
    inst_it = int((it_after - it_before).sum())
    active = int(sum(solver.stats_instance(i)["status"] == "UNSOLVED" for i in range(n_inst)))
    value = inst_it / elapsed
    log(f"timed {args.steps} steps: {elapsed * 1e3 / args.steps:.2f} ms/step, "
        f"{value:.4g} instance-iterations/s, {active} instances still iterating")

    # dominant pass kernel, from the event nodes of the timed steps' chunk graphs
    nc = sa["col_pass_launches"] - sb["col_pass_launches"]
    nr = sa["row_pass_launches"] - sb["row_pass_launches"]
    s_val = 4 if args.precision in ("mixed", "fp64a32") else 8
    s_vec = 4 if args.precision == "mixed" else 8
    col_b, row_b = pass_bytes(lp.m, lp.n, lp.nnz, s_val, s_vec)
    if nc > 0 and nr > 0:
        col_ms = (sa["col_pass_ms"] - sb["col_pass_ms"]) / nc
        row_ms = (sa["row_pass_ms"] - sb["row_pass_ms"]) / nr
        timing = (f"HIP event nodes around the passes of every {args.profile_every}th iteration "
                  f"inside the captured chunk graphs of the {args.steps} timed steps "
                  f"({nc} column and {nr} row pass launches)")
    else:
        col_ms, row_ms = solver.time_passes(20)
        timing = "HIP events around 20 launches of each pass after the timed steps"
    col_gbs = col_b / (col_ms * 1e-3) / 1e9
    row_gbs = row_b / (row_ms * 1e-3) / 1e9
    dom = "col" if col_ms >= row_ms else "row"
    ach = col_gbs if dom == "col" else row_gbs
    prec_name = args.precision or "fp64"
    out = {
        "metric": METRIC, "value": value, "unit": "instance-iterations/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": elapsed * 1e3 / args.steps, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None,
        "dtype": {"fp64": "f64", "mixed": "f32->f64", "fp64a32": "f64 (A in f32)"}[prec_name],
        "data": "synthetic",
        "config": {"workload": lpgen.WORKLOADS["batch256"], "name": "batch256",
                   "instances": n_inst, "m": lp.m, "n": lp.n, "nnz": lp.nnz,
                   "precision": prec_name, "tol": args.tol, "check_every": ce,
                   "step": f"one chunk: {ce} iterations of every instance with its checks and "
                           f"per-instance decisions (one chunk-graph launch)",
                   "autotune": not args.no_autotune},
        "iters_per_s": ce * args.steps / elapsed,
        "instances_iterating_in_timed_steps": active,
        "power_method": {"iters": int(st0["power_iters"]), "ms": st0["t_power_ms"]},
        "schedule": sched,
        "create_s": {"total": t_create, "preprocessing": sb["t_prep_ms"] / 1e3,
                     "autotune": sb["t_tune_ms"] / 1e3, "on": "device"},
        "roofline": {
            "bound": "hbm", "achieved": ach, "peak": PEAK_HBM_GBS, "unit": "GB/s",
            "frac": ach / PEAK_HBM_GBS, "traffic": read_traffic(dom, "batch256"),
            "kernel": ("k_pass<ColOp> (x-step over A^T)" if dom == "col"
                       else "k_pass<RowOp> (y-step over A)"),
            "alg_bytes_per_launch": col_b if dom == "col" else row_b,
            "avg_launch_ms": col_ms if dom == "col" else row_ms, "timing": timing},
        "passes": {"col_ms": col_ms, "row_ms": row_ms, "col_gbs": col_gbs, "row_gbs": row_gbs,
                   "both_passes_gbs": (col_b + row_b) / ((col_ms + row_ms) * 1e-3) / 1e9},
    }

    # ---- time to tolerance: one capped solve from the origin on the same handle
    if not args.no_ttt and time.perf_counter() + args.ttt_cap + 20 < deadline:
        log(f"time to tolerance: solve capped at {args.ttt_cap:.0f}s")
        solver.solve()
        out["time_to_tol"] = dict(ttt_fields(solver, lp, t_create), cap_s=args.ttt_cap,
                                  precision=prec_name)
        log(f"  {out['time_to_tol']['solved']}/{n_inst} solved")
    solver.close()
    del solver

    # ---- FP32 -> FP64 on the same instances (or plain FP64 if the main run was mixed)
    other = "fp64" if prec_name == "mixed" else "mixed"
    if not args.no_compare and time.perf_counter() + args.ttt_cap + 40 < deadline:
        log(f"compare: {other} batched solve capped at {args.ttt_cap:.0f}s")
        t0 = time.perf_counter()
        s2 = hprlp.Solver(lp, batched=True, **dict(opts, profile=0, precision={
            "fp64": hprlp.FP64, "mixed": hprlp.MIXED}[other]))
        tc = time.perf_counter() - t0
        s2.solve()
        out[f"compare_{other}_batched"] = dict(ttt_fields(s2, lp, tc), cap_s=args.ttt_cap,
                                               precision=other)
        log(f"  {out[f'compare_{other}_batched']['solved']}/{n_inst} solved")
        s2.close()
        del s2
    # ---- the single-LP FP64 solver over the instances in sequence, same cap
    seq_cap = min(args.ttt_cap, args.seq_cap)
    if not args.no_compare and time.perf_counter() + seq_cap + 30 < deadline:
        log(f"compare: single-LP FP64 solver over the instances in sequence, {seq_cap:.0f}s")
        nsolved, it_sum, ndone, t_used = 0, 0, 0, 0.0
        for i in range(n_inst):
            left = seq_cap - t_used
            if left <= 0:
                break
            s = hprlp.Solver(lp.instance(i), tol=args.tol, time_limit=left, check_every=ce)
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            r = s.solve()
            torch.cuda.synchronize()
            t_used += time.perf_counter() - t1
            nsolved += r.status == "OPTIMAL"
            it_sum += r.stats["iters"]
            ndone += 1
            s.close()
        out["compare_fp64_sequential"] = {
            "time_s": t_used, "instances_attempted": ndone, "solved": nsolved,
            "instance_iters_per_s": it_sum / max(t_used, 1e-9),
            "note": "solves only (creates excluded), same cap as the batched solves"}
        log(f"  {nsolved} solved of {ndone} attempted")

    if not args.no_cpu_baseline and time.perf_counter() + 60 < deadline:
        log("timing the CPU oracle on a sample of instances")
        out["cpu_baseline"] = cpu_baseline_batched(lp, host_threads(), args.cpu_sample_iters,
                                                   deadline - 20)
        log(f"  oracle: {out['cpu_baseline']['value']:.4g} instance-iterations/s on "
            f"{out['cpu_baseline']['cores']} threads")
    out["wall_s"] = time.perf_counter() - T_PROC0
    print(json.dumps(out), flush=True)


# ------------------------------------------------------------------------ single LP

def run_single(args):
    """One step = one solve of a single LP from the origin, capped at --time-limit."""
    import numpy as np
    import torch
    import lpgen
    from paper_2408_12179_amd import hprlp

    prec = args.precision or {"zipf4m": "mixed", "transport10m": "mixed"}.get(args.config, "fp64")
    t0 = time.perf_counter()
    lp = lpgen.make(args.config)
    log(f"{args.config}: m={lp.m} n={lp.n} nnz={lp.nnz} generated in "
        f"{time.perf_counter() - t0:.1f}s")
    P = {"mixed": hprlp.MIXED, "fp64a32": hprlp.FP64_A32}.get(prec, hprlp.FP64)
    sampled = not (args.no_profile or lp.nnz < 100_000)
    opts = dict(tol=args.tol, time_limit=args.time_limit, precision=P, check_every=150,
                profile=50 if sampled else 0, autotune=0 if args.no_autotune else 1,
                setup_on_host=1 if args.setup_on_host else 0,
                t1_zero=1 if args.t1_zero else 0, tile_order=args.tile_order,
                bundle_rows=args.bundle_rows)
    if args.stall_checks is not None:
        opts["stall_checks"] = args.stall_checks
    t0 = time.perf_counter()
    solver = hprlp.Solver(lp, **opts)
    t_create = time.perf_counter() - t0
    sched = {"A": solver.schedule(0), "AT": solver.schedule(1)}
    log(f"create {t_create:.2f}s; A: {sched['A']}; A^T: {sched['AT']}")
    for w in range(args.warmup):
        sol = solver.solve()
        log(f"warmup {w}: {sol.status} {sol.stats['iters']} it")
    torch.cuda.synchronize()
    times, stats = [], []
    for k in range(args.steps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        sol = solver.solve()
        torch.cuda.synchronize()
        times.append(time.perf_counter() - t0)
        stats.append(sol.stats)
        st = sol.stats
        log(f"step {k}: {sol.status} {st['iters']} it in {times[-1]:.2f}s (kkt "
            f"{max(st['rel_p'], st['rel_d'], st['rel_gap']):.2e})")
    st = stats[-1]
    value = float(np.mean(times))
    solved = all(s["status"] == "OPTIMAL" for s in stats)
    iters = int(st["iters"])
    s_val = 4 if prec in ("mixed", "fp64a32") else 8
    col_b, row_b = pass_bytes(lp.m, lp.n, lp.nnz, s_val, 8)
    if prec == "mixed" and iters > 0:
        # the timed launches sample every 50th iteration: a share iters_fp32 / iters of them
        # runs the FP32 phase (4-byte vectors), the rest the FP64 phase (8-byte vectors)
        f32 = st["iters_fp32"] / iters
        c4, r4 = pass_bytes(lp.m, lp.n, lp.nnz, s_val, 4)
        col_b, row_b = f32 * c4 + (1 - f32) * col_b, f32 * r4 + (1 - f32) * row_b
    out = {
        "metric": METRIC, "value": value, "unit": "s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": value * 1e3, "higher_is_better": False,
        "scaling": "weak", "vs_baseline": None,
        "dtype": "f32->f64" if prec == "mixed" else "f64", "data": "synthetic",
        "config": {"workload": lpgen.WORKLOADS[args.config], "name": args.config,
                   "m": lp.m, "m1": lp.m1, "n": lp.n, "nnz": lp.nnz, "precision": prec,
                   "tol": args.tol, "time_limit_s": args.time_limit, "check_every": 150,
                   "step": "one solve from the origin capped at time_limit_s",
                   "autotune": not args.no_autotune, "t1_zero": bool(args.t1_zero)},
        "solved": solved, "status": st["status"], "iters": iters,
        "power_iters": int(st["power_iters"]), "restarts": int(st["restarts"]),
        "rel_kkt": max(st["rel_p"], st["rel_d"], st["rel_gap"]),
        "iters_per_s": iters / max((st["t_solve_ms"] - st["t_power_ms"]) / 1e3, 1e-9),
        "schedule": sched,
        "create_s": {"total": t_create, "preprocessing": st["t_prep_ms"] / 1e3,
                     "autotune": st["t_tune_ms"] / 1e3,
                     "on": "host" if args.setup_on_host else "device"},
    }
    if lp.cert is not None:
        out["obj_rel_err_vs_certificate"] = abs(st["pobj"] - lp.cert.obj) / (1 + abs(lp.cert.obj))
    if prec == "mixed":
        out["iters_fp32"] = int(st["iters_fp32"])
    if st["col_pass_launches"] > 0:
        col_ms = st["col_pass_ms"] / st["col_pass_launches"]
        row_ms = st["row_pass_ms"] / st["row_pass_launches"]
        has_split = sched["A"]["chunks"] > 0 or sched["AT"]["chunks"] > 0
        split_pi = st["split_ms"] / max(st["col_pass_launches"], 1) if has_split else None
        timing = "HIP events around every 50th iteration's passes inside the timed solve"
    else:
        col_ms, row_ms = solver.time_passes(20)
        split_pi = None
        timing = "HIP events around 20 launches of each pass after the timed solve"
        if prec == "mixed":  # launched after the solve, in the phase it ended in
            s_vec = 4 if st["iters_fp32"] == iters else 8
            col_b, row_b = pass_bytes(lp.m, lp.n, lp.nnz, s_val, s_vec)
    row_kernel = "k_pass<RowOp> (y-step over A)"
    if args.t1_zero:  # residual pass over A, then the dense product with G = (A A^T)^-1
        row_b += 8 * lp.m * lp.m
        row_kernel = "k_pass<T1ResidOp> + k_t1_solve (T1 = 0 y-step: residual over A, G r)"
    col_gbs = col_b / (col_ms * 1e-3) / 1e9
    row_gbs = row_b / (row_ms * 1e-3) / 1e9
    dom = "col" if col_ms >= row_ms else "row"
    ach = col_gbs if dom == "col" else row_gbs
    out["roofline"] = {
        "bound": "hbm", "achieved": ach, "peak": PEAK_HBM_GBS, "unit": "GB/s",
        "frac": ach / PEAK_HBM_GBS,
        "traffic": None if args.t1_zero and dom == "row" else read_traffic(dom, args.config),
        "kernel": ("k_pass<ColOp> (x-step over A^T)" if dom == "col" else row_kernel),
        "alg_bytes_per_launch": col_b if dom == "col" else row_b,
        "avg_launch_ms": col_ms if dom == "col" else row_ms, "timing": timing,
    }
    out["passes"] = {"col_ms": col_ms, "row_ms": row_ms, "col_gbs": col_gbs,
                     "row_gbs": row_gbs, "split_ms_per_iter": split_pi,
                     "both_passes_gbs": (col_b + row_b) / ((col_ms + row_ms) * 1e-3) / 1e9}
    if args.compare:
        fp64 = dict(opts, precision=hprlp.FP64, profile=0)
        if args.t1_zero:  # the reference point is the default variant, T1 = lambda I - A A^T
            fp64["t1_zero"] = 0
        log("compare: plain FP64 solve of the same LP")
        s64 = hprlp.Solver(lp, **fp64)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        r = s64.solve()
        torch.cuda.synchronize()
        t64 = time.perf_counter() - t1
        out["compare_fp64"] = {"time_s": t64, "status": r.status, "iters": r.stats["iters"],
                               "rel_kkt": max(r.stats["rel_p"], r.stats["rel_d"],
                                              r.stats["rel_gap"]),
                               "speedup_of_this_run": t64 / value}
        if lp.cert is not None:
            out["compare_fp64"]["obj_rel_err_vs_certificate"] = \
                abs(r.stats["pobj"] - lp.cert.obj) / (1 + abs(lp.cert.obj))
        s64.close()
    if not args.no_cpu_baseline:
        log("timing the CPU oracle on a bounded sample")
        out["cpu_baseline"] = cpu_baseline_single(lp, iters, int(st["power_iters"]))
        if not solved:
            out["cpu_baseline"]["sample"] += " (a lower bound: the GPU run hit its time cap)"
    out["wall_s"] = time.perf_counter() - T_PROC0
    print(json.dumps(out), flush=True)
    solver.close()


# ------------------------------------------------------------------------ ablation

ABLATION = [
    ("DR", dict(rho=1.0, use_halpern=0, use_restart=0, sigma_update=0)),
    ("+ restart, Halpern", dict(rho=1.0, use_halpern=1, use_restart=1, sigma_update=0)),
    ("+ sigma update", dict(rho=1.0, use_halpern=1, use_restart=1, sigma_update=1)),
    ("+ relaxation rho = 2 (HPR-LP)", dict(rho=2.0, use_halpern=1, use_restart=1, sigma_update=1)),
]


def ablation(args):
    """The ablation steps on the first 64 batch256 instances (same seeds and size range)."""
    import numpy as np
    import lpgen
    from paper_2408_12179_amd import hprlp
    lp = lpgen.batched_lp(64, m_range=(1000, 50000), name="batch256[:64]")
    rows = []
    for name, kw in ABLATION:
        s = hprlp.Solver(lp, batched=True, check_every=100, tol=args.tol,
                         time_limit=args.time_limit, autotune=1, **kw)
        t0 = time.perf_counter()
        sol = s.solve()
        wall = time.perf_counter() - t0
        per = [s.stats_instance(i) for i in range(len(lp.inst_m1))]
        solved = [p["status"] == "OPTIMAL" for p in per]
        its = np.array([p["iters"] for p in per], dtype=float)
        sgm = float(np.exp(np.mean(np.log(its + 10.0))) - 10.0)  # unsolved: iterations run
        rows.append({"variant": name, **kw, "solved": int(sum(solved)),
                     "instances": len(per), "sgm10_iters": sgm, "wall_s": wall,
                     "batch_iters": int(sol.stats["iters"])})
        log(f"ablation {name}: {sum(solved)}/{len(per)} solved, SGM10 iterations {sgm:.0f}, "
            f"{wall:.1f} s")
        s.close()
    # the same steps on the tiny LP, solved alone: iterations to the tolerance
    tiny = lpgen.make("tiny")
    tiny_rows = []
    for name, kw in ABLATION:
        s = hprlp.Solver(tiny, tol=args.tol, max_iter=200_000, **kw)
        sol = s.solve()
        tiny_rows.append({"variant": name, "status": sol.status,
                          "iters": int(sol.stats["iters"]),
                          "solve_ms": sol.stats["t_solve_ms"]})
        log(f"ablation tiny {name}: {sol.status} in {sol.stats['iters']} iterations")
        s.close()
    print(json.dumps({"ablation": rows, "workload": "first 64 batch256 instances",
                      "tol": args.tol, "time_limit_s": args.time_limit,
                      "note": "unsolved instances count with the iterations run",
                      "ablation_tiny": tiny_rows}), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--config", default="batch256",
                    choices=["batch256", "tiny", "zipf1m", "zipf4m", "transport10m", "qap40",
                             "ot4m"])
    ap.add_argument("--precision", default=None, choices=["fp64", "mixed", "fp64a32"])
    ap.add_argument("--tol", type=float, default=1e-8)
    ap.add_argument("--ttt-cap", type=float, default=60.0,
                    help="batch256: cap of each time-to-tolerance solve (seconds)")
    ap.add_argument("--seq-cap", type=float, default=30.0,
                    help="batch256: cap of the sequential single-LP comparison (seconds)")
    ap.add_argument("--wall-budget", type=float, default=450.0,
                    help="batch256: optional legs run only while the run fits in this many "
                         "seconds from process start")
    ap.add_argument("--profile-every", type=int, default=10,
                    help="batch256: event nodes around the passes of every N-th iteration")
    ap.add_argument("--cpu-sample-iters", type=int, default=400)
    ap.add_argument("--time-limit", type=float, default=60.0,
                    help="single-LP configs and --ablation: seconds per solve")
    ap.add_argument("--no-autotune", action="store_true")
    ap.add_argument("--no-compare", action="store_true")
    ap.add_argument("--compare", action="store_true",
                    help="single-LP configs: also run the plain-FP64 GPU solver")
    ap.add_argument("--ablation", action="store_true",
                    help="run the ablation steps of Section 4.2 instead of the benchmark")
    ap.add_argument("--t1-zero", action="store_true",
                    help="the T1 = 0 variant (equality-only LPs, exact y-step through A A^T)")
    ap.add_argument("--setup-on-host", action="store_true",
                    help="preprocess on the host instead of the GPU (bit-identical arrays)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--bundle-rows", type=int, default=-1, choices=[-1, 0, 1],
                    help="row bundles: -1 shift-structured runs of A (default), 0 none, 1 all")
    ap.add_argument("--tile-order", type=int, default=0, choices=[-1, 0, 1],
                    help="nonzeros inside tiles: 0 row order, 1 column order, -1 autotuner")
    ap.add_argument("--stall-checks", type=int, default=None,
                    help="MIXED: checks of the FP32-stall rule (0: switch at tol_switch only)")
    ap.add_argument("--no-ttt", action="store_true",
                    help="batch256: skip the time-to-tolerance solve (profiling runs)")
    ap.add_argument("--no-profile", action="store_true",
                    help="single-LP configs: no HIP events around sampled pass launches")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus > 1 or world > 1:
        print(f"bench.py: one GPU only (asked for {max(args.gpus, world)}); the batched and "
              "single-LP paths would shard by instance / by rows, but no multi-GPU run is "
              "part of this benchmark.", file=sys.stderr)
        sys.exit(2)
    if args.ablation:
        ablation(args)
    elif args.config == "batch256":
        run_batched(args)
    else:
        run_single(args)


if __name__ == "__main__":
    main()
