"""Benchmark of the MI355X HPR-LP solver.

Metric (one JSON line on stdout): time to relative KKT 1e-8, with the SpMV HBM bandwidth of
the dominant pass kernel.  One step = one full solve through the C ABI: the power method for
lambda, then Algorithm 2 (column pass, row pass, checks, restarts, sigma updates) until the
relative KKT residual of w_bar is <= tol, with the inputs resident in HBM (preconditioning,
schedule autotuning and upload happen once, in create, before the timed region; the paper
also excludes preprocessing and counts the power method, Section 4.1).  A solve that hits the
per-step time cap counts as the cap (the paper's convention for unsolved instances) and the
line says solved=false.

Default workload: the single large sparse LP (m = 500k, half equality; n = 1M; row lengths
U{5..40}; Zipf(1.1) column popularity; plain FP64).  --config selects the other workloads:
  zipf4m        the same generator at m = 2M, n = 4M, FP32 -> FP64
  batch256      256 independent LPs (m_i ~ U{1k..50k}, n_i = 2 m_i) packed block-diagonally,
                solved in one batched run (check_every = 100)
  transport10m  2000 x 5000 transportation LP (n = 10M), FP32 -> FP64
  qap40         LP relaxation of a random QAP with N = 40 in the form of Section 4.4
                (n = 2.56M, m = 1.41M equality rows, nnz = 7.8M), FP64
  ot4m          balanced optimal transport 2048 x 2048 (m = 4095 equality rows, n = 4.19M),
                FP64; with --t1-zero the T1 = 0 variant of Section 3.2 (exact y-step)
--compare adds the plain-FP64 GPU solver on the same instances under the same time budget:
the FP64 single-LP solve for the mixed-precision workloads (with --t1-zero: the default
variant T1 = lambda I - A A^T), and for batch256 the single-LP FP64 solver run on the
instances one after another.
--ablation instead runs the four steps of the paper's ablation (Section 4.2, Fig. 1: DR;
+ restart and Halpern; + sigma update; + relaxation rho = 2, i.e. HPR-LP) on the first 64
batch256 instances, each variant as one batched solve capped at --time-limit, and prints one
JSON line with the solved counts and shifted geometric means of the iteration counts.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0
METRIC = "time to rel. KKT 1e-8 + SpMV HBM GB/s; FP32→FP64 & batched vs plain FP64"


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


def cpu_baseline(lp, gpu_iters, gpu_power_iters, sample_iters=300, sample_power=60):
    """The oracle (plain FP64 C, one thread) timed on a bounded sample of the same workload:
    sample_power power iterations and sample_iters HPR-LP iterations, extrapolated to the
    GPU run's counts."""
    import oracle
    t0 = time.perf_counter()
    r = oracle.solve(lp, max_iter=sample_iters, power_max_iter=sample_power, power_tol=0.0)
    wall = time.perf_counter() - t0
    it_rate = r.iters / max(r.t_solve - r.t_power, 1e-9)
    pw_rate = r.power_iters / max(r.t_power, 1e-9)
    est = gpu_power_iters / pw_rate + gpu_iters / it_rate
    return {"value": est, "unit": "s", "cores": 1, "kind": "oracle",
            "sample": f"{r.power_iters} power iterations + {r.iters} HPR-LP iterations of the "
                      f"same LP on 1 host core ({wall:.1f} s wall incl. its preconditioning), "
                      f"extrapolated to the GPU run's {gpu_power_iters} power + {gpu_iters} "
                      f"iterations",
            "oracle_iters_per_s": it_rate}


def cpu_baseline_batched(lp, inst_iters, power_iters, n_sample=16, sample_iters=800,
                         sample_power=100):
    """The oracle on n_sample instances spread over the batch (sample_power power and
    sample_iters HPR-LP iterations each); its cost per nonzero-iteration, applied to every
    instance's own iteration count in the GPU run (and the power iterations)."""
    import numpy as np
    import oracle
    n_inst = len(lp.inst_m1)
    idx = np.linspace(0, n_inst - 1, n_sample).astype(int)
    it_s, pw_s = 0.0, 0.0
    t0 = time.perf_counter()
    for i in idx:
        inst = lp.instance(int(i))
        r = oracle.solve(inst, max_iter=sample_iters, power_max_iter=sample_power,
                         power_tol=0.0, check_every=100)
        it_s += (r.t_solve - r.t_power) / r.iters * 1.0 / inst.nnz
        pw_s += r.t_power / r.power_iters / inst.nnz
    wall = time.perf_counter() - t0
    it_s /= len(idx)
    pw_s /= len(idx)
    nnz_i = np.diff(lp.rowptr[lp.inst_row_off])
    est = float(np.sum(np.asarray(inst_iters) * nnz_i) * it_s + power_iters * lp.nnz * pw_s)
    return {"value": est, "unit": "s", "cores": 1, "kind": "oracle",
            "sample": f"instances {list(map(int, idx))}: {sample_power} power + {sample_iters} "
                      f"HPR-LP iterations each on 1 host core ({wall:.1f} s wall incl. their "
                      f"preconditioning); cost per nonzero-iteration applied to every "
                      f"instance's iteration count in the GPU run"}


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
        print(f"[bench] ablation {name}: {sum(solved)}/{len(per)} solved, SGM10 iterations "
              f"{sgm:.0f}, {wall:.1f} s", file=sys.stderr, flush=True)
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
        print(f"[bench] ablation tiny {name}: {sol.status} in {sol.stats['iters']} iterations",
              file=sys.stderr, flush=True)
        s.close()
    print(json.dumps({"ablation": rows, "workload": "first 64 batch256 instances",
                      "tol": args.tol, "time_limit_s": args.time_limit,
                      "note": "unsolved instances count with the iterations run",
                      "ablation_tiny": tiny_rows}), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1)
    ap.add_argument("--warmup", type=int, default=0)
    ap.add_argument("--config", default="zipf1m",
                    choices=["tiny", "zipf1m", "zipf4m", "batch256", "transport10m", "qap40",
                             "ot4m"])
    ap.add_argument("--precision", default=None, choices=["fp64", "mixed", "fp64a32"])
    ap.add_argument("--tol", type=float, default=1e-8)
    ap.add_argument("--time-limit", type=float, default=60.0, help="seconds per solve")
    ap.add_argument("--no-autotune", action="store_true")
    ap.add_argument("--compare", action="store_true",
                    help="also run the plain-FP64 GPU solver on the same instances")
    ap.add_argument("--ablation", action="store_true",
                    help="run the ablation steps of Section 4.2 instead of the benchmark")
    ap.add_argument("--t1-zero", action="store_true",
                    help="the T1 = 0 variant (equality-only LPs, exact y-step through A A^T)")
    ap.add_argument("--setup-on-host", action="store_true",
                    help="preprocess on the host instead of the GPU (bit-identical arrays)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-profile", action="store_true",
                    help="do not time pass launches with HIP events (default: every 50th "
                         "iteration of a single-LP solve with >= 1e5 nonzeros is bracketed "
                         "by events)")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus > 1 or world > 1:
        print(f"bench.py: one GPU only (asked for {max(args.gpus, world)}); the batched and "
              "single-LP paths would shard by instance / by rows, but no multi-GPU run is "
              "part of this benchmark.", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    import lpgen
    from paper_2408_12179_amd import hprlp

    if args.ablation:
        ablation(args)
        return
    batched = args.config == "batch256"
    prec = args.precision or {"zipf4m": "mixed", "transport10m": "mixed"}.get(args.config, "fp64")
    ce = 100 if batched else 150
    t0 = time.perf_counter()
    lp = lpgen.make(args.config)
    print(f"[bench] {args.config}: m={lp.m} n={lp.n} nnz={lp.nnz} generated in "
          f"{time.perf_counter() - t0:.1f}s", file=sys.stderr, flush=True)
    P = {"mixed": hprlp.MIXED, "fp64a32": hprlp.FP64_A32}.get(prec, hprlp.FP64)
    # HIP events around sampled pass launches inside the timed solve, except where the solve
    # runs as captured graphs (batches, and single LPs under 1e5 nonzeros: launch-bound)
    sampled = not (args.no_profile or batched or lp.nnz < 100_000)
    opts = dict(tol=args.tol, time_limit=args.time_limit, precision=P, check_every=ce,
                profile=50 if sampled else 0, autotune=0 if args.no_autotune else 1,
                setup_on_host=1 if args.setup_on_host else 0,
                t1_zero=1 if args.t1_zero else 0)
    t0 = time.perf_counter()
    solver = hprlp.Solver(lp, batched=batched, **opts)
    t_create = time.perf_counter() - t0
    sched = {"A": solver.schedule(0), "AT": solver.schedule(1)}
    print(f"[bench] create ({'host' if args.setup_on_host else 'device'} preprocessing, "
          f"schedules{'' if args.no_autotune else ' + autotune'}, upload) {t_create:.2f}s; "
          f"A: {sched['A']}; A^T: {sched['AT']}", file=sys.stderr, flush=True)

    for w in range(args.warmup):
        sol = solver.solve()
        print(f"[bench] warmup {w}: {sol.status} {sol.stats['iters']} it", file=sys.stderr,
              flush=True)
    torch.cuda.synchronize()
    times, stats, sol = [], [], None
    for k in range(args.steps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        sol = solver.solve()
        torch.cuda.synchronize()
        times.append(time.perf_counter() - t0)
        stats.append(sol.stats)
        st = sol.stats
        print(f"[bench] step {k}: {sol.status} {st['iters']} it in {times[-1]:.2f}s "
              f"(kkt {max(st['rel_p'], st['rel_d'], st['rel_gap']):.2e})", file=sys.stderr,
              flush=True)
    st = stats[-1]
    value = float(np.mean(times))
    solved = all(s["status"] == "OPTIMAL" for s in stats)
    iters = int(st["iters"])
    s_val = 4 if prec in ("mixed", "fp64a32") else 8
    s_vec = 4 if (prec == "mixed" and st["iters_fp32"] == iters) else 8
    col_b, row_b = pass_bytes(lp.m, lp.n, lp.nnz, s_val, s_vec)
    out = {
        "metric": METRIC, "value": value, "unit": "s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": value * 1e3, "higher_is_better": False,
        "scaling": "weak", "vs_baseline": None,
        "dtype": "f32->f64" if prec == "mixed" else "f64", "data": "synthetic",
        "config": {"workload": lpgen.WORKLOADS[args.config], "name": args.config,
                   "m": lp.m, "m1": lp.m1, "n": lp.n, "nnz": lp.nnz, "precision": prec,
                   "tol": args.tol, "time_limit_s": args.time_limit, "check_every": ce,
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
    inst_iters = None
    if batched:
        n_inst = len(lp.inst_m1)
        per = [solver.stats_instance(i) for i in range(n_inst)]
        inst_iters = [p["iters"] for p in per]
        errs = []
        for i, p in enumerate(per):
            inst = lp.instance(i)
            if inst.cert is not None and p["status"] == "OPTIMAL":
                errs.append(abs(p["pobj"] - inst.cert.obj) / (1 + abs(inst.cert.obj)))
        out["batched"] = {
            "instances": n_inst,
            "solved": sum(p["status"] == "OPTIMAL" for p in per),
            "inst_iters_p50": float(np.percentile(inst_iters, 50)),
            "inst_iters_max": int(max(inst_iters)),
            "instance_iters_per_s": float(sum(inst_iters)) / value,
            "compactions": int(st["n_compactions"]),
            "max_obj_rel_err_vs_certificate": max(errs) if errs else None,
        }
    elif lp.cert is not None:
        out["obj_rel_err_vs_certificate"] = abs(st["pobj"] - lp.cert.obj) / (1 + abs(lp.cert.obj))
    if prec == "mixed":
        out["iters_fp32"] = int(st["iters_fp32"])

    # pass timing: HIP events around sampled pass launches inside the timed solve (single
    # LP), or around launches of both passes right after it (a batch runs as graphs)
    if st["col_pass_launches"] > 0:
        col_ms = st["col_pass_ms"] / st["col_pass_launches"]
        row_ms = st["row_pass_ms"] / st["row_pass_launches"]
        # time between the main kernel's end event and the pass's end event: the split-row
        # finisher where a schedule has split rows, otherwise just the event gap
        has_split = sched["A"]["chunks"] > 0 or sched["AT"]["chunks"] > 0
        split_pi = st["split_ms"] / max(st["col_pass_launches"], 1) if has_split else None
        timing = "HIP events around every 50th iteration's passes inside the timed solve"
    else:
        col_ms, row_ms = solver.time_passes(20)
        split_pi = None
        timing = "HIP events around 20 launches of each pass after the timed solve"
        if prec == "mixed" and st["iters_fp32"] < iters:
            s_vec = 8
            col_b, row_b = pass_bytes(lp.m, lp.n, lp.nnz, s_val, s_vec)
    row_kernel = "k_pass<RowOp> (y-step over A)"
    if args.t1_zero:  # residual pass over A, then the dense product with G = (A A^T)^-1
        row_b += 8 * lp.m * lp.m
        row_kernel = "k_t1_resid + k_t1_solve (T1 = 0 y-step: residual over A, G r)"
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
        if batched:
            del fp64["autotune"]
            print("[bench] compare: single-LP FP64 solver over the instances in sequence",
                  file=sys.stderr, flush=True)
            nsolved, it_sum, ndone, t_used = 0, 0, 0, 0.0
            budget = args.time_limit
            for i in range(len(lp.inst_m1)):
                left = budget - t_used
                if left <= 0:
                    break
                s = hprlp.Solver(lp.instance(i), **dict(fp64, time_limit=left))
                torch.cuda.synchronize()
                t1 = time.perf_counter()
                r = s.solve()
                torch.cuda.synchronize()
                t_used += time.perf_counter() - t1
                nsolved += r.status == "OPTIMAL"
                it_sum += r.stats["iters"]
                ndone += 1
                s.close()
                if i % 32 == 0:
                    print(f"[bench]   instance {i}: {r.status} {r.stats['iters']} it, "
                          f"{t_used:.1f}s used", file=sys.stderr, flush=True)
            out["compare_fp64_sequential"] = {
                "time_s": t_used, "instances_attempted": ndone, "solved": nsolved,
                "instance_iters_per_s": it_sum / max(t_used, 1e-9),
                "note": "same time budget, solves only (creates excluded)"}
        else:
            if args.t1_zero:  # the reference point is the default variant, T1 = lambda I - A A^T
                fp64["t1_zero"] = 0
            print("[bench] compare: plain FP64 solve of the same LP"
                  + (" with T1 = lambda I - A A^T" if args.t1_zero else ""),
                  file=sys.stderr, flush=True)
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
        print("[bench] timing the CPU oracle on a bounded sample", file=sys.stderr, flush=True)
        if batched:
            out["cpu_baseline"] = cpu_baseline_batched(lp, inst_iters, int(st["power_iters"]))
        else:
            out["cpu_baseline"] = cpu_baseline(lp, iters, int(st["power_iters"]))
        if not solved:
            out["cpu_baseline"]["sample"] += " (a lower bound: the GPU run hit its time cap)"
    print(json.dumps(out), flush=True)
    solver.close()


if __name__ == "__main__":
    main()
