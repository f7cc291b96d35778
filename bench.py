#!/usr/bin/env python3
"""Benchmark: time to 1e-4 relative KKT of FP32 PDLP on one MI355X, with SpMV HBM bandwidth.

One step = one full cold-start PDLP solve (scaling and matrix already on the device, as set up by
pdlp_create) of the general sparse LP: m = 500,000 rows, n = 1,000,000 columns, Zipf(1.5) row lengths
capped at 5,000 (27.35M nonzeros for seed 0), 40 % equality / 60 % <= rows, 70 % boxed / 30 % free
columns, FP32 iterates and matrix with FP64 norms, to relative KKT error 1e-4.

Printed: one JSON line: metric, value = median seconds per solve (the production configuration:
each evaluation interval replayed from a captured hipGraph); the roofline of the dominant iteration
kernel by measured time, from a separate solve of the same LP whose kernel dispatches record HIP
start and stop events on the handle's stream; the FP64 cold solve; other seeds of the same generator (bounded);
the learned warm start on held-out LPs; and the FP64 CPU oracle timed on a bounded sample as
cpu_baseline. Progress goes to stderr.
"""
import argparse
import json
import os
import platform
import statistics
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0  # MI355X HBM3E, 8 TB/s

# HBM bytes per launch of the dominant kernel measured by rocprofv3 (FETCH_SIZE x 2.000 + WRITE_SIZE
# x 1.000, the factors of a 256 MiB device copy), keyed by workload, kernel and the SHA-1 of the
# sources the kernels and their launch configuration are built from; any change to them makes the
# figure stale (reported null).
KERNEL_SOURCES = ["pdlp_internal.h", "pdlp_kernels.h", "pdlp.hip"]
MEASURED_TRAFFIC = {  # {(workload, kernel, sha1): HBM bytes per launch}; commands and raw figures in profiles/
    # A side (k_panel + k_dual) on the 500k x 1M general sparse LP: FETCH_SIZE (100,391 + 58,435) KiB x 2
    # + WRITE_SIZE (21,122 + 6,113) KiB
    ("zipf", "dual", "a4ad068062111aa284e73b81559ce42b8d16c195"): 353_164_288,
    # k_primal_cb on the same LP: FETCH_SIZE 111,420 KiB x 2 + WRITE_SIZE 13,682 KiB
    ("zipf", "primal", "a4ad068062111aa284e73b81559ce42b8d16c195"): 242_198_528,
    # the energy-shaped LP: k_dual FETCH_SIZE 258,247 KiB x 2 + WRITE_SIZE 60,546 KiB; k_primal
    # FETCH_SIZE 290,683 KiB x 2 + WRITE_SIZE 152,442 KiB (mean over accepted and deferred launches)
    ("energy", "dual", "a4ad068062111aa284e73b81559ce42b8d16c195"): 590_888_960,
    ("energy", "primal", "a4ad068062111aa284e73b81559ce42b8d16c195"): 751_419_392,
}


def oracle_reference(args, info, chk):
    """The stored FP64 oracle solve of the same LP to the same tolerance (written by
    tests/golden/make_zipf500k_oracle.py), next to this solve's objectives. Both points meet the
    relative KKT tolerance, so their objectives may differ by up to the tolerance's duality gap."""
    path = os.path.join(ROOT, "tests", "golden", "zipf500k_seed0_oracle.json")
    if args.workload != "zipf" or args.seed != 0 or not os.path.exists(path):
        return None
    with open(path) as f:
        ref = json.load(f)["solves"].get("%g" % args.tol)
    if ref is None:
        return None
    pobj = info["primal_obj"]
    return {"source": "FP64 oracle solve, tests/golden/zipf500k_seed0_oracle.json", "tol": ref["tol"],
            "attempts": ref["iterations"], "pobj": ref["pobj"], "dobj": ref["dobj"],
            "primal_obj_rel_diff": abs(pobj - ref["pobj"]) / max(1.0, abs(ref["pobj"])),
            "this_dobj_oracle_evaluated": chk.get("dobj")}


def kernel_source_sha1():
    import hashlib
    h = hashlib.sha1()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_2503_10344_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def algorithmic_bytes(kernel, m, n, nnz, tb):
    """Bytes one launch must move (values tb bytes, indices 4 bytes, each vector element once).

    dual   (A x' + dual update): A values + columns, row offsets, gather of x', read y, ax, b and
           the row senses, write y' and ax'.
    primal (A'y' + primal update + averages, accepted attempt): A' values + columns, row offsets,
           gather of y', write A'y', read x, c, l, u, write x', and the FP64 averages. FP32 pairs
           the average updates of consecutive accepted attempts: one attempt of a pair leaves them
           alone, the other reads the older x and y and reads + writes x-bar and y-bar once, i.e.
           per accepted attempt (16 + 4) / 2 = 10 bytes per column and (16 + 2 * 4) / 2 = 12 per
           row. FP64 updates every attempt (read+write x-bar, read y, read+write y-bar) and also
           reads+writes A'y-bar and A x-bar and reads A x (FP32 recomputes those two products
           before each evaluation instead).
    """
    if kernel == "dual":
        return nnz * (tb + 4) + 4 * (m + 1) + tb * n + m * (5 * tb + 1)
    if tb == 4:
        return nnz * (tb + 4) + 4 * (n + 1) + tb * m + (6 * tb + 10) * n + 12 * m
    return nnz * (tb + 4) + 4 * (n + 1) + tb * m + 10 * tb * n + 6 * tb * m


def cpu_model():
    try:
        for ln in open("/proc/cpuinfo"):
            if ln.startswith("model name"):
                return ln.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor()


def make_workload(name, seed):
    from paper_2503_10344_amd import generators as g
    if name == "zipf":
        lp = g.general_sparse(seed)
        desc = (f"general sparse LP, m=500000, n=1000000, Zipf(1.5) row lengths capped at 5000, "
                f"nnz={lp.nnz}, 40% = / 60% <= rows, 70% boxed [0,10] / 30% free columns, seed {seed}")
    elif name == "setcover":
        lp = g.set_cover(seed)
        desc = f"set-cover LP relaxation, m=2000, n=5000, 5 ones per column, seed {seed}"
    elif name == "energy":
        lp = g.energy(seed)
        desc = (f"energy-system-shaped LP, 8760 steps x 100 nodes x 6 technologies, m={lp.m}, n={lp.n}, "
                f"nnz={lp.nnz}, seed {seed}")
    else:
        raise SystemExit(f"unknown workload {name}")
    return lp, desc


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="zipf",
                    choices=["zipf", "setcover", "energy", "batch", "fixing", "propagation", "resolve",
                             "snapshots"])
    ap.add_argument("--fixing-lp", default="zipf", choices=["zipf", "energy"],
                    help="with --workload fixing or propagation: the LP whose size they run at")
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--tol", type=float, default=1e-4)
    ap.add_argument("--iter-limit", type=int, default=500_000)
    ap.add_argument("--no-fp64", action="store_true", help="skip the FP64 cold-solve comparison")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-iters", type=int, default=1000, help="oracle attempts in the CPU sample")
    ap.add_argument("--no-warm-start", action="store_true", help="skip the learned warm-start comparison")
    ap.add_argument("--warm-instances", type=int, default=200)
    ap.add_argument("--other-seeds", default="1,2", help="further seeds of the workload, solved once each")
    ap.add_argument("--other-seeds-limit", type=int, default=300_000)
    ap.add_argument("--batch-count", type=int, default=256)
    ap.add_argument("--col-blocks", type=int, default=0,
                    help="pdlp_options.col_blocks for the solves (0 auto, 1 forced where possible, -1 off)")
    ap.add_argument("--calib-copy-mib", type=int, default=0,
                    help="first copy this many MiB device-to-device (a kernel of known size for scaling "
                         "hardware byte counters)")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU: the library runs the PDLP solve on a single MI355X and has no "
              "multi-GPU path; run it with --gpus 1.", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2503_10344_amd import pdlp

    torch.cuda.set_device(0)
    if args.workload == "batch":
        return bench_batch(args)
    if args.workload == "fixing":
        return bench_fixing(args)
    if args.workload == "propagation":
        return bench_propagation(args)
    if args.workload == "resolve":
        return bench_resolve(args)
    if args.workload == "snapshots":
        return bench_snapshots(args)
    if args.calib_copy_mib > 0:
        src = torch.ones(args.calib_copy_mib * 2**18, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        log(f"calibration copy: {args.calib_copy_mib} MiB read + {args.calib_copy_mib} MiB written")
        del src, dst
    t = time.time()
    lp, desc = make_workload(args.workload, args.seed)
    log(f"workload generated in {time.time() - t:.1f} s: m={lp.m} n={lp.n} nnz={lp.nnz}")

    # ---------------- FP32 solves (the measured configuration: hipGraphs, no timing events) ----------
    t = time.time()
    p = pdlp.Problem(lp, precision="fp32", col_blocks=args.col_blocks)
    torch.cuda.synchronize()
    create_s = time.time() - t
    sched = p.schedule()
    log(f"create (upload, transpose, scaling, autotune) {create_s:.2f} s; schedule {sched}")
    for w in range(args.warmup):
        info = p.solve(tol=args.tol, iter_limit=args.iter_limit)
        log(f"warmup {w}: {info['status_name']} iters={info['iterations']} {info['solve_seconds']:.3f} s")
    times, iters = [], []
    info = None
    for s in range(args.steps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        info = p.solve(tol=args.tol, iter_limit=args.iter_limit)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        times.append(dt)
        iters.append(info["iterations"])
        log(f"step {s}: {info['status_name']} iters={info['iterations']} restarts={info['restarts']} "
            f"rel_kkt={info['rel_kkt']:.2e} obj={info['primal_obj']:.10g} {dt:.3f} s")
    sol = p.get()
    sec = statistics.median(times)
    it = int(statistics.median(iters))
    p.close()

    # ---------------- kernel durations: a separate solve with HIP events around every launch ---------
    # (graphs are off in that mode; the trajectory is the same bit for bit)
    pk = pdlp.Problem(lp, precision="fp32", kernel_timing=True, col_blocks=args.col_blocks)
    ik = pk.solve(tol=args.tol, iter_limit=args.iter_limit)
    ks = pk.kernel_stats()
    pk.close()
    log(f"timing solve: {ik['iterations']} iterations (timed solves: {it}), {ik['solve_seconds']:.3f} s with events")
    tb = 4
    kern = {}
    # the A side of an attempt is k_panel (column-panel sums of the long rows, when used) + k_dual
    a_us = ks["dual"]["avg_ms"] * 1e3 + (ks["panel"]["avg_ms"] * 1e3 if ks["panel"]["launches"] else 0.0)
    sides = {"dual": (a_us, ks["dual"]["launches"]), "primal": (ks["primal"]["avg_ms"] * 1e3, ks["primal"]["launches"])}
    for name, (us, launches) in sides.items():
        bytes_ = algorithmic_bytes(name, lp.m, lp.n, lp.nnz, tb)
        gbs = bytes_ / (us * 1e-6) / 1e9 if us > 0 else None
        kern[name] = dict(launches=launches, avg_us=us, alg_bytes=bytes_, gbs=gbs,
                          frac=(gbs / PEAK_HBM_GBS) if gbs else None,
                          traffic=MEASURED_TRAFFIC.get((args.workload, name, kernel_source_sha1())))
    if ks["panel"]["launches"]:
        kern["dual"]["of_which_k_panel_us"] = ks["panel"]["avg_ms"] * 1e3
    dname = max(kern, key=lambda k: kern[k]["avg_us"])  # dominant by measured time per attempt
    dom = kern[dname]
    traffic = MEASURED_TRAFFIC.get((args.workload, dname, kernel_source_sha1()))
    label = {"dual": "k_panel + k_dual (A x' with the dual update and step-size sums)",
             "primal": ("k_primal_cb (A'y' by column blocks, with the primal update and the averages)"
                        if ks["col_blocks"]["launches"] else "k_primal (A'y' with the primal update and the averages)")}[dname]
    roofline = {"bound": "hbm", "achieved": round(dom["gbs"], 1), "peak": PEAK_HBM_GBS, "unit": "GB/s",
                "frac": round(dom["gbs"] / PEAK_HBM_GBS, 4), "traffic": traffic,
                "kernel": label, "alg_bytes_per_launch": dom["alg_bytes"], "avg_launch_us": round(dom["avg_us"], 2)}
    log(f"kernels: {json.dumps(kern)}")

    # ---------------- FP64 cold solve (comparison) ----------------
    fp64 = None
    if not args.no_fp64:
        t = time.time()
        p64 = pdlp.Problem(lp, precision="fp64")
        c64 = time.time() - t
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        i64 = p64.solve(tol=args.tol, iter_limit=args.iter_limit)
        torch.cuda.synchronize()
        s64 = time.perf_counter() - t0
        fp64 = dict(seconds=round(s64, 4), iterations=i64["iterations"], status=i64["status_name"],
                    primal_obj=i64["primal_obj"], create_s=round(c64, 2))
        log(f"fp64 cold: {i64['status_name']} iters={i64['iterations']} {s64:.3f} s obj={i64['primal_obj']:.10g}")
        p64.close()

    # ---------------- other seeds of the same generator (time to tolerance is heavy-tailed) ----------
    others = []
    for sd in [int(v) for v in args.other_seeds.split(",") if v.strip()]:
        if args.workload != "zipf":
            break
        lpo, _ = make_workload(args.workload, sd)
        po = pdlp.Problem(lpo, precision="fp32")
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        io = po.solve(tol=args.tol, iter_limit=args.other_seeds_limit)
        torch.cuda.synchronize()
        dto = time.perf_counter() - t0
        others.append({"seed": sd, "status": io["status_name"], "iterations": io["iterations"], "seconds": round(dto, 3),
                       "rel_kkt": io["rel_kkt"], "nnz": lpo.nnz, "iteration_cap": args.other_seeds_limit})
        log(f"seed {sd}: {io['status_name']} iters={io['iterations']} rel_kkt={io['rel_kkt']:.2e} {dto:.3f} s")
        po.close()
        del lpo

    # ---------------- CPU baseline: the FP64 oracle on a bounded sample ----------------
    cpu, chk = None, {"rel_kkt": None}
    if not args.no_cpu_baseline:
        import oracle
        # the oracle's FP64 re-evaluation of the returned point (original data) comes with this leg
        t = time.time()
        chk = oracle.kkt(lp, sol.x, sol.y)
        log(f"oracle re-evaluation of the returned point: rel_kkt={chk['rel_kkt']:.3e} ({time.time() - t:.1f} s)")
        n1, n2 = 8, max(16, args.cpu_iters)
        t = time.time()
        oracle.solve(lp, tol=0.0, iter_limit=n1)
        t1 = time.time() - t
        t = time.time()
        oracle.solve(lp, tol=0.0, iter_limit=n2)
        t2 = time.time() - t
        per_iter = (t2 - t1) / (n2 - n1)
        setup = max(t1 - n1 * per_iter, 0.0)
        est = setup + per_iter * it
        cpu = {"value": round(est, 2), "unit": "s", "cores": oracle.num_threads(), "kind": "oracle",
               "sample": (f"FP64 oracle (C, OpenMP row loops) run for {n1} and {n2} PDHG attempts on the same "
                          f"instance ({t1:.1f} s and {t2:.1f} s incl. scaling); time-to-tolerance extrapolated as "
                          f"setup {setup:.2f} s + {per_iter * 1e3:.1f} ms/attempt x {it} attempts (the GPU's count); "
                          f"host CPU: {cpu_model()}")}
        log(f"cpu baseline: {json.dumps(cpu)}")

    # ---------------- learned warm start vs cold FP32 (held-out energy-shaped LPs) ----------------
    warm = None
    if not args.no_warm_start:
        warm = warm_start_comparison(args.warm_instances, args.tol)

    out = {
        "metric": "time to 1e-4 rel. KKT + SpMV HBM GB/s; FP32/warm-start vs FP64 cold PDLP",
        "value": round(sec, 4),
        "unit": "s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(sec * 1e3, 2),
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": desc, "precision": "FP32 iterates and matrix, FP64 norms/KKT/restarts",
                   "start": "cold", "tol": args.tol, "m": lp.m, "n": lp.n, "nnz": lp.nnz,
                   "tile_nnz": sched["tile_nnz"]},
        "iterations": it,
        "iters_per_s": round(it / sec, 1),
        "status": info["status_name"],
        "rel_kkt": info["rel_kkt"],
        "oracle_rel_kkt": chk["rel_kkt"],
        "primal_obj": info["primal_obj"],
        "oracle_reference": oracle_reference(args, info, chk),
        "create_s": round(create_s, 3),
        "roofline": roofline,
        "kernels": {k: {kk: (round(vv, 3) if isinstance(vv, float) else vv) for kk, vv in v.items()}
                    for k, v in kern.items()},
        "fp64_cold": fp64,
        "other_seeds": others,
        "warm_start": warm,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


def warm_start_comparison(count, tol):
    """Cold FP32 vs the committed trained warm start (inference included) on held-out seeds."""
    from paper_2503_10344_amd import generators as g
    from paper_2503_10344_amd import pdlp, warmstart
    net, mode = warmstart.load_trained()
    rows = []
    for s in range(warmstart.TEST_SEEDS[0], warmstart.TEST_SEEDS[0] + count):
        lp = g.warmstart_family(s)
        with pdlp.Problem(lp) as p:
            p.solve(tol=tol)   # warm-up of this handle's graphs
            cold = p.solve(tol=tol)
            w = warmstart.warm_solve(net, p, tol=tol, mode=mode)
        rows.append((cold["iterations"], cold["solve_seconds"], w["iterations"], w["seconds"], w["fallback"],
                     w["predict_seconds"]))
    med = lambda k: statistics.median(r[k] for r in rows)  # noqa: E731
    res = {"instances": f"energy-shaped LPs, m 10k-100k, held-out seeds {warmstart.TEST_SEEDS[0]}.."
                        f"{warmstart.TEST_SEEDS[0] + count - 1}", "mode": mode,
           "cold_total_s": round(sum(r[1] for r in rows), 3), "warm_total_s": round(sum(r[3] for r in rows), 3),
           "cold_median_s": round(med(1), 4), "warm_median_s": round(med(3), 4),
           "cold_median_iterations": med(0), "warm_median_iterations": med(2),
           "median_predict_ms": round(1e3 * med(5), 3),
           "fallback_rate": round(sum(r[4] for r in rows) / len(rows), 3),
           "warm_faster_fraction": round(sum(r[3] < r[1] for r in rows) / len(rows), 3)}
    log(f"warm start: {json.dumps(res)}")
    return res


def bench_batch(args):
    """Many uneven LPs in one handle: makespan of the batched solve vs the same LPs one by one."""
    import torch
    from paper_2503_10344_amd import generators as g
    from paper_2503_10344_amd import pdlp
    t = time.time()
    lps = g.batch(args.seed, count=args.batch_count)
    nnz = sum(lp.nnz for lp in lps)
    log(f"{len(lps)} instances generated in {time.time() - t:.1f} s: sum m={sum(lp.m for lp in lps)} "
        f"sum n={sum(lp.n for lp in lps)} nnz={nnz}")
    t = time.time()
    b = pdlp.Batch(lps, precision="fp32", col_blocks=args.col_blocks)
    torch.cuda.synchronize()
    create_s = time.time() - t
    for w in range(args.warmup):
        b.solve(tol=args.tol, iter_limit=args.iter_limit)
    times, infos = [], None
    for s in range(args.steps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        infos = b.solve(tol=args.tol, iter_limit=args.iter_limit)
        torch.cuda.synchronize()
        times.append(time.perf_counter() - t0)
        log(f"step {s}: makespan {times[-1]:.3f} s, max iterations {max(i['iterations'] for i in infos)}")
    b.close()
    seq, seq_it = 0.0, []
    for lp in lps:
        with pdlp.Problem(lp, precision="fp32", col_blocks=args.col_blocks) as p:
            p.solve(tol=args.tol, iter_limit=args.iter_limit)
            i = p.solve(tol=args.tol, iter_limit=args.iter_limit)
            seq += i["solve_seconds"]
            seq_it.append(i["iterations"])
    sec = statistics.median(times)
    it = [i["iterations"] for i in infos]
    # aggregate algorithmic traffic over the makespan: every instance's attempts times its bytes per
    # attempt (both sides of an attempt), all kernels of the batch together
    alg = sum(i["iterations"] * (algorithmic_bytes("dual", lp.m, lp.n, lp.nnz, 4) +
                                 algorithmic_bytes("primal", lp.m, lp.n, lp.nnz, 4)) for i, lp in zip(infos, lps))
    gbs = alg / sec / 1e9
    roofline = {"bound": "hbm", "achieved": round(gbs, 1), "peak": PEAK_HBM_GBS, "unit": "GB/s",
                "frac": round(gbs / PEAK_HBM_GBS, 4), "traffic": None,
                "kernel": "all iteration kernels of the batch: sum over instances of attempts x algorithmic bytes "
                          "per attempt (A x' + dual update, A'y' + primal update + averages), over the makespan",
                "alg_bytes_total": int(alg)}
    log(f"batch roofline: {json.dumps(roofline)}")
    cpu = None
    if not args.no_cpu_baseline:
        cpu = batch_cpu_baseline(lps, it)
        log(f"cpu baseline: {json.dumps(cpu)}")
    out = {"metric": "makespan to 1e-4 rel. KKT of a batch of LPs (FP32 PDLP)", "value": round(sec, 4), "unit": "s",
           "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(sec * 1e3, 2),
           "higher_is_better": False, "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
           "config": {"workload": f"{len(lps)} LPs (even: set cover, odd: multi-knapsack), m ~ U[1000, 50000], "
                                  f"n = 2.5 m, nnz={nnz}, batch seed {args.seed}", "tol": args.tol},
           "optimal": sum(i["status_name"] == "optimal" for i in infos), "iterations_max": max(it),
           "iterations_median": statistics.median(it), "sequential_s": round(seq, 3),
           "speedup_vs_sequential": round(seq / sec, 2), "create_s": round(create_s, 2),
           "roofline": roofline, "cpu_baseline": cpu}
    print(json.dumps(out), flush=True)


def batch_cpu_baseline(lps, iterations, every=8, n1=8, n2=136):
    """The FP64 oracle on a sample of the batch (every `every`-th instance): setup and per-attempt
    time from runs of n1 and n2 attempts, per-attempt time per (nnz + m + n) fitted by least squares
    over the sample, extrapolated to every instance's GPU attempt count and summed (the instances
    one after the other on the host's cores)."""
    import numpy as np
    import oracle
    xs, per, setup = [], [], []
    t_all = time.time()
    for k in range(0, len(lps), every):
        lp = lps[k]
        t = time.time()
        oracle.solve(lp, tol=0.0, iter_limit=n1)
        t1 = time.time() - t
        t = time.time()
        oracle.solve(lp, tol=0.0, iter_limit=n2)
        t2 = time.time() - t
        pa = (t2 - t1) / (n2 - n1)
        xs.append(lp.nnz + lp.m + lp.n)
        per.append(pa)
        setup.append(max(t1 - n1 * pa, 0.0))
    xs, per, setup = np.array(xs, float), np.array(per), np.array(setup)
    A = np.stack([np.ones_like(xs), xs], axis=1)
    cp = np.linalg.lstsq(A, per, rcond=None)[0]
    cs = np.linalg.lstsq(A, setup, rcond=None)[0]
    est = 0.0
    for lp, k in zip(lps, iterations):
        w = lp.nnz + lp.m + lp.n
        est += max(cs[0] + cs[1] * w, 0.0) + max(cp[0] + cp[1] * w, 0.0) * k
    return {"value": round(float(est), 2), "unit": "s", "cores": oracle.num_threads(), "kind": "oracle",
            "sample": (f"FP64 oracle (C, OpenMP row loops) on {len(xs)} of the {len(lps)} instances (one in {every}), "
                       f"{n1} and {n2} attempts each ({time.time() - t_all:.1f} s in all); setup and per-attempt time "
                       f"fitted linearly in nnz + m + n and summed over all instances with the GPU's attempt counts, "
                       f"solved one after the other; host CPU: {cpu_model()}")}


def bench_fixing(args):
    """LP-based variable strategies and LP-based fixing at the size of a full LP: time per call with
    the inputs resident in HBM (GPU tensors in and out: the figure reported as value), the same
    calls with host arrays (PCIe included), and the oracle (numpy) on the same inputs."""
    import numpy as np
    import torch
    from paper_2503_10344_amd import generators as g
    from paper_2503_10344_amd import pdlp
    import oracle.fix_oracle as fo
    torch.cuda.set_device(0)
    lp, desc = make_workload(args.fixing_lp, args.seed)
    d = g.fixing_inputs(args.seed, lp)
    dev = {k: torch.from_numpy(np.ascontiguousarray(v)).cuda() for k, v in d.items()}
    dl, du = torch.from_numpy(lp.l).cuda(), torch.from_numpy(lp.u).cuda()
    k = int(np.sum(d["var_type"] != 0))
    log(f"{desc}; {k} binary / integer variables (seeded types, point, duals, reduced costs)")
    combos = {"frac": (pdlp.ORDER_FRAC, pdlp.ORDER_NONE), "redcost": (pdlp.ORDER_REDCOST, pdlp.ORDER_NONE),
              "dual": (pdlp.ORDER_DUAL, pdlp.ORDER_NONE), "type": (pdlp.ORDER_TYPE, pdlp.ORDER_NONE),
              "frac+dual": (pdlp.ORDER_FRAC, pdlp.ORDER_DUAL), "frac+redcost": (pdlp.ORDER_FRAC, pdlp.ORDER_REDCOST)}

    def timed(fn):
        for _ in range(args.warmup):
            fn()
        ts, res = [], None
        for _ in range(args.steps):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            res = fn()
            torch.cuda.synchronize()
            ts.append(time.perf_counter() - t0)
        return 1e3 * statistics.median(ts), res

    out = {}
    p = pdlp.Problem(lp, precision="fp32")
    for name, (s_, t_) in combos.items():
        ms_dev, got_dev = timed(lambda: p.variable_strategy(s_, dev["var_type"], x=dev["x"], y=dev["y"],
                                                            rc=dev["rc"], tiebreak=t_))
        ms_host, got = timed(lambda: p.variable_strategy(s_, d["var_type"], x=d["x"], y=d["y"], rc=d["rc"],
                                                         tiebreak=t_))
        t0 = time.perf_counter()
        want = fo.variable_order(s_, t_, d["x"], d["y"], d["rc"], d["var_type"], lp.m, lp.n, lp.row_ptr, lp.col)
        cpu = time.perf_counter() - t0
        out[name] = {"ms": round(ms_dev, 3), "ms_host_arrays": round(ms_host, 3), "oracle_ms": round(1e3 * cpu, 1),
                     "equal_to_oracle": bool(np.array_equal(got, want) and np.array_equal(got_dev.cpu().numpy(), want))}
        log(f"{name}: {json.dumps(out[name])}")
    ms_dev, vals_dev = timed(lambda: p.lp_fixing(dev["var_type"], dev["x"], dl, du, dev["uniform"]))
    ms_host, vals = timed(lambda: p.lp_fixing(d["var_type"], d["x"], lp.l, lp.u, d["uniform"]))
    t0 = time.perf_counter()
    want = fo.lp_fixing(d["x"], d["var_type"], d["uniform"], lp.l, lp.u)
    fix = {"ms": round(ms_dev, 3), "ms_host_arrays": round(ms_host, 3),
           "oracle_ms": round(1e3 * (time.perf_counter() - t0), 1),
           "equal_to_oracle": bool(np.array_equal(vals, want) and np.array_equal(vals_dev.cpu().numpy(), want))}
    log(f"lp_fixing: {json.dumps(fix)}")
    p.close()
    res = {"metric": "LP-based variable strategy (Frac, ties by Dual) + LP-based fixing, time per call",
           "value": round(out["frac+dual"]["ms"] + fix["ms"], 3), "unit": "ms", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": round(out["frac+dual"]["ms"] + fix["ms"], 3),
           "higher_is_better": False, "scaling": "weak", "vs_baseline": None,
           "dtype": "f64 keys, int32 indices", "data": "synthetic",
           "config": {"workload": f"{desc}; {k} binary/integer variables",
                      "inputs": "resident in HBM (GPU tensors); ms_host_arrays: host arrays, PCIe included"},
           "orders": out, "lp_fixing": fix,
           "cpu_baseline": {"value": round(out["frac+dual"]["oracle_ms"] + fix["oracle_ms"], 1), "unit": "ms",
                            "cores": 1, "kind": "oracle",
                            "sample": "numpy oracle (lexsort, one thread) on the same inputs, one call each"}}
    print(json.dumps(res), flush=True)


def bench_propagation(args):
    """Linear-constraint propagation over a full LP's rows after fixings: time to the fixpoint with
    the bounds resident in HBM, per-round HBM throughput, and the C oracle on the same start."""
    import numpy as np
    import torch
    from paper_2503_10344_amd import generators as g
    from paper_2503_10344_amd import pdlp
    import oracle
    torch.cuda.set_device(0)
    lp, desc = make_workload(args.fixing_lp, args.seed)
    rng = np.random.default_rng([13, args.seed])
    l, u = lp.l.copy(), lp.u.copy()
    if args.fixing_lp == "zipf":
        vt = np.zeros(lp.n, np.uint8)  # continuous; 30 % of the columns fixed at the generator's feasible point
        pick = rng.random(lp.n) < 0.3
        l[pick] = lp.meta["x0"][pick]
        u[pick] = lp.meta["x0"][pick]
        start = "continuous columns, 30 % fixed at a feasible point"
    else:
        vt = g.fixing_inputs(args.seed, lp)["var_type"]
        start = "the LP's own bounds, seeded binary / integer types"
    max_rounds = 100
    prop = pdlp.Propagator(lp, vt)
    ts, res = [], None
    for s_ in range(args.warmup + args.steps):
        tl, tu = torch.from_numpy(l).cuda(), torch.from_numpy(u).cuda()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        res = prop.propagate(tl, tu, max_rounds)
        torch.cuda.synchronize()
        if s_ >= args.warmup:
            ts.append(time.perf_counter() - t0)
    prop.close()
    gl, gu, st, rounds = res
    t0 = time.perf_counter()
    ol, ou, ost, orr = oracle.propagate(lp, vt, l, u, max_rounds)
    cpu = time.perf_counter() - t0
    same = bool(np.array_equal(gl.cpu().numpy(), ol) and np.array_equal(gu.cpu().numpy(), ou) and (st, rounds) == (ost, orr))
    ms = 1e3 * statistics.median(ts)
    # algorithmic bytes of a round: two passes over each row (value, column, both bounds of the
    # column: 28 B per nonzero each), row offsets, b and sense, and the bound update (six 8-byte
    # vectors over the columns)
    per_round = 56 * lp.nnz + 13 * lp.m + 48 * lp.n
    gbs = per_round * rounds / (ms * 1e-3) / 1e9
    out = {"metric": "linear-constraint propagation to the fixpoint, time per call", "value": round(ms, 3), "unit": "ms",
           "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms, 3),
           "higher_is_better": False, "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
           "config": {"workload": f"{desc}; start: {start}", "max_rounds": max_rounds,
                      "inputs": "bounds resident in HBM (GPU tensors)"},
           "status": st, "rounds": rounds, "ms_per_round": round(ms / max(rounds, 1), 3),
           "bounds_moved": int(np.sum((ol != l) | (ou != u))), "equal_to_oracle": same,
           "roofline": {"bound": "hbm", "achieved": round(gbs, 1), "peak": PEAK_HBM_GBS, "unit": "GB/s",
                        "frac": round(gbs / PEAK_HBM_GBS, 4), "traffic": None,
                        "alg_bytes_per_round": per_round, "note": "wall time per round incl. the flag read-back"},
           "cpu_baseline": {"value": round(1e3 * cpu, 1), "unit": "ms", "cores": 1, "kind": "oracle",
                            "sample": f"C oracle (one thread), the same start, {orr} rounds"}}
    log(json.dumps(out))
    print(json.dumps(out), flush=True)


def bench_resolve(args):
    """Re-solves after fixings on the 256-LP batch: solve, fix from the LP solution (set cover: x >= 0.99
    to 1; multi-knapsack: x <= 0.01 to 0; both keep the LP feasible), update every instance's bounds,
    then re-solve cold and warm-started from the first solutions, next to a new batch made with the
    fixed bounds."""
    import numpy as np
    import torch
    from paper_2503_10344_amd import generators as g
    from paper_2503_10344_amd import pdlp
    t = time.time()
    lps = g.batch(args.seed, count=args.batch_count)
    log(f"{len(lps)} instances generated in {time.time() - t:.1f} s")

    def timed_solve(bt, **kw):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        infos = bt.solve(tol=args.tol, iter_limit=args.iter_limit, **kw)
        torch.cuda.synchronize()
        return time.perf_counter() - t0, infos

    b = pdlp.Batch(lps, precision="fp32")
    timed_solve(b)  # warm-up
    t_first, first = timed_solve(b)
    sols = [b.get(i) for i in range(len(lps))]
    fixed, nfix = [], 0
    for i, (lp, s_) in enumerate(zip(lps, sols)):
        l, u = lp.l.copy(), lp.u.copy()
        if i % 2 == 0:
            pick = s_.x >= 0.99
            l[pick] = 1.0
        else:
            pick = s_.x <= 0.01
            u[pick] = 0.0
        nfix += int(pick.sum())
        fixed.append(g.LP(lp.m, lp.n, lp.row_ptr, lp.col, lp.val, lp.c, lp.b, lp.sense, l, u))
    t0 = time.perf_counter()
    for i, fx in enumerate(fixed):
        b.update_bounds(i, fx.l, fx.u)
    t_update = time.perf_counter() - t0
    t_cold, cold = timed_solve(b)
    t_warm, warm = timed_solve(b, x0s=[s_.x for s_ in sols], y0s=[s_.y for s_ in sols],
                               omega0s=[f["omega"] for f in first])
    worst = max(i_["rel_kkt"] for i_ in warm)  # the library's FP64 re-evaluation of each returned point
    b.close()
    t0 = time.perf_counter()
    nb = pdlp.Batch(fixed, precision="fp32")
    torch.cuda.synchronize()
    t_create = time.perf_counter() - t0
    t_new, new = timed_solve(nb)
    nb.close()
    it = lambda infos: (max(i["iterations"] for i in infos), int(sum(i["iterations"] for i in infos)))  # noqa: E731
    res = {"metric": "makespan of re-solving a batch of LPs after fixings, warm-started from the first solve",
           "value": round(t_warm, 4), "unit": "s", "n_gpus": 1, "steps": 1, "warmup": 1, "ms_per_step": round(1e3 * t_warm, 2),
           "higher_is_better": False, "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
           "config": {"workload": f"{len(lps)} LPs of the batch workload (seed {args.seed}); {nfix} variables fixed from "
                                  "the first solution", "tol": args.tol},
           "first_solve_s": round(t_first, 4), "bound_update_s": round(t_update, 4),
           "resolve_cold_s": round(t_cold, 4), "resolve_warm_s": round(t_warm, 4),
           "new_batch_create_s": round(t_create, 3), "new_batch_solve_s": round(t_new, 4),
           "iterations_max_total": {"first": it(first), "cold": it(cold), "warm": it(warm), "new_batch": it(new)},
           "warm_used": int(sum(i["warm_started"] for i in warm)),
           "all_optimal": bool(all(i["status"] == pdlp.OPTIMAL for i in warm)),
           "worst_rel_kkt_warm": worst}
    log(json.dumps(res))
    print(json.dumps(res), flush=True)


def bench_snapshots(args, k=8, rel_tol=1e-3):
    """Reference snapshots on the general sparse LP: the FP32 solve to tol with and without keeping the
    newest k restart points of relative KKT error <= rel_tol (the solve itself is unchanged), the time
    to read them back, how far apart they are, and how many LP-based fixings each one changes against
    the final solution (the same seeded samples), i.e. how many distinct fix-and-propagate starts one
    solve yields."""
    import numpy as np
    import torch
    from paper_2503_10344_amd import generators as g
    from paper_2503_10344_amd import pdlp
    lp, desc = make_workload(args.fixing_lp, args.seed)
    d = g.fixing_inputs(args.seed, lp)
    p = pdlp.Problem(lp, precision="fp32")

    def timed_solve():
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        info = p.solve(tol=args.tol, iter_limit=args.iter_limit)
        torch.cuda.synchronize()
        return time.perf_counter() - t0, info

    t_off, info_off = timed_solve()
    x_off = p.get().x
    p.set_snapshots(k, rel_tol)
    t_on, info_on = timed_solve()
    sol = p.get()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    snaps = p.snapshots()
    t_get = time.perf_counter() - t0
    same = bool(info_on["iterations"] == info_off["iterations"] and np.array_equal(sol.x, x_off))
    log(f"solve without snapshots {t_off:.3f} s, with {t_on:.3f} s; {snaps.attempt.size} snapshots at "
        f"{list(map(int, snaps.attempt))}; read back in {t_get:.3f} s")
    nx = max(np.linalg.norm(sol.x), 1e-30)
    dist_final = [float(np.linalg.norm(snaps.x[q] - sol.x) / nx) for q in range(snaps.attempt.size)]
    dist_next = [float(np.linalg.norm(snaps.x[q + 1] - snaps.x[q]) / nx) for q in range(snaps.attempt.size - 1)]
    vt = d["var_type"]
    ints = vt != 0
    fix_final = p.lp_fixing(vt, sol.x, lp.l, lp.u, d["uniform"])
    changed = [int(np.sum(p.lp_fixing(vt, snaps.x[q], lp.l, lp.u, d["uniform"])[ints] != fix_final[ints]))
               for q in range(snaps.attempt.size)]
    p.close()
    over = t_on - t_off
    cpu = None
    if not args.no_cpu_baseline:
        import oracle
        n1, n2 = 8, 72
        t = time.time()
        oracle.solve(lp, tol=0.0, iter_limit=n1)
        t1 = time.time() - t
        t = time.time()
        oracle.solve(lp, tol=0.0, iter_limit=n2)
        t2 = time.time() - t
        t = time.time()
        for q in range(snaps.attempt.size):
            oracle.kkt(lp, snaps.x[q], snaps.y[q])
        t_kkt = time.time() - t
        per = (t2 - t1) / (n2 - n1)
        est = max(t1 - n1 * per, 0.0) + per * info_on["iterations"] + t_kkt
        cpu = {"value": round(est, 2), "unit": "s", "cores": oracle.num_threads(), "kind": "oracle",
               "sample": (f"FP64 oracle run for {n1} and {n2} attempts ({t1:.1f} s, {t2:.1f} s), extrapolated to "
                          f"{info_on['iterations']} attempts, plus its KKT evaluation of the {snaps.attempt.size} "
                          f"snapshots ({t_kkt:.1f} s); host CPU: {cpu_model()}")}
        log(f"cpu baseline: {json.dumps(cpu)}")
    res = {"metric": f"FP32 solve to {args.tol:g} rel. KKT keeping the newest {k} restart points with rel. KKT <= "
                     f"{rel_tol:g} as reference solutions",
           "value": round(t_on, 4), "unit": "s", "n_gpus": 1, "steps": 1, "warmup": 0,
           "ms_per_step": round(1e3 * t_on, 2), "higher_is_better": False, "scaling": "weak", "vs_baseline": None,
           "dtype": "f32", "data": "synthetic",
           "config": {"workload": f"{desc}; {int(ints.sum())} seeded binary/integer variables for the fixings",
                      "k": k, "rel_tol": rel_tol, "tol": args.tol},
           "solve_without_snapshots_s": round(t_off, 4), "overhead_s": round(over, 4),
           "overhead_frac": round(over / t_off, 4), "solve_unchanged": same,
           "iterations": info_on["iterations"], "read_back_s": round(t_get, 4),
           "snapshots": {"attempt": [int(a) for a in snaps.attempt],
                         "rel_kkt": [float("%.4g" % r) for r in snaps.rel_kkt],
                         "rel_dist_to_final": [float("%.4g" % v) for v in dist_final],
                         "rel_dist_to_next": [float("%.4g" % v) for v in dist_next],
                         "lp_fixings_changed_vs_final": changed},
           "roofline": None, "cpu_baseline": cpu}
    log(json.dumps(res))
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
