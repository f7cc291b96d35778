"""Learned warm start for PDLP: training data from solver runs, training, warm-started solves.

Pipeline (all arithmetic in the HIP library):
  1. make_shards: draw LPs of the energy-shaped family, solve them to the tolerance with the batched
     FP32 solver, keep each batch handle together with its solutions (x*, y*) and final primal
     weights omega* as training targets.
  2. train: Adam over the shards (one shard = one minibatch), shuffled each epoch.
  3. warm_solve: predict (x0, y0, omega0) for a problem and solve from there. The solver itself
     discards a predicted point whose relative KKT error is not below the cold start's; a warm solve
     that runs out of its iteration budget is repeated from the cold start (both counted).

Command line:  python -m paper_2503_10344_amd.warmstart --train 2000 --out weights.npz
"""
from __future__ import annotations

import argparse
import json
import os
import statistics
import sys
import time
from dataclasses import dataclass, field

import numpy as np

from . import generators as gen
from . import pdlp

TRAIN_SEEDS = (0, 20_000)
VAL_SEEDS = (20_000, 21_000)
TEST_SEEDS = (1_000_000, 1_000_200)
# which predicted parts seed the solve: all, omega alone, x and omega, y and omega, x and y
MODES = ("full", "omega", "primal_omega", "dual_omega", "primal_dual")


WEIGHTS = os.path.join(os.path.dirname(os.path.abspath(__file__)), "weights", "warmstart_energy.npz")


def load_trained(path: str = WEIGHTS):
    """The committed trained network and the warm-start mode chosen on the validation seeds."""
    with np.load(path, allow_pickle=False) as f:
        params, mode = f["params"], str(f["mode"])
    return pdlp.WarmStartNet(params=params), mode


def _log(*a):
    print("[warmstart]", *a, file=sys.stderr, flush=True)


@dataclass
class Shard:
    batch: pdlp.Batch
    seeds: list
    x: np.ndarray
    y: np.ndarray
    omega: np.ndarray
    iterations: list = field(default_factory=list)
    converged: list = field(default_factory=list)


def family(seed: int, m_lo: int, m_hi: int):
    return gen.warmstart_family(seed, m_lo=m_lo, m_hi=m_hi)


def make_shards(seeds, per_shard=16, tol=1e-4, iter_limit=100_000, m_lo=10_000, m_hi=100_000, log=_log):
    """Solve the instances in batches; each batch handle becomes one training minibatch."""
    shards = []
    seeds = list(seeds)
    t0 = time.time()
    for s in range(0, len(seeds), per_shard):
        ss = seeds[s:s + per_shard]
        lps = [family(q, m_lo, m_hi) for q in ss]
        b = pdlp.Batch(lps, precision="fp32")
        infos = b.solve(tol=tol, iter_limit=iter_limit)
        sols = [b.get(i) for i in range(len(lps))]
        shards.append(Shard(b, ss, np.concatenate([v.x for v in sols]), np.concatenate([v.y for v in sols]),
                            np.array([i["omega"] for i in infos]), [i["iterations"] for i in infos],
                            [i["status_name"] == "optimal" for i in infos]))
        if log and (len(shards) % 10 == 0 or s + per_shard >= len(seeds)):
            log(f"solved {s + len(ss)}/{len(seeds)} instances ({time.time() - t0:.1f} s)")
    return shards


def train(net: pdlp.WarmStartNet, shards, epochs=30, lr=1e-3, seed=0, schedule="constant", log=_log):
    """Adam over the shards; schedule "constant" keeps lr, "cosine" decays it to lr/20."""
    rng = np.random.default_rng(seed)
    hist = []
    for ep in range(epochs):
        t = time.time()
        lr_ep = lr
        if schedule == "cosine":
            lr_ep = lr * (0.05 + 0.95 * 0.5 * (1.0 + np.cos(np.pi * ep / max(epochs, 1))))
        losses = [net.train_step(shards[k].batch, shards[k].x, shards[k].y, shards[k].omega, lr=lr_ep)
                  for k in rng.permutation(len(shards))]
        hist.append(float(np.mean(losses)))
        if log:
            log(f"epoch {ep}: mean loss {hist[-1]:.4g} ({time.time() - t:.1f} s)")
    return hist


def validation_loss(net, shards):
    return float(np.mean([net.gradients(s.batch, s.x, s.y, s.omega)[0] for s in shards]))


def warm_solve(net, problem: pdlp.Problem, tol=1e-4, iter_limit=100_000, mode="full") -> dict:
    """Predict a start and solve from it; inference time is part of the reported time."""
    if mode == "cold":
        info = problem.solve(tol=tol, iter_limit=iter_limit)
        return dict(iterations=info["iterations"], seconds=info["solve_seconds"], predict_seconds=0.0,
                    status=info["status_name"], fallback=True, rel_kkt=info["rel_kkt"],
                    primal_obj=info["primal_obj"])
    if mode not in MODES:
        raise ValueError(f"unknown warm-start mode {mode}")
    t = time.perf_counter()
    x0, y0, om = net.predict(problem)
    t_pred = time.perf_counter() - t
    if mode in ("omega", "dual_omega"):
        x0 = None
    if mode in ("omega", "primal_omega"):
        y0 = None
    if mode == "primal_dual":
        om = 0.0
    info = problem.solve(tol=tol, iter_limit=iter_limit, x0=x0, y0=y0, omega0=om)
    iters, secs = info["iterations"], t_pred + info["solve_seconds"]
    rerun = False
    if info["status_name"] != "optimal":
        cold = problem.solve(tol=tol, iter_limit=iter_limit)
        iters += cold["iterations"]
        secs += cold["solve_seconds"]
        rerun, info = True, cold
    return dict(iterations=iters, seconds=secs, predict_seconds=t_pred, status=info["status_name"],
                fallback=bool(info.get("fallback_used", 0)) or rerun, rel_kkt=info["rel_kkt"],
                primal_obj=info["primal_obj"])


def warm_solve_batch(net, batch: pdlp.Batch, tol=1e-4, iter_limit=100_000, mode="full") -> list:
    """Predict starts for every instance of a batch in one pass and solve them together; instances
    that end at the budget are not repeated here (per-instance results carry the status)."""
    if mode not in MODES and mode != "cold":
        raise ValueError(f"unknown warm-start mode {mode}")
    if mode == "cold":
        return batch.solve(tol=tol, iter_limit=iter_limit)
    x0, y0, om = net.predict(batch)
    xs, ys, co, ro = [], [], 0, 0
    for m, n in batch.dims:
        xs.append(x0[co:co + n] if mode not in ("omega", "dual_omega") else None)
        ys.append(y0[ro:ro + m] if mode not in ("omega", "primal_omega") else None)
        co += n
        ro += m
    oms = om if mode != "primal_dual" else None
    if all(v is None for v in xs):
        xs = None
    if all(v is None for v in ys):
        ys = None
    return batch.solve(tol=tol, iter_limit=iter_limit, x0s=xs, y0s=ys, omega0s=oms)


def evaluate(net, seeds, tol=1e-4, iter_limit=100_000, modes=MODES, m_lo=10_000, m_hi=100_000, log=_log):
    """Cold vs warm on each instance (same handle, cold first)."""
    rows = []
    t0 = time.time()
    for k, s in enumerate(seeds):
        lp = family(s, m_lo, m_hi)
        with pdlp.Problem(lp, precision="fp32") as p:
            cold = p.solve(tol=tol, iter_limit=iter_limit)
            row = dict(seed=s, m=lp.m, n=lp.n, cold_iterations=cold["iterations"], cold_seconds=cold["solve_seconds"],
                       cold_status=cold["status_name"], cold_obj=cold["primal_obj"])
            for mode in modes:
                w = warm_solve(net, p, tol, iter_limit, mode)
                row.update({f"{mode}_{k2}": v for k2, v in w.items()})
        rows.append(row)
        if log and ((k + 1) % 25 == 0 or k + 1 == len(seeds)):
            log(f"evaluated {k + 1}/{len(seeds)} ({time.time() - t0:.1f} s)")
    return rows


def summarize(rows, modes=MODES):
    out = dict(instances=len(rows),
               cold_median_iterations=statistics.median(r["cold_iterations"] for r in rows),
               cold_median_seconds=statistics.median(r["cold_seconds"] for r in rows))
    for mode in modes:
        it = [r[f"{mode}_iterations"] for r in rows]
        sec = [r[f"{mode}_seconds"] for r in rows]
        ratio = [r[f"{mode}_iterations"] / max(r["cold_iterations"], 1) for r in rows]
        out[mode] = dict(median_iterations=statistics.median(it), median_seconds=statistics.median(sec),
                         median_iteration_ratio=statistics.median(ratio),
                         geomean_iteration_ratio=float(np.exp(np.mean(np.log(ratio)))),
                         total_iteration_ratio=sum(it) / max(sum(r["cold_iterations"] for r in rows), 1),
                         total_seconds_ratio=sum(sec) / max(sum(r["cold_seconds"] for r in rows), 1e-30),
                         fallback_rate=float(np.mean([r[f"{mode}_fallback"] for r in rows])),
                         faster_fraction=float(np.mean([r[f"{mode}_iterations"] < r["cold_iterations"] for r in rows])))
    return out


def choose_mode(val):
    """The mode with the smallest total solve time on the validation seeds (inference included:
    what a caller of many solves pays); cold if no mode beats the cold start."""
    best = min(MODES, key=lambda md: (val[md]["total_seconds_ratio"], md))
    return best if val[best]["total_seconds_ratio"] < 1.0 else "cold"


def main(argv=None):
    ap = argparse.ArgumentParser(description="train and evaluate the learned PDLP warm start")
    ap.add_argument("--train", type=int, default=2000, help="training instances (seeds 0..N-1)")
    ap.add_argument("--val", type=int, default=200, help="validation instances (loss and mode choice)")
    ap.add_argument("--test", type=int, default=200)
    ap.add_argument("--per-shard", type=int, default=16)
    ap.add_argument("--epochs", type=int, default=30)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--schedule", default="constant", choices=["constant", "cosine"])
    ap.add_argument("--omega-weight", type=float, default=10.0, help="weight of the log-omega loss term")
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--m-lo", type=int, default=10_000)
    ap.add_argument("--m-hi", type=int, default=100_000)
    ap.add_argument("--tol", type=float, default=1e-4)
    ap.add_argument("--out", default=None, help="write the trained parameters here (.npz)")
    ap.add_argument("--report", default=None, help="write the JSON report here")
    ap.add_argument("--evaluate", default=None, metavar="WEIGHTS",
                    help="only evaluate these trained weights (.npz) on the held-out seeds, in their mode")
    ap.add_argument("--reselect", default=None, metavar="OUT",
                    help="with --evaluate: choose the mode again on the validation seeds, save to OUT (.npz)")
    args = ap.parse_args(argv)

    if args.evaluate:
        net, mode = load_trained(args.evaluate)
        if args.reselect:
            # choose the mode again on the validation seeds (the solver may have changed since)
            val_rows = evaluate(net, range(VAL_SEEDS[0], VAL_SEEDS[0] + args.val), args.tol,
                                m_lo=args.m_lo, m_hi=args.m_hi)
            val = summarize(val_rows)
            mode = choose_mode(val)
            _log(f"validation: {json.dumps(val)}; chosen mode {mode}")
            np.savez(args.reselect, params=net.params(), mode=np.array(mode))
        modes = tuple(dict.fromkeys((mode, "full", "omega")))
        rows = evaluate(net, range(TEST_SEEDS[0], TEST_SEEDS[0] + args.test), args.tol, modes=modes,
                        m_lo=args.m_lo, m_hi=args.m_hi)
        report = dict(weights=args.evaluate, mode=mode, test=summarize(rows, modes=modes), tol=args.tol,
                      m_range=[args.m_lo, args.m_hi])
        if args.reselect:
            report["validation"] = val
        print(json.dumps(report), flush=True)
        if args.report:
            with open(args.report, "w") as f:
                json.dump(dict(report, test_rows=rows), f)
        return

    t = time.time()
    shards = make_shards(range(TRAIN_SEEDS[0], TRAIN_SEEDS[0] + args.train), args.per_shard, args.tol,
                         m_lo=args.m_lo, m_hi=args.m_hi)
    gen_s = time.time() - t
    vshards = make_shards(range(VAL_SEEDS[0], VAL_SEEDS[0] + args.val), args.per_shard, args.tol,
                          m_lo=args.m_lo, m_hi=args.m_hi, log=None)
    net = pdlp.WarmStartNet(seed=args.seed, omega_weight=args.omega_weight)
    v0 = validation_loss(net, vshards)
    t = time.time()
    hist = train(net, shards, args.epochs, args.lr, args.seed, args.schedule)
    train_s = time.time() - t
    v1 = validation_loss(net, vshards)
    _log(f"validation loss {v0:.4g} -> {v1:.4g}")
    del shards
    val_rows = evaluate(net, range(VAL_SEEDS[0], VAL_SEEDS[0] + args.val), args.tol,
                        m_lo=args.m_lo, m_hi=args.m_hi)
    val = summarize(val_rows)
    best = choose_mode(val)
    _log(f"validation: {json.dumps(val)}; chosen mode {best}")
    # held-out: the chosen mode, plus the two single-choice modes for context
    test_modes = tuple(dict.fromkeys((best, "full", "omega")))
    test_rows = evaluate(net, range(TEST_SEEDS[0], TEST_SEEDS[0] + args.test), args.tol, modes=test_modes,
                         m_lo=args.m_lo, m_hi=args.m_hi)
    test = summarize(test_rows, modes=test_modes)
    report = dict(train_instances=args.train, epochs=args.epochs, lr=args.lr, schedule=args.schedule,
                  omega_weight=args.omega_weight,
                  data_seconds=round(gen_s, 1),
                  train_seconds=round(train_s, 1), loss_history=hist, val_loss_before=v0, val_loss_after=v1,
                  validation=val, mode=best, test=test, m_range=[args.m_lo, args.m_hi], tol=args.tol)
    print(json.dumps(report), flush=True)
    if args.out:
        np.savez(args.out, params=net.params(), mode=np.array(best))
    if args.report:
        with open(args.report, "w") as f:
            json.dump(dict(report, test_rows=test_rows, validation_rows=val_rows), f)


if __name__ == "__main__":
    main()
