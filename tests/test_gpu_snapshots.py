"""Reference snapshots (pdlp_set_snapshots / pdlp_get_snapshots) against the oracle.

* FP64 tracks the oracle: the restart points the GPU keeps (rel_tol = inf) are taken at the same
  attempts as the oracle's and equal them within the tracking bound (tests/tracking.py: twice the
  oracle's own divergence under other summation orders, at least 1e-9), up to the first discrete
  decision whose margin that divergence could flip; a finite rel_tol keeps the same attempts as the
  oracle's selection.
* Taking snapshots does not change the solve (bitwise, FP32 and FP64); the ring keeps the newest k;
  a batch instance's snapshots are bitwise the single solve's; argument and order errors.
* Full size (500k x 1M, FP32, 1e-4): every snapshot's KKT error, re-evaluated by the oracle, matches
  the one the solve measured, and the points respect bounds and dual signs.
"""
import ctypes
import sys

import numpy as np
import pytest

import oracle
import tracking
from oracle import snap_oracle as so

try:  # import at collection time: the first import on a fresh machine can take a minute
    import torch  # noqa: F401
except Exception:  # pragma: no cover
    torch = None
from paper_2503_10344_amd import generators as g

pytestmark = pytest.mark.gpu


def say(*a):
    print("[gpu-test]", *a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def pdlp():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2503_10344_amd import pdlp as mod
    mod.load()
    return mod


@pytest.mark.parametrize("name", ["general", "energy", "knapsack"])
def test_snapshots_track_the_oracle_fp64(pdlp, name):
    lp = {"general": lambda: g.general_sparse(7, m=400, n=800, cap=200),
          "energy": lambda: g.energy(1, T=24, N=5, K=3, E=8),
          "knapsack": lambda: g.multi_knapsack(1, m=150, n=400)}[name]()
    K = 1024
    ref = so.reference_snapshots(lp, k=100, rel_tol=np.inf, iter_limit=K)
    tr = ref.result.trace
    bound = tracking.tracking_bound(lp, K, tr)
    risky = np.nonzero(tr["margin"] < np.maximum(1e-12, 100.0 * bound))[0]
    cut = int(risky[0]) + 1 if risky.size else K + 1  # first attempt whose decision could flip
    with pdlp.Problem(lp, precision="fp64", tile_nnz=1024, warm_fallback=False) as p:
        p.set_snapshots(64, np.inf)
        p.solve(tol=0.0, iter_limit=K)
        s = p.snapshots()
    n_cmp = int(np.sum(ref.attempt < cut))
    say(name, "oracle restarts", list(ref.attempt), "gpu", list(s.attempt), "compared before attempt", cut)
    assert n_cmp >= 2
    assert np.array_equal(s.attempt[:n_cmp], ref.attempt[:n_cmp])
    for q in range(n_cmp):
        a = int(ref.attempt[q])
        ex = np.linalg.norm(s.x[q] - ref.x[q]) / max(np.linalg.norm(ref.x[q]), 1e-30)
        ey = np.linalg.norm(s.y[q] - ref.y[q]) / max(np.linalg.norm(ref.y[q]), 1e-30)
        assert max(ex, ey) <= bound[a - 1], (name, a, ex, ey, bound[a - 1])
        assert abs(s.rel_kkt[q] - ref.rel_kkt[q]) <= 1e-4 * ref.rel_kkt[q] + 1e-9, (a, s.rel_kkt[q], ref.rel_kkt[q])
    # a finite threshold between two of the compared KKT errors keeps the oracle's attempts
    r = np.sort(ref.rel_kkt[:n_cmp])
    gaps = [(r[i + 1] / r[i], i) for i in range(len(r) - 1) if r[i] > 0]
    ratio, i = max(gaps)
    assert ratio > 1.01
    tol = float(np.sqrt(r[i] * r[i + 1]))
    with pdlp.Problem(lp, precision="fp64", tile_nnz=1024, warm_fallback=False) as p:
        p.set_snapshots(64, tol)
        p.solve(tol=0.0, iter_limit=K)
        st = p.snapshots()
    want = ref.attempt[:n_cmp][ref.rel_kkt[:n_cmp] <= tol]
    assert np.array_equal(st.attempt[: want.size], want), (list(st.attempt), list(want))


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_snapshots_do_not_change_the_solve(pdlp, prec):
    lp = g.general_sparse(7, m=3000, n=6000, cap=1000)
    with pdlp.Problem(lp, precision=prec, tile_nnz=1024) as p:
        a = p.solve(tol=1e-4, iter_limit=400_000)
        sa = p.get()
    with pdlp.Problem(lp, precision=prec, tile_nnz=1024) as p:
        p.set_snapshots(6, 1e-2)
        b = p.solve(tol=1e-4, iter_limit=400_000)
        sb = p.get()
        s = p.snapshots()
    say(prec, "iterations", a["iterations"], b["iterations"], "snapshots at", list(s.attempt),
        "rel", ["%.2e" % v for v in s.rel_kkt])
    assert a["iterations"] == b["iterations"] and a["status"] == b["status"] == pdlp.OPTIMAL
    assert np.array_equal(sa.x, sb.x) and np.array_equal(sa.y, sb.y)
    assert 1 <= s.attempt.size <= 6
    assert np.all(np.diff(s.attempt) > 0) and np.all(s.attempt % 64 == 0) and s.attempt[-1] <= b["iterations"]
    assert np.all(s.rel_kkt <= 1e-2)
    for q in range(s.attempt.size):
        k = oracle.kkt(lp, s.x[q], s.y[q])["rel_kkt"]
        # FP64 evaluates the same point; FP32 evaluated FP32 products (and the FP32 data)
        slack = 1e-9 if prec == "fp64" else 2e-2
        assert abs(k - s.rel_kkt[q]) <= slack * s.rel_kkt[q] + 1e-6, (q, k, s.rel_kkt[q])


def test_ring_batch_and_errors(pdlp):
    lps = [g.general_sparse(7, m=400, n=800, cap=200), g.energy(1, T=24, N=5, K=3, E=8),
           g.multi_knapsack(1, m=150, n=400)]
    with pdlp.Batch(lps, precision="fp32", tile_nnz=1024) as bt:
        bt.set_snapshots(8, np.inf)
        bt.solve(tol=0.0, iter_limit=1024)
        got8 = [bt.snapshots(i) for i in range(3)]
        two = bt.snapshots(1, cap=2)
        bt.set_snapshots(2, np.inf)
        bt.solve(tol=0.0, iter_limit=1024)
        got2 = [bt.snapshots(i) for i in range(3)]
        cnt = ctypes.c_int32(0)  # instance index out of range, through the C ABI
        assert pdlp.load().pdlp_batch_get_snapshots(bt.h, 3, 4, None, None, None, None, ctypes.byref(cnt)) == -1
    for i, lp in enumerate(lps):
        with pdlp.Problem(lp, precision="fp32", tile_nnz=1024) as p:
            p.set_snapshots(8, np.inf)
            p.solve(tol=0.0, iter_limit=1024)
            one = p.snapshots()
        say("instance", i, "batch", list(got8[i].attempt), "single", list(one.attempt))
        assert np.array_equal(got8[i].attempt, one.attempt)
        assert np.array_equal(got8[i].x, one.x) and np.array_equal(got8[i].y, one.y)
        assert np.array_equal(got8[i].rel_kkt, one.rel_kkt)
        # a 2-slot ring holds the newest two, oldest first
        assert np.array_equal(got2[i].attempt, one.attempt[-2:])
        assert np.array_equal(got2[i].x, one.x[-2:]) and np.array_equal(got2[i].y, one.y[-2:])
    assert np.array_equal(two.attempt, got8[1].attempt[-2:]) and np.array_equal(two.x, got8[1].x[-2:])
    with pdlp.Problem(lps[0], precision="fp32") as p:
        with pytest.raises(pdlp.PDLPError):
            p.snapshots(cap=4)                # before a solve
        with pytest.raises(pdlp.PDLPError):
            p.set_snapshots(-1, 1e-3)
        with pytest.raises(pdlp.PDLPError):
            p.set_snapshots(4, np.nan)
        p.set_snapshots(4, 1e-3)
        p.solve(tol=1e-4)
        cnt = ctypes.c_int32(0)  # negative cap, through the C ABI
        assert pdlp.load().pdlp_get_snapshots(p.h, -1, None, None, None, None, ctypes.byref(cnt)) == -1
        p.set_snapshots(0, 1e-3)              # off: the next solve keeps none
        p.solve(tol=1e-4)
        assert p.snapshots(cap=4).attempt.size == 0


def test_full_size_snapshots(pdlp):
    lp = g.general_sparse(0)
    with pdlp.Problem(lp, precision="fp32") as p:
        p.set_snapshots(4, 1e-3)
        info = p.solve(tol=1e-4)
        s = p.snapshots()
    say("500k x 1M: iterations", info["iterations"], "snapshots at", list(s.attempt),
        "rel", ["%.2e" % v for v in s.rel_kkt])
    assert info["status"] == pdlp.OPTIMAL and 1 <= s.attempt.size <= 4
    lo, hi = lp.l, lp.u
    tol = 1e-6 * np.maximum(1.0, np.abs(np.where(np.isfinite(hi), hi, lo)))
    for q in range(s.attempt.size):
        k = oracle.kkt(lp, s.x[q], s.y[q])["rel_kkt"]
        say("snapshot", int(s.attempt[q]), "measured %.4e oracle %.4e" % (s.rel_kkt[q], k))
        assert abs(k - s.rel_kkt[q]) <= 2e-2 * s.rel_kkt[q] + 1e-6
        x, y = s.x[q], s.y[q]
        assert np.all(x >= lo - tol) and np.all(x <= hi + tol)
        assert np.all(y[lp.sense == ord("L")] <= 0.0) and np.all(y[lp.sense == ord("G")] >= 0.0)
    for q in range(s.attempt.size - 1):
        assert np.linalg.norm(s.x[q + 1] - s.x[q]) > 0.0
