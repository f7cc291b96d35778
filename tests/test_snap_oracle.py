"""Pins of the reference-snapshot oracle (oracle/snap_oracle.py), CPU only.

* Restart schedule. With tol = 0 the artificial-restart criterion (attempts since the last restart
  at least 0.36 of all attempts) forces restarts at the first two evaluations, 64 and 128, and after
  any restart at r forces the next one no later than the first evaluation k = r + 64 j with
  64 j >= 0.36 k. Snapshots with rel_tol = inf are exactly the restart points, at multiples of the
  evaluation period.
* Restart to the average. When the attempt of a restart to the average was itself rejected, every
  iterate the average holds is in the trace, so the restart point must equal the mean of the
  iterates committed since the previous restart weighted by the step size each accepted attempt
  used (the trace's step size after the attempt before it). Recomputed here from the traced
  iterates; this fixes the weights, the reset of the weight sum at a restart and the choice of the
  average.
* Threshold and ring. rel_tol keeps exactly the restart points whose KKT error is at most rel_tol;
  k keeps the newest k of those, oldest first.
* Planted mistakes in a copy of the selection (wrong flag bit, ring kept from the front) fail a pin.
"""
import numpy as np
import pytest

import oracle
from oracle import snap_oracle as so
from paper_2503_10344_amd import generators as g

LPS = {
    "general": lambda: g.general_sparse(7, m=400, n=800, cap=200),
    "energy": lambda: g.energy(1, T=24, N=5, K=3, E=8),
    "knapsack": lambda: g.multi_knapsack(1, m=150, n=400),
}


def _schedule_ok(attempts, every=64):
    a = [int(v) for v in attempts]
    if a[:2] != [every, 2 * every] or any(v % every for v in a):
        return False
    for r, nxt in zip(a, a[1:]):
        k = r + every
        while (k - r) < 0.36 * k:
            k += every
        if nxt > k:
            return False
    return True


@pytest.mark.parametrize("name", sorted(LPS))
def test_restart_schedule(name):
    lp = LPS[name]()
    s = so.reference_snapshots(lp, k=100, rel_tol=np.inf, iter_limit=1024)
    _, att, _ = so.restart_points(lp, iter_limit=1024)
    assert np.array_equal(s.attempt, att) and len(att) >= 4
    assert _schedule_ok(s.attempt), list(s.attempt)
    # with a 32-attempt evaluation period the forced restarts are at 32 and 64
    s32 = so.reference_snapshots(lp, k=100, rel_tol=np.inf, iter_limit=512, eval_every=32)
    assert _schedule_ok(s32.attempt, 32), list(s32.attempt)


def _average_since(tr, prev, a):
    acc = [i for i in range(prev + 1, a) if tr["flags"][i - 1] & so.ACCEPTED]
    w = np.array([tr["eta"][i - 2] for i in acc])
    xb = (w[:, None] * np.array([tr["x"][i - 1] for i in acc])).sum(0) / w.sum()
    yb = (w[:, None] * np.array([tr["y"][i - 1] for i in acc])).sum(0) / w.sum()
    return xb, yb, len(acc)


def test_restart_to_average_is_the_weighted_mean():
    lp = LPS["general"]()
    s = so.reference_snapshots(lp, k=100, rel_tol=np.inf, iter_limit=512)
    tr = s.result.trace
    i = int(np.nonzero(s.attempt == 512)[0][0])
    prev, a = int(s.attempt[i - 1]), 512
    assert s.to_average[i] and not (tr["flags"][a - 1] & so.ACCEPTED)  # the case this pin needs
    xb, yb, nacc = _average_since(tr, prev, a)
    assert nacc > 100
    ex = np.linalg.norm(xb - s.x[i]) / np.linalg.norm(s.x[i])
    ey = np.linalg.norm(yb - s.y[i]) / np.linalg.norm(s.y[i])
    # a mean of ~190 FP64 vectors and the oracle's running update differ by rounding only
    assert ex < 1e-13 and ey < 1e-13, (ex, ey)
    # the current iterate at that restart is not the restart point (the choice matters)
    cur = tr["x"][a - 2]
    assert np.linalg.norm(cur - s.x[i]) > 1e-6 * np.linalg.norm(s.x[i])


@pytest.mark.parametrize("name", sorted(LPS))
def test_threshold_and_ring(name):
    lp = LPS[name]()
    full = so.reference_snapshots(lp, k=100, rel_tol=np.inf, iter_limit=1024)
    for q, a in enumerate(full.attempt):
        assert full.rel_kkt[q] == oracle.kkt(lp, full.x[q], full.y[q])["rel_kkt"]
    tol = float(np.median(full.rel_kkt))
    sel = so.reference_snapshots(lp, k=100, rel_tol=tol, iter_limit=1024)
    assert np.array_equal(sel.attempt, full.attempt[full.rel_kkt <= tol])
    assert np.all(sel.rel_kkt <= tol)
    two = so.reference_snapshots(lp, k=2, rel_tol=tol, iter_limit=1024)
    assert np.array_equal(two.attempt, sel.attempt[-2:])
    assert np.array_equal(two.x, sel.x[-2:]) and np.array_equal(two.y, sel.y[-2:])
    none = so.reference_snapshots(lp, k=0, rel_tol=tol, iter_limit=1024)
    assert none.attempt.size == 0 and none.x.shape == (0, lp.n)
    # distinct points: the method keeps moving between restarts
    d = [np.linalg.norm(full.x[q + 1] - full.x[q]) for q in range(len(full.attempt) - 1)]
    assert min(d) > 0.0


def test_pins_catch_planted_mistakes(monkeypatch):
    lp = LPS["general"]()
    # reading the accepted bit instead of the restarted bit
    monkeypatch.setattr(so, "RESTARTED", so.ACCEPTED)
    s = so.reference_snapshots(lp, k=100, rel_tol=np.inf, iter_limit=512)
    assert not _schedule_ok(s.attempt)
    monkeypatch.setattr(so, "RESTARTED", 4)
    # keeping the oldest k instead of the newest k
    orig = so.reference_snapshots

    def oldest_first(lp_, k, rel_tol, **kw):
        r = orig(lp_, 100, rel_tol, **kw)
        return so.Snapshots(r.attempt[:k], r.x[:k], r.y[:k], r.rel_kkt[:k], r.to_average[:k], r.result)

    full = orig(lp, 100, np.inf, iter_limit=512)
    bad = oldest_first(lp, 2, np.inf, iter_limit=512)
    assert not np.array_equal(bad.attempt, full.attempt[-2:])
