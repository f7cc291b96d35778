"""Reference snapshots of the oracle's PDLP solve (test infrastructure).

TEST INFRASTRUCTURE ONLY: the test suite uses this module; the GPU library never does, and it
shares no code with it.

The paper's conclusion (section 5) proposes taking several LP reference solutions for
fix-and-propagate from the cycling convergence of PDLP, and gives no rule for it. The reading taken
here: a snapshot is a restart point of the solve, i.e. the candidate (current iterate or average)
that the restarted method moves to at an evaluation, kept when its relative KKT error in the
original space is at most rel_tol; of those, the newest k are kept, oldest first.

The oracle's solve records the committed iterate after every attempt (original space), after a
restart has moved it, and flags the attempts at which a restart happened. So the restart points are
the traced iterates at the flagged attempts; each is re-evaluated with the oracle's KKT function.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from . import kkt, solve

RESTARTED, TO_AVERAGE, ACCEPTED = 4, 8, 1


@dataclass
class Snapshots:
    attempt: np.ndarray   # [count] attempt count at which each restart point was taken
    x: np.ndarray         # [count, n] original space
    y: np.ndarray         # [count, m]
    rel_kkt: np.ndarray   # [count] relative KKT error (oracle KKT evaluation)
    to_average: np.ndarray  # [count] whether the restart moved to the average
    result: object        # the oracle solve (with its full trace)


def restart_points(lp, tol: float = 0.0, iter_limit: int = 512, eval_every: int = 64):
    """Every restart point of the oracle's solve: (solve result, attempts, to_average flags)."""
    res = solve(lp, tol=tol, iter_limit=iter_limit, eval_every=eval_every, trace_len=iter_limit)
    flags = res.trace["flags"][: res.iterations]
    idx = np.nonzero(flags & RESTARTED)[0]
    return res, idx + 1, (flags[idx] & TO_AVERAGE) != 0


def reference_snapshots(lp, k: int, rel_tol: float, tol: float = 0.0, iter_limit: int = 512,
                        eval_every: int = 64) -> Snapshots:
    """The newest k restart points with relative KKT error <= rel_tol, oldest first."""
    res, attempts, to_avg = restart_points(lp, tol, iter_limit, eval_every)
    tr = res.trace
    keep = []
    for a, av in zip(attempts, to_avg):
        x, y = tr["x"][a - 1], tr["y"][a - 1]
        r = kkt(lp, x, y)["rel_kkt"]
        if r <= rel_tol:
            keep.append((a, x, y, r, av))
    keep = keep[-k:] if k > 0 else []
    if not keep:
        return Snapshots(np.zeros(0, np.int64), np.zeros((0, lp.n)), np.zeros((0, lp.m)), np.zeros(0),
                         np.zeros(0, bool), res)
    return Snapshots(np.array([q[0] for q in keep], np.int64), np.array([q[1] for q in keep]),
                     np.array([q[2] for q in keep]), np.array([q[3] for q in keep]),
                     np.array([q[4] for q in keep]), res)
