"""LP-based variable strategies and LP-based fixing, plain numpy in FP64 (test infrastructure).

TEST INFRASTRUCTURE ONLY: the test suite and the benchmark's CPU leg use this module; the GPU
library never does, and it shares no code with it.

What it computes follows section 2 of the paper ("LP-based variable strategies", "LP-based fixing",
"Tiebreaking and hybrid strategies"). The paper states the keys but not every direction or tie rule;
the readings taken here:
  * Only binary and integer variables are ordered; continuous ones are left out.
  * Frac: ascending fractionality frac_j = min(x_j - floor x_j, ceil x_j - x_j), i.e. the most nearly
    integral variables first (fractionality as confidence).
  * RedCost: descending |r_j| (high absolute reduced cost first).
  * Dual: constraints in descending |y_i| (equal |y_i|: lower row index first); walking them in that
    order, each constraint contributes the integer variables it contains that no earlier constraint
    contributed, and each contribution is ordered by RedCost. Variables in no constraint come last, in
    RedCost order. Equivalently, a variable's group is the smallest rank of a constraint containing it.
  * Type: binaries first, then integers (stable).
  * A tiebreak strategy orders what the primary strategy ranks equally; when every key is equal the
    lower variable index comes first.
  * LP-based fixing: d_j = x_j - floor x_j; with one uniform sample s_j in (0, 1) per variable
    (supplied by the caller), the fixing value is floor x_j if s_j > d_j, else ceil x_j, then clamped
    to [ceil l_j, floor u_j]. Continuous variables keep x_j.
"""
from __future__ import annotations

import numpy as np

CONTINUOUS, BINARY, INTEGER = 0, 1, 2
NONE, FRAC, REDCOST, DUAL, TYPE = 0, 1, 2, 3, 4
NAMES = {FRAC: "frac", REDCOST: "redcost", DUAL: "dual", TYPE: "type"}


def fractionality(x):
    """Distance of each value to the nearest integer (section 2, Frac)."""
    x = np.asarray(x, np.float64)
    return np.minimum(x - np.floor(x), np.ceil(x) - x)


def dual_groups(m, n, row_ptr, col, y):
    """Rank of the first constraint, in descending |y| order, that contains each variable (m if the
    column is empty): the grouping of the Dual strategy."""
    rows = np.arange(m)
    order = np.lexsort((rows, -np.abs(np.asarray(y, np.float64))))  # |y| descending, index ascending
    rank = np.empty(m, np.int64)
    rank[order] = np.arange(m)
    row_of = np.repeat(rows, np.diff(np.asarray(row_ptr, np.int64)))
    group = np.full(n, m, np.int64)
    np.minimum.at(group, np.asarray(col, np.int64), rank[row_of])
    return group


def _keys(strategy, x, rc, vtype, group):
    """Sort keys of one strategy, most significant first, each ascending."""
    if strategy == FRAC:
        return [fractionality(x)]
    if strategy == REDCOST:
        return [-np.abs(rc)]
    if strategy == DUAL:
        return [group, -np.abs(rc)]
    if strategy == TYPE:
        return [vtype.astype(np.int64)]
    if strategy == NONE:
        return []
    raise ValueError(f"unknown strategy {strategy}")


def variable_order(strategy, tiebreak, x, y, rc, var_type, m, n, row_ptr, col):
    """Indices of the binary and integer variables in the order the strategy (ties broken by the
    tiebreak strategy, then by index) fixes them."""
    vtype = np.asarray(var_type, np.uint8)
    if strategy not in NAMES or (tiebreak not in NAMES and tiebreak != NONE):
        raise ValueError("bad strategy")
    x = np.zeros(n) if x is None else np.asarray(x, np.float64)
    rc = np.zeros(n) if rc is None else np.asarray(rc, np.float64)
    group = None
    if DUAL in (strategy, tiebreak):
        group = dual_groups(m, n, row_ptr, col, y)
    keys = _keys(strategy, x, rc, vtype, group) + _keys(tiebreak, x, rc, vtype, group)
    idx = np.nonzero(vtype != CONTINUOUS)[0]
    # np.lexsort sorts by its last key first: list the keys least significant first
    cols = [idx] + [k[idx] for k in reversed(keys)]
    return idx[np.lexsort(cols)]


def lp_fixing(x, var_type, uniform, l, u):
    """Fixing values of the LP-based value strategy (continuous variables keep x)."""
    x = np.asarray(x, np.float64)
    lo, hi = np.floor(x), np.ceil(x)
    d = x - lo
    a = np.where(np.asarray(uniform, np.float64) > d, lo, hi)
    a = np.clip(a, np.ceil(np.asarray(l, np.float64)), np.floor(np.asarray(u, np.float64)))
    return np.where(np.asarray(var_type) == CONTINUOUS, x, a)


def branching(l, u, a, c):
    """Bound changes (lower, upper) of the integer-aware branching rule (section 2, Alg. 1), in
    increasing priority (the last is explored first). With the fixing value a strictly inside
    [l, u]: the restriction away from the objective direction, the one towards it, then x = a
    (c > 0 prefers smaller values). With a on a bound: the other bound, then a."""
    if l < a < u:
        up, down, fix = (a + 1, u), (l, a - 1), (a, a)
        return [up, down, fix] if c > 0 else [down, up, fix]
    if a == l:
        return [(u, u), (l, l)]
    return [(l, l), (u, u)]
