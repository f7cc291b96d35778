"""Pins of the LP-based variable strategies and LP-based fixing oracle (CPU).

* a hand-worked six-variable example: every strategy and the hybrid tiebreaks, and the fixing values
  (expected lists derived by hand from the definitions, written out below);
* the Dual strategy against a literal walk over the constraints (sorted with Python's sort, one
  constraint at a time, as the paper describes it) on seeded instances;
* every order against a pairwise comparison built from the definitions with Python's math module,
  and as a permutation of the binary and integer variables;
* fixing: exact rounding frequencies over a grid of samples (a value rounds up for a share d of the
  samples), integral values stay, bounds clamp.
Planted mistakes in a copy of the oracle must fail at least one pin.
"""
import functools
import math

import numpy as np
import pytest

from oracle import fix_oracle as fo
from paper_2503_10344_amd import generators as gen

# --- the hand-worked example -----------------------------------------------------------------
# variables 0..5: binary, integer, continuous, binary, integer, binary
# rows: 0 = {0, 2}, 1 = {1, 3}, 2 = {3, 4}; variable 5 is in no row
HAND = dict(
    m=3, n=6,
    row_ptr=np.array([0, 2, 4, 6], np.int32), col=np.array([0, 2, 1, 3, 3, 4], np.int32),
    var_type=np.array([1, 2, 0, 1, 2, 1], np.uint8),
    x=np.array([0.3, 2.75, 1.234, 1.0, 4.25, 0.9]),
    rc=np.array([2.0, -3.0, 7.0, 2.0, -5.0, 0.0]),
    y=np.array([0.5, -4.0, 4.0]),
)
# fractionalities of the ordered variables: 0: 0.3, 1: 0.25, 3: 0, 4: 0.25, 5: 0.1
# |rc|: 0: 2, 1: 3, 3: 2, 4: 5, 5: 0; |y| order of the rows: 1, 2 (tie, lower index), 0
# Dual walk: row 1 gives {1, 3} -> by |rc| 1, 3; row 2 gives {4}; row 0 gives {0}; then 5
HAND_ORDERS = {
    (fo.FRAC, fo.NONE): [3, 5, 1, 4, 0],
    (fo.REDCOST, fo.NONE): [4, 1, 0, 3, 5],
    (fo.DUAL, fo.NONE): [1, 3, 4, 0, 5],
    (fo.TYPE, fo.NONE): [0, 3, 5, 1, 4],
    (fo.FRAC, fo.REDCOST): [3, 5, 4, 1, 0],   # 1 and 4 tie at 0.25; |rc| 5 > 3
    (fo.FRAC, fo.DUAL): [3, 5, 1, 4, 0],      # 1 (row 1) before 4 (row 2)
    (fo.REDCOST, fo.FRAC): [4, 1, 3, 0, 5],   # 0 and 3 tie at |rc| 2; frac 0 < 0.3
    (fo.TYPE, fo.FRAC): [3, 5, 0, 1, 4],
    (fo.DUAL, fo.FRAC): [1, 3, 4, 0, 5],
}
HAND_L = np.array([0.0, 0.0, -np.inf, 0.0, 0.0, 0.0])
HAND_U = np.array([1.0, 10.0, np.inf, 1.0, 10.0, 1.0])
HAND_S = np.array([0.5, 0.5, 0.5, 0.5, 0.9, 0.05])
# 0: d 0.3 < 0.5 -> 0; 1: d 0.75 >= 0.5 -> 3; 2 continuous; 3: integral -> 1; 4: d 0.25 < 0.9 -> 4;
# 5: d 0.9 >= 0.05 -> 1
HAND_VALUES = [0.0, 3.0, 1.234, 1.0, 4.0, 1.0]


def _order(fo_, inst, s, t):
    return list(fo_.variable_order(s, t, inst["x"], inst["y"], inst["rc"], inst["var_type"], inst["m"],
                                   inst["n"], inst["row_ptr"], inst["col"]))


def pin_hand_orders(fo_=fo):
    for (s, t), want in HAND_ORDERS.items():
        assert _order(fo_, HAND, s, t) == want, (s, t)


def pin_hand_fixing(fo_=fo):
    got = fo_.lp_fixing(HAND["x"], HAND["var_type"], HAND_S, HAND_L, HAND_U)
    assert list(got) == HAND_VALUES, got


def _instance(seed, m=40, n=90):
    lp = gen.set_cover(seed, m=m, n=n, k=3) if seed % 2 == 0 else gen.general_sparse(seed, m=m, n=n, cap=12)
    d = gen.fixing_inputs(seed, lp)
    return dict(m=lp.m, n=lp.n, row_ptr=lp.row_ptr, col=lp.col, l=lp.l, u=lp.u, **d)


def _literal_dual(inst, with_groups=False):
    """The Dual strategy as the paper words it: constraints by descending |y|, each contributing its
    not yet seen integer variables ordered by reduced cost; then the variables of no constraint.
    With with_groups, also the step of the walk at which each variable was taken."""
    y, rc, vt = inst["y"], inst["rc"], inst["var_type"]
    rows = sorted(range(inst["m"]), key=lambda i: (-abs(float(y[i])), i))
    seen, out, group = set(), [], {}
    by_rc = lambda j: (-abs(float(rc[j])), j)  # noqa: E731
    for step, i in enumerate(rows):
        new = [int(j) for j in inst["col"][inst["row_ptr"][i]:inst["row_ptr"][i + 1]] if vt[j] != 0 and int(j) not in seen]
        new.sort(key=by_rc)
        seen.update(new)
        group.update({j: step for j in new})
        out += new
    rest = sorted((j for j in range(inst["n"]) if vt[j] != 0 and j not in seen), key=by_rc)
    group.update({j: len(rows) for j in rest})
    return (out + rest, group) if with_groups else out + rest


def pin_dual_is_the_literal_walk(fo_=fo):
    for seed in range(6):
        inst = _instance(seed)
        assert _order(fo_, inst, fo.DUAL, fo.NONE) == _literal_dual(inst), seed


def _pairwise_key(inst, strategy, j, group):
    x, rc, vt = float(inst["x"][j]), float(inst["rc"][j]), int(inst["var_type"][j])
    if strategy == fo.FRAC:
        return (min(x - math.floor(x), math.ceil(x) - x),)
    if strategy == fo.REDCOST:
        return (-abs(rc),)
    if strategy == fo.DUAL:  # the walk's step, then reduced cost inside it
        return (group[j], -abs(rc))
    if strategy == fo.TYPE:
        return (vt,)
    return ()


def pin_orders_follow_pairwise_definition(fo_=fo):
    combos = [(s, t) for s in (fo.FRAC, fo.REDCOST, fo.DUAL, fo.TYPE)
              for t in (fo.NONE, fo.FRAC, fo.REDCOST, fo.DUAL, fo.TYPE) if t != s]
    for seed in range(4):
        inst = _instance(seed)
        _, group = _literal_dual(inst, with_groups=True)
        ints = sorted(int(j) for j in np.nonzero(inst["var_type"] != 0)[0])
        for s, t in combos:
            got = _order(fo_, inst, s, t)
            assert sorted(got) == ints, (seed, s, t)

            def cmp(a, b):
                ka = _pairwise_key(inst, s, a, group) + _pairwise_key(inst, t, a, group) + (a,)
                kb = _pairwise_key(inst, s, b, group) + _pairwise_key(inst, t, b, group) + (b,)
                return -1 if ka < kb else (1 if ka > kb else 0)
            assert got == sorted(ints, key=functools.cmp_to_key(cmp)), (seed, s, t)


def pin_fixing_frequencies(fo_=fo):
    T = 1000
    s = (np.arange(T) + 0.5) / T
    for x, lo_int, d in ((0.3, 0.0, 0.3), (7.625, 7.0, 0.625), (-2.75, -3.0, 0.25), (5.0, 5.0, 0.0)):
        vals = fo_.lp_fixing(np.full(T, x), np.full(T, 2, np.uint8), s, np.full(T, -100.0), np.full(T, 100.0))
        ups = int(np.sum(vals == lo_int + 1))
        assert ups == round(d * T), (x, ups)
        assert np.all((vals == lo_int) | (vals == lo_int + 1))


def pin_fixing_clamps_to_integral_bounds(fo_=fo):
    x = np.array([10.0 + 1e-9, -1e-12, 2.5, 0.5])
    vt = np.array([2, 2, 2, 0], np.uint8)
    s = np.array([0.01, 0.99, 0.01, 0.5])
    got = fo_.lp_fixing(x, vt, s, np.array([0.0, 0.0, 2.2, 0.0]), np.array([10.0, 5.0, 2.9, 1.0]))
    # 11 -> clamped to 10; -1 -> clamped to 0; 3 -> clamped to floor(2.9) = 2; continuous keeps x
    assert list(got) == [10.0, 0.0, 2.0, 0.5], got


PINS = [pin_hand_orders, pin_hand_fixing, pin_dual_is_the_literal_walk, pin_orders_follow_pairwise_definition,
        pin_fixing_frequencies, pin_fixing_clamps_to_integral_bounds]


@pytest.mark.parametrize("pin", PINS, ids=[p.__name__ for p in PINS])
def test_pin(pin):
    pin()


MUTANTS = {
    "frac_descending": ("return [fractionality(x)]", "return [-fractionality(x)]"),
    "redcost_signed": ("if strategy == REDCOST:\n        return [-np.abs(rc)]",
                       "if strategy == REDCOST:\n        return [-rc]"),
    "redcost_ascending": ("if strategy == REDCOST:\n        return [-np.abs(rc)]",
                          "if strategy == REDCOST:\n        return [np.abs(rc)]"),
    "dual_rows_ascending": ("np.lexsort((rows, -np.abs(np.asarray(y, np.float64))))",
                            "np.lexsort((rows, np.abs(np.asarray(y, np.float64))))"),
    "dual_rows_signed": ("np.lexsort((rows, -np.abs(np.asarray(y, np.float64))))",
                         "np.lexsort((rows, -np.asarray(y, np.float64)))"),
    "dual_group_is_last_row": ("group = np.full(n, m, np.int64)\n    np.minimum.at(",
                               "group = np.full(n, -1, np.int64)\n    np.maximum.at("),
    "dual_without_redcost": ("return [group, -np.abs(rc)]", "return [group]"),
    "type_integers_first": ("return [vtype.astype(np.int64)]", "return [-vtype.astype(np.int64)]"),
    "tiebreak_ignored": ("keys = _keys(strategy, x, rc, vtype, group) + _keys(tiebreak, x, rc, vtype, group)",
                         "keys = _keys(strategy, x, rc, vtype, group)"),
    "tiebreak_outranks_primary": (
        "keys = _keys(strategy, x, rc, vtype, group) + _keys(tiebreak, x, rc, vtype, group)",
        "keys = _keys(tiebreak, x, rc, vtype, group) + _keys(strategy, x, rc, vtype, group)"),
    "index_ties_reversed": ("cols = [idx] + ", "cols = [-idx] + "),
    "continuous_included": ("idx = np.nonzero(vtype != CONTINUOUS)[0]", "idx = np.arange(vtype.size)"),
    "fixing_comparison_reversed": ("a = np.where(np.asarray(uniform, np.float64) > d, lo, hi)",
                                   "a = np.where(np.asarray(uniform, np.float64) < d, lo, hi)"),
    "fixing_distance_to_upper": ("d = x - lo", "d = hi - x"),
    "fixing_not_clamped": ("a = np.clip(a, np.ceil(np.asarray(l, np.float64)), np.floor(np.asarray(u, np.float64)))",
                           "a = a"),
    "frac_distance_to_lower_only": ("return np.minimum(x - np.floor(x), np.ceil(x) - x)",
                                    "return x - np.floor(x)"),
}


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_pins_catch_mutant(name):
    """A plausible mistake planted in a copy of the oracle fails at least one pin."""
    import importlib.util
    import types
    old, new = MUTANTS[name]
    path = importlib.util.find_spec("oracle.fix_oracle").origin
    src = open(path).read()
    assert src.count(old) == 1, name
    mod = types.ModuleType("fix_oracle_mutant")
    exec(compile(src.replace(old, new), path + ":" + name, "exec"), mod.__dict__)
    failed = []
    for pin in PINS:
        try:
            pin(fo_=mod)
        except Exception:   # an assertion or a shape error both count as caught
            failed.append(pin.__name__)
    assert failed, f"mutant {name} passed every pin"
