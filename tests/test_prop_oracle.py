"""Pins of the linear-constraint propagation oracle and of the branching rule (CPU).

* a hand-worked six-variable example (a fixing forcing a binary to 0, an integer >= row, an equality
  between continuous variables), a tiny improvement of a continuous bound that must be ignored,
  integer rounding within 1e-6, one and two infinite activity terms; expected bounds, status and
  round count derived by hand below;
* infeasibility found in the first round;
* a chain x_{k+1} - x_k >= 1 whose closed form after r Jacobi rounds is l_k = min(k, r),
  u_k = 10 - min(4 - k, r) (one step per round; a Gauss-Seidel sweep would finish in one);
* brute force on tiny integer programs: propagation never removes a feasible integer point, and
  reports infeasible only when there is none; the result is a fixpoint; tighter input bounds give
  tighter or equal output bounds;
* the branching rule of Alg. 1 on hand cases.
Planted mistakes in a copy of the C oracle (rebuilt on the CPU) must fail at least one pin.
"""
import itertools

import numpy as np
import pytest

import oracle
from oracle import fix_oracle as fo
from paper_2503_10344_amd import generators as gen

L_, G_, E_ = ord("L"), ord("G"), ord("E")


def _lp(rows, n, b, sense, l, u):
    """LP from a list of rows, each a list of (column, value)."""
    rp = np.zeros(len(rows) + 1, np.int32)
    col, val = [], []
    for i, r in enumerate(rows):
        rp[i + 1] = rp[i] + len(r)
        col += [c for c, _ in r]
        val += [v for _, v in r]
    return gen.LP(len(rows), n, rp, np.array(col, np.int32), np.array(val, np.float64), np.zeros(n),
                  np.array(b, np.float64), np.array(sense, np.uint8), np.array(l, np.float64), np.array(u, np.float64))


def _run(lib, lp, vt, l=None, u=None, rounds=100):
    return oracle.propagate(lp, vt, lp.l if l is None else l, lp.u if u is None else u, rounds, lib_path=lib)


def pin_hand_example(lib=oracle.PROP_LIB):
    # x0 + x1 <= 1 (binaries, x0 fixed to 1); 2 x2 + 3 x3 >= 7 (integers in [0, 2]);
    # x4 - x5 = 0 (continuous, x4 in [0, 5], x5 in [1, 3])
    lp = _lp([[(0, 1.0), (1, 1.0)], [(2, 2.0), (3, 3.0)], [(4, 1.0), (5, -1.0)]], 6, [1.0, 7.0, 0.0],
             [L_, G_, E_], [1, 0, 0, 0, 0, 1], [1, 1, 2, 2, 5, 3])
    vt = np.array([1, 1, 2, 2, 0, 0], np.uint8)
    l, u, st, r = _run(lib, lp, vt)
    # first round: u1 = (1 - 1)/1 = 0; l2 = ceil((7 - 6)/2) = 1, l3 = ceil((7 - 4)/3) = 1;
    # u4 = 0 - (-3) = 3, l4 = 0 - (-1) = 1; the second round changes nothing
    assert list(l) == [1, 0, 1, 1, 1, 1] and list(u) == [1, 0, 2, 2, 3, 3], (l, u)
    assert (st, r) == (oracle.PROP_FIXPOINT, 2)


def pin_small_continuous_gain_ignored(lib=oracle.PROP_LIB):
    # x <= 0.9999999 on a continuous x in [0, 1]: a gain of 1e-7 < 1e-3 is not taken;
    # integers in [0, 5]: y <= 2.9999995 rounds to 3 (within 1e-6), y <= 2.5 to 2, z >= 2.0000005 to 2
    lp = _lp([[(0, 1.0)], [(1, 1.0)], [(2, 1.0)], [(3, 1.0)]], 4, [0.9999999, 2.9999995, 2.5, 2.0000005],
             [L_, L_, L_, G_], [0, 0, 0, 0], [1, 5, 5, 5])
    l, u, st, r = _run(lib, lp, np.array([0, 2, 2, 2], np.uint8))
    assert list(u) == [1.0, 3.0, 2.0, 5.0] and list(l) == [0.0, 0.0, 0.0, 2.0], (l, u)
    assert st == oracle.PROP_FIXPOINT


def pin_infinite_bounds(lib=oracle.PROP_LIB):
    # x0 + x1 + x2 <= 5, continuous, x2 in [0, 1]
    rows = [[(0, 1.0), (1, 1.0), (2, 1.0)]]
    # two infinite lower bounds: the minimum activity is -inf for every residual, nothing is derived
    lp = _lp(rows, 3, [5.0], [L_], [-np.inf, -np.inf, 0], [10, 10, 1])
    l, u, st, r = _run(lib, lp, np.zeros(3, np.uint8))
    assert list(u) == [10, 10, 1] and (st, r) == (oracle.PROP_FIXPOINT, 1), u
    # one infinite lower bound: only that variable gets a bound, u0 = 5 - (0 + 0)
    lp = _lp(rows, 3, [5.0], [L_], [-np.inf, 0, 0], [10, 10, 1])
    l, u, st, r = _run(lib, lp, np.zeros(3, np.uint8))
    assert list(u) == [5, 10, 1] and l[0] == -np.inf, (l, u)


def pin_infeasible_in_first_round(lib=oracle.PROP_LIB):
    lp = _lp([[(0, 1.0), (1, 1.0)]], 2, [3.0], [G_], [0, 0], [1, 1])
    _, _, st, r = _run(lib, lp, np.array([1, 1], np.uint8))
    assert (st, r) == (oracle.PROP_INFEASIBLE, 1)
    # crossed bounds and no rows: only the bound check can see it
    empty = _lp([], 2, [], [], [0, 2], [1, 1])
    _, _, st, r = _run(lib, empty, np.array([2, 2], np.uint8))
    assert (st, r) == (oracle.PROP_INFEASIBLE, 1)


def _chain():
    rows = [[(k, -1.0), (k + 1, 1.0)] for k in range(4)]
    return _lp(rows, 5, [1.0] * 4, [G_] * 4, [0] * 5, [10] * 5)


def pin_chain_one_step_per_round(lib=oracle.PROP_LIB):
    lp = _chain()
    vt = np.full(5, 2, np.uint8)
    for r in range(1, 5):
        l, u, st, done = _run(lib, lp, vt, rounds=r)
        assert list(l) == [min(k, r) for k in range(5)], (r, l)
        assert list(u) == [10 - min(4 - k, r) for k in range(5)], (r, u)
        assert (st, done) == (oracle.PROP_ROUND_LIMIT, r)
    l, u, st, done = _run(lib, lp, vt)
    assert (st, done) == (oracle.PROP_FIXPOINT, 5) and list(l) == [0, 1, 2, 3, 4]


def _tiny(seed):
    rng = np.random.default_rng([5, seed])
    n, m = int(rng.integers(3, 6)), int(rng.integers(2, 5))
    rows = []
    for _ in range(m):
        cols = rng.choice(n, size=int(rng.integers(1, n + 1)), replace=False)
        rows.append([(int(c), float(rng.choice([-3, -2, -1, 1, 2, 3]))) for c in sorted(cols)])
    sense = rng.choice([L_, G_, E_], size=m, p=[0.45, 0.45, 0.1])
    l = rng.integers(-2, 1, n).astype(float)
    u = l + rng.integers(1, 4, n)
    b = [float(rng.integers(-4, 5)) for _ in range(m)]
    return _lp(rows, n, b, sense, l, u)


def _feasible_points(lp):
    A = lp.to_scipy().toarray()
    pts = []
    for p in itertools.product(*[range(int(a), int(b) + 1) for a, b in zip(lp.l, lp.u)]):
        ax = A @ np.array(p, float)
        ok = all((s != L_ or v <= bb + 1e-9) and (s != G_ or v >= bb - 1e-9) and (s != E_ or abs(v - bb) <= 1e-9)
                 for v, bb, s in zip(ax, lp.b, lp.sense))
        if ok:
            pts.append(p)
    return np.array(pts, float).reshape(-1, lp.n)


def pin_never_cuts_a_feasible_point(lib=oracle.PROP_LIB):
    for seed in range(60):
        lp = _tiny(seed)
        vt = np.full(lp.n, 2, np.uint8)
        F = _feasible_points(lp)
        l, u, st, r = _run(lib, lp, vt)
        if st == oracle.PROP_INFEASIBLE:
            assert F.shape[0] == 0, seed
            continue
        assert st == oracle.PROP_FIXPOINT, seed
        assert np.all(F >= l - 1e-9) and np.all(F <= u + 1e-9), seed
        # a fixpoint: propagating again changes nothing, in one round
        l2, u2, st2, r2 = _run(lib, lp, vt, l, u)
        assert np.array_equal(l2, l) and np.array_equal(u2, u) and (st2, r2) == (oracle.PROP_FIXPOINT, 1), seed
        # tighter input bounds give tighter or equal results
        j = seed % lp.n
        lt, ut = lp.l.copy(), lp.u.copy()
        ut[j] = lt[j]
        l3, u3, st3, _ = _run(lib, lp, vt, lt, ut)
        if st3 != oracle.PROP_INFEASIBLE:
            assert np.all(l3 >= l) and np.all(u3 <= u), seed


def pin_branching_rule(lib=None):
    assert fo.branching(0, 5, 2, 1.0) == [(3, 5), (0, 1), (2, 2)]
    assert fo.branching(0, 5, 2, -1.0) == [(0, 1), (3, 5), (2, 2)]
    assert fo.branching(0, 5, 2, 0.0) == [(0, 1), (3, 5), (2, 2)]
    assert fo.branching(0, 5, 0, 1.0) == [(5, 5), (0, 0)]
    assert fo.branching(0, 5, 5, 1.0) == [(0, 0), (5, 5)]
    assert fo.branching(0, 1, 1, -2.0) == [(0, 0), (1, 1)]


PINS = [pin_hand_example, pin_small_continuous_gain_ignored, pin_infinite_bounds, pin_infeasible_in_first_round,
        pin_chain_one_step_per_round, pin_never_cuts_a_feasible_point]


@pytest.mark.parametrize("pin", PINS + [pin_branching_rule], ids=[p.__name__ for p in PINS + [pin_branching_rule]])
def test_pin(pin):
    pin()


MUTANTS = {
    "residual_keeps_own_term": ("if (mininf == 0) res = minf - a * t;", "if (mininf == 0) res = minf;"),
    "infinite_count_ignored": ("else if (mininf == 1 && isinf(t)) res = minf;", "else if (isinf(t)) res = minf;"),
    "integer_rounds_outward": ("const double q = floor(p + kFeasTol);", "const double q = ceil(p + kFeasTol);"),
    "integer_no_tolerance": ("const double q = ceil(p - kFeasTol);", "const double q = ceil(p);"),
    "equality_one_sided": ("ge = sense[i] == 'G' || sense[i] == 'E';", "ge = sense[i] == 'G';"),
    "gauss_seidel_reads": ("const double a = val[k], lo = l[j], hi = u[j];",
                           "const double a = val[k], lo = ln[j], hi = un[j];"),
    "continuous_threshold_dropped": ("return p < cur - kContTol * rmax(1.0, fabs(cur)) ? p : cur;",
                                     "return p < cur ? p : cur;"),
    "negative_coefficient_side_swapped": ("if (a > 0.0) un[j] = fmin(un[j], tighten_upper(hi, p, integral));\n"
                                          "            else ln[j] = fmax(ln[j], tighten_lower(lo, p, integral));",
                                          "if (a > 0.0) un[j] = fmin(un[j], tighten_upper(hi, p, integral));\n"
                                          "            else un[j] = fmin(un[j], tighten_upper(hi, p, integral));"),
    "min_activity_uses_upper": ("const double tmin = a > 0.0 ? lo : hi, tmax = a > 0.0 ? hi : lo;",
                                "const double tmin = a > 0.0 ? hi : lo, tmax = a > 0.0 ? hi : lo;"),
    "column_infeasibility_missed": ("if (l[j] > u[j] + kFeasTol) col_infeasible = 1;", "(void)0;"),
}


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_pins_catch_mutant(name, tmp_path):
    """A plausible mistake planted in a copy of the C oracle fails at least one pin."""
    old, new = MUTANTS[name]
    src = open(oracle.PROP_SRC).read()
    assert src.count(old) == 1, name
    path = tmp_path / "prop_mutant.c"
    path.write_text(src.replace(old, new))
    lib = str(tmp_path / f"libprop_{name}.so")
    oracle.build_prop(str(path), lib)
    failed = []
    for pin in PINS:
        try:
            pin(lib=lib)
        except Exception:
            failed.append(pin.__name__)
    assert failed, f"mutant {name} passed every pin"
