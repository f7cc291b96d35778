"""The oracle against what the mathematics and independent solvers fix (CPU only)."""
import numpy as np
import pytest

import oracle
import oracle_pins as P


@pytest.mark.parametrize("pin", P.ALL_PINS, ids=lambda f: f.__name__)
def test_pin(pin, oracle_lib):
    pin()


def test_sum_orders_are_roundings_of_the_same_method():
    """The oracle's alternative summation orders (used to size the GPU tracking bound) change only
    the rounding: the first attempts agree to a few ulps, the solves reach the same optimum, and the
    orders are really different (the traces are not bitwise equal)."""
    from paper_2503_10344_amd import generators as g
    lp = g.general_sparse(2, m=120, n=240, cap=60)
    base = oracle.solve(lp, tol=0.0, iter_limit=8, trace_len=8).trace
    fin = oracle.solve(lp, tol=1e-7, iter_limit=400_000)
    for so in (1, 2):
        t = oracle.solve(lp, tol=0.0, iter_limit=8, trace_len=8, sum_order=so).trace
        d = np.abs(t["x"][0] - base["x"][0]).max() / np.abs(base["x"][0]).max()
        assert 0.0 < np.abs(t["x"] - base["x"]).max() and d <= 1e-14, (so, d)
        r = oracle.solve(lp, tol=1e-7, iter_limit=400_000, sum_order=so)
        assert r.status == oracle.OPTIMAL
        assert abs(r.pobj - fin.pobj) <= 1e-6 * max(1.0, abs(fin.pobj)), (so, r.pobj, fin.pobj)
