"""Linear-constraint propagation on the GPU against the C oracle: bounds, status and round count
must be equal (bounds compared as numbers; row sums keep row order on both sides and the tightest
proposal of a set does not depend on order, so no rounding tolerance is needed).

Starting bounds (the state fix-and-propagate propagates after fixings): a seeded share of the
variables fixed to a feasible point's values on set-cover and multi-knapsack rows (binaries) and on
general sparse rows (continuous, free columns: infinite activity terms), and the energy-shaped LP's
own bounds with seeded integer types; then an infeasible fixing, a round limit, GPU-resident bounds,
edge cases and the full 500k x 1M and 7.0M x 9.6M LPs.
"""
import sys

import numpy as np
import pytest

import oracle

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


def _start(lp, family, seed):
    """Variable types and starting bounds: a seeded share of the variables fixed to the values of a
    feasible point (so propagation must not find infeasibility), or, for the energy-shaped rows, the
    LP's own bounds with seeded integer types."""
    rng = np.random.default_rng([13, seed])
    l, u = lp.l.copy(), lp.u.copy()
    if family in ("setcover", "knapsack"):
        vt = np.ones(lp.n, np.uint8)
        point = g.feasible_binary_point(seed, lp)
        pick = rng.random(lp.n) < (0.85 if family == "setcover" else 0.6)
    elif family == "general":
        vt = np.zeros(lp.n, np.uint8)       # continuous: the generator's point x0 is feasible
        point = lp.meta["x0"]
        pick = rng.random(lp.n) < 0.3
    else:
        return g.fixing_inputs(seed, lp)["var_type"], l, u
    l[pick] = point[pick]
    u[pick] = point[pick]
    return vt, l, u


def _compare(pdlp, lp, vt, l, u, max_rounds=100, label=""):
    ol, ou, ost, orr = oracle.propagate(lp, vt, l, u, max_rounds)
    with pdlp.Propagator(lp, vt) as p:
        gl, gu, gst, grr = p.propagate(l, u, max_rounds)
    moved = int(np.sum((ol != l) | (ou != u)))
    say(label, "status", gst, "rounds", grr, "bounds moved", moved)
    assert (gst, grr) == (ost, orr), (label, gst, grr, ost, orr)
    assert np.array_equal(gl, ol) and np.array_equal(gu, ou), label
    return moved, gst, grr


@pytest.mark.parametrize("family", ["setcover", "knapsack", "general", "energy"])
def test_propagation_matches_oracle(pdlp, family):
    if family == "setcover":
        lp = g.set_cover(1, m=6000, n=15000)
    elif family == "knapsack":
        lp = g.multi_knapsack(2, m=3000, n=8000)
    elif family == "general":
        lp = g.general_sparse(3, m=20000, n=50000, cap=400)
    else:
        lp = g.energy(4, T=48, N=20, K=6, E=40)
    vt, l, u = _start(lp, family, 5)
    moved, st, r = _compare(pdlp, lp, vt, l, u, label=family)
    assert moved > 0 and st == pdlp.PROP_FIXPOINT and r >= 2


def test_infeasible_fixing_and_round_limit(pdlp):
    lp = g.set_cover(6, m=500, n=1200)
    vt = np.ones(lp.n, np.uint8)
    l, u = lp.l.copy(), lp.u.copy()
    row = 7
    u[lp.col[lp.row_ptr[row]:lp.row_ptr[row + 1]]] = 0.0  # every cover of row 7 fixed to 0
    _, st, r = _compare(pdlp, lp, vt, l, u, label="infeasible")
    assert (st, r) == (pdlp.PROP_INFEASIBLE, 1)
    # a chain x_{k+1} - x_k >= 1 moves one step per round: a round limit stops it
    n = 40
    rp = np.arange(0, 2 * (n - 1) + 1, 2, dtype=np.int32)
    col = np.array([[k, k + 1] for k in range(n - 1)], np.int32).ravel()
    val = np.tile([-1.0, 1.0], n - 1)
    chain = g.LP(n - 1, n, rp, col, val, np.zeros(n), np.ones(n - 1), np.full(n - 1, ord("G"), np.uint8),
                 np.zeros(n), np.full(n, 100.0))
    vt = np.full(n, 2, np.uint8)
    _, st, r = _compare(pdlp, chain, vt, chain.l, chain.u, max_rounds=7, label="chain")
    assert (st, r) == (pdlp.PROP_ROUND_LIMIT, 7)
    _, st, r = _compare(pdlp, chain, vt, chain.l, chain.u, label="chain to fixpoint")
    assert (st, r) == (pdlp.PROP_FIXPOINT, n)


def test_device_bounds_and_edge_cases(pdlp):
    import torch
    lp = g.general_sparse(8, m=5000, n=12000, cap=200)
    vt, l, u = _start(lp, "general", 9)
    ol, ou, ost, orr = oracle.propagate(lp, vt, l, u, 100)
    with pdlp.Propagator(lp, vt) as p:
        tl, tu = torch.from_numpy(l.copy()).cuda(), torch.from_numpy(u.copy()).cuda()
        gl, gu, gst, grr = p.propagate(tl, tu)
        assert gl.is_cuda and (gst, grr) == (ost, orr)
        assert np.array_equal(gl.cpu().numpy(), ol) and np.array_equal(gu.cpu().numpy(), ou)
        with pytest.raises(pdlp.PDLPError):
            p.propagate(np.full(lp.n, np.nan), u)
        with pytest.raises(pdlp.PDLPError):
            p.propagate(l, u, max_rounds=0)
    # no rows; crossed bounds are infeasible in the first round
    empty = g.LP(0, 4, np.zeros(1, np.int32), np.zeros(0, np.int32), np.zeros(0), np.zeros(4), np.zeros(0),
                 np.zeros(0, np.uint8), np.zeros(4), np.ones(4))
    with pdlp.Propagator(empty, np.full(4, 2, np.uint8)) as p:
        assert p.propagate(empty.l, empty.u)[2:] == (pdlp.PROP_FIXPOINT, 1)
        assert p.propagate(np.array([0, 2, 0, 0.0]), empty.u)[2:] == (pdlp.PROP_INFEASIBLE, 1)


@pytest.mark.parametrize("which", ["general", "energy"])
def test_full_size_propagation_matches_oracle(pdlp, which):
    lp = g.general_sparse(0) if which == "general" else g.energy(0)
    vt, l, u = _start(lp, which, 11)
    # at most 20 rounds (a long chain of rows moves one step per round)
    moved, st, r = _compare(pdlp, lp, vt, l, u, max_rounds=20, label=f"{which} full size")
    assert moved > 0
