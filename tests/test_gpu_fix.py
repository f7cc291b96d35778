"""LP-based variable strategies and LP-based fixing on the GPU against the oracle (bit-exact).

Orders are integer results of comparisons on exactly computed keys (fractionality and |r| are exact
in FP64 on both sides), so every strategy and tiebreak must give the oracle's permutation exactly,
and the fixing values must be equal bit for bit. Inputs are seeded draws (generators.fixing_inputs)
with many equal keys. Sizes: tens of thousands of variables (several 4,096-item sort tiles and a
ragged tail), edge cases, and the full 500k x 1M and 7.0M x 9.6M LPs.
"""
import sys

import numpy as np
import pytest

from oracle import fix_oracle as fo

try:  # import at collection time: the first import on a fresh machine can take a minute
    import torch  # noqa: F401
except Exception:  # pragma: no cover
    torch = None
from paper_2503_10344_amd import generators as g

pytestmark = pytest.mark.gpu

STRATEGIES = [fo.FRAC, fo.REDCOST, fo.DUAL, fo.TYPE]
COMBOS = [(s, fo.NONE) for s in STRATEGIES] + [(fo.FRAC, fo.DUAL), (fo.FRAC, fo.REDCOST), (fo.REDCOST, fo.FRAC),
                                               (fo.DUAL, fo.FRAC), (fo.TYPE, fo.FRAC), (fo.FRAC, fo.TYPE)]


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


def _oracle_order(lp, d, s, t):
    return fo.variable_order(s, t, d["x"], d["y"], d["rc"], d["var_type"], lp.m, lp.n, lp.row_ptr, lp.col)


def _check_all(pdlp, lp, d, combos=COMBOS, label=""):
    with pdlp.Problem(lp, precision="fp32", tile_nnz=512) as p:
        for s, t in combos:
            got = p.variable_strategy(s, d["var_type"], x=d["x"], y=d["y"], rc=d["rc"], tiebreak=t)
            want = _oracle_order(lp, d, s, t)
            assert got.size == want.size and np.array_equal(got, want), (label, s, t)
        vals = p.lp_fixing(d["var_type"], d["x"], lp.l, lp.u, d["uniform"])
    np.testing.assert_array_equal(vals, fo.lp_fixing(d["x"], d["var_type"], d["uniform"], lp.l, lp.u))
    say(label, "orders and fixing values equal the oracle's;", int(np.sum(d["var_type"] != 0)), "integer variables")


@pytest.mark.parametrize("family", ["setcover", "general", "energy"])
def test_orders_and_fixing_match_oracle(pdlp, family):
    if family == "setcover":
        lp = g.set_cover(3, m=6000, n=15000)            # all binary: 15k keys, four tiles
    elif family == "general":
        lp = g.general_sparse(4, m=20000, n=50000, cap=400)
    else:
        lp = g.energy(5, T=48, N=20, K=6, E=40)
    d = g.fixing_inputs(7, lp)
    _check_all(pdlp, lp, d, label=family)


def test_edge_cases(pdlp):
    lp = g.general_sparse(8, m=300, n=700, cap=40)
    d = g.fixing_inputs(9, lp)
    with pdlp.Problem(lp, precision="fp64") as p:
        # no integer variables: an empty order
        none = np.zeros(lp.n, np.uint8)
        assert p.variable_strategy(fo.FRAC, none, x=d["x"]).size == 0
        # one integer variable
        one = none.copy()
        one[123] = 2
        assert list(p.variable_strategy(fo.DUAL, one, y=d["y"], rc=d["rc"])) == [123]
        # every key equal: index order (Dual still groups by the first row holding a variable)
        allint = np.full(lp.n, 2, np.uint8)
        flat = dict(var_type=allint, x=np.round(d["x"]), y=np.zeros(lp.m), rc=np.zeros(lp.n))
        for s in STRATEGIES:
            got = p.variable_strategy(s, allint, x=flat["x"], y=flat["y"], rc=flat["rc"])
            if s == fo.DUAL:
                assert np.array_equal(got, _oracle_order(lp, flat, s, fo.NONE))
            else:
                assert np.array_equal(got, np.arange(lp.n)), s
        # a needed input missing, or an unknown strategy, is an argument error
        with pytest.raises(pdlp.PDLPError):
            p.variable_strategy(fo.DUAL, d["var_type"], x=d["x"], rc=d["rc"])
        with pytest.raises(pdlp.PDLPError):
            p.variable_strategy(9, d["var_type"], x=d["x"])
        with pytest.raises(pdlp.PDLPError):
            p.lp_fixing(d["var_type"], d["x"], lp.l, lp.u, np.zeros(lp.n))  # samples must lie in (0, 1)
    # no constraints at all: Dual falls back to RedCost order; empty columns come last
    box = g.LP(0, 50, np.zeros(1, np.int32), np.zeros(0, np.int32), np.zeros(0), np.ones(50), np.zeros(0),
               np.zeros(0, np.uint8), np.zeros(50), np.full(50, 3.0))
    db = g.fixing_inputs(10, box)
    with pdlp.Problem(box) as p:
        got = p.variable_strategy(fo.DUAL, db["var_type"], y=db["y"], rc=db["rc"])
    assert np.array_equal(got, _oracle_order(box, db, fo.DUAL, fo.NONE))


def test_device_resident_inputs_give_the_same_results(pdlp):
    """GPU tensors in and out (no PCIe): the same order and values as the host path."""
    import torch
    lp = g.general_sparse(6, m=8000, n=20000, cap=300)
    d = g.fixing_inputs(13, lp)
    dev = {k: torch.from_numpy(np.ascontiguousarray(v)).cuda() for k, v in d.items()}
    lo, up = torch.from_numpy(lp.l).cuda(), torch.from_numpy(lp.u).cuda()
    with pdlp.Problem(lp, precision="fp32") as p:
        for s, t in ((fo.FRAC, fo.DUAL), (fo.DUAL, fo.NONE), (fo.TYPE, fo.REDCOST)):
            host = p.variable_strategy(s, d["var_type"], x=d["x"], y=d["y"], rc=d["rc"], tiebreak=t)
            on_gpu = p.variable_strategy(s, dev["var_type"], x=dev["x"], y=dev["y"], rc=dev["rc"], tiebreak=t)
            assert on_gpu.is_cuda and np.array_equal(on_gpu.cpu().numpy(), host), (s, t)
        vals = p.lp_fixing(dev["var_type"], dev["x"], lo, up, dev["uniform"])
    assert vals.is_cuda
    np.testing.assert_array_equal(vals.cpu().numpy(), fo.lp_fixing(d["x"], d["var_type"], d["uniform"], lp.l, lp.u))


def test_order_of_a_solved_lp_is_sorted_by_its_keys(pdlp):
    """Chained on the device's own solution: the Frac order is a permutation of the binaries whose
    fractionality never decreases, ties in index order (a property, so no oracle input comes from
    the GPU)."""
    lp = g.set_cover(2, m=2000, n=5000)
    vt = np.ones(lp.n, np.uint8)
    with pdlp.Problem(lp, precision="fp32") as p:
        p.solve(tol=1e-4)
        sol = p.get()
        order = p.variable_strategy(fo.FRAC, vt, x=sol.x)
        vals = p.lp_fixing(vt, sol.x, lp.l, lp.u, np.full(lp.n, 0.5))
    assert np.array_equal(np.sort(order), np.arange(lp.n))
    f = np.minimum(sol.x - np.floor(sol.x), np.ceil(sol.x) - sol.x)[order]
    assert np.all(np.diff(f) >= 0)
    ties = np.diff(f) == 0
    assert np.all(np.diff(order)[ties] > 0)
    assert set(np.unique(vals)) <= {0.0, 1.0}


@pytest.mark.parametrize("which", ["general", "energy"])
def test_full_size_orders_match_oracle(pdlp, which):
    lp = g.general_sparse(0) if which == "general" else g.energy(0)
    d = g.fixing_inputs(12, lp)
    say(which, "full size:", lp.m, "rows", lp.n, "columns", int(np.sum(d["var_type"] != 0)), "integer variables")
    _check_all(pdlp, lp, d, combos=[(fo.FRAC, fo.DUAL), (fo.DUAL, fo.NONE), (fo.REDCOST, fo.FRAC)], label=which)
