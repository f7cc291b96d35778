"""Re-solves after fixings: new bounds on an existing handle (pdlp_update_bounds /
pdlp_batch_update_bounds) behave exactly like a new handle made with those bounds, and a re-solve
warm-started from the previous solution reaches the tolerance on the fixed LP as the oracle
re-evaluates it.

Fixings are seeded: a share of the binaries fixed at the values of a feasible 0/1 point of the LP
(generators.feasible_binary_point), so the fixed LP stays feasible and no input of a check comes
from the GPU.
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


def _fixed(lp, seed, share=0.3):
    point = g.feasible_binary_point(seed, lp)
    pick = np.random.default_rng([19, seed]).random(lp.n) < share
    l, u = lp.l.copy(), lp.u.copy()
    l[pick] = point[pick]
    u[pick] = point[pick]
    fixed = g.LP(lp.m, lp.n, lp.row_ptr, lp.col, lp.val, lp.c, lp.b, lp.sense, l, u, name=lp.name + " fixed")
    return fixed


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_updated_bounds_solve_like_a_new_handle(pdlp, prec):
    lp = g.set_cover(0)
    fx = _fixed(lp, 1)
    with pdlp.Problem(lp, precision=prec, tile_nnz=512) as a:
        a.solve(tol=1e-4)
        a.update_bounds(fx.l, fx.u)
        ia = a.solve(tol=1e-4)
        sa = a.get()
    with pdlp.Problem(fx, precision=prec, tile_nnz=512) as b:
        ib = b.solve(tol=1e-4)
        sb = b.get()
    say(prec, "after update", ia["iterations"], "new handle", ib["iterations"])
    assert ia["iterations"] == ib["iterations"] and ia["status"] == ib["status"] == pdlp.OPTIMAL
    assert np.array_equal(sa.x, sb.x) and np.array_equal(sa.y, sb.y)


def test_warm_resolve_after_fixings(pdlp):
    lp = g.set_cover(2)
    fx = _fixed(lp, 3)
    with pdlp.Problem(lp, precision="fp32") as p:
        first = p.solve(tol=1e-4)
        s0 = p.get()
        p.update_bounds(fx.l, fx.u)
        cold = p.solve(tol=1e-4)
        warm = p.solve(tol=1e-4, x0=s0.x, y0=s0.y, omega0=first["omega"])
        sw = p.get()
    k = oracle.kkt(fx, sw.x, sw.y)
    say("initial", first["iterations"], "re-solve cold", cold["iterations"], "warm", warm["iterations"],
        "warm used", warm["warm_started"], "oracle rel_kkt %.2e" % k["rel_kkt"])
    assert warm["status"] == pdlp.OPTIMAL and k["rel_kkt"] <= 1e-4
    # FP32 iterates are clipped to the FP32-rounded scaled bounds, so the unscaled x may pass a bound
    # by the rounding of one FP32 value (2^-24 relative) and of the unscaling
    tol = 1e-6 * np.maximum(1.0, np.abs(fx.u))
    assert np.all(sw.x >= fx.l - tol) and np.all(sw.x <= fx.u + tol)
    fixed = fx.l == fx.u
    assert np.all(np.abs(sw.x[fixed] - fx.l[fixed]) <= tol[fixed])


def test_batch_update_matches_single(pdlp):
    lps = [g.set_cover(10, m=300, n=700), g.multi_knapsack(12, m=150, n=400), g.set_cover(11, m=500, n=1100)]
    fx = _fixed(lps[1], 4, share=0.5)
    with pdlp.Batch(lps, precision="fp32", tile_nnz=1024) as bt:
        bt.solve(tol=1e-4)
        bt.update_bounds(1, fx.l, fx.u)
        infos = bt.solve(tol=1e-4)
        got = [bt.get(i) for i in range(3)]
    for i, lp in enumerate([lps[0], fx, lps[2]]):
        with pdlp.Problem(lp, precision="fp32", tile_nnz=1024) as p:
            p.solve(tol=1e-4)
            s = p.get()
        assert infos[i]["iterations"] == s.info["iterations"], i
        assert np.array_equal(got[i].x, s.x) and np.array_equal(got[i].y, s.y), i


def test_bad_bounds_are_rejected(pdlp):
    lp = g.set_cover(1, m=200, n=500)
    with pdlp.Problem(lp) as p:
        bad_l = lp.l.copy()
        bad_l[3] = 2.0  # above u
        with pytest.raises(pdlp.PDLPError):
            p.update_bounds(bad_l, lp.u)
        nan_u = lp.u.copy()
        nan_u[0] = np.nan
        with pytest.raises(pdlp.PDLPError):
            p.update_bounds(lp.l, nan_u)
        inf_l = lp.l.copy()
        inf_l[1] = np.inf
        with pytest.raises(pdlp.PDLPError):
            p.update_bounds(inf_l, np.full(lp.n, np.inf))
        # the handle still solves the original LP
        assert p.solve(tol=1e-4)["status"] == pdlp.OPTIMAL
    with pdlp.Batch([lp], precision="fp32") as bt:
        with pytest.raises(pdlp.PDLPError):
            bt.update_bounds(1, lp.l, lp.u)
