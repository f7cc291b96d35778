"""Degenerate LPs on the GPU: no constraints, a single variable and row, infeasible and unbounded
problems, and such instances inside a batch (also through the warm-start network)."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

from oracle import gnn_oracle as go  # noqa: E402
from paper_2503_10344_amd import generators as g  # noqa: E402
from paper_2503_10344_amd import pdlp  # noqa: E402


def box_only(seed, n=300):
    """min c'x over a box, no rows: x_j = l_j if c_j > 0, u_j if c_j < 0 (closed form)."""
    rng = np.random.default_rng(seed)
    c = rng.normal(size=n)
    l = rng.uniform(-3, 0, n)
    u = l + rng.uniform(0.5, 4, n)
    lp = g.LP(0, n, np.zeros(1, np.int32), np.zeros(0, np.int32), np.zeros(0), c, np.zeros(0),
              np.zeros(0, np.uint8), l, u)
    return lp, np.where(c > 0, l, u)


def one_by_one():
    """min 3x s.t. 2x >= 4, 0 <= x <= 10: x = 2, y = 1.5 (closed form)."""
    return g.LP(1, 1, np.array([0, 1], np.int32), np.array([0], np.int32), np.array([2.0]), np.array([3.0]),
                np.array([4.0]), np.array([ord("G")], np.uint8), np.array([0.0]), np.array([10.0]))


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_no_constraints(prec):
    lp, xs = box_only(1)
    with pdlp.Problem(lp, precision=prec) as p:
        info = p.solve(tol=1e-6, iter_limit=20_000)
        sol = p.get()
    assert info["status_name"] == "optimal"
    assert sol.y.size == 0
    np.testing.assert_allclose(sol.x, xs, rtol=0, atol=1e-5 * (1 + np.abs(xs)).max())
    np.testing.assert_allclose(sol.rc, lp.c, rtol=1e-12, atol=0)   # r = c - A'y with no rows


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_single_variable_single_row(prec):
    with pdlp.Problem(one_by_one(), precision=prec) as p:
        info = p.solve(tol=1e-8 if prec == "fp64" else 1e-6, iter_limit=50_000)
        sol = p.get()
    assert info["status_name"] == "optimal"
    assert abs(sol.x[0] - 2.0) <= 1e-5 and abs(sol.y[0] - 1.5) <= 1e-5
    assert abs(info["primal_obj"] - 6.0) <= 1e-5


def test_infeasible_and_unbounded_stop_cleanly():
    # infeasible: x >= 1 and x <= 0.5 with 0 <= x <= 10
    inf_lp = g.LP(2, 1, np.array([0, 1, 2], np.int32), np.array([0, 0], np.int32), np.array([1.0, 1.0]),
                  np.array([1.0]), np.array([1.0, 0.5]), np.array([ord("G"), ord("L")], np.uint8),
                  np.array([0.0]), np.array([10.0]))
    # unbounded: min -x1 s.t. x1 - x2 = 0, x >= 0
    unb_lp = g.LP(1, 2, np.array([0, 2], np.int32), np.array([0, 1], np.int32), np.array([1.0, -1.0]),
                  np.array([-1.0, 0.0]), np.array([0.0]), np.array([ord("E")], np.uint8),
                  np.zeros(2), np.full(2, np.inf))
    for lp in (inf_lp, unb_lp):
        for prec in ("fp32", "fp64"):
            with pdlp.Problem(lp, precision=prec) as p:
                info = p.solve(tol=1e-4, iter_limit=5_000)
            # no optimality claim; the solve ends at the budget (or flags a numerical breakdown)
            assert info["status_name"] in ("iteration_limit", "numerical"), (prec, info["status_name"])
            assert info["iterations"] <= 5_000 + 64


def empty_lines():
    """4 x 5 with an empty row (0 <= 2) and two empty columns (x2 -> 0 at c = 3, x4 -> 1 at c = -1)."""
    rp = np.array([0, 2, 2, 4, 6], np.int32)
    ci = np.array([0, 1, 1, 3, 0, 3], np.int32)
    v = np.array([1.0, 1.0, 1.0, 1.0, 1.0, -1.0])
    sense = np.array([ord("G"), ord("L"), ord("E"), ord("L")], np.uint8)
    return g.LP(4, 5, rp, ci, v, np.array([1.0, 2.0, 3.0, 1.0, -1.0]), np.array([1.0, 2.0, 1.0, 0.5]), sense,
                np.zeros(5), np.ones(5))


@pytest.mark.parametrize("col_blocks", [0, 1])
def test_batch_with_degenerate_members_matches_single(col_blocks):
    """col_blocks = 1 puts every member with rows and columns on column blocks and row blocks
    (a row-less member, a 1 x 1 member, empty rows and columns)."""
    lps = [box_only(2, n=50)[0], one_by_one(), g.set_cover(4, m=120, n=300, k=4), box_only(3, n=7)[0],
           empty_lines()]
    with pdlp.Batch(lps, precision="fp32", tile_nnz=512, col_blocks=col_blocks) as b:
        infos = b.solve(tol=1e-6, iter_limit=30_000)
        sols = [b.get(i) for i in range(len(lps))]
    for lp, info, sol in zip(lps, infos, sols):
        assert info["status_name"] == "optimal", (lp.name, info["status_name"])
        with pdlp.Problem(lp, precision="fp32", tile_nnz=512, col_blocks=col_blocks) as p:
            one = p.solve(tol=1e-6, iter_limit=30_000)
            s1 = p.get()
        assert info["iterations"] == one["iterations"] and info["status_name"] == one["status_name"]
        np.testing.assert_array_equal(sol.x, s1.x)
        np.testing.assert_array_equal(sol.y, s1.y)


def test_network_on_degenerate_batch_matches_oracle():
    """Forward pass over a batch with a row-less instance and a 1 x 1 instance."""
    from test_gpu_gnn import oracle_graph, _rel
    lps = [box_only(5, n=40)[0], one_by_one(), g.set_cover(6, m=90, n=200, k=3)]
    with pdlp.Batch(lps, precision="fp32") as b:
        G, *_ = oracle_graph(b, lps)
        net = pdlp.WarmStartNet(seed=2)
        p = net.params()
        xh, yh, lw = net.predict_raw(b)
        x0, y0, om = net.predict(b)
    ox, oy, olw, _ = go.forward(p.astype(np.float64), G, emulate_bf16=True)
    assert _rel(xh, ox) <= 1e-4 and _rel(yh, oy) <= 1e-4 and _rel(lw, olw) <= 1e-4
    assert np.all(np.isfinite(x0)) and np.all(np.isfinite(y0)) and np.all(om > 0)
