"""GPU parity at the full workload sizes, in the configuration the benchmark times (FP32 handle,
chunk size chosen at create time, hipGraph launches, kernel timing on).

The oracle cannot take these LPs to tolerance within a test, so each check is one it can afford:
  * sampled products: 4,096 random rows of A x plus the 64 longest rows and some empty ones, and the
    same for the columns of A'y; the expected entries are the oracle's CSR product over just those
    rows of A (or of the oracle's transpose). Tolerance as in the small SpMV test: FP32
    |err| <= 2e-6 (|A||x|)_i, FP64 1e-12.
  * scaling: the oracle's full Ruiz + Pock-Chambolle pass (C, a second or two) against the handle's
    Dr and Dc, 1e-12 relative (the two take the Pock-Chambolle sums in different orders).
  * first attempts: the FP64 handle's iterates after attempts 1..3 against the oracle's trace within
    1e-9 relative (the small tracking tests measure ~1e-13 this early); the FP32 handle after
    attempts 1..2 within 1e-5 relative. The initial primal weight ||c~|| / ||b~|| within
    1e-12 + 2 N u (N = max(m, n), u = 2^-53): the oracle sums each squared norm serially, with the
    worst-case relative error (N - 1) u of such a sum (energy-shaped LP: measured 1.1e-12, N ~ 1e7). FP32 rounding of the inputs and products gives
    a few 1e-7 per element (unit roundoff 6e-8, one rounding per stored value and per product, sums
    of up to 5,000 terms growing as their square root); 1e-5 leaves room for the extrapolation
    2 A x' - A x doubling it, and is far below what a wrong sign, index or dropped term would give.
    Attempts after an accept/reject decision whose relative margin in the oracle is below the
    tolerance are not compared.
  * end to end: the FP32 solve reaches relative KKT 1e-4 as the oracle re-evaluates the returned
    point on the original data (a property that holds at any size).
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

FP32_PRODUCT = 2e-6
FP64_PRODUCT = 1e-12
FP64_ITERATE = 1e-9
FP32_ITERATE = 1e-5


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


def _sub_csr(row_ptr, col, val, rows):
    """Rows `rows` of a CSR matrix as a CSR matrix of their own."""
    lens = (row_ptr[rows + 1] - row_ptr[rows]).astype(np.int64)
    rp = np.zeros(rows.size + 1, np.int64)
    np.cumsum(lens, out=rp[1:])
    idx = np.concatenate([np.arange(row_ptr[r], row_ptr[r + 1]) for r in rows]) if rp[-1] else np.zeros(0, int)
    return rp.astype(np.int32), col[idx], val[idx]


def _sample(lengths, rng, k=4096):
    """k random indices, the 64 longest and up to 16 empty ones."""
    longest = np.argsort(lengths, kind="stable")[-64:]
    empty = np.nonzero(lengths == 0)[0][:16]
    pick = rng.choice(lengths.size, size=min(k, lengths.size), replace=False)
    return np.unique(np.concatenate([pick, longest, empty]))


def _sampled_products(p, lp, At, prec, rng):
    """Sampled entries of A x and A'y, plain and as the iteration forms them (FP32 handles may
    sum long rows of A by column panels and A'y by column blocks), against the oracle."""
    tol = FP32_PRODUCT if prec == "fp32" else FP64_PRODUCT
    x = rng.standard_normal(lp.n)
    y = rng.standard_normal(lp.m)
    ax = p.spmv(x)
    aty = p.spmv(y, trans=True)
    ax_it = p.spmv(x, iteration=True)
    aty_it = p.spmv(y, trans=True, iteration=True)
    for name, (rp, ci, v), vec, out in (("A x", (lp.row_ptr, lp.col, lp.val), x, ax),
                                        ("A'y", At, y, aty),
                                        ("A x (iteration)", (lp.row_ptr, lp.col, lp.val), x, ax_it),
                                        ("A'y (iteration)", At, y, aty_it)):
        rows = _sample(np.diff(rp), rng)
        srp, sci, sv = _sub_csr(rp, ci, v, rows)
        ref = oracle.spmv(srp, sci, sv, vec)
        bound = oracle.spmv(srp, sci, np.abs(sv), np.abs(vec))
        err = np.abs(out[rows] - ref)
        say(prec, name, rows.size, "sampled entries, worst err / (|A||x|) %.2e"
            % float(np.max(err / np.maximum(bound, 1e-300))))
        assert np.all(err <= tol * bound + 1e-30), (name, prec)


def _first_attempts(pdlp, lp, trace, K, prec, **opts):
    tol = FP64_ITERATE if prec == "fp64" else FP32_ITERATE
    cut = K
    close = np.nonzero(trace["margin"][:K] < 10 * tol)[0]
    if close.size:
        cut = int(close[0])
        say(prec, "decision margin below tolerance at attempt", cut + 1)
    with pdlp.Problem(lp, precision=prec, **opts) as p:
        for k in range(1, cut + 1):
            p.solve(tol=0.0, iter_limit=k)
            sol = p.get()
            assert sol.info["iterations"] == k
            xo, yo = trace["x"][k - 1], trace["y"][k - 1]
            ex = np.linalg.norm(sol.x - xo) / max(np.linalg.norm(xo), 1e-30)
            ey = np.linalg.norm(sol.y - yo) / max(np.linalg.norm(yo), 1e-30)
            eom = abs(sol.info["omega"] - trace["omega"][k - 1]) / trace["omega"][k - 1]
            say(prec, "attempt", k, "rel err x %.2e y %.2e omega %.2e" % (ex, ey, eom))
            assert ex <= tol and ey <= tol, (prec, k, ex, ey)
            assert eom <= 1e-12 + 2.0 * max(lp.m, lp.n) * 2.0**-53, (prec, k, eom)
    return cut


def _full_size_checks(pdlp, lp, label, seed):
    rng = np.random.default_rng(seed)
    At = oracle.transpose(lp.m, lp.n, lp.row_ptr, lp.col, lp.val)
    Dr, Dc, _ = oracle.scale(lp)
    K = 3
    orc = oracle.solve(lp, tol=0.0, iter_limit=K, trace_len=K)
    for prec in ("fp32", "fp64"):
        with pdlp.Problem(lp, precision=prec, kernel_timing=True) as p:
            say(label, prec, "schedule", p.schedule())
            s = p.scaling()
            er = float(np.max(np.abs(s["Dr"] - Dr) / Dr))
            ec = float(np.max(np.abs(s["Dc"] - Dc) / Dc))
            say(label, prec, "scaling rel err Dr %.2e Dc %.2e" % (er, ec))
            assert er <= 1e-12 and ec <= 1e-12
            _sampled_products(p, lp, At, prec, rng)
    n64 = _first_attempts(pdlp, lp, orc.trace, K, "fp64", kernel_timing=True)
    n32 = _first_attempts(pdlp, lp, orc.trace, 2, "fp32", kernel_timing=True)
    assert n64 >= 1 and n32 >= 1


@pytest.fixture(scope="module")
def general_lp():
    say("generating the 500,000 x 1,000,000 general sparse LP (seed 0)")
    return g.general_sparse(0)


@pytest.fixture(scope="module")
def energy_lp():
    say("generating the 8760 x 100 x 6 energy-shaped LP (seed 0)")
    return g.energy(0)


def test_general_sparse_full_size_parity(pdlp, general_lp):
    _full_size_checks(pdlp, general_lp, "general 500k x 1M", 21)


def test_energy_full_size_parity(pdlp, energy_lp):
    _full_size_checks(pdlp, energy_lp, "energy 7.0M x 9.6M", 22)


@pytest.mark.parametrize("which", ["general", "energy"])
def test_full_size_solve_reaches_tolerance(pdlp, which, request):
    lp = request.getfixturevalue(f"{which}_lp")
    with pdlp.Problem(lp, precision="fp32", kernel_timing=True) as p:
        info = p.solve(tol=1e-4, iter_limit=500_000)
        sol = p.get()
    k = oracle.kkt(lp, sol.x, sol.y)
    say(which, info["status_name"], "attempts", info["iterations"], "%.2f s" % info["solve_seconds"],
        "device rel_kkt %.3e, oracle re-evaluation %.3e" % (info["rel_kkt"], k["rel_kkt"]))
    assert info["status"] == pdlp.OPTIMAL
    assert k["rel_kkt"] <= 1e-4
    # the objective the device reports is the one of the returned point
    assert abs(k["pobj"] - info["primal_obj"]) <= 1e-9 * max(1.0, abs(k["pobj"]))


def test_batch_full_size_members_reach_tolerance_and_match_single_solves(pdlp):
    """256 LPs (about 1e8 nonzeros) in one handle: every member's returned point passes the oracle's
    re-evaluation, and sampled members are bitwise the single-problem solve with the same chunk size
    (the chunk size fixes the grouping of the FP64 partial sums, hence the rounding of a
    trajectory) and the same column-block choice (the batch holds more than 2^20 nonzeros and every
    member's columns have at most 64 entries, so the batch gives every member column blocks; alone
    a member is below 2^20 nonzeros and takes them only with col_blocks = 1)."""
    say("generating the 256-LP batch (seed 0)")
    lps = g.batch(0)
    with pdlp.Batch(lps, precision="fp32") as bt:
        sched = bt.schedule()
        say("batch schedule", sched)
        infos = bt.solve(tol=1e-4, iter_limit=500_000)
        sols = [bt.get(i) for i in range(len(lps))]
    worst = 0.0
    for i, (lp, s) in enumerate(zip(lps, sols)):
        assert infos[i]["status"] == pdlp.OPTIMAL, i
        worst = max(worst, oracle.kkt(lp, s.x, s.y)["rel_kkt"])
    say("batch: all", len(lps), "optimal; worst oracle rel_kkt %.3e" % worst)
    assert worst <= 1e-4
    for i in (0, 1, 127, 255):
        with pdlp.Problem(lps[i], precision="fp32", tile_nnz=sched["tile_nnz"], col_blocks=1) as p:
            p.solve(tol=1e-4, iter_limit=500_000)
            s = p.get()
        say("batch member", i, "iterations", sols[i].info["iterations"], "single", s.info["iterations"])
        assert s.info["iterations"] == sols[i].info["iterations"]
        assert np.array_equal(s.x, sols[i].x) and np.array_equal(s.y, sols[i].y)
