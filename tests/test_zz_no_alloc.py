"""The allocation-free variable-strategy entry point (pdlp_variable_strategy_noalloc) against the
allocating one (pdlp_variable_strategy) and the oracle, through the C-ABI: two calls in a row, the
second on a smaller problem, must give the same order bit for bit (integer work: the sort keys are
exact functions of the inputs); inputs in host memory and a problem beyond the static buffer are
rejected before any work."""
import ctypes as C
import sys

import numpy as np
import pytest

from oracle import fix_oracle as fo
from paper_2503_10344_amd import generators as g

pytestmark = pytest.mark.gpu


def say(*a):
    print("[gpu-test]", *a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def env():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2503_10344_amd import pdlp
    pdlp.load()
    return torch, pdlp


def _orders(torch, pdlp, lp, d, strategy, tiebreak):
    """(allocating entry point, allocation-free entry point, oracle) orders for the same inputs,
    all in device memory."""
    lib = pdlp.load()
    dev = torch.device("cuda:0")
    vt = torch.from_numpy(np.ascontiguousarray(d["var_type"], np.uint8)).to(dev)
    x, y, rc = (torch.from_numpy(np.ascontiguousarray(d[k], np.float64)).to(dev) for k in ("x", "y", "rc"))
    torch.cuda.synchronize()
    out = []
    with pdlp.Problem(lp) as p:
        for fn in (lib.pdlp_variable_strategy, lib.pdlp_variable_strategy_noalloc):
            order = torch.full((max(lp.n, 1),), -7, dtype=torch.int32, device=dev)
            cnt = C.c_int32(-1)
            rc_ = fn(p.h, strategy, tiebreak, vt.data_ptr(), x.data_ptr(), y.data_ptr(), rc.data_ptr(),
                     order.data_ptr(), C.byref(cnt))
            assert rc_ == 0, lib.pdlp_last_error().decode()
            out.append(order[:cnt.value].cpu().numpy())
    ref = fo.variable_order(strategy, tiebreak, d["x"], d["y"], d["rc"], d["var_type"], lp.m, lp.n, lp.row_ptr,
                            lp.col)
    return out[0], out[1], ref


def test_noalloc_matches_allocating_entry_point_twice(env):
    torch, pdlp = env
    big = g.general_sparse(4, m=60_000, n=120_000, cap=2000)
    small = g.set_cover(5, m=700, n=1500)
    for lp, strategy, tiebreak in ((big, pdlp.ORDER_FRAC, pdlp.ORDER_DUAL), (small, pdlp.ORDER_DUAL, pdlp.ORDER_FRAC),
                                   (small, pdlp.ORDER_REDCOST, pdlp.ORDER_TYPE)):
        d = g.fixing_inputs(11, lp)
        say("noalloc", lp.name, "strategy", strategy, "tiebreak", tiebreak, "n", lp.n)
        a, b, ref = _orders(torch, pdlp, lp, d, strategy, tiebreak)
        say("  ordered", a.size, "variables")
        assert a.size > 1000 or lp is small
        assert np.array_equal(a, b)
        assert np.array_equal(b, ref)


def test_noalloc_rejects_host_inputs_and_oversized_problems(env):
    torch, pdlp = env
    lib = pdlp.load()
    lp = g.set_cover(6, m=300, n=800)
    d = g.fixing_inputs(6, lp)
    vt = np.ascontiguousarray(d["var_type"], np.uint8)
    x = np.ascontiguousarray(d["x"], np.float64)
    order = np.zeros(lp.n, np.int32)
    cnt = C.c_int32(-1)
    with pdlp.Problem(lp) as p:
        rc_ = lib.pdlp_variable_strategy_noalloc(p.h, pdlp.ORDER_FRAC, pdlp.ORDER_NONE, vt.ctypes.data, x.ctypes.data,
                                                 None, None, order.ctypes.data, C.byref(cnt))
        assert rc_ == -1 and "device pointers" in lib.pdlp_last_error().decode()
    # a Frac order of 3.5M columns needs about 20 bytes per column, 71 MB: more than the 64 MiB buffer
    n = 3_500_000
    rp = np.array([0, n], np.int32)
    big = g.LP(1, n, rp, np.arange(n, dtype=np.int32), np.ones(n), np.ones(n), np.ones(1), np.array([ord("G")], np.uint8),
               np.zeros(n), np.ones(n), name="wide")
    dev = torch.device("cuda:0")
    vt_d = torch.ones(n, dtype=torch.uint8, device=dev)
    x_d = torch.full((n,), 0.25, dtype=torch.float64, device=dev)
    order_d = torch.empty(n, dtype=torch.int32, device=dev)
    with pdlp.Problem(big) as p:
        rc_ = lib.pdlp_variable_strategy_noalloc(p.h, pdlp.ORDER_FRAC, pdlp.ORDER_NONE, vt_d.data_ptr(),
                                                 x_d.data_ptr(), None, None, order_d.data_ptr(), C.byref(cnt))
        assert rc_ == -1 and "64 MiB" in lib.pdlp_last_error().decode()
        # the allocating entry point still serves it, and the handle is intact
        k = p.variable_strategy(pdlp.ORDER_FRAC, vt_d, x=x_d, tiebreak=pdlp.ORDER_NONE)
        assert k.numel() == n and torch.equal(k.cpu(), torch.arange(n, dtype=torch.int32))
