"""The bound to which the GPU's FP64 iterates must track the oracle's (test helper, CPU).

Two exact implementations of the same method differ only in rounding: the order of every sum
(matrix rows, reductions, norms), and the last bit of library functions. PDHG amplifies such
differences from attempt to attempt, so no fixed relative bound holds for all attempts. The
reference divergence D_k is measured on the oracle itself: the running maximum, over attempts
1..k, of the relative difference between its iterates and those of the same oracle with every sum
taken in another valid order (reversed, and even indices before odd ones). The GPU, whose sums use
yet another order (lane-strided partial sums and shuffle trees), must stay within
    B_k = max(1e-9, 2 D_k),
i.e. the flat 1e-9 wherever the order-induced divergence stays below 5e-10, and at most twice the
spread of the oracle's own summation orders beyond that.
"""
import numpy as np

import oracle

ALT_ORDERS = (1, 2)
FACTOR = 2.0
FLOOR = 1e-9


def order_divergence(lp, K, trace):
    """D_k for k = 1..K (running maximum) against `trace`, the forward-order oracle's trace."""
    div = np.zeros(K)
    for so in ALT_ORDERS:
        t2 = oracle.solve(lp, tol=0.0, iter_limit=K, trace_len=K, sum_order=so).trace
        for key in ("x", "y"):
            d = np.linalg.norm(t2[key] - trace[key], axis=1) / np.maximum(np.linalg.norm(trace[key], axis=1), 1e-30)
            div = np.maximum(div, d)
    return np.maximum.accumulate(div)


def tracking_bound(lp, K, trace):
    """B_k = max(1e-9, 2 D_k) for k = 1..K."""
    return np.maximum(FLOOR, FACTOR * order_divergence(lp, K, trace))
