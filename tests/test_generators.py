"""Seeded generators: determinism and the statistics the workloads are specified by."""
import numpy as np

from paper_2503_10344_amd import generators as g


def _same(a, b):
    for f in ("row_ptr", "col", "val", "c", "b", "sense", "l", "u"):
        assert np.array_equal(getattr(a, f), getattr(b, f)), f


def test_deterministic():
    _same(g.set_cover(3, 200, 500), g.set_cover(3, 200, 500))
    _same(g.general_sparse(2, 2000, 4000), g.general_sparse(2, 2000, 4000))
    _same(g.energy(1, T=10, N=4, K=3, E=6), g.energy(1, T=10, N=4, K=3, E=6))
    _same(g.batch_member(0, 5, 1000, 2000), g.batch_member(0, 5, 1000, 2000))


def _csr_ok(lp):
    rp = lp.row_ptr.astype(np.int64)
    assert rp[0] == 0 and np.all(np.diff(rp) >= 0) and rp[-1] == lp.col.size == lp.val.size
    assert lp.col.min() >= 0 and lp.col.max() < lp.n
    for i in range(0, lp.m, max(1, lp.m // 200)):
        seg = lp.col[rp[i]:rp[i + 1]]
        assert np.all(np.diff(seg) > 0)  # sorted, no duplicates
    assert np.all(lp.l <= lp.u)


def test_set_cover_shape():
    lp = g.set_cover(0)
    _csr_ok(lp)
    assert (lp.m, lp.n, lp.nnz) == (2000, 5000, 25000)
    assert np.bincount(lp.col, minlength=lp.n).tolist() == [5] * 5000
    assert lp.row_lengths().min() >= 1
    assert lp.c.min() >= 1 and lp.c.max() <= 100 and np.all(lp.c == np.round(lp.c))
    assert np.all(lp.sense == ord("G")) and np.all(lp.b == 1)


def test_general_sparse_statistics():
    lp = g.general_sparse(0, m=20000, n=40000)
    _csr_ok(lp)
    lens = lp.row_lengths()
    assert lens.max() <= 5000 and lens.min() >= 1
    # Zipf(1.5) on {1..5000}: P(L = 1) = 1/zeta_5000(1.5) ~ 0.386, mean ~ 54.2
    assert abs((lens == 1).mean() - 0.386) < 0.02
    assert 40 < lens.mean() < 70
    eq = (lp.sense == ord("E")).mean()
    assert abs(eq - 0.4) < 0.02
    free = ~np.isfinite(lp.l)
    assert abs(free.mean() - 0.3) < 0.02
    assert np.all(lp.l[~free] == 0) and np.all(lp.u[~free] == 10)
    pm1 = np.isin(lp.val, (-1.0, 1.0)).mean()
    assert abs(pm1 - 0.05) < 0.01


def test_energy_block_counts():
    T, N, K, E = 24, 10, 6, 20
    lp = g.energy(0, T=T, N=N, K=K, E=E)
    _csr_ok(lp)
    assert lp.m == T * (N * K + 2 * N)
    assert lp.n == T * (N * K + 3 * N + E) + N * K
    assert lp.nnz == T * (2 * N * K + (N * K + 2 * N + 2 * E) + 4 * N)
    assert (lp.sense == ord("L")).sum() == T * N * K
    # the full-size instance has the sizes the workload states
    T, N, K, E = 8760, 100, 6, 200
    assert T * (N * K + 2 * N) == 7_008_000
    assert T * (2 * N * K + (N * K + 2 * N + 2 * E) + 4 * N) == 24_528_000


def test_batch_member_ranges():
    for i in range(4):
        lp = g.batch_member(0, i, 1000, 3000)
        _csr_ok(lp)
        assert 1000 <= lp.m <= 3000 and lp.n == round(2.5 * lp.m)
        deg = np.bincount(lp.col, minlength=lp.n)
        assert deg.min() >= 4 and deg.max() <= 8
