"""Seeded synthetic LP generators.

These build the instances that stand in for the paper's data sets (MIPLIB 2017 and the UNSEEN energy
system models, section "Energy system optimization models", Table 1), which are not available here.
The module holds instance construction only: no part of the PDHG method lives here. Both the GPU path
and the CPU oracle read problems produced by it.

Every problem is the LP of eq. (1) with row senses widened to <=, >= and = (energy models carry
equalities), returned as CSR with int32 indices and float64 values, senses as ASCII codes 'L', 'G', 'E'
and bounds that may be +-inf.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

INF = np.inf
L_, G_, E_ = ord("L"), ord("G"), ord("E")


@dataclass
class LP:
    m: int
    n: int
    row_ptr: np.ndarray  # int32 [m+1]
    col: np.ndarray      # int32 [nnz]
    val: np.ndarray      # float64 [nnz]
    c: np.ndarray        # float64 [n]
    b: np.ndarray        # float64 [m]
    sense: np.ndarray    # uint8 [m], ord('L'|'G'|'E')
    l: np.ndarray        # float64 [n], may be -inf
    u: np.ndarray        # float64 [n], may be +inf
    name: str = ""
    meta: dict = field(default_factory=dict)

    @property
    def nnz(self) -> int:
        return int(self.row_ptr[-1])

    def row_lengths(self) -> np.ndarray:
        return np.diff(self.row_ptr.astype(np.int64))

    def to_scipy(self):
        import scipy.sparse as sp
        return sp.csr_matrix((self.val, self.col, self.row_ptr), shape=(self.m, self.n))


def _csr_from_triplets(m: int, n: int, rows, cols, vals):
    rows = np.asarray(rows, dtype=np.int64)
    cols = np.asarray(cols, dtype=np.int64)
    vals = np.asarray(vals, dtype=np.float64)
    order = np.lexsort((cols, rows))
    rows, cols, vals = rows[order], cols[order], vals[order]
    if rows.size:
        dup = (rows[1:] == rows[:-1]) & (cols[1:] == cols[:-1])
        if dup.any():
            raise ValueError("duplicate (row, col) entries")
    counts = np.bincount(rows, minlength=m) if rows.size else np.zeros(m, np.int64)
    row_ptr = np.zeros(m + 1, dtype=np.int64)
    np.cumsum(counts, out=row_ptr[1:])
    if row_ptr[-1] >= 2**31:
        raise ValueError("nnz exceeds int32 range")
    return row_ptr.astype(np.int32), cols.astype(np.int32), vals


def _distinct_in_segments(rng, seg_len: np.ndarray, universe: int) -> np.ndarray:
    """For segment s draw seg_len[s] distinct integers uniformly from [0, universe).

    Returns the flat array, segments contiguous and each segment sorted ascending.
    """
    seg_len = np.asarray(seg_len, dtype=np.int64)
    if seg_len.size and seg_len.max() > universe:
        raise ValueError("segment longer than the universe it draws from")
    total = int(seg_len.sum())
    seg_id = np.repeat(np.arange(seg_len.size, dtype=np.int64), seg_len)
    vals = rng.integers(0, universe, size=total, dtype=np.int64)
    while True:
        order = np.lexsort((vals, seg_id))
        vals = vals[order]  # seg_id is already sorted, so it is unchanged by the permutation
        dup = np.zeros(total, dtype=bool)
        if total > 1:
            dup[1:] = (vals[1:] == vals[:-1]) & (seg_id[1:] == seg_id[:-1])
        nd = int(dup.sum())
        if nd == 0:
            return vals
        vals[dup] = rng.integers(0, universe, size=nd, dtype=np.int64)


# ----------------------------------------------------------------------------------------------
# Tiny dense LPs (for brute-force vertex enumeration)
# ----------------------------------------------------------------------------------------------
def tiny_lp(seed: int, m: int = 4, n: int = 4, density: float = 0.8) -> LP:
    """Small LP with integer data, a finite box, mixed senses, feasible by construction."""
    rng = np.random.default_rng(seed)
    A = rng.integers(-5, 6, size=(m, n)).astype(np.float64)
    A[rng.random((m, n)) > density] = 0.0
    for i in range(m):  # no empty rows
        if not A[i].any():
            A[i, rng.integers(0, n)] = float(rng.integers(1, 6))
    lo = rng.integers(-3, 1, size=n).astype(np.float64)
    hi = lo + rng.integers(1, 6, size=n)
    x0 = lo + (hi - lo) * rng.random(n)
    sense = rng.choice(np.array([L_, G_, E_], dtype=np.uint8), size=m, p=[0.45, 0.35, 0.2])
    ax0 = A @ x0
    slack = rng.integers(0, 4, size=m).astype(np.float64)
    b = np.where(sense == L_, np.ceil(ax0) + slack, np.where(sense == G_, np.floor(ax0) - slack, ax0))
    c = rng.integers(-9, 10, size=n).astype(np.float64)
    rows, cols = np.nonzero(A)
    rp, ci, v = _csr_from_triplets(m, n, rows, cols, A[rows, cols])
    return LP(m, n, rp, ci, v, c, b, sense, lo, hi, name=f"tiny[{seed}]")


# ----------------------------------------------------------------------------------------------
# Set cover (LP relaxation of a set-cover MIP)
# ----------------------------------------------------------------------------------------------
def set_cover(seed: int, m: int = 2000, n: int = 5000, k: int = 5) -> LP:
    """Columns with k ones in distinct uniform rows, c_j ~ U{1..100}, rows A x >= 1, 0 <= x <= 1.

    If a row is left empty the whole draw is repeated with the next sub-seed.
    """
    sub = 0
    while True:
        rng = np.random.default_rng([seed, sub])
        rows = _distinct_in_segments(rng, np.full(n, k), m)
        if np.bincount(rows, minlength=m).min() > 0:
            break
        sub += 1
    cols = np.repeat(np.arange(n), k)
    c = rng.integers(1, 101, size=n).astype(np.float64)
    rp, ci, v = _csr_from_triplets(m, n, rows, cols, np.ones(rows.size))
    return LP(m, n, rp, ci, v, c, np.ones(m), np.full(m, G_, np.uint8), np.zeros(n), np.ones(n),
              name=f"setcover[{seed}] {m}x{n}", meta={"sub_seed": sub})


def multi_knapsack(seed, m: int = 2000, n: int = 5000, kmin: int = 4, kmax: int = 8) -> LP:
    """Columns with U{kmin..kmax} entries a ~ U{1..100} in distinct rows; rows <= 0.3 * row sum;
    c = -p with p ~ U{1..100}; 0 <= x <= 1."""
    rng = np.random.default_rng(seed)
    kcol = rng.integers(kmin, kmax + 1, size=n)
    rows = _distinct_in_segments(rng, kcol, m)
    cols = np.repeat(np.arange(n), kcol)
    a = rng.integers(1, 101, size=rows.size).astype(np.float64)
    rp, ci, v = _csr_from_triplets(m, n, rows, cols, a)
    rsum = np.add.reduceat(v, rp[:-1]) if v.size else np.zeros(m)
    rsum[np.diff(rp) == 0] = 0.0
    b = 0.3 * rsum
    c = -rng.integers(1, 101, size=n).astype(np.float64)
    return LP(m, n, rp, ci, v, c, b, np.full(m, L_, np.uint8), np.zeros(n), np.ones(n),
              name=f"knapsack {m}x{n}")


# ----------------------------------------------------------------------------------------------
# General sparse LP with Zipf row lengths
# ----------------------------------------------------------------------------------------------
def zipf_row_lengths(rng, m: int, exponent: float = 1.5, cap: int = 5000) -> np.ndarray:
    support = np.arange(1, cap + 1, dtype=np.float64)
    p = support ** (-exponent)
    cdf = np.cumsum(p)
    cdf /= cdf[-1]
    return (np.searchsorted(cdf, rng.random(m), side="right") + 1).astype(np.int64).clip(1, cap)


def general_sparse(seed: int, m: int = 500_000, n: int = 1_000_000, exponent: float = 1.5,
                   cap: int = 5000, frac_eq: float = 0.4, frac_boxed: float = 0.7) -> LP:
    """General sparse LP.

    Row lengths ~ Zipf(exponent) on {1..cap}, distinct uniform columns; values N(0,1) with 5 %
    replaced by +-1; 40 % equality rows and 60 % <= rows; bounds [0, 10] on 70 % of the columns and
    free on the rest. b = A x0 (+ U[0,1] slack on <= rows) for x0 uniform in the bounds (U[-10, 10] on
    free columns). c ~ N(0,1) on boxed columns; on free columns c = A^T y0 for a y0 that is sign-feasible
    for the row senses, which makes the LP dual feasible and therefore bounded.
    """
    rng = np.random.default_rng(seed)
    cap = min(cap, n)
    lens = zipf_row_lengths(rng, m, exponent, cap)
    cols = _distinct_in_segments(rng, lens, n)
    rows = np.repeat(np.arange(m, dtype=np.int64), lens)
    vals = rng.standard_normal(cols.size)
    pm = rng.random(cols.size) < 0.05
    vals[pm] = np.where(rng.random(int(pm.sum())) < 0.5, -1.0, 1.0)
    # rows and cols are already in CSR order (row-major, columns sorted within each row)
    row_ptr = np.zeros(m + 1, dtype=np.int64)
    np.cumsum(lens, out=row_ptr[1:])
    if row_ptr[-1] >= 2**31:
        raise ValueError("nnz exceeds int32 range")
    rp, ci = row_ptr.astype(np.int32), cols.astype(np.int32)
    sense = np.where(rng.random(m) < frac_eq, E_, L_).astype(np.uint8)
    boxed = rng.random(n) < frac_boxed
    lo = np.where(boxed, 0.0, -INF)
    hi = np.where(boxed, 10.0, INF)
    x0 = np.where(boxed, 10.0 * rng.random(n), -10.0 + 20.0 * rng.random(n))
    import scipy.sparse as sp
    A = sp.csr_matrix((vals, ci, rp), shape=(m, n))
    ax0 = A @ x0
    b = np.where(sense == E_, ax0, ax0 + rng.random(m))
    dbar = max(cols.size / max(n, 1), 1.0)
    g = rng.standard_normal(m)
    y0 = np.where(sense == E_, g, -np.abs(g)) / np.sqrt(dbar)
    aty0 = A.T @ y0
    c = np.where(boxed, rng.standard_normal(n), aty0)
    return LP(m, n, rp, ci, vals, c, b, sense, lo, hi,
              name=f"zipf[{seed}] {m}x{n}", meta={"exponent": exponent, "cap": cap, "x0": x0})


# ----------------------------------------------------------------------------------------------
# Energy-system-shaped LP (dispatch + capacity expansion + storage + transport network)
# ----------------------------------------------------------------------------------------------
def energy(seed: int, T: int = 8760, N: int = 100, K: int = 6, E: int = 200) -> LP:
    """Hourly dispatch / expansion LP shaped like the paper's energy system models.

    Columns, time-major: per step t the dispatch g[t,n,k] >= 0, storage level s[t,n] in [0, 4 d_n],
    charge ch[t,n] and discharge dis[t,n] in [0, d_n], line flows f[t,e] in [-F_e, F_e]; then the
    capacities cap[n,k] >= 0 shared by all steps. Rows, time-major: per step the capacity rows
    g - a[t,n,k] cap <= 0, the node balances sum_k g + dis - ch + (incident flows) = d[t,n] and the
    storage links s_t - s_{t-1} - 0.9 ch + dis = 0 (cyclic in t). Demand ~ lognormal(0, 0.5),
    availability ~ U[0,1], costs ~ U[1,100] on dispatch and capacity.
    """
    if T < 2 or N < 3:
        raise ValueError("energy(): needs T >= 2 and N >= 3")
    rng = np.random.default_rng(seed)
    E = max(E, N)
    # network: ring plus random chords
    ring = [(i, (i + 1) % N) for i in range(N)] if N > 2 else []
    chords = []
    while len(ring) + len(chords) < E:
        a, b = rng.integers(0, N, size=2)
        if a != b:
            chords.append((int(a), int(b)))
    lines = np.array(ring + chords, dtype=np.int64).reshape(-1, 2)
    E = lines.shape[0]
    d = rng.lognormal(0.0, 0.5, size=(T, N))
    dmean = d.mean(axis=0)
    avail = rng.random((T, N, K))
    cost_g = rng.uniform(1.0, 100.0, size=(N, K))
    cost_cap = rng.uniform(1.0, 100.0, size=(N, K))
    Fcap = rng.uniform(0.5, 2.0, size=E) * d.mean()

    per_t_cols = N * K + 3 * N + E
    ncol = T * per_t_cols + N * K
    per_t_rows = N * K + 2 * N
    mrow = T * per_t_rows

    t = np.arange(T, dtype=np.int64)[:, None]
    nn = np.arange(N, dtype=np.int64)[None, :]
    base_c = t * per_t_cols
    g_idx = base_c[:, :, None] + (np.arange(N)[:, None] * K + np.arange(K)[None, :])[None, :, :]
    s_idx = base_c + N * K + nn
    ch_idx = base_c + N * K + N + nn
    dis_idx = base_c + N * K + 2 * N + nn
    f_idx = base_c + N * K + 3 * N + np.arange(E)[None, :]
    cap_idx = T * per_t_cols + (np.arange(N)[:, None] * K + np.arange(K)[None, :])

    base_r = t * per_t_rows
    capr = base_r[:, :, None] + (np.arange(N)[:, None] * K + np.arange(K)[None, :])[None, :, :]
    balr = base_r + N * K + nn
    stor = base_r + N * K + N + nn

    R, C, V = [], [], []
    # capacity rows: g - a cap <= 0
    R += [capr.ravel(), capr.ravel()]
    C += [g_idx.ravel(), np.broadcast_to(cap_idx[None], (T, N, K)).ravel()]
    V += [np.ones(T * N * K), -avail.ravel()]
    # balance rows
    R += [np.repeat(balr.ravel(), K)]
    C += [g_idx.reshape(T * N, K).ravel()]
    V += [np.ones(T * N * K)]
    R += [balr.ravel(), balr.ravel()]
    C += [dis_idx.ravel(), ch_idx.ravel()]
    V += [np.ones(T * N), -np.ones(T * N)]
    src, dst = lines[:, 0], lines[:, 1]
    R += [(base_r + N * K + src[None, :]).ravel(), (base_r + N * K + dst[None, :]).ravel()]
    C += [f_idx.ravel(), f_idx.ravel()]
    V += [-np.ones(T * E), np.ones(T * E)]
    # storage rows: s_t - s_{t-1} - 0.9 ch + dis = 0 (cyclic)
    prev_s = np.roll(s_idx, 1, axis=0)
    R += [stor.ravel()] * 4
    C += [s_idx.ravel(), prev_s.ravel(), ch_idx.ravel(), dis_idx.ravel()]
    V += [np.ones(T * N), -np.ones(T * N), -0.9 * np.ones(T * N), np.ones(T * N)]
    rows = np.concatenate(R)
    cols = np.concatenate(C)
    vals = np.concatenate(V)
    rp, ci, v = _csr_from_triplets(mrow, ncol, rows, cols, vals)

    c = np.zeros(ncol)
    c[g_idx.ravel()] = np.broadcast_to(cost_g[None], (T, N, K)).ravel()
    c[cap_idx.ravel()] = cost_cap.ravel()
    lo = np.zeros(ncol)
    hi = np.full(ncol, INF)
    hi[s_idx.ravel()] = np.broadcast_to(4.0 * dmean[None, :], (T, N)).ravel()
    hi[ch_idx.ravel()] = np.broadcast_to(dmean[None, :], (T, N)).ravel()
    hi[dis_idx.ravel()] = np.broadcast_to(dmean[None, :], (T, N)).ravel()
    lo[f_idx.ravel()] = np.broadcast_to(-Fcap[None, :], (T, E)).ravel()
    hi[f_idx.ravel()] = np.broadcast_to(Fcap[None, :], (T, E)).ravel()
    b = np.zeros(mrow)
    b[balr.ravel()] = d.ravel()
    sense = np.full(mrow, E_, np.uint8)
    sense[capr.ravel()] = L_
    return LP(mrow, ncol, rp, ci, v, c, b, sense, lo, hi,
              name=f"energy[{seed}] T={T} N={N} K={K} E={E}", meta={"T": T, "N": N, "K": K, "E": E})


# ----------------------------------------------------------------------------------------------
# Batched family: uneven set-cover / multi-knapsack relaxations
# ----------------------------------------------------------------------------------------------
def batch_member(batch_seed: int, i: int, m_lo: int = 1000, m_hi: int = 50_000) -> LP:
    rng = np.random.default_rng([batch_seed, i])
    m = int(rng.integers(m_lo, m_hi + 1))
    n = int(round(2.5 * m))
    sub_seed = [batch_seed, i, 1]
    if i % 2 == 0:
        k = int(rng.integers(4, 9))
        lp = set_cover(int(np.random.default_rng(sub_seed).integers(0, 2**31 - 1)), m, n, k)
    else:
        lp = multi_knapsack(np.random.default_rng(sub_seed).integers(0, 2**31 - 1), m, n)
    lp.name = f"batch[{batch_seed},{i}] " + lp.name
    return lp


def batch(batch_seed: int, count: int = 256, m_lo: int = 1000, m_hi: int = 50_000) -> list:
    return [batch_member(batch_seed, i, m_lo, m_hi) for i in range(count)]


# ----------------------------------------------------------------------------------------------
# Family used for the learned warm start (small energy-shaped LPs)
# ----------------------------------------------------------------------------------------------
def warmstart_family(seed: int, m_lo: int = 10_000, m_hi: int = 100_000) -> LP:
    rng = np.random.default_rng([7, seed])
    N = int(rng.integers(5, 21))
    m_target = float(rng.uniform(m_lo, m_hi))
    T = max(2, int(round(m_target / (N * 8))))
    return energy(int(rng.integers(0, 2**31 - 1)), T=T, N=N, K=6, E=2 * N)


# ----------------------------------------------------------------------------------------------
# Inputs of the LP-based variable strategies and LP-based fixing (random draws only)
# ----------------------------------------------------------------------------------------------
VAR_CONTINUOUS, VAR_BINARY, VAR_INTEGER = 0, 1, 2


def fixing_inputs(seed: int, lp: LP, int_share: float = 0.6, tie_share: float = 0.3) -> dict:
    """Seeded stand-ins for an LP solution and a MIP's integrality: variable types (binary where the
    bounds are [0, 1], otherwise integer with probability int_share, else continuous), a point x
    inside the bounds, duals y, reduced costs rc and one uniform sample in (0, 1) per variable.

    A share tie_share of x, |y| and rc is drawn from small grids (eighths, a few magnitudes), so that
    orderings meet many equal keys; some x are integral and some rc are zero.
    """
    rng = np.random.default_rng([11, seed])
    n, m = lp.n, lp.m
    lo = np.where(np.isfinite(lp.l), lp.l, -20.0)
    hi = np.where(np.isfinite(lp.u), lp.u, 20.0)
    hi = np.maximum(hi, lo)
    binary = (lp.l == 0.0) & (lp.u == 1.0)
    vtype = np.where(binary, VAR_BINARY,
                     np.where(rng.random(n) < int_share, VAR_INTEGER, VAR_CONTINUOUS)).astype(np.uint8)
    x = lo + (hi - lo) * rng.random(n)
    grid = rng.random(n) < tie_share
    x = np.where(grid, np.clip(np.floor(x) + rng.integers(0, 9, n) / 8.0, lo, hi), x)
    y = rng.standard_normal(m) * np.exp(rng.normal(0.0, 1.0, m))
    ygrid = rng.random(m) < tie_share
    y = np.where(ygrid, rng.choice([-2.0, -0.5, 0.0, 0.5, 2.0], m), y)
    rc = rng.standard_normal(n) * np.exp(rng.normal(0.0, 1.0, n))
    rgrid = rng.random(n) < tie_share
    rc = np.where(rgrid, rng.choice([-1.0, 0.0, 0.0, 0.25, 1.0], n), rc)
    uniform = (rng.integers(0, 2**53, n, dtype=np.int64).astype(np.float64) + 0.5) * 2.0**-53
    return dict(var_type=vtype, x=x, y=y, rc=rc, uniform=uniform)


def feasible_binary_point(seed: int, lp: LP) -> np.ndarray:
    """A random 0/1 point satisfying every row of a set-cover (>= 1) or multi-knapsack (<=) LP: a
    random cover (one random column of each row set to 1), or items added in random order while
    every row stays within its capacity."""
    rng = np.random.default_rng([17, seed])
    x = np.zeros(lp.n)
    if np.all(lp.sense == G_):
        for i in rng.permutation(lp.m):
            cols = lp.col[lp.row_ptr[i]:lp.row_ptr[i + 1]]
            if not np.any(x[cols] > 0):
                x[rng.choice(cols)] = 1.0
        return x
    At = lp.to_scipy().T.tocsr()
    load = np.zeros(lp.m)
    for j in rng.permutation(lp.n):
        rows, a = At.indices[At.indptr[j]:At.indptr[j + 1]], At.data[At.indptr[j]:At.indptr[j + 1]]
        if np.all(load[rows] + a <= lp.b[rows]):
            load[rows] += a
            x[j] = 1.0
    return x
