"""Pins of the warm-start network oracle against things other than itself.

* gradients: central finite differences of the loss (the exact FP64 network);
* message directions: a hand-wired network whose output is a closed form evaluated with explicit
  loops over the nonzeros;
* features: hand-computed values on a 2 x 3 problem;
* equivariance: permuting variables and constraints of an instance permutes the outputs;
* independence: a batch of two instances gives each instance's own outputs;
* BF16 rounding: torch's float32 -> bfloat16 conversion (round to nearest even).
"""
import math

import numpy as np
import pytest
import torch

from oracle import gnn_oracle as go


def _graph(seed, m, n, K=1, dens=0.4, go=go):
    rng = np.random.default_rng(seed)
    rows, cols, vals = [], [], []
    row0, col0 = [0], [0]
    c, b, l, u, sense = [], [], [], [], []
    for q in range(K):
        mq, nq = m + q, n + 2 * q
        A = rng.normal(size=(mq, nq)) * (rng.random((mq, nq)) < dens)
        for i in range(mq):
            if not A[i].any():
                A[i, rng.integers(nq)] = 1.5
        r, cc = np.nonzero(A)
        rows += list(r + row0[-1]); cols += list(cc + col0[-1]); vals += list(A[r, cc])
        row0.append(row0[-1] + mq); col0.append(col0[-1] + nq)
        c += list(rng.normal(size=nq) * 3)
        b += list(rng.normal(size=mq))
        lo = np.where(rng.random(nq) < 0.7, rng.uniform(-2, 0, nq), -np.inf)
        hi = np.where(rng.random(nq) < 0.6, rng.uniform(1, 5, nq), np.inf)
        l += list(lo); u += list(hi)
        sense += list(rng.choice(np.frombuffer(b"LGE", np.uint8), size=mq))
    import scipy.sparse as sp
    M = sp.csr_matrix((vals, (rows, cols)), shape=(row0[-1], col0[-1]))
    M.sort_indices()
    return go.Graph(M.indptr, M.indices, M.data, np.array(c), np.array(b), np.array(l), np.array(u),
                    np.array(sense, np.uint8), np.array(row0), np.array(col0))


def _targets(G, seed):
    rng = np.random.default_rng(seed)
    return rng.normal(size=G.n), rng.normal(size=G.m), rng.normal(size=G.K)


def pin_bf16_rounding_matches_torch(go=go):
    rng = np.random.default_rng(0)
    v = np.concatenate([rng.normal(size=5000) * 10.0 ** rng.integers(-30, 30, 5000),
                        [0.0, -0.0, 1.0, 1.00390625, 1.01171875, 3.0e38, -1e-40]])
    v32 = v.astype(np.float32)
    ref = torch.from_numpy(v32).to(torch.bfloat16).to(torch.float64).numpy()
    np.testing.assert_array_equal(go.bf16(v32), ref)
    # exact ties go to even: 1 + 2^-8 sits halfway between 1 and 1 + 2^-7
    assert go.bf16(np.float32(1.0 + 2.0 ** -8)) == 1.0
    assert go.bf16(np.float32(1.0 + 3 * 2.0 ** -8)) == 1.0 + 2.0 ** -6


def pin_features_by_hand(go=go):
    # 2 constraints x 3 variables; row 0 = {0, 2}, row 1 = {1, 2}
    G = go.Graph(np.array([0, 2, 4]), np.array([0, 2, 1, 2]), np.array([1.0, -2.0, 3.0, 0.5]),
                 np.array([1.0, -np.e + 1, 0.0]), np.array([3.0, -1.0]),
                 np.array([0.0, -np.inf, -1.0]), np.array([np.inf, 2.0, 1.0]),
                 np.frombuffer(b"GE", np.uint8), np.array([0, 2]), np.array([0, 3]))
    fv, fc = go.features(G)
    l2, l3 = math.log(2.0), math.log(3.0)
    expect_v = [[l2, 1, 0, 0, 0, l2 / 4, 1, 0],
                [-1.0, 0, 1, 0, math.log(3.0), l2 / 4, 1, 0],
                [0, 1, 1, -l2, l2, l3 / 4, 1, 0]]
    expect_c = [[math.log(4.0), 0, 1, 0, l3 / 4, 1, 0, 0],
                [-l2, 0, 0, 1, l3 / 4, 1, 0, 0]]
    np.testing.assert_allclose(fv, expect_v, rtol=1e-6, atol=1e-7)
    np.testing.assert_allclose(fc, expect_c, rtol=1e-6, atol=1e-7)


def pin_message_directions_closed_form(go=go):
    """Wire the network so that x-hat = relu(A' relu(A relu(A' relu(A ... slog c)))) in channel 0."""
    G = _graph(3, 5, 7, go=go)
    P = {name: np.zeros(sh) for name, sh in go.param_shapes()}
    P["Wv_in"][0, 0] = 1.0           # hv[:,0] = relu(slog c)
    P["Wc_in"][0, 1] = 1.0           # hc[:,1] = relu(slog b)   (carried to check W1)
    for l in range(go.LAYERS):
        P[f"W2_{l}"][0, 0] = 1.0     # hc0 = relu(A hv0)
        P[f"W1_{l}"][1, 1] = 0.5     # hc1 = relu(0.5 hc1)
        P[f"W4_{l}"][0, 0] = 1.0     # hv0 = relu(A' hc0)
        P[f"W3_{l}"][0, 2] = 2.0     # hv2 = relu(2 hv0_prev)
    P["wx"][0] = 1.0; P["wx"][2] = 10.0; P["bx"][0] = 0.25
    P["wy"][0] = 1.0; P["wy"][1] = 3.0; P["by"][0] = -1.0
    P["wov"][0] = 1.0; P["woc"][1] = 1.0; P["bo"][0] = 0.5
    xh, yh, lw, _ = go.forward(go.pack(P), G, emulate_bf16=False)

    rp, ci, va = G.A.indptr, G.A.indices, G.A.data
    f32 = lambda t: float(np.float32(t))   # features are formed in binary32
    v0 = [max(f32(math.copysign(math.log1p(abs(cj)), cj)), 0.0) for cj in G.c]
    c1 = [max(f32(math.copysign(math.log1p(abs(bi)), bi)), 0.0) for bi in G.b]
    v_prev = v0
    for _ in range(go.LAYERS):
        c0 = [max(sum(va[e] * v0[ci[e]] for e in range(rp[i], rp[i + 1])), 0.0) for i in range(G.m)]
        c1 = [0.5 * t for t in c1]
        nv = [0.0] * G.n
        for i in range(G.m):
            for e in range(rp[i], rp[i + 1]):
                nv[ci[e]] += va[e] * c0[i]
        v_prev, v0 = v0, [max(t, 0.0) for t in nv]
        v2 = [2.0 * max(t, 0.0) for t in v_prev]
    expect_x = [v0[j] + 10.0 * v2[j] + 0.25 for j in range(G.n)]
    expect_y = [c0[i] + 3.0 * c1[i] - 1.0 for i in range(G.m)]
    expect_w = sum(v0) / G.n + sum(c1) / G.m + 0.5
    np.testing.assert_allclose(xh, expect_x, rtol=1e-12, atol=1e-12)
    np.testing.assert_allclose(yh, expect_y, rtol=1e-12, atol=1e-12)
    np.testing.assert_allclose(lw, [expect_w], rtol=1e-12)


def pin_gradients_by_finite_differences(go=go):
    G = _graph(1, 6, 9, K=2, go=go)
    xs, ys, lws = _targets(G, 2)
    flat = go.init_params(5)
    rng = np.random.default_rng(9)
    flat += rng.normal(size=flat.size) * 0.05     # non-zero biases
    w_om = 3.0   # a weight other than 1 on the log-omega term
    L, g = go.loss_and_grad(flat, G, xs, ys, lws, emulate_bf16=False, omega_weight=w_om)
    offs, o = {}, 0
    for name, sh in go.param_shapes():
        offs[name] = (o, int(np.prod(sh)))
        o += int(np.prod(sh))
    idx = []
    for name, (o, k) in offs.items():
        idx += list(o + rng.choice(k, size=min(k, 6), replace=False))
    h = 1e-6
    worst = 0.0
    for i in idx:
        fp = flat.copy(); fp[i] += h
        fm = flat.copy(); fm[i] -= h
        Lp, _ = go.loss_and_grad(fp, G, xs, ys, lws, emulate_bf16=False, omega_weight=w_om)
        Lm, _ = go.loss_and_grad(fm, G, xs, ys, lws, emulate_bf16=False, omega_weight=w_om)
        fd = (Lp - Lm) / (2 * h)
        err = abs(fd - g[i]) / max(1e-6, abs(fd), abs(g[i]))
        worst = max(worst, err)
        assert err < 1e-5 or abs(fd - g[i]) < 1e-9, (i, fd, g[i])
    assert L > 0 and np.isfinite(worst)


def pin_permutation_equivariance(go=go):
    G = _graph(4, 6, 8, go=go)
    flat = go.init_params(1) + np.random.default_rng(2).normal(size=go.num_params()) * 0.05
    xh, yh, lw, _ = go.forward(flat, G, emulate_bf16=False)
    rng = np.random.default_rng(3)
    pr, pc = rng.permutation(G.m), rng.permutation(G.n)
    A = G.A[pr][:, pc].tocsr()
    A.sort_indices()
    G2 = go.Graph(A.indptr, A.indices, A.data, G.c[pc], G.b[pr], G.l[pc], G.u[pc], G.sense[pr],
                  np.array([0, G.m]), np.array([0, G.n]))
    xh2, yh2, lw2, _ = go.forward(flat, G2, emulate_bf16=False)
    np.testing.assert_allclose(xh2, xh[pc], rtol=1e-11, atol=1e-12)
    np.testing.assert_allclose(yh2, yh[pr], rtol=1e-11, atol=1e-12)
    np.testing.assert_allclose(lw2, lw, rtol=1e-12)


def pin_instances_are_independent(go=go):
    G = _graph(6, 5, 7, K=2, go=go)
    flat = go.init_params(4)
    xh, yh, lw, _ = go.forward(flat, G, emulate_bf16=True)
    for q in range(2):
        r0, r1, c0, c1 = G.row0[q], G.row0[q + 1], G.col0[q], G.col0[q + 1]
        A = G.A[r0:r1][:, c0:c1].tocsr()
        Gq = go.Graph(A.indptr, A.indices, A.data, G.c[c0:c1], G.b[r0:r1], G.l[c0:c1], G.u[c0:c1],
                      G.sense[r0:r1], np.array([0, r1 - r0]), np.array([0, c1 - c0]))
        xq, yq, lq, _ = go.forward(flat, Gq, emulate_bf16=True)
        np.testing.assert_allclose(xq, xh[c0:c1], rtol=1e-12, atol=1e-13)
        np.testing.assert_allclose(yq, yh[r0:r1], rtol=1e-12, atol=1e-13)
        np.testing.assert_allclose(lq, lw[q:q + 1], rtol=1e-12)


def pin_bf16_emulation_is_close_to_exact(go=go):
    """The BF16-emulated network stays within BF16's relative precision of the exact one."""
    G = _graph(8, 20, 30, go=go)
    flat = go.init_params(6)
    xe, ye, _, _ = go.forward(flat, G, emulate_bf16=False)
    xb, yb, _, _ = go.forward(flat, G, emulate_bf16=True)
    assert np.linalg.norm(xb - xe) <= 0.05 * np.linalg.norm(xe) + 1e-6
    assert np.linalg.norm(yb - ye) <= 0.05 * np.linalg.norm(ye) + 1e-6
    assert not np.array_equal(xb, xe)



PINS = [pin_bf16_rounding_matches_torch, pin_features_by_hand, pin_message_directions_closed_form, pin_gradients_by_finite_differences, pin_permutation_equivariance, pin_instances_are_independent, pin_bf16_emulation_is_close_to_exact]


@pytest.mark.parametrize("pin", PINS, ids=lambda f: f.__name__)
def test_pin(pin):
    pin()


MUTANTS = {
    "stale_constraint_state": ("mv = G.AT @ hc_new", "mv = G.AT @ hc"),
    "transposed_backward_message": ("dhc = dhc + G.A @ dmv", "dhc = dhc + G.A @ dmv[:, ::-1]"),
    "backward_sign": ("dhv_prev = dhv_prev + G.AT @ dmc", "dhv_prev = dhv_prev - G.AT @ dmc"),
    "relu_mask_wrong_layer": ("dpv = dhv * (hv_l > 0)", "dpv = dhv * (hv_p > 0)"),
    "pooled_grad_wrong_side": ('g["wov"] = C["pv"].T @ dlw', 'g["wov"] = C["pc"].T @ dlw'),
    "lower_bound_feature_uses_upper": ("slog(np.where(lf, G.l, 0.0))", "slog(np.where(lf, G.u, 0.0))"),
    "sum_instead_of_mean_pool": ("return s / np.maximum(cnt, 1.0)[:, None], cnt", "return s, cnt"),
    "dual_loss_normalised_by_columns": ("dyh = 2.0 * ey / np.maximum(mq[G.rinst], 1.0) / K",
                                        "dyh = 2.0 * ey / np.maximum(nq[G.rinst], 1.0) / K"),
    "bf16_rounds_ties_up": ("u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000", "u = (u + 0x8000) & 0xFFFF0000"),
    "degree_feature_scale": ("fv[:, 5] = np.log1p(degc) / 4.0", "fv[:, 5] = np.log1p(degc) / 2.0"),
    "omega_weight_missing_in_gradient": ("dlw = 2.0 * omega_weight * ew / K", "dlw = 2.0 * ew / K"),
}


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_pins_catch_mutant(name):
    """A plausible mistake planted in a copy of the oracle fails at least one pin."""
    import importlib.util
    import types
    old, new = MUTANTS[name]
    path = importlib.util.find_spec("oracle.gnn_oracle").origin
    src = open(path).read()
    assert src.count(old) == 1, name
    mod = types.ModuleType("gnn_oracle_mutant")
    exec(compile(src.replace(old, new), path + ":" + name, "exec"), mod.__dict__)
    failed = []
    for pin in PINS:
        try:
            pin(go=mod)
        except Exception:   # an assertion or a shape error both count as caught
            failed.append(pin.__name__)
    assert failed, f"mutant {name} passed every pin"
