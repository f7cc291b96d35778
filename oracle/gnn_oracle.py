"""FP64 oracle of the learned warm start: a bipartite variable-constraint message-passing network.

TEST INFRASTRUCTURE ONLY (used by the tests, never by the GPU library). It shares no code with the
HIP kernels; the parameter layout and the feature definitions are an interface both sides implement
independently.

The warm-start model is not in the paper (it is an extension on top of the PDLP solve of the
initial LP relaxation, section 2). Its definition here:

  features (internal numbering, scaled problem; slog(v) = sign(v) log(1 + |v|)):
    variable j:   [slog c_j, [l_j finite], [u_j finite], slog l_j or 0, slog u_j or 0,
                   log(1 + deg_j) / 4, 1, 0]
    constraint i: [slog b_i, [sense L], [sense G], [sense E], log(1 + deg_i) / 4, 1, 0, 0]
  embedding:  hv = relu(fv Wv_in + bv_in),  hc = relu(fc Wc_in + bc_in)             (8 -> 64)
  3 layers:   mc = A hv ; hc = relu(hc W1 + mc W2 + b1)
              mv = A' hc ; hv = relu(hv W3 + mv W4 + b3)                         (64 -> 64)
  heads:      xhat = hv wx + bx ; yhat = hc wy + by ;
              log omega_q = mean_q(hv) wov + mean_q(hc) woc + bo     (per instance q)
  loss:       mean over instances of  mean_j (xhat - x*)^2 + mean_i (yhat - y*)^2
                                       + w_omega (log omega - log omega*)^2     (w_omega >= 0)

The GPU runs the dense layers on BF16 matrix cores with FP32 accumulation: both operands of every
dense product (activations and weights, forward and backward) are rounded to BF16 (round to nearest
even), nothing else is. With emulate_bf16=True the oracle applies the same roundings and
accumulates in FP64; with emulate_bf16=False it is the exact FP64 network (used for the
finite-difference pins).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

H = 64
F = 8
LAYERS = 3


def param_shapes():
    """Order and shapes of the flat parameter vector."""
    s = [("Wv_in", (F, H)), ("bv_in", (H,)), ("Wc_in", (F, H)), ("bc_in", (H,))]
    for l in range(LAYERS):
        s += [(f"W1_{l}", (H, H)), (f"W2_{l}", (H, H)), (f"b1_{l}", (H,)),
              (f"W3_{l}", (H, H)), (f"W4_{l}", (H, H)), (f"b3_{l}", (H,))]
    s += [("wx", (H,)), ("bx", (1,)), ("wy", (H,)), ("by", (1,)), ("wov", (H,)), ("woc", (H,)), ("bo", (1,))]
    return s


def num_params() -> int:
    return int(sum(np.prod(sh) for _, sh in param_shapes()))


def unpack(flat):
    out, o = {}, 0
    for name, sh in param_shapes():
        k = int(np.prod(sh))
        out[name] = np.asarray(flat[o:o + k], dtype=np.float64).reshape(sh)
        o += k
    return out


def pack(d):
    return np.concatenate([np.asarray(d[name], np.float64).ravel() for name, _ in param_shapes()])


def bf16(a):
    """Round to bfloat16 (nearest, ties to even) from the IEEE binary32 encoding."""
    x = np.asarray(a, dtype=np.float32)
    u = x.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def slog(v):
    return np.sign(v) * np.log1p(np.abs(v))


class Graph:
    """The scaled problem in internal numbering, as the GPU holds it (values in FP32)."""

    def __init__(self, row_ptr, col, val, c, b, l, u, sense, row0, col0):
        self.m = len(row_ptr) - 1
        self.n = len(c)
        self.A = sp.csr_matrix((np.asarray(val, np.float32).astype(np.float64), col, row_ptr),
                               shape=(self.m, self.n))
        self.AT = self.A.T.tocsr()
        self.c, self.b = np.asarray(c, np.float64), np.asarray(b, np.float64)
        self.l, self.u = np.asarray(l, np.float64), np.asarray(u, np.float64)
        self.sense = np.asarray(sense, np.uint8)
        self.row0, self.col0 = np.asarray(row0), np.asarray(col0)
        self.K = len(row0) - 1
        self.rinst = np.repeat(np.arange(self.K), np.diff(self.row0))
        self.cinst = np.repeat(np.arange(self.K), np.diff(self.col0))


def features(G: Graph):
    degc = np.diff(G.AT.indptr).astype(np.float64)
    degr = np.diff(G.A.indptr).astype(np.float64)
    lf = np.isfinite(G.l)
    uf = np.isfinite(G.u)
    fv = np.zeros((G.n, F))
    fv[:, 0] = slog(G.c)
    fv[:, 1] = lf
    fv[:, 2] = uf
    fv[:, 3] = np.where(lf, slog(np.where(lf, G.l, 0.0)), 0.0)
    fv[:, 4] = np.where(uf, slog(np.where(uf, G.u, 0.0)), 0.0)
    fv[:, 5] = np.log1p(degc) / 4.0
    fv[:, 6] = 1.0
    fc = np.zeros((G.m, F))
    fc[:, 0] = slog(G.b)
    fc[:, 1] = G.sense == ord("L")
    fc[:, 2] = G.sense == ord("G")
    fc[:, 3] = G.sense == ord("E")
    fc[:, 4] = np.log1p(degr) / 4.0
    fc[:, 5] = 1.0
    # the GPU computes features in FP32
    return fv.astype(np.float32).astype(np.float64), fc.astype(np.float32).astype(np.float64)


def _mm(x, W, emulate):
    return (bf16(x) @ bf16(W)) if emulate else x @ W


def _seg_mean(h, inst, K):
    cnt = np.bincount(inst, minlength=K).astype(np.float64)
    s = np.zeros((K, h.shape[1]))
    np.add.at(s, inst, h)
    return s / np.maximum(cnt, 1.0)[:, None], cnt


def forward(flat, G: Graph, emulate_bf16=True):
    P = unpack(flat)
    e = emulate_bf16
    fv, fc = features(G)
    cache = {"fv": fv, "fc": fc}
    hv = np.maximum(_mm(fv, P["Wv_in"], e) + P["bv_in"], 0.0)
    hc = np.maximum(_mm(fc, P["Wc_in"], e) + P["bc_in"], 0.0)
    cache["hv0"], cache["hc0"] = hv, hc
    for l in range(LAYERS):
        mc = G.A @ hv
        hc_new = np.maximum(_mm(hc, P[f"W1_{l}"], e) + _mm(mc, P[f"W2_{l}"], e) + P[f"b1_{l}"], 0.0)
        mv = G.AT @ hc_new
        hv_new = np.maximum(_mm(hv, P[f"W3_{l}"], e) + _mm(mv, P[f"W4_{l}"], e) + P[f"b3_{l}"], 0.0)
        cache[f"mc{l}"], cache[f"mv{l}"] = mc, mv
        hv, hc = hv_new, hc_new
        cache[f"hv{l + 1}"], cache[f"hc{l + 1}"] = hv, hc
    xhat = hv @ P["wx"] + P["bx"][0]
    yhat = hc @ P["wy"] + P["by"][0]
    pv, _ = _seg_mean(hv, G.cinst, G.K)
    pc, _ = _seg_mean(hc, G.rinst, G.K)
    logw = pv @ P["wov"] + pc @ P["woc"] + P["bo"][0]
    cache.update(pv=pv, pc=pc)
    return xhat, yhat, logw, cache


def loss_and_grad(flat, G: Graph, xs, ys, logws, emulate_bf16=True, omega_weight=1.0):
    """Loss and its gradient (flat, same layout as the parameters)."""
    P = unpack(flat)
    e = emulate_bf16
    xhat, yhat, logw, C = forward(flat, G, e)
    K = G.K
    nq = np.diff(G.col0).astype(np.float64)
    mq = np.diff(G.row0).astype(np.float64)
    ex, ey, ew = xhat - xs, yhat - ys, logw - logws
    L = 0.0
    for q in range(K):
        a, b_ = G.col0[q], G.col0[q + 1]
        c0, c1 = G.row0[q], G.row0[q + 1]
        L += ((np.mean(ex[a:b_] ** 2) if b_ > a else 0.0) + (np.mean(ey[c0:c1] ** 2) if c1 > c0 else 0.0)
              + omega_weight * ew[q] ** 2)
    L /= K
    dxh = 2.0 * ex / np.maximum(nq[G.cinst], 1.0) / K
    dyh = 2.0 * ey / np.maximum(mq[G.rinst], 1.0) / K
    dlw = 2.0 * omega_weight * ew / K
    g = {name: np.zeros(sh) for name, sh in param_shapes()}
    hv, hc = C[f"hv{LAYERS}"], C[f"hc{LAYERS}"]
    g["wx"] = hv.T @ dxh
    g["bx"][0] = dxh.sum()
    g["wy"] = hc.T @ dyh
    g["by"][0] = dyh.sum()
    g["wov"] = C["pv"].T @ dlw
    g["woc"] = C["pc"].T @ dlw
    g["bo"][0] = dlw.sum()
    dhv = np.outer(dxh, P["wx"]) + (dlw / np.maximum(nq, 1.0))[G.cinst][:, None] * P["wov"][None, :]
    dhc = np.outer(dyh, P["wy"]) + (dlw / np.maximum(mq, 1.0))[G.rinst][:, None] * P["woc"][None, :]

    def mmT(dpre, W):  # gradient w.r.t. the input of x W
        return (bf16(dpre) @ bf16(W).T) if e else dpre @ W.T

    def wgrad(x, dpre):
        return (bf16(x).T @ bf16(dpre)) if e else x.T @ dpre

    for l in reversed(range(LAYERS)):
        hv_l, hc_l = C[f"hv{l + 1}"], C[f"hc{l + 1}"]
        hv_p, hc_p = C[f"hv{l}"], C[f"hc{l}"]
        mv, mc = C[f"mv{l}"], C[f"mc{l}"]
        dpv = dhv * (hv_l > 0)
        g[f"W3_{l}"] = wgrad(hv_p, dpv)
        g[f"W4_{l}"] = wgrad(mv, dpv)
        g[f"b3_{l}"] = dpv.sum(axis=0)
        dhv_prev = mmT(dpv, P[f"W3_{l}"])
        dmv = mmT(dpv, P[f"W4_{l}"])
        dhc = dhc + G.A @ dmv
        dpc = dhc * (hc_l > 0)
        g[f"W1_{l}"] = wgrad(hc_p, dpc)
        g[f"W2_{l}"] = wgrad(mc, dpc)
        g[f"b1_{l}"] = dpc.sum(axis=0)
        dhc_prev = mmT(dpc, P[f"W1_{l}"])
        dmc = mmT(dpc, P[f"W2_{l}"])
        dhv_prev = dhv_prev + G.AT @ dmc
        dhv, dhc = dhv_prev, dhc_prev
    dpv = dhv * (C["hv0"] > 0)
    dpc = dhc * (C["hc0"] > 0)
    g["Wv_in"] = wgrad(C["fv"], dpv)
    g["bv_in"] = dpv.sum(axis=0)
    g["Wc_in"] = wgrad(C["fc"], dpc)
    g["bc_in"] = dpc.sum(axis=0)
    return L, pack(g)


def init_params(seed: int):
    """Glorot-uniform weights, zero biases (the GPU library draws its own; this is for tests)."""
    rng = np.random.default_rng(seed)
    d = {}
    for name, sh in param_shapes():
        if len(sh) == 2:
            lim = np.sqrt(6.0 / (sh[0] + sh[1]))
            d[name] = rng.uniform(-lim, lim, size=sh)
        elif name in ("wx", "wy", "wov", "woc"):
            lim = np.sqrt(6.0 / (H + 1))
            d[name] = rng.uniform(-lim, lim, size=sh)
        else:
            d[name] = np.zeros(sh)
    return pack(d)
