"""FP64 CPU oracle for the PDLP solve (test infrastructure).

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the benchmark's CPU-baseline leg use
this package; the GPU library never does. The arithmetic lives in ``pdhg_oracle.c`` (plain C, FP64),
which shares no code with the GPU path; this module only compiles it and marshals numpy arrays.

Functions and the passages they follow (the paper names PDLP but does not define it, so the steps
follow the published PDLP method; every constant is a reading):
  solve     -- restarted, diagonally preconditioned PDHG to a relative KKT tolerance (eq. (1); the
               low-accuracy regime of section 4, tolerances 1e-4 / 1e-6)
  kkt       -- relative primal / dual / gap errors of a point on the unscaled LP (termination test)
  scale     -- Ruiz inf-norm passes then one Pock-Chambolle alpha = 1 pass
  pdhg_step -- one PDHG step on an unscaled LP
  step_rule, restart_rule, primal_weight, kkt_weighted, initial_weight, initial_step -- the scalar
               rules of the method (adaptive step, restart test, primal weight update, weighted KKT
               error, start values), exactly the functions the solve calls
  spmv, transpose -- plain CSR product and counting-sort transpose
  propagate -- linear-constraint bound propagation in Jacobi rounds (prop_oracle.c; the paper uses
               the framework's linear-constraint propagator without defining it: a reading)
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(_HERE, "pdhg_oracle.c")
LIB = os.path.join(_HERE, "liboracle.so")

OPTIMAL, ITER_LIMIT, NUMERICAL = 1, 2, 3


def build(openmp: bool = True, src: str = SRC, out: str = LIB) -> str:
    cmd = ["gcc", "-O3", "-fPIC", "-shared", "-std=c99", src, "-o", out, "-lm"]
    if openmp:
        cmd.insert(1, "-fopenmp")
    subprocess.run(cmd, check=True)
    return out


class _LP(C.Structure):
    _fields_ = [("m", C.c_int32), ("n", C.c_int32),
                ("row_ptr", C.c_void_p), ("col", C.c_void_p), ("val", C.c_void_p),
                ("c", C.c_void_p), ("b", C.c_void_p), ("sense", C.c_void_p),
                ("l", C.c_void_p), ("u", C.c_void_p)]


class _Opts(C.Structure):
    _fields_ = [("tol", C.c_double), ("iter_limit", C.c_int64), ("ruiz_iters", C.c_int32),
                ("pock_chambolle", C.c_int32), ("eval_every", C.c_int32), ("trace_len", C.c_int32),
                ("x0", C.c_void_p), ("y0", C.c_void_p), ("omega0", C.c_double),
                ("trace_x", C.c_void_p), ("trace_y", C.c_void_p), ("trace_eta", C.c_void_p),
                ("trace_omega", C.c_void_p), ("trace_flags", C.c_void_p), ("trace_margin", C.c_void_p),
                ("trace_cond", C.c_void_p), ("sum_order", C.c_int32), ("pad_", C.c_int32)]


class _Res(C.Structure):
    _fields_ = [("status", C.c_int32), ("restarts", C.c_int32), ("iterations", C.c_int64),
                ("rel_p", C.c_double), ("rel_d", C.c_double), ("rel_gap", C.c_double),
                ("pobj", C.c_double), ("dobj", C.c_double), ("omega", C.c_double),
                ("eta", C.c_double), ("which", C.c_int32), ("pad", C.c_int32),
                ("omega_init", C.c_double), ("eta_init", C.c_double)]


_lib_cache: dict = {}


def load(path: str = LIB):
    if path in _lib_cache:
        return _lib_cache[path]
    if path == LIB and (not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC)):
        build()
    lib = C.CDLL(path)
    for name in ("orc_solve", "orc_kkt", "orc_scale", "orc_pdhg_step", "orc_num_threads", "orc_step_rule",
                 "orc_restart_rule"):
        getattr(lib, name).restype = C.c_int
    for name in ("orc_primal_weight", "orc_kkt_weighted", "orc_initial_weight", "orc_initial_step"):
        getattr(lib, name).restype = C.c_double
    lib.orc_spmv.restype = None
    lib.orc_transpose.restype = None
    _lib_cache[path] = lib
    return lib


def _p(a):
    return a.ctypes.data_as(C.c_void_p) if a is not None else None


def _arrays(lp):
    arrs = dict(row_ptr=np.ascontiguousarray(lp.row_ptr, np.int32),
                col=np.ascontiguousarray(lp.col, np.int32),
                val=np.ascontiguousarray(lp.val, np.float64),
                c=np.ascontiguousarray(lp.c, np.float64), b=np.ascontiguousarray(lp.b, np.float64),
                sense=np.ascontiguousarray(lp.sense, np.uint8),
                l=np.ascontiguousarray(lp.l, np.float64), u=np.ascontiguousarray(lp.u, np.float64))
    s = _LP(lp.m, lp.n, *[_p(arrs[k]) for k in ("row_ptr", "col", "val", "c", "b", "sense", "l", "u")])
    return s, arrs


@dataclass
class Result:
    status: int
    iterations: int
    restarts: int
    rel_p: float
    rel_d: float
    rel_gap: float
    pobj: float
    dobj: float
    omega: float
    eta: float
    which: int
    x: np.ndarray
    y: np.ndarray
    rc: np.ndarray
    trace: dict | None = None
    omega_init: float = 0.0
    eta_init: float = 0.0

    @property
    def rel_kkt(self) -> float:
        return max(self.rel_p, self.rel_d, self.rel_gap)


def solve(lp, tol: float = 1e-4, iter_limit: int = 1_000_000, ruiz_iters: int = 10,
          pock_chambolle: bool = True, eval_every: int = 64, x0=None, y0=None, omega0: float = 0.0,
          trace_len: int = 0, sum_order: int = 0, lib_path: str = LIB) -> Result:
    """sum_order 1 takes every sum of the method in reverse index order, 2 the even indices first
    and then the odd ones (different, equally valid roundings of the same arithmetic)."""
    lib = load(lib_path)
    s, keep = _arrays(lp)
    x = np.zeros(lp.n)
    y = np.zeros(lp.m)
    rc = np.zeros(lp.n)
    x0a = None if x0 is None else np.ascontiguousarray(x0, np.float64)
    y0a = None if y0 is None else np.ascontiguousarray(y0, np.float64)
    tr = None
    if trace_len > 0:
        tr = dict(x=np.zeros((trace_len, lp.n)), y=np.zeros((trace_len, lp.m)),
                  eta=np.zeros(trace_len), omega=np.zeros(trace_len),
                  flags=np.zeros(trace_len, np.int32), margin=np.full(trace_len, np.inf),
                  cond=np.ones(trace_len))
    o = _Opts(tol, iter_limit, ruiz_iters, 1 if pock_chambolle else 0, eval_every, trace_len,
              _p(x0a), _p(y0a), omega0,
              *([_p(tr[k]) for k in ("x", "y", "eta", "omega", "flags", "margin", "cond")] if tr else [None] * 7),
              int(sum_order), 0)
    r = _Res()
    rc_ = lib.orc_solve(C.byref(s), C.byref(o), _p(x), _p(y), _p(rc), C.byref(r))
    if rc_ != 0:
        raise MemoryError("oracle solve failed to allocate")
    return Result(r.status, r.iterations, r.restarts, r.rel_p, r.rel_d, r.rel_gap, r.pobj, r.dobj,
                  r.omega, r.eta, r.which, x, y, rc, tr, r.omega_init, r.eta_init)


def step_rule(omega, dx2, dy2, inter, eta, k, lib_path: str = LIB):
    """The adaptive step-size rule after attempt k: (accepted, eta_bar, eta_new)."""
    lib = load(lib_path)
    eb, en = C.c_double(), C.c_double()
    acc = lib.orc_step_rule(C.c_double(omega), C.c_double(dx2), C.c_double(dy2), C.c_double(inter),
                            C.c_double(eta), C.c_int64(k), C.byref(eb), C.byref(en))
    return bool(acc), eb.value, en.value


def restart_rule(kkt_cur, kkt_avg, kkt_anchor, kkt_prev, t_since, k, lib_path: str = LIB):
    """The restart decision at an evaluation: (restart, use_average, candidate KKT)."""
    lib = load(lib_path)
    ua, kc = C.c_int32(), C.c_double()
    r = lib.orc_restart_rule(C.c_double(kkt_cur), C.c_double(kkt_avg), C.c_double(kkt_anchor),
                             C.c_double(kkt_prev), C.c_int64(t_since), C.c_int64(k), C.byref(ua), C.byref(kc))
    return bool(r), bool(ua.value), kc.value


def primal_weight(omega, dx, dy, lib_path: str = LIB) -> float:
    """The primal weight after a restart whose point lies dx, dy from the anchor."""
    return float(load(lib_path).orc_primal_weight(C.c_double(omega), C.c_double(dx), C.c_double(dy)))


def kkt_weighted(omega, rp2, rd2, gap, lib_path: str = LIB) -> float:
    return float(load(lib_path).orc_kkt_weighted(C.c_double(omega), C.c_double(rp2), C.c_double(rd2),
                                                 C.c_double(gap)))


def initial_weight(omega0, norm_c_scaled, norm_b_scaled, lib_path: str = LIB) -> float:
    return float(load(lib_path).orc_initial_weight(C.c_double(omega0), C.c_double(norm_c_scaled),
                                                   C.c_double(norm_b_scaled)))


def initial_step(scaled_val, lib_path: str = LIB) -> float:
    v = np.ascontiguousarray(scaled_val, np.float64)
    return float(load(lib_path).orc_initial_step(_p(v), C.c_int64(v.size)))


def kkt(lp, x, y, lib_path: str = LIB) -> dict:
    lib = load(lib_path)
    s, keep = _arrays(lp)
    xa = np.ascontiguousarray(x, np.float64)
    ya = np.ascontiguousarray(y, np.float64)
    out = np.zeros(7)
    lib.orc_kkt(C.byref(s), _p(xa), _p(ya), _p(out))
    return dict(rel_p=out[0], rel_d=out[1], rel_gap=out[2], pobj=out[3], dobj=out[4],
                norm_rp=out[5], norm_rd=out[6], rel_kkt=float(max(out[0], out[1], out[2])))


def scale(lp, ruiz_iters: int = 10, pock_chambolle: bool = True, lib_path: str = LIB):
    lib = load(lib_path)
    rp = np.ascontiguousarray(lp.row_ptr, np.int32)
    ci = np.ascontiguousarray(lp.col, np.int32)
    v = np.ascontiguousarray(lp.val, np.float64)
    Dr = np.zeros(lp.m)
    Dc = np.zeros(lp.n)
    sv = np.zeros(max(v.size, 1))
    lib.orc_scale(C.c_int32(lp.m), C.c_int32(lp.n), _p(rp), _p(ci), _p(v), C.c_int32(ruiz_iters),
                  C.c_int32(1 if pock_chambolle else 0), _p(Dr), _p(Dc), _p(sv))
    return Dr, Dc, sv[: v.size]


def pdhg_step(lp, x, y, tau: float, sigma: float, lib_path: str = LIB):
    lib = load(lib_path)
    s, keep = _arrays(lp)
    xa = np.ascontiguousarray(x, np.float64)
    ya = np.ascontiguousarray(y, np.float64)
    xn = np.zeros(lp.n)
    yn = np.zeros(lp.m)
    lib.orc_pdhg_step(C.byref(s), _p(xa), _p(ya), C.c_double(tau), C.c_double(sigma), _p(xn), _p(yn))
    return xn, yn


def spmv(row_ptr, col, val, x, lib_path: str = LIB):
    lib = load(lib_path)
    rp = np.ascontiguousarray(row_ptr, np.int32)
    ci = np.ascontiguousarray(col, np.int32)
    v = np.ascontiguousarray(val, np.float64)
    xa = np.ascontiguousarray(x, np.float64)
    m = rp.size - 1
    y = np.zeros(m)
    lib.orc_spmv(C.c_int32(m), _p(rp), _p(ci), _p(v), _p(xa), _p(y))
    return y


def transpose(m: int, n: int, row_ptr, col, val, lib_path: str = LIB):
    lib = load(lib_path)
    rp = np.ascontiguousarray(row_ptr, np.int32)
    ci = np.ascontiguousarray(col, np.int32)
    v = np.ascontiguousarray(val, np.float64)
    nnz = int(rp[-1])
    trp = np.zeros(n + 1, np.int32)
    tci = np.zeros(max(nnz, 1), np.int32)
    tv = np.zeros(max(nnz, 1))
    lib.orc_transpose(C.c_int32(m), C.c_int32(n), _p(rp), _p(ci), _p(v), _p(trp), _p(tci), _p(tv))
    return trp, tci[:nnz], tv[:nnz]


def num_threads(lib_path: str = LIB) -> int:
    return int(load(lib_path).orc_num_threads())


# ---- linear-constraint propagation (prop_oracle.c, a library of its own) ----
PROP_SRC = os.path.join(_HERE, "prop_oracle.c")
PROP_LIB = os.path.join(_HERE, "liboracle_prop.so")
PROP_FIXPOINT, PROP_INFEASIBLE, PROP_ROUND_LIMIT = 0, 1, 2


def build_prop(src: str = PROP_SRC, out: str = PROP_LIB) -> str:
    subprocess.run(["gcc", "-O2", "-fPIC", "-shared", "-std=c99", "-ffp-contract=off", src, "-o", out, "-lm"],
                   check=True)
    return out


def load_prop(path: str = PROP_LIB):
    if path in _lib_cache:
        return _lib_cache[path]
    if path == PROP_LIB and (not os.path.exists(PROP_LIB) or os.path.getmtime(PROP_LIB) < os.path.getmtime(PROP_SRC)):
        build_prop()
    lib = C.CDLL(path)
    lib.orc_propagate.restype = C.c_int
    _lib_cache[path] = lib
    return lib


def propagate(lp, var_type, l, u, max_rounds: int = 100, lib_path: str = PROP_LIB):
    """Bounds after linear-constraint propagation in Jacobi rounds (prop_oracle.c states the rule).
    Returns (l, u, status, rounds)."""
    lib = load_prop(lib_path)
    rp = np.ascontiguousarray(lp.row_ptr, np.int32)
    ci = np.ascontiguousarray(lp.col, np.int32)
    v = np.ascontiguousarray(lp.val, np.float64)
    b = np.ascontiguousarray(lp.b, np.float64)
    sn = np.ascontiguousarray(lp.sense, np.uint8)
    vt = np.ascontiguousarray(var_type, np.uint8)
    lo = np.array(l, np.float64, copy=True)
    hi = np.array(u, np.float64, copy=True)
    rounds = C.c_int32()
    st = lib.orc_propagate(C.c_int32(lp.m), C.c_int32(lp.n), _p(rp), _p(ci), _p(v), _p(b), _p(sn), _p(vt), _p(lo),
                           _p(hi), C.c_int32(max_rounds), C.byref(rounds))
    if st < 0:
        raise MemoryError("oracle propagation failed to allocate")
    return lo, hi, int(st), int(rounds.value)
