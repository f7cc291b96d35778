"""Thin Python binding of libpdlp (ctypes). Argument marshalling only: every step of the solve runs
in the library's HIP kernels.

The functions keep the C names (pdlp_create, pdlp_solve, pdlp_get, ...). `Problem` wraps a handle
for convenience. PyTorch supplies streams and, optionally, device memory: tensors on the GPU may be
passed directly (their data pointers are handed over with device_ptrs set).
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libpdlp.so")

FP32, FP64 = 0, 1
STATUS = {0: "none", 1: "optimal", 2: "iteration_limit", 3: "numerical"}
OPTIMAL, ITER_LIMIT, NUMERICAL = 1, 2, 3
VAR_CONTINUOUS, VAR_BINARY, VAR_INTEGER = 0, 1, 2
ORDER_NONE, ORDER_FRAC, ORDER_REDCOST, ORDER_DUAL, ORDER_TYPE = 0, 1, 2, 3, 4
PROP_FIXPOINT, PROP_INFEASIBLE, PROP_ROUND_LIMIT = 0, 1, 2
ERR = {-1: "PDLP_ERR_ARG", -2: "PDLP_ERR_CSR", -3: "PDLP_ERR_OOM", -4: "PDLP_ERR_HIP", -5: "PDLP_ERR_STATE"}


class PDLPError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{ERR.get(code, code)}: {msg}")
        self.code = code


class Options(C.Structure):
    _fields_ = [("precision", C.c_int32), ("eval_every", C.c_int32), ("ruiz_iters", C.c_int32),
                ("pock_chambolle", C.c_int32), ("use_graphs", C.c_int32), ("device_ptrs", C.c_int32),
                ("tile_nnz", C.c_int32), ("verbose", C.c_int32), ("device_mem_limit", C.c_int64),
                ("stream", C.c_void_p), ("warm_fallback", C.c_int32), ("kernel_timing", C.c_int32),
                ("work_blocks", C.c_int32), ("single_avg_updates", C.c_int32), ("panel_rows", C.c_int32),
                ("col_blocks", C.c_int32), ("reserved", C.c_int32 * 2)]


class Result(C.Structure):
    _fields_ = [("status", C.c_int32), ("restarts", C.c_int32), ("iterations", C.c_int64),
                ("rel_primal", C.c_double), ("rel_dual", C.c_double), ("rel_gap", C.c_double),
                ("primal_obj", C.c_double), ("dual_obj", C.c_double), ("omega", C.c_double),
                ("eta", C.c_double), ("solve_seconds", C.c_double), ("used_average", C.c_int32),
                ("warm_started", C.c_int32), ("fallback_used", C.c_int32), ("final_checks", C.c_int32)]

    def as_dict(self) -> dict:
        d = {k: getattr(self, k) for k, _ in self._fields_}
        d["rel_kkt"] = max(self.rel_primal, self.rel_dual, self.rel_gap)
        d["status_name"] = STATUS.get(self.status, str(self.status))
        return d


class ProblemDesc(C.Structure):
    _fields_ = [("m", C.c_int32), ("n", C.c_int32), ("nnz", C.c_int64), ("row_ptr", C.c_void_p),
                ("col_idx", C.c_void_p), ("val", C.c_void_p), ("c", C.c_void_p), ("b", C.c_void_p),
                ("sense", C.c_void_p), ("l", C.c_void_p), ("u", C.c_void_p)]


EXPORTS = ["pdlp_options_default", "pdlp_create", "pdlp_solve", "pdlp_get", "pdlp_spmv",
           "pdlp_get_scaling", "pdlp_get_internal", "pdlp_get_schedule", "pdlp_kernel_stats", "pdlp_device_bytes", "pdlp_destroy",
           "pdlp_error_string", "pdlp_last_error", "pdlp_batch_create", "pdlp_batch_solve",
           "pdlp_batch_get", "pdlp_batch_get_schedule", "pdlp_batch_destroy", "pdlp_update_bounds",
           "pdlp_batch_update_bounds", "pdlp_variable_strategy", "pdlp_variable_strategy_noalloc",
           "pdlp_lp_fixing", "pdlp_prop_create", "pdlp_propagate", "pdlp_prop_destroy", "pdlp_branching",
           "pdlp_set_snapshots", "pdlp_get_snapshots", "pdlp_batch_set_snapshots", "pdlp_batch_get_snapshots"]

_lib = None


def load(path: str = LIB_PATH):
    """Load libpdlp.so. Raises if it has not been built: there is no fallback path."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"libpdlp.so not found at {path}; build it with "
                           "`python -m paper_2503_10344_amd.build` (hipcc, gfx950)")
    try:  # share torch's HIP runtime when torch is present (one runtime per process)
        import torch  # noqa: F401
    except Exception:
        pass
    lib = C.CDLL(path)
    vp, i32, i64, dp = C.c_void_p, C.c_int32, C.c_int64, C.c_double
    lib.pdlp_options_default.argtypes = [C.POINTER(Options)]
    lib.pdlp_options_default.restype = None
    lib.pdlp_create.argtypes = [C.POINTER(vp), i32, i32, i64, vp, vp, vp, vp, vp, vp, vp, vp, C.POINTER(Options)]
    lib.pdlp_create.restype = C.c_int
    lib.pdlp_solve.argtypes = [vp, dp, i64, vp, vp, dp]
    lib.pdlp_solve.restype = C.c_int
    lib.pdlp_get.argtypes = [vp, vp, vp, vp, C.POINTER(Result)]
    lib.pdlp_get.restype = C.c_int
    lib.pdlp_spmv.argtypes = [vp, i32, vp, vp]
    lib.pdlp_spmv.restype = C.c_int
    lib.pdlp_get_scaling.argtypes = [vp, vp, vp, vp]
    lib.pdlp_get_scaling.restype = C.c_int
    lib.pdlp_get_internal.argtypes = [vp, vp, vp, vp, vp, vp, vp, vp, vp]
    lib.pdlp_get_internal.restype = C.c_int
    lib.pdlp_get_schedule.argtypes = [vp, C.POINTER(i32), C.POINTER(i32), C.POINTER(i32)]
    lib.pdlp_get_schedule.restype = C.c_int
    lib.pdlp_batch_get_schedule.argtypes = [vp, C.POINTER(i32), C.POINTER(i32), C.POINTER(i32)]
    lib.pdlp_batch_get_schedule.restype = C.c_int
    lib.pdlp_update_bounds.argtypes = [vp, vp, vp]
    lib.pdlp_update_bounds.restype = C.c_int
    lib.pdlp_batch_update_bounds.argtypes = [vp, i32, vp, vp]
    lib.pdlp_batch_update_bounds.restype = C.c_int
    lib.pdlp_kernel_stats.argtypes = [vp, i32, C.POINTER(i64), C.POINTER(dp)]
    lib.pdlp_kernel_stats.restype = C.c_int
    lib.pdlp_device_bytes.argtypes = [vp]
    lib.pdlp_device_bytes.restype = i64
    lib.pdlp_destroy.argtypes = [vp]
    lib.pdlp_destroy.restype = None
    lib.pdlp_error_string.argtypes = [C.c_int]
    lib.pdlp_error_string.restype = C.c_char_p
    lib.pdlp_last_error.argtypes = []
    lib.pdlp_last_error.restype = C.c_char_p
    lib.pdlp_batch_create.argtypes = [C.POINTER(vp), i32, C.POINTER(ProblemDesc), C.POINTER(Options)]
    lib.pdlp_batch_create.restype = C.c_int
    lib.pdlp_batch_solve.argtypes = [vp, dp, i64, C.POINTER(vp), C.POINTER(vp), vp]
    lib.pdlp_batch_solve.restype = C.c_int
    lib.pdlp_batch_get.argtypes = [vp, i32, vp, vp, vp, C.POINTER(Result)]
    lib.pdlp_batch_get.restype = C.c_int
    lib.pdlp_batch_destroy.argtypes = [vp]
    lib.pdlp_batch_destroy.restype = None
    lib.pdlp_batch_get_scaling.argtypes = [vp, vp, vp, vp]
    lib.pdlp_batch_get_scaling.restype = C.c_int
    lib.pdlp_batch_get_internal.argtypes = [vp, vp, vp, vp, vp, vp, vp, vp, vp]
    lib.pdlp_batch_get_internal.restype = C.c_int
    # learned warm start
    lib.pdlp_gnn_num_params.argtypes = []
    lib.pdlp_gnn_num_params.restype = i64
    lib.pdlp_gnn_create.argtypes = [C.POINTER(vp), C.c_uint64]
    lib.pdlp_gnn_create.restype = C.c_int
    lib.pdlp_gnn_get_params.argtypes = [vp, vp]
    lib.pdlp_gnn_get_params.restype = C.c_int
    lib.pdlp_gnn_set_params.argtypes = [vp, vp]
    lib.pdlp_gnn_set_params.restype = C.c_int
    lib.pdlp_gnn_predict.argtypes = [vp, vp, vp, vp, vp]
    lib.pdlp_gnn_predict.restype = C.c_int
    lib.pdlp_gnn_predict_batch.argtypes = [vp, vp, vp, vp, vp]
    lib.pdlp_gnn_predict_batch.restype = C.c_int
    lib.pdlp_gnn_predict_raw.argtypes = [vp, vp, vp, vp, vp]
    lib.pdlp_gnn_predict_raw.restype = C.c_int
    lib.pdlp_gnn_gradients.argtypes = [vp, vp, vp, vp, vp, C.POINTER(dp), vp]
    lib.pdlp_gnn_gradients.restype = C.c_int
    lib.pdlp_gnn_train_step.argtypes = [vp, vp, vp, vp, vp, C.c_float, C.POINTER(dp)]
    lib.pdlp_gnn_train_step.restype = C.c_int
    lib.pdlp_gnn_set_omega_weight.argtypes = [vp, C.c_float]
    lib.pdlp_gnn_set_omega_weight.restype = C.c_int
    lib.pdlp_gnn_destroy.argtypes = [vp]
    lib.pdlp_gnn_destroy.restype = None
    # LP-based variable strategies and fixing
    lib.pdlp_variable_strategy.argtypes = [vp, i32, i32, vp, vp, vp, vp, vp, C.POINTER(i32)]
    lib.pdlp_variable_strategy.restype = C.c_int
    lib.pdlp_variable_strategy_noalloc.argtypes = [vp, i32, i32, vp, vp, vp, vp, vp, C.POINTER(i32)]
    lib.pdlp_variable_strategy_noalloc.restype = C.c_int
    lib.pdlp_lp_fixing.argtypes = [vp, vp, vp, vp, vp, vp, vp]
    lib.pdlp_lp_fixing.restype = C.c_int
    # linear-constraint propagation and branching
    lib.pdlp_prop_create.argtypes = [C.POINTER(vp), i32, i32, i64, vp, vp, vp, vp, vp, vp, C.POINTER(Options)]
    lib.pdlp_prop_create.restype = C.c_int
    lib.pdlp_propagate.argtypes = [vp, vp, vp, i32, C.POINTER(i32), C.POINTER(i32)]
    lib.pdlp_propagate.restype = C.c_int
    lib.pdlp_prop_destroy.argtypes = [vp]
    lib.pdlp_prop_destroy.restype = None
    lib.pdlp_branching.argtypes = [dp, dp, dp, dp, vp, vp, C.POINTER(i32)]
    lib.pdlp_branching.restype = C.c_int
    # reference snapshots
    lib.pdlp_set_snapshots.argtypes = [vp, i32, dp]
    lib.pdlp_set_snapshots.restype = C.c_int
    lib.pdlp_batch_set_snapshots.argtypes = [vp, i32, dp]
    lib.pdlp_batch_set_snapshots.restype = C.c_int
    lib.pdlp_get_snapshots.argtypes = [vp, i32, vp, vp, vp, vp, C.POINTER(i32)]
    lib.pdlp_get_snapshots.restype = C.c_int
    lib.pdlp_batch_get_snapshots.argtypes = [vp, i32, i32, vp, vp, vp, vp, C.POINTER(i32)]
    lib.pdlp_batch_get_snapshots.restype = C.c_int
    _lib = lib
    return lib


def _check(rc: int):
    if rc != 0:
        lib = load()
        raise PDLPError(rc, lib.pdlp_last_error().decode())


def _torch():
    import torch
    return torch


def _is_cuda(a):
    return getattr(a, "is_cuda", False)


def _vec(a, length, name):
    """Contiguous float64 copy of a vector the C side reads `length` entries of; a wrong length
    raises here instead of letting the library read past the end of the array."""
    v = np.ascontiguousarray(a, np.float64)
    if v.ndim != 1 or v.size != length:
        raise ValueError(f"{name} must have {length} entries, got shape {v.shape}")
    return v


def _dptr(a):
    """Device pointer of a contiguous GPU torch tensor."""
    if not (_is_cuda(a) and a.is_contiguous()):
        raise ValueError("expected a contiguous torch tensor on the GPU")
    return C.c_void_p(a.data_ptr())


def _ptr(a):
    """Pointer of a numpy array or a torch tensor (None stays None)."""
    if a is None:
        return None
    if hasattr(a, "data_ptr"):
        return C.c_void_p(a.data_ptr())
    return a.ctypes.data_as(C.c_void_p)


def options(precision="fp32", eval_every=64, ruiz_iters=10, pock_chambolle=True, use_graphs=True,
            device_ptrs=False, tile_nnz=0, verbose=0, device_mem_limit=0, stream=None,
            warm_fallback=2, kernel_timing=False, work_blocks=0, single_avg_updates=False,
            panel_rows=0, col_blocks=0) -> Options:
    o = Options()
    load().pdlp_options_default(C.byref(o))
    o.precision = FP64 if str(precision).lower() in ("fp64", "f64", "double", "1") else FP32
    o.eval_every = eval_every
    o.ruiz_iters = ruiz_iters
    o.pock_chambolle = 1 if pock_chambolle else 0
    o.use_graphs = 1 if use_graphs else 0
    o.device_ptrs = 1 if device_ptrs else 0
    o.tile_nnz = tile_nnz
    o.verbose = verbose
    o.device_mem_limit = device_mem_limit
    o.warm_fallback = int(warm_fallback)  # 0 keep, 1 cold start, 2 cold point keeping omega0
    o.kernel_timing = 1 if kernel_timing else 0
    o.work_blocks = work_blocks
    o.single_avg_updates = 1 if single_avg_updates else 0
    o.panel_rows = panel_rows
    o.col_blocks = col_blocks
    if stream is None:
        try:
            import torch
            if torch.cuda.is_available():
                stream = torch.cuda.current_stream().cuda_stream
        except Exception:
            stream = None
    o.stream = stream
    return o


# ---- functions with the C names ---------------------------------------------------------------
def pdlp_create(m, n, nnz, row_ptr, col_idx, val, c, b, sense, l, u, opt: Options | None = None):
    lib = load()
    h = C.c_void_p()
    _check(lib.pdlp_create(C.byref(h), m, n, nnz, _ptr(row_ptr), _ptr(col_idx), _ptr(val), _ptr(c),
                           _ptr(b), _ptr(sense), _ptr(l), _ptr(u), C.byref(opt) if opt else None))
    return h


def pdlp_solve(h, tol=1e-4, iter_limit=1_000_000, x0=None, y0=None, omega0=0.0):
    _check(load().pdlp_solve(h, tol, iter_limit, _ptr(x0), _ptr(y0), omega0))


def pdlp_get(h, x=None, y=None, red_cost=None) -> Result:
    r = Result()
    _check(load().pdlp_get(h, _ptr(x), _ptr(y), _ptr(red_cost), C.byref(r)))
    return r


def pdlp_spmv(h, trans, x, y):
    _check(load().pdlp_spmv(h, int(trans), _ptr(x), _ptr(y)))


def pdlp_destroy(h):
    load().pdlp_destroy(h)


# ---- convenience wrapper ----------------------------------------------------------------------
def _lp_arrays(lp):
    return dict(row_ptr=np.ascontiguousarray(lp.row_ptr, np.int32), col=np.ascontiguousarray(lp.col, np.int32),
                val=np.ascontiguousarray(lp.val, np.float64), c=np.ascontiguousarray(lp.c, np.float64),
                b=np.ascontiguousarray(lp.b, np.float64), sense=np.ascontiguousarray(lp.sense, np.uint8),
                l=np.ascontiguousarray(lp.l, np.float64), u=np.ascontiguousarray(lp.u, np.float64))


@dataclass
class Solution:
    x: np.ndarray
    y: np.ndarray
    rc: np.ndarray
    info: dict


@dataclass
class Snapshots:
    """Restart points of a solve kept as reference solutions, oldest first (original space)."""
    x: np.ndarray        # [count, n]
    y: np.ndarray        # [count, m]
    attempt: np.ndarray  # [count] attempt count at which each was taken
    rel_kkt: np.ndarray  # [count] relative KKT error as the solve measured it


def _get_snapshots(call, cap, n, m) -> Snapshots:
    """call(cap, x, y, attempt, rel, count) for one instance; host arrays."""
    x, y = np.zeros((cap, n)), np.zeros((cap, m))
    att, rel = np.zeros(cap, np.int64), np.zeros(cap)
    cnt = C.c_int32(0)
    _check(call(int(cap), _ptr(x), _ptr(y), _ptr(att), _ptr(rel), C.byref(cnt)))
    k = cnt.value
    return Snapshots(x[:k].copy(), y[:k].copy(), att[:k].copy(), rel[:k].copy())


class Problem:
    """A solver handle for one LP (generators.LP or any object with the same fields)."""

    def __init__(self, lp, precision="fp32", **opts):
        self.m, self.n = int(lp.m), int(lp.n)
        self.arr = _lp_arrays(lp)
        self.nnz = int(self.arr["row_ptr"][-1])
        self.opt = options(precision=precision, **opts)
        a = self.arr
        self.h = pdlp_create(self.m, self.n, self.nnz, a["row_ptr"], a["col"], a["val"], a["c"], a["b"],
                             a["sense"], a["l"], a["u"], self.opt)

    def solve(self, tol=1e-4, iter_limit=1_000_000, x0=None, y0=None, omega0=0.0) -> dict:
        x0a = None if x0 is None else _vec(x0, self.n, "x0")
        y0a = None if y0 is None else _vec(y0, self.m, "y0")
        pdlp_solve(self.h, tol, iter_limit, x0a, y0a, omega0)
        return pdlp_get(self.h).as_dict()

    def get(self) -> Solution:
        x, y, rc = np.zeros(self.n), np.zeros(self.m), np.zeros(self.n)
        r = pdlp_get(self.h, x, y, rc)
        return Solution(x, y, rc, r.as_dict())

    def spmv(self, x, trans=False, iteration=False) -> np.ndarray:
        """A x (A'x with trans). iteration=True: the product the way the PDHG iteration forms it (in
        FP32 handles that use them: long rows of A by column panels, A'x by column blocks)."""
        x = _vec(x, self.m if trans else self.n, "x")
        y = np.zeros(self.n if trans else self.m)
        pdlp_spmv(self.h, (3 if trans else 2) if iteration else (1 if trans else 0), x, y)
        return y

    def set_snapshots(self, k, rel_tol):
        """Keep the newest k restart points with relative KKT error <= rel_tol in later solves."""
        _check(load().pdlp_set_snapshots(self.h, int(k), float(rel_tol)))
        self.snap_k = int(k)

    def snapshots(self, cap=None) -> Snapshots:
        cap = getattr(self, "snap_k", 0) if cap is None else cap
        lib = load()
        return _get_snapshots(lambda *a: lib.pdlp_get_snapshots(self.h, *a), cap, self.n, self.m)

    def scaling(self):
        Dr, Dc, sv = np.zeros(self.m), np.zeros(self.n), np.zeros(self.nnz)
        _check(load().pdlp_get_scaling(self.h, _ptr(Dr), _ptr(Dc), _ptr(sv)))
        return dict(Dr=Dr, Dc=Dc, scaled_val=sv)

    def internal(self):
        m, n, z = self.m, self.n, self.nnz
        out = dict(row_ptr=np.zeros(m + 1, np.int32), col=np.zeros(z, np.int32), val=np.zeros(z),
                   t_row_ptr=np.zeros(n + 1, np.int32), t_col=np.zeros(z, np.int32), t_val=np.zeros(z),
                   row_perm=np.zeros(m, np.int32), col_perm=np.zeros(n, np.int32))
        _check(load().pdlp_get_internal(self.h, *[_ptr(out[k]) for k in ("row_ptr", "col", "val", "t_row_ptr",
                                                                          "t_col", "t_val", "row_perm", "col_perm")]))
        return out

    def schedule(self) -> dict:
        tn, ta, tt = C.c_int32(), C.c_int32(), C.c_int32()
        _check(load().pdlp_get_schedule(self.h, C.byref(tn), C.byref(ta), C.byref(tt)))
        return dict(tile_nnz=tn.value, tiles_a=ta.value, tiles_at=tt.value)

    def update_bounds(self, l, u):
        """New column bounds (after fixings) for the next solve; see pdlp_update_bounds."""
        lo, hi = _vec(l, self.n, "l"), _vec(u, self.n, "u")
        _check(load().pdlp_update_bounds(self.h, _ptr(lo), _ptr(hi)))

    def kernel_stats(self) -> dict:
        out = {}
        for k, name in ((0, "dual"), (1, "primal"), (2, "panel"), (3, "col_blocks"), (4, "row_blocks")):
            n, ms = C.c_int64(), C.c_double()
            _check(load().pdlp_kernel_stats(self.h, k, C.byref(n), C.byref(ms)))
            out[name] = dict(launches=n.value, total_ms=ms.value,
                             avg_ms=(ms.value / n.value) if n.value else float("nan"))
        return out

    def device_bytes(self) -> int:
        return int(load().pdlp_device_bytes(self.h))

    def variable_strategy(self, strategy, var_type, x=None, y=None, rc=None, tiebreak=ORDER_NONE):
        """Indices of the binary and integer variables in fixing order (see include/pdlp_fix.h).
        Inputs are numpy arrays, or contiguous torch tensors on the GPU (uint8 types, float64 values):
        then the result is a torch int32 tensor on the GPU and nothing crosses PCIe."""
        if _is_cuda(var_type):
            _torch().cuda.current_stream().synchronize()  # inputs written on torch's stream are complete
            order = _torch().empty(max(self.n, 1), dtype=_torch().int32, device=var_type.device)
            args = [_dptr(var_type)] + [None if a is None else _dptr(a) for a in (x, y, rc)] + [_dptr(order)]
        else:
            vt = np.ascontiguousarray(var_type, np.uint8)
            arrs = [None if a is None else np.ascontiguousarray(a, np.float64) for a in (x, y, rc)]
            order = np.zeros(max(self.n, 1), np.int32)
            args = [_ptr(vt)] + [None if a is None else _ptr(a) for a in arrs] + [_ptr(order)]
        cnt = C.c_int32()
        _check(load().pdlp_variable_strategy(self.h, int(strategy), int(tiebreak), *args, C.byref(cnt)))
        return order[:cnt.value].clone() if _is_cuda(order) else order[:cnt.value].copy()

    def variable_strategy_noalloc(self, strategy, var_type, order, x=None, y=None, rc=None, tiebreak=ORDER_NONE):
        """The same order computed without any device allocation (include/pdlp_fix.h): every argument
        is a contiguous torch tensor on the handle's GPU, `order` (int32, at least n entries) is the
        caller's output buffer. Returns the number of ordered variables."""
        _torch().cuda.current_stream().synchronize()  # inputs written on torch's stream are complete
        args = [_dptr(var_type)] + [None if a is None else _dptr(a) for a in (x, y, rc)] + [_dptr(order)]
        cnt = C.c_int32()
        _check(load().pdlp_variable_strategy_noalloc(self.h, int(strategy), int(tiebreak), *args, C.byref(cnt)))
        return cnt.value

    def lp_fixing(self, var_type, x, l, u, uniform):
        """Fixing value of every variable under LP-based fixing (continuous ones keep x); numpy
        arrays in and out, or GPU torch tensors in and out."""
        if _is_cuda(var_type):
            _torch().cuda.current_stream().synchronize()
            out = _torch().empty(self.n, dtype=_torch().float64, device=var_type.device)
            args = [_dptr(v) for v in (var_type, x, l, u, uniform, out)]
        else:
            a = [np.ascontiguousarray(v, np.float64) for v in (x, l, u, uniform)]
            vt = np.ascontiguousarray(var_type, np.uint8)
            out = np.zeros(self.n)
            args = [_ptr(vt)] + [_ptr(v) for v in a] + [_ptr(out)]
        _check(load().pdlp_lp_fixing(self.h, *args))
        return out

    def close(self):
        if getattr(self, "h", None):
            pdlp_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()


def pdlp_batch_create(descs, opt: Options | None = None):
    lib = load()
    h = C.c_void_p()
    arr = (ProblemDesc * len(descs))(*descs)
    _check(lib.pdlp_batch_create(C.byref(h), len(descs), arr, C.byref(opt) if opt else None))
    return h


def pdlp_batch_solve(h, tol=1e-4, iter_limit=1_000_000, x0s=None, y0s=None, omega0s=None):
    _check(load().pdlp_batch_solve(h, tol, iter_limit, x0s, y0s, omega0s))


def pdlp_batch_get(h, i, x=None, y=None, red_cost=None) -> Result:
    r = Result()
    _check(load().pdlp_batch_get(h, i, _ptr(x), _ptr(y), _ptr(red_cost), C.byref(r)))
    return r


def pdlp_batch_destroy(h):
    load().pdlp_batch_destroy(h)


class Batch:
    """A handle solving many LPs together (one launch per kernel covers every instance)."""

    def __init__(self, lps, precision="fp32", **opts):
        self.arrs = [_lp_arrays(lp) for lp in lps]
        self.dims = [(int(lp.m), int(lp.n)) for lp in lps]
        descs = []
        for (m, n), a in zip(self.dims, self.arrs):
            descs.append(ProblemDesc(m, n, int(a["row_ptr"][-1]), _ptr(a["row_ptr"]), _ptr(a["col"]),
                                     _ptr(a["val"]), _ptr(a["c"]), _ptr(a["b"]), _ptr(a["sense"]),
                                     _ptr(a["l"]), _ptr(a["u"])))
        self.opt = options(precision=precision, **opts)
        self.h = pdlp_batch_create(descs, self.opt)

    def __len__(self):
        return len(self.dims)

    def solve(self, tol=1e-4, iter_limit=1_000_000, x0s=None, y0s=None, omega0s=None):
        k = len(self.dims)
        keep = []

        def ptr_array(vs, side):
            if vs is None:
                return None
            if len(vs) != k:
                raise ValueError(f"one start vector (or None) per instance: {k} expected, got {len(vs)}")
            arr = (C.c_void_p * k)()
            for i, v in enumerate(vs):
                if v is not None:
                    a = _vec(v, self.dims[i][side], f"start vector of instance {i}")
                    keep.append(a)
                    arr[i] = a.ctypes.data
            return arr

        xa, ya = ptr_array(x0s, 1), ptr_array(y0s, 0)
        om = None
        if omega0s is not None:
            oa = _vec(omega0s, k, "omega0s")
            keep.append(oa)
            om = oa.ctypes.data_as(C.c_void_p)
        pdlp_batch_solve(self.h, tol, iter_limit, xa, ya, om)
        return [pdlp_batch_get(self.h, i).as_dict() for i in range(k)]

    def get(self, i) -> Solution:
        m, n = self.dims[i]
        x, y, rc = np.zeros(n), np.zeros(m), np.zeros(n)
        r = pdlp_batch_get(self.h, i, x, y, rc)
        return Solution(x, y, rc, r.as_dict())

    def set_snapshots(self, k, rel_tol):
        """Keep the newest k restart points with relative KKT error <= rel_tol per instance."""
        _check(load().pdlp_batch_set_snapshots(self.h, int(k), float(rel_tol)))
        self.snap_k = int(k)

    def snapshots(self, i, cap=None) -> Snapshots:
        m, n = self.dims[i]
        cap = getattr(self, "snap_k", 0) if cap is None else cap
        lib = load()
        return _get_snapshots(lambda *a: lib.pdlp_batch_get_snapshots(self.h, int(i), *a), cap, n, m)

    def update_bounds(self, i, l, u):
        """New column bounds of instance i for the next batched solve."""
        if 0 <= int(i) < len(self.dims):
            lo, hi = _vec(l, self.dims[int(i)][1], "l"), _vec(u, self.dims[int(i)][1], "u")
        else:  # the library rejects the index
            lo, hi = np.ascontiguousarray(l, np.float64), np.ascontiguousarray(u, np.float64)
        _check(load().pdlp_batch_update_bounds(self.h, int(i), _ptr(lo), _ptr(hi)))

    def schedule(self) -> dict:
        tn, ta, tt = C.c_int32(), C.c_int32(), C.c_int32()
        _check(load().pdlp_batch_get_schedule(self.h, C.byref(tn), C.byref(ta), C.byref(tt)))
        return dict(tile_nnz=tn.value, tiles_a=ta.value, tiles_at=tt.value)

    @property
    def m(self):
        return sum(d[0] for d in self.dims)

    @property
    def n(self):
        return sum(d[1] for d in self.dims)

    @property
    def nnz(self):
        return sum(int(a["row_ptr"][-1]) for a in self.arrs)

    def scaling(self):
        """Dr [sum m], Dc [sum n] and the scaled values, over the concatenated instances."""
        Dr, Dc, sv = np.zeros(self.m), np.zeros(self.n), np.zeros(self.nnz)
        _check(load().pdlp_batch_get_scaling(self.h, _ptr(Dr), _ptr(Dc), _ptr(sv)))
        return dict(Dr=Dr, Dc=Dc, scaled_val=sv)

    def internal(self):
        m, n, z = self.m, self.n, self.nnz
        out = dict(row_ptr=np.zeros(m + 1, np.int32), col=np.zeros(z, np.int32), val=np.zeros(z),
                   t_row_ptr=np.zeros(n + 1, np.int32), t_col=np.zeros(z, np.int32), t_val=np.zeros(z),
                   row_perm=np.zeros(m, np.int32), col_perm=np.zeros(n, np.int32))
        _check(load().pdlp_batch_get_internal(self.h, *[_ptr(out[k]) for k in (
            "row_ptr", "col", "val", "t_row_ptr", "t_col", "t_val", "row_perm", "col_perm")]))
        return out

    def close(self):
        if getattr(self, "h", None):
            pdlp_batch_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()


class WarmStartNet:
    """The learned warm start (a 3-round bipartite message-passing network, width 64).

    predict(handle) returns (x0, y0, omega0) in the original space for a Problem or a Batch (batch
    vectors concatenated in instance order); train_step / gradients take a Batch and its targets.
    All arithmetic runs in the HIP library.
    """

    def __init__(self, seed=0, params=None, omega_weight=1.0):
        lib = load()
        self.num_params = int(lib.pdlp_gnn_num_params())
        h = C.c_void_p()
        _check(lib.pdlp_gnn_create(C.byref(h), C.c_uint64(seed)))
        self.h = h
        if params is not None:
            self.set_params(params)
        if omega_weight != 1.0:
            self.set_omega_weight(omega_weight)

    def set_omega_weight(self, w):
        """Weight of the log-omega term of the training loss (default 1)."""
        _check(load().pdlp_gnn_set_omega_weight(self.h, C.c_float(w)))

    def params(self) -> np.ndarray:
        p = np.zeros(self.num_params, np.float32)
        _check(load().pdlp_gnn_get_params(self.h, _ptr(p)))
        return p

    def set_params(self, p):
        p = np.ascontiguousarray(p, np.float32)
        if p.size != self.num_params:
            raise ValueError(f"expected {self.num_params} parameters, got {p.size}")
        _check(load().pdlp_gnn_set_params(self.h, _ptr(p)))

    def predict(self, handle):
        lib = load()
        if isinstance(handle, Batch):
            x0, y0, om = np.zeros(handle.n), np.zeros(handle.m), np.zeros(len(handle))
            _check(lib.pdlp_gnn_predict_batch(self.h, handle.h, _ptr(x0), _ptr(y0), _ptr(om)))
            return x0, y0, om
        x0, y0, om = np.zeros(handle.n), np.zeros(handle.m), np.zeros(1)
        _check(lib.pdlp_gnn_predict(self.h, handle.h, _ptr(x0), _ptr(y0), _ptr(om)))
        return x0, y0, float(om[0])

    def predict_raw(self, batch):
        xh, yh, lw = np.zeros(batch.n, np.float32), np.zeros(batch.m, np.float32), np.zeros(len(batch), np.float32)
        _check(load().pdlp_gnn_predict_raw(self.h, batch.h, _ptr(xh), _ptr(yh), _ptr(lw)))
        return xh, yh, lw

    @staticmethod
    def _targets(batch, x_star, y_star, omega_star):
        xs = np.ascontiguousarray(x_star, np.float64)
        ys = np.ascontiguousarray(y_star, np.float64)
        om = np.ascontiguousarray(omega_star, np.float64)
        if xs.size != batch.n or ys.size != batch.m or om.size != len(batch):
            raise ValueError("target sizes do not match the batch")
        return xs, ys, om

    def gradients(self, batch, x_star, y_star, omega_star):
        xs, ys, om = self._targets(batch, x_star, y_star, omega_star)
        g = np.zeros(self.num_params, np.float32)
        loss = C.c_double()
        _check(load().pdlp_gnn_gradients(self.h, batch.h, _ptr(xs), _ptr(ys), _ptr(om), C.byref(loss), _ptr(g)))
        return loss.value, g

    def train_step(self, batch, x_star, y_star, omega_star, lr=1e-3) -> float:
        xs, ys, om = self._targets(batch, x_star, y_star, omega_star)
        loss = C.c_double()
        _check(load().pdlp_gnn_train_step(self.h, batch.h, _ptr(xs), _ptr(ys), _ptr(om), C.c_float(lr),
                                          C.byref(loss)))
        return loss.value

    def close(self):
        if getattr(self, "h", None):
            load().pdlp_gnn_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Propagator:
    """Linear-constraint propagation over the rows of an LP / MIP (see include/pdlp_prop.h)."""

    def __init__(self, lp, var_type, stream=None, device_mem_limit=0):
        self.n = int(lp.n)
        self.arr = _lp_arrays(lp)
        self.vt = np.ascontiguousarray(var_type, np.uint8)
        self.opt = options(stream=stream, device_mem_limit=device_mem_limit)
        a = self.arr
        h = C.c_void_p()
        _check(load().pdlp_prop_create(C.byref(h), int(lp.m), self.n, int(a["row_ptr"][-1]), _ptr(a["row_ptr"]),
                                       _ptr(a["col"]), _ptr(a["val"]), _ptr(a["b"]), _ptr(a["sense"]), _ptr(self.vt),
                                       C.byref(self.opt)))
        self.h = h

    def propagate(self, l, u, max_rounds=100):
        """Propagated copies of the bounds, the status (PROP_*) and the rounds run. numpy arrays, or
        GPU torch float64 tensors (propagated in place and returned)."""
        if _is_cuda(l):
            _torch().cuda.current_stream().synchronize()
            lo, hi, pl, pu = l, u, _dptr(l), _dptr(u)
        else:
            lo = np.array(l, np.float64, copy=True)
            hi = np.array(u, np.float64, copy=True)
            pl, pu = _ptr(lo), _ptr(hi)
        r, st = C.c_int32(), C.c_int32()
        _check(load().pdlp_propagate(self.h, pl, pu, int(max_rounds), C.byref(r), C.byref(st)))
        return lo, hi, st.value, r.value

    def close(self):
        if getattr(self, "h", None):
            load().pdlp_prop_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()


def branching(l, u, a, c):
    """Bound changes of the integer-aware branching rule, in increasing priority: [(lower, upper), ...]."""
    lo, hi, k = (C.c_double * 3)(), (C.c_double * 3)(), C.c_int32()
    _check(load().pdlp_branching(float(l), float(u), float(a), float(c), lo, hi, C.byref(k)))
    return [(lo[i], hi[i]) for i in range(k.value)]
