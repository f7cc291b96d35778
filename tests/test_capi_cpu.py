"""The C-ABI library on the CPU: it loads, exports every function include/pdlp.h declares, and
rejects malformed input before touching a GPU (validation runs on the host)."""
import ctypes as C
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "pdlp.h")
HEADERS = [os.path.join(ROOT, "include", h) for h in ("pdlp.h", "pdlp_gnn.h", "pdlp_fix.h", "pdlp_prop.h")]


@pytest.fixture(scope="module")
def lib():
    from paper_2503_10344_amd import pdlp
    if not os.path.exists(pdlp.LIB_PATH):
        from paper_2503_10344_amd import build
        build.build()
    return pdlp.load()


def declared_functions():
    src = "\n".join(open(h).read() for h in HEADERS)
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[a-z_0-9]+\s*\**\s*(pdlp_[a-z_0-9]+)\s*\(", src, flags=re.M)
    return sorted(set(names))


def test_header_declares_the_boundary():
    names = declared_functions()
    for must in ("pdlp_create", "pdlp_solve", "pdlp_get", "pdlp_destroy", "pdlp_batch_create",
                 "pdlp_batch_solve", "pdlp_batch_get", "pdlp_gnn_create", "pdlp_gnn_predict",
                 "pdlp_gnn_train_step"):
        assert must in names


def test_library_exports_every_declared_symbol(lib):
    missing = [name for name in declared_functions() if not hasattr(lib, name)]
    assert not missing, missing


def test_struct_layout_matches_header(lib, tmp_path):
    """The ctypes mirrors have the sizes and field offsets a C compiler gives the header's structs."""
    from paper_2503_10344_amd import pdlp
    prog = tmp_path / "layout.c"
    fields = {"pdlp_options": [f for f, _ in pdlp.Options._fields_],
              "pdlp_result": [f for f, _ in pdlp.Result._fields_],
              "pdlp_problem_desc": [f for f, _ in pdlp.ProblemDesc._fields_]}
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "pdlp.h"', "int main(void){"]
    for st, fs in fields.items():
        lines.append(f'printf("{st} %zu\\n", sizeof({st}));')
        for f in fs:
            lines.append(f'printf("{st}.{f} %zu\\n", offsetof({st}, {f}));')
    lines.append("return 0;}")
    prog.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    import subprocess
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), str(prog), "-o", str(exe)], check=True)
    out = dict(ln.split() for ln in subprocess.run([str(exe)], capture_output=True, text=True,
                                                     check=True).stdout.splitlines())
    for st, cls in (("pdlp_options", pdlp.Options), ("pdlp_result", pdlp.Result),
                    ("pdlp_problem_desc", pdlp.ProblemDesc)):
        assert int(out[st]) == C.sizeof(cls), st
        for f, _ in cls._fields_:
            assert int(out[f"{st}.{f}"]) == getattr(cls, f).offset, (st, f)
    o = pdlp.Options()
    lib.pdlp_options_default(C.byref(o))
    assert (o.precision, o.eval_every, o.ruiz_iters, o.pock_chambolle, o.use_graphs) == (0, 64, 10, 1, 1)
    assert o.warm_fallback == 2 and o.tile_nnz == 0


def _create(lib, lp, **over):
    from paper_2503_10344_amd import pdlp
    a = pdlp._lp_arrays(lp)
    for k, v in over.items():
        a[k] = v
    h = C.c_void_p()
    o = pdlp.Options()
    lib.pdlp_options_default(C.byref(o))
    rc = lib.pdlp_create(C.byref(h), lp.m, lp.n, int(a["row_ptr"][-1]), pdlp._ptr(a["row_ptr"]),
                         pdlp._ptr(a["col"]), pdlp._ptr(a["val"]), pdlp._ptr(a["c"]), pdlp._ptr(a["b"]),
                         pdlp._ptr(a["sense"]), pdlp._ptr(a["l"]), pdlp._ptr(a["u"]), C.byref(o))
    return rc, lib.pdlp_last_error().decode()


def _small():
    from paper_2503_10344_amd import generators as g
    return g.general_sparse(0, m=30, n=50, cap=10)


def test_rejects_bad_csr(lib):
    lp = _small()
    rp = lp.row_ptr.copy()
    rp[5], rp[6] = rp[6], rp[5] + 0  # make row_ptr decrease
    if rp[5] <= rp[6]:
        rp[6] = rp[5] - 1
    rc, msg = _create(lib, lp, row_ptr=rp)
    assert rc == -2, msg
    col = lp.col.copy()
    col[0] = lp.n + 3
    rc, msg = _create(lib, lp, col=col)
    assert rc == -2 and "out of range" in msg
    # duplicate column in a row
    r = int(np.nonzero(np.diff(lp.row_ptr) >= 2)[0][0])
    col = lp.col.copy()
    col[lp.row_ptr[r] + 1] = col[lp.row_ptr[r]]
    rc, msg = _create(lib, lp, col=col)
    assert rc == -2 and "duplicate" in msg


def test_rejects_bad_data(lib):
    lp = _small()
    c = lp.c.copy()
    c[3] = np.nan
    assert _create(lib, lp, c=c)[0] == -1
    v = lp.val.copy()
    v[0] = np.inf
    assert _create(lib, lp, val=v)[0] == -1
    lo = lp.l.copy()
    lo[0], up0 = 5.0, lp.u.copy()
    up0[0] = 1.0
    assert _create(lib, lp, l=lo, u=up0)[0] == -1
    s = lp.sense.copy()
    s[0] = ord("X")
    assert _create(lib, lp, sense=s)[0] == -1


def test_rejects_sizes_beyond_int32_indices(lib):
    """Indices are 32-bit: 2^31 - 1 or more nonzeros, or negative sizes, are rejected before any
    input is read (the data pointers below are far too short to be read)."""
    from paper_2503_10344_amd import pdlp
    o = pdlp.Options()
    lib.pdlp_options_default(C.byref(o))
    one_i = np.zeros(2, np.int32)
    one_d = np.zeros(2)
    sense = np.full(2, ord("E"), np.uint8)
    for m, n, nnz in ((1, 1, 2**31 - 1), (1, 1, 2**31), (1, 1, 2**40), (-1, 1, 0), (1, -1, 0), (1, 1, -1)):
        h = C.c_void_p()
        rc = lib.pdlp_create(C.byref(h), m, n, nnz, pdlp._ptr(one_i), pdlp._ptr(one_i), pdlp._ptr(one_d),
                             pdlp._ptr(one_d), pdlp._ptr(one_d), pdlp._ptr(sense), pdlp._ptr(one_d),
                             pdlp._ptr(one_d), C.byref(o))
        assert rc == -1, (m, n, nnz)
        assert not h.value


def test_null_arguments(lib):
    assert lib.pdlp_create(None, 1, 1, 0, None, None, None, None, None, None, None, None, None) == -1
    assert lib.pdlp_solve(None, 1e-4, 10, None, None, 0.0) == -1
    assert lib.pdlp_get(None, None, None, None, None) == -1
    assert lib.pdlp_batch_get_schedule(None, None, None, None) == -1
    assert lib.pdlp_update_bounds(None, None, None) == -1
    assert lib.pdlp_batch_update_bounds(None, 0, None, None) == -1
    cnt = C.c_int32()
    assert lib.pdlp_variable_strategy(None, 1, 0, None, None, None, None, None, C.byref(cnt)) == -1
    assert lib.pdlp_lp_fixing(None, None, None, None, None, None, None) == -1
    assert lib.pdlp_prop_create(None, 1, 1, 0, None, None, None, None, None, None, None) == -1
    assert lib.pdlp_propagate(None, None, None, 10, None, None) == -1
    assert lib.pdlp_set_snapshots(None, 4, 1e-3) == -1
    assert lib.pdlp_batch_set_snapshots(None, 4, 1e-3) == -1
    assert lib.pdlp_get_snapshots(None, 4, None, None, None, None, C.byref(cnt)) == -1
    assert lib.pdlp_batch_get_snapshots(None, 0, 4, None, None, None, None, C.byref(cnt)) == -1


def test_branching_rule_matches_oracle(lib):
    """pdlp_branching is host code: checked here against the oracle on every case of small domains."""
    from oracle import fix_oracle as fo
    from paper_2503_10344_amd import pdlp
    for l in range(-2, 3):
        for u in range(l, l + 4):
            for a in range(l, u + 1):
                for c in (-1.5, 0.0, 2.0):
                    assert pdlp.branching(l, u, a, c) == fo.branching(l, u, a, c), (l, u, a, c)
    for bad in ((0, 5, 6, 1.0), (0, 5, 2.5, 1.0), (0, 5, float("nan"), 1.0)):
        with pytest.raises(pdlp.PDLPError):
            pdlp.branching(*bad)
    assert lib.pdlp_error_string(-2) == b"malformed CSR matrix"


def test_gnn_header_compiles_as_c_and_parameter_count(lib, tmp_path):
    """pdlp_gnn.h is plain C, and the library's parameter count is the oracle's."""
    import subprocess
    from oracle import gnn_oracle
    prog = tmp_path / "g.c"
    prog.write_text('#include "pdlp_gnn.h"\nint main(void){return pdlp_gnn_num_params == 0;}\n')
    subprocess.run(["gcc", "-c", "-I", os.path.join(ROOT, "include"), str(prog), "-o", str(tmp_path / "g.o")],
                   check=True)
    assert lib.pdlp_gnn_num_params() == gnn_oracle.num_params() == 50947


def test_gnn_rejects_null_arguments(lib):
    assert lib.pdlp_gnn_create(None, 0) == -1
    assert lib.pdlp_gnn_predict(None, None, None, None, None) == -1
    assert lib.pdlp_gnn_train_step(None, None, None, None, None, C.c_float(1e-3), None) == -1
    assert lib.pdlp_batch_get_internal(None, *([None] * 8)) == -1
    assert lib.pdlp_gnn_set_omega_weight(None, C.c_float(1.0)) == -1


def test_binding_checks_vector_lengths(lib):
    """Vectors the library reads n or m entries of are checked in the binding: a short array raises
    ValueError instead of being read past its end (no GPU needed: the check comes before any call)."""
    from paper_2503_10344_amd import pdlp
    prob = pdlp.Problem.__new__(pdlp.Problem)  # no device handle: only the checks run
    prob.m, prob.n, prob.h = 3, 5, None
    for kw in (dict(x0=np.zeros(4)), dict(y0=np.zeros(2)), dict(x0=np.zeros((5, 1)))):
        with pytest.raises(ValueError):
            prob.solve(**kw)
    with pytest.raises(ValueError):
        prob.spmv(np.zeros(3))
    with pytest.raises(ValueError):
        prob.spmv(np.zeros(5), trans=True)
    with pytest.raises(ValueError):
        prob.update_bounds(np.zeros(5), np.zeros(4))
    bt = pdlp.Batch.__new__(pdlp.Batch)
    bt.dims, bt.h = [(3, 5), (2, 4)], None
    with pytest.raises(ValueError):
        bt.solve(x0s=[np.zeros(5), np.zeros(5)])
    with pytest.raises(ValueError):
        bt.solve(y0s=[np.zeros(3)])
    with pytest.raises(ValueError):
        bt.solve(omega0s=[1.0])
    with pytest.raises(ValueError):
        bt.update_bounds(1, np.zeros(5), np.zeros(5))
