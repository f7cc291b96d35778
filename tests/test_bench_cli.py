"""The benchmark's command line on the CPU: it measures one GPU and says so when asked for more,
before touching a GPU; every workload name it accepts is one it dispatches."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_exits_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120, cwd=ROOT)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def test_every_workload_choice_is_dispatched():
    src = open(os.path.join(ROOT, "bench.py")).read()
    start = src.index('"--workload"')
    choices = src[src.index("choices=[", start) + len("choices=["): src.index("]", start)]
    names = [c.strip().strip('"') for c in choices.replace("\n", " ").split(",") if c.strip()]
    assert "zipf" in names and "snapshots" in names
    for name in names:
        if name in ("zipf", "setcover", "energy"):
            assert f'name == "{name}"' in src  # make_workload builds it
        else:
            assert f'args.workload == "{name}"' in src, name


def _bench():
    sys.path.insert(0, ROOT)
    import bench
    return bench


def test_algorithmic_bytes_of_the_500k_x_1m_lp():
    """The per-launch byte counts the roofline divides by, for the 500k x 1M LP in FP32: A side =
    8 B per nonzero (value + column), 4 B per row offset, one gather of x' (4 B per column), and per
    row y, Ax, b read, the sense byte, y' and Ax' written (21 B); the primal side likewise with the
    transpose, plus the paired FP64 averages (10 B per column and 12 B per row)."""
    b = _bench()
    m, n, nnz = 500_000, 1_000_000, 27_350_943
    assert b.algorithmic_bytes("dual", m, n, nnz, 4) == 8 * nnz + 4 * (m + 1) + 4 * n + 21 * m == 235_307_548
    assert b.algorithmic_bytes("primal", m, n, nnz, 4) == 8 * nnz + 4 * (n + 1) + 4 * m + 34 * n + 12 * m \
        == 264_807_548


def test_oracle_reference_is_the_stored_solve_of_the_same_lp_and_tolerance():
    b = _bench()

    class A:
        workload, seed, tol = "zipf", 0, 1e-4
    ref = b.oracle_reference(A, {"primal_obj": -3_166_000.0}, {"dobj": -3_165_900.0})
    assert ref["attempts"] == 16_512 and ref["tol"] == 1e-4
    assert abs(ref["primal_obj_rel_diff"] - abs(-3_166_000.0 - ref["pobj"]) / abs(ref["pobj"])) < 1e-15
    for w, s, t in (("energy", 0, 1e-4), ("zipf", 1, 1e-4), ("zipf", 0, 1e-6)):
        A.workload, A.seed, A.tol = w, s, t
        assert b.oracle_reference(A, {"primal_obj": 0.0}, {}) is None
