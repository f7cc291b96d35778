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
