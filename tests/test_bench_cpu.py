"""Host-side checks of bench.py: its one-GPU contract and the digest that
keys the committed counter measurements to the pass kernel's code (a
comment edit keeps them, a code edit retires them)."""
import subprocess
import sys
from pathlib import Path

import pytest

ROOT = Path(__file__).resolve().parent.parent
sys.path.insert(0, str(ROOT))

import bench  # noqa: E402


def test_bench_refuses_more_than_one_gpu():
    r = subprocess.run([sys.executable, str(ROOT / "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def test_code_digest_ignores_comments_and_blank_lines():
    code = "int f(int a) {\n    return a + 1;\n}\n"
    commented = "// adds one\nint f(int a) {  // the argument\n\n    return a + 1;\n}\n"
    assert bench.code_digest(code) == bench.code_digest(commented)


def test_code_digest_ignores_line_wrapping():
    one = "#define L(a, b) call(a, b, 1)\nint g() { return f(1, 2, 3); }\n"
    wrapped = "#define L(a, b) \\\n    call(a, b, 1)\nint g() {\n    return f(1,\n             2, 3);\n}\n"
    assert bench.code_digest(one) == bench.code_digest(wrapped)


def test_code_digest_sees_code_changes():
    a = "int f(int a) {\n    return a + 1;\n}\n"
    b = "int f(int a) {\n    return a + 2;\n}\n"
    assert bench.code_digest(a) != bench.code_digest(b)



def _parse(argv):
    saved = sys.argv
    sys.argv = ["bench.py", *argv]
    try:
        return bench.parse()
    finally:
        sys.argv = saved


def test_driver_argv_times_whole_production_turns():
    # the round-end command: --gpus 1 --steps 20 --warmup 5
    a = _parse(["--gpus", "1", "--steps", "20", "--warmup", "5"])
    assert (a.gpus, a.steps, a.warmup, a.workload) == (1, 20, 5, "production")
    plan = bench.resolve_turns(a.workload, a.steps, a.warmup, 100)
    assert plan["timed_turns"] == 10 and plan["steps"] == 1000
    assert plan["warmup_turns"] == 2 and plan["warmup"] == 200
    assert plan["steps_requested"] == 20 and plan["warmup_requested"] == 5


def test_requests_are_lower_bounds_rounded_up_to_turns():
    assert bench.resolve_turns("production", 1001, 0, 100)["steps"] == 1100
    assert bench.resolve_turns("production", 3000, 250, 100)["warmup"] == 300
    assert bench.resolve_turns("small", 170, 1, 16)["steps"] == 176
    assert bench.resolve_turns("batch", 20, 5, 16)["steps"] == 5 * 16
    assert bench.resolve_turns("large", 1, 1, 200)["steps"] == 400
    # defaults, and odd but legal integers
    d = bench.resolve_turns("production", None, None, 100)
    assert (d["timed_turns"], d["warmup_turns"]) == (20, 2)
    assert bench.resolve_turns("production", 0, -3, 100)["timed_turns"] == 10


def test_driver_argv_reaches_the_gpu_check_on_a_cpu_host():
    # no GPU here: the run stops at the GPU check (exit 1), never at the
    # argument check (exit 2); on a GPU host this would run the whole bench
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is visible: the command would run the benchmark")
    r = subprocess.run([sys.executable, str(ROOT / "bench.py"), "--gpus", "1", "--steps", "20",
                        "--warmup", "5"], capture_output=True, text=True, timeout=300)
    assert r.returncode == 1, r.stderr
    assert "needs a GPU" in r.stderr


def test_cpu_model_is_named():
    assert isinstance(bench.cpu_model(), str) and bench.cpu_model()
