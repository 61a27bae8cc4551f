"""Host-side checks of bench.py: its one-GPU contract and the digest that
keys the committed counter measurements to the pass kernel's code (a
comment edit keeps them, a code edit retires them)."""
import subprocess
import sys
from pathlib import Path

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

