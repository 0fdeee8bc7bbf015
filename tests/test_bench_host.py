"""Host-side checks of bench.py: the one-GPU guard, and the source hash that
decides whether the stored HBM counters still describe the current kernel
(the roofline's traffic is reported only while they do)."""
import os
import subprocess
import sys

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_exits_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_code_hash_ignores_comments_and_layout_only():
    a = "int f(int x) {\n  return x + 1; // one more\n}\n/* note */"
    b = "int f(int x) { return x + 1; }  // edited comment\n"
    c = "int f(int x) { return x + 2; }"
    assert bench.code_hash([a]) == bench.code_hash([b])
    assert bench.code_hash([a]) != bench.code_hash([c])
    assert bench.code_hash(["int a;", "int b;"]) != bench.code_hash(["int b;", "int a;"])

