"""bench.py's command-line contract, checked without a GPU: more than one GPU is refused with a
message, and every leg the default run calls is defined."""
import ast
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    msg = json.loads(r.stdout.strip().splitlines()[-1])
    assert "one GPU" in msg["error"]


def test_default_legs_are_defined():
    tree = ast.parse(open(os.path.join(ROOT, "bench.py")).read())
    defined = {n.name for n in tree.body if isinstance(n, ast.FunctionDef)}
    called = {n.func.id for n in ast.walk(tree) if isinstance(n, ast.Call) and isinstance(n.func, ast.Name)}
    for name in ("main", "make_data", "make_event", "serve_bench", "cpu_baseline", "host_terms", "percentiles"):
        assert name in defined
    local = {c for c in called if c in defined or c.startswith(("make_", "serve_", "cpu_"))}
    assert local <= defined, local - defined
