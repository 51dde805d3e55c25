"""Checks of bench.py that need no GPU: every function its sections call is
defined, the default section list names only sections main() handles, and
--gpus above 1 is refused with a message."""
import ast
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
BENCH = os.path.join(ROOT, "bench.py")


def _tree():
    with open(BENCH) as f:
        return ast.parse(f.read())


def test_called_bench_functions_are_defined():
    tree = _tree()
    defined = {n.name for n in tree.body if isinstance(n, ast.FunctionDef)}
    called = {n.func.id for n in ast.walk(tree)
              if isinstance(n, ast.Call) and isinstance(n.func, ast.Name)
              and n.func.id.startswith(("bench_", "cpu_", "timed_", "traffic_", "ratio_"))}
    assert called, "no bench functions found"
    assert called <= defined, f"called but not defined: {sorted(called - defined)}"


def test_default_sections_are_handled():
    tree = _tree()
    with open(BENCH) as f:
        src = f.read()
    default = None
    for n in ast.walk(tree):
        if (isinstance(n, ast.Call) and isinstance(n.func, ast.Attribute)
                and n.func.attr == "add_argument" and n.args
                and isinstance(n.args[0], ast.Constant) and n.args[0].value == "--sections"):
            for kw in n.keywords:
                if kw.arg == "default":
                    default = kw.value.value
    assert default, "--sections has no default"
    for sec in default.split(","):
        if sec == "plain":               # the headline product always runs
            continue
        assert f'"{sec}"' in src, f"section {sec} is not handled in main()"


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, BENCH, "--gpus", "2"], capture_output=True, text=True,
                       cwd=ROOT, timeout=120)
    assert r.returncode != 0
    assert "one GPU" in (r.stdout + r.stderr)
