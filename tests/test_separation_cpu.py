"""Structural checks: the product path never touches the oracle, the oracle
never touches the product path, and bench.py refuses multi-GPU runs."""
import os
import re
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PKG = os.path.join(ROOT, "paper_2306_09427_amd")


def _files(d, exts):
    for base, _, names in os.walk(d):
        if "_build" in base or "__pycache__" in base:
            continue
        for n in names:
            if n.endswith(exts):
                yield os.path.join(base, n)


def test_product_does_not_reference_oracle():
    for f in _files(PKG, (".py", ".hip", ".h", ".cpp")):
        src = open(f).read()
        assert not re.search(r"^\s*(import|from)\s+oracle", src, re.M), f
        assert "dr_oracle" not in src and "liboracle" not in src, f


def test_oracle_does_not_reference_product():
    for f in _files(os.path.join(ROOT, "oracle"), (".py", ".c", ".h")):
        src = open(f).read()
        assert "paper_2306_09427_amd" not in src and "rve_batch" not in src and "librvebatch" not in src, f


def test_generator_holds_no_method_arithmetic():
    """synth.py calls no fiber-law or relaxation functions (only geometry)."""
    import ast
    tree = ast.parse(open(os.path.join(PKG, "synth.py")).read())
    called = set()
    for node in ast.walk(tree):
        if isinstance(node, ast.Call):
            f = node.func
            called.add(f.attr if isinstance(f, ast.Attribute) else getattr(f, "id", ""))
    assert not called & {"exp", "expm1", "solve", "stress", "forces"}, called & {"exp", "expm1", "solve"}


def test_bench_refuses_multi_gpu():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2 and "one GPU" in r.stderr


def test_run_config_needs_a_gpu():
    """The workload runner has no CPU path: without a GPU it exits with a
    message instead of falling back."""
    import pytest
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    r = subprocess.run([sys.executable, "-m", "paper_2306_09427_amd.run_config", "--config", "1"], cwd=ROOT,
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2 and "needs a GPU" in r.stderr
