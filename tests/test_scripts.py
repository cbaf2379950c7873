"""Host-side checks of the scripts the GPU runs read: every name a function
of bench.py, the binding or the graft entry loads is defined (a misspelt
name would only surface at the end of a long GPU run), and bench.py refuses
more than one GPU with a message."""
import ast
import builtins
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SCRIPTS = ["bench.py", "__graft_entry__.py", os.path.join("paper_2012_03550_amd", "binding.py"),
           os.path.join("paper_2012_03550_amd", "synth.py"), os.path.join("paper_2012_03550_amd", "serve.py"),
           os.path.join("paper_2012_03550_amd", "tune.py")]


def _bound_names(node):
    out = set()
    for n in ast.walk(node):
        if isinstance(n, ast.Name) and isinstance(n.ctx, (ast.Store, ast.Del)):
            out.add(n.id)
        elif isinstance(n, ast.arg):
            out.add(n.arg)
        elif isinstance(n, (ast.Import, ast.ImportFrom)):
            for a in n.names:
                out.add((a.asname or a.name).split(".")[0])
        elif isinstance(n, (ast.FunctionDef, ast.AsyncFunctionDef, ast.ClassDef)):
            out.add(n.name)
        elif isinstance(n, ast.ExceptHandler) and n.name:
            out.add(n.name)
        elif isinstance(n, ast.Global):
            out.update(n.names)
    return out


def undefined_names(path):
    tree = ast.parse(open(path).read(), path)
    module_names = _bound_names(tree)  # generous: any name bound anywhere in the module
    bad = []
    for n in ast.walk(tree):
        if isinstance(n, ast.Name) and isinstance(n.ctx, ast.Load):
            if n.id not in module_names and not hasattr(builtins, n.id) and n.id != "__file__":
                bad.append((n.id, n.lineno))
    return bad


@pytest.mark.parametrize("rel", SCRIPTS)
def test_no_undefined_names(rel):
    assert undefined_names(os.path.join(ROOT, rel)) == []


def _function_locals_check(path):
    """Names loaded inside a function that are bound neither in it nor at module level."""
    tree = ast.parse(open(path).read(), path)
    top = set()
    for n in tree.body:
        if isinstance(n, (ast.FunctionDef, ast.ClassDef)):
            top.add(n.name)
        elif isinstance(n, ast.Assign):
            for t in n.targets:
                top.update(x.id for x in ast.walk(t) if isinstance(x, ast.Name))
        elif isinstance(n, (ast.Import, ast.ImportFrom)):
            top.update((a.asname or a.name).split(".")[0] for a in n.names)
    bad = []
    for fn in [n for n in tree.body if isinstance(n, ast.FunctionDef)]:
        local = _bound_names(fn)
        for n in ast.walk(fn):
            if isinstance(n, ast.Name) and isinstance(n.ctx, ast.Load):
                if n.id not in local and n.id not in top and not hasattr(builtins, n.id):
                    bad.append((fn.name, n.id, n.lineno))
    return bad


def test_bench_functions_use_only_their_own_or_module_names():
    assert _function_locals_check(os.path.join(ROOT, "bench.py")) == []


def test_bench_refuses_more_than_one_gpu():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode != 0
    assert "one GPU" in r.stderr
