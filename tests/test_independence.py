"""Structural checks: the oracle and the GPU path share no code.

The GPU package never imports the oracle and its HIP sources include nothing
from it; the oracle includes nothing from the GPU sources and imports nothing
from the package; the benchmark reaches the oracle only from its CPU-baseline
leg.  The seeded input generators are the one module both sides read.
"""
import ast
import os
import re

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PKG = os.path.join(ROOT, "paper_1604_07163_amd")
ORACLE = os.path.join(ROOT, "oracle")


def files(top, exts):
    for d, _, names in os.walk(top):
        for n in names:
            if n.endswith(exts):
                yield os.path.join(d, n)


def imported_modules(path):
    """(module name, enclosing function or None) for every import in a file."""
    tree = ast.parse(open(path).read(), path)
    out = []

    def visit(node, fn):
        for child in ast.iter_child_nodes(node):
            f = child.name if isinstance(child, (ast.FunctionDef, ast.AsyncFunctionDef)) else fn
            if isinstance(child, ast.Import):
                out.extend((a.name, fn) for a in child.names)
            elif isinstance(child, ast.ImportFrom):
                base = "." * child.level + (child.module or "")
                out.append((base, fn))
                out.extend((f"{base}.{a.name}", fn) for a in child.names)
            visit(child, f)

    visit(tree, None)
    return out


def test_gpu_package_never_imports_the_oracle():
    for p in files(PKG, (".py",)):
        for mod, _ in imported_modules(p):
            assert not mod.split(".")[0] == "oracle", (p, mod)


def test_hip_sources_include_nothing_from_the_oracle():
    srcs = list(files(PKG, (".hip", ".hpp", ".h", ".cpp"))) + list(files(os.path.join(ROOT, "include"), (".h",)))
    assert srcs
    for p in srcs:
        for inc in re.findall(r'#include\s*[<"]([^>"]+)[>"]', open(p).read()):
            assert "oracle" not in inc, (p, inc)


def test_oracle_includes_and_imports_nothing_from_the_gpu_path():
    for p in files(ORACLE, (".c", ".h")):
        for inc in re.findall(r'#include\s*[<"]([^>"]+)[>"]', open(p).read()):
            assert inc in {"math.h", "stdint.h", "stdlib.h", "string.h", "stdio.h", "float.h"}, (p, inc)
    for p in files(ORACLE, (".py",)):
        for mod, _ in imported_modules(p):
            assert "paper_1604_07163_amd" not in mod and "gmg" != mod.split(".")[-1], (p, mod)


def test_benchmark_reaches_the_oracle_only_from_the_cpu_baseline():
    uses = [fn for mod, fn in imported_modules(os.path.join(ROOT, "bench.py")) if mod.split(".")[0] == "oracle"]
    assert uses and set(uses) == {"cpu_baseline"}


def test_shared_input_module_calls_neither_side():
    """The one module both sides use draws inputs; it imports neither the
    oracle nor the GPU binding."""
    mods = {m for m, _ in imported_modules(os.path.join(PKG, "inputs.py"))}
    assert mods <= {"__future__", "__future__.annotations", "numpy", "scipy.ndimage",
                    "scipy.ndimage.gaussian_filter", "torch"}, mods


def test_stored_expected_values_come_from_the_oracle_only():
    """The script that writes the golden files runs the oracle and reads only
    the input generators from the package."""
    mods = {m for m, _ in imported_modules(os.path.join(ROOT, "tests", "golden", "make_golden.py"))}
    pkg = {m for m in mods if m.startswith("paper_1604_07163_amd")}
    assert pkg == {"paper_1604_07163_amd", "paper_1604_07163_amd.inputs"}, pkg
    assert "oracle" in mods


def test_missing_library_fails_loudly(monkeypatch, tmp_path):
    """Without the built HIP library the binding raises; there is no fallback."""
    import pytest

    from paper_1604_07163_amd import gmg

    monkeypatch.setattr(gmg, "_lib", None)
    monkeypatch.setattr(gmg, "LIB_PATH", str(tmp_path / "libgmg.so"))
    with pytest.raises(RuntimeError, match="not built"):
        gmg.lib()
