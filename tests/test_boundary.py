"""Host checks of the separation between the product path and the oracle: the package
never imports the oracle, the oracle never imports the package, the seeded input
module holds no method code, and only smoke() and bench.py's CPU baseline reach the
oracle (inside those functions)."""
import ast
import glob
import os

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def imported_modules(tree):
    for node in ast.walk(tree):
        if isinstance(node, ast.Import):
            for a in node.names:
                yield node, a.name
        elif isinstance(node, ast.ImportFrom) and node.module:
            yield node, node.module


def parse(path):
    return ast.parse(open(path, encoding="utf-8").read(), filename=path)


def test_package_does_not_import_the_oracle():
    for path in glob.glob(os.path.join(ROOT, "paper_1707_06551_amd", "**", "*.py"), recursive=True):
        for _node, mod in imported_modules(parse(path)):
            assert not mod.split(".")[0] == "oracle", (path, mod)


def test_oracle_does_not_import_the_package():
    for path in glob.glob(os.path.join(ROOT, "oracle", "*.py")):
        for _node, mod in imported_modules(parse(path)):
            assert not mod.startswith("paper_1707_06551_amd"), (path, mod)


def test_input_generators_import_no_method_code():
    tree = parse(os.path.join(ROOT, "paper_1707_06551_amd", "inputs.py"))
    assert {mod.split(".")[0] for _n, mod in imported_modules(tree)} <= {"math", "numpy"}


def test_oracle_is_reached_only_from_smoke_and_the_cpu_baseline():
    # bench.py: the CPU-baseline leg is cpu_baseline and its helpers cpu_baseline_*
    allowed = {"__graft_entry__.py": {"smoke"}, "bench.py": {"cpu_baseline"}}
    for fname, funcs in allowed.items():
        tree = parse(os.path.join(ROOT, fname))
        inside = set()
        for fn in ast.walk(tree):
            if isinstance(fn, ast.FunctionDef) and (fn.name in funcs or (fname == "bench.py" and any(
                    fn.name.startswith(f + "_") for f in funcs))):
                inside |= {id(n) for n in ast.walk(fn)}
        for node, mod in imported_modules(tree):
            if mod.split(".")[0] == "oracle":
                assert id(node) in inside, (fname, mod, node.lineno)


def test_native_sources_do_not_reference_the_oracle():
    for path in glob.glob(os.path.join(ROOT, "paper_1707_06551_amd", "csrc", "*")) + \
            glob.glob(os.path.join(ROOT, "include", "*.h")):
        text = open(path, encoding="utf-8").read()
        assert "oracle" not in text.lower(), path


def test_product_path_fails_loudly_without_the_library(monkeypatch):
    # no fallback: with libbie.so absent the binding raises before any work is done
    import pytest

    from paper_1707_06551_amd import bie
    monkeypatch.setattr(bie, "LIB_PATH", os.path.join(ROOT, "no_such_dir", "libbie.so"))
    monkeypatch.setattr(bie, "_lib", None)
    with pytest.raises(RuntimeError, match="missing"):
        bie.lib()
