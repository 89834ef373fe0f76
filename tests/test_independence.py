"""The oracle and the HIP path share no code: neither imports the other, the
shared input generator holds no import of either, and outside the tests only
the benchmark's CPU-baseline leg and smoke() reach the oracle (static check of
the sources)."""
import ast
import os

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PKG = os.path.join(ROOT, "paper_1509_00680_amd")


def _imports(path):
    """(module, enclosing top-level function or None) of every import."""
    tree = ast.parse(open(path).read(), path)
    out = []

    def visit(node, fn):
        for child in ast.iter_child_nodes(node):
            f = fn
            if isinstance(child, (ast.FunctionDef, ast.AsyncFunctionDef)) and fn is None:
                f = child.name
            if isinstance(child, ast.Import):
                out.extend((a.name, f) for a in child.names)
            elif isinstance(child, ast.ImportFrom):
                out.append(((child.module or "") if not child.level else "." + (child.module or ""), f))
            visit(child, f)

    visit(tree, None)
    return out


def _py(dirname):
    return [os.path.join(dirname, f) for f in sorted(os.listdir(dirname)) if f.endswith(".py")]


def test_oracle_imports_nothing_of_the_hip_path():
    for path in _py(os.path.join(ROOT, "oracle")):
        for mod, _ in _imports(path):
            assert not mod.startswith("paper_1509_00680_amd"), (path, mod)
        assert "libgps" not in open(path).read(), path


def test_package_never_imports_the_oracle():
    for path in _py(PKG):
        for mod, _ in _imports(path):
            assert not mod.startswith("oracle"), (path, mod)


def test_input_generator_is_neutral():
    # the seeded input generator serves both sides and imports neither
    for mod, _ in _imports(os.path.join(PKG, "workloads.py")):
        assert not mod.startswith("oracle") and not mod.startswith("paper_1509_00680_amd")
        assert mod not in (".", ".gps", ".build"), mod


def test_oracle_reached_only_by_the_cpu_baseline_and_smoke():
    allowed = {"bench.py": {"oracle_accuracy", "_oracle_electrolyte", "cpu_baseline"},
               "__graft_entry__.py": {"smoke"}}
    for name, fns in allowed.items():
        for mod, fn in _imports(os.path.join(ROOT, name)):
            if mod.startswith("oracle"):
                assert fn in fns, (name, mod, fn)
