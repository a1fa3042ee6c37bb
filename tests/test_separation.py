"""The product path and the oracle stay apart: the package (HIP library,
binding, build step, input generators) imports no part of the oracle, the
HIP sources include nothing from it and it includes nothing of theirs,
every oracle file declares itself test infrastructure, and outside the
tests only the benchmark's CPU-baseline leg and the entry point's build
and smoke steps touch it."""
import ast
import glob
import os
import re

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PKG = os.path.join(ROOT, "paper_2606_12753_amd")
ORACLE = os.path.join(ROOT, "oracle")


def _oracle_imports(path):
    """(line, enclosing top-level function or None) of every import of the
    oracle package in a Python file."""
    tree = ast.parse(open(path).read(), filename=path)
    found = []

    def visit(node, func):
        for child in ast.iter_child_nodes(node):
            f = func
            if isinstance(child, (ast.FunctionDef, ast.AsyncFunctionDef)) and func is None:
                f = child.name
            names = []
            if isinstance(child, ast.Import):
                names = [a.name for a in child.names]
            elif isinstance(child, ast.ImportFrom) and child.module:
                names = [child.module]
            if any(n == "oracle" or n.startswith("oracle.") for n in names):
                found.append((child.lineno, f))
            visit(child, f)

    visit(tree, None)
    return found


def test_package_imports_no_oracle():
    files = glob.glob(os.path.join(PKG, "**", "*.py"), recursive=True)
    assert files
    for path in files:
        assert _oracle_imports(path) == [], path


def test_oracle_used_only_by_the_permitted_entry_points():
    bench = _oracle_imports(os.path.join(ROOT, "bench.py"))
    assert bench and all(f == "cpu_baseline" for _, f in bench), bench
    entry = _oracle_imports(os.path.join(ROOT, "__graft_entry__.py"))
    assert entry and all(f in ("build", "smoke") for _, f in entry), entry


def test_hip_and_oracle_sources_share_no_header():
    inc = re.compile(r'#\s*include\s*"([^"]+)"')
    for path in glob.glob(os.path.join(PKG, "csrc", "*")):
        for name in inc.findall(open(path).read()):
            assert "oracle" not in name and "flopcount" not in name, (path, name)
    for path in glob.glob(os.path.join(ORACLE, "*.[ch]")) + glob.glob(os.path.join(ORACLE, "*.hpp")):
        for name in inc.findall(open(path).read()):
            assert os.path.dirname(name) == "" and name.startswith(("mhd_oracle", "flopcount")), \
                (path, name)


def test_oracle_files_declare_test_infrastructure():
    paths = [p for ext in ("py", "c", "h", "hpp")
             for p in glob.glob(os.path.join(ORACLE, f"*.{ext}"))]
    assert paths
    for path in paths:
        head = re.sub(r"[\s*/#]+", " ", "".join(open(path).readlines()[:12]).lower())
        assert "test infrastructure" in head, path


def test_input_generators_use_neither_side():
    """The seeded input module serves both sides, so it imports neither the
    library binding nor the oracle."""
    tree = ast.parse(open(os.path.join(PKG, "workloads.py")).read())
    mods = set()
    for node in ast.walk(tree):
        if isinstance(node, ast.Import):
            mods.update(a.name for a in node.names)
        elif isinstance(node, ast.ImportFrom):
            mods.add(("." * node.level) + (node.module or ""))
    assert not any("oracle" in m or m.endswith("mhd") or m == ".mhd" for m in mods), mods
