"""The oracle and the library share no code (CPU only, reads the sources).

* nothing in the package (Python, HIP, C++) or the public header imports or
  includes anything from oracle/;
* nothing in oracle/ imports the package or includes its headers (the tests
  hand both sides the same seeded arrays from the package's input generators);
* outside tests/, the oracle is imported only by bench.py's cpu_baseline and
  by __graft_entry__'s build (which compiles it) and smoke.
"""
import ast
import os
import re

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PKG = os.path.join(ROOT, "paper_2607_25444_amd")
ORC = os.path.join(ROOT, "oracle")


def _files(top, exts):
    for d, dirs, names in os.walk(top):
        dirs[:] = [x for x in dirs if not x.startswith(("_build", "__pycache__"))]
        for n in names:
            if n.endswith(exts):
                yield os.path.join(d, n)


def _imports(path):
    """(module, enclosing top-level function or None) of every import."""
    tree = ast.parse(open(path).read(), path)
    out = []

    def visit(node, fn):
        for ch in ast.iter_child_nodes(node):
            f = ch.name if isinstance(ch, (ast.FunctionDef, ast.AsyncFunctionDef)) and fn is None else fn
            if isinstance(ch, ast.Import):
                out.extend((a.name, fn) for a in ch.names)
            elif isinstance(ch, ast.ImportFrom):
                out.append(("." * ch.level + (ch.module or ""), fn))
            visit(ch, f)

    visit(tree, None)
    return out


def _includes(path):
    return re.findall(r'^\s*#\s*include\s*[<"]([^>"]+)[>"]', open(path).read(), re.M)


def test_package_does_not_use_the_oracle():
    for p in _files(PKG, (".py",)):
        for mod, _ in _imports(p):
            assert not mod.lstrip(".").startswith("oracle"), (p, mod)
    for p in list(_files(PKG, (".hip", ".cpp", ".hpp", ".h"))) + list(_files(os.path.join(ROOT, "include"), (".h",))):
        for inc in _includes(p):
            assert "oracle" not in inc, (p, inc)


def test_oracle_does_not_use_the_package():
    for p in _files(ORC, (".py",)):
        for mod, _ in _imports(p):
            assert "paper_2607_25444_amd" not in mod and not mod.startswith("bench"), (p, mod)
    for p in _files(ORC, (".c", ".h")):
        for inc in _includes(p):
            assert "csrc" not in inc and "cac.h" not in inc and "paper_2607_25444_amd" not in inc, (p, inc)


def test_oracle_entry_points_outside_tests():
    allowed = {"bench.py": {"cpu_baseline"}, "__graft_entry__.py": {"build", "smoke"}}
    for name, fns in allowed.items():
        for mod, fn in _imports(os.path.join(ROOT, name)):
            if mod.startswith("oracle"):
                assert fn in fns, (name, mod, fn)
