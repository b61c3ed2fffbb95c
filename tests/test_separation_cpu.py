"""The oracle and the product path share nothing: no module of the package
imports the oracle, the HIP sources include nothing from it, and the oracle
imports nothing from the package (the seeded input generator is the one
module both read, and it holds no arithmetic of the method)."""
import ast
import os
import re

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PKG = os.path.join(ROOT, "paper_1906_03958_amd")
ORACLE = os.path.join(ROOT, "oracle")


def _imports(path):
    tree = ast.parse(open(path).read())
    out = set()
    for node in ast.walk(tree):
        if isinstance(node, ast.Import):
            out |= {a.name.split(".")[0] for a in node.names}
        elif isinstance(node, ast.ImportFrom) and node.module:
            out.add(node.module.split(".")[0])
    return out


def _files(root, exts):
    for d, _, names in os.walk(root):
        for f in names:
            if f.endswith(exts):
                yield os.path.join(d, f)


def test_package_does_not_import_the_oracle():
    for f in _files(PKG, (".py",)):
        assert "oracle" not in _imports(f), f


def test_hip_sources_include_nothing_from_the_oracle():
    inc = re.compile(r'#\s*include\s*[<"]([^>"]+)[>"]')
    for f in _files(os.path.join(PKG, "csrc"), (".hip", ".h", ".cpp")):
        for name in inc.findall(open(f).read()):
            assert "oracle" not in name, (f, name)


def test_oracle_imports_nothing_from_the_package():
    for f in _files(ORACLE, (".py",)):
        assert "paper_1906_03958_amd" not in _imports(f), f
    src = open(os.path.join(ORACLE, "psst_oracle.c")).read()
    assert "psst.h" not in src and "csrc" not in src
