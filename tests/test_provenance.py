"""Where stored expected values come from, and what may call the oracle.

* Every golden file under tests/golden/ names the script that wrote it, and
  that script imports nothing but the oracle, the seeded input generators
  and the standard library / NumPy: no stored value comes from the HIP path.
* The oracle and the HIP package share no code: neither imports the other.
* Outside tests/, only bench.py (its CPU-baseline leg) and
  __graft_entry__.py (its smoke check) import the oracle.
"""

import ast
import json
import os

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
GOLDEN = os.path.join(ROOT, "tests", "golden")
PKG = "paper_2401_06277_amd"
ALLOWED_GOLDEN_IMPORTS = {"oracle", "stokes_inputs", "numpy", "json", "os", "sys", "time",
                          "__future__", "math"}


def _imported_modules(path):
    tree = ast.parse(open(path).read(), filename=path)
    mods = set()
    for node in ast.walk(tree):
        if isinstance(node, ast.Import):
            mods.update(a.name.split(".")[0] for a in node.names)
        elif isinstance(node, ast.ImportFrom):
            if node.level == 0 and node.module:
                mods.add(node.module.split(".")[0])
            elif node.level > 0:
                mods.add(".")
    return mods


def _py_files(d):
    for base, _, files in os.walk(d):
        if "__pycache__" in base:
            continue
        for f in files:
            if f.endswith(".py"):
                yield os.path.join(base, f)


def test_golden_files_name_an_oracle_only_script():
    jsons = [f for f in os.listdir(GOLDEN) if f.endswith(".json")]
    assert jsons
    for f in jsons:
        with open(os.path.join(GOLDEN, f)) as fh:
            d = json.load(fh)
        script = d["written_by"].split()[0]
        path = os.path.join(ROOT, script)
        assert os.path.dirname(path) == GOLDEN and os.path.exists(path), (f, script)
        mods = _imported_modules(path)
        assert mods <= ALLOWED_GOLDEN_IMPORTS, (script, mods - ALLOWED_GOLDEN_IMPORTS)


def test_oracle_and_hip_package_share_no_code():
    for path in _py_files(os.path.join(ROOT, "oracle")):
        assert PKG not in _imported_modules(path), path
    for path in _py_files(os.path.join(ROOT, PKG)):
        assert "oracle" not in _imported_modules(path), path
    for base, _, files in os.walk(os.path.join(ROOT, PKG, "csrc")):
        for f in files:
            text = open(os.path.join(base, f), errors="replace").read()
            assert "oracle/" not in text, f


def test_only_the_checkers_import_the_oracle_outside_tests():
    users = []
    for f in os.listdir(ROOT):
        if f.endswith(".py") and "oracle" in _imported_modules(os.path.join(ROOT, f)):
            users.append(f)
    for d in (PKG, "stokes_inputs"):
        for path in _py_files(os.path.join(ROOT, d)):
            if "oracle" in _imported_modules(path):
                users.append(os.path.relpath(path, ROOT))
    assert sorted(users) == ["__graft_entry__.py", "bench.py"], users
