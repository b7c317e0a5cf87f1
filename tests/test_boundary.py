"""The product path and the oracle stay apart (CPU): nothing in the package imports the oracle, the
oracle imports nothing of the package or of the shared input generators' arithmetic, and the binding
fails loudly (no fallback) when the library has not been built."""
import ast
import os

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _imports(path):
    tree = ast.parse(open(path).read(), path)
    names = set()
    for node in ast.walk(tree):
        if isinstance(node, ast.Import):
            names |= {a.name.split(".")[0] for a in node.names}
        elif isinstance(node, ast.ImportFrom) and node.module and node.level == 0:
            names.add(node.module.split(".")[0])
    return names


def _py_files(sub):
    for d, _, files in os.walk(os.path.join(ROOT, sub)):
        for f in files:
            if f.endswith(".py"):
                yield os.path.join(d, f)


def test_package_never_imports_the_oracle():
    bad = [p for p in _py_files("paper_1905_01348_amd") if "oracle" in _imports(p)]
    assert not bad, bad


def test_oracle_never_imports_the_package_or_synth():
    bad = [p for p in _py_files("oracle") if _imports(p) & {"paper_1905_01348_amd", "synth", "torch"}]
    assert not bad, bad


def test_synth_holds_no_library_or_oracle_code():
    bad = [p for p in _py_files("synth") if _imports(p) & {"paper_1905_01348_amd", "oracle"}]
    assert not bad, bad


def test_binding_raises_without_the_library(monkeypatch, tmp_path):
    from paper_1905_01348_amd import fock as F

    monkeypatch.setattr(F, "_lib", None)
    monkeypatch.setattr(F, "LIB_PATH", str(tmp_path / "libfock.so"))
    with pytest.raises(RuntimeError, match="not built"):
        F.load()
