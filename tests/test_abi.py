"""The C-ABI library loads and exports every function include/spx.h declares; no GPU call."""
import os
import re
import subprocess

from paper_2308_15964_amd import spx

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    text = open(os.path.join(ROOT, "include", "spx.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"\b(spx_[a-z0-9_]+)\s*\(", text)
    return [n for n in dict.fromkeys(names) if not n.endswith("_fn")]


def test_header_matches_binding_list():
    assert declared_functions() == spx.EXPORTS


def test_library_exports_every_declared_symbol():
    lib = spx.lib()
    for name in declared_functions():
        assert hasattr(lib, name), name
    out = subprocess.run(["nm", "-D", "--defined-only", spx.LIB_PATH], capture_output=True, text=True).stdout
    exported = {line.split()[-1] for line in out.splitlines() if line.strip()}
    for name in declared_functions():
        assert name in exported, name


def test_error_message_roundtrip():
    import pytest

    with pytest.raises(spx.SpxError) as e:
        spx.Graph.build(1, [(0, 9, 0)])
    assert "mode" in str(e.value)
