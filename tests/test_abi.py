"""Host-side checks of the C ABI (no GPU needed): the built library loads and
exports every function that include/demag.h declares, and the binding knows
each of them."""
import os
import re

from paper_1212_3509_amd import api

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    names = set()
    for fn in os.listdir(os.path.join(ROOT, "include")):
        if fn.endswith(".h"):
            src = open(os.path.join(ROOT, "include", fn)).read()
            src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
            names |= set(re.findall(r"\b(demag_[a-z0-9_]+)\s*\(", src))
    return names


def test_library_exports_every_declared_symbol():
    lib = api.library()
    declared = _declared()
    assert "demag_apply_full" in declared and "demag_assemble_factors" in declared
    for name in declared:
        assert hasattr(lib, name), name


def test_binding_covers_declarations():
    assert _declared() <= set(api.exported_symbols())


def test_bench_refuses_several_gpus():
    """bench.py measures one GPU; asking for more exits with status 2 and a
    message, before anything touches a device."""
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    res = subprocess.run([sys.executable, os.path.join(root, "bench.py"), "--gpus", "2"], capture_output=True,
                         text=True, timeout=120)
    assert res.returncode == 2
    assert "single GPU" in res.stderr
