"""The C-ABI library loads on the CPU host and exports every function the
public header declares (no compute call: that needs a GPU)."""
import os
import re

import paper_2303_03848_amd as bsp

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "bsparareal.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"^(?:const\s+)?[a-z_]+\s*\*?\s*([a-z_]+)\s*\(", src, flags=re.M)))


def test_header_declares_expected_entry_points():
    names = _declared()
    assert set(bsp.EXPORTS) <= set(names), names
    assert len(names) == len(bsp.EXPORTS), names


def test_library_exports_every_declared_symbol():
    lib = bsp.load_library()
    for name in _declared():
        assert hasattr(lib, name), name


def test_no_cpu_fallback_in_binding():
    """The binding never imports the oracle."""
    pkg = os.path.join(ROOT, "paper_2303_03848_amd")
    for fn in os.listdir(pkg):
        if fn.endswith(".py"):
            src = open(os.path.join(pkg, fn)).read()
            assert not re.search(r"^\s*(import|from)\s+oracle", src, flags=re.M), fn
