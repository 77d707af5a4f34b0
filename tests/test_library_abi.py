"""CPU checks of the C ABI: the built library loads and exports every entry
point that include/vif.h declares (no compute calls: no GPU here)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_2507_05064_amd", "libvif.so")


def _declared():
    names = set()
    for h in os.listdir(os.path.join(ROOT, "include")):
        if h.endswith(".h"):
            txt = open(os.path.join(ROOT, "include", h)).read()
            names |= set(re.findall(r"^\s*(?:[A-Za-z_][\w\s\*]*?)\b(vif_\w+)\s*\(", txt, re.M))
    return names


@pytest.mark.skipif(not os.path.exists(LIB), reason="libvif.so not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    declared = _declared()
    assert "vif_create" in declared and "vif_nll_grad" in declared
    for name in sorted(declared):
        assert hasattr(lib, name), name


def test_binding_lists_every_declared_symbol():
    from paper_2507_05064_amd import vif
    assert _declared() == set(vif.EXPORTS)


def test_binding_refuses_without_gpu():
    import torch
    from paper_2507_05064_amd.vif import VifContext
    if torch.cuda.is_available():
        pytest.skip("GPU present")
    with pytest.raises(RuntimeError):
        VifContext(10, 2, 0, 2)
