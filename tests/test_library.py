"""Host-only checks of the C-ABI library: it is built for gfx950, loads, and exports exactly
the entry points include/thc.h declares (no GPU call is made)."""
import ctypes
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "thc.h")
LIB = os.path.join(ROOT, "paper_2111_11473_amd", "libthc.so")


def _declared():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(thc_[a-z_0-9]+)\s*\(", txt)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        pytest.fail("libthc.so is not built (run __graft_entry__.build())")
    return ctypes.CDLL(LIB)


def test_header_declares_the_binding_symbols():
    from paper_2111_11473_amd import thc
    assert _declared() == sorted(thc.SYMBOLS)


def test_library_exports_every_declared_symbol(lib):
    for name in _declared():
        assert hasattr(lib, name), name
    out = subprocess.run(["nm", "-D", "--defined-only", LIB], capture_output=True, text=True).stdout
    exported = set(re.findall(r"\bT (thc_[a-z_0-9]+)$", out, flags=re.M))
    assert exported == set(_declared())


def test_library_contains_gfx950_code():
    """The device code object bundled in the library targets gfx950 (MI355X)."""
    data = open(LIB, "rb").read()
    assert b"amdgcn-amd-amdhsa--gfx950" in data


def test_binding_refuses_host_tensors():
    import torch
    from paper_2111_11473_amd import thc
    with pytest.raises(TypeError):
        thc._ptr(torch.zeros(3, dtype=torch.float64))
