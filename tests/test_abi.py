"""The C-ABI library loads and exports every symbol include/ctrex.h declares.

CPU-only: no compute call is made (there is no device here).
"""

import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared(header):
    text = open(os.path.join(ROOT, "include", header)).read()
    return sorted(set(re.findall(r"CTREX_API\s+[\w\s\*]*?\b(ctrex_\w+)\s*\(", text)))


def _lib():
    from paper_2609_30166_amd import _lib

    if not os.path.exists(_lib.library_path()):
        pytest.skip("libctrex.so not built (run __graft_entry__.build())")
    return _lib.lib()


def test_header_declares_the_boundary():
    names = _declared("ctrex.h")
    for need in ("ctrex_set_geometry", "ctrex_forward_project", "ctrex_back_project",
                 "ctrex_sirt_iterate"):
        assert need in names


@pytest.mark.parametrize("header", ["ctrex.h", "ctrex_nn.h"])
def test_every_declared_symbol_is_exported(header):
    L = _lib()
    names = _declared(header)
    assert names
    for name in names:
        assert hasattr(L, name), name


def test_binding_covers_every_declared_symbol():
    """Every entry point of the headers has a ctypes signature."""
    from paper_2609_30166_amd import _lib as binding

    src = open(binding.__file__).read()
    for header in ("ctrex.h", "ctrex_nn.h"):
        for name in _declared(header):
            assert '"%s"' % name in src, name


def test_create_without_device_reports_device_error():
    L = _lib()
    import torch

    if torch.cuda.is_available():
        pytest.skip("a device is present")
    ctx = ctypes.c_void_p()
    assert L.ctrex_create(ctypes.byref(ctx), 0) == -5
    assert L.ctrex_last_error(None) == b"null context"
    L.ctrex_destroy(None)


def test_package_has_no_cpu_fallback():
    """The product path must not import the oracle."""
    pkg = os.path.join(ROOT, "paper_2609_30166_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".cpp", ".hip", ".h")):
                text = open(os.path.join(dirpath, f)).read()
                assert "import oracle" not in text and "from oracle" not in text, f
