"""Host-side checks of the C-ABI library (no GPU compute)."""
import ctypes
import os
import re

import pytest

from paper_2505_00529_amd import qoc

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_symbols():
    text = open(os.path.join(ROOT, "include", "qoc.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = set(re.findall(r"\b(qoc_[a-z_0-9]+)\s*\(", text))
    return sorted(names)


def test_library_exports_every_declared_symbol():
    lib = qoc.lib()
    names = _declared_symbols()
    assert len(names) >= 30
    for name in names:
        assert hasattr(lib, name), name
        assert name in qoc.SIGNATURES, name


def test_status_strings():
    lib = qoc.lib()
    for code in range(-8, 1):
        s = lib.qoc_status_string(code)
        assert s and s.decode() != "unknown status"
    assert lib.qoc_status_string(-99).decode() == "unknown status"
    assert lib.qoc_last_error(None).decode() == "NULL handle"


def test_null_handle_calls_are_rejected():
    lib = qoc.lib()
    assert lib.qoc_set_weights(None, 1.0, 1.0) == qoc.QOC_ERR_INVALID_ARG
    assert lib.qoc_cost(None, None, None) == qoc.QOC_ERR_INVALID_ARG
    assert lib.qoc_set_checkpoint_interval(None, 10) == qoc.QOC_ERR_INVALID_ARG
    assert lib.qoc_create(0, None, None) == qoc.QOC_ERR_INVALID_ARG
    lib.qoc_destroy(None)


def test_create_without_device_fails_cleanly():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a device is present")
    h = ctypes.c_void_p()
    st = qoc.lib().qoc_create(0, None, ctypes.byref(h))
    assert st in (qoc.QOC_ERR_DEVICE, qoc.QOC_ERR_INVALID_ARG)
    assert not h.value
