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


def _device_disassembly():
    """Disassembly of every gfx950 code object in the built library (each translation unit's
    offload bundle in the .hip_fatbin section)."""
    import subprocess
    import tempfile

    llvm = "/opt/rocm/llvm/bin"
    for tool in ("clang-offload-bundler", "llvm-objdump"):
        if not os.path.exists(os.path.join(llvm, tool)):
            pytest.skip(f"{tool} not available")
    with tempfile.TemporaryDirectory() as tmp:
        fat = os.path.join(tmp, "fatbin")
        # with no output operand objcopy would rewrite the library in place (under a process that
        # may have it mapped); write its copy to a scratch file instead
        subprocess.run(["objcopy", "--dump-section", f".hip_fatbin={fat}", qoc.LIB_PATH,
                        os.path.join(tmp, "copy.so")], check=True)
        data = open(fat, "rb").read()
        magic = b"__CLANG_OFFLOAD_BUNDLE__"
        starts = [m.start() for m in re.finditer(re.escape(magic), data)]
        assert starts, "no offload bundle in the library"
        text = []
        for k, a in enumerate(starts):
            b = starts[k + 1] if k + 1 < len(starts) else len(data)
            part = os.path.join(tmp, f"b{k}")
            elf = os.path.join(tmp, f"c{k}.elf")
            open(part, "wb").write(data[a:b])
            subprocess.run([os.path.join(llvm, "clang-offload-bundler"), "--unbundle", "--type=o", f"--input={part}",
                            "--targets=hipv4-amdgcn-amd-amdhsa--gfx950", f"--output={elf}"], check=True)
            out = subprocess.run([os.path.join(llvm, "llvm-objdump"), "-d", "--mcpu=gfx950", elf],
                                 check=True, capture_output=True, text=True).stdout
            text.append(out)
        return text


def test_device_code_has_no_packed_fp32_arithmetic():
    """The library is built with the packed-FP32 target feature off for the device pass: no
    v_pk_add_f32 / v_pk_mul_f32 / v_pk_fma_f32 anywhere in its gfx950 code."""
    texts = _device_disassembly()
    assert sum(t.count("\n") for t in texts) > 10000
    for t in texts:
        for op in ("v_pk_add_f32", "v_pk_mul_f32", "v_pk_fma_f32"):
            assert op not in t, op
