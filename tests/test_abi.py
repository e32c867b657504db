"""CPU checks of the C-ABI library: it loads, exports every function that
include/qdcb.h declares, reports its ABI version, and shares no code with
the oracle (no compute call needs a GPU here)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HDR = os.path.join(ROOT, "include", "qdcb.h")
LIB = os.path.join(ROOT, "paper_2606_04316_amd", "libqdcb.so")


def declared_functions():
    src = open(HDR).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(qdcb_[a-z_]+)\s*\(", src)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        from paper_2606_04316_amd import build
        build.build()
    return ctypes.CDLL(LIB)


def test_every_declared_symbol_is_exported(lib):
    names = declared_functions()
    assert len(names) >= 12
    for n in names:
        assert hasattr(lib, n), n


def test_abi_version_and_error_string(lib):
    lib.qdcb_abi_version.restype = ctypes.c_int
    assert lib.qdcb_abi_version() == 1
    lib.qdcb_last_error.restype = ctypes.c_char_p
    assert isinstance(lib.qdcb_last_error(), bytes)  # "" until a call on this thread fails


def test_null_arguments_are_rejected_without_a_device(lib):
    # argument validation happens before any device call
    assert lib.qdcb_basis_schwarz(None, None) == -1
    assert lib.qdcb_plan_footprint(None, None) == -1
    lib.qdcb_last_error.restype = ctypes.c_char_p
    assert b"NULL" in lib.qdcb_last_error()


def test_oracle_and_gpu_path_share_no_code():
    csrc = os.path.join(ROOT, "paper_2606_04316_amd", "csrc")
    for f in os.listdir(csrc):
        txt = open(os.path.join(csrc, f)).read()
        assert "oracle" not in txt.lower(), f
    for f in ("qdcb.py", "build.py", "__init__.py"):
        txt = open(os.path.join(ROOT, "paper_2606_04316_amd", f)).read()
        assert "import oracle" not in txt and "from oracle" not in txt, f
    for f in os.listdir(os.path.join(ROOT, "oracle")):
        if f.endswith((".c", ".h", ".py")):
            txt = open(os.path.join(ROOT, "oracle", f)).read()
            assert "qdcb" not in txt.replace("QDCB_ORACLE_H", ""), f
            assert "paper_2606_04316_amd" not in txt, f
