"""The C-ABI library loads on any machine and exports every function that
include/gpupegas.h declares; the struct layouts of the binding match the
header.  No compute call is made (CPU only)."""
import ctypes
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "gpupegas.h")
LIB = os.path.join(ROOT, "paper_1311_0861_amd", "libgpupegas.so")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(gp_[a-z_0-9]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        from paper_1311_0861_amd import build
        build.build()
    return ctypes.CDLL(LIB)


def test_library_exports_every_declared_function(lib):
    names = declared_functions()
    assert len(names) >= 15, names
    for n in names:
        assert hasattr(lib, n), n
    out = subprocess.run(["nm", "-D", "--defined-only", LIB], capture_output=True, text=True).stdout
    exported = set(re.findall(r"\bT (gp_\w+)", out))
    assert set(names) <= exported, set(names) - exported


def test_status_strings_without_gpu(lib):
    lib.gp_status_str.restype = ctypes.c_char_p
    lib.gp_status_str.argtypes = [ctypes.c_int32]
    assert lib.gp_status_str(0) == b"ok"
    assert b"order" in lib.gp_status_str(-7)


def test_struct_layouts_match_header():
    from paper_1311_0861_amd import gpupegas as gp
    # gp_config: 6 int32 + 6 double + 6 double + 2 int32 = 24 + 96 + 8
    assert ctypes.sizeof(gp.gp_config) == 128
    assert gp.gp_config.lo.offset == 24 and gp.gp_config.precision.offset == 120
    # gp_diag: int64 + 16 doubles + 2 uint32
    assert ctypes.sizeof(gp.gp_diag) == 8 + 16 * 8 + 8
    assert gp.gp_diag.err.offset == 136
    src = open(os.path.join(ROOT, "paper_1311_0861_amd", "csrc", "common.hpp")).read()
    assert "kDiagCap = 4096" in src


def test_null_and_bad_arguments_rejected(lib):
    lib.gp_create.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]
    lib.gp_create.restype = ctypes.c_int32
    assert lib.gp_create(None, None, None) == -1
    lib.gp_step.argtypes = [ctypes.c_void_p, ctypes.c_int32]
    lib.gp_step.restype = ctypes.c_int32
    assert lib.gp_step(None, 1) == -1
    lib.gp_destroy.argtypes = [ctypes.c_void_p]
    lib.gp_destroy.restype = ctypes.c_int32
    assert lib.gp_destroy(None) == -1


def test_product_package_does_not_touch_oracle():
    """The GPU path never imports or links the oracle."""
    pkg = os.path.join(ROOT, "paper_1311_0861_amd")
    for dirpath, _, files in os.walk(pkg):
        for fn in files:
            if fn.endswith((".py", ".hip", ".hpp", ".h", ".cpp")):
                text = open(os.path.join(dirpath, fn)).read()
                for pat in ("import oracle", "from oracle", "liboracle", "orc_"):
                    assert pat not in text, (fn, pat)
