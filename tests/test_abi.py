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


def test_struct_layouts_match_header(tmp_path):
    """Every field offset and the size of gp_config and gp_diag, as a C
    compiler lays them out from the header, equal the binding's."""
    from paper_1311_0861_amd import gpupegas as gp
    prog = ['#include <stddef.h>', '#include <stdio.h>', '#include "gpupegas.h"', "int main(void) {"]
    for st in (gp.gp_config, gp.gp_diag):
        cname = st.__name__
        prog.append('  printf("%s size %%zu\\n", sizeof(%s));' % (cname, cname))
        for name, _ in st._fields_:
            prog.append('  printf("%s %s %%zu\\n", offsetof(%s, %s));' % (cname, name, cname, name))
    prog += ["  return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(prog) + "\n")
    exe = tmp_path / "layout"
    subprocess.check_call(["gcc", "-std=c99", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)])
    got = {}
    for line in subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.splitlines():
        a, b, v = line.split()
        got[(a, b)] = int(v)
    for st in (gp.gp_config, gp.gp_diag):
        cname = st.__name__
        assert got[(cname, "size")] == ctypes.sizeof(st), cname
        for name, _ in st._fields_:
            assert got[(cname, name)] == getattr(st, name).offset, (cname, name)
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


def test_create_failure_reason_without_gpu():
    """A refused configuration is rejected before any HIP call, and
    gp_last_error(NULL) then says why the calling thread's create failed."""
    from paper_1311_0861_amd import gpupegas as gp
    cfg = {"n": (16, 16, 16), "lo": (-1.0,) * 3, "hi": (1.0,) * 3, "gamma": 0.5}
    with pytest.raises(gp.GpError, match="invalid configuration"):
        gp.gp_create(cfg)
    assert b"invalid configuration" in gp.lib.gp_last_error(None)
    with pytest.raises(gp.GpError, match="run 1: invalid configuration"):
        gp.gp_batch_create([dict(cfg, gamma=5.0 / 3.0), cfg])
    assert gp.lib.gp_batch_last_error(None).startswith(b"run 1")


def test_binding_shares_one_hip_runtime_with_torch():
    """Importing the binding before torch still leaves a single HIP runtime
    mapped in the process (two runtimes each claim the device)."""
    code = ("import sys; sys.path.insert(0, %r)\n"
            "from paper_1311_0861_amd import gpupegas\n"
            "import torch\n"
            "maps = open('/proc/self/maps').read().split()\n"
            "print(sorted({m for m in maps if 'libamdhip64' in m}))\n") % ROOT
    out = subprocess.run(["python", "-c", code], capture_output=True, text=True, timeout=300)
    assert out.returncode == 0, out.stderr
    libs = eval(out.stdout.strip().splitlines()[-1])
    assert len(libs) == 1, libs


def test_product_package_does_not_touch_oracle():
    """The GPU path never imports or links the oracle."""
    pkg = os.path.join(ROOT, "paper_1311_0861_amd")
    for dirpath, _, files in os.walk(pkg):
        for fn in files:
            if fn.endswith((".py", ".hip", ".hpp", ".h", ".cpp")):
                text = open(os.path.join(dirpath, fn)).read()
                for pat in ("import oracle", "from oracle", "liboracle", "orc_"):
                    assert pat not in text, (fn, pat)
