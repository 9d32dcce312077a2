"""The library's host code (argument validation, sizes, the stability limit,
layouts, teardown: everything the C ABI does without a GPU) built with
AddressSanitizer and UndefinedBehaviorSanitizer on the host side only, and
driven by the plain C program of tests/c/abi_host.c.  The device code is the
ordinary build's."""
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PKG = os.path.join(ROOT, "paper_2404_01035_amd")
OBJ = os.path.join(ROOT, "_build", "obj")
CLANG = "/opt/rocm/llvm/bin/clang"

sys.path.insert(0, ROOT)


def _objects():
    from paper_2404_01035_amd import build

    objs = []
    for src in build.sources():
        if os.path.basename(src) == "api.cpp":
            continue
        o = os.path.join(OBJ, os.path.basename(src) + ".o")
        if not os.path.exists(o) or os.path.getmtime(o) < os.path.getmtime(src):
            return None
        objs.append(o)
    return objs


@pytest.mark.skipif(not os.path.exists(CLANG), reason="no ROCm clang")
def test_host_code_is_clean_under_asan_and_ubsan(tmp_path):
    from paper_2404_01035_amd import build

    objs = _objects()
    if objs is None:
        pytest.skip("the library's objects are not built (run the build first)")
    san = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
           "-Xarch_host", "-fno-sanitize-recover=undefined", "-Xarch_host", "-fno-omit-frame-pointer"]
    api_o = tmp_path / "api_san.o"
    flags = [f for f in build.COMMON if f != "-O3"] + ["-O1", "-g"]
    r = subprocess.run([build.HIPCC, *flags, *san, "-c", os.path.join(PKG, "csrc", "api.cpp"), "-o", str(api_o)],
                       capture_output=True, text=True, timeout=600)
    assert r.returncode == 0, r.stderr[-3000:]
    lib = tmp_path / "libmpstep.so"
    r = subprocess.run([build.HIPCC, f"--offload-arch={build.ARCH}", "-shared", "-fPIC", *san, "-o", str(lib),
                        str(api_o), *objs], capture_output=True, text=True, timeout=600)
    assert r.returncode == 0, r.stderr[-3000:]
    exe = tmp_path / "abi_host_san"
    r = subprocess.run([CLANG, "-std=c99", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined",
                        "-I", os.path.join(ROOT, "include"), os.path.join(ROOT, "tests", "c", "abi_host.c"),
                        "-o", str(exe), str(lib), f"-Wl,-rpath,{tmp_path}", "-lm"],
                       capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stderr[-3000:]
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=300, env=env)
    assert r.returncode == 0 and r.stdout.strip() == "ok", (r.returncode, r.stdout, r.stderr[-4000:])
    assert "runtime error" not in r.stderr and "ERROR: AddressSanitizer" not in r.stderr, r.stderr[-4000:]
