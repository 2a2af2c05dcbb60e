"""The host C++ of the library (transcription, symbolic analysis, C ABI) built
with AddressSanitizer and UndefinedBehaviorSanitizer and driven through its
host paths and error paths by a small C program, against a device layer that
reports no device (tests/sanitize/).  Runs without a GPU."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2606_04725_amd", "csrc")
HERE = os.path.join(ROOT, "tests", "sanitize")
CLANG = "/opt/rocm/llvm/bin/clang++"
CLANG_C = "/opt/rocm/llvm/bin/clang"
FLAGS = ["-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined", "-fno-sanitize-recover=all"]


@pytest.mark.skipif(not (os.path.exists(CLANG) and os.path.exists(CLANG_C)), reason="ROCm clang not installed")
def test_host_code_under_sanitizers(tmp_path):
    objs = []
    inc = [f"-I{os.path.join(ROOT, 'include')}", "-I/opt/rocm/include", "-D__HIP_PLATFORM_AMD__"]
    for src in ("family.cpp", "symbolic.cpp", "capi.cpp", os.path.join(HERE, "device_stub.cpp")):
        path = src if os.path.isabs(src) else os.path.join(CSRC, src)
        obj = str(tmp_path / (os.path.basename(src) + ".o"))
        subprocess.run([CLANG, "-std=c++17", *FLAGS, *inc, "-c", path, "-o", obj], check=True)
        objs.append(obj)
    drv = str(tmp_path / "driver.o")
    subprocess.run([CLANG_C, "-std=c11", *FLAGS, *inc, "-c", os.path.join(HERE, "driver.c"), "-o", drv], check=True)
    exe = str(tmp_path / "sanitize_driver")
    subprocess.run([CLANG, *FLAGS, drv, *objs, "-o", exe, "-lm"], check=True)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0:exitcode=23",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=600)
    print(r.stdout)
    assert r.returncode == 0, r.stderr[-4000:]
    assert "sanitize: ok" in r.stdout
