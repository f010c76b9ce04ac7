"""The library's host code (argument validation, workspace layouts and their
size arithmetic) built with AddressSanitizer and UndefinedBehaviorSanitizer
and driven by tests/host_checks/harness.cpp without a GPU: every case either
needs no device or must be refused before the device is touched.  The device
code is compiled as usual; the sanitizers instrument the host side only."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2602_14683_amd", "csrc")
HARNESS = os.path.join(ROOT, "tests", "host_checks", "harness.cpp")
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")
HIPCC = shutil.which("hipcc") or os.path.join(ROCM, "bin", "hipcc")
CLANG = os.path.join(ROCM, "llvm", "bin", "clang++")
SAN = ["-Xarch_host", "-fsanitize=address,undefined", "-Xarch_host", "-fno-sanitize-recover=undefined",
       "-Xarch_host", "-fno-omit-frame-pointer", "-Xarch_host", "-g"]


def _sources():
    from paper_2602_14683_amd import build
    return build.SOURCES


@pytest.mark.skipif(not (os.path.exists(HIPCC) and os.path.exists(CLANG)), reason="hipcc / ROCm clang not found")
def test_host_code_under_asan_and_ubsan(tmp_path):
    import concurrent.futures
    objs = []

    def compile_one(k_src):
        k, src = k_src
        obj = str(tmp_path / f"o{k}.o")
        lang = ["-x", "hip"] if src.endswith(".cpp") else []
        cmd = [HIPCC, "-O1", "-std=c++17", "-fPIC", "--offload-arch=gfx950", "-Xclang", "-target-feature",
               "-Xclang", "-packed-fp32-ops", "-I", CSRC] + SAN + lang + ["-c", os.path.join(CSRC, src), "-o", obj]
        res = subprocess.run(cmd, capture_output=True, text=True)
        assert res.returncode == 0, res.stderr[-3000:]
        return obj

    with concurrent.futures.ThreadPoolExecutor(min(8, os.cpu_count() or 1)) as ex:
        objs = list(ex.map(compile_one, enumerate(_sources())))
    hobj = str(tmp_path / "harness.o")
    res = subprocess.run([CLANG, "-O1", "-g", "-std=c++17", "-fsanitize=address,undefined",
                          "-fno-sanitize-recover=undefined", "-I", os.path.join(ROOT, "include"),
                          "-I", os.path.join(ROCM, "include"), "-D__HIP_PLATFORM_AMD__", "-c", HARNESS, "-o", hobj],
                         capture_output=True, text=True)
    assert res.returncode == 0, res.stderr[-3000:]
    exe = str(tmp_path / "harness")
    res = subprocess.run([CLANG, "-fsanitize=address,undefined", "-o", exe, hobj] + objs +
                         ["-L", os.path.join(ROCM, "lib"), "-lamdhip64", "-lrocprofiler-sdk-roctx",
                          "-Wl,-rpath," + os.path.join(ROCM, "lib")],
                         capture_output=True, text=True)
    assert res.returncode == 0, res.stderr[-3000:]
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1",
               HIP_VISIBLE_DEVICES=os.environ.get("HIP_VISIBLE_DEVICES", ""))
    res = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=300)
    assert res.returncode == 0, (res.stdout[-2000:], res.stderr[-4000:])
    assert "runtime error" not in res.stderr and "AddressSanitizer" not in res.stderr, res.stderr[-4000:]
    assert "host checks passed" in res.stdout
