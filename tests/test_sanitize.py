"""CPU sanitizer builds: the oracle (oracle/sco.c) and the host code of the C ABI
(paper_2410_21207_amd/csrc/sc_api.cpp: validation, workspace layouts, the batch planner) built
with AddressSanitizer and UndefinedBehaviorSanitizer (g++/gcc, host code only; the kernel
launchers are replaced by stand-ins that report an error), then run over many shapes and
argument errors.  A sanitizer finding aborts the program and fails the test."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HERE = os.path.join(ROOT, "tests", "sanitize")
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")
SAN = ["-O1", "-g", "-fsanitize=address,undefined", "-fno-omit-frame-pointer", "-fno-sanitize-recover=undefined"]


def _run(exe, tmp_path, leaks):
    env = dict(os.environ, ASAN_OPTIONS=f"detect_leaks={1 if leaks else 0}:abort_on_error=0",
               UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([exe], capture_output=True, text=True, timeout=600, env=env, cwd=tmp_path)
    out = r.stdout + r.stderr
    assert r.returncode == 0, out[-4000:]
    assert "runtime error" not in out and "AddressSanitizer" not in out, out[-4000:]
    return out


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc missing")
def test_oracle_under_sanitizers(tmp_path):
    exe = str(tmp_path / "oracle_asan")
    subprocess.run(["gcc", "-std=c99"] + SAN + [os.path.join(ROOT, "oracle", "sco.c"),
                                                os.path.join(HERE, "oracle_driver.c"), "-o", exe],
                   check=True, capture_output=True, text=True)
    assert "all expectations held" in _run(exe, tmp_path, leaks=True)


@pytest.mark.skipif(shutil.which("g++") is None or not os.path.exists(os.path.join(ROCM, "lib", "libamdhip64.so")),
                    reason="g++ or the HIP runtime missing")
def test_abi_host_code_under_sanitizers(tmp_path):
    exe = str(tmp_path / "api_asan")
    csrc = os.path.join(ROOT, "paper_2410_21207_amd", "csrc")
    r = subprocess.run(["g++", "-std=c++17"] + SAN +
                       ["-D__HIP_PLATFORM_AMD__", "-I", os.path.join(ROCM, "include"), "-I", os.path.join(ROOT, "include"),
                        "-I", csrc, os.path.join(csrc, "sc_api.cpp"), os.path.join(HERE, "kernel_stubs.cpp"),
                        os.path.join(HERE, "api_driver.cpp"), "-L", os.path.join(ROCM, "lib"), "-lamdhip64",
                        "-Wl,-rpath," + os.path.join(ROCM, "lib"), "-o", exe], capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-4000:]
    # the HIP runtime's own allocations are not ours to check for leaks
    assert "all expectations held" in _run(exe, tmp_path, leaks=False)
