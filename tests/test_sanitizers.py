"""The FP64 oracle and the library's host UCT tree under AddressSanitizer
and UndefinedBehaviorSanitizer: a host-only driver (tests/sanitize/
driver.cpp) built with gcc/g++ and the sanitizers, no GPU code, run once.
Any out-of-bounds access, leak, use after free or undefined operation in
either makes the run fail."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer", "-g", "-O1"]


@pytest.mark.skipif(shutil.which("g++") is None or not os.path.isdir("/opt/rocm/include"),
                    reason="needs g++ and the HIP headers")
def test_oracle_and_host_tree_are_clean_under_asan_and_ubsan(tmp_path):
    inc = ["-I", os.path.join(ROOT, "include"), "-I", os.path.join(ROOT, "paper_2207_06649_amd", "csrc"),
           "-I", os.path.join(ROOT, "oracle"), "-I", "/opt/rocm/include", "-D__HIP_PLATFORM_AMD__"]
    oracle_o = str(tmp_path / "oracle.o")
    subprocess.run(["gcc", "-std=c11", "-D_GNU_SOURCE", *SAN, "-c", os.path.join(ROOT, "oracle", "pmbs_oracle.c"),
                    "-o", oracle_o], check=True)
    exe = str(tmp_path / "driver")
    subprocess.run(["g++", "-std=c++17", *SAN, *inc, os.path.join(ROOT, "tests", "sanitize", "driver.cpp"),
                    os.path.join(ROOT, "paper_2207_06649_amd", "csrc", "pmbs_tree.cpp"), oracle_o,
                    "-o", exe, "-lpthread", "-lm"], check=True)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=300)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "ok" in r.stdout
