"""The library's host-side logic under AddressSanitizer and
UndefinedBehaviorSanitizer, on the CPU.

paper_2511_22468_amd/csrc/host_logic.h holds what the C ABI decides on the host
before any launch: the launch geometry of the pair kernels, the buffer-size
queries, the host-galaxy parameter check and the ring of tape descriptors the
reverse sweeps are checked against.  It includes no HIP, so
tests/c/host_logic_test.cpp builds it with g++ and both sanitizers and runs its
checks; the library links the same header through hipcc.
"""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "tests", "c", "host_logic_test.cpp")
FLAGS = ["-std=c++17", "-O1", "-g", "-Wall", "-Wextra", "-Werror", "-fno-omit-frame-pointer",
         "-fsanitize=address,undefined", "-fno-sanitize-recover=all"]


def compile_and_run(src, exe):
    if shutil.which("g++") is None:
        pytest.skip("g++ missing")
    r = subprocess.run(["g++"] + FLAGS + [f"-I{ROOT}/include", src, "-o", exe],
                       capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
               UBSAN_OPTIONS="print_stacktrace=1")
    return subprocess.run([exe], capture_output=True, text=True, timeout=120, env=env)


def test_host_logic_under_sanitizers(tmp_path):
    r = compile_and_run(SRC, str(tmp_path / "host_logic_test"))
    assert r.returncode == 0, r.stdout + r.stderr
    assert "host logic ok" in r.stdout
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr


def test_the_sanitizer_build_reports_overflow(tmp_path):
    # the same flags turn a signed overflow into a failing run, so a clean run of
    # the host-logic checks means none happened there
    src = tmp_path / "overflow.cpp"
    src.write_text("#include <stdint.h>\n#include <stdlib.h>\n"
                   "int main(int argc, char**) {\n"
                   "    int64_t a = INT64_MAX - 1 + (int64_t)argc;\n"
                   "    volatile int64_t b = a * 9;\n"
                   "    return b == 0 ? 0 : 0;\n}\n")
    r = compile_and_run(str(src), str(tmp_path / "overflow"))
    assert r.returncode != 0
    assert "runtime error" in r.stderr
