"""The C ABI from plain C: tests/c/abi_consumer.c includes only include/*.h and the
HIP runtime header, links libdnb.so and libamdhip64, and exercises the library
without Python or torch.  Compiled on the CPU (the headers are valid C11);
compiled and run on the GPU."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "tests", "c", "abi_consumer.c")
PKG = os.path.join(ROOT, "paper_2511_22468_amd")
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")


def build(out):
    if shutil.which("gcc") is None or not os.path.exists(os.path.join(PKG, "libdnb.so")):
        pytest.skip("gcc or libdnb.so missing")
    cmd = ["gcc", "-std=c11", "-Wall", "-Wextra", "-Werror", "-D__HIP_PLATFORM_AMD__",
           f"-I{ROCM}/include", f"-I{ROOT}/include", SRC, f"-L{PKG}", "-ldnb", f"-L{ROCM}/lib",
           "-lamdhip64", f"-Wl,-rpath,{PKG}", f"-Wl,-rpath,{ROCM}/lib", "-lm", "-o", out]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    return out


def test_headers_compile_as_c(tmp_path):
    build(str(tmp_path / "abi_consumer"))


@pytest.mark.gpu
def test_c_program_runs_on_the_gpu(tmp_path):
    exe = build(str(tmp_path / "abi_consumer"))
    r = subprocess.run([exe], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "abi consumer ok" in r.stdout
