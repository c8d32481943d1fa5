"""CPU sanitizer builds (AddressSanitizer + UndefinedBehaviorSanitizer, host code only):
the oracle driven through every entry point by tests/native/oracle_sanitize.c, and libspvar's
host code (device code built unoptimised, only the host side instrumented) driven through its
table arithmetic, sample split, R99 and pre-device argument checks by
tests/native/library_host_checks.cpp.  No GPU is used."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
NATIVE = os.path.join(ROOT, "tests", "native")
CSRC = os.path.join(ROOT, "paper_1706_07826_amd", "csrc")
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer"]


def _run(cmd, env=None, timeout=600):
    p = subprocess.run(cmd, capture_output=True, text=True, env=env, timeout=timeout)
    assert p.returncode == 0, f"{' '.join(cmd)}\n{p.stdout[-2000:]}\n{p.stderr[-4000:]}"
    return p


def test_oracle_under_address_and_undefined_sanitizers(tmp_path):
    exe = str(tmp_path / "oracle_asan")
    _run(["gcc", "-O1", "-g", "-std=c99", "-fopenmp", *SAN, "-o", exe, os.path.join(NATIVE, "oracle_sanitize.c"),
          "-lm"])
    p = _run([exe], env=dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=1"))
    assert "all checks passed" in p.stdout


@pytest.mark.slow
def test_library_host_code_under_address_and_undefined_sanitizers(tmp_path):
    hipcc = shutil.which("hipcc")
    clangxx = "/opt/rocm/llvm/bin/clang++"
    if not hipcc or not os.path.exists(clangxx):
        pytest.skip("hipcc / ROCm clang++ not installed")
    lib = str(tmp_path / "libspvar_hostasan.so")
    srcs = sorted(os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith((".hip", ".cpp")))
    # sanitizers on the host side only (-Xarch_host before each); device code built at -O0
    _run([hipcc, "--offload-arch=gfx950", "-O1", "-Xarch_device", "-O0", "-std=c++17", "-fPIC", "-shared",
          "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
          "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
          "-I", os.path.join(ROOT, "include"), "-I", CSRC, "-o", lib, *srcs], timeout=900)
    obj = str(tmp_path / "oracle_asan.o")
    _run(["gcc", "-c", "-O1", "-g", "-std=c99", "-fPIC", "-fopenmp", *SAN, "-o", obj,
          os.path.join(ROOT, "oracle", "spvar_oracle.c")])
    exe = str(tmp_path / "host_checks")
    _run([clangxx, "-O1", "-g", "-std=c++17", *SAN, "-D__HIP_PLATFORM_AMD__", "-I", os.path.join(ROOT, "include"),
          "-I", "/opt/rocm/include", "-o", exe, os.path.join(NATIVE, "library_host_checks.cpp"), obj,
          "-L", str(tmp_path), "-lspvar_hostasan", f"-Wl,-rpath,{tmp_path}", "-lm", "-fopenmp"])
    p = _run([exe], env=dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=1"))
    assert "all passed" in p.stdout
