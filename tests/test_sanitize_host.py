"""AddressSanitizer + UndefinedBehaviorSanitizer builds of the CPU code: the
FP64 oracle (every entry point, orthorhombic and triclinic cells, variable and
self radii, a sampled subset, the masked stencil and CG) and the plan-time
host code of the library (sphere-class tables in both layouts, the NK arms,
the moment tables, the plane-sweep tables), each driven by a small program
under tests/native that also checks the tables' index invariants.  Host code
only: built with gcc/g++, no GPU code involved."""
import os
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
NATIVE = os.path.join(ROOT, "tests", "native")
CSRC = os.path.join(ROOT, "paper_2011_07209_amd", "csrc")
SAN = ["-O1", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer"]
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")


def _sanitizers_available(tmp_path):
    src = tmp_path / "probe.c"
    src.write_text("int main(void){return 0;}\n")
    r = subprocess.run(["gcc", *SAN, str(src), "-o", str(tmp_path / "probe")], capture_output=True)
    return r.returncode == 0


def _run(exe):
    r = subprocess.run([str(exe)], capture_output=True, text=True, env=ENV, timeout=300)
    print(r.stdout[-4000:])
    print(r.stderr[-8000:])
    assert r.returncode == 0, "sanitized run failed"
    assert "ERROR: AddressSanitizer" not in r.stderr and "runtime error" not in r.stderr
    assert r.stdout.strip().endswith("failures 0")


def test_oracle_under_sanitizers(tmp_path):
    if not _sanitizers_available(tmp_path):
        pytest.skip("gcc without ASan/UBSan runtime")
    exe = tmp_path / "oracle_san"
    subprocess.run(["gcc", "-std=c11", "-fopenmp", *SAN, "-Wall", "-o", str(exe),
                    os.path.join(NATIVE, "oracle_sanitize_main.c"), "-lm"], check=True)
    _run(exe)


def test_host_plan_code_under_sanitizers(tmp_path):
    if not _sanitizers_available(tmp_path):
        pytest.skip("gcc without ASan/UBSan runtime")
    if not os.path.exists("/opt/rocm/include/hip/hip_runtime.h"):
        pytest.skip("HIP headers not installed")
    exe = tmp_path / "host_san"
    subprocess.run(["g++", "-std=c++17", *SAN, "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include",
                    "-I", os.path.join(ROOT, "include"), "-I", CSRC, "-o", str(exe),
                    os.path.join(NATIVE, "host_plan_sanitize_main.cpp"), os.path.join(CSRC, "plan_geometry.cpp"),
                    os.path.join(CSRC, "nk_stencil.cpp")], check=True)
    _run(exe)
