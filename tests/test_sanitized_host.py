"""The host code under AddressSanitizer and UndefinedBehaviorSanitizer.

Builds, into a temporary directory, the FP64 oracle (oracle/gsr_oracle.c)
and the host half of the library (gsr_api.cpp: plan creation, argument
validation and workspace layout; gsr_partition.cpp: the host KD-tree
partition), both with -fsanitize=address,undefined, the device launchers
replaced by stand-ins that report no device (tests/sanitize/host_stubs.cpp).
Then runs the CPU tests of those parts in a child process against these
builds (GSR_LIBRARY / GSR_ORACLE_LIBRARY), with the sanitizer runtime
preloaded and any report fatal."""
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2510_01767_amd", "csrc")
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")
SAN = ["-fsanitize=address,undefined", "-fno-omit-frame-pointer", "-fno-sanitize-recover=undefined", "-g", "-O1"]
# CPU tests of the sanitized parts (the export test and the bench tests need the full library)
SUITES = ["tests/test_abi_host.py", "tests/test_partition.py", "tests/test_oracle_pins.py",
          "tests/test_oracle_guard_pins.py", "tests/test_oracle_fcs_pins.py", "tests/test_oracle_densify_pins.py"]


def _have_toolchain():
    return (shutil.which("gcc") and shutil.which("g++") and os.path.exists(os.path.join(ROCM, "include", "hip"))
            and os.path.exists(os.path.join(ROCM, "lib", "libamdhip64.so")))


@pytest.mark.slow
@pytest.mark.skipif(not _have_toolchain(), reason="needs gcc/g++ and the ROCm host runtime")
def test_host_code_is_clean_under_asan_and_ubsan(tmp_path):
    inc = ["-I", os.path.join(ROOT, "include"), "-I", CSRC, "-I", os.path.join(ROCM, "include")]
    oracle_so = str(tmp_path / "libgsr_oracle_san.so")
    subprocess.check_call(["gcc", "-std=c11", "-fopenmp", "-fPIC", "-shared", *SAN, "-o", oracle_so,
                           os.path.join(ROOT, "oracle", "gsr_oracle.c"), "-lm"])
    objs = []
    for src in (os.path.join(CSRC, "gsr_api.cpp"), os.path.join(CSRC, "gsr_partition.cpp"),
                os.path.join(ROOT, "tests", "sanitize", "host_stubs.cpp")):
        obj = str(tmp_path / (os.path.basename(src) + ".o"))
        subprocess.check_call(["g++", "-std=c++17", "-D__HIP_PLATFORM_AMD__", "-fPIC", *SAN, *inc, "-c", src,
                               "-o", obj])
        objs.append(obj)
    lib_so = str(tmp_path / "libgsr_host_san.so")
    subprocess.check_call(["g++", "-shared", *SAN, "-o", lib_so, *objs, "-L", os.path.join(ROCM, "lib"),
                           "-lamdhip64", "-Wl,-rpath," + os.path.join(ROCM, "lib")])
    asan_rt = subprocess.check_output(["gcc", "-print-file-name=libasan.so"], text=True).strip()
    ubsan_rt = subprocess.check_output(["gcc", "-print-file-name=libubsan.so"], text=True).strip()
    env = dict(os.environ)
    env.update(GSR_LIBRARY=lib_so, GSR_ORACLE_LIBRARY=oracle_so, LD_PRELOAD=f"{asan_rt}:{ubsan_rt}",
               ASAN_OPTIONS="detect_leaks=0:abort_on_error=1:halt_on_error=1",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1", OMP_NUM_THREADS="2",
               HIP_VISIBLE_DEVICES="", CUDA_VISIBLE_DEVICES="")
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-x", "-p", "no:cacheprovider", "-m", "not gpu",
                        "-k", "not every_declared_function and not bench", *SUITES],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=900)
    out = r.stdout[-4000:] + r.stderr[-4000:]
    assert r.returncode == 0, out
    assert "ERROR: AddressSanitizer" not in out and "runtime error:" not in out, out
    assert " passed" in r.stdout, out
