"""Host AddressSanitizer and UndefinedBehaviorSanitizer run (CPU only): the
host-side grid builder and C-ABI glue of libsgcm (grid.cpp, capi.cpp; the
device-table hooks stubbed out) and the oracle are built with
-fsanitize=address,undefined and driven through small cases and invalid
arguments by tests/asan_driver.py in a subprocess with the sanitizer runtime
preloaded; any report fails the test."""
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1507_04769_amd", "csrc")
SAN = ["-fsanitize=address,undefined", "-fno-omit-frame-pointer", "-fno-sanitize-recover=undefined"]

STUB = """#include "sgcm_internal.h"
namespace sgcm {
void free_device_tables(Grid&) {}
int upload_device_tables(Grid&, int, void*) { return SGCM_EUNSUPPORTED; }
}
"""


@pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")
def test_host_paths_under_address_sanitizer(tmp_path):
    stub = tmp_path / "stub.cpp"
    stub.write_text(STUB)
    glue = tmp_path / "libsgcm_host_asan.so"
    orc = tmp_path / "liboracle_asan.so"
    subprocess.check_call(["g++", "-std=c++17", "-O1", "-g", "-shared", "-fPIC"] + SAN +
                          ["-I" + os.path.join(ROOT, "include"), "-I" + CSRC, os.path.join(CSRC, "capi.cpp"),
                           os.path.join(CSRC, "grid.cpp"), str(stub), "-o", str(glue)])
    subprocess.check_call(["g++", "-std=c++17", "-O1", "-g", "-fopenmp", "-shared", "-fPIC"] + SAN +
                          [os.path.join(ROOT, "oracle", "sgcm_oracle.cpp"), "-o", str(orc)])
    runtime = subprocess.run(["g++", "-print-file-name=libasan.so"], capture_output=True, text=True).stdout.strip()
    env = dict(os.environ, LD_PRELOAD=runtime, SGCM_ORACLE_LIB=str(orc), OMP_NUM_THREADS="2",
               ASAN_OPTIONS="detect_leaks=0:abort_on_error=1", UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([sys.executable, os.path.join(ROOT, "tests", "asan_driver.py"), str(glue)],
                       capture_output=True, text=True, env=env, timeout=600)
    report = r.stderr[-4000:]
    assert r.returncode == 0, report
    assert "asan ok" in r.stdout
    assert "AddressSanitizer" not in r.stderr and "runtime error" not in r.stderr, report
