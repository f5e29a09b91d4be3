"""The host-side result conversion (paper_1712_03560_amd/csrc/oasm_hostpar.h)
split over threads, on the CPU: under ThreadSanitizer (no data race between
the conversion threads) and under AddressSanitizer/UBSan, each conversion
equal record for record to a serial one (tests/native/hostpar_tsan_driver.cpp)."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "tests", "native", "hostpar_tsan_driver.cpp")
INC = ["-I", os.path.join(ROOT, "include"), "-I", os.path.join(ROOT, "paper_1712_03560_amd", "csrc")]


@pytest.mark.parametrize("san", ["thread", "address,undefined"])
def test_conversion_threads_clean(tmp_path, san):
    if shutil.which("g++") is None:
        pytest.skip("no C++ compiler")
    exe = tmp_path / "hostpar"
    build = subprocess.run(["g++", "-std=c++17", "-O1", "-g", f"-fsanitize={san}", "-fno-sanitize-recover=all",
                            "-fno-omit-frame-pointer", "-pthread", *INC, SRC, "-o", str(exe)],
                           capture_output=True, text=True)
    if build.returncode != 0 and "sanitize" in build.stderr:
        pytest.skip("sanitizer runtime not available: " + build.stderr[-200:])
    assert build.returncode == 0, build.stderr
    env = dict(os.environ, TSAN_OPTIONS="halt_on_error=1", ASAN_OPTIONS="detect_leaks=1",
               UBSAN_OPTIONS="print_stacktrace=1")
    res = subprocess.run([str(exe)], capture_output=True, text=True, env=env, timeout=300)
    assert res.returncode == 0, res.stdout[-2000:] + res.stderr[-4000:]
    assert "ok (0 mismatches)" in res.stdout
