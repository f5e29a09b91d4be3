"""The oracle under AddressSanitizer and UndefinedBehaviorSanitizer (CPU):
every function of oasm_oracle.c driven on seeded random inputs with exact-size
buffers and capacities below the counts (oracle/sanitize_driver.c)."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_oracle_clean_under_asan_ubsan(tmp_path):
    if shutil.which("gcc") is None:
        pytest.skip("no C compiler")
    exe = tmp_path / "oracle_asan"
    src = [os.path.join(ROOT, "oracle", f) for f in ("oasm_oracle.c", "sanitize_driver.c")]
    build = subprocess.run(["gcc", "-std=c99", "-O1", "-g", "-fsanitize=address,undefined",
                            "-fno-sanitize-recover=all", "-fno-omit-frame-pointer", *src, "-o", str(exe)],
                           capture_output=True, text=True)
    if build.returncode != 0 and "sanitize" in build.stderr:
        pytest.skip("sanitizer runtime not available: " + build.stderr[-200:])
    assert build.returncode == 0, build.stderr
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")
    res = subprocess.run([str(exe), "600"], capture_output=True, text=True, env=env, timeout=300)
    assert res.returncode == 0, res.stdout[-2000:] + res.stderr[-4000:]
    assert "600 cases ok" in res.stdout
