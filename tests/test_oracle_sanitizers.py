"""The oracle built with AddressSanitizer and UndefinedBehaviorSanitizer
(errors fatal) runs its pins cleanly: no out-of-bounds access, use after
free or undefined arithmetic in the checker itself."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.slow
def test_oracle_pins_under_address_and_undefined_sanitizers(tmp_path):
    asan = subprocess.run(["g++", "-print-file-name=libasan.so"], capture_output=True, text=True).stdout.strip()
    ubsan = subprocess.run(["g++", "-print-file-name=libubsan.so"], capture_output=True, text=True).stdout.strip()
    if not os.path.isabs(asan) or not os.path.exists(asan):
        pytest.skip("libasan is not available to g++")
    lib = tmp_path / "liboracle_san.so"
    subprocess.run(["g++", "-O1", "-g", "-std=c++17", "-fopenmp", "-fPIC", "-shared", "-ffp-contract=off",
                    "-fno-omit-frame-pointer", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
                    "-o", str(lib), os.path.join(ROOT, "oracle", "gesr_oracle.cpp")], check=True)
    env = dict(os.environ, GESR_ORACLE_LIB=str(lib), LD_PRELOAD=" ".join(p for p in (asan, ubsan) if p),
               ASAN_OPTIONS="detect_leaks=0:abort_on_error=1", UBSAN_OPTIONS="print_stacktrace=1",
               OMP_NUM_THREADS="4")
    tests = [os.path.join(ROOT, "tests", f) for f in
             ("test_oracle_pins.py", "test_oracle_fd.py", "test_oracle_channels.py", "test_parity_model.py")]
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-x", "-p", "no:cacheprovider", "-m", "not slow",
                        *tests], cwd=ROOT, env=env, capture_output=True, text=True, timeout=1800)
    tail = (r.stdout + r.stderr)[-3000:]
    assert r.returncode == 0, tail
    assert "ERROR: AddressSanitizer" not in r.stderr and "runtime error" not in r.stderr, tail
