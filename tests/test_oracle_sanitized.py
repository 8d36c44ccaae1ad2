"""The oracle's pins under AddressSanitizer and UndefinedBehaviorSanitizer:
the oracle library is rebuilt with -fsanitize=address,undefined and the pins
run against it in a child process with the sanitizer runtime preloaded.  Any
out-of-bounds access, use after free or undefined behaviour in the oracle
aborts the child (no CPU time is spent here on the slow pins)."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _runtime(name):
    try:
        p = subprocess.run(["gcc", f"-print-file-name={name}"], capture_output=True, text=True, check=True)
    except (OSError, subprocess.CalledProcessError):
        return None
    path = p.stdout.strip()
    return path if os.path.isabs(path) and os.path.exists(path) else None


@pytest.mark.slow
def test_oracle_pins_under_asan_and_ubsan(tmp_path):
    asan = _runtime("libasan.so")
    if asan is None:
        pytest.skip("no gcc AddressSanitizer runtime")
    sys.path.insert(0, ROOT)
    from oracle import build as B
    lib = B.build(out=str(tmp_path / "liboracle_san.so"), sanitize=True)
    env = dict(os.environ)
    env.update(JFNK_ORACLE_LIB=lib, LD_PRELOAD=asan,
               ASAN_OPTIONS="detect_leaks=0:abort_on_error=1:halt_on_error=1",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    p = subprocess.run([sys.executable, "-m", "pytest", "-q", "-x", "-p", "no:cacheprovider",
                        os.path.join(ROOT, "tests", "test_oracle_pins.py"), "-m", "not slow"],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    out = p.stdout + p.stderr
    assert "AddressSanitizer" not in out and "runtime error" not in out, out[-4000:]
    assert p.returncode == 0, out[-4000:]
    assert " passed" in out
