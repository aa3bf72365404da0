"""The oracle's C++ under AddressSanitizer and UndefinedBehaviorSanitizer: its own pin tests run in
a child process against a sanitized build (oracle/libvxo_san.so, g++ -fsanitize=address,undefined,
no recovery from undefined behaviour), with libasan preloaded into the interpreter."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _runtime(name):
    try:
        p = subprocess.run(["gcc", f"-print-file-name={name}"], capture_output=True, text=True, check=True).stdout
    except (OSError, subprocess.CalledProcessError):
        return None
    p = p.strip()
    return p if os.path.isabs(p) and os.path.exists(p) else None


@pytest.mark.slow
def test_oracle_pins_clean_under_asan_ubsan():
    asan, ubsan = _runtime("libasan.so"), _runtime("libubsan.so")
    if not asan or not ubsan:
        pytest.skip("gcc sanitizer runtimes not installed")
    # the sanitizer runtimes go first in the child's preload list; anything already listed stays
    pre = os.environ.get("LD_PRELOAD", "")
    env = dict(os.environ, VXO_SANITIZE="1", LD_PRELOAD=f"{asan}:{ubsan}" + (f":{pre}" if pre else ""),
               ASAN_OPTIONS="detect_leaks=0:abort_on_error=1", UBSAN_OPTIONS="print_stacktrace=1")
    subprocess.run([sys.executable, "-c", "import oracle; oracle.build(force=True)"], cwd=ROOT, env=env, check=True)
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-x", "-p", "no:cacheprovider",
                        "tests/test_oracle_pins.py", "tests/test_oracle_fit.py", "tests/test_oracle_compact.py",
                        "tests/test_oracle_sample.py", "tests/test_oracle_occupancy.py", "tests/test_oracle_sggxh.py"],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=900)
    tail = (r.stdout + r.stderr)[-3000:]
    assert r.returncode == 0, tail
    assert "ERROR: AddressSanitizer" not in tail and "runtime error" not in tail, tail
