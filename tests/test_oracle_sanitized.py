"""The oracle's C code under AddressSanitizer and UndefinedBehaviorSanitizer
(host code only): the CPU pins of the oracle run in a child process whose
oracle library is the sanitized build; any out-of-bounds access, leak-free
heap misuse or undefined behaviour aborts that process."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _asan_runtime():
    try:
        p = subprocess.run(["gcc", "-print-file-name=libasan.so"], capture_output=True, text=True, check=True)
    except (OSError, subprocess.CalledProcessError):
        return None
    path = p.stdout.strip()
    return path if os.path.isabs(path) and os.path.exists(path) else None


@pytest.mark.slow
def test_oracle_pins_under_sanitizers():
    asan = _asan_runtime()
    if asan is None:
        pytest.skip("gcc's AddressSanitizer runtime is not installed")
    env = dict(os.environ)
    env.update(DN_ORACLE_SANITIZE="1", LD_PRELOAD=asan,
               ASAN_OPTIONS="detect_leaks=0:abort_on_error=1:halt_on_error=1",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1", OMP_NUM_THREADS="4")
    cmd = [sys.executable, "-c", "import oracle; oracle.build(force=True)"]
    subprocess.run(cmd, cwd=ROOT, env={k: v for k, v in env.items() if k != "LD_PRELOAD"}, check=True)
    tests = [os.path.join(ROOT, "tests", t) for t in ("test_oracle_pins.py", "test_oracle_l1_pins.py",
                                                     "test_oracle_mesh_pins.py", "test_oracle_laser_pins.py")]
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-x", "-p", "no:cacheprovider",
                        "-k", "not torch"] + tests, cwd=ROOT, env=env, capture_output=True, text=True,
                       timeout=900)
    tail = (r.stdout + r.stderr)[-3000:]
    assert r.returncode == 0, tail
    assert "ERROR: AddressSanitizer" not in tail and "runtime error" not in tail, tail
