"""The oracle under AddressSanitizer and UndefinedBehaviorSanitizer: its
checking build (oracle.build(sanitize=True)) runs every oracle pin test in
a child process with the sanitizer runtime preloaded; any out-of-bounds
access, use after free or undefined operation ends that process with a
report.  CPU only (the GPU library's device code cannot be sanitized on
this hardware; its bounds are checked on the host before each launch)."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
ORACLE_TESTS = ["test_oracle_pins.py", "test_oracle_pp_taps.py", "test_oracle_spatial.py", "test_oracle_recon.py",
                "test_oracle_adjoint.py", "test_oracle_specular.py", "test_oracle_aperture.py"]


def _asan_runtime():
    try:
        path = subprocess.run(["gcc", "-print-file-name=libasan.so"], capture_output=True, text=True,
                              check=True).stdout.strip()
    except (OSError, subprocess.CalledProcessError):
        return None
    return path if os.path.isabs(path) and os.path.exists(path) else None


def test_oracle_pins_under_sanitizers():
    runtime = _asan_runtime()
    if runtime is None:
        pytest.skip("gcc's AddressSanitizer runtime is not installed")
    sys.path.insert(0, ROOT)
    import oracle
    oracle.build(force=True, sanitize=True)
    env = dict(os.environ, HDOF_ORACLE_SANITIZED="1", LD_PRELOAD=runtime,
               ASAN_OPTIONS="detect_leaks=0:halt_on_error=1", UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    files = [os.path.join(ROOT, "tests", f) for f in ORACLE_TESTS if os.path.exists(os.path.join(ROOT, "tests", f))]
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider", *files],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=900)
    out = r.stdout + r.stderr
    assert r.returncode == 0, out[-4000:]
    assert "runtime error" not in out and "AddressSanitizer" not in out, out[-4000:]
    assert " passed" in out
