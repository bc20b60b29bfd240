"""The oracle built with AddressSanitizer and UndefinedBehaviorSanitizer
(every report fatal) runs the whole pin suite, including the corrupt and
truncated stream cases, in a child process: an out-of-bounds access, a use
after free, a signed overflow or a shift out of range anywhere in the
oracle ends that process with an error."""
import os
import subprocess
import sys

import pytest

import oracle

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _asan_runtime():
    try:
        p = subprocess.check_output(["gcc", "-print-file-name=libasan.so"], text=True).strip()
    except (OSError, subprocess.CalledProcessError):
        return None
    return p if os.path.isabs(p) and os.path.exists(p) else None


@pytest.mark.slow
def test_pins_pass_under_asan_and_ubsan(tmp_path):
    rt = _asan_runtime()
    if rt is None:
        pytest.skip("gcc's AddressSanitizer runtime is not installed")
    so = oracle.build_sanitized(str(tmp_path / "liboracle_san.so"))
    env = dict(os.environ, LD_PRELOAD=rt, ASAN_OPTIONS="detect_leaks=0:abort_on_error=0",
               UBSAN_OPTIONS="print_stacktrace=1", ISX_ORACLE_LIB=so)
    # the child reports which oracle library it loaded, then runs the pins
    probe = subprocess.run([sys.executable, "-c",
                            "import oracle; oracle.lib(); "
                            "print([l.split()[-1] for l in open('/proc/self/maps') if 'liboracle' in l][0])"],
                           cwd=ROOT, env=env, capture_output=True, text=True, timeout=120)
    assert probe.returncode == 0, probe.stderr[-2000:]
    assert probe.stdout.strip() == so
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-x", "-p", "no:cacheprovider",
                        os.path.join(ROOT, "tests", "test_oracle_pins.py")],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=900)
    assert r.returncode == 0, (r.stdout[-3000:], r.stderr[-3000:])
    assert "passed" in r.stdout and "failed" not in r.stdout
