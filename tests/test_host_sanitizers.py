"""The C ABI's host runtime (argument validation, table building, staging,
the host-only calls) under AddressSanitizer and UndefinedBehaviorSanitizer:
the sanitizer build of the library runs the whole host-side ABI suite in a
child process (the ASan runtime has to be preloaded before Python starts).
CPU only; no device code is instrumented."""
import os
import subprocess
import sys

import pytest

from paper_2605_30541_amd import build as B

HERE = os.path.dirname(os.path.abspath(__file__))


def test_abi_suite_is_clean_under_asan_and_ubsan():
    rt = B.sanitizer_runtime()
    if rt is None or not os.path.exists(B.HIPCC):
        pytest.skip("no ROCm clang ASan runtime or hipcc here")
    lib = B.build_sanitized()
    env = dict(os.environ, SGWAVE_LIBRARY=lib, LD_PRELOAD=rt,
               ASAN_OPTIONS="detect_leaks=0:halt_on_error=1:abort_on_error=0",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-x", "-p", "no:cacheprovider",
                        os.path.join(HERE, "test_abi.py")], env=env, capture_output=True, text=True, timeout=900,
                       cwd=os.path.dirname(HERE))
    out = r.stdout + r.stderr
    assert r.returncode == 0, out[-4000:]
    assert "AddressSanitizer" not in out and "runtime error" not in out, out[-4000:]
    assert " passed" in out
    # the child really ran the instrumented library
    probe = subprocess.run([sys.executable, "-c",
                            "from paper_2605_30541_amd import sgwave; sgwave.lib(); "
                            "print(open('/proc/self/maps').read().count(%r))" % lib],
                           env=env, capture_output=True, text=True, timeout=300, cwd=os.path.dirname(HERE))
    assert probe.returncode == 0 and int(probe.stdout.split()[-1]) > 0, probe.stdout + probe.stderr
