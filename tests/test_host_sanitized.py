"""The host-side ABI tests (plan validation, workspace checks, tunings, the
GenASiS builder) rerun against the host-sanitized library: every host code
path they reach runs under AddressSanitizer and UndefinedBehaviorSanitizer,
which abort the run on the first error.  CPU only."""
import os
import subprocess
import sys

import sanitized_host_build as shb

HERE = os.path.dirname(os.path.abspath(__file__))


def test_host_abi_tests_clean_under_asan_and_ubsan():
    lib = shb.build()
    env = dict(os.environ)
    env.update(MPOLE_LIBRARY=lib, LD_PRELOAD=shb.asan_runtime(),
               ASAN_OPTIONS="detect_leaks=0:abort_on_error=1", UBSAN_OPTIONS="print_stacktrace=1")
    cmd = [sys.executable, "-m", "pytest", "-q", "-x", "-p", "no:cacheprovider", "-m", "not gpu",
           os.path.join(HERE, "test_abi_host.py"), os.path.join(HERE, "test_genasis_host.py")]
    r = subprocess.run(cmd, env=env, cwd=os.path.dirname(HERE), capture_output=True, text=True, timeout=900)
    tail = (r.stdout + r.stderr)[-4000:]
    assert r.returncode == 0, tail
    assert "passed" in r.stdout and "AddressSanitizer" not in tail and "runtime error" not in tail, tail
