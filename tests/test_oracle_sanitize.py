"""The oracle built with AddressSanitizer and UndefinedBehaviorSanitizer (gcc) runs its public entry
points over every class, route and option on small deterministic inputs (oracle/sanitize_check.c):
no report, exit status 0. CPU only."""
import os
import shutil
import subprocess
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
ORACLE = os.path.join(ROOT, "oracle")


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not found")
def test_oracle_under_address_and_undefined_behaviour_sanitizers():
    with tempfile.TemporaryDirectory() as d:
        exe = os.path.join(d, "sanitize_check")
        cmd = ["gcc", "-O1", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
               "-fno-omit-frame-pointer", "-fopenmp", "-ffp-contract=off", "-I", ORACLE, "-o", exe,
               os.path.join(ORACLE, "sanitize_check.c"), os.path.join(ORACLE, "ada_oracle.c"), "-lm"]
        b = subprocess.run(cmd, capture_output=True, text=True)
        if b.returncode != 0 and ("asan" in b.stderr.lower() or "ubsan" in b.stderr.lower()):
            pytest.skip("sanitizer runtime libraries not available: " + b.stderr[-300:])
        assert b.returncode == 0, b.stderr[-2000:]
        env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1",
                   OMP_NUM_THREADS="2")
        r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=300)
        assert r.returncode == 0, (r.stdout[-1000:], r.stderr[-3000:])
        assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr, r.stderr[-3000:]
        assert r.stdout.strip().endswith("OK")
