"""The oracle under the address and undefined-behaviour sanitizers (CPU).

tests/oracle_sanitized_run.c drives every oracle entry point (both
precisions and shapes, both walls, photons and in-place pairs, a spread of
the threshold, capacity freezes, explicit seeding, the event map, the
generators and the conversion table); it is built here with gcc
-fsanitize=address,undefined and no recovery, so any out-of-bounds access,
leak, overflow or other undefined behaviour fails the test."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.skipif(shutil.which("gcc") is None, reason="no gcc")
def test_oracle_runs_clean_under_sanitizers(tmp_path):
    exe = tmp_path / "oracle_sanitized"
    cmd = ["gcc", "-std=c11", "-O1", "-g", "-ffp-contract=off", "-fno-omit-frame-pointer",
           "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
           "-I", os.path.join(ROOT, "oracle"), "-o", str(exe),
           os.path.join(ROOT, "tests", "oracle_sanitized_run.c"),
           os.path.join(ROOT, "oracle", "pic_oracle.c"), "-lm"]
    subprocess.run(cmd, check=True, capture_output=True)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=1",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    r = subprocess.run([str(exe)], capture_output=True, text=True, env=env, timeout=600)
    assert r.returncode == 0, (r.stdout[-2000:], r.stderr[-4000:])
    assert "ok" in r.stdout
