"""The FP64 oracle under AddressSanitizer and UndefinedBehaviorSanitizer (CPU).

Builds ``oracle_sanitize_main.c`` (which includes the oracle's single C source)
with gcc, ``-fsanitize=address,undefined`` and no recovery, and runs it: any
out-of-bounds access, leak, use after free, signed overflow or other undefined
behaviour in the oracle's neighbour search, sweeps, step or wall treatment
ends the run with a non-zero status.  Host code only.
"""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.mark.skipif(shutil.which("gcc") is None, reason="needs gcc")
def test_oracle_clean_under_sanitizers(tmp_path):
    exe = tmp_path / "oracle_sanitize"
    cmd = ["gcc", "-std=c11", "-O1", "-g", "-fno-omit-frame-pointer", "-ffp-contract=off",
           "-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-Wall",
           "-Wno-unknown-pragmas", "-o", str(exe),
           os.path.join(HERE, "oracle_sanitize_main.c"), "-lm"]
    subprocess.run(cmd, check=True, capture_output=True, text=True)
    env = dict(os.environ,
               ASAN_OPTIONS="detect_leaks=1:abort_on_error=0:verify_asan_link_order=0",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    r = subprocess.run([str(exe)], capture_output=True, text=True, env=env, timeout=300)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "oracle sanitizer run clean" in r.stdout
