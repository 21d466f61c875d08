"""The FP64 oracle under AddressSanitizer and UndefinedBehaviorSanitizer.

tests/helpers/oracle_sanitize.c compiles the oracle's source into a small
program (gcc, no OpenMP) that runs every entry point on graphs using all of
its features (absorbing, mirror and self-loop vertices, zero jump
probabilities, cubic coefficients, semi-infinite edges, the split cap,
sources, traces longer than their buffer) and checks that particles are
conserved.  Any out-of-bounds access, leak, signed overflow, misaligned or
invalid shift aborts it.
"""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))


def test_oracle_clean_under_asan_and_ubsan(tmp_path):
    if shutil.which("gcc") is None:
        pytest.skip("no gcc")
    exe = str(tmp_path / "oracle_sanitize")
    src = os.path.join(HERE, "helpers", "oracle_sanitize.c")
    subprocess.run(["gcc", "-std=c11", "-O1", "-g", "-ffp-contract=off",
                    "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
                    "-fno-omit-frame-pointer", "-Wno-unknown-pragmas", "-o", exe, src, "-lm"],
                   check=True)
    # verify_asan_link_order=0: the process may have other libraries
    # preloaded ahead of the sanitizer runtime
    env = dict(os.environ,
               ASAN_OPTIONS="detect_leaks=1:abort_on_error=0:verify_asan_link_order=0",
               UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=300)
    assert r.returncode == 0, r.stderr[-4000:]
    assert "oracle_sanitize: ok" in r.stdout
    assert "runtime error" not in r.stderr
