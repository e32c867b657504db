"""CPU builds with AddressSanitizer and UndefinedBehaviorSanitizer (leak
detection on): the oracle driven through every entry point on a tiny s/p/d
system (oracle/sanitize_check.c), and the library's host code driven through
the entry points that need no device (paper_2606_04316_amd/sanitize_check.c:
tuning cache, RKB small components, argument checks).  A sanitizer report or
a failed check fails the test."""
import os
import subprocess

import pytest


def _run(exe, args=(), env_extra=None):
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1", OMP_NUM_THREADS="2")
    if env_extra:
        env.update(env_extra)
    r = subprocess.run([exe, *args], capture_output=True, text=True, env=env, timeout=600)
    out = r.stdout + r.stderr
    print(out[-3000:])
    assert "AddressSanitizer" not in out and "LeakSanitizer" not in out, out[-3000:]
    assert "runtime error" not in out, out[-3000:]
    assert r.returncode == 0 and "all checks passed" in r.stdout
    return out


def test_oracle_under_sanitizers():
    import oracle
    _run(oracle.build_sanitized())


def test_library_host_code_under_sanitizers(tmp_path):
    from paper_2606_04316_amd import build
    _run(build.build_sanitized(), [str(tmp_path / "tune.jsonl")])
