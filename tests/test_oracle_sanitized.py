"""The CPU oracle built with AddressSanitizer and UndefinedBehaviorSanitizer
(host code only, plain g++) runs every entry point, including the removal
and error branches, without a report (oracle_sanitize_driver.py in a process
of its own, the ASan runtime preloaded into the Python interpreter)."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _runtime(name):
    try:
        p = subprocess.run(["g++", f"-print-file-name={name}"], capture_output=True, text=True, check=True)
    except (OSError, subprocess.CalledProcessError):
        return None
    path = p.stdout.strip()
    return path if os.path.isabs(path) and os.path.exists(path) else None


def test_oracle_clean_under_address_and_ub_sanitizers(tmp_path):
    sys.path.insert(0, ROOT)
    from oracle import build as B
    asan = _runtime("libasan.so")
    if asan is None:
        pytest.skip("no AddressSanitizer runtime for g++ on this host")
    lib = B.build(out=str(tmp_path / "libpn_oracle_san.so"), sanitize=True)
    env = dict(os.environ, PN_ORACLE_LIB=lib, LD_PRELOAD=asan,
               ASAN_OPTIONS="detect_leaks=0:abort_on_error=0:exitcode=23",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1:exitcode=24")
    p = subprocess.run([sys.executable, os.path.join(ROOT, "tests", "oracle_sanitize_driver.py")], env=env,
                       capture_output=True, text=True, timeout=600)
    report = p.stdout[-4000:] + p.stderr[-4000:]
    assert p.returncode == 0, report
    assert "driver ok" in p.stdout, report
    assert "runtime error" not in p.stderr and "AddressSanitizer" not in p.stderr, report
