"""The server's host thread pool (csrc/host_pool.h), built on its own with g++
under ThreadSanitizer: every item runs once, its writes are visible to the
caller, and no data race is reported."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.skipif(shutil.which("g++") is None, reason="g++ not available")
def test_host_pool_under_thread_sanitizer(tmp_path):
    exe = tmp_path / "host_pool_check"
    build = ["g++", "-std=c++17", "-O1", "-g", "-fsanitize=thread", "-pthread",
             "-I" + os.path.join(ROOT, "paper_2505_12414_amd", "csrc"),
             os.path.join(ROOT, "tests", "host_pool_check.cpp"), "-o", str(exe)]
    r = subprocess.run(build, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    env = dict(os.environ, TSAN_OPTIONS="halt_on_error=1 exitcode=66")
    r = subprocess.run([str(exe)], capture_output=True, text=True, env=env, timeout=300)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "OK" in r.stdout
    assert "WARNING: ThreadSanitizer" not in r.stderr
