"""CPU tests of the serve scheduler (csrc/serve_sched.h) with a fake backend
(tests/sched_fake.cpp): admission never exceeds the arena, a full queue
answers TN_E_AGAIN, stopping cancels queued requests, a failing request
fails alone, requests that can never fit fail with TN_E_NOMEM, a request
waiting for memory does not block smaller ones, memory released by other
users of the arena admits waiting requests, and a request that stays
unadmitted with the scheduler idle ends instead of waiting for ever.  The
same program also runs under ThreadSanitizer and AddressSanitizer (host code
only; g++, no GPU)."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(os.path.dirname(HERE), "paper_2507_20667_amd", "csrc")
SRC = os.path.join(HERE, "sched_fake.cpp")


def _build_and_run(tmp_path, extra, env=None):
    exe = str(tmp_path / "sched_fake")
    cmd = ["g++", "-std=c++17", "-O1", "-g", "-pthread", "-I", CSRC, SRC, "-o", exe] + extra
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    r = subprocess.run([exe], capture_output=True, text=True, timeout=240,
                       env=dict(os.environ, **(env or {})))
    print(r.stdout)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "ALL PASSED" in r.stdout
    return r


@pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")
def test_scheduler_fake_backend(tmp_path):
    _build_and_run(tmp_path, [])


@pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")
def test_scheduler_thread_sanitizer(tmp_path):
    r = _build_and_run(tmp_path, ["-fsanitize=thread"], {"TSAN_OPTIONS": "halt_on_error=1"})
    assert "WARNING: ThreadSanitizer" not in r.stderr


@pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")
def test_scheduler_address_sanitizer(tmp_path):
    r = _build_and_run(tmp_path, ["-fsanitize=address,undefined", "-fno-omit-frame-pointer"],
                       {"ASAN_OPTIONS": "detect_leaks=1"})
    assert "ERROR: AddressSanitizer" not in r.stderr
