"""The serving scheduler (paper_1711_01177_amd/csrc/grim_serve.cpp) on the CPU
(no GPU): the same source the library links, built against a host-memory
backend (tests/native/serve_fake_backend.cpp: worker threads as streams, a
stand-in filter, injected launch failures) and driven by
tests/native/serve_check.cpp from several threads with concurrent
cancellations.  It runs once under ThreadSanitizer and once under
AddressSanitizer + UndefinedBehaviorSanitizer; any sanitizer report or failed
check fails the test."""
import os
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1711_01177_amd", "csrc")
NATIVE = os.path.join(ROOT, "tests", "native")
SOURCES = [os.path.join(CSRC, "grim_serve.cpp"), os.path.join(NATIVE, "serve_fake_backend.cpp"),
           os.path.join(NATIVE, "serve_check.cpp")]
FLAGS = {
    "thread": ["-fsanitize=thread"],
    "address,undefined": ["-fsanitize=address,undefined", "-fno-sanitize-recover=all",
                          "-fno-omit-frame-pointer"],
}
ENV = {
    "thread": {"TSAN_OPTIONS": "halt_on_error=1:exitcode=66:second_deadlock_stack=1"},
    "address,undefined": {"ASAN_OPTIONS": "halt_on_error=1:exitcode=86:detect_leaks=1",
                          "UBSAN_OPTIONS": "halt_on_error=1:print_stacktrace=1:exitcode=87"},
}


@pytest.mark.parametrize("sanitizer", sorted(FLAGS))
def test_scheduler_under_sanitizer(sanitizer, tmp_path):
    exe = str(tmp_path / "serve_check")
    cmd = ["g++", "-std=c++17", "-O1", "-g", "-Wall", "-Wextra", "-Werror", *FLAGS[sanitizer],
           f"-I{os.path.join(ROOT, 'include')}", f"-I{CSRC}", *SOURCES, "-o", exe, "-lpthread"]
    subprocess.check_call(cmd)
    env = dict(os.environ)
    env.pop("LD_PRELOAD", None)
    env.update(ENV[sanitizer])
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=900)
    assert r.returncode == 0, (r.returncode, r.stdout[-2000:], r.stderr[-6000:])
    assert "all scenarios passed" in r.stdout
    assert "failed launches" in r.stdout
