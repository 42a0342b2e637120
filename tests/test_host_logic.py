"""Host logic of the library that needs no device, compiled from the
library's own headers with g++ and run: the serving pool allocator and
latency percentiles, and the serving core (admission, release,
cancellation, statistics) driven by a fake executor on host threads --
plain, under ThreadSanitizer, and under AddressSanitizer with
UndefinedBehaviorSanitizer."""
import os
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CPP = os.path.join(ROOT, "tests", "cpp")


def build_and_run(tmp_path, source, flags, expect):
    exe = str(tmp_path / (os.path.splitext(source)[0] + "_" + str(abs(hash(tuple(flags))))))
    subprocess.check_call(["g++", "-std=c++17", "-g", "-Wall", "-pthread", *flags, "-o", exe,
                           os.path.join(CPP, source)])
    env = dict(os.environ, TSAN_OPTIONS="halt_on_error=1", ASAN_OPTIONS="detect_leaks=1")
    out = subprocess.run([exe], capture_output=True, text=True, timeout=300, env=env)
    assert out.returncode == 0, out.stdout + out.stderr
    assert "WARNING" not in out.stderr, out.stderr
    assert expect in out.stdout


def test_pool_allocator_and_percentiles(tmp_path):
    build_and_run(tmp_path, "test_pool.cpp", ["-O1"], "pool ok")


@pytest.mark.parametrize("flags", [["-O2"], ["-O1", "-fsanitize=thread"],
                                   ["-O1", "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined"]],
                         ids=["plain", "tsan", "asan_ubsan"])
def test_serving_core_with_a_fake_executor(tmp_path, flags):
    build_and_run(tmp_path, "test_serve_core.cpp", flags, "serve core ok")
