"""Host logic of the library that needs no device: the serving pool
allocator and latency percentiles (compiled from the library's own header
with g++ and run)."""
import os
import subprocess

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_pool_allocator_and_percentiles(tmp_path):
    exe = str(tmp_path / "test_pool")
    subprocess.check_call(["g++", "-O1", "-std=c++17", "-Wall", "-o", exe,
                           os.path.join(ROOT, "tests", "cpp", "test_pool.cpp")])
    out = subprocess.run([exe], capture_output=True, text=True, timeout=60)
    assert out.returncode == 0, out.stderr
    assert "pool ok" in out.stdout
