"""The device allocator's segment bookkeeping (hmx_segcache.h), compiled for the host with g++
and run on a malloc backend: trimmed buffers hand their tail to later requests, frees merge,
only entirely free blocks are released, and a seeded random sequence of allocations, shrinks,
frees and releases keeps live buffers disjoint and their contents intact."""
import os
import subprocess

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_segment_cache_on_the_host(tmp_path):
    exe = str(tmp_path / "segcache_check")
    src = os.path.join(ROOT, "tests", "segcache_check.cpp")
    r = subprocess.run(["g++", "-std=c++17", "-O1", "-Wall", "-Werror", "-fsanitize=address,undefined",
                        src, "-o", exe], capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    r = subprocess.run([exe], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0 and r.stdout.strip().endswith("ok"), r.stdout + r.stderr
