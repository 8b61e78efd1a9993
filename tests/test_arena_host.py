"""The graph-capture ownership rules of the library's context memory
(paper_2304_07325_amd/csrc/symba_arena.h), compiled with g++ without HIP and
run on the host: the capture arena is append-only, aligned and bounded; the
partial-sum buffer is kept, grown, retired or refused as documented."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.skipif(shutil.which("g++") is None, reason="g++ not available")
def test_arena_rules(tmp_path):
    exe = str(tmp_path / "arena_test")
    subprocess.run(["g++", "-O1", "-g", "-std=c++17", "-Wall", "-I",
                    os.path.join(ROOT, "paper_2304_07325_amd", "csrc"), "-o", exe,
                    os.path.join(ROOT, "tests", "csrc", "arena_test.cpp")], check=True)
    r = subprocess.run([exe], capture_output=True, text=True, timeout=60)
    assert r.returncode == 0 and r.stdout.strip().endswith("ok"), r.stdout
