"""The request loop's arena allocator (C++), compiled on its own with the
host compiler and address/undefined-behaviour sanitizers, run against a
byte-map model."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.skipif(shutil.which("g++") is None, reason="no host C++ compiler")
def test_arena_against_model(tmp_path):
    exe = os.path.join(str(tmp_path), "arena_test")
    subprocess.run(["g++", "-std=c++17", "-O1", "-g", "-fsanitize=address,undefined",
                    "-fno-sanitize-recover=all",
                    "-I" + os.path.join(ROOT, "paper_1403_7295_amd", "csrc"),
                    os.path.join(ROOT, "tests", "cpp", "arena_test.cpp"), "-o", exe], check=True)
    r = subprocess.run([exe], capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stderr
    assert "arena ok" in r.stdout
