"""Bucket order of the grouped strip launch (csrc/strip_pack.h), on the CPU.

The header is compiled with g++ into a native driver (tests/native/
pack_check.cpp) under the address and undefined-behaviour sanitizers and run
on random buckets: every strip once, whole problems kept in one wavefront
where the strip counts allow it."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2608_25469_amd", "csrc")


def test_bucket_order(tmp_path):
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("g++ not available")
    exe = str(tmp_path / "pack_check")
    subprocess.run([gxx, "-O1", "-g", "-std=c++17", "-fsanitize=address,undefined",
                    "-fno-sanitize-recover=undefined", f"-I{CSRC}",
                    os.path.join(ROOT, "tests", "native", "pack_check.cpp"), "-o", exe],
                   check=True, capture_output=True, text=True)
    r = subprocess.run([exe], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "pack ok" in r.stdout
