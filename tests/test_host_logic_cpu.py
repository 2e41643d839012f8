"""Host logic of the launches, on the CPU: the bucket order of the grouped
strip launch (csrc/strip_pack.h) and the tile shape of a lower-triangular
product (csrc/tile_choice.h: five shapes, 128 x 128 down to 32 x 32).

Each header is compiled with g++ into a native driver (tests/native/) under
the address and undefined-behaviour sanitizers: random buckets (every strip
once, whole problems kept in one wavefront where the strip counts allow it);
non-empty tile counts against a brute force and the shapes chosen for sizes
worked out by hand."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2608_25469_amd", "csrc")


def run_native(tmp_path, name, expect):
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("g++ not available")
    exe = str(tmp_path / name)
    subprocess.run([gxx, "-O1", "-g", "-std=c++17", "-fsanitize=address,undefined",
                    "-fno-sanitize-recover=undefined", f"-I{CSRC}",
                    os.path.join(ROOT, "tests", "native", name + ".cpp"), "-o", exe],
                   check=True, capture_output=True, text=True)
    r = subprocess.run([exe], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stdout + r.stderr
    assert expect in r.stdout


def test_bucket_order(tmp_path):
    run_native(tmp_path, "pack_check", "pack ok")


def test_lower_tile_shape(tmp_path):
    run_native(tmp_path, "tile_check", "tile choice ok")
