"""The serving queue under ThreadSanitizer (CPU only).

The library's host code is rebuilt with ThreadSanitizer instrumentation
(device code unchanged, linked from the regular build), and a native driver
(tests/native/queue_stress.cpp) hammers the queue's simulation backend from
four threads: concurrent submits, polls, waits, releases and statistics
against the scheduler thread.  The run must finish, report no data race, and
return every byte of the budget."""
import os
import shutil
import subprocess
from concurrent.futures import ThreadPoolExecutor

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2608_25469_amd", "csrc")
BUILD = os.path.join(ROOT, "paper_2608_25469_amd", "_build")
HIPCC = "/opt/rocm/bin/hipcc"
CLANG = "/opt/rocm/lib/llvm/bin/clang++"
HOST_TUS = ["serve", "api", "alloc", "batched", "grouped", "blocked", "graph", "prof"]
# every translation unit with device code, from the regular build
DEVICE_OBJS = sorted(os.path.basename(f) + ".o" for f in os.listdir(CSRC) if f.endswith(".hip"))

pytestmark = pytest.mark.slow


def test_queue_is_race_free(tmp_path):
    if not (os.path.exists(HIPCC) and os.path.exists(CLANG)):
        pytest.skip("ROCm toolchain not available")
    objs = [os.path.join(BUILD, o) for o in DEVICE_OBJS]
    if not all(os.path.exists(o) for o in objs):
        pytest.skip("library objects not built (python -m paper_2608_25469_amd.build)")
    inc = os.path.join(ROOT, "include")
    tsan = ["-Xarch_host", "-fsanitize=thread"]

    def host(tu):
        out = str(tmp_path / f"{tu}.o")
        subprocess.run([HIPCC, "-O1", "-g", "-std=c++17", "-fPIC", "--offload-arch=gfx950",
                        "-Wno-unused-command-line-argument", *tsan, f"-I{inc}", "-x", "hip", "-c",
                        os.path.join(CSRC, tu + ".cpp"), "-o", out], check=True, capture_output=True)
        return out

    with ThreadPoolExecutor(max_workers=min(8, os.cpu_count() or 2)) as ex:
        host_objs = list(ex.map(host, HOST_TUS))
    drv = str(tmp_path / "queue_stress.o")
    subprocess.run([CLANG, "-O1", "-g", "-std=c++17", *tsan, f"-I{inc}", "-c",
                    os.path.join(ROOT, "tests", "native", "queue_stress.cpp"), "-o", drv], check=True)
    exe = str(tmp_path / "queue_stress")
    subprocess.run([HIPCC, "-g", "--offload-arch=gfx950", "-Wno-unused-command-line-argument", *tsan,
                    drv, *host_objs, *objs, "-o", exe], check=True, capture_output=True)
    r = subprocess.run([exe], capture_output=True, text=True, timeout=240)
    out = r.stdout + r.stderr
    assert "ThreadSanitizer" not in out, out[-4000:]
    assert r.returncode == 0, out[-2000:]
    line = [ln for ln in r.stdout.splitlines() if ln.startswith("submitted")][-1]
    f = dict(zip(line.split()[0::2], map(int, line.split()[1::2])))
    assert f["submitted"] == f["completed"] == 1200 and f["failed"] == 0 and f["in_use"] == 0
