"""Build the gfx950 HIP library ``libhsma.so`` in-tree.

Every ``csrc/*.hip`` and ``csrc/*.cpp`` is compiled by hipcc for gfx950 (one
process per translation unit, in parallel) and linked into
``paper_2608_25469_amd/libhsma.so``.  Run ``python -m paper_2608_25469_amd.build``.
"""
from __future__ import annotations

import concurrent.futures as cf
import glob
import os
import shutil
import subprocess
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libhsma.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

ARCH = "gfx950"
COMMON = [
    "-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
    # Packed FP32 instructions are kept out of every kernel.
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    # The small-solve kernels rely on complete unrolling of long loop nests.
    "-mllvm", "-pragma-unroll-threshold=500000",
    "-Wno-unused-command-line-argument",
    f"-I{os.path.join(HERE, '..', 'include')}",
]


def _headers_mtime() -> float:
    hs = glob.glob(os.path.join(CSRC, "*.h")) + glob.glob(os.path.join(HERE, "..", "include", "*.h"))
    return max([os.path.getmtime(h) for h in hs] + [os.path.getmtime(__file__)])


def _compile(src: str, incremental: bool = False) -> str:
    obj = os.path.join(BUILD, os.path.basename(src) + ".o")
    if incremental and os.path.exists(obj) and \
            os.path.getmtime(obj) > max(os.path.getmtime(src), _headers_mtime()):
        return f"{os.path.basename(src)} up to date"
    # .cpp files hold host-only code but use the HIP runtime API; they are
    # compiled as HIP so the same toolchain and headers apply.
    cmd = [HIPCC, *COMMON, "-x", "hip", "-c", src, "-o", obj]
    t0 = time.time()
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"compile failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    return f"{os.path.basename(src)} {time.time() - t0:.1f}s"


def build(verbose: bool = True, jobs: int | None = None, incremental: bool = False) -> str:
    """Compile every source (``incremental``: only those older than their
    object file and every header are skipped) and link the library."""
    os.makedirs(BUILD, exist_ok=True)
    srcs = sorted(glob.glob(os.path.join(CSRC, "*.hip")) + glob.glob(os.path.join(CSRC, "*.cpp")))
    jobs = jobs or min(len(srcs), max(1, (os.cpu_count() or 4)))
    with cf.ThreadPoolExecutor(max_workers=jobs) as ex:
        for msg in ex.map(lambda src: _compile(src, incremental), srcs):
            if verbose:
                print("  built", msg, flush=True)
    objs = [os.path.join(BUILD, os.path.basename(s) + ".o") for s in srcs]
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = [HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *objs,
           "-Wno-unused-command-line-argument"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, LIB)
    if verbose:
        print("  linked", LIB, flush=True)
    return LIB


def clean() -> None:
    shutil.rmtree(BUILD, ignore_errors=True)


if __name__ == "__main__":
    t = time.time()
    build(incremental="--incremental" in sys.argv)
    print(f"done in {time.time() - t:.1f}s", file=sys.stderr)
