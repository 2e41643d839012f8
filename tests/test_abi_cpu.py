"""The C ABI without a GPU: the library loads, exports every function the
header declares, and rejects bad arguments before touching the device."""
import ctypes
import os
import re

import pytest

import paper_2608_25469_amd as hs

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "hsma.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(hsma_[a-z0-9_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(hs.LIB_PATH):
        pytest.fail("libhsma.so is not built (python -m paper_2608_25469_amd.build)")
    return hs.lib()


def test_exports_every_declared_symbol(lib):
    names = declared_functions()
    assert "hsma_trsm" in names and "hsma_trsm_ex" in names
    for n in names:
        assert hasattr(lib, n), f"{n} declared in hsma.h but not exported"


def test_status_strings(lib):
    for code in range(12):
        s = lib.hsma_status_string(code)
        assert s and len(s) > 3
    assert lib.hsma_version().startswith(b"0.")


def _call(lib, diag=0, m=4, n=3, alpha=1.0, A=16, lda=4, B=32, ldb=4, dtype=0):
    al = (ctypes.c_double * 2)(alpha, 0.0) if alpha is not None else None
    return lib.hsma_trsm(diag, m, n, al, ctypes.c_void_p(A) if A else None, lda,
                         ctypes.c_void_p(B) if B else None, ldb, dtype, None)


def test_validation_order(lib):
    # 1. enumerators
    assert _call(lib, diag=2) == 1
    assert _call(lib, dtype=7) == 1
    assert _call(lib, diag=-1, m=-1) == 1          # enum checked before sizes
    # 2. sizes
    assert _call(lib, m=-1) == 2
    assert _call(lib, n=-5) == 2
    # 3. leading dimensions
    assert _call(lib, m=5, lda=4) == 2
    assert _call(lib, m=5, lda=5, ldb=4) == 2
    assert _call(lib, m=0, lda=0) == 2              # ld >= max(1, m)
    # 4. quick return before pointer checks
    assert _call(lib, m=0, lda=1, ldb=1, A=0, B=0, alpha=None) == 0
    assert _call(lib, n=0, A=0, B=0, alpha=None) == 0
    # 5. alpha pointer
    assert _call(lib, alpha=None) == 3
    # 6. B null; A null only matters when alpha != 0
    assert _call(lib, B=0) == 3
    assert _call(lib, A=0) == 3


def test_ex_option_checks(lib):
    al = (ctypes.c_double * 2)(1.0, 0.0)
    for bad in (dict(block_size=48), dict(path=3), dict(block_size=-16)):
        o = hs.TrsmOptions(**bad)
        st = lib.hsma_trsm_ex(0, 4, 3, al, ctypes.c_void_p(16), 4, ctypes.c_void_p(32), 4, 0,
                              ctypes.byref(o), None, None)
        assert st == 1, bad
    for bad in (dict(precision=2), dict(refine_steps=5), dict(refine_steps=-2),
                dict(want_backward_error=2), dict(refine_tol=-1.0), dict(use_graph=3)):
        o = hs.TrsmOptions(**bad)
        st = lib.hsma_trsm_ex(0, 4, 3, al, ctypes.c_void_p(16), 4, ctypes.c_void_p(32), 4, 0,
                              ctypes.byref(o), None, None)
        assert st == 1, bad
    o = hs.TrsmOptions()
    o.reserved[1] = 1
    st = lib.hsma_trsm_ex(0, 4, 3, al, ctypes.c_void_p(16), 4, ctypes.c_void_p(32), 4, 0,
                          ctypes.byref(o), None, None)
    assert st == 1


def test_block_size_lookup_rule(lib):
    # Exact table scales return their entry; other scales the nearest one in
    # log2(m), then log2(n), ties to the smaller scale.
    import math
    src = open(os.path.join(ROOT, "paper_2608_25469_amd", "csrc", "tuning_gfx950.h")).read()
    rows = [tuple(map(int, t)) for t in re.findall(r"\{(\d), (\d+), (\d+), (\d+)\}", src)]
    assert rows

    def expect(dt, m, n):
        cand = [r for r in rows if r[0] == dt]
        key = lambda r: (round(abs(math.log2(r[1]) - math.log2(m)), 9),
                         round(abs(math.log2(r[2]) - math.log2(n)), 9), r[1], r[2])
        return min(cand, key=key)[3]

    for dt in (0, 1):
        for m in (65, 100, 128, 181, 1000, 3000, 5000, 20000, 100000):
            for n in (1, 64, 1000, 16384):
                assert lib.hsma_lookup_block_size(dt, m, n) == expect(dt, m, n), (dt, m, n)


def test_batched_validation_without_device(lib):
    """Every descriptor is checked before anything touches the device."""
    P = hs.Problem
    good = P(0, 0, 4, 3, 1.0, 0.0, ctypes.c_void_p(16), 4, ctypes.c_void_p(32), 4)
    bad_lda = P(0, 0, 4, 3, 1.0, 0.0, ctypes.c_void_p(16), 3, ctypes.c_void_p(32), 4)
    bad_alpha = P(0, 0, 4, 3, 1.0, 0.5, ctypes.c_void_p(16), 4, ctypes.c_void_p(32), 4)
    bad_enum = P(0, 9, 4, 3, 1.0, 0.0, ctypes.c_void_p(16), 4, ctypes.c_void_p(32), 4)
    for probs, idx, st in (([good, bad_lda], 1, 2), ([bad_alpha, good], 0, 1),
                           ([good, good, bad_enum], 2, 1)):
        arr = (P * len(probs))(*probs)
        first = ctypes.c_int64(-7)
        assert lib.hsma_trsm_batched(arr, len(probs), ctypes.byref(first), None) == st
        assert first.value == idx
        plan = ctypes.c_void_p()
        first.value = -7
        assert lib.hsma_batch_plan_create(arr, len(probs), ctypes.byref(first), ctypes.byref(plan)) == st
        assert first.value == idx and not plan.value
    assert lib.hsma_trsm_batched(None, 3, None, None) == 3
    assert lib.hsma_trsm_batched(None, -1, None, None) == 2
    assert lib.hsma_trsm_batched(None, 0, None, None) == 0


STRUCTS = {
    "hsma_trsm_options": hs.TrsmOptions,
    "hsma_trsm_report": hs.TrsmReport,
    "hsma_problem": hs.Problem,
    "hsma_phase_stat": hs.PhaseStat,
    "hsma_queue_config": hs.QueueConfig,
    "hsma_request": hs.Request,
    "hsma_request_info": hs.RequestInfo,
    "hsma_queue_statistics": hs.QueueStatistics,
    "hsma_latency_summary": hs.LatencySummary,
}


def test_binding_structs_match_header(tmp_path):
    """Size and every field offset of the ctypes mirrors equal the C
    compiler's layout of the header's structs."""
    import shutil
    import subprocess
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no host C compiler")
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "hsma.h"', "int main(void) {"]
    for cname, py in STRUCTS.items():
        lines.append(f'printf("{cname} size %zu\\n", sizeof({cname}));')
        for f in py._fields_:
            lines.append(f'printf("{cname} {f[0]} %zu\\n", offsetof({cname}, {f[0]}));')
    lines += ["return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.run([cc, "-std=c11", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)],
                   check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split("\n")
    got = {}
    for ln in out:
        if ln:
            a, b, c = ln.split()
            got[(a, b)] = int(c)
    for cname, py in STRUCTS.items():
        assert got[(cname, "size")] == ctypes.sizeof(py), cname
        for f in py._fields_:
            assert got[(cname, f[0])] == getattr(py, f[0]).offset, (cname, f[0])


def test_generate_inputs_validation(lib):
    g = lib.hsma_generate_inputs
    assert g(3, 4, 4, 1, ctypes.c_void_p(16), ctypes.c_void_p(32), None) == 1
    assert g(0, -1, 4, 1, ctypes.c_void_p(16), ctypes.c_void_p(32), None) == 2
    assert g(0, 4, -1, 1, ctypes.c_void_p(16), ctypes.c_void_p(32), None) == 2
    assert g(0, 0, 4, 1, None, None, None) == 0
    assert g(0, 4, 4, 1, None, ctypes.c_void_p(32), None) == 3
    assert g(1, 4, 4, 1, ctypes.c_void_p(16), None, None) == 3


def test_noalloc_rejects_oversized_workspace_before_device(lib):
    """hsma_trsm_noalloc validates like hsma_trsm and refuses a blocked
    problem whose workspace exceeds its fixed scratch array before any device
    call (fake pointers are never dereferenced)."""
    f = lib.hsma_trsm_noalloc
    f.argtypes = [ctypes.c_int32, ctypes.c_int64, ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p,
                  ctypes.c_int64, ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, ctypes.c_void_p]
    f.restype = ctypes.c_int32
    lib.hsma_noalloc_scratch_bytes.restype = ctypes.c_uint64
    assert lib.hsma_noalloc_scratch_bytes() == 64 << 20
    one = (ctypes.c_double * 2)(1.0, 0.0)
    fake = ctypes.c_void_p(0x1000)
    assert f(0, 40000, 1, one, fake, 40000, fake, 40000, 0, None) == 12
    assert f(0, 30000, 1, one, fake, 30000, fake, 30000, 1, None) == 12
    # the documented validation order comes first
    assert f(2, 40000, 1, one, fake, 40000, fake, 40000, 0, None) == 1
    assert f(0, 5, 1, one, fake, 4, fake, 5, 0, None) == 2
    assert f(0, 0, 1, one, None, 1, None, 1, 0, None) == 0
    assert f(0, 5, 1, None, fake, 5, fake, 5, 0, None) == 3
    assert lib.hsma_status_string(12)


def test_general_validation_order_without_device(lib):
    """hsma_trsm_general checks its arguments in the documented order before
    any device call (fake pointers are never dereferenced)."""
    f = lib.hsma_trsm_general
    i32, i64, vp = ctypes.c_int32, ctypes.c_int64, ctypes.c_void_p
    f.argtypes = [i32, i32, i32, i32, i64, i64, vp, vp, i64, vp, i64, i32, vp]
    f.restype = i32
    one = (ctypes.c_double * 2)(1.0, 0.0)
    zero = (ctypes.c_double * 2)(0.0, 0.0)
    A, B = ctypes.c_void_p(16), ctypes.c_void_p(32)

    def call(side=0, uplo=0, trans=0, diag=0, m=4, n=3, alpha=one, A=A, lda=4, B=B, ldb=4, dt=0):
        return f(side, uplo, trans, diag, m, n, alpha, A, lda, B, ldb, dt, None)
    assert call(side=2) == 1 and call(uplo=-1) == 1 and call(trans=3) == 1
    assert call(diag=2) == 1 and call(dt=5) == 1
    assert call(m=-1) == 2 and call(n=-1) == 2
    assert call(side=1, lda=2) == 2            # right side: lda >= n = 3
    assert call(side=0, lda=3) == 2            # left side: lda >= m = 4
    assert call(ldb=3) == 2
    assert call(side=1, m=5, n=0, lda=1, ldb=5) == 0
    assert call(alpha=None) == 3
    assert call(B=None) == 3
    assert call(A=None) == 3
    assert call(side=1, uplo=1, trans=2, A=None, alpha=zero, m=0) == 0
