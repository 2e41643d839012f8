"""hsma_trsm_noalloc (the entry point for callers that cannot allocate)
against hsma_trsm through the C ABI: same kernels and schedule, so the
results must be equal bit for bit; two calls in a row on each path, the
second with a smaller problem (the scratch array keeps the first call's
contents, which must not leak into the second)."""
import ctypes

import numpy as np
import pytest

import oracle
import workloads as W
from parity import assert_parity

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu
hs = pytest.importorskip("paper_2608_25469_amd")


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)
    hs.lib()


def _abi(fn, L, B, alpha, unit, cx):
    a = complex(alpha)
    al = (ctypes.c_double * 2)(a.real, a.imag)
    st = fn(hs.UNIT if unit else hs.NON_UNIT, B.shape[0], B.shape[1], al,
            ctypes.c_void_p(L.data_ptr()), hs.leading_dim(L), ctypes.c_void_p(B.data_ptr()),
            hs.leading_dim(B), hs.C64F if cx else hs.R64F,
            ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    return st


@pytest.mark.parametrize("cx", [False, True], ids=["real", "complex"])
def test_noalloc_equals_trsm_twice_second_smaller(cx):
    lib = hs.lib()
    alpha = complex(-1.0, 0.5) if cx else -1.0
    # blocked, blocked smaller, small, blocked at the largest size the
    # scratch array holds for the data type, then a small one again
    shapes = [(1500, 300, False), (700, 90, True), (40, 33, False),
              (16384 if not cx else 8192, 64, False), (300, 7, True)]
    for k, (m, n, unit) in enumerate(shapes):
        L, B = W.problem(4000 + k, m, n, cx)
        Ld = hs.to_colmajor(L)
        B1, B2 = hs.to_colmajor(B), hs.to_colmajor(B)
        print(f"noalloc case m={m} n={n} complex={cx} unit={unit}", flush=True)
        assert _abi(lib.hsma_trsm, Ld, B1, alpha, unit, cx) == 0
        assert _abi(lib.hsma_trsm_noalloc, Ld, B2, alpha, unit, cx) == 0
        torch.cuda.synchronize()
        X1, X2 = hs.from_colmajor(B1), hs.from_colmajor(B2)
        assert X2.tobytes() == X1.tobytes(), (m, n, cx, unit)
        cols = list(range(0, n, max(1, n // 8)))
        assert_parity(L, np.asfortranarray(B[:, cols]), np.asfortranarray(X2[:, cols]), alpha,
                      unit=unit, tag=("noalloc", m, n, cx))
        del Ld, B1, B2
        torch.cuda.empty_cache()


def test_noalloc_alpha_zero_and_oversize():
    lib = hs.lib()
    L, B = W.problem(5, 200, 10, False)
    Ld, Bd = hs.to_colmajor(L), hs.to_colmajor(B)
    assert _abi(lib.hsma_trsm_noalloc, Ld, Bd, 0.0, False, False) == 0
    torch.cuda.synchronize()
    assert np.all(hs.from_colmajor(Bd) == 0)
    # larger than the scratch array: refused, B untouched
    Bd = hs.to_colmajor(B)
    al = (ctypes.c_double * 2)(1.0, 0.0)
    st = lib.hsma_trsm_noalloc(0, 40000, 1, al, ctypes.c_void_p(Ld.data_ptr()), 40000,
                               ctypes.c_void_p(Bd.data_ptr()), 40000, 0, None)
    assert st == 12
    torch.cuda.synchronize()
    assert hs.from_colmajor(Bd).tobytes() == np.asfortranarray(B).tobytes()
