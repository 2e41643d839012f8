"""The CPU oracle against its pins (closed forms, exact arithmetic, a library
solver, invariants).  No GPU needed."""
import pytest

import oracle
import pins


@pytest.fixture(scope="module")
def orc():
    return oracle._load()


@pytest.mark.parametrize("pin", pins.ALL_PINS, ids=lambda f: f.__name__)
def test_pin(orc, pin):
    pin(orc)


def test_thread_count_does_not_change_result(orc):
    import numpy as np
    import workloads as W
    L, B = W.problem(5, 200, 37, True)
    t0 = orc.num_threads()
    try:
        orc.set_num_threads(1)
        X1 = orc.solve(L, B, 0.5 - 1j)
        orc.set_num_threads(max(2, t0))
        X2 = orc.solve(L, B, 0.5 - 1j)
    finally:
        orc.set_num_threads(t0)
    assert np.ascontiguousarray(X1).tobytes() == np.ascontiguousarray(X2).tobytes()


def test_leading_dimensions_and_padding(orc):
    import numpy as np
    import workloads as W
    for cx in (False, True):
        L, B = W.problem(6, 23, 9, cx, lda=31, ldb=27)
        Lc = np.asfortranarray(L)
        Bc = np.asfortranarray(B)
        X = orc.solve(Lc, Bc, 1.0)
        orc.trsm(L, B, 1.0)
        assert np.array_equal(B, X)
        pad = B.base[23:, :]
        assert np.all(pad == W.PAD_SENTINEL)
