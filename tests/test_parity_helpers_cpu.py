"""The GPU tests' own helpers, on the CPU: the padding view of a column-major
tensor reaches exactly the rows beyond m, and each parity bar fails on a
planted error that the others would let through."""
import numpy as np
import pytest

from parity import column_rel_errors, elementwise_rel_error, padding_rows

torch = pytest.importorskip("torch")
hs = pytest.importorskip("paper_2608_25469_amd")


@pytest.mark.parametrize("m,n,ld", [(5, 3, 9), (1, 1, 4), (7, 1, 7), (16, 16, 21)])
def test_padding_rows_cover_rows_beyond_m(m, n, ld):
    t = hs.colmajor(m, n, torch.float64, ld=ld, device="cpu", fill=0.0)
    pad = padding_rows(t)
    assert tuple(pad.shape) == (n, ld - m)
    pad.fill_(7.0)
    # the matrix itself is untouched, and every padding slot is written
    assert not torch.any(t != 0.0)
    store = t.as_strided((n * ld,), (1,), t.storage_offset())
    expect = np.zeros((n, ld))
    expect[:, m:] = 7.0
    assert np.array_equal(store.numpy().reshape(n, ld), expect)


def test_column_bar_sees_a_small_wrong_column():
    ref = np.ones((8, 4))
    ref[:, 3] = 1e-9
    X = ref.copy()
    X[:, 3] *= 1.0 + 1e-6
    # the Frobenius norm of the difference hides the column ...
    assert np.linalg.norm(X - ref) / np.linalg.norm(ref) < 1e-12
    # ... its own relative error does not
    assert column_rel_errors(X, ref)[3] > 1e-7


def test_elementwise_bar_sees_one_wrong_entry():
    ref = np.ones((50, 3))
    X = ref.copy()
    X[17, 1] += 1e-10
    assert elementwise_rel_error(X, ref) == pytest.approx(1e-10, rel=1e-3)
