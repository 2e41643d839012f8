"""Parity criteria shared by the GPU tests: the library's result against the
oracle's on the same inputs.

Three bars, all of which must hold (FP64 paths):
  - normwise:    ||X - X_ref||_F / ||X_ref||_F <= 1e-12 (the paper's Table 2
                 metric, Sec. 5.1);
  - per column:  max_j ||x_j - xref_j||_2 / ||xref_j||_2 <= 1e-12, so a wrong
                 column of small magnitude cannot hide under the norm of the
                 others (columns are independent solves, Sec. 4.2.1);
  - element:     max_ij |x_ij - xref_ij| / max_ij |xref_ij| <= 1e-12;
and the normwise backward error of X computed by the oracle (Dot2 residual)
stays <= 10 m 2^-53.
"""
import numpy as np

import oracle

U = 2.0 ** -53
REL_BAR = 1e-12


def padding_rows(t):
    """Rows m .. ld - 1 of every column of the column-major m x n tensor t
    (a view of its storage, shape (n, ld - m)).  A slice of t itself cannot
    reach them: t covers rows 0 .. m - 1 only."""
    m, n = t.shape
    ld = t.stride(1)
    full = t.as_strided((n, ld), (ld, 1), t.storage_offset())
    return full[:, m:]


def column_rel_errors(X, ref):
    """Per-column relative 2-norm errors (a zero reference column counts its
    absolute error)."""
    X = np.asarray(X)
    ref = np.asarray(ref)
    num = np.linalg.norm(X - ref, axis=0)
    den = np.linalg.norm(ref, axis=0)
    return np.where(den > 0, num / np.where(den > 0, den, 1.0), num)


def elementwise_rel_error(X, ref):
    X = np.asarray(X)
    ref = np.asarray(ref)
    if X.size == 0:
        return 0.0
    scale = np.max(np.abs(ref))
    err = np.max(np.abs(X - ref))
    return float(err / scale) if scale > 0 else float(err)


def assert_parity(L, B, X, alpha, unit=False, tag="", ref=None, bar=REL_BAR, eta_bar=None,
                  check_eta=True):
    """All parity bars for one result; returns (fro, worst column, element, eta).
    ``check_eta=False`` skips the backward error (inputs regenerated on the host
    that agree with the device's only to rounding)."""
    if ref is None:
        ref = oracle.solve(L, B, alpha, unit=unit)
    m = B.shape[0]
    assert np.all(np.isfinite(X)), (tag, "non-finite result")
    fro = oracle.rel_err_fro(X, ref)
    col = float(np.max(column_rel_errors(X, ref))) if X.size else 0.0
    ele = elementwise_rel_error(X, ref)
    assert fro <= bar, (tag, "frobenius", fro)
    assert col <= bar, (tag, "worst column", col)
    assert ele <= bar, (tag, "element", ele)
    eta = None
    if check_eta:
        eta = oracle.backward_error(L, np.asfortranarray(X), np.asfortranarray(B), alpha, unit=unit)
        assert eta <= (eta_bar if eta_bar is not None else 10 * m * U), (tag, "backward error", eta)
    return fro, col, ele, eta
