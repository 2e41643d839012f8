"""The general BLAS TRSM on the GPU (hsma_trsm_general) against the oracle's
direct substitution on op(A) (Sec. 2.1's op(A) X = alpha B, either side):
every side x stored triangle x op(A) x data type x diagonal kind, at sizes on
the small path (order <= 64), the blocked path with ragged tails, and
right-hand sides wider than one 64-column panel; exact closed forms bit for
bit; padding rows untouched; alpha = 0 reads nothing."""
import itertools

import numpy as np
import pytest

import oracle
import workloads as W
from parity import U, column_rel_errors, elementwise_rel_error, padding_rows

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu
hs = pytest.importorskip("paper_2608_25469_amd")

VARIANTS = [(s, u, t) for s in "LR" for u in "LU" for t in "NTC"]


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)
    hs.lib()


def stored(M_lower, uplo):
    return np.asfortranarray((M_lower if uplo == "L" else M_lower.T).copy())


def run(A, B, alpha, side, uplo, trans, unit=False, ldb=None, lda=None):
    Ad = hs.to_colmajor(A, ld=lda)
    Bd = hs.to_colmajor(B, ld=ldb)
    if ldb is not None:
        padding_rows(Bd).fill_(W.PAD_SENTINEL)
    hs.trsm_general(Ad, Bd, alpha, side=side, uplo=uplo, trans=trans, unit=unit)
    torch.cuda.synchronize()
    pad = padding_rows(Bd).cpu().numpy() if ldb is not None else None
    return hs.from_colmajor(Bd), pad


def check(A, B, X, alpha, side, uplo, trans, unit, tag):
    ref = oracle.solve_general(A, B, alpha, side, uplo, trans, unit)
    k = B.shape[0] if side == "L" else B.shape[1]
    assert np.all(np.isfinite(X)), tag
    fro = oracle.rel_err_fro(X, ref)
    col = float(np.max(column_rel_errors(X, ref)))
    ele = elementwise_rel_error(X, ref)
    eta = oracle.backward_error_general(A, np.asfortranarray(X), B, alpha, side, uplo, trans, unit)
    assert fro <= 1e-12 and col <= 1e-12 and ele <= 1e-12, (tag, fro, col, ele)
    assert eta <= 10 * k * U, (tag, eta)


@pytest.mark.parametrize("side,uplo,trans", VARIANTS, ids=lambda v: str(v))
def test_variant_against_oracle(side, uplo, trans):
    # (k, other dimension): small path, small with a wide right-hand side,
    # blocked with ragged tails
    for k, other in ((37, 50), (64, 130), (300, 129), (1061, 77)):
        for cx in (False, True):
            for unit in (False, True):
                m, n = (k, other) if side == "L" else (other, k)
                Lk, _ = W.problem(500 + k, k, 1, cx)
                A = stored(Lk, uplo)
                B = W.rhs_matrix(np.random.default_rng(k + other), m, n, cx)
                if unit:
                    A[np.diag_indices(k)] = np.nan   # must not be read
                alpha = complex(-0.75, 0.5) if cx else 1.25
                X, _ = run(A, B, alpha, side, uplo, trans, unit)
                check(A, B, X, alpha, side, uplo, trans, unit, (side, uplo, trans, k, other, cx, unit))


@pytest.mark.parametrize("side,uplo,trans", VARIANTS, ids=lambda v: str(v))
def test_variant_exact_closed_forms(side, uplo, trans):
    """Bidiagonal and block-nilpotent operators: running sums and
    alpha (2I - op(A)) B, bit for bit, on the small and blocked paths."""
    rng = np.random.default_rng(7)
    for cx in (False, True):
        for k, other in ((40, 9), (300, 11)):
            m, n = (k, other) if side == "L" else (other, k)
            d = (1 + 1j) if cx else 4.0
            A = stored(W.bidiagonal_lower(k, d, complex_=cx), uplo)
            B = W.integer_rhs(rng, m, n, -50, 50, complex_=cx)
            X, _ = run(A, B, 1.0, side, uplo, trans)
            ref = oracle.solve_general(A, B, 1.0, side, uplo, trans)
            assert np.array_equal(X, ref), ("bidiagonal", side, uplo, trans, cx, k)
            m1 = k // 3
            C = W.integer_rhs(rng, k - m1, m1, -2, 2, complex_=cx)
            An = stored(W.block_nilpotent(m1, k - m1, C), uplo)
            An[np.diag_indices(k)] = np.nan
            X, _ = run(An, B, -1.0, side, uplo, trans, unit=True)
            ref = oracle.solve_general(An, B, -1.0, side, uplo, trans, unit=True)
            assert np.array_equal(X, ref), ("nilpotent", side, uplo, trans, cx, k)


def test_variant_leading_dimensions_padding_and_alpha_zero():
    for side, uplo, trans in itertools.product("LR", "LU", "NTC"):
        for cx in (False, True):
            k, other = (150, 20)
            m, n = (k, other) if side == "L" else (other, k)
            Lk, _ = W.problem(41, k, 1, cx)
            A = stored(Lk, uplo)
            B = W.rhs_matrix(np.random.default_rng(3), m, n, cx)
            X, pad = run(A, B, 1.0, side, uplo, trans, ldb=m + 5, lda=k + 3)
            assert np.all(pad == W.PAD_SENTINEL), (side, uplo, trans, cx)
            check(A, B, X, 1.0, side, uplo, trans, False, ("ld", side, uplo, trans, cx))
            An = np.full(A.shape, np.nan, dtype=A.dtype, order="F")
            Bn = np.full(B.shape, np.nan, dtype=B.dtype, order="F")
            X0, _ = run(An, Bn, 0.0, side, uplo, trans)
            assert np.all(X0 == 0), ("alpha 0", side, uplo, trans, cx)
