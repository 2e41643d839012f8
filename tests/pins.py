"""The oracle's pins: checks that tie the CPU oracle to facts fixed by the paper
and by the mathematics, not to itself.

Each ``pin_*`` function takes an oracle front end (``oracle.OracleLib``) and
raises AssertionError on failure.  ``test_oracle_pins.py`` runs them on the
real oracle; ``test_oracle_mutants.py`` runs them on deliberately broken copies
and checks that every planted mistake trips at least one pin.

The operation is x_ij = (alpha b_ij - sum_{k<i} l_ik x_kj) / l_ii (paper,
Sec. 2.1 and Sec. 4.2.1) with BLAS conventions for what the paper leaves open.
"""
from __future__ import annotations

import itertools
import math
from fractions import Fraction

import numpy as np

import workloads as W

U = 2.0 ** -53


def _bits_equal(a: np.ndarray, b: np.ndarray) -> bool:
    """Exact equality of every value (no tolerance; +0 and -0 compare equal)."""
    a = np.asarray(a)
    b = np.asarray(b)
    return a.shape == b.shape and bool(np.all(np.isfinite(a))) and np.array_equal(a, b)


def _scale(alpha, B):
    """alpha * B with one rounding per real product and per sum, formed from
    separate real array operations (numpy's own complex multiply may fuse)."""
    if not np.iscomplexobj(B):
        return alpha * B
    ar, ai = float(np.real(alpha)), float(np.imag(alpha))
    re = ar * B.real - ai * B.imag
    im = ar * B.imag + ai * B.real
    out = np.empty(B.shape, dtype=np.complex128, order="F")
    out.real = re
    out.imag = im
    return out


# ---------------------------------------------------------------------------
# P1: identity L gives X = alpha B exactly
# ---------------------------------------------------------------------------
def pin_identity(orc):
    rng = np.random.default_rng(101)
    for cx in (False, True):
        for unit in (False, True):
            for m, n in ((1, 1), (7, 3), (33, 17)):
                L = W.identity_lower(m, cx, unit=unit)
                B = W.rhs_matrix(rng, m, n, cx)
                alpha = complex(0.75, -1.5) if cx else -2.5
                X = orc.solve(L, B, alpha, unit=unit)
                assert _bits_equal(X, _scale(alpha, B)), ("identity", cx, unit, m, n)


# ---------------------------------------------------------------------------
# P2: diagonal L with power-of-two entries gives x = alpha b / d exactly
# ---------------------------------------------------------------------------
def pin_diagonal(orc):
    rng = np.random.default_rng(102)
    m, n = 9, 5
    d = 2.0 ** rng.integers(-3, 4, size=m) * rng.choice([-1.0, 1.0], size=m)
    B = W.rhs_matrix(rng, m, n)
    X = orc.solve(W.diagonal_lower(d), B, 1.5)
    assert _bits_equal(X, (1.5 * B) / d[:, None])
    # Complex: d = 2^k (1+i) has inverse 2^-k (1-i)/2, exact in binary.
    k = rng.integers(-2, 3, size=m)
    dc = (2.0 ** k) * (1 + 1j)
    Bc = W.integer_rhs(rng, m, n, -50, 50, complex_=True)
    Xc = orc.solve(W.diagonal_lower(dc, complex_=True), Bc, 1.0)
    expect = Bc * (1 - 1j) * (2.0 ** -(k + 1))[:, None]
    assert _bits_equal(Xc, expect)


# ---------------------------------------------------------------------------
# P3: bidiagonal L = d (I - S) has inverse (1/d) * (lower all-ones), so
#     X = (alpha/d) * cumulative row sums of B.  Integer data keeps it exact.
# ---------------------------------------------------------------------------
def pin_bidiagonal(orc):
    rng = np.random.default_rng(103)
    for m, n in ((1, 3), (5, 4), (64, 9), (200, 6)):
        L = W.bidiagonal_lower(m, 4.0)
        B = W.integer_rhs(rng, m, n, -100, 100)
        X = orc.solve(L, B, 2.0)
        assert _bits_equal(X, np.cumsum(B, axis=0) * 0.5), ("bidiag real", m, n)
        # Complex: d = 1 + i, 1/d = (1 - i)/2.
        Lc = W.bidiagonal_lower(m, 1 + 1j, complex_=True)
        Bc = W.integer_rhs(rng, m, n, -100, 100, complex_=True)
        Xc = orc.solve(Lc, Bc, 1.0)
        assert _bits_equal(Xc, np.cumsum(Bc, axis=0) * ((1 - 1j) / 2)), ("bidiag cx", m, n)


# ---------------------------------------------------------------------------
# P4: L = [[I, 0], [C, I]] has inverse [[I, 0], [-C, I]]
# ---------------------------------------------------------------------------
def pin_block_nilpotent(orc):
    rng = np.random.default_rng(104)
    for cx in (False, True):
        for m1, m2, n in ((3, 4, 2), (16, 16, 5), (40, 25, 7)):
            C = W.integer_rhs(rng, m2, m1, -3, 3, complex_=cx)
            L = W.block_nilpotent(m1, m2, C)
            B = W.integer_rhs(rng, m1 + m2, n, -20, 20, complex_=cx)
            expect = B.copy()
            expect[m1:] = B[m1:] - C @ B[:m1]
            X = orc.solve(L, B, 1.0)
            assert _bits_equal(X, expect), ("nilpotent", cx, m1, m2)
            # The same with a unit diagonal that is NaN and must not be read.
            Lu = L.copy(order="F")
            Lu[np.diag_indices(m1 + m2)] = np.nan
            Xu = orc.solve(Lu, B, 1.0, unit=True)
            assert _bits_equal(Xu, expect), ("nilpotent unit", cx, m1, m2)


# ---------------------------------------------------------------------------
# P5: integer round trip: unit-lower integer L, integer X, B := L X exactly;
#     the solve must return X exactly while every partial sum stays integral
#     and below 2^53.
# ---------------------------------------------------------------------------
def pin_integer_roundtrip(orc):
    rng = np.random.default_rng(105)
    for cx in (False, True):
        for m, n in ((6, 3), (24, 8), (48, 5)):
            L = W.unit_lower_integer(rng, m, complex_=cx)
            X = W.integer_rhs(rng, m, n, -4, 4, complex_=cx)
            Lt = np.tril(np.nan_to_num(L, nan=0.0), -1) + np.eye(m)
            # Exact integer product (values are small integers).
            if cx:
                Lr, Li = Lt.real.astype(np.int64), Lt.imag.astype(np.int64)
                Xr, Xi = X.real.astype(np.int64), X.imag.astype(np.int64)
                B = (Lr @ Xr - Li @ Xi) + 1j * (Lr @ Xi + Li @ Xr)
            else:
                B = Lt.astype(np.int64) @ X.astype(np.int64)
            B = np.asfortranarray(B.astype(X.dtype))
            got = orc.solve(L, B, 1.0, unit=True)
            assert _bits_equal(got, X), ("roundtrip", cx, m, n)


# ---------------------------------------------------------------------------
# P6: brute force on tiny dyadic problems.  The exact solution comes from
#     Cramer's rule with rational determinants (a formula independent of
#     substitution), and the oracle's answer must satisfy the classical
#     componentwise backward-error bound of forward substitution,
#     |L x - alpha b| <= gamma_{m+1} (|L| |x| + |alpha b|),  gamma_k = k u/(1-k u),
#     checked in exact rational arithmetic.
# ---------------------------------------------------------------------------
def _det(M):
    n = len(M)
    total = Fraction(0)
    for perm in itertools.permutations(range(n)):
        sign = 1
        for i in range(n):
            for j in range(i + 1, n):
                if perm[i] > perm[j]:
                    sign = -sign
        p = Fraction(sign)
        for i in range(n):
            p *= M[i][perm[i]]
        total += p
    return total


def pin_bruteforce_rational(orc):
    rng = np.random.default_rng(106)
    for trial in range(12):
        m = int(rng.integers(1, 6))
        n = int(rng.integers(1, 4))
        Lf = np.zeros((m, m))
        for i in range(m):
            for k in range(i):
                Lf[i, k] = rng.integers(-16, 17) / 16.0
            Lf[i, i] = rng.choice([0.5, 0.75, 1.0, 1.25, 1.5, 3.0, -2.0])
        Bf = rng.integers(-64, 65, size=(m, n)) / 8.0
        alpha = float(rng.choice([1.0, -0.5, 3.0]))
        L = np.asfortranarray(Lf.copy())
        L[np.triu_indices(m, 1)] = np.nan
        X = orc.solve(L, np.asfortranarray(Bf), alpha)
        Lq = [[Fraction(Lf[i, k]) for k in range(m)] for i in range(m)]
        detL = _det(Lq)
        gamma = Fraction((m + 1)) * Fraction(U) / (1 - (m + 1) * Fraction(U))

        def cramer(rhs):
            out = []
            for i in range(m):
                Mi = [row[:] for row in Lq]
                for r in range(m):
                    Mi[r][i] = rhs[r]
                out.append(_det(Mi) / detL)
            return out

        # |inv(L)| column by column, exactly.
        absinv = [[abs(v) for v in cramer([Fraction(int(r == c)) for r in range(m)])]
                  for c in range(m)]  # absinv[c][r] = |inv(L)[r, c]|
        for j in range(n):
            rhs = [Fraction(alpha) * Fraction(Bf[i, j]) for i in range(m)]
            exact = cramer(rhs)
            xq = [Fraction(X[i, j]) for i in range(m)]
            # componentwise residual bound: |L x - alpha b| <= gamma (|L||x| + |alpha b|)
            cap = [gamma * (sum(abs(Lq[i][k]) * abs(xq[k]) for k in range(i + 1)) + abs(rhs[i]))
                   for i in range(m)]
            for i in range(m):
                r = sum(Lq[i][k] * xq[k] for k in range(i + 1)) - rhs[i]
                assert abs(r) <= cap[i], ("componentwise backward error", trial, i, j)
            # hence the forward error |x - x*| <= |inv(L)| cap
            for i in range(m):
                fe = sum(absinv[c][i] * cap[c] for c in range(m))
                assert abs(xq[i] - exact[i]) <= fe, ("cramer forward error", trial, i, j)


# ---------------------------------------------------------------------------
# P7: agreement with a library triangular solver (LAPACK trtrs via scipy)
# ---------------------------------------------------------------------------
def pin_library(orc):
    import scipy.linalg as sl
    for cx in (False, True):
        for unit in (False, True):
            for m, n in ((17, 5), (130, 40), (700, 33)):
                L, B = W.problem(7 + m, m, n, cx)
                alpha = complex(1.0, 0.5) if cx else -1.25
                X = orc.solve(L, B, alpha, unit=unit)
                ref = sl.solve_triangular(L, alpha * B, lower=True, unit_diagonal=unit,
                                          check_finite=False)
                rel = np.linalg.norm(X - ref) / np.linalg.norm(ref)
                assert rel <= 1e-13, ("scipy", cx, unit, m, n, rel)


# ---------------------------------------------------------------------------
# P8: invariants
# ---------------------------------------------------------------------------
def pin_invariants(orc):
    for cx in (False, True):
        L, B = W.problem(108, 96, 24, cx)
        a = complex(0.5, -0.25) if cx else 0.75
        X1 = orc.solve(L, B, a)
        # Linearity in alpha: doubling alpha doubles X exactly.
        X2 = orc.solve(L, B, 2 * a)
        assert _bits_equal(X2, 2 * X1)
        # Column independence: a subset of columns solves identically.
        cols = [3, 0, 17, 23]
        Xs = orc.solve(L, np.asfortranarray(B[:, cols]), a)
        assert _bits_equal(Xs, X1[:, cols])
        # Block consistency: X1 = L11^-1 a B1, X2 = L22^-1 (a B2 - L21 X1).
        h = 40
        top = orc.solve(np.asfortranarray(L[:h, :h]), np.asfortranarray(B[:h]), a)
        L21 = L[h:, :h]
        rhs = np.asfortranarray(a * B[h:] - L21 @ top)
        bot = orc.solve(np.asfortranarray(L[h:, h:]), rhs, 1.0)
        full = np.vstack([top, bot])
        assert np.linalg.norm(full - X1) / np.linalg.norm(X1) <= 1e-13
        # Row (dot) form and column (axpy) form agree to rounding.
        Xr = orc.solve(L, B, a, rowform=True)
        assert np.linalg.norm(Xr - X1) / np.linalg.norm(X1) <= 1e-13
        Xru = orc.solve(L, B, a, unit=True, rowform=True)
        Xcu = orc.solve(L, B, a, unit=True)
        assert np.linalg.norm(Xru - Xcu) / np.linalg.norm(Xcu) <= 1e-13


# ---------------------------------------------------------------------------
# alpha = 0: B is zeroed and neither A nor B is read (NaN inputs stay out).
# ---------------------------------------------------------------------------
def pin_alpha_zero(orc):
    for cx in (False, True):
        m, n = 6, 4
        L = np.full((m, m), np.nan, dtype=np.complex128 if cx else np.float64, order="F")
        B = np.full((m, n), np.nan, dtype=L.dtype, order="F")
        X = orc.solve(L, B, 0.0)
        assert np.all(X == 0) and not np.any(np.signbit(X.real))


# ---------------------------------------------------------------------------
# The backward-error checker against closed forms: zero for an exact
# solution; for X = X* + delta e_p e_q^T it is |delta| max_r |l_rp| over the
# denominator computed from the norms directly.
# ---------------------------------------------------------------------------
def pin_backward_error_checker(orc):
    rng = np.random.default_rng(109)
    for cx in (False, True):
        m, n = 12, 5
        L = W.unit_lower_integer(rng, m, complex_=cx)
        Lt = np.tril(np.nan_to_num(L, nan=0.0), -1) + np.eye(m)
        X = W.integer_rhs(rng, m, n, -3, 3, complex_=cx)
        B = np.asfortranarray(Lt @ X)  # small integers: exact in float
        assert orc.backward_error(L, X, B, 1.0, unit=True) == 0.0
        p, q, delta = 4, 2, 2.0 ** -10
        Xp = X.copy(order="F")
        Xp[p, q] += delta
        eta = orc.backward_error(L, Xp, B, 1.0, unit=True)
        num = delta * np.max(np.abs(Lt[:, p]))
        den = np.max(np.abs(Lt).sum(1)) * np.max(np.abs(Xp).sum(1)) + np.max(np.abs(B).sum(1))
        assert abs(eta - num / den) <= 1e-14 * (num / den), (cx, eta, num / den)


# ---------------------------------------------------------------------------
# The general BLAS TRSM: op(A) X = alpha B (left) or X op(A) = alpha B
# (right), A's lower or upper triangle stored, op(A) = A, A^T or A^H.
# ---------------------------------------------------------------------------
VARIANTS = [(side, uplo, trans) for side in "LR" for uplo in "LU" for trans in "NTC"]


def _stored(M_lower, uplo):
    """A holding the lower-triangular M (uplo "L") or its transpose M^T, an
    upper-triangular matrix (uplo "U"); the other triangle stays NaN."""
    A = M_lower if uplo == "L" else M_lower.T
    return np.asfortranarray(A.copy())


def _dense_op(A, uplo, trans):
    """op(A) as a dense array with zeros outside the stored triangle."""
    k = A.shape[0]
    Z = np.where(np.tril(np.ones((k, k), bool)) if uplo == "L" else np.triu(np.ones((k, k), bool)),
                 A, 0)
    if trans == "N":
        return Z
    if trans == "T":
        return Z.T
    return Z.conj().T


def _op_is_lower(uplo, trans):
    return (uplo == "L") == (trans == "N")


def pin_general_bidiagonal(orc):
    """op(A) bidiagonal, d'(I - S) or d'(I - S^T) (S the sub-diagonal shift),
    has inverse (1/d') times the lower or upper all-ones triangle, so X is a
    running sum of B: down the rows on the left, along the columns on the
    right, from the end the triangle starts at.  Exact with integer B."""
    rng = np.random.default_rng(110)
    for side, uplo, trans in VARIANTS:
        for cx in (False, True):
            d = (1 + 1j) if cx else 4.0
            alpha = 1.0 if cx else 2.0
            for m, n in ((1, 3), (5, 4), (29, 6)):
                k = m if side == "L" else n
                A = _stored(W.bidiagonal_lower(k, d, complex_=cx), uplo)
                B = W.integer_rhs(rng, m, n, -100, 100, complex_=cx)
                X = orc.solve_general(A, B, alpha, side, uplo, trans)
                dp = np.conj(d) if trans == "C" else d
                scale = alpha / dp      # exact: 0.5, (1 -/+ i)/2
                ax = 0 if side == "L" else 1
                lower = _op_is_lower(uplo, trans)
                # left: lower -> prefix sums, upper -> suffix sums (down the rows);
                # right: lower -> suffix sums, upper -> prefix sums (along a row)
                prefix = lower if side == "L" else not lower
                S = np.cumsum(B, axis=ax) if prefix else \
                    np.flip(np.cumsum(np.flip(B, axis=ax), axis=ax), axis=ax)
                assert _bits_equal(X, S * scale), ("general bidiagonal", side, uplo, trans, cx, m, n)


def pin_general_block_nilpotent(orc):
    """op(A) = I + N with N^2 = 0 (A = [[I, 0], [C, I]] or its transpose)
    has inverse I - N = 2I - op(A), so X = alpha (2I - op(A)) B on the left and
    alpha B (2I - op(A)) on the right, exactly for integer data; also with a
    NaN unit diagonal that must not be read."""
    rng = np.random.default_rng(111)
    for side, uplo, trans in VARIANTS:
        for cx in (False, True):
            for m1, m2, other in ((3, 4, 5), (17, 12, 6)):
                k = m1 + m2
                C = W.integer_rhs(rng, m2, m1, -3, 3, complex_=cx)
                A = _stored(W.block_nilpotent(m1, m2, C), uplo)
                m, n = (k, other) if side == "L" else (other, k)
                B = W.integer_rhs(rng, m, n, -20, 20, complex_=cx)
                alpha = -1.0
                inv = 2 * np.eye(k) - _dense_op(A, uplo, trans)
                expect = alpha * (inv @ B if side == "L" else B @ inv)
                X = orc.solve_general(A, B, alpha, side, uplo, trans)
                assert _bits_equal(X, expect), ("general nilpotent", side, uplo, trans, cx)
                Au = A.copy(order="F")
                Au[np.diag_indices(k)] = np.nan
                Xu = orc.solve_general(Au, B, alpha, side, uplo, trans, unit=True)
                assert _bits_equal(Xu, expect), ("general nilpotent unit", side, uplo, trans, cx)


def pin_general_bruteforce_rational(orc):
    """Every variant on tiny dyadic real problems against the exact rational
    solution (inverse by Cramer's rule): componentwise residual within
    gamma_{k+1}(|op(A)||X| + |alpha B|), which bounds the forward error."""
    rng = np.random.default_rng(112)
    for t, (side, uplo, trans) in enumerate(VARIANTS * 2):
        m = int(rng.integers(1, 5))
        n = int(rng.integers(1, 5))
        k = m if side == "L" else n
        M = np.zeros((k, k))
        for i in range(k):
            for j in range(i):
                M[i, j] = rng.integers(-16, 17) / 16.0
            M[i, i] = rng.choice([0.5, 0.75, 1.25, 1.5, 3.0, -2.0])
        Ml = M.copy()
        Ml[np.triu_indices(k, 1)] = np.nan
        A = _stored(Ml, uplo)
        Bf = rng.integers(-64, 65, size=(m, n)) / 8.0
        alpha = float(rng.choice([1.0, -0.5, 3.0]))
        X = orc.solve_general(A, np.asfortranarray(Bf), alpha, side, uplo, trans)
        Op = _dense_op(A, uplo, trans)
        Oq = [[Fraction(Op[i, j]) for j in range(k)] for i in range(k)]
        det = _det(Oq)
        inv = [[None] * k for _ in range(k)]
        for c in range(k):
            for r in range(k):
                Mi = [row[:] for row in Oq]
                for q in range(k):
                    Mi[q][r] = Fraction(int(q == c))
                inv[r][c] = _det(Mi) / det
        gamma = Fraction(k + 1) * Fraction(U) / (1 - (k + 1) * Fraction(U))
        Xq = [[Fraction(X[i, j]) for j in range(n)] for i in range(m)]
        Bq = [[Fraction(alpha) * Fraction(Bf[i, j]) for j in range(n)] for i in range(m)]
        if side == "L":
            res = [[sum(Oq[i][q] * Xq[q][j] for q in range(k)) - Bq[i][j] for j in range(n)]
                   for i in range(m)]
            cap = [[gamma * (sum(abs(Oq[i][q]) * abs(Xq[q][j]) for q in range(k)) + abs(Bq[i][j]))
                    for j in range(n)] for i in range(m)]
            exact = [[sum(inv[i][q] * Bq[q][j] for q in range(k)) for j in range(n)] for i in range(m)]
            fe = [[sum(abs(inv[i][q]) * cap[q][j] for q in range(k)) for j in range(n)]
                  for i in range(m)]
        else:
            res = [[sum(Xq[i][q] * Oq[q][j] for q in range(k)) - Bq[i][j] for j in range(n)]
                   for i in range(m)]
            cap = [[gamma * (sum(abs(Xq[i][q]) * abs(Oq[q][j]) for q in range(k)) + abs(Bq[i][j]))
                    for j in range(n)] for i in range(m)]
            exact = [[sum(Bq[i][q] * inv[q][j] for q in range(k)) for j in range(n)] for i in range(m)]
            fe = [[sum(cap[i][q] * abs(inv[q][j]) for q in range(k)) for j in range(n)]
                  for i in range(m)]
        for i in range(m):
            for j in range(n):
                assert abs(res[i][j]) <= cap[i][j], ("general residual", t, side, uplo, trans, i, j)
                assert abs(Xq[i][j] - exact[i][j]) <= fe[i][j], ("general forward", t, side, uplo, trans)


def pin_general_library(orc):
    """Every variant against LAPACK trtrs (scipy): left side directly; right
    side through X op(A) = alpha B  <=>  op(A)^T X^T = alpha B^T."""
    import scipy.linalg as sl
    for side, uplo, trans in VARIANTS:
        for cx in (False, True):
            for unit in (False, True):
                for m, n in ((17, 9), (120, 40)):
                    k = m if side == "L" else n
                    Lk, _ = W.problem(8 + k, k, 1, cx)
                    B = W.rhs_matrix(np.random.default_rng(9 + m + n), m, n, cx)
                    A = _stored(Lk, uplo)
                    Z = np.nan_to_num(A, nan=0.0)
                    alpha = complex(1.0, 0.5) if cx else -1.25
                    X = orc.solve_general(A, B, alpha, side, uplo, trans, unit)
                    if side == "L":
                        ref = sl.solve_triangular(Z, alpha * B, lower=uplo == "L", trans=trans,
                                                  unit_diagonal=unit, check_finite=False)
                    elif trans == "N":
                        ref = sl.solve_triangular(Z, alpha * B.T, lower=uplo == "L", trans="T",
                                                  unit_diagonal=unit, check_finite=False).T
                    elif trans == "T":
                        ref = sl.solve_triangular(Z, alpha * B.T, lower=uplo == "L", trans="N",
                                                  unit_diagonal=unit, check_finite=False).T
                    else:
                        ref = sl.solve_triangular(Z.conj(), alpha * B.T, lower=uplo == "L",
                                                  trans="N", unit_diagonal=unit,
                                                  check_finite=False).T
                    rel = np.linalg.norm(X - ref) / np.linalg.norm(ref)
                    assert rel <= 1e-13, ("general scipy", side, uplo, trans, cx, unit, rel)


def pin_general_consistency(orc):
    """The left, lower, no-transpose case of the general solver is the
    oracle's row form, bit for bit (the same order of operations)."""
    for cx in (False, True):
        for unit in (False, True):
            L, B = W.problem(31, 70, 13, cx)
            alpha = complex(0.5, 2.0) if cx else 0.75
            X = orc.solve_general(L, B, alpha, "L", "L", "N", unit)
            Xr = orc.solve(L, B, alpha, unit=unit, rowform=True)
            assert X.tobytes() == np.asfortranarray(Xr).tobytes(), ("general vs row form", cx, unit)
            Bn = np.full((13, 70), np.nan, dtype=B.dtype, order="F")
            Ln = np.full(L.shape, np.nan, dtype=L.dtype, order="F")
            Z = orc.solve_general(Ln, Bn, 0.0, "R", "U", "C", unit)
            assert np.all(Z == 0), "alpha = 0 reads nothing"


def pin_general_backward_error_checker(orc):
    """Hand-computed values of the general checker (chosen so that a wrong
    index, a dropped absolute value or a dropped conjugation changes them)."""
    F = lambda a, dt=np.float64: np.asfortranarray(np.array(a, dtype=dt))
    nan = np.nan
    # left, lower, N: A = [[2, .], [-1, 4]], X = [1; 1], B = [3; 6]:
    # A X - B = [-1; -3], ||A|| = 5, eta = 3 / (5 * 1 + 1 * 6) = 3/11
    A = F([[2.0, nan], [-1.0, 4.0]])
    eta = orc.backward_error_general(A, F([[1.0], [1.0]]), F([[3.0], [6.0]]), 1.0, "L", "L", "N")
    assert abs(eta - 3.0 / 11.0) <= 1e-15, eta
    # right, lower, T: op(A) = A^T = [[2, -1], [0, 4]], X = [1 2], B = [3 6]:
    # X op(A) = [2 7], R = [-1 1], ||op(A)|| = 4, eta = 2 / (4 * 3 + 9) = 2/21
    eta = orc.backward_error_general(A, F([[1.0, 2.0]]), F([[3.0, 6.0]]), 1.0, "R", "L", "T")
    assert abs(eta - 2.0 / 21.0) <= 1e-15, eta
    # complex, left, lower, C: A = [[2, .], [i, 4]], op(A) = A^H = [[2, -i], [0, 4]],
    # X = [1; 1], alpha = i, B = [1; -4i]: op(A) X = [2 - i; 4], alpha B = [i; 4],
    # R = [2 - 2i; 0], eta = sqrt(8) / (4 * 1 + 1 * 4)
    Ac = F([[2.0, nan], [1j, 4.0]], np.complex128)
    X = F([[1.0], [1.0]], np.complex128)
    B = F([[1.0], [-4j]], np.complex128)
    eta = orc.backward_error_general(Ac, X, B, 1j, "L", "L", "C")
    assert abs(eta - np.sqrt(8.0) / 8.0) <= 1e-15, eta


# ---------------------------------------------------------------------------
# Cholesky factorization A = L L^H (the TRSM's consumer in the second
# workload) and the solve L L^H X = B by two triangular solves.
# ---------------------------------------------------------------------------
def _integer_factor(rng, n, cx):
    """Lower L with a power-of-two diagonal and small integer (Gaussian
    integer) entries below it; A = L L^H is then exact, and so is every step
    of the factorization of A (perfect-square pivots, divisions by powers
    of two)."""
    L = np.zeros((n, n), dtype=np.complex128 if cx else np.float64)
    for j in range(n):
        L[j, j] = float(rng.choice([1.0, 2.0, 4.0]))
        for i in range(j + 1, n):
            v = float(rng.integers(-2, 3))
            L[i, j] = v + 1j * float(rng.integers(-2, 3)) if cx else v
    A = L @ L.conj().T
    return np.asfortranarray(L), np.asfortranarray(A)


def pin_cholesky_exact(orc):
    rng = np.random.default_rng(120)
    for cx in (False, True):
        for n in (1, 2, 7, 20):
            L, A = _integer_factor(rng, n, cx)
            Au = A.copy(order="F")
            Au[np.triu_indices(n, 1)] = np.nan          # never read
            got, info = orc.potrf(Au)
            assert info == 0, ("cholesky info", cx, n, info)
            assert _bits_equal(np.tril(got), L), ("cholesky exact", cx, n)
            assert np.all(np.isnan(got[np.triu_indices(n, 1)])), ("upper touched", cx, n)


def pin_cholesky_library(orc):
    import scipy.linalg as sl
    rng = np.random.default_rng(121)
    for cx in (False, True):
        for n in (5, 64, 150):
            M = rng.standard_normal((n, n)) + (1j * rng.standard_normal((n, n)) if cx else 0)
            A = np.asfortranarray(M @ M.conj().T + n * np.eye(n))
            got, info = orc.potrf(A)
            ref = sl.cholesky(A, lower=True)
            assert info == 0
            rel = np.linalg.norm(np.tril(got) - ref) / np.linalg.norm(ref)
            assert rel <= 1e-13, ("cholesky scipy", cx, n, rel)
            B = np.asfortranarray(rng.standard_normal((n, 3)) + (1j if cx else 0) * rng.standard_normal((n, 3)))
            X = orc.cholesky_solve(np.asfortranarray(np.tril(got)), B)
            Xr = np.linalg.solve(A, B)
            rel = np.linalg.norm(X - Xr) / np.linalg.norm(Xr)
            assert rel <= 1e-12, ("cholesky solve", cx, n, rel)


def pin_cholesky_not_definite(orc):
    """The first non-positive pivot stops the factorization with its
    1-based column index."""
    for cx in (False, True):
        A = np.asfortranarray(np.diag([4.0, 9.0, 1.0, -1.0, 16.0]).astype(np.complex128 if cx else np.float64))
        _, info = orc.potrf(A)
        assert info == 4, ("not definite", cx, info)
        A = np.asfortranarray(np.array([[1.0, 2.0], [2.0, 1.0]], dtype=np.complex128 if cx else np.float64))
        _, info = orc.potrf(A)          # pivot 1 - 4 = -3 in column 2
        assert info == 2, ("not definite 2x2", cx, info)


# Cheap pins first: the mutant test stops at the first pin that fails.
ALL_PINS = [
    pin_identity, pin_diagonal, pin_bidiagonal, pin_block_nilpotent,
    pin_integer_roundtrip, pin_alpha_zero, pin_backward_error_checker,
    pin_general_bidiagonal, pin_general_block_nilpotent, pin_general_consistency,
    pin_general_backward_error_checker, pin_general_bruteforce_rational,
    pin_cholesky_exact, pin_cholesky_not_definite,
    pin_bruteforce_rational, pin_invariants, pin_library, pin_general_library,
    pin_cholesky_library,
]
