"""Single-precision solves (STRSM, CTRSM; the paper's other two data types,
Sec. 5) on the GPU against the oracle.

The library computes in FP32 (FP32 matrix cores and FP32 accumulation), the
oracle in FP64 on the same FP32 inputs (promoted exactly), so the oracle's
result is the exact answer of the FP32 problem to ~1e-16.  Bars, from FP32
arithmetic (u = 2^-24) as the FP64 bars are from FP64 arithmetic:
  - normwise backward error (oracle Dot2 residual of the FP32 result)
    <= 10 k u, k the order of the triangular matrix;
  - relative error against the oracle, Frobenius, per column and per element,
    <= kappa_inf(op(A)) * 10 k u (the backward error times the condition
    number bounds the forward error);
  - exact closed forms (integer data, partial sums below 2^24) bit for bit.
"""
import numpy as np
import pytest

import oracle
import workloads as W
from parity import column_rel_errors, elementwise_rel_error, padding_rows

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu
hs = pytest.importorskip("paper_2608_25469_amd")

U32 = 2.0 ** -24
VARIANTS = [(s, u, t) for s in "LR" for u in "LU" for t in "NTC"]


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)
    hs.lib()


def f32(a):
    return np.asfortranarray(a.astype(np.complex64 if np.iscomplexobj(a) else np.float32))


def f64(a):
    return np.asfortranarray(a.astype(np.complex128 if np.iscomplexobj(a) else np.float64))


def kappa_lower(L64, unit):
    """max(kappa_inf, kappa_1) of tril(L) (unit diagonal as 1), through the
    oracle's inverse; kappa_1 is kappa_inf of the transpose, so this bounds
    every op(A) of the general solves too."""
    k = L64.shape[0]
    Lz = np.tril(np.nan_to_num(L64, nan=0.0))
    if unit:
        Lz[np.diag_indices(k)] = 1.0
    inv = oracle.solve(L64, np.asfortranarray(np.eye(k, dtype=L64.dtype)), 1.0, unit=unit)
    k_inf = np.max(np.sum(np.abs(Lz), axis=1)) * np.max(np.sum(np.abs(inv), axis=1))
    k_one = np.max(np.sum(np.abs(Lz), axis=0)) * np.max(np.sum(np.abs(inv), axis=0))
    return max(k_inf, k_one)


def check(L32, B32, X32, alpha, unit, tag, kappa, general=None):
    L64, B64, X64 = f64(L32), f64(B32), f64(X32)
    if general is None:
        ref = oracle.solve(L64, B64, alpha, unit=unit)
        eta = oracle.backward_error(L64, X64, B64, alpha, unit=unit)
        k = B32.shape[0]
    else:
        side, uplo, trans = general
        ref = oracle.solve_general(L64, B64, alpha, side, uplo, trans, unit)
        eta = oracle.backward_error_general(L64, X64, B64, alpha, side, uplo, trans, unit)
        k = B32.shape[0] if side == "L" else B32.shape[1]
    assert np.all(np.isfinite(X64)), tag
    bar_eta = 10 * k * U32
    bar = kappa * bar_eta
    fro = oracle.rel_err_fro(X64, ref)
    col = float(np.max(column_rel_errors(X64, ref)))
    ele = elementwise_rel_error(X64, ref)
    assert eta <= bar_eta, (tag, "backward error", eta, bar_eta)
    assert fro <= bar and col <= bar and ele <= bar, (tag, fro, col, ele, bar)
    return fro, eta


def run(L32, B32, alpha, unit=False, block_size=0, path=0, ldb=None):
    Ld = hs.to_colmajor(L32)
    Bd = hs.to_colmajor(B32, ld=ldb)
    if ldb is not None:
        padding_rows(Bd).fill_(W.PAD_SENTINEL)
    _, rep = hs.trsm(Ld, Bd, alpha, unit=unit, block_size=block_size, path=path, report=True)
    torch.cuda.synchronize()
    pad = padding_rows(Bd).cpu().numpy() if ldb is not None else None
    return hs.from_colmajor(Bd), rep, pad


@pytest.mark.parametrize("cx", [False, True], ids=["strsm", "ctrsm"])
@pytest.mark.parametrize("unit", [False, True], ids=["nonunit", "unit"])
def test_single_small_every_m(cx, unit):
    alpha = complex(0.75, -0.5) if cx else -1.5
    for m in range(1, 65):
        L, _ = W.problem(3000 + m, m, 1, cx)
        L32 = f32(L)
        kap = kappa_lower(f64(L32), unit)
        for n in (1, 13, 64, 65, 130):
            B32 = f32(W.rhs_matrix(np.random.default_rng(m * 7 + n), m, n, cx))
            X, rep, _ = run(L32, B32, alpha, unit=unit)
            assert rep["path"] == 1
            check(L32, B32, X, alpha, unit, ("small", m, n, cx, unit), kap)


@pytest.mark.parametrize("cx", [False, True], ids=["strsm", "ctrsm"])
@pytest.mark.parametrize("ib", [16, 32, 64, 128, 256])
def test_single_blocked_sizes(cx, ib):
    alpha = complex(-1.0, 0.25) if cx else -1.0
    for m, n in ((65, 7), (129, 33), (300, 129), (1061, 200)):
        for unit in (False, True):
            L, B = W.problem(4000 + m + ib, m, n, cx)
            L32, B32 = f32(L), f32(B)
            kap = kappa_lower(f64(L32), unit)
            X, rep, _ = run(L32, B32, alpha, unit=unit, block_size=ib)
            assert rep["path"] == 2 and rep["block_size"] == ib
            check(L32, B32, X, alpha, unit, ("blocked", m, n, cx, ib, unit), kap)


@pytest.mark.parametrize("ib", [0, 16, 64, 256])
def test_single_exact(ib):
    """Bidiagonal L = d(I - S): X = (alpha/d) cumsum(B); [[I, 0], [C, I]]:
    X = B with the lower part minus C times the upper; exact in FP32."""
    rng = np.random.default_rng(12)
    for m in (40, 300, 777):
        if (ib == 0) != (m <= 64):
            continue
        B = W.integer_rhs(rng, m, 9, -50, 50)
        X, _, _ = run(f32(W.bidiagonal_lower(m, 4.0)), f32(B), 2.0, block_size=ib)
        assert np.array_equal(X, f32(np.cumsum(B, axis=0) * 0.5)), (m, ib)
        Bc = W.integer_rhs(rng, m, 9, -50, 50, complex_=True)
        Xc, _, _ = run(f32(W.bidiagonal_lower(m, 1 + 1j, complex_=True)), f32(Bc), 1.0, block_size=ib)
        assert np.array_equal(Xc, f32(np.cumsum(Bc, axis=0) * (0.5 - 0.5j))), (m, ib, "cx")
        m1 = m // 3
        C = W.integer_rhs(rng, m - m1, m1, -2, 2)
        Ln = W.block_nilpotent(m1, m - m1, C)
        expect = B.copy()
        expect[m1:] = B[m1:] - C @ B[:m1]
        Xn, _, _ = run(f32(Ln), f32(B), 1.0, block_size=ib)
        assert np.array_equal(Xn, f32(expect)), (m, ib, "nilpotent")


def test_single_alpha_zero_padding_and_rejections():
    for m, ib in ((37, 0), (150, 32)):
        for cx in (False, True):
            L, B = W.problem(9, m, 20, cx)
            L32, B32 = f32(L), f32(B)
            X, _, pad = run(L32, B32, 1.0, block_size=ib, ldb=m + 11)
            assert np.all(pad == np.float32(W.PAD_SENTINEL)), (m, cx)
            check(L32, B32, X, 1.0, False, ("pad", m, cx), kappa_lower(f64(L32), False))
            Ln = np.full(L32.shape, np.nan, dtype=L32.dtype, order="F")
            Bn = np.full(B32.shape, np.nan, dtype=B32.dtype, order="F")
            X0, _, _ = run(Ln, Bn, 0.0)
            assert np.all(X0 == 0)
    L, B = W.problem(1, 100, 10, False)
    Ld, Bd = hs.to_colmajor(f32(L)), hs.to_colmajor(f32(B))
    for kw in ({"mixed": True}, {"refine_steps": 1}, {"backward_error": True}):
        with pytest.raises(hs.HsmaError) as e:
            hs.trsm(Ld, Bd, 1.0, **kw)
        assert e.value.status == 6, kw


@pytest.mark.parametrize("side,uplo,trans", VARIANTS, ids=lambda v: str(v))
def test_single_general_variants(side, uplo, trans):
    for k, other in ((37, 50), (300, 70)):
        for cx in (False, True):
            m, n = (k, other) if side == "L" else (other, k)
            Lk, _ = W.problem(600 + k, k, 1, cx)
            A = f32(Lk if uplo == "L" else np.asfortranarray(Lk.T))
            B = f32(W.rhs_matrix(np.random.default_rng(k + other), m, n, cx))
            alpha = complex(-0.75, 0.5) if cx else 1.25
            Ad, Bd = hs.to_colmajor(A), hs.to_colmajor(B)
            hs.trsm_general(Ad, Bd, alpha, side=side, uplo=uplo, trans=trans)
            torch.cuda.synchronize()
            X = hs.from_colmajor(Bd)
            kap = kappa_lower(f64(f32(Lk)), False)
            check(A, B, X, alpha, False, ("general", side, uplo, trans, k, cx), kap,
                  general=(side, uplo, trans))
