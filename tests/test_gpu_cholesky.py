"""Cholesky factorization on the library's TRSM (the second workload: the
right-side conjugate-transpose TRSM inside a recursive potrf) and the
two-TRSM solve, against the oracle's column Cholesky and its two
substitutions."""
import numpy as np
import pytest

import oracle
import workloads as W
from parity import column_rel_errors, elementwise_rel_error

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu
hs = pytest.importorskip("paper_2608_25469_amd")

U = 2.0 ** -53


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)
    hs.lib()


def hpd(n, cx, seed):
    """A = M M^H / n + I: Hermitian positive definite, kappa ~ 5."""
    rng = np.random.default_rng(seed)
    M = rng.standard_normal((n, n)) + (1j * rng.standard_normal((n, n)) if cx else 0)
    return np.asfortranarray(M @ M.conj().T / n + np.eye(n))


@pytest.mark.parametrize("cx", [False, True], ids=["dpotrf", "zpotrf"])
def test_potrf_against_oracle(cx):
    for n in (1, 17, 64, 65, 128, 300, 1000, 2049):
        A = hpd(n, cx, 100 + n)
        Ap = A.copy(order="F")
        Ap[np.triu_indices(n, 1)] = np.nan          # must be neither read nor written
        Ad = hs.to_colmajor(Ap)
        hs.potrf(Ad)
        torch.cuda.synchronize()
        G = hs.from_colmajor(Ad)
        assert np.all(np.isnan(G[np.triu_indices(n, 1)])), ("upper touched", n, cx)
        Lg = np.tril(G)
        ref, info = oracle.potrf(A)
        assert info == 0
        Lr = np.tril(ref)
        fro = np.linalg.norm(Lg - Lr) / np.linalg.norm(Lr)
        col = float(np.max(column_rel_errors(Lg, Lr)))
        ele = elementwise_rel_error(Lg, Lr)
        assert fro <= 1e-12 and col <= 1e-12 and ele <= 1e-12, (n, cx, fro, col, ele)
        # backward error of the factorization: ||L L^H - A|| / ||A|| <= 10 n u
        res = np.linalg.norm(Lg @ Lg.conj().T - A, np.inf) / np.linalg.norm(A, np.inf)
        assert res <= 10 * n * U, (n, cx, res)


def test_potrf_exact_integer_factor():
    """L with a power-of-two diagonal and small integer entries: every step of
    factoring A = L L^H is exact in the base kernel, so L comes back bit for
    bit."""
    rng = np.random.default_rng(9)
    for cx in (False, True):
        for n in (5, 33, 64):
            L = np.zeros((n, n), dtype=np.complex128 if cx else np.float64)
            for j in range(n):
                L[j, j] = float(rng.choice([1.0, 2.0, 4.0]))
                for i in range(j + 1, n):
                    L[i, j] = float(rng.integers(-2, 3)) + (1j * float(rng.integers(-2, 3)) if cx else 0)
            A = np.asfortranarray(L @ L.conj().T)
            Ad = hs.to_colmajor(A)
            hs.potrf(Ad)
            torch.cuda.synchronize()
            assert np.array_equal(np.tril(hs.from_colmajor(Ad)), L), (n, cx)


@pytest.mark.parametrize("cx", [False, True], ids=["real", "complex"])
def test_potrs_against_oracle(cx):
    for n, nrhs in ((40, 7), (300, 33), (1500, 100)):
        A = hpd(n, cx, 200 + n)
        B = W.rhs_matrix(np.random.default_rng(n), n, nrhs, cx)
        Ad, Bd = hs.to_colmajor(A), hs.to_colmajor(B)
        hs.potrf(Ad)
        hs.potrs(Ad, Bd)
        torch.cuda.synchronize()
        X = hs.from_colmajor(Bd)
        Lr, _ = oracle.potrf(A)
        Xr = oracle.cholesky_solve(np.asfortranarray(np.tril(Lr)), B)
        fro = oracle.rel_err_fro(X, Xr)
        col = float(np.max(column_rel_errors(X, Xr)))
        assert fro <= 1e-12 and col <= 1e-12, (n, cx, fro, col)
        Xn = np.linalg.solve(A, B)
        assert oracle.rel_err_fro(X, Xn) <= 1e-11, (n, cx)


def test_potrf_validation():
    A = hs.to_colmajor(np.eye(4))
    with pytest.raises(hs.HsmaError) as e:
        hs.potrf(A.float())
    assert e.value.status in (2, 6)
