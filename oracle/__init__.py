"""CPU oracle for left-side, lower-triangular, no-transpose TRSM, and for the
general BLAS TRSM (either side, either stored triangle, op(A) = A, A^T, A^H).

TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the
benchmark's CPU-baseline leg may import this package.  The GPU library never
imports it, and it never imports the GPU library.

The arithmetic lives in ``trsm_oracle.c`` (plain C, fp64, compiled with
``-ffp-contract=off``); this module only compiles it with gcc and marshals
numpy arrays to it.  Every function follows the forward-substitution equation
of the paper (Sec. 2.1 and Sec. 4.2.1): x_ij = (alpha b_ij - sum_{k<i} l_ik
x_kj) / l_ii, under BLAS TRSM conventions for the points the paper leaves open
(column-major storage, unit diagonal never read, alpha == 0 zero-fills B).

Arrays are numpy arrays in Fortran (column-major) order: float64 for real
problems, complex128 for complex ones.  B is overwritten in place, exactly as
the library does.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "trsm_oracle.c")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lock = threading.Lock()
_lib = None

_CFLAGS = ["-O2", "-fopenmp", "-ffp-contract=off", "-fno-fast-math",
           "-fPIC", "-shared", "-std=c11"]


def build(force: bool = True) -> str:
    """Compile the oracle with gcc into ``oracle/liboracle.so``."""
    if not force and os.path.exists(_LIB_PATH) and \
            os.path.getmtime(_LIB_PATH) >= os.path.getmtime(_SRC):
        return _LIB_PATH
    tmp = _LIB_PATH + ".tmp%d" % os.getpid()
    subprocess.check_call(["gcc", *_CFLAGS, _SRC, "-o", tmp, "-lm"])
    os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _bind(lib):
    i64, dp, c_int = ctypes.c_int64, ctypes.c_void_p, ctypes.c_int
    for name in ("oracle_trsm_d", "oracle_trsm_d_rowform"):
        f = getattr(lib, name)
        f.argtypes = [c_int, i64, i64, ctypes.c_double, dp, i64, dp, i64]
        f.restype = None
    for name in ("oracle_trsm_z", "oracle_trsm_z_rowform"):
        f = getattr(lib, name)
        f.argtypes = [c_int, i64, i64, dp, dp, i64, dp, i64]
        f.restype = None
    lib.oracle_backward_error_d.argtypes = [c_int, i64, i64, ctypes.c_double, dp, i64,
                                            dp, i64, dp, i64, dp]
    lib.oracle_backward_error_d.restype = ctypes.c_double
    lib.oracle_backward_error_z.argtypes = [c_int, i64, i64, dp, dp, i64,
                                            dp, i64, dp, i64, dp]
    lib.oracle_backward_error_z.restype = ctypes.c_double
    for name in ("oracle_trsm_general_d",):
        f = getattr(lib, name)
        f.argtypes = [c_int, c_int, c_int, c_int, i64, i64, ctypes.c_double, dp, i64, dp, i64]
        f.restype = None
    lib.oracle_trsm_general_z.argtypes = [c_int, c_int, c_int, c_int, i64, i64, dp, dp, i64, dp, i64]
    lib.oracle_trsm_general_z.restype = None
    lib.oracle_backward_error_general.argtypes = [c_int, c_int, c_int, c_int, c_int, i64, i64, dp,
                                                  dp, i64, dp, i64, dp, i64, dp]
    lib.oracle_backward_error_general.restype = ctypes.c_double
    for name in ("oracle_potrf_d", "oracle_potrf_z"):
        f = getattr(lib, name)
        f.argtypes = [i64, dp, i64]
        f.restype = c_int
    lib.oracle_num_threads.argtypes = []
    lib.oracle_num_threads.restype = c_int
    lib.oracle_set_num_threads.argtypes = [c_int]
    lib.oracle_set_num_threads.restype = None
    return lib


def _ptr(a: np.ndarray) -> int:
    return a.ctypes.data


def _check_fortran(name, a, dtype):
    if not isinstance(a, np.ndarray) or a.dtype != dtype:
        raise TypeError(f"{name} must be a numpy {np.dtype(dtype)} array")
    if a.ndim != 2:
        raise ValueError(f"{name} must be 2-D")
    if a.size and not a.flags.f_contiguous:
        # Allow column-major views with a leading dimension (strided columns).
        es = a.itemsize
        if a.strides[0] != es or a.strides[1] % es:
            raise ValueError(f"{name} must be column-major with unit row stride")


def _ld(a: np.ndarray) -> int:
    if a.shape[1] <= 1:
        return max(1, a.shape[0])
    return a.strides[1] // a.itemsize


class OracleLib:
    """numpy front end over one compiled copy of ``trsm_oracle.c``."""

    def __init__(self, path: str):
        self.path = path
        self.lib = _bind(ctypes.CDLL(path))

    def num_threads(self) -> int:
        return self.lib.oracle_num_threads()

    def set_num_threads(self, t: int) -> None:
        self.lib.oracle_set_num_threads(int(t))

    def trsm(self, L: np.ndarray, B: np.ndarray, alpha=1.0, unit: bool = False,
             rowform: bool = False) -> np.ndarray:
        """Overwrite B (m x n, column-major) with alpha * inv(tril(L)) * B.

        L is m x m (only its lower triangle is read; its diagonal is not read
        when ``unit``).  ``rowform`` selects the literal row (dot-product) order
        of the paper's equation instead of the column (axpy) order; both
        compute the same function and exist so the tests can compare them.
        """
        lib = self.lib
        if B.dtype == np.float64:
            _check_fortran("L", L, np.float64)
            _check_fortran("B", B, np.float64)
            m, n = B.shape
            if L.shape[0] != m or L.shape[1] < m:
                raise ValueError("L must be at least m x m")
            if np.iscomplexobj(alpha) and np.imag(alpha) != 0:
                raise ValueError("complex alpha with a real problem")
            f = lib.oracle_trsm_d_rowform if rowform else lib.oracle_trsm_d
            f(int(bool(unit)), m, n, float(np.real(alpha)), _ptr(L), _ld(L), _ptr(B), _ld(B))
            return B
        if B.dtype == np.complex128:
            _check_fortran("L", L, np.complex128)
            _check_fortran("B", B, np.complex128)
            m, n = B.shape
            if L.shape[0] != m or L.shape[1] < m:
                raise ValueError("L must be at least m x m")
            al = np.array([np.real(alpha), np.imag(alpha)], dtype=np.float64)
            f = lib.oracle_trsm_z_rowform if rowform else lib.oracle_trsm_z
            f(int(bool(unit)), m, n, _ptr(al), _ptr(L), _ld(L), _ptr(B), _ld(B))
            return B
        raise TypeError("B must be float64 or complex128")

    def solve(self, L: np.ndarray, B: np.ndarray, alpha=1.0, unit: bool = False,
              rowform: bool = False) -> np.ndarray:
        """Out-of-place convenience: returns alpha * inv(tril(L)) * B."""
        X = np.array(B, dtype=B.dtype, order="F", copy=True)
        return self.trsm(L, X, alpha=alpha, unit=unit, rowform=rowform)

    def backward_error(self, L: np.ndarray, X: np.ndarray, B0: np.ndarray, alpha=1.0,
                       unit: bool = False) -> float:
        """eta = ||L X - alpha B0||_inf / (||L||_inf ||X||_inf + |alpha| ||B0||_inf).

        The residual is formed with compensated (Dot2) dot products; norms are
        the maximum absolute row sums (complex modulus for complex data).  Only
        the lower triangle of L is used, with a unit diagonal when ``unit``.
        """
        lib = self.lib
        m, n = X.shape
        if B0.shape != (m, n):
            raise ValueError("X and B0 must have the same shape")
        if X.dtype == np.float64:
            for nm, a in (("L", L), ("X", X), ("B0", B0)):
                _check_fortran(nm, a, np.float64)
            R = np.empty((m, n), dtype=np.float64, order="F")
            return lib.oracle_backward_error_d(int(bool(unit)), m, n, float(np.real(alpha)),
                                               _ptr(L), _ld(L), _ptr(X), _ld(X),
                                               _ptr(B0), _ld(B0), _ptr(R))
        if X.dtype == np.complex128:
            for nm, a in (("L", L), ("X", X), ("B0", B0)):
                _check_fortran(nm, a, np.complex128)
            R = np.empty((m, n), dtype=np.complex128, order="F")
            al = np.array([np.real(alpha), np.imag(alpha)], dtype=np.float64)
            return lib.oracle_backward_error_z(int(bool(unit)), m, n, _ptr(al),
                                               _ptr(L), _ld(L), _ptr(X), _ld(X),
                                               _ptr(B0), _ld(B0), _ptr(R))
        raise TypeError("X must be float64 or complex128")


    def trsm_general(self, A, B, alpha=1.0, side="L", uplo="L", trans="N", unit=False):
        """General BLAS TRSM in place on B: op(A) X = alpha B (side "L") or
        X op(A) = alpha B (side "R"); ``uplo`` names the stored triangle of A and
        ``trans`` is "N", "T" or "C" (conjugate transpose).  Direct substitution
        on op(A) (trsm_oracle.c, "The general BLAS TRSM")."""
        lib = self.lib
        sd, ul, tr = _general_codes(side, uplo, trans)
        m, n = _general_shapes(A, B, sd)
        if B.dtype == np.float64:
            _check_fortran("A", A, np.float64)
            _check_fortran("B", B, np.float64)
            if np.imag(alpha) != 0:
                raise ValueError("complex alpha for real data")
            lib.oracle_trsm_general_d(sd, ul, tr, int(bool(unit)), m, n, float(np.real(alpha)),
                                      _ptr(A), _ld(A), _ptr(B), _ld(B))
            return B
        if B.dtype == np.complex128:
            _check_fortran("A", A, np.complex128)
            _check_fortran("B", B, np.complex128)
            al = np.array([np.real(alpha), np.imag(alpha)], dtype=np.float64)
            lib.oracle_trsm_general_z(sd, ul, tr, int(bool(unit)), m, n, _ptr(al), _ptr(A), _ld(A),
                                      _ptr(B), _ld(B))
            return B
        raise TypeError("B must be float64 or complex128")


    def solve_general(self, A, B, alpha=1.0, side="L", uplo="L", trans="N", unit=False):
        """Out-of-place :func:`trsm_general`."""
        X = np.array(B, dtype=B.dtype, order="F", copy=True)
        return self.trsm_general(A, X, alpha, side, uplo, trans, unit)


    def backward_error_general(self, A, X, B0, alpha=1.0, side="L", uplo="L", trans="N",
                               unit=False) -> float:
        """eta = ||R||_inf / (||op(A)||_inf ||X||_inf + |alpha| ||B0||_inf) with
        R = op(A) X - alpha B0 (left) or X op(A) - alpha B0 (right), Dot2 residual."""
        lib = self.lib
        sd, ul, tr = _general_codes(side, uplo, trans)
        m, n = _general_shapes(A, X, sd)
        if B0.shape != (m, n):
            raise ValueError("X and B0 must have the same shape")
        cx = X.dtype == np.complex128
        dt = np.complex128 if cx else np.float64
        for nm, a in (("A", A), ("X", X), ("B0", B0)):
            _check_fortran(nm, a, dt)
        R = np.empty((m, n), dtype=dt, order="F")
        al = np.array([np.real(alpha), np.imag(alpha)], dtype=np.float64)
        return lib.oracle_backward_error_general(int(cx), sd, ul, tr, int(bool(unit)), m, n, _ptr(al),
                                                 _ptr(A), _ld(A), _ptr(X), _ld(X), _ptr(B0), _ld(B0),
                                                 _ptr(R))


    def potrf(self, A):
        """Cholesky factor of a Hermitian positive definite A (lower triangle
        read): returns (L, info) with L's strict upper triangle as given."""
        L = np.array(A, dtype=A.dtype, order="F", copy=True)
        n = L.shape[0]
        if L.shape[1] < n:
            raise ValueError("A must be n x n")
        if L.dtype == np.float64:
            info = self.lib.oracle_potrf_d(n, _ptr(L), _ld(L))
        elif L.dtype == np.complex128:
            info = self.lib.oracle_potrf_z(n, _ptr(L), _ld(L))
        else:
            raise TypeError("A must be float64 or complex128")
        return L, int(info)

    def cholesky_solve(self, L, B):
        """X with L L^H X = B: L Y = B, then L^H X = Y (two triangular solves)."""
        Y = self.solve(L, B, 1.0)
        return self.solve_general(L, Y, 1.0, "L", "L", "C")


SIDES = {"L": 0, "R": 1}
UPLOS = {"L": 0, "U": 1}
TRANS = {"N": 0, "T": 1, "C": 2}


def _general_codes(side, uplo, trans):
    return SIDES[side.upper()], UPLOS[uplo.upper()], TRANS[trans.upper()]


def _general_shapes(A, B, side):
    m, n = B.shape
    ka = m if side == 0 else n
    if A.shape[0] != ka or A.shape[1] < ka:
        raise ValueError(f"A must be {ka} x {ka}")
    return m, n


def trsm_general(A, B, alpha=1.0, side="L", uplo="L", trans="N", unit=False):
    """Module-level :meth:`OracleLib.trsm_general` on the default build."""
    return _load().trsm_general(A, B, alpha, side, uplo, trans, unit)


def solve_general(A, B, alpha=1.0, side="L", uplo="L", trans="N", unit=False):
    """Module-level :meth:`OracleLib.solve_general` on the default build."""
    return _load().solve_general(A, B, alpha, side, uplo, trans, unit)


def backward_error_general(A, X, B0, alpha=1.0, side="L", uplo="L", trans="N", unit=False):
    """Module-level :meth:`OracleLib.backward_error_general` on the default build."""
    return _load().backward_error_general(A, X, B0, alpha, side, uplo, trans, unit)


def potrf(A):
    """Module-level :meth:`OracleLib.potrf` on the default build."""
    return _load().potrf(A)


def cholesky_solve(L, B):
    """Module-level :meth:`OracleLib.cholesky_solve` on the default build."""
    return _load().cholesky_solve(L, B)


def _load() -> OracleLib:
    global _lib
    with _lock:
        if _lib is None:
            _lib = OracleLib(build(force=False))
        return _lib


def num_threads() -> int:
    return _load().num_threads()


def set_num_threads(t: int) -> None:
    _load().set_num_threads(t)


def trsm(L, B, alpha=1.0, unit=False, rowform=False):
    """Module-level :meth:`OracleLib.trsm` on the default build."""
    return _load().trsm(L, B, alpha, unit, rowform)


def solve(L, B, alpha=1.0, unit=False, rowform=False):
    """Module-level :meth:`OracleLib.solve` on the default build."""
    return _load().solve(L, B, alpha, unit, rowform)


def backward_error(L, X, B0, alpha=1.0, unit=False) -> float:
    """Module-level :meth:`OracleLib.backward_error` on the default build."""
    return _load().backward_error(L, X, B0, alpha, unit)


def compile_variant(src_text: str, out_path: str) -> str:
    """Compile C source text (a copy of the oracle, possibly edited by a test)
    with the oracle's own flags.  Used by the tests that check the pins catch
    planted mistakes."""
    src = out_path + ".c"
    with open(src, "w") as f:
        f.write(src_text)
    subprocess.check_call(["gcc", *_CFLAGS, src, "-o", out_path, "-lm"])
    return out_path


def source_text() -> str:
    with open(_SRC) as f:
        return f.read()


def rel_err_fro(X: np.ndarray, Xref: np.ndarray) -> float:
    """Normwise relative error ||X - Xref||_F / ||Xref||_F (the paper's Table 2 metric)."""
    num = np.linalg.norm(np.asarray(X) - np.asarray(Xref))
    den = np.linalg.norm(np.asarray(Xref))
    return float(num / den) if den > 0 else float(num)

