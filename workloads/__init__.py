"""Seeded synthetic inputs for the TRSM workloads.

This module only draws numbers: it holds none of the solver's arithmetic.  The
tests, the benchmark and the oracle's pins all take their inputs from here, so
the GPU path and the CPU oracle see identical data.

The paper measures on "random values" (Sec. 5.1) without saying which; the
recipes below fix them:

* numpy ``default_rng(seed)`` (PCG64) draws everything, in this order:
  1. an m x m U(-1, 1) matrix, filled in column-major order (for complex
     problems the full real part, then the full imaginary part); its strict
     lower triangle divided by m becomes the off-diagonal of L;
  2. the diagonal: length-m U(1, 2) (complex: then an imaginary part
     U(-0.5, 0.5));
  3. B: m x n N(0, 1), column-major (complex: real part, then imaginary part).
* The upper triangle of L is filled with NaN, so a kernel that reads it
  poisons its result.  Padding rows (between m and the leading dimension) are
  filled with a sentinel the tests check is untouched.

Arrays are numpy arrays in Fortran (column-major) order, float64 for real
problems and complex128 for complex ones.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import List, Optional, Sequence, Tuple

import numpy as np

# Sentinel written into padding rows of B (rows m..ldb-1).
PAD_SENTINEL = 1234.5625


def flops(m: int, n: int, complex_: bool) -> float:
    """Flop count behind every GFLOP/s figure (the paper states none).

    Real: m*n divisions plus m(m-1)/2*n multiply-adds, i.e. m^2 n.  Complex
    (6 flops per multiply, 2 per add): 4 m^2 n + 2 m n, the usual ZTRSM count.
    The extra work of explicit diagonal-block inverses is not counted.
    """
    if complex_:
        return 4.0 * m * m * n + 2.0 * m * n
    return float(m) * m * n


def algorithmic_bytes(m: int, n: int, complex_: bool) -> float:
    """Minimum HBM traffic of one solve: the lower triangle of L read once, B
    read once and written once."""
    es = 16 if complex_ else 8
    return es * (m * (m + 1) / 2.0 + 2.0 * m * n)


def _embed(a: np.ndarray, ld: Optional[int], fill) -> np.ndarray:
    """Return a column-major view of ``a`` whose leading dimension is ``ld``."""
    m, n = a.shape
    if ld is None or ld == m:
        return np.asfortranarray(a)
    if ld < m:
        raise ValueError("leading dimension smaller than the row count")
    buf = np.empty((ld, n), dtype=a.dtype, order="F")
    buf[...] = fill
    buf[:m, :] = a
    return buf[:m, :]


def _fill_upper(a: np.ndarray, value, include_diag: bool = False) -> None:
    """Write ``value`` above the diagonal (and on it, if ``include_diag``),
    one column at a time so large matrices need no index arrays."""
    m = a.shape[0]
    for j in range(a.shape[1]):
        top = min(j + 1 if include_diag else j, m)
        if top > 0:
            a[:top, j] = value


def lower_matrix(rng: np.random.Generator, m: int, complex_: bool = False,
                 lda: Optional[int] = None, offdiag_scale: float = 1.0) -> np.ndarray:
    """Random lower-triangular L with the workloads' distribution.

    Real: l_ij ~ U(-1,1)/m for j < i, l_ii ~ U(1,2).  Complex: real and
    imaginary off-diagonal parts ~ U(-1,1)/m, diagonal real part ~ U(1,2),
    imaginary part ~ U(-0.5,0.5).  ``offdiag_scale`` multiplies the strict
    lower triangle (used to set the conditioning of the mixed-precision case).
    Upper triangle = NaN.
    """
    if complex_:
        re = rng.uniform(-1.0, 1.0, size=m * m).reshape((m, m), order="F")
        im = rng.uniform(-1.0, 1.0, size=m * m).reshape((m, m), order="F")
        full = (re + 1j * im).astype(np.complex128)
        del re, im
        dre = rng.uniform(1.0, 2.0, size=m)
        dim = rng.uniform(-0.5, 0.5, size=m)
        diag = dre + 1j * dim
    else:
        full = rng.uniform(-1.0, 1.0, size=m * m).reshape((m, m), order="F")
        diag = rng.uniform(1.0, 2.0, size=m)
    full *= offdiag_scale / m
    _fill_upper(full, np.nan)
    full[np.diag_indices(m)] = diag
    return _embed(full, lda, np.nan)


def rhs_matrix(rng: np.random.Generator, m: int, n: int, complex_: bool = False,
               ldb: Optional[int] = None) -> np.ndarray:
    """B ~ N(0,1) (complex: independent N(0,1) real and imaginary parts)."""
    if complex_:
        re = rng.standard_normal(size=m * n).reshape((m, n), order="F")
        im = rng.standard_normal(size=m * n).reshape((m, n), order="F")
        b = (re + 1j * im).astype(np.complex128)
    else:
        b = rng.standard_normal(size=m * n).reshape((m, n), order="F")
    return _embed(b, ldb, PAD_SENTINEL)


def problem(seed: int, m: int, n: int, complex_: bool = False,
            lda: Optional[int] = None, ldb: Optional[int] = None,
            offdiag_scale: float = 1.0) -> Tuple[np.ndarray, np.ndarray]:
    """One (L, B) pair drawn with ``default_rng(seed)`` in the documented order."""
    rng = np.random.default_rng(seed)
    L = lower_matrix(rng, m, complex_, lda, offdiag_scale)
    B = rhs_matrix(rng, m, n, complex_, ldb)
    return L, B


# --------------------------------------------------------------------------
# Named workloads
# --------------------------------------------------------------------------

# Single small real solve: m = n = 32, non-unit, alpha = 1, seed 0.
SINGLE_SMALL = dict(seed=0, m=32, n=32, complex_=False, alpha=1.0)

# Large real solve: m = n = 16384, alpha = -1, seed 2; large complex solve:
# m = n = 8192, alpha = (-1, 0), also seed 2.
LARGE_REAL = dict(seed=2, m=16384, n=16384, complex_=False, alpha=-1.0)
LARGE_COMPLEX = dict(seed=2, m=8192, n=8192, complex_=True, alpha=complex(-1.0, 0.0))

# Mixed-precision case: m = 8192, n = 4096, alpha = 1, seed 3, the strict
# lower triangle scaled to reach a target condition number.
MIXED = dict(seed=3, m=8192, n=4096, complex_=False, alpha=1.0)

def mixed_scale(m: int, kappa: float) -> float:
    """Off-diagonal scale s giving L(s) = D + s N0 an estimated kappa_inf of
    ``kappa`` (table written by tests/golden/make_mixed_scales.py, which uses
    only the oracle's solver; sizes 1024 and 8192)."""
    import json
    import os
    path = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                        "tests", "golden", "mixed_scales.json")
    with open(path) as f:
        tab = json.load(f)
    return float(tab[str(m)][f"{kappa:.0e}"]["scale"])


def mixed_problem(m: int = 8192, n: int = 4096, kappa: float = 1e3, seed: int = 3):
    """The mixed-precision workload: the standard real draw with its strict
    lower triangle scaled so that kappa_inf(L) is about ``kappa``."""
    return problem(seed, m, n, False, offdiag_scale=mixed_scale(m, kappa))


# Batched small complex solves: 10 000 problems, m and n i.i.d. U{8..64},
# alpha = (1, 0.5), seed 1.
BATCHED = dict(seed=1, count=10000, lo=8, hi=64, complex_=True, alpha=complex(1.0, 0.5))
# The same shapes as real problems (DTRSM), alpha = 0.5.
BATCHED_REAL = dict(seed=1, count=10000, lo=8, hi=64, complex_=False, alpha=0.5)


@dataclass
class Batch:
    """A set of independent problems, each its own column-major arrays."""
    shapes: List[Tuple[int, int]]
    L: List[np.ndarray]
    B: List[np.ndarray]
    alpha: complex
    complex_: bool
    unit: List[bool] = field(default_factory=list)

    def total_flops(self) -> float:
        return sum(flops(m, n, self.complex_) for m, n in self.shapes)

    def total_bytes(self) -> float:
        return sum(algorithmic_bytes(m, n, self.complex_) for m, n in self.shapes)


def batch_shapes(seed: int, count: int, lo: int = 8, hi: int = 64) -> List[Tuple[int, int]]:
    """(m, n) pairs, each coordinate i.i.d. uniform on {lo..hi}; m's drawn first."""
    rng = np.random.default_rng(seed)
    ms = rng.integers(lo, hi + 1, size=count)
    ns = rng.integers(lo, hi + 1, size=count)
    return [(int(a), int(b)) for a, b in zip(ms, ns)]


def batched(seed: int = 1, count: int = 10000, lo: int = 8, hi: int = 64,
            complex_: bool = True, alpha=complex(1.0, 0.5)) -> Batch:
    """The batched workload: the shapes come from ``default_rng(seed)``; then
    each problem's L and B, in problem order, from ``default_rng([seed, 1])``."""
    shapes = batch_shapes(seed, count, lo, hi)
    rng = np.random.default_rng([seed, 1])
    Ls, Bs = [], []
    for m, n in shapes:
        Ls.append(lower_matrix(rng, m, complex_))
        Bs.append(rhs_matrix(rng, m, n, complex_))
    return Batch(shapes=shapes, L=Ls, B=Bs, alpha=alpha, complex_=complex_,
                 unit=[False] * count)


# --------------------------------------------------------------------------
# Structured matrices with closed-form inverses (used by the pins)
# --------------------------------------------------------------------------

def identity_lower(m: int, complex_: bool = False, unit: bool = False) -> np.ndarray:
    """Identity L (NaN above the diagonal; NaN on the diagonal when ``unit``)."""
    dt = np.complex128 if complex_ else np.float64
    L = np.zeros((m, m), dtype=dt, order="F")
    _fill_upper(L, np.nan)
    L[np.diag_indices(m)] = np.nan if unit else 1.0
    return L


def diagonal_lower(d: Sequence, complex_: bool = False) -> np.ndarray:
    m = len(d)
    dt = np.complex128 if complex_ else np.float64
    L = np.zeros((m, m), dtype=dt, order="F")
    _fill_upper(L, np.nan)
    L[np.diag_indices(m)] = np.asarray(d, dtype=dt)
    return L


def bidiagonal_lower(m: int, d, complex_: bool = False) -> np.ndarray:
    """L = d (I - S), S the sub-diagonal shift: l_ii = d, l_{i+1,i} = -d."""
    dt = np.complex128 if complex_ else np.float64
    L = np.zeros((m, m), dtype=dt, order="F")
    _fill_upper(L, np.nan)
    L[np.diag_indices(m)] = d
    idx = np.arange(m - 1)
    L[idx + 1, idx] = -d
    return L


def integer_rhs(rng: np.random.Generator, m: int, n: int, lo: int, hi: int,
                complex_: bool = False) -> np.ndarray:
    """Integer-valued B (uniform on {lo..hi}), stored as float64/complex128."""
    re = rng.integers(lo, hi + 1, size=(m, n)).astype(np.float64)
    if complex_:
        im = rng.integers(lo, hi + 1, size=(m, n)).astype(np.float64)
        return np.asfortranarray(re + 1j * im)
    return np.asfortranarray(re)


def unit_lower_integer(rng: np.random.Generator, m: int, values=(-1, 0, 1),
                       complex_: bool = False) -> np.ndarray:
    """Unit-lower L with strict lower entries drawn from ``values``; NaN
    diagonal (a unit-diagonal solve must not read it) and NaN upper part."""
    v = np.asarray(values, dtype=np.float64)
    re = v[rng.integers(0, len(v), size=(m, m))]
    if complex_:
        im = v[rng.integers(0, len(v), size=(m, m))]
        L = np.asfortranarray(re + 1j * im)
    else:
        L = np.asfortranarray(re)
    _fill_upper(L, np.nan, include_diag=True)
    return L


def block_nilpotent(m1: int, m2: int, C: np.ndarray) -> np.ndarray:
    """L = [[I, 0], [C, I]] with C of shape (m2, m1); NaN upper triangle."""
    m = m1 + m2
    dt = C.dtype
    L = np.zeros((m, m), dtype=dt, order="F")
    L[np.diag_indices(m)] = 1.0
    L[m1:, :m1] = C
    _fill_upper(L, np.nan)
    return L


# --------------------------------------------------------------------------
# Serving stream
# --------------------------------------------------------------------------

@dataclass
class Request:
    rid: int
    t_arrival: float      # seconds from stream start
    m: int
    n: int
    complex_: bool
    alpha: float          # real; imaginary part 0 for complex requests


def serving_stream(seed: int = 4, rate: float = 20000.0, duration: float = 60.0,
                   m_range=(8, 4096), n_range=(1, 512), p_complex: float = 0.3,
                   alpha_range=(-2.0, 2.0)) -> List[Request]:
    """Open-loop Poisson arrivals (exponential gaps at ``rate``/s) for
    ``duration`` seconds.  Per request, m = floor(exp U(ln lo, ln hi+1)) and n
    likewise, clamped; complex with probability ``p_complex``; alpha real
    uniform on ``alpha_range``."""
    rng = np.random.default_rng(seed)
    est = int(rate * duration * 1.2) + 64
    gaps = rng.exponential(1.0 / rate, size=est)
    t = np.cumsum(gaps)
    t = t[t < duration]
    k = len(t)
    um = rng.uniform(math.log(m_range[0]), math.log(m_range[1] + 1), size=k)
    un = rng.uniform(math.log(n_range[0]), math.log(n_range[1] + 1), size=k)
    ms = np.clip(np.floor(np.exp(um)).astype(np.int64), m_range[0], m_range[1])
    ns = np.clip(np.floor(np.exp(un)).astype(np.int64), n_range[0], n_range[1])
    cx = rng.uniform(0.0, 1.0, size=k) < p_complex
    al = rng.uniform(alpha_range[0], alpha_range[1], size=k)
    return [Request(i, float(t[i]), int(ms[i]), int(ns[i]), bool(cx[i]), float(al[i]))
            for i in range(k)]


# ---------------------------------------------------------------------------
# Counter-based synthetic inputs (serving requests)
# ---------------------------------------------------------------------------
#
# Philox4x32-10 (Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as
# easy as 1, 2, 3", SC'11): a 4 x 32-bit counter and a 2 x 32-bit key go
# through ten rounds; each round multiplies words 0 and 2 by fixed odd
# constants, and the new words are (hi(M1 c2) ^ c1 ^ k0, lo(M1 c2),
# hi(M0 c0) ^ c3 ^ k1, lo(M0 c0)); the key is bumped by two Weyl constants
# between rounds.  The device library draws serving inputs with its own
# implementation of the same published generator; this one lets the host
# regenerate them for verification.

PHILOX_M0, PHILOX_M1 = 0xD2511F53, 0xCD9E8D57
PHILOX_W0, PHILOX_W1 = 0x9E3779B9, 0xBB67AE85
_MASK32 = np.uint64(0xFFFFFFFF)


def philox4x32_10(counter, key):
    """Philox4x32-10 on arrays: ``counter`` is a sequence of four uint32
    arrays (or scalars), ``key`` a pair of uint32 values.  Returns four
    uint32 arrays."""
    c = [np.asarray(x, dtype=np.uint64) & _MASK32 for x in counter]
    k0, k1 = np.uint64(int(key[0]) & 0xFFFFFFFF), np.uint64(int(key[1]) & 0xFFFFFFFF)
    m0, m1 = np.uint64(PHILOX_M0), np.uint64(PHILOX_M1)
    w0, w1 = np.uint64(PHILOX_W0), np.uint64(PHILOX_W1)
    for r in range(10):
        if r:
            k0 = (k0 + w0) & _MASK32
            k1 = (k1 + w1) & _MASK32
        p0 = m0 * c[0]            # < 2^64: exact in uint64
        p1 = m1 * c[2]
        c = [(p1 >> np.uint64(32)) ^ c[1] ^ k0, p1 & _MASK32,
             (p0 >> np.uint64(32)) ^ c[3] ^ k1, p0 & _MASK32]
    return [x.astype(np.uint32) for x in c]


def philox_uniforms(e: np.ndarray, tag: int, key: int):
    """Two 53-bit uniforms on [0, 1) per element index ``e`` (uint64 array):
    counter (e mod 2^32, e div 2^32, tag, 0), key (key mod 2^32, key div 2^32);
    u1 from output words (x0, x1), u2 from (x2, x3), each the top 53 bits of
    the 64-bit word x_lo + 2^32 x_hi, times 2^-53."""
    e = np.asarray(e, dtype=np.uint64)
    x = philox4x32_10([e & _MASK32, e >> np.uint64(32), np.full(e.shape, tag, np.uint64),
                       np.zeros(e.shape, np.uint64)],
                      (key & 0xFFFFFFFF, (key >> 32) & 0xFFFFFFFF))
    a = (x[1].astype(np.uint64) << np.uint64(32)) | x[0].astype(np.uint64)
    b = (x[3].astype(np.uint64) << np.uint64(32)) | x[2].astype(np.uint64)
    u1 = (a >> np.uint64(11)).astype(np.float64) * 2.0 ** -53
    u2 = (b >> np.uint64(11)).astype(np.float64) * 2.0 ** -53
    return u1, u2


def serving_key(seed: int, rid: int) -> int:
    """Philox key of serving request ``rid`` of a stream drawn with ``seed``."""
    return ((seed & 0xFFFFFFFF) << 32) | (rid & 0xFFFFFFFF)


def synthetic_inputs(m: int, n: int, key: int, complex_: bool = False):
    """L (m x m) and B (m x n) of a synthetic serving request, column-major:
    element e (column-major index) of L from philox_uniforms(e, 0, key), of B
    from tag 1.  L: strict lower (2 u1 - 1)/m (complex: imaginary part
    (2 u2 - 1)/m), diagonal 1 + u1 (complex: imaginary u2 - 1/2), upper
    triangle 0.  B: sqrt(-2 ln(1 - u1)) cos(2 pi u2) (complex: imaginary part
    with sin) -- the Box-Muller transform, so B ~ N(0, 1) as in the standard
    workload, and L has its off-diagonal U(-1, 1)/m and diagonal U(1, 2)."""
    e = np.arange(m * m, dtype=np.uint64)
    u1, u2 = philox_uniforms(e, 0, key)
    i = (e % np.uint64(max(m, 1))).astype(np.int64)
    j = (e // np.uint64(max(m, 1))).astype(np.int64)
    low, diag = i > j, i == j
    re = np.where(low, (2.0 * u1 - 1.0) / m, np.where(diag, 1.0 + u1, 0.0))
    if complex_:
        im = np.where(low, (2.0 * u2 - 1.0) / m, np.where(diag, u2 - 0.5, 0.0))
        L = (re + 1j * im).reshape(m, m, order="F")
    else:
        L = re.reshape(m, m, order="F")
    eb = np.arange(m * n, dtype=np.uint64)
    v1, v2 = philox_uniforms(eb, 1, key)
    r = np.sqrt(-2.0 * np.log(1.0 - v1))
    th = 6.283185307179586 * v2
    if complex_:
        B = (r * np.cos(th) + 1j * (r * np.sin(th))).reshape(m, n, order="F")
    else:
        B = (r * np.cos(th)).reshape(m, n, order="F")
    return np.asfortranarray(L), np.asfortranarray(B)
