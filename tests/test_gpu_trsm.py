"""GPU parity: the HIP path against the CPU oracle on identical seeded inputs.

Bar (normwise): relative Frobenius error against the oracle <= 1e-12 and
backward error ||L X - alpha B||_inf / (||L|| ||X|| + |alpha| ||B||) <= 10 m 2^-53.
Structured inputs with exactly representable answers must match bit for bit.
"""
import numpy as np
import pytest

import oracle
import workloads as W
from parity import assert_parity, padding_rows

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

hs = pytest.importorskip("paper_2608_25469_amd")

U = 2.0 ** -53


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)
    hs.lib()  # raises if the library is missing: no silent fallback


def run(L, B, alpha, unit=False, block_size=0, path=0, ldb=None, lda=None):
    """Solve on the GPU; returns (X, report, padding rows of B as numpy)."""
    Ld = hs.to_colmajor(L, ld=lda)
    Bd = hs.to_colmajor(B, ld=ldb)
    if ldb is not None:
        # sentinel in the padding rows
        padding_rows(Bd).fill_(W.PAD_SENTINEL)
    _, rep = hs.trsm(Ld, Bd, alpha, unit=unit, block_size=block_size, path=path, report=True)
    torch.cuda.synchronize()
    X = hs.from_colmajor(Bd)
    pad = None
    if ldb is not None:
        pad = padding_rows(Bd).cpu().numpy()
    return X, rep, pad


def check(L, B, X, alpha, unit=False, tag=""):
    """Frobenius, per-column and element-wise error against the oracle, and
    the oracle's backward error of X (see tests/parity.py)."""
    fro, _, _, eta = assert_parity(L, B, X, alpha, unit=unit, tag=tag)
    return fro, eta


# ---------------------------------------------------------------------------
# small kernel: every m in 1..64
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("cx", [False, True], ids=["real", "complex"])
@pytest.mark.parametrize("unit", [False, True], ids=["nonunit", "unit"])
def test_small_every_m(cx, unit):
    alpha = complex(0.75, -0.5) if cx else -1.5
    for m in range(1, 65):
        for n in (1, 13, 64, 65, 130):
            L, B = W.problem(1000 + m, m, n, cx)
            X, rep, _ = run(L, B, alpha, unit=unit)
            assert rep["path"] == 1
            check(L, B, X, alpha, unit, tag=(m, n, cx, unit))


def test_single_small_workload():
    """The single small real solve: m = n = 32, seed 0, alpha = 1."""
    c = W.SINGLE_SMALL
    L, B = W.problem(c["seed"], c["m"], c["n"], c["complex_"])
    X, rep, _ = run(L, B, c["alpha"])
    assert rep["path"] == 1
    check(L, B, X, c["alpha"], tag="single-small")


# ---------------------------------------------------------------------------
# blocked path: every I_B, ragged sizes, both dtypes
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("cx", [False, True], ids=["real", "complex"])
@pytest.mark.parametrize("ib", [16, 32, 64, 128, 256])
def test_blocked_sizes(cx, ib):
    alpha = complex(-1.0, 0.25) if cx else -1.0
    for m, n in ((65, 7), (127, 64), (129, 33), (300, 129), (1000, 77), (1061, 200)):
        for unit in (False, True):
            L, B = W.problem(2000 + m + ib, m, n, cx)
            X, rep, _ = run(L, B, alpha, unit=unit, block_size=ib)
            assert rep["path"] == 2 and rep["block_size"] == ib
            check(L, B, X, alpha, unit, tag=(m, n, cx, ib, unit))


def test_blocked_default_table():
    for cx in (False, True):
        L, B = W.problem(7, 700, 50, cx)
        X, rep, _ = run(L, B, 1.0)
        assert rep["path"] == 2 and rep["block_size"] == hs.lookup_block_size(cx, 700, 50)
        check(L, B, X, 1.0, tag=("table", cx))


# ---------------------------------------------------------------------------
# exact answers, bit for bit, on every path
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("ib", [0, 16, 64, 256])
def test_bidiagonal_exact(ib):
    rng = np.random.default_rng(3)
    for m in (40, 64, 300, 777):
        if ib == 0 and m > 64:
            continue
        if ib and m <= 64:
            continue
        B = W.integer_rhs(rng, m, 9, -50, 50)
        X, _, _ = run(W.bidiagonal_lower(m, 4.0), B, 2.0, block_size=ib)
        assert np.array_equal(X, np.cumsum(B, axis=0) * 0.5), (m, ib)
        Bc = W.integer_rhs(rng, m, 9, -50, 50, complex_=True)
        Xc, _, _ = run(W.bidiagonal_lower(m, 1 + 1j, complex_=True), Bc, 1.0, block_size=ib)
        assert np.array_equal(Xc, np.cumsum(Bc, axis=0) * (0.5 - 0.5j)), (m, ib, "cx")


@pytest.mark.parametrize("ib", [0, 32, 128])
def test_block_nilpotent_exact(ib):
    rng = np.random.default_rng(4)
    for cx in (False, True):
        for m1, m2 in ((20, 30), (130, 200), (256, 256)):
            if (ib == 0) != (m1 + m2 <= 64):
                continue
            C = W.integer_rhs(rng, m2, m1, -2, 2, complex_=cx)
            L = W.block_nilpotent(m1, m2, C)
            B = W.integer_rhs(rng, m1 + m2, 11, -20, 20, complex_=cx)
            expect = B.copy()
            expect[m1:] = B[m1:] - C @ B[:m1]
            X, _, _ = run(L, B, 1.0, block_size=ib)
            assert np.array_equal(X, expect), (cx, m1, m2, ib)
            Lu = L.copy(order="F")
            Lu[np.diag_indices(m1 + m2)] = np.nan
            Xu, _, _ = run(Lu, B, 1.0, unit=True, block_size=ib)
            assert np.array_equal(Xu, expect), (cx, m1, m2, ib, "unit")


def test_identity_exact():
    rng = np.random.default_rng(5)
    for m, ib in ((33, 0), (64, 0), (200, 64), (513, 256)):
        for cx in (False, True):
            for unit in (False, True):
                L = W.identity_lower(m, cx, unit=unit)
                B = W.rhs_matrix(rng, m, 17, cx)
                X, _, _ = run(L, B, 1.0, unit=unit, block_size=ib)
                assert np.array_equal(X, B), (m, ib, cx, unit)


# ---------------------------------------------------------------------------
# BLAS conventions
# ---------------------------------------------------------------------------
def test_alpha_zero_reads_nothing():
    for m, cx in ((10, False), (100, True)):
        L = np.full((m, m), np.nan, dtype=np.complex128 if cx else np.float64, order="F")
        B = np.full((m, 5), np.nan, dtype=L.dtype, order="F")
        X, _, _ = run(L, B, 0.0)
        assert np.all(X == 0)


def test_padding_rows_untouched():
    # m, n <= 16 take the fused kernel (B staged through LDS), m = 37 the
    # strip kernel, m = 150 the blocked path
    for m, n, ib in ((1, 16, 0), (7, 5, 0), (16, 16, 0), (37, 20, 0), (150, 20, 32)):
        for cx in (False, True):
            L, B = W.problem(9, m, n, cx)
            alpha = complex(0.5, -1.0) if cx else 1.0
            X, _, pad = run(L, B, alpha, block_size=ib, ldb=m + 11, lda=m + 3)
            assert np.all(pad == W.PAD_SENTINEL), (m, cx)
            check(L, B, X, alpha, tag=("pad", m, cx))


def test_leading_dimension_of_L():
    for m, ib in ((50, 0), (260, 64)):
        for cx in (False, True):
            L, B = W.problem(10, m, 30, cx)
            X, _, _ = run(L, B, 1.0, block_size=ib, lda=m + 9)
            check(L, B, X, 1.0, tag=("lda", m, cx))


def _device_at_offset(a, ld, fill=0.0):
    """a (m x n, Fortran order) in a float64 device buffer whose data start 8
    bytes in (8-byte, not 16-byte, alignment), leading dimension ld, padding
    rows filled with `fill`.  Returns (buffer, address of a)."""
    m, n = a.shape
    host = np.full((ld, n), fill, dtype=a.dtype, order="F")
    host[:m] = a
    flat = np.ascontiguousarray(host.reshape(-1, order="F")).view(np.float64)
    buf = torch.from_numpy(np.concatenate([[0.0], flat])).to("cuda")
    return buf, buf.data_ptr() + 8


def _read_at_offset(buf, m, n, ld, cx):
    flat = np.ascontiguousarray(buf.cpu().numpy()[1:])
    full = (flat.view(np.complex128) if cx else flat).reshape(ld, n, order="F")
    return np.asfortranarray(full[:m]), np.asfortranarray(full[m:])


def test_operands_at_eight_byte_offsets():
    """L and B 8 bytes into their allocations, with odd leading dimensions:
    the small paths' 16-byte accesses (two real rows, one complex element;
    the fused kernel for m, n <= 16, the strip kernel above) must read and
    write exactly the right elements, and leave B's padding rows alone."""
    import ctypes
    for cx in (False, True):
        for m, n in ((5, 9), (16, 16), (7, 20), (33, 70), (64, 37), (50, 5)):
            L, B = W.problem(77 + m, m, n, cx)
            lda = m + 2 if m % 2 else m + 1
            ldb = m + 2 if m % 2 else m + 3
            Lbuf, La = _device_at_offset(L, lda)
            Bbuf, Ba = _device_at_offset(B, ldb, fill=W.PAD_SENTINEL)
            alpha = complex(0.5, -0.25) if cx else -0.5
            code = hs.C64F if cx else hs.R64F
            st = hs.lib().hsma_trsm(hs.NON_UNIT, m, n, hs._alpha_buf(alpha, code), ctypes.c_void_p(La), lda,
                                    ctypes.c_void_p(Ba), ldb, code, None)
            assert st == 0, st
            torch.cuda.synchronize()
            X, pad = _read_at_offset(Bbuf, m, n, ldb, cx)
            assert np.all(pad == W.PAD_SENTINEL), (m, n, cx)
            check(L, B, X, alpha, tag=("offset", m, n, cx))


def test_deterministic_repeats():
    for m, ib in ((48, 0), (400, 64)):
        L, B = W.problem(11, m, 100, True)
        X0, _, _ = run(L, B, 1.0, block_size=ib)
        for _ in range(5):
            X1, _, _ = run(L, B, 1.0, block_size=ib)
            assert X1.tobytes() == X0.tobytes()


# ---------------------------------------------------------------------------
# HIP-graph replay of the blocked schedule
# ---------------------------------------------------------------------------
def test_graph_replay_matches_eager_every_time():
    """Capture once, replay several times with eager work in between; every
    replay must equal the eager solve of the same input bit for bit."""
    for cx, m, n, ib in ((False, 600, 100, 64), (True, 300, 40, 32)):
        L, B = W.problem(21, m, n, cx)
        Ld = hs.to_colmajor(L)
        Bg = hs.to_colmajor(B)
        Be = hs.to_colmajor(B)
        B0 = hs.to_colmajor(B)
        hs.trsm(Ld, Be, -1.0, block_size=ib)
        torch.cuda.synchronize()
        ref = hs.from_colmajor(Be)
        for rep in range(4):
            Bg.copy_(B0)
            hs.trsm(Ld, Bg, -1.0, block_size=ib, graph=True)
            torch.cuda.synchronize()
            assert hs.from_colmajor(Bg).tobytes() == ref.tobytes(), (cx, rep)
            # unrelated eager work between replays
            Be.copy_(B0)
            hs.trsm(Ld, Be, -1.0, block_size=ib)
            torch.cuda.synchronize()
        check(L, B, hs.from_colmajor(Bg), -1.0, tag=("graph", cx))
    hs.graph_cache_clear()


def test_graph_one_capture_per_shape_new_pointers_and_alpha():
    """One graph per shape: calls with other A, B and alpha of the same shape
    replay the instantiated graphs with their arguments updated in place (no
    new instantiation after the two the shape keeps), and every replay equals
    the eager solve of its own inputs bit for bit, with eager work and a
    second shape interleaved."""
    hs.graph_cache_clear()
    for cx, m, n, ib in ((False, 500, 70, 64), (True, 260, 33, 32)):
        probs = [W.problem(70 + k, m, n, cx) for k in range(5)]
        alphas = [(-1.0, 0.5, 2.0, -0.75, 1.0)[k] if not cx else complex(-1.0 + 0.25 * k, 0.5 - k)
                  for k in range(5)]
        dev = [(hs.to_colmajor(L), hs.to_colmajor(B)) for L, B in probs]
        refs = []
        for (L, B), a in zip(probs, alphas):
            Le, Be = hs.to_colmajor(L), hs.to_colmajor(B)
            hs.trsm(Le, Be, a, block_size=ib)
            refs.append(Be)
        torch.cuda.synchronize()
        before = hs.graph_stats()
        for rnd in range(3):
            for k, ((Ld, Bd), a) in enumerate(zip(dev, alphas)):
                Bd.copy_(hs.to_colmajor(probs[k][1]))
                hs.trsm(Ld, Bd, a, block_size=ib, graph=True)
                # another shape in between
                L2, B2 = W.problem(99, 130, 7, cx)
                hs.trsm(hs.to_colmajor(L2), hs.to_colmajor(B2), 1.0, block_size=32, graph=True)
                torch.cuda.synchronize()
                assert hs.from_colmajor(Bd).tobytes() == hs.from_colmajor(refs[k]).tobytes(), (cx, rnd, k)
        after = hs.graph_stats()
        # two graphs for this shape and two for the interleaved one, at most
        assert after["captures"] - before["captures"] <= 4, (before, after)
        assert after["updates"] - before["updates"] >= 10, (before, after)
        assert after["replays"] - before["replays"] == 30
    hs.graph_cache_clear()


def test_plain_solve_on_side_streams():
    """A plain solve (the options-free entry point) runs on torch's current
    stream, or on the stream passed as an object or a raw handle: the
    binding's stream lookup returns the side stream's handle inside its
    context, and every result equals the default stream's bit for bit."""
    for m, n, cx in ((32, 32, False), (40, 70, True), (300, 64, False)):
        L, B = W.problem(4242 + m, m, n, cx)
        Ld = hs.to_colmajor(L)
        ref = hs.to_colmajor(B)
        hs.trsm(Ld, ref, 1.0)
        torch.cuda.synchronize()
        want = hs.from_colmajor(ref).tobytes()
        side = torch.cuda.Stream()
        outs = [hs.to_colmajor(B) for _ in range(3)]
        torch.cuda.synchronize()
        with torch.cuda.stream(side):
            assert hs._stream_handle(None) == side.cuda_stream
            hs.trsm(Ld, outs[0], 1.0)
        hs.trsm(Ld, outs[1], 1.0, stream=side)
        hs.trsm(Ld, outs[2], 1.0, stream=side.cuda_stream)
        side.synchronize()
        assert hs._stream_handle(None) == torch.cuda.current_stream().cuda_stream
        for k, o in enumerate(outs):
            assert hs.from_colmajor(o).tobytes() == want, (m, n, cx, k)
