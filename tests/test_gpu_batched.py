"""Batched solves on the GPU: every problem against the oracle, the batch
against one-at-a-time calls (bit for bit), and the plan API."""
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
    hs.lib()


def mixed_problems(seed, count, max_m=64, max_n=64, big=()):
    rng = np.random.default_rng(seed)
    probs = []
    for i in range(count):
        m = int(rng.integers(1, max_m + 1))
        n = int(rng.integers(1, max_n + 1))
        cx = bool(rng.integers(0, 2))
        unit = bool(rng.integers(0, 4) == 0)
        L, B = W.problem(seed * 100000 + i, m, n, cx)
        alpha = complex(rng.uniform(-2, 2), rng.uniform(-1, 1)) if cx else float(rng.uniform(-2, 2))
        probs.append((L, B, alpha, unit))
    for j, (m, n, cx) in enumerate(big):
        L, B = W.problem(seed * 100000 + 90000 + j, m, n, cx)
        probs.append((L, B, complex(-1, 0.5) if cx else -0.75, False))
    return probs


def to_dev(probs):
    out = []
    for L, B, a, u in probs:
        out.append((hs.to_colmajor(L), hs.to_colmajor(B), a, u))
    return out


def test_batched_matches_oracle_and_single_calls():
    probs = mixed_problems(1, 300, max_n=150, big=[(100, 30, False), (200, 70, True)])
    dev = to_dev(probs)
    hs.trsm_batched(dev)
    torch.cuda.synchronize()
    dev1 = to_dev(probs)
    for L, B, a, u in dev1:
        hs.trsm(L, B, a, unit=u)
    torch.cuda.synchronize()
    for (L, B, a, u), (_, Bd, _, _), (_, Bs, _, _) in zip(probs, dev, dev1):
        X = hs.from_colmajor(Bd)
        Xs = hs.from_colmajor(Bs)
        assert X.tobytes() == Xs.tobytes(), "batched differs from single call"
        assert_parity(L, B, X, a, unit=u, tag=("batched", B.shape))


def test_batched_every_m_with_three_or_four_blocks():
    """m = 33 .. 64 (three or four 16-row blocks), real and complex: four
    16-column problems of one m share a wavefront (each strip its own
    problem), beside 40- and 64-column problems and a 5-column one.  Real
    batches keep two finished blocks in LDS and read older ones back from B;
    single calls keep them all, so equal bits check both walks."""
    rng = np.random.default_rng(77)
    probs = []
    for m in range(33, 65):
        for cx in (False, True):
            for j, n in enumerate((16, 16, 16, 16, 40, 64, 5)):
                L, B = W.problem(1000 * m + 10 * j + cx, m, n, cx)
                unit = bool(rng.integers(0, 3) == 0)
                alpha = complex(rng.uniform(-2, 2), rng.uniform(-1, 1)) if cx else float(rng.uniform(-2, 2))
                probs.append((L, B, alpha, unit))
    dev = to_dev(probs)
    hs.trsm_batched(dev)
    torch.cuda.synchronize()
    dev1 = to_dev(probs)
    for L, B, a, u in dev1:
        hs.trsm(L, B, a, unit=u)
    torch.cuda.synchronize()
    for (L, B, a, u), (_, Bd, _, _), (_, Bs, _, _) in zip(probs, dev, dev1):
        X = hs.from_colmajor(Bd)
        assert X.tobytes() == hs.from_colmajor(Bs).tobytes(), ("batched differs from single call", B.shape)
        assert_parity(L, B, X, a, unit=u, tag=("every m", B.shape, np.iscomplexobj(B), u))


def test_batched_workload_subset():
    """2000 problems drawn like the 10 000-problem complex workload."""
    b = W.batched(count=2000)
    pl, pb, vl, vb = hs.pack_batch(b.L, b.B)
    hs.trsm_batched([(L, B, b.alpha, False) for L, B in zip(vl, vb)])
    torch.cuda.synchronize()
    for i in range(0, 2000, 7):
        X = hs.from_colmajor(vb[i])
        assert_parity(b.L[i], b.B[i], X, b.alpha, tag=(i, b.shapes[i]))


def test_plan_repeats_bitwise():
    probs = mixed_problems(2, 120)
    dev_a = to_dev(probs)
    plan = hs.BatchPlan([hs.problem_struct(*p) for p in dev_a])
    dev_b = to_dev(probs)
    hs.trsm_batched(dev_b)
    plan.execute()
    torch.cuda.synchronize()
    for (_, Ba, _, _), (_, Bb, _, _) in zip(dev_a, dev_b):
        assert hs.from_colmajor(Ba).tobytes() == hs.from_colmajor(Bb).tobytes()
    # second execution solves again in place: compare with a second one-shot
    plan.execute()
    hs.trsm_batched(dev_b)
    torch.cuda.synchronize()
    for (_, Ba, _, _), (_, Bb, _, _) in zip(dev_a, dev_b):
        assert hs.from_colmajor(Ba).tobytes() == hs.from_colmajor(Bb).tobytes()
    plan.close()


def test_batched_alpha_zero_and_empty():
    L = hs.to_colmajor(np.full((5, 5), np.nan))
    B = hs.to_colmajor(np.full((5, 3), np.nan))
    E = hs.colmajor(0, 4, torch.float64)
    hs.trsm_batched([(L, B, 0.0, False), (L[:0, :0], E, 1.0, False)])
    torch.cuda.synchronize()
    assert np.all(hs.from_colmajor(B) == 0)


def test_batched_rejects_bad_descriptor_before_enqueue():
    probs = mixed_problems(3, 5)
    dev = to_dev(probs)
    before = [hs.from_colmajor(B).copy() for _, B, _, _ in dev]
    structs = [hs.problem_struct(*p) for p in dev]
    structs[3].lda = 0
    with pytest.raises(hs.HsmaError) as e:
        hs.trsm_batched(structs)
    assert e.value.first_bad == 3 and e.value.status == 2
    torch.cuda.synchronize()
    for (_, B, _, _), b0 in zip(dev, before):
        assert np.array_equal(hs.from_colmajor(B), b0, equal_nan=True)


def test_grouped_blocked_bitwise_equal_to_single():
    """Problems with m > 64 in one batch share grouped launches (every
    problem keeps its own schedule): each result must be bit for bit the
    single-call result, across data types, diagonal kinds, ragged m, I_B
    values from the table and alpha = 0."""
    rng = np.random.default_rng(11)
    shapes = [(65, 1), (66, 130), (100, 7), (127, 64), (128, 128), (129, 33), (200, 200),
              (255, 17), (256, 300), (300, 65), (511, 40), (512, 512), (777, 91), (1024, 8),
              (1100, 260), (1500, 100), (2048, 33), (4100, 20)]
    probs = []
    for i, (m, n) in enumerate(shapes):
        for cx in (False, True):
            L, B = W.problem(5000 + 2 * i + cx, m, n, cx)
            unit = (i + cx) % 4 == 3
            a = complex(rng.uniform(-2, 2), rng.uniform(-1, 1)) if cx else float(rng.uniform(-2, 2))
            if i == 5:
                a = 0.0
            probs.append((L, B, a, unit))
    dev = to_dev(probs)
    hs.trsm_batched(dev)
    torch.cuda.synchronize()
    dev1 = to_dev(probs)
    for L, B, a, u in dev1:
        hs.trsm(L, B, a, unit=u)
    torch.cuda.synchronize()
    for k, ((L, B, a, u), (_, Bd, _, _), (_, Bs, _, _)) in enumerate(zip(probs, dev, dev1)):
        X = hs.from_colmajor(Bd)
        assert X.tobytes() == hs.from_colmajor(Bs).tobytes(), f"problem {k} {B.shape}"
        if B.shape[0] <= 1100:
            ref = oracle.solve(L, B, a, unit=u)
            assert oracle.rel_err_fro(X, ref) <= 1e-12


def test_more_items_than_one_grid_row():
    """70 000 tiny problems (more than 65 535 workgroups in one launch, one
    per item).  Inputs are small integers with diagonals in {1, 2, 4}, so
    every solution is exact in FP64 and is checked bit for bit against the
    2 x 2 forward substitution written out."""
    count = 70_000
    rng = np.random.default_rng(17)
    l00 = rng.choice([1.0, 2.0, 4.0], count)
    l11 = rng.choice([1.0, 2.0, 4.0], count)
    l10 = rng.integers(-3, 4, count).astype(np.float64)
    b0 = rng.integers(-8, 9, count).astype(np.float64)
    b1 = rng.integers(-8, 9, count).astype(np.float64)
    # Problem i: L column-major 2 x 2 at offset 4i (lda 2), B 2 x 1 at offset 2i.
    Lh = np.zeros((count, 4))
    Lh[:, 0], Lh[:, 1], Lh[:, 3] = l00, l10, l11
    Lh[:, 2] = 99.0  # upper triangle: never read as a coefficient
    Bh = np.stack([b0, b1], axis=1)
    Ld = torch.from_numpy(Lh.reshape(-1)).cuda()
    Bd = torch.from_numpy(Bh.reshape(-1)).cuda()
    lp, bp = Ld.data_ptr(), Bd.data_ptr()
    probs = [hs.Problem(0, 0, 2, 1, 1.0, 0.0, lp + 32 * i, 2, bp + 16 * i, 2) for i in range(count)]
    hs.trsm_batched(probs)
    torch.cuda.synchronize()
    X = Bd.cpu().numpy().reshape(count, 2)
    x0 = b0 * (1.0 / l00)
    x1 = (b1 - l10 * x0) * (1.0 / l11)
    assert np.array_equal(X[:, 0], x0)
    assert np.array_equal(X[:, 1], x1)


def test_fused_very_small_padded_and_alpha_zero():
    """The fused kernel on problems whose B and L carry padding rows (ldb =
    m + 5, lda = m + 3): the padding of B keeps its sentinel, problems with
    alpha = 0 come back as exact zeros, and the rest match the oracle and
    their single calls bit for bit."""
    rng = np.random.default_rng(78)
    probs, dev = [], []
    for i in range(600):
        m, n = int(rng.integers(1, 17)), int(rng.integers(1, 17))
        cx, unit = bool(i % 2), bool(i % 3 == 0)
        L, B = W.problem(60000 + i, m, n, cx)
        if i % 7 == 0:
            alpha = 0.0
        else:
            alpha = complex(rng.uniform(-2, 2), rng.uniform(-1, 1)) if cx else float(rng.uniform(-2, 2))
        probs.append((L, B, alpha, unit))
    def padded():
        out = []
        for L, B, a, u in probs:
            Bd = hs.to_colmajor(B, ld=B.shape[0] + 5)
            padding_rows(Bd).fill_(W.PAD_SENTINEL)
            out.append((hs.to_colmajor(L, ld=L.shape[0] + 3), Bd, a, u))
        return out
    dev = padded()
    hs.trsm_batched(dev)
    torch.cuda.synchronize()
    dev1 = padded()
    for L, B, a, u in dev1:
        hs.trsm(L, B, a, unit=u)
    torch.cuda.synchronize()
    for k, ((L, B, a, u), (_, Bd, _, _), (_, Bs, _, _)) in enumerate(zip(probs, dev, dev1)):
        m = B.shape[0]
        assert np.all(padding_rows(Bd).cpu().numpy() == W.PAD_SENTINEL), ("padding", k)
        X = hs.from_colmajor(Bd)
        assert X.tobytes() == hs.from_colmajor(Bs).tobytes(), ("batched differs from single", k)
        if a == 0:
            assert not np.any(X), ("alpha zero", k)
        else:
            assert_parity(L, B, X, a, unit=u, tag=("fused padded", k, B.shape))


def test_fused_very_small_batch():
    """Problems with m, n <= 16 run four per wavefront (the fused kernel),
    alone and in batches: every one matches the oracle and its own single
    call bit for bit, in a batch that also holds larger small problems and a
    blocked one, with problems of both data types and diagonal kinds."""
    rng = np.random.default_rng(77)
    probs = []
    for i in range(3001):
        m, n = int(rng.integers(1, 17)), int(rng.integers(1, 17))
        cx, unit = bool(i % 2), bool(i % 5 == 0)
        L, B = W.problem(50000 + i, m, n, cx)
        alpha = complex(rng.uniform(-2, 2), rng.uniform(-1, 1)) if cx else float(rng.uniform(-2, 2))
        probs.append((L, B, alpha, unit))
    probs += mixed_problems(9, 40, big=[(90, 20, True)])
    dev = to_dev(probs)
    hs.trsm_batched(dev)
    torch.cuda.synchronize()
    dev1 = to_dev(probs)
    for L, B, a, u in dev1:
        hs.trsm(L, B, a, unit=u)
    torch.cuda.synchronize()
    for k, ((L, B, a, u), (_, Bd, _, _), (_, Bs, _, _)) in enumerate(zip(probs, dev, dev1)):
        X = hs.from_colmajor(Bd)
        assert X.tobytes() == hs.from_colmajor(Bs).tobytes(), ("batched differs from single", k)
        assert_parity(L, B, X, a, unit=u, tag=("fused", k, B.shape))
