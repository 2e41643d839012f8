"""Serving on the GPU: the device input generator against the host one, each
queued result against the same solve run alone (bit for bit) and against the
oracle, with requests arriving while earlier ones run."""
import time

import numpy as np
import pytest

import oracle
import workloads as W
from parity import assert_parity

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


@pytest.mark.parametrize("m,n,cx", [(1, 1, False), (37, 5, True), (300, 70, False),
                                    (129, 3, True), (64, 200, False)])
def test_device_generator_matches_host(m, n, cx):
    key = W.serving_key(4, 1000 + m)
    Ld, Bd = hs.generate_inputs(m, n, key, complex_=cx)
    torch.cuda.synchronize()
    Lh, Bh = W.synthetic_inputs(m, n, key, cx)
    # L uses only exactly rounded operations: identical bits
    assert np.array_equal(hs.from_colmajor(Ld), Lh)
    # B goes through log, sqrt, cos, sin: a few ulps apart at most
    Bg = hs.from_colmajor(Bd)
    assert np.all(np.abs(Bg - Bh) <= 1e-14 * np.maximum(1.0, np.abs(Bh)))


def _problems(seed):
    """Small, medium and a few large problems of both data types."""
    rng = np.random.default_rng(seed)
    shapes = [(int(m), int(n)) for m, n in zip(rng.integers(1, 65, 24), rng.integers(1, 140, 24))]
    shapes += [(int(m), int(n)) for m, n in zip(rng.integers(65, 700, 12), rng.integers(1, 300, 12))]
    shapes += [(1500, 257), (2100, 64), (1024, 1024)]
    probs = []
    for i, (m, n) in enumerate(shapes):
        cx = i % 3 == 1
        unit = i % 5 == 2
        L, B = W.problem(seed * 1000 + i, m, n, cx)
        alpha = complex(rng.uniform(-2, 2), 0.0) if cx else float(rng.uniform(-2, 2))
        probs.append((L, B, alpha, unit, cx))
    return probs


def test_queue_results_equal_alone_and_oracle():
    probs = _problems(7)
    # alone: one hsma_trsm per problem
    alone = []
    for L, B, a, u, cx in probs:
        Ld, Bd = hs.to_colmajor(L), hs.to_colmajor(B)
        hs.trsm(Ld, Bd, a, unit=u)
        alone.append(Bd)
    torch.cuda.synchronize()
    # in the mix: submitted in waves while earlier waves run
    dev = [(hs.to_colmajor(L), hs.to_colmajor(B)) for L, B, _, _, _ in probs]
    torch.cuda.synchronize()
    order = np.random.default_rng(3).permutation(len(probs))
    tickets = {}
    with hs.Queue(n_streams=4) as q:
        for wave in np.array_split(order, 6):
            reqs = []
            for i in wave:
                L, B, a, u, cx = probs[i]
                Ld, Bd = dev[i]
                reqs.append(hs.request(B.shape[0], B.shape[1], a, unit=u, complex_=cx, L=Ld, B=Bd))
            for i, t in zip(wave, q.submit(reqs, tensors=[dev[i] for i in wave])):
                tickets[int(i)] = t
            time.sleep(0.002)
        infos = {i: q.wait(t, 60) for i, t in tickets.items()}
        st = q.stats()
    assert st["completed"] == len(probs) and st["failed"] == 0
    overlapped = sum(1 for i in infos for j in infos
                     if i != j and infos[j]["t_admit_ns"] < infos[i]["t_done_ns"]
                     and infos[i]["t_admit_ns"] < infos[j]["t_done_ns"])
    assert overlapped > 0, "no two requests were in flight together"
    for i, (L, B, a, u, cx) in enumerate(probs):
        assert infos[i]["path"] == (1 if B.shape[0] <= 64 else 2)
        X = hs.from_colmajor(dev[i][1])
        Xa = hs.from_colmajor(alone[i])
        assert X.tobytes() == Xa.tobytes(), f"problem {i} differs from its solve alone"
        if i % 2 == 0 or B.shape[0] <= 700:
            assert_parity(L, B, X, a, unit=u, tag=("served", i, B.shape))


def test_synthetic_requests_against_oracle():
    shapes = [(8, 1, False), (40, 64, True), (64, 300, False), (65, 7, True), (257, 130, False),
              (600, 33, True), (1100, 200, False)]
    keys = [W.serving_key(4, 500 + i) for i in range(len(shapes))]
    with hs.Queue() as q:
        tk = q.submit([hs.request(m, n, -1.25, complex_=cx, key=k, release_on_completion=False)
                       for (m, n, cx), k in zip(shapes, keys)])
        # load that frees itself, interleaved
        q.submit([hs.request(48, 48, 1.0, key=W.serving_key(9, i)) for i in range(200)])
        for (m, n, cx), k, t in zip(shapes, keys, tk):
            info = q.wait(t, 60)
            assert info["status"] == 0 and info["lda"] == m and info["ldb"] == m
            X = hs.matrix_from_pointer(info["B"], m, n, m, cx)
            Lh, Bh = W.synthetic_inputs(m, n, k, cx)
            # the device draws B with its own libm: inputs agree to ~1e-15, so
            # the bars are the relative-error ones, not the backward error
            assert_parity(Lh, Bh, X, -1.25, tag=("synthetic", m, n, cx), check_eta=False)
            q.release(t)
        for _ in range(200):
            if q.stats()["completed"] == 207:
                break
            time.sleep(0.01)
        st = q.stats()
        assert st["completed"] == 207
        assert st["bytes_in_use"] == 0
        assert st["p50_ns"] > 0 and st["p99_ns"] >= st["p50_ns"]


def test_fire_and_forget_load_frees_everything():
    """Fire-and-forget synthetic load (release_on_completion = 2) mixed with
    kept requests: the forgotten records are gone, every byte of budget comes
    back, and the kept results still match the oracle."""
    shapes = [(30, 5, False), (200, 17, True), (700, 3, False)]
    keys = [W.serving_key(5, 900 + i) for i in range(len(shapes))]
    with hs.Queue() as q:
        q.stats_reset(hs.clock_ns())
        forgot = q.submit([hs.request(8 + (i * 37) % 900, 1 + i % 50, 0.5, complex_=bool(i % 3 == 0),
                                      key=W.serving_key(6, i), forget=True) for i in range(300)])
        kept = q.submit([hs.request(m, n, 2.0, complex_=cx, key=k, release_on_completion=False)
                         for (m, n, cx), k in zip(shapes, keys)])
        for (m, n, cx), k, t in zip(shapes, keys, kept):
            info = q.wait(t, 60)
            X = hs.matrix_from_pointer(info["B"], m, n, m, cx)
            Lh, Bh = W.synthetic_inputs(m, n, k, cx)
            assert_parity(Lh, Bh, X, 2.0, tag=("kept", m, n, cx), check_eta=False)
            q.release(t)
        for _ in range(2000):
            if q.stats()["completed"] == 303:
                break
            time.sleep(0.01)
        st = q.stats()
        assert st["completed"] == 303 and st["failed"] == 0
        assert st["bytes_in_use"] == 0 and st["inflight"] == 0
        assert st["all"]["count"] == 303
        assert sum(c["count"] for c in st["by_class"].values()) == 303
        assert all(q.poll(t)[0] == 11 for t in forgot)
