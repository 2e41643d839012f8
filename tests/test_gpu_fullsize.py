"""Parity at the benchmark's full sizes, in the launch configuration the
benchmark times: DTRSM m = n = 16384 (alpha = -1, seed 2) and ZTRSM
m = n = 8192 (alpha = (-1, 0), seed 2) with the tuning table's I_B, checked
on sampled columns against the oracle (columns are independent solves,
Sec. 4.2.1, so a sample of columns is an exact sub-problem); and the whole
10 000-problem batched workload, every problem against the oracle.

At these sizes the top-level trailing update is an (m/2) x n x (m/2)
product of thousands of 128 x 128 tiles, the update configuration that
carries most of the large solves' time.
"""
import time

import numpy as np
import pytest

import oracle
import workloads as W
from parity import U, assert_parity, column_rel_errors

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu
hs = pytest.importorskip("paper_2608_25469_amd")


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)
    hs.lib()


def _large(cfg, ncols):
    m, n, cx, alpha = cfg["m"], cfg["n"], cfg["complex_"], cfg["alpha"]
    t0 = time.time()
    L, B = W.problem(cfg["seed"], m, n, cx)
    print(f"inputs m={m} n={n} complex={cx} in {time.time() - t0:.1f}s", flush=True)
    Ld, Bd = hs.to_colmajor(L), hs.to_colmajor(B)
    _, rep = hs.trsm(Ld, Bd, alpha, report=True)
    torch.cuda.synchronize()
    assert rep["path"] == 2 and rep["block_size"] == hs.lookup_block_size(cx, m, n)
    cols = np.unique(np.linspace(0, n - 1, num=ncols).astype(int))
    X = np.asfortranarray(Bd[:, cols.tolist()].cpu().numpy())
    del Ld, Bd
    torch.cuda.empty_cache()
    Bs = np.asfortranarray(B[:, cols])
    t0 = time.time()
    fro, col, ele, eta = assert_parity(L, Bs, X, alpha, tag=("full size", m, n, cx))
    print(f"m={m} complex={cx}: {len(cols)} columns fro={fro:.2e} worst column={col:.2e} "
          f"element={ele:.2e} eta={eta:.2e} (oracle {time.time() - t0:.1f}s)", flush=True)
    # the Table 2 magnitude (~1e-16 .. 1e-15 at m = 1024 .. 8192)
    assert fro <= 1e-14, fro


def test_dtrsm_16384_sampled_columns():
    _large(W.LARGE_REAL, 16)


def test_ztrsm_8192_sampled_columns():
    _large(W.LARGE_COMPLEX, 16)


def test_batched_workload_every_problem():
    """The 10 000-problem complex workload as the benchmark runs it (a plan
    executed on resident descriptors), every problem against the oracle."""
    b = W.batched(**{k: W.BATCHED[k] for k in ("seed", "count", "lo", "hi", "complex_", "alpha")})
    pl, pb, vl, vb = hs.pack_batch(b.L, b.B)
    plan = hs.BatchPlan([hs.problem_struct(L, B, b.alpha) for L, B in zip(vl, vb)])
    plan.execute()
    torch.cuda.synchronize()
    host = pb.cpu().numpy()
    worst = 0.0
    for i, (L, B) in enumerate(zip(b.L, b.B)):
        off = (vb[i].data_ptr() - pb.data_ptr()) // 16
        m, n = b.shapes[i]
        X = np.asfortranarray(host[off:off + m * n].reshape((n, m)).T)
        ref = oracle.solve(L, B, b.alpha)
        worst = max(worst, float(np.max(column_rel_errors(X, ref))))
        assert_parity(L, B, X, b.alpha, tag=(i, m, n), ref=ref)
    plan.close()
    print(f"10000 problems: worst column error {worst:.2e}", flush=True)
