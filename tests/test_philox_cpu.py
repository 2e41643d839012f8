"""Host Philox4x32-10 and the synthetic serving inputs drawn from it.

The generator is pinned by the published known-answer vectors; the input
recipe by its distributional and structural facts."""
import json
import os

import numpy as np
import pytest

import workloads as W

HERE = os.path.dirname(os.path.abspath(__file__))


def _kat():
    with open(os.path.join(HERE, "golden", "philox4x32_10_kat.json")) as f:
        return json.load(f)["vectors"]


@pytest.mark.parametrize("v", _kat())
def test_known_answer_vectors(v):
    c = [int(x, 16) for x in v["counter"]]
    k = [int(x, 16) for x in v["key"]]
    out = [int(x) for x in W.philox4x32_10(c, k)]
    assert out == [int(x, 16) for x in v["out"]]


def test_vectorised_matches_scalar():
    rng = np.random.default_rng(5)
    cs = rng.integers(0, 2**32, size=(4, 17), dtype=np.uint64)
    key = (0x12345678, 0x9ABCDEF0)
    vec = W.philox4x32_10(list(cs), key)
    for j in range(17):
        one = W.philox4x32_10([int(cs[i, j]) for i in range(4)], key)
        assert [int(x) for x in one] == [int(vec[i][j]) for i in range(4)]


def test_uniforms_range_and_moments():
    u1, u2 = W.philox_uniforms(np.arange(200000, dtype=np.uint64), 0, W.serving_key(4, 3))
    for u in (u1, u2):
        assert u.min() >= 0.0 and u.max() < 1.0
        assert abs(u.mean() - 0.5) < 0.005
        assert abs(u.var() - 1.0 / 12.0) < 0.002
    # 53-bit values: u * 2^53 is an integer
    assert np.all(np.floor(u1 * 2.0**53) == u1 * 2.0**53)
    # different tags and keys give different streams
    v1, _ = W.philox_uniforms(np.arange(1000, dtype=np.uint64), 1, W.serving_key(4, 3))
    w1, _ = W.philox_uniforms(np.arange(1000, dtype=np.uint64), 0, W.serving_key(4, 4))
    assert not np.array_equal(u1[:1000], v1) and not np.array_equal(u1[:1000], w1)


@pytest.mark.parametrize("cx", [False, True])
def test_synthetic_inputs_structure(cx):
    m, n = 300, 200
    L, B = W.synthetic_inputs(m, n, W.serving_key(4, 11), cx)
    assert L.flags.f_contiguous and B.flags.f_contiguous
    assert L.shape == (m, m) and B.shape == (m, n)
    assert np.all(np.triu(L, 1) == 0)
    d = np.diag(L)
    assert np.all(d.real >= 1.0) and np.all(d.real < 2.0)
    if cx:
        assert np.all(np.abs(d.imag) <= 0.5)
    low = L[np.tril_indices(m, -1)]
    assert np.abs(low.real).max() <= 1.0 / m
    assert abs(low.real.mean()) < 0.05 / m
    b = B.real.ravel()
    assert abs(b.mean()) < 0.02 and abs(b.var() - 1.0) < 0.03
    # same key -> same data; the first column of L does not depend on m's later columns
    L2, B2 = W.synthetic_inputs(m, n, W.serving_key(4, 11), cx)
    assert np.array_equal(L, L2) and np.array_equal(B, B2)
