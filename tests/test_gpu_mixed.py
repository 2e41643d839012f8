"""Mixed-precision mode (FP32 matrix-core updates, FP64 residual refinement)
and the backward-error report, against the oracle."""
import numpy as np
import pytest

import oracle
import workloads as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu
hs = pytest.importorskip("paper_2608_25469_amd")


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)
    hs.lib()


def sample_eta(L, X, B, cols, alpha=1.0):
    return oracle.backward_error(L, np.asfortranarray(X[:, cols]), np.asfortranarray(B[:, cols]), alpha)


@pytest.mark.parametrize("kappa", [1e3, 1e6])
def test_mixed_auto_refinement_reaches_target(kappa):
    m, n = 1024, 192
    L, B = W.mixed_problem(m, n, kappa)
    Ld, Bd = hs.to_colmajor(L), hs.to_colmajor(B)
    _, rep = hs.trsm(Ld, Bd, 1.0, mixed=True, refine_steps=-1, refine_tol=1e-13, report=True)
    X = hs.from_colmajor(Bd)
    assert rep["path"] == 2 and 0 <= rep["refine_steps"] <= 4
    assert 0 <= rep["backward_error"] <= 1e-13, rep
    cols = list(range(0, n, 12))
    eta = sample_eta(L, X, B, cols)
    assert eta <= 1e-13, eta
    # forward error against the oracle, reported: bounded by kappa * eta
    ref = oracle.solve(L, np.asfortranarray(B[:, cols]), 1.0)
    fe = oracle.rel_err_fro(X[:, cols], ref)
    assert fe <= 10 * kappa * 1e-13, fe


def test_mixed_without_refinement_is_single_precision_level():
    m, n = 1024, 128
    L, B = W.mixed_problem(m, n, 1e3)
    Ld, Bd = hs.to_colmajor(L), hs.to_colmajor(B)
    _, rep = hs.trsm(Ld, Bd, 1.0, mixed=True, refine_steps=0, backward_error=True, report=True)
    X = hs.from_colmajor(Bd)
    eta = sample_eta(L, X, B, list(range(0, n, 8)))
    # FP32 products: far above FP64 rounding, far below O(1)
    assert 1e-14 < eta < 1e-5, eta
    assert rep["refine_steps"] == 0
    # the library's eta is over all columns, the oracle's over every eighth
    assert 0.2 * eta <= rep["backward_error"] <= 5 * eta, (rep["backward_error"], eta)


def test_fixed_steps_and_fp64_report():
    m, n = 700, 64
    L, B = W.mixed_problem(1024, n, 1e4)
    L, B = np.asfortranarray(L[:m, :m]), np.asfortranarray(B[:m])
    Ld, Bd = hs.to_colmajor(L), hs.to_colmajor(B)
    _, rep = hs.trsm(Ld, Bd, -0.5, mixed=True, refine_steps=2, backward_error=True, report=True)
    assert rep["refine_steps"] == 2 and 0 <= rep["backward_error"] <= 1e-13
    X = hs.from_colmajor(Bd)
    eta = sample_eta(L, X, B, list(range(0, n, 4)), -0.5)
    assert eta <= 1e-13
    # plain FP64 path with the backward-error report
    Bd2 = hs.to_colmajor(B)
    _, rep2 = hs.trsm(Ld, Bd2, -0.5, backward_error=True, report=True)
    X2 = hs.from_colmajor(Bd2)
    eta2 = oracle.backward_error(L, X2, B, -0.5)
    assert rep2["refine_steps"] == 0
    assert eta2 <= 10 * m * 2.0 ** -53
    assert rep2["backward_error"] <= 10 * m * 2.0 ** -53


def test_mixed_exact_on_bidiagonal():
    """Integer data with partial sums below 2^24 is exact in FP32 too, so the
    mixed path must return the closed form bit for bit."""
    rng = np.random.default_rng(8)
    m = 600
    B = W.integer_rhs(rng, m, 20, -20, 20)
    Ld = hs.to_colmajor(W.bidiagonal_lower(m, 4.0))
    Bd = hs.to_colmajor(B)
    hs.trsm(Ld, Bd, 2.0, mixed=True, block_size=64)
    torch.cuda.synchronize()
    assert np.array_equal(hs.from_colmajor(Bd), np.cumsum(B, axis=0) * 0.5)


def test_mixed_rejects_complex():
    L, B = W.problem(1, 100, 10, True)
    with pytest.raises(hs.HsmaError) as e:
        hs.trsm(hs.to_colmajor(L), hs.to_colmajor(B), 1.0, mixed=True)
    assert e.value.status == 6


@pytest.mark.parametrize("cx", [False, True], ids=["real", "complex"])
@pytest.mark.parametrize("unit", [False, True], ids=["nonunit", "unit"])
def test_fp64_backward_error_report_against_oracle(cx, unit):
    """The FP64 path's reported backward error is a real measurement: it lies
    within a factor of 10 of the oracle's (Dot2 residual) on the same result,
    both ways.  A residual walked in the solve's own order would report far
    less (the update rounding cancels out of it)."""
    for m, n, ib in ((2048, 96, 128), (700, 40, 64), (48, 30, 0)):
        L, B = W.problem(300 + m, m, n, cx)
        alpha = complex(-1.0, 0.0) if cx else -1.0
        Ld, Bd = hs.to_colmajor(L), hs.to_colmajor(B)
        _, rep = hs.trsm(Ld, Bd, alpha, unit=unit, block_size=ib, backward_error=True, report=True)
        X = hs.from_colmajor(Bd)
        eta = oracle.backward_error(L, X, B, alpha, unit=unit)
        assert rep["refine_steps"] == 0
        assert 0.1 * eta <= rep["backward_error"] <= 10 * eta, (m, cx, unit, rep["backward_error"], eta)
        assert rep["backward_error"] <= 10 * m * 2.0 ** -53


@pytest.mark.parametrize("unit", [False, True], ids=["nonunit", "unit"])
def test_complex_refinement_fp64(unit):
    """Complex data: fixed FP64 refinement steps and the stop-at-tolerance
    mode; the result meets the oracle's parity bars and the reported backward
    error bounds the oracle's."""
    from parity import assert_parity
    m, n = 900, 50
    L, B = W.problem(77, m, n, True)
    alpha = complex(0.5, -1.25)
    for steps in (1, 2, -1):
        Ld, Bd = hs.to_colmajor(L), hs.to_colmajor(B)
        _, rep = hs.trsm(Ld, Bd, alpha, unit=unit, refine_steps=steps, backward_error=True,
                         refine_tol=1e-14, report=True)
        X = hs.from_colmajor(Bd)
        _, _, _, eta = assert_parity(L, B, X, alpha, unit=unit, tag=("complex refine", steps))
        assert rep["refine_steps"] == (steps if steps > 0 else rep["refine_steps"])
        assert 0 <= rep["refine_steps"] <= 4
        assert 0.1 * eta <= rep["backward_error"] <= 10 * eta, (steps, rep["backward_error"], eta)


def test_refinement_reduces_fp64_residual_for_bad_conditioning():
    """At kappa ~1e6 one FP64 refinement step does not raise the backward
    error (the independent residual sees the solve's true error)."""
    m, n = 1024, 64
    L, B = W.mixed_problem(m, n, 1e6)
    Ld = hs.to_colmajor(L)
    etas = []
    for steps in (0, 1):
        Bd = hs.to_colmajor(B)
        _, rep = hs.trsm(Ld, Bd, 1.0, refine_steps=steps, backward_error=True, report=True)
        X = hs.from_colmajor(Bd)
        eta = oracle.backward_error(L, X, B, 1.0)
        etas.append(eta)
        assert 0.1 * eta <= rep["backward_error"] <= 10 * eta
    assert etas[1] <= 2 * etas[0] + 1e-17, etas
