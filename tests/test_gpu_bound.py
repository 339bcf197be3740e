"""GPU: the error bound every exact rank rests on, checked pair by pair.

The count kernels decide s(u,p) > u.q from a matrix-core score s_hat and a
per-user, per-item-block bound eps with |s_hat - s(u,p)| <= eps, where
s(u,p) is the FP64 spec dot (Def. 1 with the dot product of the masters).
Only the scores inside [u.q - eps, u.q + eps] go to the FP64 recheck, so a
single pair whose error exceeds its eps could give a wrong rank without any
parity test noticing.  rkr_score_error recomputes the spec dot beside every
score of the count kernel and reports the largest |s_hat - s| / eps and the
number of pairs above 1: over a billion pairs of random data and several
inputs built to stress the bound (cancellation, extreme and mixed norms,
entries near the FP32 underflow, integer data, low rank), no pair may exceed
its bound.  rkr_score_error_at does the same for the form the BF16 exact and
screening passes take, with the query's thresholds folded into the
accumulators.
"""
import numpy as np
import pytest

from paper_2504_13446_amd import rkr, workloads as W

pytestmark = pytest.mark.gpu

_PAIRS = {"n": 0}


def _check(U, P, masters, score, slack=1.0):
    idx = rkr.Index(rkr.to_device(U, masters), rkr.to_device(P, masters), score=score)
    try:
        ratio, over = idx.score_error()
    finally:
        idx.close()
    _PAIRS["n"] += U.shape[0] * P.shape[0]
    print(f"  {masters}/{score} n={U.shape[0]} m={P.shape[0]} d={U.shape[1]}: "
          f"max |s_hat - s| / eps = {ratio:.4g}, pairs over = {over}", flush=True)
    assert over == 0
    assert ratio <= slack
    return ratio


def _masters(X, masters):
    X = np.ascontiguousarray(X, np.float32)
    return W.f32_to_bf16_bits(X) if masters == "bf16" else X


@pytest.mark.parametrize("masters,score", [("bf16", "bf16"), ("f32", "f32"), ("f32", "fp8"), ("f32", "bf16")])
def test_random_data_16k_squared(masters, score):
    """16,384 users x 16,384 items (2.7e8 pairs per case, 1.1e9 over the four)."""
    w = W.make("batch" if masters == "bf16" else "single", n=16_384, m=16_384, nq=1)
    ratio = _check(w.U, w.P, masters, score)
    assert ratio > 1e-3            # the check sees real rounding errors, not zeros


@pytest.mark.parametrize("score", ["bf16", "f32", "fp8"])
def test_cancellation(score):
    """Rows of large entries of alternating sign against nearly constant rows:
    partial sums grow to |u||p| while the dots stay near zero, so the error of
    the low-precision products dominates and the bound's norm terms are tight."""
    rng = np.random.default_rng(21)
    n, m, d = 4096, 4096, 128
    sign = np.where(np.arange(d) % 2 == 0, 1.0, -1.0)
    U = sign[None, :] * rng.uniform(1e3, 2e3, size=(n, 1)) * (1 + 1e-3 * rng.standard_normal((n, d)))
    P = 1.0 + 1e-2 * rng.standard_normal((m, d))
    _check(_masters(U, "f32"), _masters(P, "f32"), "f32", score)


@pytest.mark.parametrize("score", ["bf16", "f32", "fp8"])
def test_extreme_and_mixed_norms(score):
    """Row norms from 2^-36 to 2^36 on both sides (products from 2^-72 to
    2^72), and rows mixing entries 2^20 apart in magnitude."""
    rng = np.random.default_rng(22)
    n, m, d = 4096, 4096, 96
    U = rng.standard_normal((n, d)) * np.exp2(rng.integers(-36, 37, size=(n, 1)))
    P = rng.standard_normal((m, d)) * np.exp2(rng.integers(-36, 37, size=(m, 1)))
    U[: n // 4] *= np.exp2(rng.integers(-10, 11, size=(n // 4, d)))
    P[: m // 4] *= np.exp2(rng.integers(-10, 11, size=(m // 4, d)))
    _check(_masters(U, "f32"), _masters(P, "f32"), "f32", score)


@pytest.mark.parametrize("masters,score", [("f32", "bf16"), ("f32", "f32"), ("f32", "fp8"), ("bf16", "bf16")])
def test_entries_near_underflow(masters, score):
    """Entries of 2^-50 .. 2^-60 (products near the FP32 normal limit 2^-126
    and below it), alone and beside ordinary entries in the same row."""
    rng = np.random.default_rng(23)
    n, m, d = 2048, 4096, 64
    U = rng.standard_normal((n, d)) * np.exp2(rng.integers(-60, -49, size=(n, d)))
    P = rng.standard_normal((m, d)) * np.exp2(rng.integers(-60, -49, size=(m, d)))
    U[n // 2:, : d // 4] = rng.standard_normal((n - n // 2, d // 4))
    P[m // 2:, : d // 4] = rng.standard_normal((m - m // 2, d // 4))
    _check(_masters(U, masters), _masters(P, masters), masters, score)


@pytest.mark.parametrize("score", ["bf16", "f32", "fp8"])
def test_integer_data(score):
    """Small integers: the spec dots are exact and many scores tie."""
    rng = np.random.default_rng(24)
    U = rng.integers(-7, 8, size=(4096, 200)).astype(np.float32)
    P = rng.integers(-7, 8, size=(4096, 200)).astype(np.float32)
    _check(U, P, "f32", score)


@pytest.mark.parametrize("score", ["bf16", "fp8"])
def test_low_rank_uneven_dimension(score):
    """Low-rank data (shared 20-dim basis) at d = 300 with ragged n and m."""
    w = W.make("uneven", n=3_001, m=5_003, d=300, nq=1)
    _check(w.U, w.P, "f32", score)


def _check_at(U, P, Q, masters, slack=1.0, score="bf16"):
    """The threshold-folded form of the BF16 passes, for each query of Q."""
    idx = rkr.Index(rkr.to_device(U, masters), rkr.to_device(P, masters), score=score)
    worst = 0.0
    try:
        for j in range(Q.shape[0]):
            ratio, over = idx.score_error_at(rkr.to_device(Q[j:j + 1], masters)[0])
            print(f"  folded {masters} n={U.shape[0]} m={P.shape[0]} d={U.shape[1]} query {j}: "
                  f"max |acc - (s - th)| / bound = {ratio:.4g}, pairs over = {over}", flush=True)
            assert over == 0
            assert ratio <= slack
            worst = max(worst, ratio)
    finally:
        idx.close()
    return worst


def test_folded_random_batch_data():
    """16,384 x 16,384 pairs of the batch workload for two of its queries, and
    for a query 2^20 times longer (|th| far above every |u||p|: the folded
    threshold's own rounding dominates)."""
    w = W.make("batch", n=16_384, m=16_384, nq=2)
    Q = np.concatenate([W.bf16_bits_to_f32(w.Qv), 2.0 ** 20 * W.bf16_bits_to_f32(w.Qv[:1])])
    ratio = _check_at(w.U, w.P, _masters(Q, "bf16"), "bf16")
    assert ratio > 1e-3


def test_folded_stress_inputs():
    """Cancellation, extreme norms and integer data, each with a query equal to
    an item (thresholds among the scores) and a zero query (th = 0)."""
    rng = np.random.default_rng(31)
    n, m, d = 4096, 4096, 128
    sign = np.where(np.arange(d) % 2 == 0, 1.0, -1.0)
    cases = [
        (sign[None, :] * rng.uniform(1e3, 2e3, size=(n, 1)) * (1 + 1e-3 * rng.standard_normal((n, d))),
         1.0 + 1e-2 * rng.standard_normal((m, d))),
        (rng.standard_normal((n, d)) * np.exp2(rng.integers(-36, 37, size=(n, 1))),
         rng.standard_normal((m, d)) * np.exp2(rng.integers(-36, 37, size=(m, 1)))),
        (rng.integers(-7, 8, size=(n, d)).astype(np.float64), rng.integers(-7, 8, size=(m, d)).astype(np.float64)),
    ]
    for U, P in cases:
        Q = np.stack([P[7], P[m // 2] * 3.0, np.zeros(d)])
        _check_at(_masters(U, "f32"), _masters(P, "f32"), _masters(Q, "f32"), "f32")


def test_folded_uneven_dimension():
    """Low-rank data at d = 300 with ragged n and m (dpad 304), two queries."""
    w = W.make("uneven", n=3_001, m=5_003, d=300, nq=2)
    _check_at(w.U, w.P, w.Qv, "f32")


def _split_stress_cases(rng, n, m, d):
    sign = np.where(np.arange(d) % 2 == 0, 1.0, -1.0)
    U1 = rng.standard_normal((n, d)) * np.exp2(rng.integers(-60, -49, size=(n, d)))
    P1 = rng.standard_normal((m, d)) * np.exp2(rng.integers(-60, -49, size=(m, d)))
    U1[n // 2:, : d // 4] = rng.standard_normal((n - n // 2, d // 4))
    P1[m // 2:, : d // 4] = rng.standard_normal((m - m // 2, d // 4))
    return {
        "cancellation": (sign[None, :] * rng.uniform(1e3, 2e3, size=(n, 1)) * (1 + 1e-3 * rng.standard_normal((n, d))),
                         1.0 + 1e-2 * rng.standard_normal((m, d))),
        "extreme norms": (rng.standard_normal((n, d)) * np.exp2(rng.integers(-36, 37, size=(n, 1)))
                          * np.exp2(rng.integers(-10, 11, size=(n, d))),
                          rng.standard_normal((m, d)) * np.exp2(rng.integers(-36, 37, size=(m, 1)))),
        "near underflow": (U1, P1),
        "integers": (rng.integers(-7, 8, size=(n, d)).astype(np.float64),
                     rng.integers(-7, 8, size=(m, d)).astype(np.float64)),
    }


def test_split_bf16_random_and_stress():
    """Split BF16 scores (hi + lo per value, three products per term): the
    low-rank single-query data at 16,384 x 16,384, and the stress inputs above
    at d = 96, against their bound, plain and with a query's thresholds folded
    in.  The split's bound is about 2^-13 of the BF16 one's width on FP32
    data, so the checks must also see errors well above zero."""
    w = W.make("single", n=16_384, m=16_384, nq=2)
    ratio = _check(w.U, w.P, "f32", "bf16x3")
    assert ratio > 1e-3
    _check_at(w.U, w.P, w.Qv, "f32", score="bf16x3")
    rng = np.random.default_rng(41)
    n, m, d = 4096, 4096, 96
    for name, (U, P) in _split_stress_cases(rng, n, m, d).items():
        print("  split BF16, " + name, flush=True)
        U32, P32 = _masters(U, "f32"), _masters(P, "f32")
        _check(U32, P32, "f32", "bf16x3")
        Q = np.stack([P[5], P[m // 3] * 2.0, np.zeros(d)])
        _check_at(U32, P32, _masters(Q, "f32"), "f32", score="bf16x3")
    # BF16 masters: lo is zero, the split score is the BF16 one
    wb = W.make("small", n=3000, m=5000, d=50, dtype="bf16")
    _check(wb.U, wb.P, "bf16", "bf16x3")


def test_pair_total():
    """The checks above covered more than a billion (user, item) pairs."""
    if _PAIRS["n"] == 0:
        pytest.skip("the bound checks did not run in this process")
    assert _PAIRS["n"] > 1_000_000_000, _PAIRS["n"]
