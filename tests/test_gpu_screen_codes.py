"""GPU: the screening pass's 7-bit code compare on inputs built to break it.

The screen drops a pair once its lower-bound count exceeds the query's bound;
an overcount would drop a pair of the exact answer, so exact top-k answers
against the oracle are the check.  Every case uses at least eight queries so
that lanes hold enough live entries for the code compare to run."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2504_13446_amd import rkr

pytestmark = pytest.mark.gpu


def _dev(x, dtype):
    return rkr.to_device(x, dtype)


def _check(idx, U, P, Qv, ks):
    R = O.ranks(U, P, Qv)
    ids, rk, off = idx.query_batch(_dev(Qv, "f32"), ks)
    ids = ids.cpu().numpy(); rk = rk.cpu().numpy()
    for i in range(Qv.shape[0]):
        wi, wr = O.topk(R[i], int(ks[i]))
        assert np.array_equal(ids[off[i]:off[i + 1]], wi), i
        assert np.array_equal(rk[off[i]:off[i + 1]], wr), i
    return idx.stats()


@pytest.mark.parametrize("score", ["bf16", "fp8", "f32"])
def test_flat_steps(score):
    """Five distinct item vectors, each repeated 160 times: after the norm sort
    whole steps hold one item, every lane sees a flat score range (scale 0,
    nothing counted by codes)."""
    rng = np.random.default_rng(71)
    d = 24
    base = rng.standard_normal((5, d)).astype(np.float32)
    P = np.repeat(base, 160, axis=0)
    U = rng.standard_normal((400, d)).astype(np.float32)
    Qv = np.concatenate([base, rng.standard_normal((5, d)).astype(np.float32)])
    idx = rkr.Index(_dev(U, "f32"), _dev(P, "f32"), score=score)
    _check(idx, U, P, Qv, np.array([1, 3, 10, 25, 50, 7, 7, 90, 2, 13], np.int32))
    idx.close()


@pytest.mark.parametrize("score", ["bf16", "f32"])
def test_offset_scores(score):
    """Scores = 1000 + a small spread: the codes' range is tiny against the
    scores' magnitude (x - mn loses no bits that matter, the codes must still
    only undercount)."""
    rng = np.random.default_rng(72)
    n, m, d = 900, 1500, 16
    U = rng.standard_normal((n, d)).astype(np.float32) * 1e-3
    U[:, 0] = 1.0
    P = rng.standard_normal((m, d)).astype(np.float32)
    P[:, 0] = 1000.0
    Qv = np.concatenate([P[rng.choice(m, 8, replace=False)], rng.standard_normal((4, d)).astype(np.float32)])
    Qv[8:, 0] = 1000.0
    idx = rkr.Index(_dev(U, "f32"), _dev(P, "f32"), score=score)
    _check(idx, U, P, Qv, np.full(12, 20, np.int32))
    idx.close()


@pytest.mark.parametrize("score", ["bf16", "fp8"])
def test_integer_ties_many_queries(score):
    """Entries in {-1, 0, 1}: scores are small integers, so most codes sit on
    the thresholds' own code; 24 queries keep the code compare on."""
    rng = np.random.default_rng(73)
    n, m, d = 700, 2100, 6
    U = rng.integers(-1, 2, size=(n, d)).astype(np.float32)
    P = rng.integers(-1, 2, size=(m, d)).astype(np.float32)
    Qv = P[rng.choice(m, 24, replace=False)]
    idx = rkr.Index(_dev(U, "f32"), _dev(P, "f32"), score=score)
    ks = np.array([1, 2, 5, 9, 17, 33, 60, 100] * 3, np.int32)
    _check(idx, U, P, Qv, ks)
    idx.close()


def test_screen_kills_what_it_should():
    """The screen's pruning power, pinned.  Seeds follow the default rule (the
    2k users of smallest -t/|u|, ties to the smaller id), the bound B_q is the
    k-th smallest seed rank, and the screen drops a pair once its certain
    count reaches B_q.  So every non-seed pair of rank <= B_q must survive,
    and a pair of rank well above B_q must not (only items inside the error
    band or sharing a threshold's 7-bit code go uncounted)."""
    from paper_2504_13446_amd import workloads as W
    w = W.make("small", n=3000, m=4000, nq=12)
    k = 20
    idx = rkr.Index(_dev(w.U, "f32"), _dev(w.P, "f32"), score="bf16")
    idx.configure(seed_mult=2)
    R = O.ranks(w.U, w.P, w.Qv).astype(np.int64)
    T = O.dots(w.U, w.Qv)                                     # [n, nq]
    nu = O.norms(w.U)
    lo = hi = 0
    for q in range(w.Qv.shape[0]):
        h = (-T[:, q] / nu).astype(np.float32)
        seeds = np.lexsort((np.arange(w.n), h))[:2 * k]
        _, wr = O.topk(R[q][seeds], k, uids=seeds)
        B = int(wr[-1])
        nonseed = np.ones(w.n, bool); nonseed[seeds] = False
        lo += int(np.sum(nonseed & (R[q] <= B)))
        hi += int(np.sum(nonseed & (R[q] <= 1.3 * B + 10)))
    ids, rk, off = idx.query_batch(_dev(w.Qv, "f32"), np.full(w.Qv.shape[0], k, np.int32))
    st = idx.stats()
    idx.close()
    assert lo <= st["survivors"] <= hi, (lo, st["survivors"], hi)


@pytest.mark.parametrize("cand", [3, 4, 5])
def test_persistent_screen_launch(cand, monkeypatch):
    """The persistent work-queue launch of the screening pass (workgroups take
    user tiles from a device counter) runs only on phases with at least one
    tile per compute unit.  140,000 users x 3,000 items x d = 32 with 16
    queries and no rank table gives every user a live pair in the first phase:
    547 tiles of 256 users (274 of 512 for tile variant 0).  Each persistent
    candidate of the tuner (3 + tile variant) is forced and the answers are
    compared with the oracle's, element by element."""
    from paper_2504_13446_amd import workloads as W
    w = W.make("small", n=140_000, m=3_000, d=32, nq=16, k=10)
    R = _ranks_cached(w)
    monkeypatch.setenv("RKR_SCREEN_CANDIDATE", str(cand))
    monkeypatch.setenv("RKR_AUTOTUNE_CACHE", "off")
    idx = rkr.Index(_dev(w.U, "f32"), _dev(w.P, "f32"), score="bf16")
    ids, rk, off = idx.query_batch(_dev(w.Qv, "f32"), w.k)
    st = idx.stats()
    idx.close()
    assert st["screen_variant"] == cand
    assert st["persistent_phases"] >= 1, st
    ids = ids.cpu().numpy(); rk = rk.cpu().numpy()
    for i in range(w.nq):
        wi, wr = O.topk(R[i], int(w.k[i]))
        assert np.array_equal(ids[off[i]:off[i + 1]], wi), i
        assert np.array_equal(rk[off[i]:off[i + 1]], wr), i


_RANKS = {}


def _ranks_cached(w):
    key = (w.name, w.n, w.m, w.d, w.nq)
    if key not in _RANKS:
        _RANKS[key] = O.ranks(w.U, w.P, w.Qv)
    return _RANKS[key]


@pytest.mark.parametrize("score", ["bf16", "fp8", "f32"])
def test_bucketed_counting_answers_equal_the_oracle(score, monkeypatch):
    """Bucketed counting (a histogram of a step's codes per user over both
    lanes of its pair, then one lookup per pair) must keep the counts lower
    bounds of the certain counts: with 64 queries and no rank table every lane
    starts with 64 live pairs, so the screen takes the histogram path; the
    answers, with it forced on and switched off, equal the oracle's."""
    from paper_2504_13446_amd import workloads as W
    w = W.make("small", n=6_000, m=5_000, d=40, nq=64, k=10)
    R = O.ranks(w.U, w.P, w.Qv)
    for hist in ("12", "0"):
        monkeypatch.setenv("RKR_SCREEN_HIST", hist)
        monkeypatch.setenv("RKR_AUTOTUNE_CACHE", "off")
        idx = rkr.Index(_dev(w.U, "f32"), _dev(w.P, "f32"), score=score)
        ids, rk, off = idx.query_batch(_dev(w.Qv, "f32"), w.k)
        idx.close()
        ids, rk = ids.cpu().numpy(), rk.cpu().numpy()
        for i in range(w.nq):
            wi, wr = O.topk(R[i], int(w.k[i]))
            assert np.array_equal(ids[off[i]:off[i + 1]], wi), (hist, i)
            assert np.array_equal(rk[off[i]:off[i + 1]], wr), (hist, i)
