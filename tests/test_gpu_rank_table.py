"""GPU: the rank table (Sec. 4.2) and the pruning it drives (Lemma 1 (2)).

The table's thresholds must equal the oracle's to the bit (both are spec dot
products with the same norm-stratified sample items, read at the same sorted
positions).  Its cells are certain counts: never above the oracle's exact
count, and below it only by items whose score lies within the low-precision
error of the threshold.  Batch answers with the table must stay identical to
the oracle's exact answers (and to the answers without the table), while the
table rules out most pairs before the screen.
"""
import numpy as np
import pytest
import torch

from oracle import oracle as O
from paper_2504_13446_amd import rkr, workloads as W

pytestmark = pytest.mark.gpu

# a loose bound, relative to |u| max|p|, on how far above a threshold an item
# the certain count misses can score: the band edge sits one error bound E
# above the threshold and the low-precision score is itself within E, so the
# window is 2E (FP32 scores: E <= 2 (dpad + 2) 2^-24 |u| max|p|, 2E about
# 2^-15.9 at dpad = 64); and on the share of the exact counts the certain
# counts may miss
REL_ERR = {"bf16": 2.0 ** -5, "fp8": 2.0 ** -2, "f32": 2.0 ** -14}
MISS = {"bf16": 0.02, "fp8": 0.4, "f32": 0.001}


def _dev(x, dtype):
    return rkr.to_device(x, dtype)


def _answers(ids, rk, off):
    ids = ids.cpu().numpy()
    rk = rk.cpu().numpy()
    return [(ids[off[i]:off[i + 1]], rk[off[i]:off[i + 1]]) for i in range(len(off) - 1)]


@pytest.mark.parametrize("score", ["bf16", "fp8", "f32"])
def test_table_against_oracle(score):
    w = W.make("small", n=1100, m=2900, nq=1)
    S = 300
    idx = rkr.Index(_dev(w.U, w.dtype), _dev(w.P, w.dtype), score=score, rank_table=S)
    t, c = idx.rank_table()
    t = t.cpu().numpy()
    c = c.cpu().numpy().astype(np.int64)
    idx.close()
    sample = O.stratified_sample(w.P, S)
    want_t, want_c = O.rank_table(w.U, w.P, sample, O.sketch_positions(S, rkr.TABLE_COLS))
    assert np.array_equal(t, want_t)
    assert np.all(c <= want_c), np.argwhere(c > want_c)[:5]
    # the shortfall is made of near ties only
    sc = O.dots(w.U, w.P)
    delta = REL_ERR[score] * O.norms(w.U)[:, None] * O.norms(w.P).max()
    near = np.stack([np.sum((sc > want_t[:, j:j + 1]) & (sc <= want_t[:, j:j + 1] + delta), axis=1)
                     for j in range(rkr.TABLE_COLS)], axis=1)
    assert np.all(want_c - c <= near)
    assert (want_c - c).sum() <= MISS[score] * want_c.sum() + rkr.TABLE_COLS * w.n


@pytest.mark.parametrize("score", ["bf16", "fp8", "f32"])
def test_pruned_batch_is_exact(score):
    """Exact and approximate answers with the table equal the oracle's (Def.
    2) or satisfy Def. 3; most non-seed pairs are ruled out by the table."""
    w = W.make("small", n=3000, m=4000, nq=12)
    ks = np.array([1, 5, 10, 20, 3, 40, 10, 10, 7, 64, 2, 15], np.int32)
    R = O.ranks(w.U, w.P, w.Qv)
    idx = rkr.Index(_dev(w.U, w.dtype), _dev(w.P, w.dtype), score=score, rank_table=512)
    Q = _dev(w.Qv, w.dtype)
    ans = _answers(*idx.query_batch(Q, ks))
    st = idx.stats()
    for i, (gi, gr) in enumerate(ans):
        wi, wr = O.topk(R[i], int(ks[i]))
        assert np.array_equal(gr, wr), i
        assert np.array_equal(gi, wi), i
    nonseed = st["pairs"] - st["seed_pairs"]
    assert st["table_pruned"] > 0.8 * nonseed, (st["table_pruned"], nonseed)
    # approximate mode: zero Def. 3 violations
    c = np.full(12, 1.5)
    aans = _answers(*idx.query_batch(Q, ks, c=c))
    for i, (gi, _) in enumerate(aans):
        _, wr = O.topk(R[i], int(ks[i]))
        viol, _ = O.def3_check(R[i][gi], wr, 1.5)
        assert viol == 0, i
    # the same answers without the table
    idx.configure(no_table=True)
    ans2 = _answers(*idx.query_batch(Q, ks))
    assert idx.stats()["table_pruned"] == 0
    for (a, b), (c2, d2) in zip(ans, ans2):
        assert np.array_equal(a, c2) and np.array_equal(b, d2)
    idx.close()


def test_pruned_candidate_lists_and_ties():
    """Candidate lists (CSR domains) and integer data full of exact ties with
    the thresholds (the thresholds are item scores, so every sample item ties
    with its own column)."""
    rng = np.random.default_rng(41)
    n, m, d = 1500, 2500, 6
    U = rng.integers(-2, 3, size=(n, d)).astype(np.float32)
    P = rng.integers(-2, 3, size=(m, d)).astype(np.float32)
    Qv = P[rng.choice(m, 9, replace=False)]
    R = O.ranks(U, P, Qv)
    ks = np.array([1, 4, 9, 16, 25, 3, 7, 30, 12], np.int32)
    lists = [np.sort(rng.choice(n, size, replace=False)) for size in (50, 300, 1500, 900, 64, 700, 200, 1000, 37)]
    off = np.zeros(10, np.int64)
    off[1:] = np.cumsum([len(x) for x in lists])
    cand = np.concatenate(lists).astype(np.int32)
    for score in ("bf16", "fp8"):
        idx = rkr.Index(_dev(U, "f32"), _dev(P, "f32"), score=score, rank_table=256)
        ans = _answers(*idx.query_batch(_dev(Qv, "f32"), ks, cand_off=off, cand_ids=torch.from_numpy(cand).cuda()))
        for i, (gi, gr) in enumerate(ans):
            wi, wr = O.topk(R[i][lists[i]], int(ks[i]), uids=lists[i])
            assert np.array_equal(gr, wr), (score, i)
            assert np.array_equal(gi, wi), (score, i)
        dense = _answers(*idx.query_batch(_dev(Qv, "f32"), ks))
        for i, (gi, gr) in enumerate(dense):
            wi, wr = O.topk(R[i], int(ks[i]))
            assert np.array_equal(gi, wi) and np.array_equal(gr, wr), (score, i)
        idx.close()


def test_table_edge_cases():
    rng = np.random.default_rng(43)
    U = rng.standard_normal((70, 9)).astype(np.float32)
    # fewer items than samples: every item is a sample
    P = rng.standard_normal((5, 9)).astype(np.float32)
    idx = rkr.Index(_dev(U, "f32"), _dev(P, "f32"), score="bf16", rank_table=4096)
    t, c = idx.rank_table()
    want_t, want_c = O.rank_table(U, P, O.stratified_sample(P, 5), O.sketch_positions(5, rkr.TABLE_COLS))
    assert np.array_equal(t.cpu().numpy(), want_t)
    assert np.all(c.cpu().numpy() <= want_c)
    R = O.ranks(U, P, P[:2])
    ids, rk, off = idx.query_batch(_dev(P[:2], "f32"), [3, 70])
    for i, kk in enumerate((3, 70)):
        wi, wr = O.topk(R[i], kk)
        assert np.array_equal(ids.cpu().numpy()[off[i]:off[i + 1]], wi)
    idx.close()
    # no items: no table
    idx = rkr.Index(_dev(U, "f32"), _dev(np.zeros((0, 9), np.float32), "f32"), rank_table=64)
    with pytest.raises(rkr.RkrError) as e:
        idx.rank_table()
    assert e.value.status == rkr.RKR_E_STATE
    idx.close()
    # an index built without a table
    idx = rkr.Index(_dev(U, "f32"), _dev(P, "f32"))
    with pytest.raises(rkr.RkrError):
        idx.rank_table()
    idx.close()
