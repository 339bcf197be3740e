"""GPU: the paper's own query on the rank table (Sec. 4.3, steps 1-3).

On small-integer data with FP32 scores every score lies a whole unit away
from any threshold it does not equal, far beyond the FP32 error bound, so the
table's certain counts are the exact counts: the device table must equal the
oracle's, and the device answer (ids and the bound or estimate each user was
chosen by) must equal the oracle's table query element by element, in both
cases of step 2.
"""
import numpy as np
import pytest
import torch

from oracle import oracle as O
from paper_2504_13446_amd import rkr

pytestmark = pytest.mark.gpu


def _dev(x):
    return rkr.to_device(x, "f32")


@pytest.fixture(scope="module")
def case():
    rng = np.random.default_rng(71)
    n, m, d, S = 2600, 3100, 6, 256
    U = rng.integers(-3, 4, size=(n, d)).astype(np.float32)
    P = rng.integers(-3, 4, size=(m, d)).astype(np.float32)
    Qv = np.vstack([P[[4, 900, 2500]], rng.integers(-3, 4, size=(2, d)).astype(np.float32)])
    idx = rkr.Index(_dev(U), _dev(P), score="f32", rank_table=S)
    t, c = idx.rank_table()
    want_t, want_c = O.rank_table(U, P, O.stratified_sample(P, S), O.sketch_positions(S, rkr.TABLE_COLS))
    yield U, P, Qv, idx, (t.cpu().numpy(), c.cpu().numpy().astype(np.int64)), (want_t, want_c)
    idx.close()


def test_table_is_exact_on_integer_data(case):
    _, _, _, _, (t, c), (want_t, want_c) = case
    assert np.array_equal(t, want_t)
    assert np.array_equal(c, want_c)


def test_table_query_matches_oracle(case):
    U, P, Qv, idx, _, (want_t, want_c) = case
    m = P.shape[0]
    n, tau = want_t.shape
    seen = [0, 0]   # step 2: first case (c R_lo_k >= R_hi_k), second case
    for qi in range(Qv.shape[0]):
        tq = O.dots(U, Qv[qi:qi + 1])[:, 0]
        L = np.sum(want_t >= tq[:, None], axis=1)
        r_lo = np.where(L > 0, 1 + want_c[np.arange(n), np.maximum(L - 1, 0)], 1)
        r_hi = np.where(L < tau, 1 + want_c[np.arange(n), np.minimum(L, tau - 1)], 1 + m)
        for k in (1, 10, 100, 700):
            for c in (1.0, 1.5, 4.0, 1e6):
                ids, est = idx.query_table(_dev(Qv[qi]), k, c)
                wi, we = O.table_query(want_t, want_c, tq, m, k, c)
                assert np.array_equal(ids.cpu().numpy(), wi), (qi, k, c)
                assert np.array_equal(est.cpu().numpy(), we), (qi, k, c)
                seen[0 if c * np.sort(r_lo)[k - 1] >= np.sort(r_hi)[k - 1] else 1] += 1
    assert seen[0] > 0 and seen[1] > 0, seen


def test_table_query_errors(case):
    U, P, Qv, idx, _, _ = case
    q = _dev(Qv[0])
    for k, c in ((0, 1.0), (U.shape[0] + 1, 1.0), (5, 0.5), (5, float("inf")), (5, float("nan"))):
        with pytest.raises(rkr.RkrError) as e:
            idx.query_table(q, k, c)
        assert e.value.status == rkr.RKR_E_INVALID, (k, c)
    plain = rkr.Index(_dev(U[:100]), _dev(P[:200]), score="f32")
    with pytest.raises(rkr.RkrError) as e:
        plain.query_table(q, 5, 1.5)
    assert e.value.status == rkr.RKR_E_STATE
    plain.close()
    bad = _dev(np.full(U.shape[1], np.nan, np.float32))
    with pytest.raises(rkr.RkrError) as e:
        idx.query_table(bad, 5, 1.5)
    assert e.value.status == rkr.RKR_E_INVALID


def test_table_query_batch_matches_oracle(case):
    """All queries in one call, each with its own k and c: every query's
    answer equals the oracle's table query."""
    U, P, Qv, idx, _, (want_t, want_c) = case
    m = P.shape[0]
    rng = np.random.default_rng(72)
    Qb = np.vstack([Qv, P[rng.choice(P.shape[0], 40, replace=False)],
                    rng.integers(-3, 4, size=(25, U.shape[1])).astype(np.float32)])
    ks = rng.integers(1, 300, size=Qb.shape[0]).astype(np.int32)
    cs = rng.choice([1.0, 1.2, 2.0, 1e6], size=Qb.shape[0])
    ids, est, off = idx.query_table_batch(_dev(Qb), ks, cs)
    ids = ids.cpu().numpy()
    est = est.cpu().numpy()
    T = O.dots(U, Qb)
    for i in range(Qb.shape[0]):
        wi, we = O.table_query(want_t, want_c, T[:, i], m, int(ks[i]), float(cs[i]))
        assert np.array_equal(ids[off[i]:off[i + 1]], wi), i
        assert np.array_equal(est[off[i]:off[i + 1]], we), i
    with pytest.raises(rkr.RkrError) as e:
        idx.query_table_batch(_dev(Qb[:3]), [5, 0, 5], [1.5, 1.5, 1.5])
    assert e.value.status == rkr.RKR_E_INVALID


def test_table_query_batch_many_query_tiles():
    """Enough users that a workgroup of the bracket kernel runs several
    32-query tiles on the table rows it holds (12,000 users, 200 queries:
    runs of two tiles and a ragged last one): every answer equals the
    oracle's table query on the oracle's own table."""
    rng = np.random.default_rng(74)
    n, m, d, S = 12000, 3100, 6, 256
    U = rng.integers(-3, 4, size=(n, d)).astype(np.float32)
    P = rng.integers(-3, 4, size=(m, d)).astype(np.float32)
    want_t, want_c = O.rank_table(U, P, O.stratified_sample(P, S), O.sketch_positions(S, rkr.TABLE_COLS))
    Qb = np.vstack([P[rng.choice(m, 150, replace=False)], rng.integers(-3, 4, size=(50, d)).astype(np.float32)])
    ks = rng.integers(1, 400, size=Qb.shape[0]).astype(np.int32)
    cs = rng.choice([1.0, 1.5, 3.0], size=Qb.shape[0])
    idx = rkr.Index(_dev(U), _dev(P), score="f32", rank_table=S)
    try:
        t, c = idx.rank_table()
        assert np.array_equal(t.cpu().numpy(), want_t)
        assert np.array_equal(c.cpu().numpy().astype(np.int64), want_c)
        ids, est, off = idx.query_table_batch(_dev(Qb), ks, cs)
        ids = ids.cpu().numpy()
        est = est.cpu().numpy()
    finally:
        idx.close()
    T = O.dots(U, Qb)
    for i in range(Qb.shape[0]):
        wi, we = O.table_query(want_t, want_c, T[:, i], m, int(ks[i]), float(cs[i]))
        assert np.array_equal(ids[off[i]:off[i + 1]], wi), i
        assert np.array_equal(est[off[i]:off[i + 1]], we), i


def test_table_query_edges():
    """Fewer users than a tile, more samples than items (every item is a
    sample), k = n, and a query above every threshold of some users."""
    rng = np.random.default_rng(73)
    n, m, d, S = 37, 50, 3, 64
    U = rng.integers(-2, 3, size=(n, d)).astype(np.float32)
    P = rng.integers(-2, 3, size=(m, d)).astype(np.float32)
    Qv = np.vstack([P[0], np.full(d, 3.0, np.float32), np.zeros(d, np.float32)])
    idx = rkr.Index(_dev(U), _dev(P), score="f32", rank_table=S)
    want_t, want_c = O.rank_table(U, P, O.stratified_sample(P, min(S, m)), O.sketch_positions(min(S, m), rkr.TABLE_COLS))
    t, c = idx.rank_table()
    assert np.array_equal(t.cpu().numpy(), want_t) and np.array_equal(c.cpu().numpy(), want_c)
    T = O.dots(U, Qv)
    ks = np.array([n, 1, 7], np.int32)
    cs = np.array([1.0, 3.0, 1.1])
    ids, est, off = idx.query_table_batch(_dev(Qv), ks, cs)
    for i in range(3):
        wi, we = O.table_query(want_t, want_c, T[:, i], m, int(ks[i]), float(cs[i]))
        assert np.array_equal(ids.cpu().numpy()[off[i]:off[i + 1]], wi), i
        assert np.array_equal(est.cpu().numpy()[off[i]:off[i + 1]], we), i
    idx.close()
