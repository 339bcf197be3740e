"""GPU parity at full size, against the oracle, with no sampling.

* The single-query workload (100,000 users x 100,000 items x d = 100, low-rank
  data, FP32 masters): every one of the 100,000 Def. 1 ranks of its query, for
  BF16, FP32 and split BF16 scores + FP64 recheck, eagerly and as a graph
  replay, equals the oracle's bit for bit (about 1e12 FP64 fma in the
  oracle: a minute or two on the host's cores).
* The batch workload (1M users x 1M items x d = 200, 256 queries, k = 100,
  with the rank table): the answer of the query with the smallest k-th rank
  equals the oracle's early-abandon exact top-k (Def. 2) element by element.
  The sampled checks of other queries are in test_gpu_full_and_errors.py.
"""
import time

import numpy as np
import pytest
import torch

from oracle import oracle as O
from paper_2504_13446_amd import rkr, workloads as W

pytestmark = pytest.mark.gpu


def _dev(x, dtype):
    return rkr.to_device(x, dtype)


def _log(msg):
    print("[fullsize %.0fs] %s" % (time.time() - _T0, msg), flush=True)


_T0 = time.time()


@pytest.mark.timeout(900)
def test_single_query_all_ranks_full_size():
    w = W.make("single")
    q = _dev(w.Qv[0], "f32")
    U, P = _dev(w.U, "f32"), _dev(w.P, "f32")
    got = {}
    for score in ("bf16", "f32", "bf16x3"):
        idx = rkr.Index(U, P, score=score)
        got[score] = idx.ranks(q).cpu().numpy()
        st = idx.stats()
        idx.configure(graph=True)
        idx.ranks(q)                                   # eager run, then capture
        got[score + "_graph"] = idx.ranks(q).cpu().numpy()
        assert idx.stats()["graph_replays"] == 1
        ids, rk = idx.query_exact(q, 50)
        got[score + "_top"] = (ids.cpu().numpy(), rk.cpu().numpy())
        idx.close()
        _log("%s: all ranks on the GPU, %d near ties rechecked" % (score, st["uncertain"]))
    t = time.time()
    R = O.ranks(w.U, w.P, w.Qv)[0]
    _log("oracle: 100,000 ranks in %.1f s on %d threads" % (time.time() - t, O.num_threads()))
    wi, wr = O.topk(R, 50)
    for score in ("bf16", "f32", "bf16x3"):
        for key in (score, score + "_graph"):
            bad = np.flatnonzero(got[key] != R)
            assert bad.size == 0, (key, bad[:10], got[key][bad[:10]], R[bad[:10]])
        ids, rk = got[score + "_top"]
        assert np.array_equal(ids, wi) and np.array_equal(rk, wr), score


@pytest.mark.timeout(900)
def test_batch_full_size_exact_and_approx():
    """The six queries of smallest k-th rank (the oracle's early abandon is
    cheapest there): the exact answers equal the oracle's element by element;
    the c = 1.5 answers have zero Def. 3 violations against the oracle's ranks
    of the returned users and of U_rr, and report exact ranks."""
    w = W.make("batch")
    idx = rkr.Index(_dev(w.U, "bf16"), _dev(w.P, "bf16"), score="bf16", rank_table=4096)
    Q = _dev(w.Qv, "bf16")
    ids, rk, off = idx.query_batch(Q, w.k)
    ida, rka, offa = idx.query_batch(Q, w.k, c=np.full(w.nq, 1.5))
    idx.close()
    ids = ids.cpu().numpy(); rk = rk.cpu().numpy()
    ida = ida.cpu().numpy(); rka = rka.cpu().numpy()
    kth = np.array([rk[off[i + 1] - 1] for i in range(w.nq)])
    Uw, Pw = O.widen(w.U), O.widen(w.P)
    order = O.norm_order(Pw)
    for i in np.argsort(kth, kind="stable")[:6]:
        i = int(i)
        st = {}
        t = time.time()
        wi, wr = O.topk_exact(Uw, Pw, O.widen(w.Qv[i]), int(w.k[i]), order=order, stats=st)
        _log("query %d (k-th rank %d): oracle top-k in %.1f s on %d threads, %.3g of the pairs visited" % (
            i, kth[i], time.time() - t, O.num_threads(), st["items_visited"] / (w.n * w.m)))
        assert np.array_equal(ids[off[i]:off[i + 1]], wi), i
        assert np.array_equal(rk[off[i]:off[i + 1]], wr), i
        gi, gr = ida[offa[i]:offa[i + 1]], rka[offa[i]:offa[i + 1]]
        assert len(set(gi.tolist())) == gi.size == int(w.k[i])
        true = O.ranks(Uw, Pw, O.widen(w.Qv[i]), uids=gi)[0]
        assert np.array_equal(gr, true), i                   # returned ranks are exact
        v, weak = O.def3_check(true, wr, 1.5)
        assert v == 0 and weak == 0, (i, v, weak)


def _def3_against_oracle(Uw, Pw, q, uids, k, got_ids, got_rk, c, order):
    """Oracle check of an approximate answer: the returned ranks are exact and
    Def. 3 holds against the oracle's exact answer over the domain."""
    wi, wr = O.topk_exact(Uw, Pw, q, k, uids=uids, order=order)
    true = O.ranks(Uw, Pw, q, uids=got_ids)[0]
    assert np.array_equal(got_rk, true)
    v, weak = O.def3_check(true, wr, c)
    assert v == 0 and weak == 0
    return wi, wr


@pytest.mark.timeout(900)
def test_uneven_full_shape_shortest_lists():
    """The uneven workload at its full shape (500,000 users x 1M items x d =
    300, FP32 masters, 1,024 candidate lists of 1k-200k users, k in {10, 50,
    100}), BF16 scores with the rank table: the whole batch, exact and c =
    1.5; the 8 queries with the shortest lists are checked against the oracle
    (exact answers element by element over their lists; returned ranks exact
    and Def. 3 with oracle ranks for the approximate answers)."""
    w = W.make("uneven")
    sizes = np.diff(w.cand_off)
    short = np.argsort(sizes, kind="stable")[:8]
    U, P, Q = _dev(w.U, "f32"), _dev(w.P, "f32"), _dev(w.Qv, "f32")
    cids = torch.from_numpy(w.cand_ids).cuda()
    idx = rkr.Index(U, P, score="bf16", rank_table=4096)
    ids, rk, off = idx.query_batch(Q, w.k, cand_off=w.cand_off, cand_ids=cids)
    ida, rka, offa = idx.query_batch(Q, w.k, c=np.full(w.nq, 1.5), cand_off=w.cand_off, cand_ids=cids)
    idx.close()
    _log("uneven batch answered, exact and c = 1.5")
    ids, rk, ida, rka = (x.cpu().numpy() for x in (ids, rk, ida, rka))
    Uw, Pw = O.widen(w.U), O.widen(w.P)
    order = O.norm_order(Pw)
    for i in short:
        i = int(i)
        lst = w.cand_ids[w.cand_off[i]:w.cand_off[i + 1]]
        k = int(w.k[i])
        t = time.time()
        wi, wr = _def3_against_oracle(Uw, Pw, O.widen(w.Qv[i]), lst, k, ida[offa[i]:offa[i + 1]],
                                      rka[offa[i]:offa[i + 1]], 1.5, order)
        _log("query %d (list of %d, k = %d): oracle in %.1f s" % (i, lst.size, k, time.time() - t))
        assert np.array_equal(ids[off[i]:off[i + 1]], wi) and np.array_equal(rk[off[i]:off[i + 1]], wr), i


@pytest.mark.timeout(900)
def test_learned_full_shape():
    """The learned workload at full shape (1M x 1M x 200, 1,024 test queries,
    k = 100): the estimator is trained on the index with the library's own
    kernels (exact ranks of 256 training queries disjoint from the test ones,
    about a million triples here; the benchmark trains on 10M), then orders
    the seeds.  For the 8 test queries of smallest k-th rank: the exact answers
    equal the oracle's, and the c = 1.5 answers have zero Def. 3 violations."""
    w = W.make("learned")
    idx = rkr.Index(_dev(w.U, "bf16"), _dev(w.P, "bf16"), score="bf16", rank_table=4096, sketch_samples=4096)
    idx.train(_dev(W.extra_queries(w, 256), "bf16"), pairs_per_query=4096, epochs=4, batch=4096, lr=1e-3, seed=5)
    st = idx.stats()
    assert st["pairs"] >= 256 * 4000
    _log("estimator trained on %d triples, MSE(ln r) %.4f" % (st["pairs"], st["mlp_loss"]))
    idx.configure(use_estimator=True)
    Q = _dev(w.Qv, "bf16")
    ids, rk, off = idx.query_batch(Q, w.k)
    ida, rka, offa = idx.query_batch(Q, w.k, c=np.full(w.nq, 1.5))
    idx.close()
    ids, rk, ida, rka = (x.cpu().numpy() for x in (ids, rk, ida, rka))
    kth = np.array([rk[off[i + 1] - 1] for i in range(w.nq)])
    Uw, Pw = O.widen(w.U), O.widen(w.P)
    order = O.norm_order(Pw)
    for i in np.argsort(kth, kind="stable")[:8]:
        i = int(i)
        t = time.time()
        wi, wr = _def3_against_oracle(Uw, Pw, O.widen(w.Qv[i]), None, int(w.k[i]), ida[offa[i]:offa[i + 1]],
                                      rka[offa[i]:offa[i + 1]], 1.5, order)
        _log("query %d (k-th rank %d): oracle in %.1f s" % (i, kth[i], time.time() - t))
        assert np.array_equal(ids[off[i]:off[i + 1]], wi) and np.array_equal(rk[off[i]:off[i + 1]], wr), i
