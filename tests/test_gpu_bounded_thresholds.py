"""GPU: the bounded FP32 thresholds of dense batches with the rank table.

Such a batch computes, for every (user, query) pair, t^ = u^.q^ on the matrix
cores and an upper bound t_up >= s64(u, q) from the same error terms as the
scores; the rank-table filter (Lemma 1 (2)) reads t_up, and FP64 thresholds
are computed only for the pairs that are counted (seeds and the pairs the
filter keeps).  A higher threshold can only lower the table's rank bound, so
the filter keeps every pair the FP64 threshold would keep: the answers must
equal the oracle's (Def. 2) and the answers with FP64 thresholds for every
pair, and the number of pairs the table rules out can only drop.
"""
import os

import numpy as np
import pytest

from oracle import oracle as O
from paper_2504_13446_amd import rkr, workloads as W

pytestmark = pytest.mark.gpu


def _answers(ids, rk, off):
    ids = ids.cpu().numpy()
    rk = rk.cpu().numpy()
    return [(ids[off[i]:off[i + 1]], rk[off[i]:off[i + 1]]) for i in range(len(off) - 1)]


def _case(name):
    rng = np.random.default_rng(77)
    if name == "iid_bf16":
        w = W.make("small", n=4000, m=5000, nq=20)
        return W.f32_to_bf16_bits(w.U), W.f32_to_bf16_bits(w.P), W.f32_to_bf16_bits(w.Qv), "bf16"
    if name == "iid_f32":
        w = W.make("small", n=4000, m=5000, nq=20)
        return w.U, w.P, w.Qv, "f32"
    if name == "iid_odd_users":
        # an odd number of users above one selection workgroup's LDS (4,096
        # keys): the 32-bit seed keys go through the select's radix passes
        w = W.make("small", n=9001, m=3000, nq=20)
        return W.f32_to_bf16_bits(w.U), W.f32_to_bf16_bits(w.P), W.f32_to_bf16_bits(w.Qv), "bf16"
    if name == "integer_ties":
        # every score an integer: thresholds tie exactly with table columns
        U = rng.integers(-3, 4, size=(3000, 8)).astype(np.float32)
        P = rng.integers(-3, 4, size=(4000, 8)).astype(np.float32)
        return U, P, P[rng.choice(4000, 20, replace=False)], "f32"
    # norms spread over many binades, and a few zero users
    U = rng.standard_normal((3000, 40)) * np.exp2(rng.integers(-30, 31, size=(3000, 1)))
    U[:7] = 0.0
    P = rng.standard_normal((4000, 40)) * np.exp2(rng.integers(-20, 21, size=(4000, 1)))
    return U.astype(np.float32), P.astype(np.float32), P[rng.choice(4000, 20, replace=False)].astype(np.float32), "f32"


@pytest.mark.parametrize("case", ["iid_bf16", "iid_f32", "iid_odd_users", "integer_ties", "spread_norms"])
def test_bounded_thresholds_keep_answers_exact(case):
    U, P, Qv, mk = _case(case)
    ks = np.array([1, 3, 5, 10, 20, 40, 7, 2, 64, 10, 10, 15, 33, 4, 8, 1, 50, 6, 12, 9], np.int32)
    R = O.ranks(O.widen(U), O.widen(P), O.widen(Qv))
    idx = rkr.Index(rkr.to_device(U, mk), rkr.to_device(P, mk), score="bf16", rank_table=512)
    Q = rkr.to_device(Qv, mk)
    got = _answers(*idx.query_batch(Q, ks))
    st = idx.stats()
    os.environ["RKR_FP64_THRESHOLDS"] = "1"
    try:
        ref = _answers(*idx.query_batch(Q, ks))
        st64 = idx.stats()
    finally:
        del os.environ["RKR_FP64_THRESHOLDS"]
    idx.close()
    for i, ((gi, gr), (fi, fr)) in enumerate(zip(got, ref)):
        wi, wr = O.topk(R[i], int(ks[i]))
        assert np.array_equal(gi, wi) and np.array_equal(gr, wr), (case, i)
        assert np.array_equal(fi, wi) and np.array_equal(fr, wr), (case, i)
    # the bounded thresholds rule out no pair the FP64 ones keep, and nearly
    # as many as they do (iid data: the bound is about 2^-13 of |u||q|)
    assert st["table_pruned"] <= st64["table_pruned"]
    if case.startswith("iid"):
        assert st["table_pruned"] >= 0.99 * st64["table_pruned"], (st["table_pruned"], st64["table_pruned"])
