"""Pins of the oracle's early-abandon exact top-k (topk_exact) for large shapes.

topk_exact must give exactly the Def. 2 answer that the plain definition
gives: Def. 1 ranks of every user (O.ranks, itself pinned in
test_oracle_pins.py by hand enumeration, closed forms and library routines),
then the k users of smallest (rank, id).  The cases put ties at the k-th rank
(integer tie storms), use low-rank data whose scores crowd together, zero
vectors, candidate domains and every item order.  Two planted mistakes, made
in a patched copy of the oracle source compiled on the CPU, must be caught by
the same comparisons: a ">=" in the abandoning count and an abandon rule that
ignores the id tie-break.
"""
import ctypes
import os
import subprocess

import numpy as np
import pytest

from oracle import oracle as O
from paper_2504_13446_amd import workloads as W


def _reference(U, P, q, k, uids=None):
    r = O.ranks(U, P, q, uids=uids)[0]
    return O.topk(r, k, uids=uids)


def _same(U, P, q, k, uids=None, order=None, topk=None):
    topk = topk or O.topk_exact
    want_ids, want_rk = _reference(U, P, q, k, uids)
    got_ids, got_rk = topk(U, P, q, k, uids=uids, order=order)
    return np.array_equal(got_ids, want_ids) and np.array_equal(got_rk, want_rk)


def _tie_storm(seed, n=240, m=300, d=3):
    rng = np.random.default_rng(seed)
    U = rng.integers(-2, 3, size=(n, d)).astype(np.float32)
    P = rng.integers(-2, 3, size=(m, d)).astype(np.float32)
    return U, P


def test_random_float_every_k():
    rng = np.random.default_rng(21)
    n, m, d = 300, 500, 12
    U = rng.standard_normal((n, d)).astype(np.float32)
    P = (rng.standard_normal((m, d)) * rng.lognormal(0, 0.5, size=(m, 1))).astype(np.float32)
    for qi in (0, 17, 499):
        for k in (1, 7, 50, n):
            assert _same(U, P, P[qi], k), (qi, k)


def test_integer_tie_storm_ties_at_the_kth_rank():
    """Entries in {-2..2}, d = 3: only a few distinct ranks, so many users tie
    at the k-th rank and only the id tie-break decides the answer."""
    hit_tie = False
    for seed in range(6):
        U, P = _tie_storm(seed)
        for qi in (0, 5, 77):
            q = P[qi]
            r = O.ranks(U, P, q)[0]
            for k in (3, 20, 64):
                kth = np.sort(r)[k - 1]
                hit_tie |= np.sum(r == kth) > 1 and np.sum(r <= kth) > k
                assert _same(U, P, q, k), (seed, qi, k)
    assert hit_tie


def test_lowrank_workload_scaled():
    w = W.make("single", n=1500, m=2000)
    for k in (10, 50):
        assert _same(w.U, w.P, w.Qv[0], k)


def test_bf16_masters_and_query_not_in_p():
    w = W.make("batch", n=900, m=1100, d=24, nq=3)
    for i in range(3):
        assert _same(w.U, w.P, w.Qv[i], 100)
    q = np.full(24, W.f32_to_bf16_bits(np.float32(0.25)), np.uint16)   # not an item of P
    assert _same(w.U, w.P, q, 40)


def test_candidate_domains():
    rng = np.random.default_rng(3)
    U, P = _tie_storm(11, n=400, m=250, d=4)
    for size, k in ((1, 1), (9, 9), (120, 10), (400, 33)):
        uids = np.sort(rng.choice(U.shape[0], size=size, replace=False))
        assert _same(U, P, P[4], k, uids=uids), (size, k)


def test_zero_vectors():
    """A zero user has rank 1 (every score is 0, nothing is strictly above);
    a zero query counts the items with a positive score."""
    rng = np.random.default_rng(8)
    U = rng.integers(-2, 3, size=(60, 5)).astype(np.float32)
    U[[3, 40]] = 0.0
    P = rng.integers(-2, 3, size=(90, 5)).astype(np.float32)
    ids, rk = O.topk_exact(U, P, P[2], 2)
    assert ids.tolist() == [3, 40] and rk.tolist() == [1, 1]
    assert _same(U, P, np.zeros(5, np.float32), 12)


def test_item_order_does_not_change_the_answer():
    U, P = _tie_storm(19)
    rng = np.random.default_rng(2)
    for order in (None, np.arange(P.shape[0]), rng.permutation(P.shape[0]),
                  np.arange(P.shape[0])[::-1].copy()):
        assert _same(U, P, P[9], 25, order=order)


def test_abandoning_skips_work():
    """On norm-sorted items most users stop long before the end."""
    w = W.make("small", n=2000, m=5000)
    st = {}
    ids, rk = O.topk_exact(w.U, w.P, w.Qv[0], 10, stats=st)
    want_ids, want_rk = _reference(w.U, w.P, w.Qv[0], 10)
    assert np.array_equal(ids, want_ids) and np.array_equal(rk, want_rk)
    assert st["items_visited"] < 0.2 * w.n * w.m
    assert 10 <= st["users_fully_counted"] < w.n


def test_certify_in_norm_order():
    U, P = _tie_storm(4, n=200, m=260, d=3)
    q = P[10]
    ids, rk = _reference(U, P, q, 15)
    order = O.norm_order(P)
    assert O.certify(U, P, q, 15, ids, rk, order=order) == (0, 0, 200)
    bad = ids.copy()
    bad[-1] = [u for u in range(200) if u not in set(ids.tolist())][-1]
    assert O.certify(U, P, q, 15, bad, rk, order=order)[:2] != (0, 0)


# ---------------------------------------------------------------------------
# planted mistakes: a patched copy of the oracle must fail the comparisons
# ---------------------------------------------------------------------------
_SRC = os.path.join(os.path.dirname(O.__file__), "rkr_oracle.c")

_MUTANTS = {
    # count scores equal to the threshold (Def. 1 says strictly above)
    "ge": ("c += (s[0] > t) + (s[1] > t) + (s[2] > t) + (s[3] > t);",
           "c += (s[0] >= t) + (s[1] >= t) + (s[2] >= t) + (s[3] >= t);"),
    # a user is abandoned once its count reaches the worst rank, whatever its
    # id: users tied at the k-th rank are then kept in visit order, not by id
    "tiebreak": ("if (stop && key > __atomic_load_n(stop, __ATOMIC_RELAXED))",
                 "if (stop && (key >> 32) >= (__atomic_load_n(stop, __ATOMIC_RELAXED) >> 32))"),
}


def _mutant_topk(tmp_path, name):
    src = open(_SRC).read()
    old, new = _MUTANTS[name]
    assert src.count(old) == 1, name
    path = tmp_path / ("mut_%s.c" % name)
    path.write_text(src.replace(old, new))
    so = tmp_path / ("mut_%s.so" % name)
    subprocess.check_call(["gcc", "-O2", "-mfma", "-ffp-contract=off", "-fopenmp", "-shared",
                           "-fPIC", "-std=c11", "-o", str(so), str(path), "-lm"])
    L = ctypes.CDLL(str(so))
    vp, i64 = ctypes.c_void_p, ctypes.c_int64
    L.orc_topk_abandon.argtypes = [vp, i64, vp, i64, vp, vp, ctypes.c_int, ctypes.c_int, vp, i64,
                                   vp, vp, vp, ctypes.c_int]
    L.orc_topk_abandon.restype = None

    def topk(U, P, q, k, uids=None, order=None):
        U = O.widen(U); P = O.widen(P); q = O.widen(np.asarray(q).reshape(1, -1))
        order = O.norm_order(P) if order is None else np.ascontiguousarray(order, np.int64)
        ids = np.empty(k, np.int64)
        rk = np.empty(k, np.int32)
        p = lambda a: a.ctypes.data_as(vp)
        L.orc_topk_abandon(p(U), U.shape[0], p(P), P.shape[0], p(order), p(q), U.shape[1], k,
                           None, U.shape[0], p(ids), p(rk), None, 1)
        return ids, rk
    return topk


@pytest.mark.parametrize("name", sorted(_MUTANTS))
def test_planted_mistakes_are_caught(tmp_path, name):
    topk = _mutant_topk(tmp_path, name)
    caught = False
    for seed in range(4):
        U, P = _tie_storm(seed)
        for qi in (0, 5, 77):
            for k in (3, 20, 64):
                caught |= not _same(U, P, P[qi], k, topk=topk)
    assert caught, name
