"""Pins of the CPU oracle against facts fixed outside the oracle itself.

Each test targets a plausible mistake: a dropped or reversed comparison
(">" vs ">="), a transposed operand, a wrong summation order, a wrong
tie-break, an off-by-one in the rank.  None of them re-types the oracle's
formula; they use hand enumeration, closed forms, library routines on exact
integer data, an independent pure-Python evaluation, and invariants.
"""
import ctypes
import json
import os

import numpy as np
import pytest
from scipy.stats import rankdata

from oracle import oracle as O

GOLD = os.path.join(os.path.dirname(__file__), "golden", "f1_hand_enumeration.json")


@pytest.fixture(scope="module")
def f1():
    with open(GOLD) as f:
        return json.load(f)


def test_f1_hand_enumeration(f1):
    U = np.array(f1["U"], np.float64)
    P = np.array(f1["P"], np.float64)
    assert np.array_equal(O.dots(U, P), np.array(f1["score_rows_u_dot_p"], np.float64))
    for case in f1["cases"]:
        r = O.ranks(U, P, np.array(case["q"], np.float64))[0]
        assert r.tolist() == case["ranks"], case["note"]
        for k, ids in case["topk"].items():
            got, _ = O.topk(r, int(k))
            assert got.tolist() == ids


def test_f1_strict_inequality(f1):
    U = np.array(f1["U"], np.float64)
    P = np.array(f1["P"] + [f1["tie_item"]["p5"]], np.float64)
    s = O.dots(U, P)[:, 4]
    assert s.tolist() == f1["tie_item"]["scores"]
    r = O.ranks(U, P, np.array(f1["tie_item"]["q"], np.float64))[0]
    assert r.tolist() == f1["tie_item"]["ranks"]


def test_f1_def3_and_criteria(f1):
    g = f1["def3"]
    U = np.array(f1["U"], np.float64)
    P = np.array(f1["P"], np.float64)
    r = O.ranks(U, P, np.array(g["q"], np.float64))[0]
    _, rr = O.topk(r, g["k"])
    assert rr.tolist() == g["exact_ranks"]
    for a in g["answers"]:
        tr = r[np.array(a["ids"])]
        assert tr.tolist() == a["true_ranks"]
        v, w = O.def3_check(tr, rr, g["c"])
        assert (v, w) == (a["violations"], a["weak_violations"]), a["note"]
        assert O.accuracy(tr, rr, g["c"]) == pytest.approx(a["accuracy"])
        assert O.overall_ratio(tr, rr) == pytest.approx(a["overall_ratio"])
    # c = 1 reduces Def. 3 to Def. 2: only the exact rank multiset passes.
    assert O.def3_check(rr, rr, 1.0)[0] == 0
    assert O.def3_check(r[[0, 1]], rr, 1.0)[0] == 1


def test_d1_closed_form():
    """d = 1: for u > 0 the rank is 1 + #{p > q}; for u < 0, 1 + #{p < q}; u = 0 gives 1.

    float32 products are exact in double, so the spec scores keep the order
    of the real products; the closed form uses sort + bisection.
    """
    rng = np.random.default_rng(7)
    P = rng.standard_normal(400).astype(np.float32)
    P[::7] = P[3]                                   # duplicated items: ties
    U = np.concatenate([rng.standard_normal(30), [0.0]]).astype(np.float32)
    qs = np.concatenate([P[[3, 10, 50]], np.float32([0.0, 9.0, -9.0])])
    srt = np.sort(P.astype(np.float64))
    got = O.ranks(U[:, None], P[:, None], qs[:, None].astype(np.float32))
    for i, q in enumerate(qs.astype(np.float64)):
        above = P.size - np.searchsorted(srt, q, side="right")
        below = np.searchsorted(srt, q, side="left")
        want = np.where(U > 0, 1 + above, np.where(U < 0, 1 + below, 1))
        assert np.array_equal(got[i], want)


@pytest.mark.parametrize("d", [3, 8, 16])
def test_rankdata_on_integer_data(d):
    """Integer data: every order of summation is exact, so numpy's matmul gives
    the true scores and scipy's competition ranking ('min') of the negated
    scores is the rank of each item q = p_j (ties everywhere)."""
    rng = np.random.default_rng(100 + d)
    U = rng.integers(-2, 3, size=(25, d)).astype(np.float32)
    P = rng.integers(-2, 3, size=(60, d)).astype(np.float32)
    S = U.astype(np.float64) @ P.astype(np.float64).T
    got = O.ranks(U, P, P)                     # queries: every item of P
    for ui in range(U.shape[0]):
        want = rankdata(-S[ui], method="min").astype(np.int64)
        assert np.array_equal(got[:, ui], want)
    # q in P: rank never exceeds m
    assert got.max() <= P.shape[0] and got.min() >= 1


_libm = ctypes.CDLL("libm.so.6")
_libm.fma.restype = ctypes.c_double
_libm.fma.argtypes = [ctypes.c_double] * 3


def _py_spec_dot(x, y):
    acc = 0.0
    for a, b in zip(x.tolist(), y.tolist()):
        acc = _libm.fma(a, b, acc)
    return acc


def test_brute_force_python_fma():
    """An independent pure-Python evaluation of Def. 1 with libm fma."""
    rng = np.random.default_rng(11)
    n, m, d = 12, 40, 9
    U = (rng.standard_normal((n, d)) * np.exp(rng.uniform(-8, 8, (n, d)))).astype(np.float32)
    P = (rng.standard_normal((m, d)) * np.exp(rng.uniform(-8, 8, (m, d)))).astype(np.float32)
    P[5] = P[6]
    Qv = P[[5, 20, 33]]
    got = O.ranks(U, P, Qv)
    for qi in range(Qv.shape[0]):
        for ui in range(n):
            t = _py_spec_dot(U[ui].astype(np.float64), Qv[qi].astype(np.float64))
            c = sum(1 for p in range(m)
                    if _py_spec_dot(U[ui].astype(np.float64), P[p].astype(np.float64)) > t)
            assert got[qi, ui] == 1 + c


def test_spec_dot_order_is_sequential_fma():
    """x = (-fl(a*a), a), y = (1, a) with a = 1 + 2^-30: the sequential fma
    chain keeps the rounding error of a*a (2^-60), while a plain product sum
    and the reversed chain both return 0.  The oracle must give the chain."""
    a = 1.0 + 2.0 ** -30
    x = np.array([-(a * a), a], np.float64)
    y = np.array([1.0, a], np.float64)
    want = _py_spec_dot(x, y)
    assert want == 2.0 ** -60
    assert O.dots(x[None], y[None])[0, 0] == want
    assert float(x[0] * y[0] + x[1] * y[1]) == 0.0
    assert _py_spec_dot(x[::-1], y[::-1]) == 0.0


def test_invariants_random():
    rng = np.random.default_rng(3)
    n, m, d = 40, 300, 12
    U = rng.standard_normal((n, d)).astype(np.float32)
    P = rng.standard_normal((m, d)).astype(np.float32)
    qi = np.array([0, 17, 123, 299])
    Qv = P[qi]
    r = O.ranks(U, P, Qv)
    assert r.min() >= 1 and r.max() <= m            # q in P => r <= m
    # q not in P: r <= m + 1, attained for a q every item beats
    far = -50.0 * U[0:1].astype(np.float32)
    rfar = O.ranks(U[0:1], P, far)
    assert rfar[0, 0] == m + 1
    # power-of-two scaling of U, or of P together with q, is exact in the spec dot
    assert np.array_equal(O.ranks(U * np.float32(2.0 ** 9), P, Qv), r)
    assert np.array_equal(O.ranks(U, P * np.float32(2.0 ** -7), Qv * np.float32(2.0 ** -7)), r)
    # permuting P leaves ranks unchanged; permuting U permutes them
    perm = rng.permutation(m)
    assert np.array_equal(O.ranks(U, P[perm], Qv), r)
    up = rng.permutation(n)
    assert np.array_equal(O.ranks(U[up], P, Qv), r[:, up])
    # user subset selection matches the full computation
    sub = np.array([5, 0, 39, 5])
    assert np.array_equal(O.ranks(U, P, Qv, uids=sub), r[:, sub])
    # monotone in the threshold: larger u.q never gives a worse rank
    T = O.dots(U, Qv)
    for ui in range(n):
        o = np.argsort(-T[ui], kind="stable")
        assert np.all(np.diff(r[o, ui]) >= 0)


def test_topk_tie_break_and_order():
    r = np.array([5, 2, 2, 9, 1, 2])
    ids, rk = O.topk(r, 4)
    assert ids.tolist() == [4, 1, 2, 5] and rk.tolist() == [1, 2, 2, 2]
    ids, rk = O.topk(r, 3, uids=np.array([50, 40, 30, 20, 10, 0]))
    assert ids.tolist() == [10, 0, 30]          # rank 1: uid 10; rank 2: uids 0 < 30 < 40


def test_certify_accepts_truth_and_rejects_planted_mistakes():
    rng = np.random.default_rng(5)
    n, m, d, k = 300, 400, 10, 12
    U = rng.standard_normal((n, d)).astype(np.float32)
    P = rng.standard_normal((m, d)).astype(np.float32)
    q = P[77]
    r = O.ranks(U, P, q)[0]
    ids, rk = O.topk(r, k)
    assert O.certify(U, P, q, k, ids, rk) == (0, 0, n)
    # planted: drop the best user, add the (k+1)-th with its true rank
    nxt, nrk = O.topk(r, k + 1)
    bad_ids = np.concatenate([ids[1:], nxt[k:]])
    bad_rk = np.concatenate([rk[1:], nrk[k:]])
    o = np.lexsort((bad_ids, bad_rk))
    assert O.certify(U, P, q, k, bad_ids[o], bad_rk[o])[1] >= 1
    # planted: wrong rank value
    rk2 = rk.copy(); rk2[3] += 1
    assert O.certify(U, P, q, k, ids, rk2)[0] == 1
    # tie-break: among users tied at the boundary rank, the smaller id must be kept
    R = rk[-1]
    tied = np.flatnonzero(r == R)
    if tied.size >= 2 and np.sum(r < R) + 1 <= k:
        pass  # the canonical answer already keeps the smallest ids
    # sampled certification examines only the listed users
    sample = rng.choice(n, 50, replace=False)
    assert O.certify(U, P, q, k, ids, rk, check=sample)[2] == 50


def test_certify_tie_break_violation():
    # Three users with the same rank; k = 2 must keep the two smallest ids.
    U = np.array([[1.0, 0.0], [1.0, 0.0], [1.0, 0.0], [-1.0, 0.0]], np.float32)
    P = np.array([[2.0, 0.0], [1.0, 0.0], [0.0, 1.0]], np.float32)
    q = P[1]
    r = O.ranks(U, P, q)[0]
    assert r.tolist() == [2, 2, 2, 2]
    assert O.certify(U, P, q, 2, [0, 1], [2, 2])[:2] == (0, 0)
    assert O.certify(U, P, q, 2, [0, 2], [2, 2])[1] == 1


def test_norm_order_integer_norms():
    """Integer rows with exact squared norms; descending order, ties by id."""
    P = np.array([[3, 4], [0, 1], [5, 0], [1, 0], [0, 0], [4, 3], [2, 2]], np.float32)
    assert O.norm_order(P).tolist() == [0, 2, 5, 6, 1, 3, 4]
    assert O.norms(P).tolist() == [5.0, 1.0, 5.0, 1.0, 0.0, 5.0, np.sqrt(8.0)]


def test_stratified_sample_positions():
    P = np.arange(10, dtype=np.float32)[::-1, None] + 1.0   # norms 10..1, already descending
    assert O.stratified_sample(P, 4).tolist() == [1, 3, 6, 8]
    assert O.stratified_sample(P, 50).tolist() == list(range(10))


def test_sketch_positions():
    pos = O.sketch_positions(4096)
    assert pos[0] == 1 and pos[-1] == 4096 and pos[5] == 16 and pos[10] == 256
    assert np.all(np.diff(pos) > 0)


def test_sketch_closed_form():
    """u = e_1 scores every item by its first coordinate exactly."""
    rng = np.random.default_rng(9)
    P = rng.standard_normal((500, 6)).astype(np.float32)
    U = np.zeros((2, 6), np.float32); U[0, 0] = 1.0; U[1, 0] = 4.0
    sample = np.arange(0, 500, 3)
    pos = np.array([1, 2, 10, 50, 167], np.int32)
    got = O.sketch(U, P, sample, pos)
    col = np.sort(P[sample, 0].astype(np.float64))[::-1]
    assert np.array_equal(got[0], col[pos - 1])
    assert np.array_equal(got[1], col[pos - 1])              # divided by the norm 4
    assert np.array_equal(O.sketch(np.zeros((1, 6), np.float32), P, sample, pos)[0], np.zeros(5))


def test_widen_bf16():
    bits = np.array([0x3F80, 0xC000, 0x0000, 0x3E20], np.uint16)   # 1, -2, 0, 0.15625
    assert O.widen(bits, "bf16").tolist() == [1.0, -2.0, 0.0, 0.15625]


def test_rank_table_integer_fixture():
    """Rank table with exact cells (Sec. 4.2): on small integers every dot is
    exact in int64, so thresholds and cells are checked against integer
    arithmetic; the data holds many ties, so '>' versus '>=' and an
    off-by-one position would both show."""
    rng = np.random.default_rng(31)
    n, m, d = 40, 300, 5
    U = rng.integers(-3, 4, size=(n, d)).astype(np.float32)
    P = rng.integers(-3, 4, size=(m, d)).astype(np.float32)
    sample = np.array(sorted(rng.choice(m, 37, replace=False)), np.int64)
    pos = np.array([1, 2, 5, 9, 20, 37], np.int32)
    t, cnt = O.rank_table(U, P, sample, pos)
    S = U.astype(np.int64) @ P.astype(np.int64).T                 # exact scores
    srt = -np.sort(-S[:, sample], axis=1)                          # descending
    want_t = srt[:, pos - 1]
    want_c = (S[:, :, None] > want_t[:, None, :]).sum(axis=1)
    assert np.array_equal(t, want_t.astype(np.float64))
    assert np.array_equal(cnt, want_c)
    assert np.all(np.diff(cnt, axis=1) >= 0)                       # lower thresholds, more above
    # the top threshold from a sample holding the best item counts nothing above it
    best = np.argmax(S, axis=1)
    for u in range(n):
        if best[u] in sample:
            assert cnt[u, 0] == np.sum(S[u] > S[u, best[u]])


def test_rank_table_brackets_ranks():
    """The bracket the table gives (Sec. 4.2): a threshold at or above u.q
    bounds the rank from below by 1 + its cell, one at or below u.q bounds it
    from above."""
    rng = np.random.default_rng(32)
    U = rng.standard_normal((60, 8)).astype(np.float32)
    P = rng.standard_normal((700, 8)).astype(np.float32)
    sample = O.stratified_sample(P, 64)
    pos = O.sketch_positions(64)
    t, cnt = O.rank_table(U, P, sample, pos)
    Qv = P[[3, 50, 400]]
    R = O.ranks(U, P, Qv)
    T = O.dots(U, Qv)
    for qi in range(3):
        for u in range(U.shape[0]):
            above = t[u] >= T[u, qi]
            below = t[u] <= T[u, qi]
            if above.any():
                assert R[qi, u] >= 1 + cnt[u][above].max()
            if below.any():
                assert R[qi, u] <= 1 + cnt[u][below].min()


def _table_case(seed, integer):
    rng = np.random.default_rng(seed)
    if integer:
        U = rng.integers(-3, 4, size=(250, 6)).astype(np.float32)
        P = rng.integers(-3, 4, size=(900, 6)).astype(np.float32)
    else:
        U = rng.standard_normal((250, 9)).astype(np.float32)
        P = rng.standard_normal((900, 9)).astype(np.float32)
    sample = O.stratified_sample(P, 128)
    t, cnt = O.rank_table(U, P, sample, O.sketch_positions(128, 32))
    Qv = P[[7, 300, 811]]
    return U, P, t, cnt, Qv, O.ranks(U, P, Qv), O.dots(U, Qv)


@pytest.mark.parametrize("integer", [False, True])
def test_table_query_first_case_meets_the_c_bound(integer):
    """Sec. 4.3 step 2, first case: with exact cells R_lo_k is at most the
    true k-th smallest rank, so every returned user (r <= r_hi <= c R_lo_k)
    has a rank within c times the k-th best one (checked by brute force)."""
    U, P, t, cnt, Qv, R, T = _table_case(61, integer)
    m = P.shape[0]
    for qi in range(Qv.shape[0]):
        for k in (1, 5, 20):
            rho_k = np.sort(R[qi])[k - 1]
            ids, est = O.table_query(t, cnt, T[:, qi], m, k, 1e9)
            assert len(ids) == k and len(set(ids.tolist())) == k
            assert np.all(R[qi][ids] <= est)            # est = r_hi, an upper bound here
            assert np.all(est <= 1e9 * rho_k)
            # a tight c: whichever case applies, the k smallest r_hi are never
            # worse than the k-th smallest r_hi itself
            ids2, est2 = O.table_query(t, cnt, T[:, qi], m, k, 1.0)
            assert len(ids2) == k and len(set(ids2.tolist())) == k


@pytest.mark.parametrize("integer", [False, True])
def test_table_query_brackets_and_filter(integer):
    """Step 1's bracket holds every exact rank (brute force); step 2 keeps
    the users whose bracket can still beat R_hi_k; step 3's estimates lie in
    their brackets; the answer lists the admitted users first."""
    U, P, t, cnt, Qv, R, T = _table_case(62, integer)
    m, n = P.shape[0], U.shape[0]
    for qi in range(Qv.shape[0]):
        tq = T[:, qi]
        L = np.sum(t >= tq[:, None], axis=1)
        r_lo = np.where(L > 0, 1 + cnt[np.arange(n), np.maximum(L - 1, 0)], 1)
        r_hi = np.where(L < t.shape[1], 1 + cnt[np.arange(n), np.minimum(L, t.shape[1] - 1)], 1 + m)
        assert np.all(r_lo <= R[qi]) and np.all(R[qi] <= r_hi)
        k = 10
        R_lo_k, R_hi_k = np.sort(r_lo)[k - 1], np.sort(r_hi)[k - 1]
        c = 1.0001
        ids, est = O.table_query(t, cnt, tq, m, k, c)
        assert len(ids) == k and len(set(ids.tolist())) == k
        assert np.all(r_lo[ids] <= R_hi_k)                   # nothing Lemma 1 (2) rules out
        assert np.all(est >= r_lo[ids]) and np.all(est <= r_hi[ids])
        if c * R_lo_k < R_hi_k:
            admitted = r_hi[ids] <= c * R_lo_k
            nadm = int(admitted.sum())
            assert np.all(admitted[:nadm]) and not np.any(admitted[nadm:])
            assert nadm == int(np.sum(r_hi <= c * R_lo_k))


def test_table_query_interpolation_ends():
    """Step 3's estimate meets the bracket at the columns' thresholds and
    falls as u.q rises between them (one user, two columns)."""
    t = np.array([[5.0, 4.0, 2.0]])
    cnt = np.array([[5, 12, 40]])
    m = 100
    lo_hi = []
    for x in (4.0 + 1e-12, 4.4, 4.9, 5.0 - 1e-12):
        # a second user with a sure rank of 1 keeps the first one in step 3
        tt = np.vstack([t, [[9.0, 8.0, 7.0]]])
        cc = np.vstack([cnt, [[0, 0, 0]]])
        ids, est = O.table_query(tt, cc, np.array([x, 10.0]), m, 2, 1.0)
        lo_hi.append(est[list(ids).index(0)])
    assert 6.0 <= lo_hi[-1] <= lo_hi[2] <= lo_hi[1] <= lo_hi[0] <= 13.0
    assert abs(lo_hi[0] - 13.0) < 1e-9 and abs(lo_hi[-1] - 6.0) < 1e-9
