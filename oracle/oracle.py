"""CPU reference for exact and c-approximate reverse k-ranks queries.

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the CPU-baseline
leg of the benchmark are the only callers.  The product library never
imports, links or runs anything here, and nothing here imports the product.

What is computed, and where the paper defines it (arXiv 2504.13446):

* ``ranks``     -- Sec. 2, Def. 1: r(q,u,P) = 1 + #{p : u.p > u.q}, strict ">".
                   Inner products use one fixed FP64 evaluation (sequential
                   fma in dimension order, see rkr_oracle.c).
* ``topk``      -- Sec. 2, Def. 2: the k users of smallest rank ("highest
                   rank" in the introduction means rank 1 is best); users
                   tied on rank are ordered by id, and the answer is listed by
                   (rank, id) ascending.
* ``def3_check``-- Sec. 2, Def. 3: the i-th user of U_c must have rank at most
                   c times the rank of the i-th user of U_rr.  Also the
                   abstract's weaker form (every rank <= c * tau, with tau the
                   k-th exact rank).
* ``accuracy``, ``overall_ratio`` -- Sec. 5, the two quality criteria.
* ``certify``   -- a checker for a claimed exact answer on all users or a
                   sample of them (see orc_certify).
* ``topk_exact``-- the Def. 2 answer for large shapes by early abandon: users
                   whose partial count already puts them behind the k best
                   found so far stop counting (Lemma 1 (2) on exact counts);
                   the result equals topk(ranks(...)) (see orc_topk_abandon).
* ``paper_table``, ``paper_table_query`` -- the paper's own method: Alg. 1
                   (Sec. 4.2: norm-sorted buckets, uniform thresholds between
                   the footnote's domain values, cells estimated from random
                   samples per bucket) and the query's three steps (Sec. 4.3).
* ``norm_order``, ``stratified_sample``, ``sketch`` -- the per-user score
                   sketch: P ordered by norm, descending (Sec. 4.2 step 1),
                   split into equal buckets with one sample from the middle
                   of each (the norm-stratified sampling of Sec. 4.2 step 3
                   with one sample per bucket), spec scores of the user
                   against the samples, sorted, read at fixed positions.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "rkr_oracle.c")
_LIB = os.path.join(_HERE, "librkr_oracle.so")

_CFLAGS = ["-O2", "-mfma", "-ffp-contract=off", "-fno-fast-math", "-fopenmp",
           "-shared", "-fPIC", "-std=c11"]


def build(force: bool = False) -> str:
    """Compile the C oracle into oracle/librkr_oracle.so."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", *_CFLAGS, "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        build()
        L = ctypes.CDLL(_LIB)
        d, i64, i32, vp = ctypes.c_double, ctypes.c_int64, ctypes.c_int32, ctypes.c_void_p
        L.orc_num_threads.restype = ctypes.c_int
        L.orc_dots.argtypes = [vp, i64, vp, i64, ctypes.c_int, vp]
        L.orc_norms.argtypes = [vp, i64, ctypes.c_int, vp]
        L.orc_ranks.argtypes = [vp, i64, vp, i64, vp, i64, ctypes.c_int, vp, i64, vp, ctypes.c_int]
        L.orc_certify.argtypes = [vp, i64, vp, i64, vp, ctypes.c_int, ctypes.c_int, vp, vp, vp,
                                  i64, vp, vp, ctypes.c_int]
        L.orc_topk_abandon.argtypes = [vp, i64, vp, i64, vp, vp, ctypes.c_int, ctypes.c_int, vp,
                                       i64, vp, vp, vp, ctypes.c_int]
        L.orc_paper_table.argtypes = [vp, i64, vp, i64, vp, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                      ctypes.c_int, vp, vp, vp, vp, ctypes.c_int]
        L.orc_norm_order.argtypes = [vp, i64, vp]
        L.orc_sketch.argtypes = [vp, i64, vp, vp, i64, ctypes.c_int, vp, ctypes.c_int, vp,
                                 ctypes.c_int]
        L.orc_rank_table.argtypes = [vp, i64, vp, i64, vp, i64, ctypes.c_int, vp, ctypes.c_int,
                                     vp, vp, ctypes.c_int]
        for f in (L.orc_dots, L.orc_norms, L.orc_ranks, L.orc_certify, L.orc_norm_order,
                  L.orc_sketch, L.orc_rank_table, L.orc_topk_abandon, L.orc_paper_table):
            f.restype = None
        _lib = L
    return _lib


def num_threads() -> int:
    return int(lib().orc_num_threads())


# --------------------------------------------------------------------------
# master values -> float64 (exact widening)
# --------------------------------------------------------------------------
def widen(x, dtype: str | None = None) -> np.ndarray:
    """Exact float64 copy of master values.

    ``dtype='bf16'`` reads uint16 bit patterns as bfloat16; float32 and
    float64 arrays widen directly.  Both widenings are exact.
    """
    x = np.asarray(x)
    if dtype == "bf16" or x.dtype == np.uint16:
        bits = x.astype(np.uint32) << np.uint32(16)
        return np.ascontiguousarray(bits.view(np.float32).astype(np.float64))
    return np.ascontiguousarray(x.astype(np.float64))


def _p(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def dots(X, Y) -> np.ndarray:
    X = widen(X); Y = widen(Y)
    out = np.empty((X.shape[0], Y.shape[0]), np.float64)
    lib().orc_dots(_p(X), X.shape[0], _p(Y), Y.shape[0], X.shape[1], _p(out))
    return out


def norms(X) -> np.ndarray:
    X = widen(X)
    out = np.empty(X.shape[0], np.float64)
    lib().orc_norms(_p(X), X.shape[0], X.shape[1], _p(out))
    return out


def ranks(U, P, Qv, uids=None, threads: int = 0) -> np.ndarray:
    """Def. 1 ranks, shape [nq, nu] (nu = len(uids) or n)."""
    U = widen(U); P = widen(P); Qv = widen(np.atleast_2d(Qv))
    n, d = U.shape
    assert P.shape[1] == d and Qv.shape[1] == d
    if uids is None:
        nu, up = n, None
        uarr = None
    else:
        uarr = np.ascontiguousarray(np.asarray(uids, np.int64))
        nu, up = uarr.shape[0], _p(uarr)
    out = np.empty((Qv.shape[0], nu), np.int32)
    lib().orc_ranks(_p(U), n, _p(P), P.shape[0], _p(Qv), Qv.shape[0], d, up, nu, _p(out),
                    int(threads))
    return out


def topk(rank_row, k: int, uids=None):
    """Def. 2 answer from a row of ranks: k users by (rank, id) ascending."""
    r = np.asarray(rank_row, np.int64)
    ids = np.arange(r.shape[0], dtype=np.int64) if uids is None else np.asarray(uids, np.int64)
    order = np.lexsort((ids, r))[:k]
    return ids[order], r[order]


def certify(U, P, q, k, ids, rks, check=None, order=None, threads: int = 0):
    """Check a claimed exact answer; returns (rank mismatches, set violations, examined).

    ``order``: the order in which the early-stopping scans visit the items
    (None: 0..m-1); norm_order(P) makes them stop sooner."""
    U = widen(U); P = widen(P); q = widen(np.asarray(q).reshape(1, -1))
    ids = np.ascontiguousarray(np.asarray(ids, np.int64))
    rks = np.ascontiguousarray(np.asarray(rks, np.int32))
    chk = np.arange(U.shape[0], dtype=np.int64) if check is None else \
        np.ascontiguousarray(np.asarray(check, np.int64))
    op = None
    if order is not None:
        order = np.ascontiguousarray(np.asarray(order, np.int64))
        assert order.shape[0] == P.shape[0]
        op = _p(order)
    out = np.zeros(3, np.int64)
    lib().orc_certify(_p(U), U.shape[0], _p(P), P.shape[0], _p(q), U.shape[1], int(k), _p(ids),
                      _p(rks), _p(chk), chk.shape[0], op, _p(out), int(threads))
    return int(out[0]), int(out[1]), int(out[2])


def topk_exact(U, P, q, k: int, uids=None, order=None, threads: int = 0, stats: dict | None = None):
    """Def. 2 answer of one query by early abandon (see orc_topk_abandon):
    the same result as topk(ranks(U, P, q)[0], k) restricted to the domain
    ``uids`` (None: every user), computed without finishing the count of users
    that cannot enter the answer.  Items are visited in ``order`` (None: the
    norm order, Sec. 4.2 step 1).  Returns (ids, ranks) by (rank, id); with a
    dict ``stats``, fills items_visited and users_fully_counted."""
    U = widen(U); P = widen(P); q = widen(np.asarray(q).reshape(1, -1))
    n, d = U.shape
    m = P.shape[0]
    if order is None:
        order = norm_order(P)
    order = np.ascontiguousarray(np.asarray(order, np.int64))
    assert order.shape[0] == m
    up, nu = None, n
    if uids is not None:
        uids = np.ascontiguousarray(np.asarray(uids, np.int64))
        up, nu = _p(uids), uids.shape[0]
    kk = int(min(k, nu))
    ids = np.empty(kk, np.int64)
    rks = np.empty(kk, np.int32)
    st = np.zeros(2, np.int64)
    lib().orc_topk_abandon(_p(U), n, _p(P), m, _p(order), _p(q), d, int(k), up, nu, _p(ids),
                           _p(rks), _p(st), int(threads))
    if stats is not None:
        stats["items_visited"] = int(st[0])
        stats["users_fully_counted"] = int(st[1])
    return ids, rks


def norm_order(P) -> np.ndarray:
    nrm = norms(P)
    out = np.empty(nrm.shape[0], np.int64)
    lib().orc_norm_order(_p(nrm), nrm.shape[0], _p(out))
    return out


def stratified_sample(P, S: int) -> np.ndarray:
    """One item from the middle of each of S equal norm buckets (ids into P)."""
    order = norm_order(P)
    m = order.shape[0]
    S = min(S, m)
    mid = ((2 * np.arange(S, dtype=np.int64) + 1) * m) // (2 * S)
    return order[mid]


def sketch_positions(S: int, levels: int = 16) -> np.ndarray:
    """1-based positions spaced geometrically from 1 to S: ceil(S ** (i / (levels-1)))."""
    i = np.arange(levels, dtype=np.float64)
    pos = np.ceil(np.power(float(S), i / (levels - 1)) - 1e-9).astype(np.int32)
    return np.clip(pos, 1, S)


def sketch(U, P, sample, pos, threads: int = 0) -> np.ndarray:
    U = widen(U); P = widen(P)
    sample = np.ascontiguousarray(np.asarray(sample, np.int64))
    pos = np.ascontiguousarray(np.asarray(pos, np.int32))
    out = np.empty((U.shape[0], pos.shape[0]), np.float64)
    lib().orc_sketch(_p(U), U.shape[0], _p(P), _p(sample), sample.shape[0], U.shape[1], _p(pos),
                     pos.shape[0], _p(out), int(threads))
    return out


def rank_table(U, P, sample, pos, threads: int = 0):
    """Rank table with exact cells (Sec. 4.2 steps 2-3): thresholds t[u][j] =
    the user's spec scores against the sample items, sorted descending, at the
    1-based positions pos; cells cnt[u][j] = #{p in P : s(u,p) > t[u][j]}
    (the paper's T_{i,j} minus its leading 1, counted over all of P)."""
    U = widen(U); P = widen(P)
    sample = np.ascontiguousarray(np.asarray(sample, np.int64))
    pos = np.ascontiguousarray(np.asarray(pos, np.int32))
    t = np.empty((U.shape[0], pos.shape[0]), np.float64)
    cnt = np.empty((U.shape[0], pos.shape[0]), np.int64)
    lib().orc_rank_table(_p(U), U.shape[0], _p(P), P.shape[0], _p(sample), sample.shape[0],
                         U.shape[1], _p(pos), pos.shape[0], _p(t), _p(cnt), int(threads))
    return t, cnt


def table_query(t, cnt, tq, m: int, k: int, c: float):
    """The paper's query on a rank table (Sec. 4.3, steps 1-3), for one query.

    t[u][j]: user u's thresholds, descending in j; cnt[u][j]: the count of
    items above t[u][j] (a table cell minus its leading 1); tq[u] = u.q (the
    spec FP64 dot); m = |P|.  Readings where the text is loose:
      * step 1: with L = #{j : t[u][j] >= u.q}, the query score lies between
        columns L-1 and L, so r_lo = 1 + cnt[L-1] (1 when L = 0) and r_hi =
        1 + cnt[L] (1 + m when L = tau);
      * step 2 ranks users by r_hi ("smallest r"), admits r_hi <= c R_lo_k,
        and drops users with r_lo > R_hi_k (Lemma 1 (2), strict);
      * step 3 interpolates linearly in u.q between the two columns:
        est = r_lo + (r_hi - r_lo) * ((t[L-1] - u.q) / (t[L-1] - t[L])), and
        est = r_lo at either end of the table or between equal thresholds;
        the estimate is rounded to FP32 for ordering, ties by user id.
    Returns (ids, est): the k users in answer order and the rank each was
    chosen by (r_hi for the users admitted in step 2, est after them)."""
    t = np.asarray(t, np.float64)
    cnt = np.asarray(cnt, np.int64)
    tq = np.asarray(tq, np.float64)
    n, tau = t.shape
    ids_all = np.arange(n, dtype=np.int64)
    # step 1: brackets
    L = np.sum(t >= tq[:, None], axis=1)
    r_lo = np.where(L > 0, 1 + cnt[ids_all, np.maximum(L - 1, 0)], 1)
    r_hi = np.where(L < tau, 1 + cnt[ids_all, np.minimum(L, tau - 1)], 1 + m)
    R_lo_k = np.sort(r_lo)[k - 1]
    R_hi_k = np.sort(r_hi)[k - 1]
    by_hi = np.lexsort((ids_all, r_hi))
    # step 2
    if c * float(R_lo_k) >= float(R_hi_k):
        sel = by_hi[:k]
        return sel.astype(np.int32), r_hi[sel].astype(np.float64)
    admit = r_hi.astype(np.float64) <= c * float(R_lo_k)
    first = by_hi[admit[by_hi]]
    rest = (~admit) & (r_lo <= R_hi_k)
    # step 3: interpolation for the users left open
    est = r_lo.astype(np.float64)
    inner = (L > 0) & (L < tau)
    tA = t[ids_all, np.maximum(L - 1, 0)]
    tB = t[ids_all, np.minimum(L, tau - 1)]
    span = np.where(inner & (tA > tB), tA - tB, 1.0)
    frac = np.where(inner & (tA > tB), (tA - tq) / span, 0.0)
    est = np.where(inner & (tA > tB), r_lo + (r_hi - r_lo).astype(np.float64) * frac, est)
    est32 = est.astype(np.float32)
    cand = ids_all[rest]
    order = cand[np.lexsort((cand, est32[cand]))]
    fill = order[:k - first.shape[0]]
    ids = np.concatenate([first, fill]).astype(np.int32)
    out = np.concatenate([r_hi[first].astype(np.float64), est[fill]])
    return ids, out


def paper_table(U, P, tau: int, omega: int, s: int, sample_pos, threads: int = 0):
    """The paper's rank table (Sec. 4.2, Alg. 1) with estimated cells (see
    orc_paper_table): returns (fmin [n], step [n], T [n, tau] float32).
    sample_pos [omega * s]: positions within each bucket (the random draws)."""
    U = widen(U); P = widen(P)
    n, d = U.shape
    m = P.shape[0]
    order = norm_order(P)
    pos = np.ascontiguousarray(np.asarray(sample_pos, np.int32).reshape(-1))
    assert pos.shape[0] == omega * s and tau >= 2
    fmin = np.empty(n, np.float64)
    step = np.empty(n, np.float64)
    T = np.empty((n, tau), np.float32)
    lib().orc_paper_table(_p(U), n, _p(P), m, _p(order), d, int(tau), int(omega), int(s), _p(pos),
                          _p(fmin), _p(step), _p(T), int(threads))
    return fmin, step, T


def paper_table_thresholds(fmin, step, tau: int) -> np.ndarray:
    """t[u][j] = fmin[u] + j * step[u] (j = 0..tau-1), one FP64 product and
    one FP64 sum each, as Alg. 1 step 2 spaces them."""
    j = np.arange(tau, dtype=np.float64)
    return np.asarray(fmin, np.float64)[:, None] + j[None, :] * np.asarray(step, np.float64)[:, None]


def paper_table_bounds(fmin, step, T, tq, m: int):
    """Query step 1 (Sec. 4.3) on the paper's table: with ascending thresholds
    t[j] and L = #{j : t[j] <= u.q}, u.q lies in [t[L-1], t[L]), so
    r_lo = T[L] (1 when L = tau) and r_hi = T[L-1] (m + 1 when L = 0), both
    FP32 as the cells.  Returns (L, r_lo, r_hi, t)."""
    T = np.asarray(T, np.float32)
    n, tau = T.shape
    t = paper_table_thresholds(fmin, step, tau)
    tq = np.asarray(tq, np.float64)
    L = np.sum(t <= tq[:, None], axis=1)
    ids = np.arange(n)
    r_lo = np.where(L == tau, np.float32(1.0), T[ids, np.minimum(L, tau - 1)]).astype(np.float32)
    r_hi = np.where(L == 0, np.float32(m + 1), T[ids, np.maximum(L - 1, 0)]).astype(np.float32)
    return L, r_lo, r_hi, t


def paper_table_query(fmin, step, T, tq, m: int, k: int, c: float):
    """The paper's query (Sec. 4.3, steps 1-3) on its own table, one query.

    Step 1 as paper_table_bounds; R_lo_k, R_hi_k are the k-th smallest r_lo
    and r_hi.  Step 2: if c R_lo_k >= R_hi_k the answer is the k users of
    smallest r_hi (ties by id); otherwise the users with r_hi <= c R_lo_k come
    first (by r_hi, id), users with r_lo > R_hi_k are ruled out (Lemma 1 (2))
    and the rest stay open.  Step 3 fills the answer with the open users of
    smallest estimate, linear in u.q between (t[L-1], r_hi) and (t[L], r_lo),
    r_lo at either end of the row or between equal thresholds, ordered by the
    estimate rounded to FP32, ties by id.  Comparisons with c R_lo_k are in
    FP64.  Returns (ids, values): the value each user was chosen by."""
    L, r_lo, r_hi, t = paper_table_bounds(fmin, step, T, tq, m)
    n, tau = t.shape
    ids_all = np.arange(n, dtype=np.int64)
    R_lo_k = np.sort(r_lo)[k - 1]
    R_hi_k = np.sort(r_hi)[k - 1]
    by_hi = np.lexsort((ids_all, r_hi))
    if c * float(R_lo_k) >= float(R_hi_k):
        sel = by_hi[:k]
        return sel.astype(np.int32), r_hi[sel].astype(np.float64)
    admit = r_hi.astype(np.float64) <= c * float(R_lo_k)
    first = by_hi[admit[by_hi]]
    rest = (~admit) & (r_lo <= R_hi_k)
    inner = (L > 0) & (L < tau)
    tA = t[ids_all, np.maximum(L - 1, 0)]
    tB = t[ids_all, np.minimum(L, tau - 1)]
    ok = inner & (tB > tA)
    lo64, hi64 = r_lo.astype(np.float64), r_hi.astype(np.float64)
    frac = np.where(ok, (np.asarray(tq, np.float64) - tA) / np.where(ok, tB - tA, 1.0), 0.0)
    est = np.where(ok, hi64 + (lo64 - hi64) * frac, lo64)
    est32 = est.astype(np.float32)
    cand = ids_all[rest]
    order = cand[np.lexsort((cand, est32[cand]))]
    fill = order[:k - first.shape[0]]
    ids = np.concatenate([first, fill]).astype(np.int32)
    vals = np.concatenate([hi64[first], est[fill]])
    return ids, vals


# --------------------------------------------------------------------------
# Def. 3 and the quality criteria of Sec. 5
# --------------------------------------------------------------------------
def def3_check(true_ranks_c, exact_ranks_rr, c: float):
    """Return (violations, abstract-form violations).

    true_ranks_c: the exact ranks of the k users returned as U_c.
    exact_ranks_rr: the k ranks of U_rr (Def. 2).
    The i-th user of each set is taken in rank order (Def. 3 pairs the
    i-th user of U_c with the i-th user of U_rr).
    """
    a = np.sort(np.asarray(true_ranks_c, np.float64))
    b = np.sort(np.asarray(exact_ranks_rr, np.float64))
    assert a.shape == b.shape
    viol = int(np.sum(a > c * b))
    tau = b[-1] if b.size else 0.0
    weak = int(np.sum(a > c * tau))
    return viol, weak


def accuracy(true_ranks_c, exact_ranks_rr, c: float) -> float:
    a = np.sort(np.asarray(true_ranks_c, np.float64))
    b = np.sort(np.asarray(exact_ranks_rr, np.float64))
    return float(np.mean(a <= c * b))


def overall_ratio(true_ranks_c, exact_ranks_rr) -> float:
    a = np.sort(np.asarray(true_ranks_c, np.float64))
    b = np.sort(np.asarray(exact_ranks_rr, np.float64))
    return float(np.mean(a / b))
