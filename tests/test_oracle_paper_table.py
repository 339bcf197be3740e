"""Pins of the oracle's version of the paper's own method: the rank table of
Alg. 1 (Sec. 4.2) with estimated cells, and the query's three steps (Sec. 4.3).

* With every item of every bucket sampled, the estimator of Sec. 4.2 step 3 is
  exact: on integer data (exact scores from numpy, thresholds recomputed in
  numpy from the footnote's domain values) every cell equals 1 + #{p : u.p > t}.
* The estimator is unbiased (Sec. 4.2): averaged over many sample draws the
  cells approach their exact values.
* Cells do not increase along a row (the thresholds ascend).
* The bracket of Fig. 1 (u1.q = 4.4 between thresholds whose cells are 13 and
  6 gives 6 <= r <= 13).
* Both cases of query step 2, Lemma 1 (2)'s filter and step 3's interpolation
  on hand-made tables.
* A planted ">=" in the cell count (a patched copy of the oracle) is caught.
"""
import ctypes
import os
import subprocess

import numpy as np
import pytest

from oracle import oracle as O
from paper_2504_13446_amd import workloads as W


def _exact_table(U, P, tau):
    """Thresholds and exact cells from numpy on integer data (every sum exact)."""
    S = U.astype(np.float64) @ P.astype(np.float64).T
    un = np.sqrt(np.sum(U.astype(np.float64) ** 2, axis=1))
    pmax = np.max(np.sqrt(np.sum(P.astype(np.float64) ** 2, axis=1)))
    fmax = un * pmax
    fmin = -fmax
    step = (fmax - fmin) / (tau - 1)
    t = fmin[:, None] + np.arange(tau, dtype=np.float64)[None, :] * step[:, None]
    cells = 1 + np.sum(S[:, :, None] > t[:, None, :], axis=1)
    return fmin, step, t, cells, S


def test_exact_when_every_item_is_sampled():
    rng = np.random.default_rng(4)
    U = rng.integers(-3, 4, size=(40, 5)).astype(np.float32)
    P = rng.integers(-3, 4, size=(90, 5)).astype(np.float32)
    tau, omega = 37, 6
    s = 90 // omega + 1                     # more than any bucket holds: all taken
    pos = W.bucket_sample_positions(90, omega, s, seed=1)
    fmin, step, T = O.paper_table(U, P, tau, omega, s, pos)
    efmin, estep, _, cells, _ = _exact_table(U, P, tau)
    assert np.array_equal(fmin, efmin) and np.array_equal(step, estep)
    assert np.array_equal(T, cells.astype(np.float32))


def test_domain_thresholds_hit_integer_scores():
    """|u| = 5 and max |p| = 5 give f_max = 25, and tau = 51 thresholds land on
    the integers -25..25, where integer scores tie with them: only scores
    strictly above count (Def. 1's strict order carried into the cells)."""
    rng = np.random.default_rng(9)
    U = np.array([[3, 4], [4, 3], [0, 5], [-5, 0]], np.float32)
    P = np.concatenate([np.array([[3, 4]], np.float32),
                        rng.integers(-3, 4, size=(60, 2)).astype(np.float32)])
    tau, omega, s = 51, 4, 20
    pos = W.bucket_sample_positions(61, omega, s, seed=2)
    fmin, step, T = O.paper_table(U, P, tau, omega, s, pos)
    assert np.all(fmin == -25.0) and np.all(step == 1.0)
    _, _, t, cells, S = _exact_table(U, P, tau)
    assert np.any(S[:, :, None] == t[:, None, :])         # ties with thresholds exist
    assert np.array_equal(T, cells.astype(np.float32))


def test_estimator_is_unbiased_over_draws():
    rng = np.random.default_rng(6)
    U = rng.integers(-3, 4, size=(12, 4)).astype(np.float32)
    P = rng.integers(-3, 4, size=(150, 4)).astype(np.float32)
    tau, omega, s = 9, 5, 6
    _, _, _, cells, _ = _exact_table(U, P, tau)
    draws = np.stack([O.paper_table(U, P, tau, omega, s, W.bucket_sample_positions(150, omega, s, seed=100 + i))[2]
                      for i in range(300)]).astype(np.float64)
    mean, sd = draws.mean(axis=0), draws.std(axis=0)
    se = sd / np.sqrt(draws.shape[0])
    assert np.all(np.abs(mean - cells) <= 5 * se + 1e-9), np.max(np.abs(mean - cells) / (se + 1e-12))
    assert np.any(sd > 0)                                  # the draws do vary


def test_rows_do_not_increase_and_stay_in_range():
    w = W.make("small", n=300, m=800, d=16, nq=1)
    tau, omega, s = 100, 8, 16
    _, _, T = O.paper_table(w.U, w.P, tau, omega, s, W.bucket_sample_positions(800, omega, s))
    assert np.all(np.diff(T, axis=1) <= 0)
    assert np.all(T >= 1) and np.all(T <= 801)


def test_fig1_bracket():
    """Fig. 1: u1.q = 4.4 falls between thresholds 4.0 and 4.5 whose cells are 13
    and 6, so 6 <= r <= 13."""
    fmin, step = np.array([4.0]), np.array([0.5])
    T = np.array([[13, 6, 2]], np.float32)
    L, r_lo, r_hi, _ = O.paper_table_bounds(fmin, step, T, [4.4], m=20)
    assert (L[0], r_lo[0], r_hi[0]) == (1, 6.0, 13.0)
    # below every threshold: r_hi = m + 1; at or above the last: r_lo = 1
    L, r_lo, r_hi, _ = O.paper_table_bounds(np.array([4.0, 4.0]), np.array([0.5, 0.5]),
                                            np.array([[13, 6, 2], [13, 6, 2]], np.float32), [3.9, 5.0], m=20)
    assert L.tolist() == [0, 3] and r_lo.tolist() == [13.0, 1.0] and r_hi.tolist() == [21.0, 2.0]


def _table(rows):
    T = np.array(rows, np.float32)
    n, tau = T.shape
    return np.zeros(n), np.ones(n), T


def test_query_first_case_takes_the_k_smallest_upper_bounds():
    # thresholds 0, 1, 2, 3; every user at u.q = 1.5: r_lo = T[2], r_hi = T[1]
    fmin, step, T = _table([[50, 9, 8, 1], [50, 7, 6, 1], [50, 7, 7, 1], [50, 20, 3, 1]])
    ids, vals = O.paper_table_query(fmin, step, T, [1.5] * 4, m=60, k=2, c=10.0)
    assert ids.tolist() == [1, 2] and vals.tolist() == [7.0, 7.0]   # tie on r_hi broken by id


def test_query_second_case_filter_and_interpolation():
    # r_lo = T[2], r_hi = T[1] at u.q in [1, 2)
    fmin, step, T = _table([[90, 10, 4, 1],      # user 0: [4, 10]
                            [90, 12, 5, 1],      # user 1: [5, 12]
                            [90, 40, 30, 1],     # user 2: [30, 40], ruled out (30 > R_hi_k)
                            [90, 20, 3, 1],      # user 3: [3, 20]
                            [90, 5, 5, 1]])      # user 4: [5, 5], admitted (5 <= c R_lo_k)
    tq = [1.25, 1.5, 1.5, 1.75, 1.5]
    ids, vals = O.paper_table_query(fmin, step, T, tq, m=99, k=3, c=1.25)
    # R_lo_k = 5 (3rd of 3,4,5,5,30), R_hi_k = 12 (3rd of 5,10,12,20,40): 1.25*5 < 12
    # admitted: r_hi <= 6.25 -> user 4; open: users 0, 1, 3 (r_lo <= 12)
    # estimates: u0 10 + (4-10)*0.25 = 8.5; u1 12 + (5-12)*0.5 = 8.5; u3 20 + (3-20)*0.75 = 7.25
    assert ids.tolist() == [4, 3, 0] and vals.tolist() == [5.0, 7.25, 8.5]


_SRC = os.path.join(os.path.dirname(O.__file__), "rkr_oracle.c")


def test_planted_ge_in_the_cells_is_caught(tmp_path):
    src = open(_SRC).read()
    old = "                        if (sc > t[j])\n                            A[j] += 1;"
    assert src.count(old) == 1
    path = tmp_path / "mut_cells.c"
    path.write_text(src.replace(old, old.replace("sc > t[j]", "sc >= t[j]")))
    so = tmp_path / "mut_cells.so"
    subprocess.check_call(["gcc", "-O2", "-mfma", "-ffp-contract=off", "-fopenmp", "-shared", "-fPIC",
                           "-std=c11", "-o", str(so), str(path), "-lm"])
    L = ctypes.CDLL(str(so))
    vp, i64, ci = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int
    L.orc_paper_table.argtypes = [vp, i64, vp, i64, vp, ci, ci, ci, ci, vp, vp, vp, vp, ci]
    L.orc_paper_table.restype = None
    U = np.array([[3, 4], [4, 3], [0, 5], [-5, 0]], np.float64)
    rng = np.random.default_rng(9)
    P = np.concatenate([np.array([[3, 4]], np.float64), rng.integers(-3, 4, size=(60, 2)).astype(np.float64)])
    tau, omega, s = 51, 4, 20
    pos = W.bucket_sample_positions(61, omega, s, seed=2)
    order = O.norm_order(P)
    fmin, step = np.empty(4), np.empty(4)
    T = np.empty((4, tau), np.float32)
    p = lambda a: a.ctypes.data_as(vp)
    L.orc_paper_table(p(U), 4, p(P), 61, p(order), 2, tau, omega, s, p(pos), p(fmin), p(step), p(T), 1)
    _, _, _, cells, _ = _exact_table(U, P, tau)
    assert not np.array_equal(T, cells.astype(np.float32))
