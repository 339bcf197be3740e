"""GPU: the all-ranks pipeline replayed as a captured hipGraph.  Every replay
is checked against the eager path and the oracle, with other eager library
work and host synchronisations between the replays; a query with more near
ties than the captured buffer holds must fall back to the eager path."""
import numpy as np
import pytest
import torch

from oracle import oracle as O
from paper_2504_13446_amd import rkr, workloads as W

pytestmark = pytest.mark.gpu


def _dev(x, dtype):
    return rkr.to_device(x, dtype)


@pytest.mark.parametrize("score", ["bf16", "fp8", "f32"])
def test_graph_replays_match_eager(score):
    w = W.make("small", n=2100, m=3300, nq=7)
    idx = rkr.Index(_dev(w.U, "f32"), _dev(w.P, "f32"), score=score)
    Q = _dev(w.Qv, "f32")
    R = O.ranks(w.U, w.P, w.Qv)
    eager = [idx.ranks(Q[i]).cpu().numpy() for i in range(5)]
    for i in range(5):
        assert np.array_equal(eager[i], R[i]), i
    idx.configure(graph=True)
    first = idx.ranks(Q[0]).cpu().numpy()          # eager run, then capture
    assert np.array_equal(first, R[0])
    for rep, i in enumerate([1, 2, 0, 3, 4, 2]):
        got = idx.ranks(Q[i]).cpu().numpy()
        st = idx.stats()
        assert st["graph_replays"] == 1, rep
        assert np.array_equal(got, eager[i]), (rep, i, np.flatnonzero(got != eager[i])[:5])
        # eager work on the same index between replays
        ids, rk, off = idx.query_batch(Q[5:7], [9, 9])
        torch.cuda.synchronize()
        for j in range(2):
            wi, wr = O.topk(R[5 + j], 9)
            assert np.array_equal(ids.cpu().numpy()[off[j]:off[j + 1]], wi)
    idx.configure(graph=False)
    assert np.array_equal(idx.ranks(Q[3]).cpu().numpy(), eager[3])
    assert idx.stats()["graph_replays"] == 0
    idx.close()


def test_graph_near_tie_overflow_falls_back():
    """Entries in {-1, 0, 1}, d = 3: an integer query ties with about a
    seventh of the items for every user (over 10^6 near-tie records), while
    a Gaussian query ties with almost none.  The graph captured after the
    Gaussian query holds too few records for the integer one: that call must
    answer eagerly (and exactly); the next call captures again."""
    rng = np.random.default_rng(17)
    n, m, d = 2000, 8000, 3
    U = rng.integers(-1, 2, size=(n, d)).astype(np.float32)
    P = rng.integers(-1, 2, size=(m, d)).astype(np.float32)
    qg = rng.standard_normal(d).astype(np.float32)
    qi = P[5].copy()
    R = O.ranks(U, P, np.stack([qg, qi]))
    idx = rkr.Index(_dev(U, "f32"), _dev(P, "f32"), score="bf16")
    idx.configure(graph=True)
    assert np.array_equal(idx.ranks(_dev(qg, "f32")).cpu().numpy(), R[0])
    assert np.array_equal(idx.ranks(_dev(qg, "f32")).cpu().numpy(), R[0])
    assert idx.stats()["graph_replays"] == 1
    got = idx.ranks(_dev(qi, "f32")).cpu().numpy()
    st = idx.stats()
    assert st["graph_replays"] == 0 and st["uncertain"] > (1 << 20), st["uncertain"]
    assert np.array_equal(got, R[1])
    # recaptured with room for the integer query's records
    assert np.array_equal(idx.ranks(_dev(qi, "f32")).cpu().numpy(), R[1])
    got = idx.ranks(_dev(qi, "f32")).cpu().numpy()
    st = idx.stats()
    assert st["graph_replays"] == 1 and st["uncertain"] > (1 << 20)
    assert np.array_equal(got, R[1])
    assert np.array_equal(idx.ranks(_dev(qg, "f32")).cpu().numpy(), R[0])
    idx.close()
