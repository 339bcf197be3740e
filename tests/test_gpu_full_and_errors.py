"""GPU: error paths through the library, approximate mode at c = 1, and the
full-size batch (the benchmark's launch configuration) checked on samples."""
import numpy as np
import pytest
import torch

from oracle import oracle as O
from paper_2504_13446_amd import rkr, workloads as W

pytestmark = pytest.mark.gpu


def _dev(x, dtype):
    return rkr.to_device(x, dtype)


def test_invalid_inputs_are_rejected():
    rng = np.random.default_rng(0)
    U = rng.standard_normal((100, 16)).astype(np.float32)
    P = rng.standard_normal((80, 16)).astype(np.float32)
    bad = U.copy(); bad[3, 4] = np.nan
    with pytest.raises(rkr.RkrError) as e:
        rkr.Index(_dev(bad, "f32"), _dev(P, "f32"))
    assert e.value.status == rkr.RKR_E_INVALID and "non-finite" in e.value.message
    big = P.copy(); big[0, 0] = 2.0 ** 60
    with pytest.raises(rkr.RkrError) as e:
        rkr.Index(_dev(U, "f32"), _dev(big, "f32"))
    assert e.value.status == rkr.RKR_E_INVALID
    idx = rkr.Index(_dev(U, "f32"), _dev(P, "f32"))
    Q = _dev(P[:3], "f32")
    with pytest.raises(rkr.RkrError) as e:
        idx.query_batch(Q, [5, 0, 5])
    assert e.value.status == rkr.RKR_E_INVALID
    with pytest.raises(rkr.RkrError):
        idx.query_batch(Q, [5, 101, 5])                        # k above the domain
    with pytest.raises(rkr.RkrError) as e:
        idx.query_batch(Q, [5, 5, 5], c=[1.5, 0.9, 1.5])
    assert "c must be >= 1" in e.value.message
    with pytest.raises(rkr.RkrError) as e:
        idx.query_batch(Q, [5, 5, 5000])
    assert e.value.status == rkr.RKR_E_INVALID
    off = np.array([0, 3, 6, 9])
    with pytest.raises(rkr.RkrError) as e:                     # duplicate id within a list
        idx.query_batch(Q, [1, 1, 1], cand_off=off,
                        cand_ids=torch.tensor([1, 2, 1, 4, 5, 6, 7, 8, 9], dtype=torch.int32, device="cuda"))
    assert "duplicated" in e.value.message
    with pytest.raises(rkr.RkrError):                          # id out of range
        idx.query_batch(Q, [1, 1, 1], cand_off=off,
                        cand_ids=torch.tensor([1, 2, 3, 4, 5, 600, 7, 8, 9], dtype=torch.int32, device="cuda"))
    with pytest.raises(rkr.RkrError):                          # offsets not monotone
        idx.query_batch(Q, [1, 1, 1], cand_off=np.array([0, 3, 2, 9]),
                        cand_ids=torch.arange(9, dtype=torch.int32, device="cuda"))
    qn = P[0].copy(); qn[1] = np.inf
    with pytest.raises(rkr.RkrError):
        idx.query_exact(_dev(qn, "f32"), 3)
    with pytest.raises(rkr.RkrError) as e:
        idx.train(Q)                                           # built without a sketch
    assert e.value.status == rkr.RKR_E_STATE
    # the index still answers correctly after the rejected calls
    R = O.ranks(U, P, P[:3])
    ids, rk, off = idx.query_batch(Q, [7, 7, 7])
    for i in range(3):
        wi, wr = O.topk(R[i], 7)
        assert np.array_equal(ids.cpu().numpy()[off[i]:off[i + 1]], wi)
    idx.close()


def test_approx_c1_equals_exact():
    w = W.make("small", n=1500, m=2500, nq=8)
    idx = rkr.Index(_dev(w.U, "f32"), _dev(w.P, "f32"))
    Q = _dev(w.Qv, "f32")
    a = idx.query_batch(Q, w.k)
    b = idx.query_batch(Q, w.k, c=1.0)
    assert torch.equal(a[0], b[0]) and torch.equal(a[1], b[1])
    idx.close()


def test_full_size_batch_sampled():
    """1M users x 1M items x d=200, 256 queries, k=100, with the rank table
    of the benchmark's configuration.  For two queries: the ranks of all 100
    returned users are recomputed by the oracle, and 3,000 other users are
    certified not to beat the k-th (rank, id): 1,500 at random and the 1,500
    best by u.q/|u| outside the answer (the ones most likely to)."""
    w = W.make("batch")
    idx = rkr.Index(_dev(w.U, "bf16"), _dev(w.P, "bf16"), score="bf16", rank_table=4096)
    ids, rk, off = idx.query_batch(_dev(w.Qv, "bf16"), w.k)
    ids = ids.cpu().numpy(); rk = rk.cpu().numpy()
    st = idx.stats()
    idx.close()
    assert st["pairs"] == 256 * 1_000_000
    assert st["table_pruned"] > 0.99 * (st["pairs"] - st["seed_pairs"])
    Uw, Pw = O.widen(w.U), O.widen(w.P)
    unorm = np.sqrt(np.einsum("ij,ij->i", Uw, Uw))
    rng = np.random.default_rng(3)
    for i in (0, 137):
        a_ids, a_rk = ids[off[i]:off[i + 1]], rk[off[i]:off[i + 1]]
        assert len(set(a_ids.tolist())) == 100
        assert np.all(np.diff(a_rk) >= 0)
        h = (Uw @ O.widen(w.Qv[i])) / np.maximum(unorm, 1e-300)
        best = [u for u in np.argsort(-h)[:1700] if u not in set(a_ids.tolist())][:1500]
        rand = rng.choice(w.n, 1500, replace=False)
        sample = np.unique(np.concatenate([np.asarray(best, np.int64), rand]))
        bad_rank, bad_set, _ = O.certify(Uw, Pw, O.widen(w.Qv[i]), 100, a_ids, a_rk, check=sample)
        assert (bad_rank, bad_set) == (0, 0), i


def test_too_many_pairs_is_rejected():
    """Pair ids are 32-bit: a batch of 2^31 or more (user, query) pairs is
    refused before any work (2^21 users x 1,024 queries, d = 1)."""
    n, nq = 1 << 21, 1024
    U = torch.ones((n, 1), dtype=torch.float32, device="cuda")
    P = torch.ones((8, 1), dtype=torch.float32, device="cuda")
    idx = rkr.Index(U, P, score="f32")
    Q = torch.ones((nq, 1), dtype=torch.float32, device="cuda")
    with pytest.raises(rkr.RkrError) as e:
        idx.query_batch(Q, [1] * nq)
    assert e.value.status == rkr.RKR_E_UNSUPPORTED
    idx.close()
