"""The seeded generators: determinism, shapes, dtype handling, candidate lists."""
import numpy as np
import torch

from paper_2504_13446_amd import workloads as W


def test_small_shapes_and_determinism():
    a = W.make("small")
    b = W.make("small")
    assert a.U.shape == (2000, 50) and a.P.shape == (5000, 50) and a.Qv.shape == (10, 50)
    assert a.U.dtype == np.float32
    assert np.array_equal(a.U, b.U) and np.array_equal(a.P, b.P)
    assert np.array_equal(a.Qv, a.P[a.qidx])
    assert len(set(a.qidx.tolist())) == 10
    assert a.k.tolist() == [10] * 10
    nrm = np.linalg.norm(a.P.astype(np.float64), axis=1)
    # log-norms ~ N(0, 0.5^2)
    assert abs(np.log(nrm).mean()) < 0.05 and abs(np.log(nrm).std() - 0.5) < 0.05


def test_bf16_rounding_matches_torch():
    rng = np.random.default_rng(0)
    x = (rng.standard_normal(100000) * np.exp(rng.uniform(-20, 20, 100000))).astype(np.float32)
    x[:4] = [1.0 + 2 ** -8, 1.0 + 3 * 2 ** -8, -1.0 - 2 ** -8, 0.0]   # exact ties
    ours = W.f32_to_bf16_bits(x)
    ref = torch.from_numpy(x).to(torch.bfloat16).view(torch.int16).numpy().view(np.uint16)
    assert np.array_equal(ours, ref)
    assert np.array_equal(W.bf16_bits_to_f32(ours), torch.from_numpy(x).to(torch.bfloat16).float().numpy())


def test_scaled_batch_is_bf16():
    w = W.make("batch", n=3000, m=2000, nq=8)
    assert w.U.dtype == np.uint16 and w.U.shape == (3000, 200)
    assert np.array_equal(w.Qv, w.P[w.qidx])


def test_lowrank_single():
    w = W.make("single", n=500, m=700)
    f = W.bf16_bits_to_f32 if w.dtype == "bf16" else np.asarray
    X = np.asarray(f(w.U), np.float64)
    s = np.linalg.svd(X - 0, compute_uv=False)
    # 20 strong directions, the rest is 0.1-scale noise
    assert s[19] > 3 * s[20]


def test_uneven_candidate_lists():
    w = W.make("uneven", n=20000, m=3000, nq=64, cand=(100, 5000))
    off, ids = w.cand_off, w.cand_ids
    assert off.shape == (65,) and off[0] == 0
    sizes = np.diff(off)
    assert sizes.min() >= 100 and sizes.max() <= 5000
    for i in range(64):
        lst = ids[off[i]:off[i + 1]]
        assert np.all(np.diff(lst) > 0) and lst.min() >= 0 and lst.max() < 20000
    assert set(np.unique(w.k).tolist()) <= {10, 50, 100}
    assert w.c == 1.5
