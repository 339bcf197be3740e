"""GPU: rkr_ranks_noalloc, the all-ranks entry point that allocates nothing.

Its output must equal rkr_ranks's (the allocating entry point, itself checked
against the oracle) bit for bit: on two calls in a row, the second on a
smaller index, on a case whose near ties overflow the scratch array (the
call then counts the users in smaller chunks), and it must refuse sizes
beyond its limits.  Device memory free before and after a call is the same.
"""
import numpy as np
import pytest
import torch

from paper_2504_13446_amd import rkr, workloads as W

pytestmark = pytest.mark.gpu


def _dev(x, dtype):
    return rkr.to_device(x, dtype)


def _both(idx, q, n):
    want = idx.ranks(q).cpu().numpy()
    out = torch.full((n,), -7, dtype=torch.int32, device="cuda")
    torch.cuda.synchronize()
    free0 = torch.cuda.mem_get_info()[0]
    rkr.rkr_ranks_noalloc(idx.h, q, out)
    torch.cuda.synchronize()
    free1 = torch.cuda.mem_get_info()[0]
    return want, out.cpu().numpy(), free0, free1


@pytest.mark.parametrize("score", ["bf16", "f32"])
def test_noalloc_equals_ranks_twice_second_smaller(score):
    big = W.make("single", n=30_000, m=20_000, nq=2)
    small = W.make("small", n=5_000, m=7_000, nq=2)
    for w in (big, small):
        idx = rkr.Index(_dev(w.U, w.dtype), _dev(w.P, w.dtype), score=score)
        for i in range(2):
            want, got, free0, free1 = _both(idx, _dev(w.Qv[i], w.dtype), w.n)
            assert np.array_equal(got, want), (w.name, i, np.flatnonzero(got != want)[:10])
            assert free1 == free0, (w.name, i, free0 - free1)
        idx.close()


def test_noalloc_near_tie_overflow_is_counted_in_chunks():
    """Entries in {-1, 0, 1}, d = 3: a quarter of the items tie with the query
    for every user, tens of millions of near ties in all, far more than the
    scratch array holds at once."""
    rng = np.random.default_rng(29)
    U = rng.integers(-1, 2, size=(20_000, 3)).astype(np.float32)
    P = rng.integers(-1, 2, size=(8_000, 3)).astype(np.float32)
    idx = rkr.Index(_dev(U, "f32"), _dev(P, "f32"), score="bf16")
    want, got, _, _ = _both(idx, _dev(P[5].copy(), "f32"), U.shape[0])
    st = idx.stats()
    idx.close()
    assert st["emit_retries"] >= 1, st
    assert np.array_equal(got, want)


def test_noalloc_refuses_sizes_beyond_its_limit():
    n = (1 << 20) + 1
    U = torch.ones((n, 1), dtype=torch.float32, device="cuda")
    P = torch.ones((4, 1), dtype=torch.float32, device="cuda")
    idx = rkr.Index(U, P, score="f32")
    out = torch.empty(n, dtype=torch.int32, device="cuda")
    with pytest.raises(rkr.RkrError) as e:
        rkr.rkr_ranks_noalloc(idx.h, P[0], out)
    assert e.value.status == rkr.RKR_E_UNSUPPORTED
    idx.close()
