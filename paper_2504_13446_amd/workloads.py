"""Seeded synthetic workloads shaped like the paper's experiments.

This module only draws inputs; it holds none of the method's arithmetic.  The
paper evaluates on matrix-factorisation embeddings of three rating datasets
with d = 200 and 1,000 random items of P as queries (Sec. 5).  Those datasets
are not available, so every workload here is synthetic:

* ``iid``       -- each vector has a N(0, I) direction, normalised, then scaled
                   to a norm rho ~ LogNormal(0, 0.5) (the paper shows roughly
                   bell-shaped norm histograms, Sec. 4.2 Fig. 2);
* ``lowrank``   -- v = B z + 0.1 xi with a shared basis B in R^{d x 20}
                   (entries N(0, 1/20)), z ~ N(0, I_20), xi ~ N(0, I_d), then
                   rescaled to a LogNormal(0, 0.5) norm (users and items share
                   B, as matrix factorisation embeddings do).

Queries are rows of P drawn uniformly without replacement (Sec. 5 uses items
of P as queries), passed as vectors in the master dtype.

Masters are float32, or bfloat16 held as uint16 bit patterns (round to
nearest even from float32).  Generation runs in float64, in row chunks.

The named workloads (``WORKLOADS``):

  small    n=2,000    m=5,000     d=50   iid     f32   10 queries  k=10
  single   n=100,000  m=100,000   d=100  lowrank f32    1 query    k=50
  batch    n=1M       m=1M        d=200  iid     bf16 256 queries  k=100
  uneven   n=500,000  m=1M        d=300  iid     f32 1,024 queries k in {10,50,100},
           candidate lists of 1k..200k users (log-uniform sizes), c=1.5
  learned  n=1M       m=1M        d=200  iid     bf16 1,024 queries k=100, c=1.5

Every draw uses numpy's PCG64 seeded from ``13446 + index`` (index 1..5 in
the order above) with independent spawned streams for U, P, queries, k and
candidate lists, so any scaled-down variant is reproducible.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

WORKLOADS = {
    "small":   dict(index=1, n=2_000, m=5_000, d=50, gen="iid", dtype="f32", nq=10, k=10),
    "single":  dict(index=2, n=100_000, m=100_000, d=100, gen="lowrank", dtype="f32", nq=1, k=50),
    "batch":   dict(index=3, n=1_000_000, m=1_000_000, d=200, gen="iid", dtype="bf16", nq=256,
                    k=100),
    "uneven":  dict(index=4, n=500_000, m=1_000_000, d=300, gen="iid", dtype="f32", nq=1024,
                    k=(10, 50, 100), c=1.5, cand=(1_000, 200_000)),
    "learned": dict(index=5, n=1_000_000, m=1_000_000, d=200, gen="iid", dtype="bf16", nq=1024,
                    k=100, c=1.5),
}

_CHUNK = 1 << 16


def f32_to_bf16_bits(x) -> np.ndarray:
    """Round float32 to bfloat16 (nearest, ties to even); returns uint16 bits."""
    b = np.ascontiguousarray(np.asarray(x, np.float32)).view(np.uint32)
    r = (b + np.uint32(0x7FFF) + ((b >> np.uint32(16)) & np.uint32(1))) >> np.uint32(16)
    return r.astype(np.uint16)


def bf16_bits_to_f32(b) -> np.ndarray:
    return (np.asarray(b, np.uint16).astype(np.uint32) << np.uint32(16)).view(np.float32)


def _vectors(rng, rows: int, d: int, gen: str, basis) -> np.ndarray:
    """float64 [rows][d] with the workload's direction and norm law."""
    if gen == "iid":
        v = rng.standard_normal((rows, d))
    elif gen == "lowrank":
        z = rng.standard_normal((rows, basis.shape[1]))
        v = z @ basis.T + 0.1 * rng.standard_normal((rows, d))
    else:
        raise ValueError(gen)
    nrm = np.sqrt(np.einsum("ij,ij->i", v, v))
    nrm[nrm == 0] = 1.0
    rho = rng.lognormal(mean=0.0, sigma=0.5, size=rows)
    return v * (rho / nrm)[:, None]


def _matrix(rng, rows: int, d: int, gen: str, basis, dtype: str) -> np.ndarray:
    out = np.empty((rows, d), np.uint16 if dtype == "bf16" else np.float32)
    for s in range(0, rows, _CHUNK):
        e = min(rows, s + _CHUNK)
        v = _vectors(rng, e - s, d, gen, basis).astype(np.float32)
        out[s:e] = f32_to_bf16_bits(v) if dtype == "bf16" else v
    return out


@dataclass
class Workload:
    name: str
    n: int
    m: int
    d: int
    dtype: str                      # "f32" or "bf16" (uint16 bit patterns)
    U: np.ndarray
    P: np.ndarray
    qidx: np.ndarray                # query rows of P
    Qv: np.ndarray                  # query vectors, master dtype [nq][d]
    k: np.ndarray                   # int32 [nq]
    c: float | None = None
    cand_off: np.ndarray | None = None   # int64 [nq+1] CSR offsets, or None (all users)
    cand_ids: np.ndarray | None = None   # int32 user ids, sorted within each list
    extra: dict = field(default_factory=dict)

    @property
    def nq(self) -> int:
        return int(self.Qv.shape[0])


def make(name: str, n: int | None = None, m: int | None = None, d: int | None = None,
         nq: int | None = None, dtype: str | None = None, gen: str | None = None,
         cand: tuple | None = None, k=None) -> Workload:
    """Draw a named workload, optionally scaled down (same law, same seeds)."""
    spec = dict(WORKLOADS[name])
    n = spec["n"] if n is None else int(n)
    m = spec["m"] if m is None else int(m)
    d = spec["d"] if d is None else int(d)
    nq = spec["nq"] if nq is None else int(nq)
    dtype = spec["dtype"] if dtype is None else dtype
    gen = spec["gen"] if gen is None else gen
    ss = np.random.SeedSequence(13446 + spec["index"])
    s_basis, s_u, s_p, s_q, s_k, s_c = ss.spawn(6)
    basis = None
    if gen == "lowrank":
        basis = np.random.default_rng(s_basis).normal(0.0, np.sqrt(1.0 / 20), size=(d, 20))
    U = _matrix(np.random.default_rng(s_u), n, d, gen, basis, dtype)
    P = _matrix(np.random.default_rng(s_p), m, d, gen, basis, dtype)
    nq = min(nq, m)
    qidx = np.random.default_rng(s_q).choice(m, size=nq, replace=False).astype(np.int64)
    Qv = np.ascontiguousarray(P[qidx])
    kspec = spec["k"] if k is None else k
    if isinstance(kspec, tuple):
        kk = np.random.default_rng(s_k).choice(np.asarray(kspec), size=nq).astype(np.int32)
    else:
        kk = np.full(nq, int(kspec), np.int32)
    cand_off = cand_ids = None
    cspec = spec.get("cand") if cand is None else cand
    if cspec is not None:
        lo, hi = cspec
        hi = min(hi, n)
        lo = min(lo, hi)
        rng = np.random.default_rng(s_c)
        sizes = np.floor(np.exp(rng.uniform(np.log(lo), np.log(hi), size=nq))).astype(np.int64)
        sizes = np.clip(sizes, 1, n)
        cand_off = np.zeros(nq + 1, np.int64)
        cand_off[1:] = np.cumsum(sizes)
        cand_ids = np.empty(int(cand_off[-1]), np.int32)
        for i in range(nq):
            ids = rng.choice(n, size=int(sizes[i]), replace=False)
            cand_ids[cand_off[i]:cand_off[i + 1]] = np.sort(ids)
        kk = np.minimum(kk, sizes.astype(np.int32))
    return Workload(name=name, n=n, m=m, d=d, dtype=dtype, U=U, P=P, qidx=qidx, Qv=Qv, k=kk,
                    c=spec.get("c"), cand_off=cand_off, cand_ids=cand_ids)


def bucket_sample_positions(m: int, omega: int, s: int, seed: int = 13446) -> np.ndarray:
    """Random draws of the paper's sampling (Sec. 4.2, Alg. 1): for each of the
    omega buckets of a partition of m items into equal parts (bucket l holds
    floor((l + 1) m / omega) - floor(l m / omega) items), s distinct positions
    within the bucket, uniform without replacement (all of them, in order,
    when the bucket holds s or fewer; the remaining slots are -1).  int32
    [omega * s]."""
    rng = np.random.default_rng(np.random.SeedSequence([seed, m, omega, s]))
    out = np.full(omega * s, -1, np.int32)
    for l in range(omega):
        size = (l + 1) * m // omega - l * m // omega
        if size <= s:
            out[l * s:l * s + size] = np.arange(size, dtype=np.int32)
        else:
            out[l * s:(l + 1) * s] = rng.choice(size, size=s, replace=False).astype(np.int32)
    return out


def extra_queries(w: Workload, nq: int, seed: int = 1) -> np.ndarray:
    """nq more query vectors: rows of P drawn uniformly without replacement
    from the rows that are not w's queries (e.g. training queries for the
    rank estimator, disjoint from the test queries).  Master dtype [nq][d]."""
    rng = np.random.default_rng(np.random.SeedSequence([13446, seed, w.m, nq]))
    rest = np.setdiff1d(np.arange(w.m, dtype=np.int64), w.qidx)
    pick = rng.choice(rest, size=min(nq, rest.size), replace=False)
    return np.ascontiguousarray(w.P[pick])
