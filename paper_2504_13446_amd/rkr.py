"""Python binding of librkr (ctypes).  Argument marshalling only.

The module-level functions carry the C names (``rkr_build``, ``rkr_query_exact``,
``rkr_query_approx``, ``rkr_query_batch``, ``rkr_ranks``, ...); they take torch
tensors for device memory and use torch's current stream.  ``Index`` wraps a
handle with the same calls as methods.

There is no CPU fallback: if librkr.so is missing or no GPU is visible, every
call raises.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "librkr.so")

RKR_OK, RKR_E_INVALID, RKR_E_NOMEM, RKR_E_DEVICE, RKR_E_UNSUPPORTED, RKR_E_STATE = range(6)
RKR_F32, RKR_BF16 = 0, 1
RKR_SCORE_F32, RKR_SCORE_BF16, RKR_SCORE_FP8, RKR_SCORE_BF16X3 = 0, 1, 2, 3
SCORES = {"f32": RKR_SCORE_F32, "bf16": RKR_SCORE_BF16, "fp8": RKR_SCORE_FP8, "bf16x3": RKR_SCORE_BF16X3}
MLP_NPARAM = 64 * 18 + 64 + 64 * 64 + 64 + 64 + 1
TABLE_COLS = 48   # RKR_TABLE_COLS of include/rkr.h
SYMBOLS = ("rkr_build", "rkr_destroy", "rkr_configure", "rkr_query_exact", "rkr_query_approx",
           "rkr_query_table", "rkr_query_table_batch", "rkr_paper_table_build", "rkr_paper_table",
           "rkr_query_paper_table", "rkr_query_paper_table_batch", "rkr_query_batch", "rkr_ranks", "rkr_ranks_noalloc", "rkr_score_error", "rkr_score_error_at", "rkr_train", "rkr_predict", "rkr_mlp_get", "rkr_mlp_set",
           "rkr_mlp_grad", "rkr_mlp_adam", "rkr_sketch", "rkr_rank_table", "rkr_stats", "rkr_last_error")


class RkrError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"rkr status {status}: {message}")
        self.status = status
        self.message = message


class BuildOpts(ctypes.Structure):
    _fields_ = [("score", ctypes.c_int32), ("recheck", ctypes.c_int32),
                ("sketch_samples", ctypes.c_int32), ("rank_table", ctypes.c_int32),
                ("stream", ctypes.c_void_p)]


class QueryOpts(ctypes.Structure):
    _fields_ = [("seed_mult", ctypes.c_int32), ("use_estimator", ctypes.c_int32),
                ("reserved0", ctypes.c_int32), ("prune_mult", ctypes.c_int32),
                ("graph", ctypes.c_int32), ("no_table", ctypes.c_int32), ("reserved", ctypes.c_int32 * 2)]


class QueryStats(ctypes.Structure):
    _fields_ = [(n, ctypes.c_int64) for n in (
        "queries", "pairs", "seed_pairs", "survivors", "refined_pairs", "uncertain", "flips",
        "compares", "emit_retries", "approx_settled")] + \
        [(n, ctypes.c_double) for n in ("ms_thresh", "ms_seed", "ms_screen", "ms_refine", "ms_select",
                                        "ms_total", "mlp_loss", "ms_screen_kernel", "ms_exact_kernel",
                                        "ms_recheck_kernel")] + [("screen_ctas", ctypes.c_int64),
                                                             ("screen_variant", ctypes.c_int64),
                                                             ("compare_slots", ctypes.c_int64),
                                                             ("graph_replays", ctypes.c_int64),
                                                             ("table_pruned", ctypes.c_int64),
                                                             ("mfma_flop", ctypes.c_int64),
                                                             ("scored_pairs", ctypes.c_int64),
                                                             ("persistent_phases", ctypes.c_int64),
                                                             ("ms_seed_kernel", ctypes.c_double),
                                                             ("scored_seed", ctypes.c_int64),
                                                             ("scored_exact", ctypes.c_int64)]

    def as_dict(self) -> dict:
        return {n: getattr(self, n) for n, _ in self._fields_}


_lib = None


def load(path: str = LIB_PATH):
    """Load librkr.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"librkr.so not found at {path}; run __graft_entry__.build() first")
    L = ctypes.CDLL(path)
    vp, i32, i64, f32, f64 = (ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_float,
                              ctypes.c_double)
    sig = {
        "rkr_build": [vp, i64, vp, i64, i32, ctypes.c_int, ctypes.POINTER(BuildOpts), ctypes.POINTER(vp)],
        "rkr_destroy": [vp],
        "rkr_configure": [vp, ctypes.POINTER(QueryOpts)],
        "rkr_query_exact": [vp, vp, i32, vp, vp],
        "rkr_query_approx": [vp, vp, i32, f64, vp, vp],
        "rkr_query_table": [vp, vp, i32, f64, vp, vp],
        "rkr_query_table_batch": [vp, i32, vp, vp, vp, vp, vp],
        "rkr_paper_table_build": [vp, i32, i32, i32, vp],
        "rkr_paper_table": [vp, vp, vp, vp],
        "rkr_query_paper_table": [vp, vp, i32, f64, vp, vp],
        "rkr_query_paper_table_batch": [vp, i32, vp, vp, vp, vp, vp],
        "rkr_query_batch": [vp, i32, vp, vp, vp, vp, vp, vp, vp],
        "rkr_ranks": [vp, vp, vp],
        "rkr_ranks_noalloc": [vp, vp, vp],
        "rkr_score_error": [vp, ctypes.POINTER(f64), ctypes.POINTER(ctypes.c_int64)],
        "rkr_score_error_at": [vp, vp, ctypes.POINTER(f64), ctypes.POINTER(ctypes.c_int64)],
        "rkr_train": [vp, i32, vp, i32, i32, i32, f32, ctypes.c_uint64],
        "rkr_predict": [vp, i32, vp, vp],
        "rkr_mlp_get": [vp, vp],
        "rkr_mlp_set": [vp, vp],
        "rkr_mlp_grad": [vp, vp, vp, i32, vp, ctypes.POINTER(f64)],
        "rkr_mlp_adam": [vp, vp, ctypes.c_float, i32, i32],
        "rkr_sketch": [vp, vp],
        "rkr_rank_table": [vp, vp, vp],
        "rkr_stats": [vp, ctypes.POINTER(QueryStats)],
        "rkr_last_error": [],
    }
    for name, args in sig.items():
        f = getattr(L, name)
        f.argtypes = args
        f.restype = ctypes.c_int if name not in ("rkr_destroy", "rkr_last_error") else None
    L.rkr_last_error.restype = ctypes.c_char_p
    _lib = L
    return L


def _check(status: int) -> None:
    if status != RKR_OK:
        msg = load().rkr_last_error()
        raise RkrError(status, msg.decode() if msg else "")


def _ptr(t) -> int | None:
    if t is None:
        return None
    if isinstance(t, torch.Tensor):
        if not t.is_cuda:
            raise ValueError("device tensor expected")
        if not t.is_contiguous():
            raise ValueError("contiguous tensor expected")
        return t.data_ptr()
    return t


def _stream() -> int:
    return torch.cuda.current_stream().cuda_stream


def _master(x: torch.Tensor) -> int:
    if x.dtype == torch.float32:
        return RKR_F32
    if x.dtype == torch.bfloat16:
        return RKR_BF16
    raise ValueError("master dtype must be float32 or bfloat16")


# ---------------------------------------------------------------------------
# C-named functions
# ---------------------------------------------------------------------------
def rkr_build(U: torch.Tensor, P: torch.Tensor, score: str = "bf16", recheck: bool = True,
              sketch_samples: int = 0, rank_table: int = 0) -> int:
    L = load()
    if U.dtype != P.dtype:
        raise ValueError("U and P must share a dtype")
    opts = BuildOpts(SCORES[score], 1 if recheck else 0, int(sketch_samples), int(rank_table), _stream())
    h = ctypes.c_void_p()
    n, d = U.shape
    m = P.shape[0]
    _check(L.rkr_build(_ptr(U), n, _ptr(P) if m > 0 else None, m, d, _master(U), ctypes.byref(opts),
                       ctypes.byref(h)))
    return h.value


def rkr_destroy(h: int) -> None:
    if h:
        load().rkr_destroy(h)


def rkr_configure(h: int, seed_mult: int = 0, use_estimator: bool = False,
                  prune_mult: int = 0, graph: bool = False, no_table: bool = False) -> None:
    o = QueryOpts(int(seed_mult), 1 if use_estimator else 0, 0, int(prune_mult),
                  1 if graph else 0, 1 if no_table else 0)
    _check(load().rkr_configure(h, ctypes.byref(o)))


def rkr_query_exact(h: int, q: torch.Tensor, k: int):
    ids = torch.empty(k, dtype=torch.int32, device=q.device)
    rk = torch.empty(k, dtype=torch.int32, device=q.device)
    _check(load().rkr_query_exact(h, _ptr(q), int(k), _ptr(ids), _ptr(rk)))
    return ids, rk


def rkr_query_approx(h: int, q: torch.Tensor, k: int, c: float):
    ids = torch.empty(k, dtype=torch.int32, device=q.device)
    rk = torch.empty(k, dtype=torch.int32, device=q.device)
    _check(load().rkr_query_approx(h, _ptr(q), int(k), float(c), _ptr(ids), _ptr(rk)))
    return ids, rk


def rkr_query_table(h: int, q: torch.Tensor, k: int, c: float):
    """The paper's table query (Sec. 4.3): (ids int32, est float64), device."""
    ids = torch.empty(k, dtype=torch.int32, device=q.device)
    est = torch.empty(k, dtype=torch.float64, device=q.device)
    _check(load().rkr_query_table(h, _ptr(q), int(k), float(c), _ptr(ids), _ptr(est)))
    return ids, est


def rkr_query_table_batch(h: int, Q: torch.Tensor, k, c):
    """The paper's table query for nq queries: (ids int32, est float64) on
    the device, concatenated by query, and the host offsets [nq + 1]."""
    nq = int(Q.shape[0])
    kk = np.ascontiguousarray(np.broadcast_to(np.asarray(k, np.int32), (nq,)))
    cc = np.ascontiguousarray(np.broadcast_to(np.asarray(c, np.float64), (nq,)))
    off = np.zeros(nq + 1, np.int64)
    off[1:] = np.cumsum(kk)
    ids = torch.empty(int(off[-1]), dtype=torch.int32, device=Q.device)
    est = torch.empty(int(off[-1]), dtype=torch.float64, device=Q.device)
    _check(load().rkr_query_table_batch(h, nq, _ptr(Q), kk.ctypes.data, cc.ctypes.data, _ptr(ids), _ptr(est)))
    return ids, est, off


def rkr_paper_table_build(h: int, tau: int, omega: int, s: int, sample_pos) -> None:
    """The paper's rank table (Alg. 1) in the index; sample_pos [omega * s]
    int32 positions within the buckets (host)."""
    pos = np.ascontiguousarray(np.asarray(sample_pos, np.int32).reshape(-1))
    assert pos.size == omega * s
    _check(load().rkr_paper_table_build(h, int(tau), int(omega), int(s), pos.ctypes.data))


def rkr_paper_table(h: int, n: int, tau: int, device="cuda"):
    """(f_min [n] float64, step [n] float64, cells [n, tau] float32) on the device."""
    fmin = torch.empty(n, dtype=torch.float64, device=device)
    step = torch.empty(n, dtype=torch.float64, device=device)
    cells = torch.empty((n, tau), dtype=torch.float32, device=device)
    _check(load().rkr_paper_table(h, _ptr(fmin), _ptr(step), _ptr(cells)))
    return fmin, step, cells


def rkr_query_paper_table_batch(h: int, Q: torch.Tensor, k, c):
    """The paper's query on its own table for nq queries: (ids int32, values
    float64) on the device, concatenated by query, and the host offsets."""
    nq = int(Q.shape[0])
    kk = np.ascontiguousarray(np.broadcast_to(np.asarray(k, np.int32), (nq,)))
    cc = np.ascontiguousarray(np.broadcast_to(np.asarray(c, np.float64), (nq,)))
    off = np.zeros(nq + 1, np.int64)
    off[1:] = np.cumsum(kk)
    ids = torch.empty(int(off[-1]), dtype=torch.int32, device=Q.device)
    val = torch.empty(int(off[-1]), dtype=torch.float64, device=Q.device)
    _check(load().rkr_query_paper_table_batch(h, nq, _ptr(Q), kk.ctypes.data, cc.ctypes.data, _ptr(ids), _ptr(val)))
    return ids, val, off


def rkr_query_paper_table(h: int, q: torch.Tensor, k: int, c: float):
    ids = torch.empty(k, dtype=torch.int32, device=q.device)
    val = torch.empty(k, dtype=torch.float64, device=q.device)
    _check(load().rkr_query_paper_table(h, _ptr(q), int(k), float(c), _ptr(ids), _ptr(val)))
    return ids, val


def rkr_query_batch(h: int, Q: torch.Tensor, k, c=None, cand_off=None, cand_ids=None):
    """Returns (ids, ranks, offsets): answers of query i are [offsets[i], offsets[i+1])."""
    nq = Q.shape[0]
    k = np.ascontiguousarray(np.broadcast_to(np.asarray(k, np.int32), (nq,)))
    off = np.zeros(nq + 1, np.int64)
    off[1:] = np.cumsum(k)
    ids = torch.empty(int(off[-1]), dtype=torch.int32, device=Q.device)
    rk = torch.empty(int(off[-1]), dtype=torch.int32, device=Q.device)
    cp = None
    if c is not None:
        c = np.ascontiguousarray(np.broadcast_to(np.asarray(c, np.float64), (nq,)))
        cp = c.ctypes.data
    co = None
    if cand_off is not None:
        cand_off = np.ascontiguousarray(np.asarray(cand_off, np.int64))
        co = cand_off.ctypes.data
    _check(load().rkr_query_batch(h, nq, _ptr(Q), k.ctypes.data, cp, co, _ptr(cand_ids), _ptr(ids),
                                  _ptr(rk)))
    return ids, rk, off


def rkr_ranks(h: int, q: torch.Tensor, n: int) -> torch.Tensor:
    out = torch.empty(n, dtype=torch.int32, device=q.device)
    _check(load().rkr_ranks(h, _ptr(q), _ptr(out)))
    return out


def rkr_score_error(h: int):
    """(largest |score - s64| / eps over every (user, item) pair, pairs above 1)."""
    r = ctypes.c_double()
    over = ctypes.c_int64()
    _check(load().rkr_score_error(h, ctypes.byref(r), ctypes.byref(over)))
    return r.value, over.value


def rkr_score_error_at(h: int, q: torch.Tensor):
    """The check in the threshold-folded form of the BF16 passes, thresholds of query q:
    (largest |acc - (s64 - th)| / bound, pairs above 1)."""
    r = ctypes.c_double()
    over = ctypes.c_int64()
    _check(load().rkr_score_error_at(h, _ptr(q), ctypes.byref(r), ctypes.byref(over)))
    return r.value, over.value


def rkr_ranks_noalloc(h: int, q: torch.Tensor, out: torch.Tensor) -> torch.Tensor:
    """rkr_ranks into a caller-provided int32 tensor, with no device allocation."""
    assert out.dtype == torch.int32 and out.is_contiguous()
    _check(load().rkr_ranks_noalloc(h, _ptr(q), _ptr(out)))
    return out


def rkr_train(h: int, Q: torch.Tensor, pairs_per_query: int = 4096, epochs: int = 4, batch: int = 4096,
              lr: float = 1e-3, seed: int = 0) -> None:
    _check(load().rkr_train(h, Q.shape[0], _ptr(Q), int(pairs_per_query), int(epochs), int(batch),
                            float(lr), int(seed)))


def rkr_predict(h: int, Q: torch.Tensor, n: int) -> torch.Tensor:
    out = torch.empty((Q.shape[0], n), dtype=torch.float32, device=Q.device)
    _check(load().rkr_predict(h, Q.shape[0], _ptr(Q), _ptr(out)))
    return out


def rkr_mlp_get(h: int) -> np.ndarray:
    out = np.empty(MLP_NPARAM, np.float32)
    _check(load().rkr_mlp_get(h, out.ctypes.data))
    return out


def rkr_mlp_set(h: int, params) -> None:
    p = np.ascontiguousarray(np.asarray(params, np.float32))
    assert p.size == MLP_NPARAM
    _check(load().rkr_mlp_set(h, p.ctypes.data))


def rkr_mlp_grad(h: int, X: torch.Tensor, z: torch.Tensor):
    g = torch.empty(MLP_NPARAM, dtype=torch.float32, device=X.device)
    loss = ctypes.c_double()
    _check(load().rkr_mlp_grad(h, _ptr(X), _ptr(z), X.shape[0], _ptr(g), ctypes.byref(loss)))
    return g, loss.value


def rkr_mlp_adam(h: int, grad: torch.Tensor, lr: float, step: int, reset: bool = False) -> None:
    assert grad.numel() == MLP_NPARAM and grad.dtype == torch.float32
    _check(load().rkr_mlp_adam(h, _ptr(grad), float(lr), int(step), 1 if reset else 0))


def rkr_sketch(h: int, n: int, device="cuda") -> torch.Tensor:
    out = torch.empty((n, 16), dtype=torch.float32, device=device)
    _check(load().rkr_sketch(h, _ptr(out)))
    return out


def rkr_rank_table(h: int, n: int, device="cuda"):
    """(thresholds [n, TABLE_COLS] float64, certain counts [n, TABLE_COLS] int32 holding uint32)."""
    t = torch.empty((n, TABLE_COLS), dtype=torch.float64, device=device)
    c = torch.empty((n, TABLE_COLS), dtype=torch.int32, device=device)
    _check(load().rkr_rank_table(h, _ptr(t), _ptr(c)))
    return t, c


def rkr_stats(h: int) -> dict:
    s = QueryStats()
    _check(load().rkr_stats(h, ctypes.byref(s)))
    return s.as_dict()


# ---------------------------------------------------------------------------
class Index:
    """An index over device tensors U [n, d] and P [m, d] (float32 or bfloat16)."""

    def __init__(self, U: torch.Tensor, P: torch.Tensor, score: str = "bf16", recheck: bool = True,
                 sketch_samples: int = 0, rank_table: int = 0):
        self.n, self.d = U.shape
        self.m = P.shape[0]
        self.device = U.device
        self.h = rkr_build(U, P, score=score, recheck=recheck, sketch_samples=sketch_samples,
                           rank_table=rank_table)

    def close(self) -> None:
        if getattr(self, "h", None):
            rkr_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def configure(self, **kw) -> None:
        rkr_configure(self.h, **kw)

    def query_exact(self, q, k):
        return rkr_query_exact(self.h, q, k)

    def query_approx(self, q, k, c):
        return rkr_query_approx(self.h, q, k, c)

    def query_table(self, q, k, c):
        return rkr_query_table(self.h, q, k, c)

    def query_table_batch(self, Q, k, c):
        return rkr_query_table_batch(self.h, Q, k, c)

    def paper_table_build(self, tau, omega, s, sample_pos):
        rkr_paper_table_build(self.h, tau, omega, s, sample_pos)
        self.paper_tau = int(tau)

    def paper_table(self):
        return rkr_paper_table(self.h, self.n, self.paper_tau)

    def query_paper_table(self, q, k, c):
        return rkr_query_paper_table(self.h, q, k, c)

    def query_paper_table_batch(self, Q, k, c):
        return rkr_query_paper_table_batch(self.h, Q, k, c)

    def query_batch(self, Q, k, c=None, cand_off=None, cand_ids=None):
        return rkr_query_batch(self.h, Q, k, c, cand_off, cand_ids)

    def score_error(self):
        return rkr_score_error(self.h)

    def score_error_at(self, q):
        return rkr_score_error_at(self.h, q)

    def ranks(self, q):
        return rkr_ranks(self.h, q, self.n)

    def train(self, Q, **kw):
        return rkr_train(self.h, Q, **kw)

    def predict(self, Q):
        return rkr_predict(self.h, Q, self.n)

    def sketch(self):
        return rkr_sketch(self.h, self.n, self.device)

    def rank_table(self):
        return rkr_rank_table(self.h, self.n, self.device)

    def stats(self) -> dict:
        return rkr_stats(self.h)


def to_device(x: np.ndarray, dtype: str, device="cuda") -> torch.Tensor:
    """Master array (float32, or bfloat16 as uint16 bits) -> device tensor."""
    x = np.ascontiguousarray(x)
    if dtype == "bf16":
        return torch.from_numpy(x.view(np.int16)).view(torch.bfloat16).to(device)
    return torch.from_numpy(x.astype(np.float32, copy=False)).to(device)
