"""GPU tests of the learned rank estimator against the FP64 references."""
import numpy as np
import pytest
import torch

from oracle import mlp as M
from oracle import oracle as O
from paper_2504_13446_amd import rkr, workloads as W

pytestmark = pytest.mark.gpu


def _dev(x, dtype):
    return rkr.to_device(x, dtype)


def _rand_params(seed, scale=1.0):
    rng = np.random.default_rng(seed)
    p = {}
    for k in M.ORDER:
        fan = M.SHAPES[k][-1] if len(M.SHAPES[k]) == 2 else 64
        p[k] = rng.standard_normal(M.SHAPES[k]) * scale / np.sqrt(fan)
    p["b3"][0] = 3.0
    return p


@pytest.fixture(scope="module")
def lowrank():
    w = W.make("single", n=3000, m=4000, nq=24)
    idx = rkr.Index(_dev(w.U, "f32"), _dev(w.P, "f32"), score="bf16", sketch_samples=512)
    yield w, idx
    idx.close()


def test_sketch_bit_exact(lowrank):
    w, idx = lowrank
    got = idx.sketch().cpu().numpy()
    S = 512
    want = O.sketch(w.U, w.P, O.stratified_sample(w.P, S), O.sketch_positions(S)).astype(np.float32)
    assert np.array_equal(got, want), np.argwhere(got != want)[:5]


def _away_from_kinks(p, X, margin=1e-4):
    """Rows whose hidden pre-activations are farther than `margin` times their
    absolute sums from 0: there the ReLU masks of an FP32 and an FP64 forward
    pass provably agree (FP32 rounding moves a pre-activation by far less than
    1e-4 of its absolute sum), so the gradient is continuous and comparable."""
    a1 = X @ p["W1"].T + p["b1"]
    s1 = np.abs(X) @ np.abs(p["W1"]).T + np.abs(p["b1"])
    h1 = np.maximum(a1, 0)
    a2 = h1 @ p["W2"].T + p["b2"]
    s2 = np.abs(h1) @ np.abs(p["W2"]).T + np.abs(p["b2"])
    ok = np.all(np.abs(a1) > margin * s1, axis=1) & np.all(np.abs(a2) > margin * s2, axis=1)
    return ok


def test_gradient_matches_fp64_reference(lowrank):
    w, idx = lowrank
    p = _rand_params(1)
    flat = M.flatten(p).astype(np.float32)
    rkr.rkr_mlp_set(idx.h, flat)
    p32 = M.unflatten(flat.astype(np.float64))       # the parameters as the GPU holds them
    rng = np.random.default_rng(2)
    X = rng.standard_normal((1200, 18)).astype(np.float32)
    X = X[_away_from_kinks(p32, X.astype(np.float64))][:777]   # several 64-sample blocks + a ragged tail
    N = X.shape[0]
    assert N == 777
    z = rng.uniform(0, 12, N).astype(np.float32)
    g, loss = rkr.rkr_mlp_grad(idx.h, torch.from_numpy(X).cuda(), torch.from_numpy(z).cuda())
    g = g.cpu().numpy().astype(np.float64)
    L, gr = M.loss_and_grad(p32, X.astype(np.float64), z.astype(np.float64))
    assert loss == pytest.approx(L, rel=1e-5)
    ref = M.flatten(gr)
    o = 0
    for k in M.ORDER:
        sz = int(np.prod(M.SHAPES[k]))
        a, b = g[o:o + sz], ref[o:o + sz]
        o += sz
        assert np.linalg.norm(a - b) <= 1e-4 * max(np.linalg.norm(b), 1e-12), k


def _abs_forward(p, X):
    a1 = np.abs(X) @ np.abs(p["W1"]).T + np.abs(p["b1"])
    a2 = a1 @ np.abs(p["W2"]).T + np.abs(p["b2"])
    return a2 @ np.abs(p["w3"]) + abs(p["b3"][0])


def test_bf16_inference_within_rounding_bound(lowrank):
    """BF16 inference vs the FP64 forward on the same features.  Rounding the
    inputs, weights and hidden activations to BF16 (relative 2^-9 each) and
    accumulating in FP32 moves each layer's pre-activation by at most about
    2^-8 of its absolute sum; ReLU is 1-Lipschitz, so over three layers
    |y_bf16 - y| <= 4 * 2^-8 * y_abs, y_abs being the forward pass of |W|, |b|, |x|."""
    w, idx = lowrank
    p = _rand_params(3)
    flat = M.flatten(p).astype(np.float32)
    rkr.rkr_mlp_set(idx.h, flat)
    p32 = M.unflatten(flat.astype(np.float64))
    Q = w.Qv[:5]
    got = idx.predict(_dev(Q, "f32")).cpu().numpy()        # [5, n]
    T = O.dots(w.U, Q)                                        # spec t(u,q), [n, 5]
    nu = O.norms(w.U)
    sk = idx.sketch().cpu().numpy().astype(np.float64)
    for qi in range(Q.shape[0]):
        X = np.concatenate([(T[:, qi] / nu).astype(np.float32)[:, None].astype(np.float64),
                            nu.astype(np.float32)[:, None].astype(np.float64), sk], axis=1)
        y, _ = M.forward(p32, X)
        tol = 4 * 2.0 ** -8 * _abs_forward(p32, X)
        err = np.abs(got[qi] - y)
        assert np.all(err <= tol), (qi, err.max(), tol[np.argmax(err)])


def test_training_and_exactness_with_estimator(lowrank):
    w, idx = lowrank
    Qtr = _dev(w.Qv[:16], "f32")
    idx.train(Qtr, pairs_per_query=512, epochs=30, batch=256, lr=3e-3, seed=5)
    st = idx.stats()
    n_train = st["pairs"]
    assert n_train >= 16 * 400
    # the fitted loss is well below the variance of ln r (the loss of the best constant)
    Rtr = O.ranks(w.U, w.P, w.Qv[:16])
    var = np.var(np.log(Rtr.astype(np.float64)))
    assert st["mlp_loss"] < 0.5 * var, (st["mlp_loss"], var)
    # exact answers stay exact when the estimator picks the seeds
    Qte = w.Qv[16:]
    R = O.ranks(w.U, w.P, Qte)
    ks = np.full(Qte.shape[0], 25, np.int32)
    idx.configure(use_estimator=False)
    a0 = idx.query_batch(_dev(Qte, "f32"), ks)
    s0 = idx.stats()
    idx.configure(use_estimator=True)
    a1 = idx.query_batch(_dev(Qte, "f32"), ks)
    s1 = idx.stats()
    for (ids, rk, off) in (a0, a1):
        ids = ids.cpu().numpy(); rk = rk.cpu().numpy()
        for i in range(Qte.shape[0]):
            wi, wr = O.topk(R[i], 25)
            assert np.array_equal(ids[off[i]:off[i + 1]], wi) and np.array_equal(rk[off[i]:off[i + 1]], wr)
    print("compares without / with estimator:", s0["compares"], s1["compares"],
          "survivors:", s0["survivors"], s1["survivors"])
    # approximate mode, verified by the screen: zero Def. 3 violations
    ids, rk, off = idx.query_batch(_dev(Qte, "f32"), ks, c=1.5)
    ids = ids.cpu().numpy()
    for i in range(Qte.shape[0]):
        _, wr = O.topk(R[i], 25)
        assert O.def3_check(R[i][ids[off[i]:off[i + 1]]], wr, 1.5)[0] == 0
    # approximate mode pruned by the estimator: the returned ranks are exact
    idx.configure(use_estimator=True, prune_mult=4)
    ids, rk, off = idx.query_batch(_dev(Qte, "f32"), ks, c=1.5)
    ids = ids.cpu().numpy(); rk = rk.cpu().numpy()
    for i in range(Qte.shape[0]):
        g = ids[off[i]:off[i + 1]]
        assert np.array_equal(rk[off[i]:off[i + 1]], R[i][g])
    idx.configure(use_estimator=False, prune_mult=0)


def test_estimator_gain_when_pruning():
    """What the trained network buys: with the candidate budget cut to exactly
    k users per query (approximate mode, no verifying screen), the users the
    estimator picks hold more of the exact answer (recall) than the users of
    best u.q/|u|, and break Def. 3 (c = 1.5) less often."""
    w = W.make("single", n=20000, m=4000, nq=48)
    idx = rkr.Index(_dev(w.U, "f32"), _dev(w.P, "f32"), score="bf16", sketch_samples=1024)
    idx.train(_dev(w.Qv[:32], "f32"), pairs_per_query=2048, epochs=20, batch=512, lr=2e-3, seed=11)
    Qte = w.Qv[32:]
    R = O.ranks(w.U, w.P, Qte)
    k = 50
    ks = np.full(Qte.shape[0], k, np.int32)
    res = {}
    for use in (True, False):
        idx.configure(use_estimator=use, prune_mult=1)
        ids, rk, off = idx.query_batch(_dev(Qte, "f32"), ks, c=1.5)
        ids = ids.cpu().numpy()
        rec, viol = [], 0
        for i in range(Qte.shape[0]):
            g = ids[off[i]:off[i + 1]]
            wi, wr = O.topk(R[i], k)
            rec.append(len(set(g.tolist()) & set(wi.tolist())) / k)
            viol += O.def3_check(R[i][g], wr, 1.5)[0]
        res[use] = (float(np.mean(rec)), viol)
    print("budget k: recall / Def.3 violations  estimator:", res[True], " u.q/|u|:", res[False])
    assert res[True][0] > res[False][0]
    assert res[True][1] <= res[False][1]
    idx.close()


def test_adam_steps_match_fp64_reference(lowrank):
    """Six Adam steps of the library's kernel from fixed FP32 gradients against
    the FP64 Adam of the oracle from the same start.  The kernel computes in
    FP32: each step moves a parameter by lr * m_hat / (sqrt(v_hat) + eps),
    with a few FP32 roundings (relative 2^-24 each) in that update and one
    in the parameter, so the parameters agree to 1e-6 of each tensor's norm
    and the accumulated updates to 1e-5 of theirs."""
    w, idx = lowrank
    p0 = _rand_params(9)
    flat0 = M.flatten(p0).astype(np.float32)
    rkr.rkr_mlp_set(idx.h, flat0)
    ref = M.unflatten(flat0.astype(np.float64))
    start = M.unflatten(flat0.astype(np.float64))
    mom = {k: np.zeros(M.SHAPES[k]) for k in M.ORDER}
    vel = {k: np.zeros(M.SHAPES[k]) for k in M.ORDER}
    rng = np.random.default_rng(12)
    lr = 1e-2
    for t in range(1, 7):
        g = (rng.standard_normal(M.n_params()) * rng.choice([1e-3, 1e-1, 1.0], M.n_params())).astype(np.float32)
        rkr.rkr_mlp_adam(idx.h, torch.from_numpy(g).cuda(), lr, t, reset=(t == 1))
        M.adam_step(ref, M.unflatten(g.astype(np.float64)), mom, vel, t, lr)
    got = M.unflatten(rkr.rkr_mlp_get(idx.h).astype(np.float64))
    for k in M.ORDER:
        a, b, s = got[k], ref[k], start[k]
        assert np.linalg.norm(a - b) <= 1e-6 * np.linalg.norm(b), k
        assert np.linalg.norm((a - s) - (b - s)) <= 1e-5 * np.linalg.norm(b - s), k
    with pytest.raises(rkr.RkrError) as e:
        rkr.rkr_mlp_adam(idx.h, torch.zeros(M.n_params(), device="cuda"), lr, 0)
    assert e.value.status == rkr.RKR_E_INVALID
