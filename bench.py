#!/usr/bin/env python3
"""Benchmark of the batched exact reverse k-ranks path on one MI355X.

A step is one rkr_query_batch call: 256 queries over |U| = |P| = 1,000,000,
d = 200, BF16 masters, k = 100, exact answers (Def. 2), all of the hot path
(thresholds, seeds, rank-table filter, screening count, refine with FP64
near-tie recheck, top-k).  Inputs are synthetic (seeded, see workloads.py) and
resident in HBM before the timed region; the index (with its rank table) is
built once, outside it, and its build time is reported.

Printed (one JSON line on stdout):
  value         queries/s of the BF16 + recheck path (exact)
  gcompare_per_s dense-equivalent rank comparisons per second (n * m * Q / t);
                gcompare_per_s_executed, the compares the kernels executed
  roofline      the dominant launch, the exact-mode count kernel (the seed
                pass and the refine pass of a step): algorithmic flop (2 d per
                (user, item) score of a user with a live pair, d unpadded,
                counted by the kernel) over its HIP-event durations, against
                the BF16 dense peak; the seed pass alone; every count launch
                of a step, by algorithmic and by executed (padded) flop; HBM
                bytes per launch from the committed counter record while the
                kernel sources match it; the compare-loop view beside it
  approx_c1_5   the same batch in approximate mode (Def. 3, c = 1.5): time,
                the Sec. 5 accuracy and overall ratio, Def. 3 violations
  paper_table_query  the paper's own method for the whole batch, c = 1.5:
                Alg. 1's table (tau = 500, omega = s = 64) built on the GPU
                and the query of Sec. 4.3 on it: build and query time, the
                Sec. 5 accuracy and overall ratio against the exact answers
  table_query   the same query on the index's exact-cell table
  without_rank_table  the same batch with the table switched off
  fp32_plain    the same pipeline (rank table, seeds) with FP32 scores and a
                plain compare (no band, no recheck), 3 timed steps, and the
                speed-up over it; the pair without the rank table beside it
  cpu_baseline  the CPU oracle on a bounded sample of users (all queries),
                scaled to queries/s
  single_all_ranks  secondary: exact ranks of all 100k users for one query on
                the single-query workload (graph replays), BF16 + recheck and
                plain FP32
  uneven, learned  the other batched workloads, each run as a child process
                with its own line embedded: 500k x 1M x 300 with 1,024 uneven
                candidate lists (c = 1.5 and exact), and 1M x 1M x 200 with
                1,024 queries and the rank estimator trained on 10M triples
                (c = 1.5 and exact, with and without the estimator)
Progress goes to stderr.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_TFLOPS = {"bf16": 2500.0, "bf16x3": 2500.0, "fp8": 5000.0, "f32": 157.3}
ALU_PEAK_TOPS = 256 * 4 * 16 * 2.4e9 / 1e12     # 32-bit vector lane-ops/s (39.3 T)
TRAFFIC = os.path.join(ROOT, "profiles", "k_count_exact_batch_1M_traffic.json")


def code_digest(path: str) -> str:
    """SHA-256 of a C++/HIP source with its // comments and blank lines
    removed: edits to comments do not invalidate a counter record."""
    import hashlib
    lines = []
    for ln in open(path, encoding="utf-8"):
        ln = ln.split("//", 1)[0].rstrip()
        if ln:
            lines.append(ln)
    return hashlib.sha256("\n".join(lines).encode()).hexdigest()


def exact_traffic(key: dict):
    """HBM bytes per launch of the exact-mode count kernel from the committed
    counter record, or None when the workload or the kernel sources differ
    from the ones the counters were read on."""
    try:
        rec = json.load(open(TRAFFIC))
        if rec["workload_key"] != key:
            return None
        for path, digest in rec["sources_sha256"].items():
            if code_digest(os.path.join(ROOT, path)) != digest:
                return None
        return rec["hbm_bytes_per_launch"]
    except (OSError, KeyError, ValueError):
        return None


METRIC = "queries/s + Gcompare/s at |U|=|P|=1M,d=200, exact top-k; BF16+recheck vs FP32 plain"


def log(msg: str) -> None:
    sys.stderr.write("[bench %.1fs] %s\n" % (time.time() - T0, msg))
    sys.stderr.flush()


T0 = time.time()


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=6)
    ap.add_argument("--workload", default="batch")
    ap.add_argument("--n", type=int, default=None)
    ap.add_argument("--m", type=int, default=None)
    ap.add_argument("--nq", type=int, default=None)
    ap.add_argument("--score", default=None, choices=["bf16", "fp8", "f32", "bf16x3"],
                    help="score precision (default: fp8 for the uneven workload, else bf16)")
    ap.add_argument("--mode", default=None, choices=["exact", "approx"],
                    help="exact (Def. 2) or approximate (Def. 3, the workload's c); default: approximate "
                         "for the workloads that name a c (uneven, learned), else exact")
    ap.add_argument("--no-fp32", action="store_true", help="skip the plain FP32 comparator")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-approx", action="store_true", help="skip the c = 1.5 approximate line")
    ap.add_argument("--no-single", action="store_true", help="skip the single-query all-ranks line")
    ap.add_argument("--rank-table", type=int, default=4096,
                    help="sample items for the index's rank table (0: no table)")
    ap.add_argument("--train-queries", type=int, default=1114,
                    help="learned workload: training queries (disjoint from the test queries)")
    ap.add_argument("--train-pairs", type=int, default=9766,
                    help="learned workload: (user, query) pairs per training query (half best by u.q/|u|, "
                         "half spread; 1,114 x 9,766 gives 10.0M triples)")
    ap.add_argument("--train-epochs", type=int, default=6)
    ap.add_argument("--seed-mult", type=int, default=0,
                    help="seeds per query, in units of k (0: the library's default)")
    ap.add_argument("--no-table-query", action="store_true", help="skip the paper's table query line")
    ap.add_argument("--no-table-compare", action="store_true",
                    help="skip timing the same batch with the rank table switched off")
    ap.add_argument("--cpu-users", type=int, default=0, help="users in the CPU sample (0: auto)")
    ap.add_argument("--no-secondary", action="store_true",
                    help="skip the uneven-list and learned-estimator workloads (run as child processes of "
                         "the batch bench)")
    ap.add_argument("--calib-copy-mib", type=int, default=0,
                    help="run one plain device copy of this many MiB first (scale for HBM counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: the library has no multi-GPU path "
              "(--gpus %d requested)" % args.gpus, file=sys.stderr)
        return 2

    import torch
    from paper_2504_13446_amd import rkr, workloads as W

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    if args.calib_copy_mib > 0:
        src = torch.empty(args.calib_copy_mib << 18, dtype=torch.float32, device="cuda")
        src.fill_(1.0)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        torch.mul(src, 1.0, out=dst)      # one elementwise kernel: reads and writes N bytes
        torch.cuda.synchronize()
        log("calibration copy: %d MiB read + %d MiB written" % (args.calib_copy_mib, args.calib_copy_mib))
        del src, dst
    log("generating workload %s" % args.workload)
    w = W.make(args.workload, n=args.n, m=args.m, nq=args.nq)
    n, m, d, nq = w.n, w.m, w.d, w.nq
    if args.score is None:
        args.score = "fp8" if w.name == "uneven" else "bf16"
    mode = args.mode or ("approx" if w.c is not None else "exact")
    cvec = np.full(nq, w.c if w.c is not None else 1.5) if mode == "approx" else None
    log("n=%d m=%d d=%d nq=%d dtype=%s" % (n, m, d, nq, w.dtype))
    U = rkr.to_device(w.U, w.dtype)
    P = rkr.to_device(w.P, w.dtype)
    Q = rkr.to_device(w.Qv, w.dtype)
    # candidate lists of the uneven workload (one CSR list per query)
    cand = {}
    if w.cand_off is not None:
        cand = {"cand_off": w.cand_off, "cand_ids": torch.from_numpy(w.cand_ids).cuda()}

    def run(index, c=cvec):
        return index.query_batch(Q, w.k, c=c, **cand)
    torch.cuda.synchronize()
    t = time.time()
    learned = w.name == "learned"
    idx = rkr.Index(U, P, score=args.score, rank_table=args.rank_table, sketch_samples=4096 if learned else 0)
    torch.cuda.synchronize()
    build_ms = (time.time() - t) * 1e3
    log("index built in %.0f ms" % build_ms)
    idx.configure(seed_mult=args.seed_mult)
    train_info = None
    if learned:
        # the rank estimator, trained on exact ranks of training queries that
        # are not test queries; the test batch then orders its seeds by it
        Qtr = rkr.to_device(W.extra_queries(w, args.train_queries), w.dtype)
        torch.cuda.synchronize()
        t = time.time()
        idx.train(Qtr, pairs_per_query=args.train_pairs, epochs=args.train_epochs, batch=4096, lr=1e-3, seed=5)
        torch.cuda.synchronize()
        s_tr = idx.stats()
        train_info = {"training_queries": int(Qtr.shape[0]), "triples": int(s_tr["pairs"]),
                      "epochs": args.train_epochs, "final_mse_ln_rank": round(float(s_tr["mlp_loss"]), 5),
                      "ms": round((time.time() - t) * 1e3, 1)}
        log("estimator trained: %s" % train_info)
        del Qtr
        idx.configure(seed_mult=args.seed_mult, use_estimator=True)

    for i in range(args.warmup):
        run(idx)
        log("warmup %d: %s" % (i, _brief(idx.stats())))
    torch.cuda.synchronize()
    per = []
    t0 = time.perf_counter()
    for i in range(args.steps):
        ids, rk, off = run(idx)
        per.append(idx.stats())
        log("step %d: %s" % (i, _brief(per[-1])))
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms_step = (t1 - t0) * 1e3 / args.steps
    qps = nq * args.steps / (t1 - t0)
    gcmp = n * m * nq / (ms_step / 1e3) / 1e9
    st = per[-1]
    mean = lambda key: float(np.mean([s_[key] for s_ in per]))
    # The dominant launch: the exact-mode count kernel (seed pass + refine pass
    # of a step, one template instance).  Its algorithmic work is 2 d flop per
    # (user, item) score of a user with a live pair (d unpadded), counted by
    # the kernel itself; its time is the HIP-event duration of its launches.
    exact_ms = mean("ms_exact_kernel")
    seed_ms = mean("ms_seed_kernel")
    screen_ms = mean("ms_screen_kernel")
    alg_exact = mean("scored_exact") * 2.0 * d
    alg_seed = mean("scored_seed") * 2.0 * d
    alg_all = mean("scored_pairs") * 2.0 * d
    exec_all = mean("mfma_flop")
    launches = 1 + int(st["refined_pairs"] > 0)
    peak = PEAK_TFLOPS[args.score]
    tf = lambda flop, ms: flop / (ms / 1e3) / 1e12 if ms > 0 else 0.0
    achieved = tf(alg_exact, exact_ms)
    cmp = mean("compares")
    cmp_rate = cmp / ((exact_ms + screen_ms) / 1e3) / 1e12 if exact_ms + screen_ms > 0 else 0.0
    ids_np = ids.cpu().numpy()
    rk_np = rk.cpu().numpy()

    out = {
        "metric": METRIC,
        "value": round(qps, 3),
        "unit": "queries/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": args.score,
        "data": "synthetic",
        "config": {"workload": w.name, "n_users": n, "m_items": m, "d": d, "queries": nq,
                   "k": int(w.k[0]) if np.all(w.k == w.k[0]) else sorted(set(int(v) for v in w.k)),
                   "masters": w.dtype, "score": args.score,
                   "mode": mode if mode == "exact" else "approx c=%g" % cvec[0],
                   "candidate_pairs": int(w.cand_off[-1]) if w.cand_off is not None else None,
                   "rank_table_samples": args.rank_table,
                   "generator": "iid N(0,I) directions x LogNormal(0,0.5) norms, seeded"},
        # rank comparisons per second: the n * m * Q the definition asks for
        # (dense equivalent), and the (score, threshold) compares executed
        "gcompare_per_s": round(gcmp, 1),
        "gcompare_per_s_executed": round(float(st["compares"]) / (ms_step / 1e3) / 1e9, 1),
        "gcompare_note": "gcompare_per_s is dense-equivalent (n*m*Q per step time); the kernels execute "
                         "gcompare_per_s_executed",
        "build_ms": round(build_ms, 1),
        "breakdown_ms": {k: round(st[k], 3) for k in ("ms_thresh", "ms_seed", "ms_screen", "ms_refine",
                                                      "ms_select", "ms_total", "ms_seed_kernel",
                                                      "ms_screen_kernel", "ms_exact_kernel", "ms_recheck_kernel")},
        "counters": {k: int(st[k]) for k in ("pairs", "seed_pairs", "survivors", "refined_pairs",
                                             "uncertain", "flips", "compares", "compare_slots", "screen_ctas",
                                             "screen_variant", "table_pruned", "mfma_flop", "scored_pairs",
                                             "scored_seed", "scored_exact")},
        "roofline": {
            "kernel": "k_pass<13, false>: the pipelined exact pass (BF16 32x32x16 MFMA, threshold folded into the "
                      "accumulators): the seed and refine launches of a step",
            "bound": "mfma", "achieved": round(achieved, 2), "peak": peak, "unit": "TFLOP/s",
            "frac": round(achieved / peak, 4),
            "traffic": exact_traffic({"workload": w.name, "n": n, "m": m, "d": d, "queries": nq,
                                      "score": args.score, "rank_table": args.rank_table}),
            "launches_per_step": launches,
            "avg_launch_ms": round(exact_ms / launches, 3),
            "algorithmic_flop_per_launch": alg_exact / launches,
            "work_unit": "2*d flop per (user, item) score of a user with a live pair, d = %d unpadded" % d,
            "target_frac": 0.5, "target_met": bool(achieved / peak >= 0.5),
            "seed_pass": {"ms": round(seed_ms, 3), "algorithmic_flop": alg_seed,
                          "achieved": round(tf(alg_seed, seed_ms), 2),
                          "frac": round(tf(alg_seed, seed_ms) / peak, 4)},
            "all_count_launches": {"ms": round(exact_ms + screen_ms, 3),
                                   "algorithmic": {"flop": alg_all,
                                                   "frac": round(tf(alg_all, exact_ms + screen_ms) / peak, 4)},
                                   "executed_padded": {"flop": exec_all,
                                                       "frac": round(tf(exec_all, exact_ms + screen_ms) / peak, 4)}},
            "alu_view": {"achieved": round(cmp_rate, 4), "peak": ALU_PEAK_TOPS, "unit": "TOP/s",
                         "frac": round(cmp_rate / ALU_PEAK_TOPS, 5), "compares_per_step": cmp}},
    }

    if train_info is not None:
        out["estimator"] = learned_line(idx, run, w, train_info, cvec, rk_np, off, ms_step)

    exact_ans = (ids_np, rk_np, off)
    if mode == "approx":
        # the same workload answered exactly: its time, and the Sec. 5 quality
        # of the approximate answers against it (the returned ranks are exact
        # for every returned user)
        run(idx, c=None)
        torch.cuda.synchronize()
        t = time.perf_counter()
        ids_e, rk_e, off_e = run(idx, c=None)
        torch.cuda.synchronize()
        ms_e = (time.perf_counter() - t) * 1e3
        se = idx.stats()
        exact_ans = (ids_e.cpu().numpy(), rk_e.cpu().numpy(), off_e)
        out["exact_same_workload"] = {"ms_per_step": round(ms_e, 2), "queries_per_s": round(nq / (ms_e / 1e3), 2),
                                      "near_ties_rechecked": int(se["uncertain"]),
                                      "recheck_fraction_of_compares": round(se["uncertain"] / max(se["compares"], 1), 6)}
        out["approx_quality"] = quality(rk_np, off, rk_e.cpu().numpy(), off_e, cvec[0])
        out["approx_quality"].update({"near_ties_rechecked": int(st["uncertain"]),
                                      "recheck_fraction_of_compares": round(st["uncertain"] / max(st["compares"], 1), 6),
                                      "queries_settled_without_refine": int(st["approx_settled"])})
        log("exact on the same workload: %.1f ms; approximate quality %s" % (ms_e, out["approx_quality"]))

    if not args.no_approx and mode == "exact" and not cand:
        out["approx_c1_5"] = approx_line(idx, Q, w, ids_np, rk_np, off)

    if args.rank_table > 0 and not args.no_table_compare:
        # the same batch with the table switched off (the screen then scans
        # every non-seed pair); warm-up lets the tuner settle on its own key
        idx.configure(no_table=True, seed_mult=args.seed_mult)
        for _ in range(6):
            run(idx)
        torch.cuda.synchronize()
        t = time.perf_counter()
        for _ in range(2):
            ids_nt, rk_nt, _ = run(idx)
        torch.cuda.synchronize()
        ms_nt = (time.perf_counter() - t) * 1e3 / 2
        same = bool(np.array_equal(ids_nt.cpu().numpy(), ids_np) and np.array_equal(rk_nt.cpu().numpy(), rk_np))
        s_nt = idx.stats()
        out["without_rank_table"] = {"ms_per_step": round(ms_nt, 2), "queries_per_s": round(nq / (ms_nt / 1e3), 3),
                                     "screen_kernel_ms": round(s_nt["ms_screen_kernel"], 2),
                                     "same_answers": same}
        out["speedup_from_rank_table"] = round(ms_nt / ms_step, 3)
        idx.configure(no_table=False, seed_mult=args.seed_mult)
        log("without the rank table: %.1f ms/step (same answers: %s)" % (ms_nt, same))

    if not args.no_table_query and mode == "exact" and not cand:
        ks = np.atleast_1d(w.k).astype(np.int32)
        if args.rank_table > 0:
            # the query of Sec. 4.3 on the index's exact-cell table
            out["table_query"] = table_query_line(idx, Q, w, ks, ids_np, rk_np, off, paper=False)
        # the paper's own method: Alg. 1's table (tau = 500, Sec. 5.1) and its query
        out["paper_table_query"] = table_query_line(idx, Q, w, ks, ids_np, rk_np, off, paper=True)

    if not args.no_single:
        out["single_all_ranks"] = single_all_ranks(rkr, W)

    if not args.no_fp32:
        # like for like: the same pipeline (rank table built the same way, same
        # seeds) with FP32 scores on the matrix cores and a plain compare of the
        # score with fl32(t): no error band, no FP64 recheck, not exact
        log("plain FP32 comparator: building (rank table %d samples)" % args.rank_table)
        t = time.time()
        idx32 = rkr.Index(U, P, score="f32", recheck=False, rank_table=args.rank_table)
        torch.cuda.synchronize()
        b32 = (time.time() - t) * 1e3
        idx32.configure(seed_mult=args.seed_mult)
        for _ in range(2):
            run(idx32)
        torch.cuda.synchronize()
        t = time.perf_counter()
        for _ in range(3):
            ids32, rk32, _ = run(idx32)
        torch.cuda.synchronize()
        ms32 = (time.perf_counter() - t) * 1e3 / 3
        s32 = idx32.stats()
        agree = float(np.mean(ids32.cpu().numpy() == ids_np))
        out["fp32_plain"] = {"ms_per_step": round(ms32, 2), "queries_per_s": round(nq / (ms32 / 1e3), 3),
                             "timed_steps": 3, "rank_table_samples": args.rank_table, "build_ms": round(b32, 1),
                             "exact_kernel_ms": round(s32["ms_exact_kernel"], 2),
                             "screen_kernel_ms": round(s32["ms_screen_kernel"], 2),
                             "answer_ids_agreeing_with_exact": round(agree, 5)}
        out["speedup_vs_fp32_plain"] = round(ms32 / ms_step, 3)
        log("plain FP32 (rank table): %.1f ms/step" % ms32)
        if args.rank_table > 0 and not args.no_table_compare:
            # the same pair without the rank table (the screen scans every pair)
            idx32.configure(no_table=True, seed_mult=args.seed_mult)
            for _ in range(2):
                run(idx32)
            torch.cuda.synchronize()
            t = time.perf_counter()
            run(idx32)
            torch.cuda.synchronize()
            ms32nt = (time.perf_counter() - t) * 1e3
            out["fp32_plain"]["without_rank_table_ms_per_step"] = round(ms32nt, 2)
            if "without_rank_table" in out:
                out["speedup_vs_fp32_plain_without_rank_table"] = round(
                    ms32nt / out["without_rank_table"]["ms_per_step"], 3)
            log("plain FP32 without the rank table: %.1f ms/step" % ms32nt)
        idx32.close()

    if not args.no_cpu:
        # the sample is checked against the exact answers (in approximate
        # mode, those of the exact leg)
        out["cpu_baseline"] = cpu_baseline(w, *exact_ans, args.cpu_users)
    idx.close()
    if not args.no_secondary and w.name == "batch":
        out["uneven"] = secondary("uneven", ["--score", "bf16", "--steps", "2", "--warmup", "1"])
        out["learned"] = secondary("learned", ["--steps", "2", "--warmup", "1"])
    print(json.dumps(out))
    sys.stdout.flush()
    return 0


def secondary(workload: str, extra: list) -> dict:
    """Another workload of the batched path, run as a child process of this
    one (its own line, embedded): the uneven candidate lists (500k x 1M x
    300, c = 1.5, BF16 scores) or the learned estimator (1M x 1M x 200,
    1,024 queries, trained on 10M triples, c = 1.5)."""
    import subprocess
    cmd = [sys.executable, os.path.abspath(__file__), "--workload", workload, "--no-cpu", "--no-fp32", "--no-single",
           "--no-table-compare", "--no-secondary", *extra]
    log("secondary workload: %s" % " ".join(cmd[2:]))
    r = subprocess.run(cmd, stdout=subprocess.PIPE, text=True)
    if r.returncode != 0:
        return {"error": "exit status %d" % r.returncode}
    line = json.loads(r.stdout.strip().splitlines()[-1])
    keep = ("value", "unit", "ms_per_step", "dtype", "config", "build_ms", "breakdown_ms", "approx_quality",
            "exact_same_workload", "estimator", "roofline")
    res = {k: line[k] for k in keep if k in line}
    res["counters"] = {k: line["counters"][k] for k in ("pairs", "seed_pairs", "survivors", "uncertain", "flips",
                                                        "table_pruned", "scored_pairs")}
    res["roofline"] = {k: res["roofline"][k] for k in ("frac", "achieved", "unit", "seed_pass")}
    return res


def learned_line(idx, run, w, train_info, cvec, rk_main, off_main, ms_main) -> dict:
    """The learned workload: what the trained estimator buys.  Exact answers
    with seeds ordered by the estimator and by the rank-table heuristic
    (u.q/|u|) must be identical; the work each needed is compared (seed pairs
    counted, pairs left after the screen, executed compares, scored pairs,
    time).  The approximate batch (c) of the main line against the same
    batch without the estimator.  And pruning: the answer taken from the 2k
    users per query of best predicted rank (estimator) or best u.q/|u|,
    counted exactly, with no verifying screen (Def. 3 not guaranteed): the
    Sec. 5 criteria, Def. 3 violations and recall of the exact top-k."""
    import torch

    def timed(c, use_est, prune=0, reps=2):
        idx.configure(use_estimator=use_est, prune_mult=prune)
        run(idx, c=c)
        torch.cuda.synchronize()
        t = time.perf_counter()
        for _ in range(reps):
            ids, rk, off = run(idx, c=c)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t) * 1e3 / reps
        st = idx.stats()
        work = {k: int(st[k]) for k in ("seed_pairs", "survivors", "refined_pairs", "compares", "scored_pairs",
                                        "uncertain")}
        return ids.cpu().numpy(), rk.cpu().numpy(), off, round(ms, 2), work

    res = {"training": train_info}
    ie, re_, oe, ms_e, work_e = timed(None, True)
    ih, rh, oh, ms_h, work_h = timed(None, False)
    res["exact"] = {"identical_answers": bool(np.array_equal(ie, ih) and np.array_equal(re_, rh)),
                    "with_estimator": {"ms_per_step": ms_e, **work_e},
                    "rank_table_heuristic": {"ms_per_step": ms_h, **work_h}}
    _, ra, oa, ms_a, work_a = timed(cvec, False)
    res["approx_without_estimator"] = {"ms_per_step": ms_a, **work_a,
                                       "quality": quality(ra, oa, re_, oe, cvec[0])}
    res["approx_with_estimator"] = {"ms_per_step": round(ms_main, 2),
                                    "quality": quality(rk_main, off_main, re_, oe, cvec[0])}
    for name, use in (("pruned_estimator", True), ("pruned_heuristic", False)):
        ip, rp, op, ms_p, work_p = timed(cvec, use, prune=2)
        rec = [len(set(ip[op[i]:op[i + 1]].tolist()) & set(ie[oe[i]:oe[i + 1]].tolist())) / float(oe[i + 1] - oe[i])
               for i in range(w.nq)]
        res[name] = {"candidates_per_query": "2k", "ms_per_step": ms_p, **work_p,
                     "quality": quality(rp, op, re_, oe, cvec[0]), "recall_of_exact_top_k": round(float(np.mean(rec)), 4)}
    idx.configure(use_estimator=True, prune_mult=0)
    log("estimator line: %s" % json.dumps(res))
    return res


def quality(rk_c, off_c, rk_x, off_x, c: float) -> dict:
    """The Sec. 5 criteria of approximate answers (true ranks rk_c) against the
    exact ones (rk_x), per query in rank order, averaged: accuracy, overall
    ratio, and Def. 3 violations."""
    acc, ratio, viol = [], [], 0
    for i in range(len(off_c) - 1):
        a = np.sort(rk_c[off_c[i]:off_c[i + 1]].astype(np.float64))
        b = np.sort(rk_x[off_x[i]:off_x[i + 1]].astype(np.float64))
        viol += int(np.sum(a > c * b))
        acc.append(float(np.mean(a <= c * b)))
        ratio.append(float(np.mean(a / b)))
    return {"c": float(c), "accuracy": round(float(np.mean(acc)), 5), "overall_ratio": round(float(np.mean(ratio)), 5),
            "def3_violations": int(viol)}


def approx_line(idx, Q, w, ids_ex, rk_ex, off, c: float = 1.5) -> dict:
    """The same batch in approximate mode (Def. 3, c = 1.5): time, and the
    paper's quality criteria of Sec. 5 per query, averaged: accuracy (the
    share of positions i with r(c_i) <= c r(rr_i)), overall ratio (mean of
    r(c_i) / r(rr_i)), and Def. 3 violations.  The ranks of the returned users
    are the ones the call returns (every returned user is counted exactly);
    U_rr's are the exact path's answer from the main leg."""
    import torch
    cc = np.full(w.nq, c)
    for _ in range(2):
        idx.query_batch(Q, w.k, c=cc)
    torch.cuda.synchronize()
    t = time.perf_counter()
    for _ in range(3):
        ids, rk, offc = idx.query_batch(Q, w.k, c=cc)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t) * 1e3 / 3
    st = idx.stats()
    rk = rk.cpu().numpy()
    acc, ratio, viol, weak = [], [], 0, 0
    for i in range(w.nq):
        # the i-th user of each answer in rank order (Def. 3 pairs them so)
        a = np.sort(rk[offc[i]:offc[i + 1]].astype(np.float64))
        b = np.sort(rk_ex[off[i]:off[i + 1]].astype(np.float64))
        viol += int(np.sum(a > c * b))
        weak += int(np.sum(a > c * b[-1]))
        acc.append(float(np.mean(a <= c * b)))
        ratio.append(float(np.mean(a / b)))
    log("approximate c=%.1f: %.1f ms/step, accuracy %.4f, overall ratio %.4f, violations %d" % (
        c, ms, np.mean(acc), np.mean(ratio), viol))
    return {"c": c, "ms_per_step": round(ms, 3), "queries_per_s": round(w.nq / (ms / 1e3), 2),
            "accuracy": round(float(np.mean(acc)), 5), "overall_ratio": round(float(np.mean(ratio)), 5),
            "def3_violations": int(viol), "abstract_form_violations": int(weak),
            "queries_settled_without_refine": int(st["approx_settled"]),
            "refined_pairs": int(st["refined_pairs"]), "seed_pairs": int(st["seed_pairs"]),
            "ranks_from": "returned ranks (exact for every returned user); U_rr from the exact leg"}


def table_query_line(idx, Q, w, ks, ids_ex, rk_ex, off, paper: bool, c: float = 1.5,
                     tau: int = 500, omega: int = 64, s: int = 64) -> dict:
    """The query of Sec. 4.3 for the whole batch in one call, c = 1.5: on the
    paper's own table (Alg. 1: tau uniform thresholds, cells estimated from s
    random samples in each of omega norm buckets), or on the index's table
    with exact lower-bound cells.  An estimate: scored with the Sec. 5
    accuracy and overall ratio against the exact answers.  The true ranks of
    the returned users come from the library's exact path (one candidate list
    per query: the users it returned)."""
    import torch
    from paper_2504_13446_amd import rkr, workloads as W
    res = {"c": c, "queries": int(w.nq)}
    if paper:
        pos = W.bucket_sample_positions(w.m, omega, s)
        torch.cuda.synchronize()
        t = time.perf_counter()
        idx.paper_table_build(tau, omega, s, pos)
        torch.cuda.synchronize()
        res.update({"tau": tau, "omega": omega, "samples_per_bucket": s,
                    "build_ms": round((time.perf_counter() - t) * 1e3, 1)})
        run = lambda: idx.query_paper_table_batch(Q, ks, c)
    else:
        res["table"] = "exact lower-bound cells at %d sampled thresholds per user" % rkr.TABLE_COLS
        run = lambda: idx.query_table_batch(Q, ks, c)
    for _ in range(2):
        run()
    torch.cuda.synchronize()
    t = time.perf_counter()
    for _ in range(3):
        ids_t, _, off_t = run()
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t) * 1e3 / 3
    cand = ids_t.clone()
    _, true_rk, off_c = idx.query_batch(Q, ks, cand_off=off_t, cand_ids=cand)
    true_rk = true_rk.cpu().numpy()
    acc, ratio, rec = [], [], []
    ids_np = ids_t.cpu().numpy()
    for i in range(w.nq):
        a = np.sort(true_rk[off_c[i]:off_c[i + 1]].astype(np.float64))
        b = np.sort(rk_ex[off[i]:off[i + 1]].astype(np.float64))
        acc.append(float(np.mean(a <= c * b)))
        ratio.append(float(np.mean(a / b)))
        rec.append(len(set(ids_np[off_t[i]:off_t[i + 1]].tolist()) & set(ids_ex[off[i]:off[i + 1]].tolist()))
                   / float(ks[i]))
    res.update({"ms_per_batch": round(ms, 3), "queries_per_s": round(w.nq / (ms / 1e3), 2),
                "accuracy": round(float(np.mean(acc)), 5), "overall_ratio": round(float(np.mean(ratio)), 5),
                "min_accuracy": round(float(np.min(acc)), 4), "recall_of_exact_top_k": round(float(np.mean(rec)), 4)})
    log("%s table query: %.2f ms per batch, accuracy %.4f, overall ratio %.4f" % (
        "paper's" if paper else "exact-cell", ms, res["accuracy"], res["overall_ratio"]))
    return res


def single_all_ranks(rkr, W) -> dict:
    """Secondary line: exact ranks of every user for one query on the
    single-query workload (100k x 100k, d = 100, low-rank, FP32 masters), as
    replays of the captured all-ranks graph (median of 10 after warm-up):
    BF16 scores + FP64 recheck, FP32 scores + FP64 recheck (the low-rank
    scores crowd near each threshold, so the narrower FP32 band pays here),
    split BF16 scores (hi + lo per value, three BF16 products per term on the
    matrix cores, a band about 2^-13 as wide as BF16's) + FP64 recheck, and
    the plain FP32 path (not exact) for the same query."""
    import torch
    w = W.make("single")
    U = rkr.to_device(w.U, w.dtype)
    P = rkr.to_device(w.P, w.dtype)
    q = rkr.to_device(w.Qv[0], w.dtype)
    res = {"workload": "single", "n_users": w.n, "m_items": w.m, "d": w.d}
    for name, kw in (("bf16_recheck", dict(score="bf16")), ("fp32_recheck", dict(score="f32")),
                     ("bf16x3_recheck", dict(score="bf16x3")), ("fp32_plain", dict(score="f32", recheck=False))):
        idx = rkr.Index(U, P, **kw)
        idx.configure(graph=True)
        for _ in range(3):
            idx.ranks(q)
        torch.cuda.synchronize()
        times = []
        for _ in range(10):
            t = time.perf_counter()
            idx.ranks(q)
            torch.cuda.synchronize()
            times.append((time.perf_counter() - t) * 1e3)
        st = idx.stats()
        ms = float(np.median(times))
        res[name] = {"ms_per_query": round(ms, 3), "gcompare_per_s": round(w.n * w.m / (ms / 1e3) / 1e9, 1),
                     "near_ties_rechecked": int(st["uncertain"]), "graph_replays": int(st["graph_replays"])}
        idx.close()
    log("single all-ranks: bf16+recheck %.2f ms, fp32+recheck %.2f ms, split bf16+recheck %.2f ms, "
        "fp32 plain %.2f ms per query" % (
            res["bf16_recheck"]["ms_per_query"], res["fp32_recheck"]["ms_per_query"],
            res["bf16x3_recheck"]["ms_per_query"], res["fp32_plain"]["ms_per_query"]))
    return res


def _brief(s: dict) -> str:
    return "total %.1f ms (thresh %.1f seed %.1f screen %.1f [kernel %.1f] refine %.1f select %.1f) " \
           "table-pruned %d survivors %d uncertain %d" % (
               s["ms_total"], s["ms_thresh"], s["ms_seed"], s["ms_screen"], s["ms_screen_kernel"], s["ms_refine"],
               s["ms_select"], s["table_pruned"], s["survivors"], s["uncertain"])


def cpu_baseline(w, ids, rk, off, users: int) -> dict:
    """The CPU oracle on a bounded sample: exact Def. 1 ranks of `users` random
    users for every query of the batch (each user's m scores are shared by the
    queries), scaled to the whole batch.  The sample also cross-checks the GPU
    answer: a sampled user outside a query's answer may not beat its k-th rank."""
    from oracle import oracle as O
    threads = O.num_threads()
    if users <= 0:
        users = max(64, 64 * threads)
    rng = np.random.default_rng(7)
    sample = np.sort(rng.choice(w.n, size=min(users, w.n), replace=False))
    log("cpu baseline: %d users x %d queries x %d items on %d threads" % (sample.size, w.nq, w.m, threads))
    Uw = O.widen(w.U)
    Pw = O.widen(w.P)
    Qw = O.widen(w.Qv)
    t = time.perf_counter()
    R = O.ranks(Uw, Pw, Qw, uids=sample)
    sec = time.perf_counter() - t
    frac = sample.size / w.n
    qps = w.nq * frac / sec
    bad = 0
    for i in range(w.nq):
        a_ids = ids[off[i]:off[i + 1]]
        a_rk = rk[off[i]:off[i + 1]]
        Rk, last = int(a_rk[-1]), int(a_ids[-1])
        ins = set(a_ids.tolist())
        for j, u in enumerate(sample):
            r = int(R[i, j])
            if u in ins:
                bad += int(r != int(a_rk[list(a_ids).index(u)]))
            elif r < Rk or (r == Rk and u < last):
                bad += 1
    log("cpu baseline: %.1f s, sample inconsistencies with the GPU answer: %d" % (sec, bad))
    return {"value": round(qps, 6), "unit": "queries/s", "cores": threads, "kind": "oracle",
            "sample": "%d random users x all %d queries x all %d items (%.3g of the batch), %.1f s"
                      % (sample.size, w.nq, w.m, frac, sec),
            "sample_inconsistencies": bad}


if __name__ == "__main__":
    sys.exit(main())
