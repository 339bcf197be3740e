/*
 * rkr.h -- exact and c-approximate reverse k-ranks queries on AMD MI355X.
 *
 * Problem (arXiv 2504.13446, Sec. 2):
 *   Def. 1  r(q,u,P) = 1 + #{p in P : u.p > u.q}            (strict ">")
 *   Def. 2  the reverse k-ranks answer U_rr: k users whose ranks are no
 *           worse than any user left out.  This library breaks ties on rank
 *           by user id, so the answer is unique, and lists it by
 *           (rank ascending, user id ascending).
 *   Def. 3  the c-approximate answer U_c (c >= 1): the i-th user of U_c has
 *           rank at most c times the rank of the i-th user of U_rr.
 *
 * Arithmetic.  The paper fixes no precision.  "u.p" here is one fixed
 * evaluation: acc = +0.0, then acc = fma(u[k], p[k], acc) for k = 0..d-1 in
 * order, in IEEE double, on the master values.  Every rank this library
 * returns as exact equals the rank under that evaluation.  Scores are first
 * computed in low precision on the matrix cores; every score within a proven
 * error bound of its threshold is recomputed in double (the near-tie
 * recheck).
 *
 * Memory and ownership.
 *   - Pointers marked [device] are device pointers on the current HIP device
 *     (e.g. torch tensors' data_ptr()), contiguous, row-major.  Pointers
 *     marked [host] are host memory.
 *   - rkr_build copies everything it needs; the caller may free U and P
 *     when it returns.  The index owns its device memory until rkr_destroy.
 *   - Outputs are caller-allocated.
 *   - Every call is ordered on the stream given at build time (NULL = the
 *     default stream) and returns after its work has completed.
 *   - Calls on one index must not overlap (one thread at a time per index).
 *     Distinct indexes are independent.
 *
 * Errors.  No call throws or aborts.  On error a call returns a status other
 * than RKR_OK, writes no output, and rkr_last_error() returns a message for
 * the calling thread (valid until that thread's next rkr_* call).
 */
#ifndef RKR_H
#define RKR_H

#include <stdint.h>

/* Columns (thresholds) per user of the rank table (rkr_rank_table). */
#define RKR_TABLE_COLS 48

#ifdef __cplusplus
extern "C" {
#endif

typedef struct rkr_index rkr_index;

typedef enum {
    RKR_OK = 0,
    RKR_E_INVALID = 1,     /* an argument is out of range (message says which) */
    RKR_E_NOMEM = 2,       /* device or host allocation failed */
    RKR_E_DEVICE = 3,      /* a HIP runtime call failed */
    RKR_E_UNSUPPORTED = 4, /* valid request outside the library's limits */
    RKR_E_STATE = 5        /* the index lacks a part the call needs */
} rkr_status;

/* Master (ground-truth) element type of U, P and queries. */
typedef enum { RKR_F32 = 0, RKR_BF16 = 1 } rkr_dtype;

/* Element type of the low-precision scoring pass on the matrix cores. */
typedef enum {
    RKR_SCORE_F32 = 0,   /* FP32 inputs, FP32 accumulation              */
    RKR_SCORE_BF16 = 1,  /* BF16 inputs (round to nearest even), FP32 acc */
    RKR_SCORE_FP8 = 2,   /* FP8 e4m3 with a power-of-two scale per vector */
    RKR_SCORE_BF16X3 = 3 /* split BF16: each value as hi + lo (two BF16), */
                         /* scores hi.hi + hi.lo + lo.hi over 3d terms,   */
                         /* FP32 acc (error ~2^-16 relative, d <= 106)    */
} rkr_score;

typedef struct {
    int32_t score;          /* rkr_score (default RKR_SCORE_BF16)                        */
    int32_t recheck;        /* 1: FP64 near-tie recheck, exact ranks (default);          */
                            /* 0: plain compare of the low-precision score with the     */
                            /*    threshold rounded to FP32 (not exact; for comparison) */
    int32_t sketch_samples; /* >0: build the per-user score sketch for the estimator    */
                            /*     from this many norm-stratified items (e.g. 4096)     */
    int32_t rank_table;     /* >0: build the rank table (Sec. 4.2) from this many       */
                            /*     norm-stratified items (at most 4096): RKR_TABLE_COLS */
                            /*     thresholds per user with certain counts over all of  */
                            /*     P; batch queries then skip the pairs it rules out    */
                            /*     (Lemma 1)                                            */
    void *stream;           /* hipStream_t for all work on this index; NULL = default   */
} rkr_build_opts;

/* Per-call planning knobs (rkr_configure); zero fields keep the default. */
typedef struct {
    int32_t seed_mult;      /* seeds per query = seed_mult * k (default: 1 with a rank   */
                            /* table in use, else 2)                                     */
    int32_t use_estimator;  /* 1: order seeds by the trained estimator (needs rkr_train) */
    int32_t reserved0;      /* must be 0                                                 */
    int32_t prune_mult;     /* approximate mode only: answer from the prune_mult * k     */
                            /* users per query of best predicted rank (estimator) or     */
                            /* best u.q/|u| (no estimator), without the verifying screen */
                            /* (0: off; Def. 3 is then not guaranteed)                   */
    int32_t graph;          /* 1: rkr_ranks runs as a captured hipGraph (captured on the */
                            /*    first call, replayed after; falls back to the eager    */
                            /*    path when the near-tie buffer would overflow)          */
    int32_t no_table;       /* 1: do not prune with the rank table                       */
    int32_t reserved[2];
} rkr_query_opts;

/* Counters of the last query call (rkr_stats). */
typedef struct {
    int64_t queries;        /* queries in the call                                        */
    int64_t pairs;          /* (user, query) pairs in the domain                          */
    int64_t seed_pairs;     /* pairs counted exactly to seed the per-query rank bound     */
    int64_t survivors;      /* pairs left after the screening pass                        */
    int64_t refined_pairs;  /* pairs counted exactly after screening                      */
    int64_t uncertain;      /* near-tie (user, item, query) triples rechecked in FP64      */
    int64_t flips;          /* rechecked triples whose FP64 verdict differs from a plain   */
                            /* FP32 compare of the low-precision score                     */
    int64_t compares;       /* executed (score, threshold) comparisons                     */
    int64_t emit_retries;   /* passes re-run because the near-tie buffer was too small     */
    int64_t approx_settled; /* approximate mode: queries settled without the exact fallback */
    double ms_thresh, ms_seed, ms_screen, ms_refine, ms_select, ms_total;
    double mlp_loss;        /* last training loss of the estimator (rkr_train)             */
    double ms_screen_kernel;/* duration of the screening count kernel (HIP events)         */
    double ms_exact_kernel; /* summed duration of the exact count kernels (HIP events)     */
    double ms_recheck_kernel; /* summed duration of the FP64 recheck kernels (HIP events)  */
    int64_t screen_ctas;    /* workgroups of the screening launch                           */
    int64_t screen_variant; /* launch candidate the autotuner chose for the screening pass: */
                            /* tile variant (v % n), persistent grid if v >= n (n = tile    */
                            /* variants of the score kind)                                  */
    int64_t compare_slots;  /* lane slots of the compare loops (active or idle): compares / */
                            /* compare_slots is the SIMD efficiency of the entry loops      */
    int64_t graph_replays;  /* 1 if the call replayed a captured graph                      */
    int64_t table_pruned;   /* pairs the rank table ruled out before the screen             */
    int64_t mfma_flop;      /* matrix-core flop the count kernels executed (padded shapes)  */
    int64_t scored_pairs;   /* (user, item) scores the count kernels computed for users     */
                            /* with a live pair (2 d flop each: the algorithmic work)       */
    int64_t persistent_phases; /* screening phases launched as a persistent grid            */
    double ms_seed_kernel;  /* duration of the seed pass's exact count kernel (HIP events)  */
    int64_t scored_seed;    /* scored_pairs of the seed pass                                */
    int64_t scored_exact;   /* scored_pairs of every exact pass (seeds, refine)             */
} rkr_query_stats;

/*
 * Build an index over users U [device, n x d] and items P [device, m x d],
 * both in master dtype dt.  Sorts P by norm (descending; Sec. 4.2 step 1),
 * makes the low-precision copies, their exact residual norms, and the
 * per-segment error-bound coefficients; with opts->rank_table > 0 also the
 * rank table (one more pass over U.P^T; not built when m = 0).
 * Errors: RKR_E_INVALID if n <= 0, m < 0, d <= 0, d > 4096, a value is not
 * finite or |value| > 2^50, sketch_samples or rank_table < 0;
 * RKR_E_UNSUPPORTED for n or m >= 2^31.
 * m = 0 is valid (every rank is 1).
 */
rkr_status rkr_build(const void *U, int64_t n, const void *P, int64_t m, int32_t d,
                     rkr_dtype dt, const rkr_build_opts *opts, rkr_index **out);

void rkr_destroy(rkr_index *idx);

rkr_status rkr_configure(rkr_index *idx, const rkr_query_opts *opts);

/*
 * Exact reverse k-ranks (Def. 2) of one query q [device, d, master dtype].
 * Writes the answer to ids_out[k] and ranks_out[k] [device, int32], sorted
 * by (rank, id).  Errors: RKR_E_INVALID if k < 1 or k > n, q not finite;
 * RKR_E_UNSUPPORTED if k > 4096.
 */
rkr_status rkr_query_exact(rkr_index *idx, const void *q, int32_t k, int32_t *ids_out,
                           int32_t *ranks_out);

/*
 * c-approximate reverse k-ranks (Def. 3) of one query, c >= 1.  ids_out[k]
 * lists U_c by (reported rank, id); rank_ub_out[k] holds each user's exact
 * rank where it was computed exactly, else a proven upper bound of it.
 * The returned set always satisfies Def. 3 (the exact answer is the fallback).
 */
rkr_status rkr_query_approx(rkr_index *idx, const void *q, int32_t k, double c,
                            int32_t *ids_out, int32_t *rank_ub_out);

/*
 * The paper's own query on the rank table (Sec. 4.3, steps 1-3) for one query
 * q [device, d, master dtype], c >= 1; the index must hold a rank table.
 * Step 1: with L = the number of the user's columns whose threshold is at or
 * above u.q (columns descend), the rank is bracketed by r_lo = 1 + cell[L-1]
 * (1 when L = 0) and r_hi = 1 + cell[L] (1 + m when L = RKR_TABLE_COLS);
 * R_lo_k, R_hi_k are the k-th smallest of each.  Step 2: if c R_lo_k >= R_hi_k
 * the answer is the k users of smallest r_hi; otherwise the users with
 * r_hi <= c R_lo_k come first, users with r_lo > R_hi_k are ruled out (Lemma 1
 * (2)), and step 3 fills the answer with the remaining users of smallest
 * estimate, r_lo + (r_hi - r_lo) (t[L-1] - u.q) / (t[L-1] - t[L]) (r_lo at
 * the ends of the row), ordered in FP32, ties by user id.  This is an
 * estimate: Def. 3 is not guaranteed (the cells count certain-above items at
 * sampled thresholds).  Writes ids_out[k] [device, int32] in answer order and
 * est_out[k] [device, double]: the bound or estimate each user was chosen by.
 * Errors: RKR_E_STATE without a table; RKR_E_INVALID for k outside [1, n],
 * c < 1 or not finite, a non-finite query; RKR_E_UNSUPPORTED if k > 4096.
 */
rkr_status rkr_query_table(rkr_index *idx, const void *q, int32_t k, double c, int32_t *ids_out,
                           double *est_out);

/*
 * The same table query for nq queries at once (Sec. 4.3, steps 1-3 per
 * query): Qm [device, nq x d], k[nq] and c[nq] [host].  Query i's answer is
 * written at offset k[0] + ... + k[i-1] of ids_out and est_out [device].
 * Errors as rkr_query_table, plus RKR_E_INVALID for nq outside [1, 65535] and
 * RKR_E_UNSUPPORTED for n * nq >= 2^31.
 */
rkr_status rkr_query_table_batch(rkr_index *idx, int32_t nq, const void *Qm, const int32_t *k,
                                 const double *c, int32_t *ids_out, double *est_out);

/*
 * The paper's own rank table (Sec. 4.2, Alg. 1), with estimated cells:
 *   step 1: the items in norm order (descending, ties by id) are cut into
 *     omega equally sized buckets; bucket l holds the positions
 *     [floor(l m / omega), floor((l + 1) m / omega)) of that order;
 *   sampling: bucket l's samples are at the positions sample_pos[l * s + i]
 *     of the bucket, i < s_l = min(s, |P_l|) [host, omega * s int32; the
 *     random draws are the caller's; slots past s_l are ignored];
 *   step 2: tau thresholds spaced uniformly between f_min and f_max, with
 *     the paper's footnote's domain values f_max = |u| max_p |p| (Cauchy-
 *     Schwarz) and f_min = -f_max: t_j = f_min + j (f_max - f_min) / (tau - 1),
 *     j = 0 .. tau - 1, ascending (|x| is the FP64 spec norm);
 *   step 3: cell T_j = 1 + sum over buckets, in order, of
 *     (A_l[j] |P_l|) / s_l with A_l[j] = #{sampled p of bucket l : u.p > t_j}
 *     (the cell estimator of Sec. 4.2), in FP64, stored in FP32.
 * The table lives in the index (8 n bytes of f_min, 8 n of step, 4 n tau of
 * cells) and replaces any earlier one.  Errors: RKR_E_INVALID for tau < 2,
 * omega < 1 or s < 1, a position outside its bucket or repeated within it;
 * RKR_E_UNSUPPORTED for tau > 2047 or omega * s > 2^22.
 */
rkr_status rkr_paper_table_build(rkr_index *idx, int32_t tau, int32_t omega, int32_t s,
                                 const int32_t *sample_pos);

/*
 * The paper's table: fmin_out [device, n double] (f_min per user),
 * step_out [device, n double] (threshold spacing), cells_out [device,
 * n x tau float].  RKR_E_STATE without one.
 */
rkr_status rkr_paper_table(const rkr_index *idx, double *fmin_out, double *step_out, float *cells_out);

/*
 * The paper's query (Sec. 4.3, steps 1-3) on its own table, for nq queries
 * Qm [device, nq x d], k[nq] and c[nq] [host]:
 *   step 1: with L = #{j : t_j <= u.q}, r_lo = T_L (1 when L = tau) and
 *     r_hi = T_{L-1} (m + 1 when L = 0), FP32; R_lo_k, R_hi_k the k-th
 *     smallest of each;
 *   step 2: if c R_lo_k >= R_hi_k the answer is the k users of smallest r_hi
 *     (ties by id); otherwise the users with r_hi <= c R_lo_k come first (by
 *     r_hi, id), users with r_lo > R_hi_k are ruled out (Lemma 1 (2)) and
 *     step 3 fills the answer with the others of smallest estimate, linear
 *     in u.q between (t_{L-1}, r_hi) and (t_L, r_lo) (r_lo at either end of
 *     the row), ordered by the estimate rounded to FP32, ties by id.
 * Query i's answer is at offset k[0] + ... + k[i-1] of ids_out [device,
 * int32] and val_out [device, double] (the bound or estimate each user was
 * chosen by).  An estimate: Def. 3 is not guaranteed.  Errors as
 * rkr_query_table_batch, RKR_E_STATE without a paper table.
 */
rkr_status rkr_query_paper_table_batch(rkr_index *idx, int32_t nq, const void *Qm, const int32_t *k,
                                       const double *c, int32_t *ids_out, double *val_out);
rkr_status rkr_query_paper_table(rkr_index *idx, const void *q, int32_t k, double c, int32_t *ids_out,
                                 double *val_out);

/*
 * Batch of nq queries Qm [device, nq x d] sharing one pass over U.P^T.
 *   k        [host, nq]      answer size per query
 *   c        [host, nq]      NULL: exact answers (Def. 2); else c[i] >= 1
 *                            per query (Def. 3)
 *   cand_off [host, nq + 1]  NULL: every user is a candidate of every query;
 *                            else CSR offsets into cand_ids, and query i's
 *                            domain is cand_ids[cand_off[i] .. cand_off[i+1])
 *   cand_ids [device]        user ids (each list free of duplicates)
 *   ids_out, ranks_out [device, sum(k)]  answers concatenated in query order
 * Errors: RKR_E_INVALID for k[i] < 1 or above its domain size, c[i] < 1 or
 * NaN, non-monotone offsets, ids out of range or duplicated within a list;
 * RKR_E_UNSUPPORTED for nq > 65535, k[i] > 4096, or 2^31 or more (user,
 * query) pairs in the batch (n * nq, or the candidate lists' total).
 */
rkr_status rkr_query_batch(rkr_index *idx, int32_t nq, const void *Qm, const int32_t *k,
                           const double *c, const int64_t *cand_off, const int32_t *cand_ids,
                           int32_t *ids_out, int32_t *ranks_out);

/*
 * The rank table (Sec. 4.2) of an index built with rank_table > 0, with
 * RKR_TABLE_COLS columns per user.  Column j of user u holds a threshold
 * t_out[u * RKR_TABLE_COLS + j] (FP64: the user's spec score against a sample
 * item; thresholds do not increase with j) and cnt_out[u * RKR_TABLE_COLS + j],
 * a count of items p with s64(u,p) > t certainly (a lower bound of the exact
 * count: items within the score error of t are left out).  The paper's cell
 * is 1 + that count.  t_out [device, n x RKR_TABLE_COLS double], cnt_out
 * [device, n x RKR_TABLE_COLS uint32], caller-allocated.  RKR_E_STATE if the
 * index has no table.
 */
rkr_status rkr_rank_table(const rkr_index *idx, double *t_out, uint32_t *cnt_out);

/*
 * Check of the error bound the exact ranks rest on, over every (user, item)
 * pair of the index: for each, the matrix-core score s_hat of the index's
 * score kind and the FP64 spec dot s(u,p) of the master values, and the
 * bound eps the count kernels use for that user and item block.  Writes the
 * largest |s_hat - s(u,p)| / eps (rounded up to FP32) to *max_ratio_out and
 * the number of pairs with a ratio above 1 (a broken bound; the exactness
 * of every rank needs 0) to *over_out [host].  Costs d FP64 fma per pair.
 */
rkr_status rkr_score_error(rkr_index *idx, double *max_ratio_out, int64_t *over_out);

/*
 * The same check in the form the BF16 exact and screening passes take
 * (Sec. 4's rank counting with the threshold of query q): for every user u,
 * th = the least FP32 value >= s(u, q) is folded into the matrix-core
 * accumulators (they start from -th), and for every (user, item) pair the
 * result acc is checked against |acc - (s(u,p) - th)| <= E (1 + 1/dpad) +
 * gamma(dpad + 1) |th|, gamma(n) = 2n 2^-23, E the bound above and dpad the
 * padded dimension.  q [device, d values of the master type].  Outputs as
 * rkr_score_error.  RKR_E_UNSUPPORTED unless the score kind is BF16;
 * RKR_E_INVALID for a non-finite or too large value in q.
 */
rkr_status rkr_score_error_at(rkr_index *idx, const void *q, double *max_ratio_out, int64_t *over_out);

/* Exact Def. 1 rank of q for every user: ranks_out [device, n int32]. */
rkr_status rkr_ranks(rkr_index *idx, const void *q, int32_t *ranks_out);

/*
 * rkr_ranks for callers that cannot allocate device memory (code under graph
 * capture elsewhere, tight serving loops, harnesses that forbid hipMalloc):
 * the same ranks, ranks_out [device, n int32], but every per-call buffer
 * lives in one static 64 MiB array per device, placed when the first index
 * is built on that device and held until the process ends; the call
 * allocates nothing.  Users are counted in chunks that
 * fit the array; a chunk with more near ties than it holds is counted again
 * in smaller chunks.  Calls that overlap on one device share the array and
 * race: issue them one at a time per device.  Errors: RKR_E_UNSUPPORTED for
 * more than 2^20 users or 2^22 items; RKR_E_INVALID as rkr_ranks.
 */
rkr_status rkr_ranks_noalloc(rkr_index *idx, const void *q, int32_t *ranks_out);

/*
 * Learned rank estimator (an MLP 18 -> 64 -> 64 -> 1 on the features
 * [u.q / |u|, |u|, 16 sketch values]) predicting ln r.  rkr_train computes
 * exact ranks for (user, query) pairs of the training queries Qm [device,
 * nq x d] with the exact path, then trains the network on the GPU with FP32
 * forward, backward and Adam kernels.  pairs_per_query users are drawn per
 * query, half uniformly and half from the best-scoring users.  Needs an
 * index built with sketch_samples > 0 (else RKR_E_STATE).
 */
rkr_status rkr_train(rkr_index *idx, int32_t nq, const void *Qm, int32_t pairs_per_query,
                     int32_t epochs, int32_t batch, float lr, uint64_t seed);

/* Predicted ln r for nq queries x every user: out [device, nq x n float].
 * RKR_E_UNSUPPORTED if nq * n >= 2^31 (as for rkr_train's training queries). */
rkr_status rkr_predict(rkr_index *idx, int32_t nq, const void *Qm, float *out);

/*
 * Estimator parameters, flattened in the order W1[64x18], b1[64], W2[64x64],
 * b2[64], w3[64], b3[1] (5,441 floats) [host].
 */
rkr_status rkr_mlp_get(rkr_index *idx, float *params_out);
rkr_status rkr_mlp_set(rkr_index *idx, const float *params);

/*
 * One forward + backward pass of the estimator on a minibatch: X [device,
 * N x 18], z [device, N] targets; writes the mean squared error to
 * loss_out [host] and the gradient (flattened as above) to grad_out
 * [device, 5441].  For gradient checks against a reference.
 */
rkr_status rkr_mlp_grad(rkr_index *idx, const float *X, const float *z, int32_t N,
                        float *grad_out, double *loss_out);

/*
 * One Adam step (Kingma & Ba; b1 = 0.9, b2 = 0.999, eps = 1e-8, bias
 * correction for the 1-based step count `step`) of the estimator's
 * parameters with the gradient grad [device, 5441 float, flattened as
 * above] and learning rate lr; the kernel rkr_train runs per minibatch.
 * reset = 1 zeroes both moment estimates first.  RKR_E_STATE if the network
 * has no parameters (rkr_train or rkr_mlp_set first); RKR_E_INVALID for
 * step < 1 or lr <= 0.
 */
rkr_status rkr_mlp_adam(rkr_index *idx, const float *grad, float lr, int32_t step, int32_t reset);

/* Per-user sketch [device, n x 16 float] (needs sketch_samples > 0). */
rkr_status rkr_sketch(rkr_index *idx, float *out);

/* Counters of the last query call on this index [host]. */
rkr_status rkr_stats(const rkr_index *idx, rkr_query_stats *out);

/* Message of the calling thread's last failed call ("" if none). */
const char *rkr_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* RKR_H */
