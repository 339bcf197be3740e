// query.h -- views and helper launchers of the query pipeline.
#pragma once
#include "kernels.h"

namespace rkr {

// Domain of a call: dense (every user x every query) or CSR candidate lists.
// Query q's domain list has positions i = 0 .. seg_off[q+1] - seg_off[q] - 1
// in ascending user id; pid(q, i) = i * nq + q (dense) or qm_pid[seg_off[q] + i].
struct QView {
    int dense;
    int nq;
    int64_t n;
    const int64_t *seg_off;   // device [nq + 1]
    const int32_t *qm_pid;    // CSR only
};

// Read-only view of a task set.
struct TView {
    int64_t ntask;
    const int32_t *len;
    const int64_t *blk_base;
    const int32_t *ent_pid;
    const uint32_t *ent_cnt;    // screening: remaining budgets
};


hipError_t q_seed_keys(const QView &v, const int32_t *pair_u, const double *t64, const double *unorm3,
                       const float *pred, int64_t total, uint64_t *keys, hipStream_t st);
hipError_t q_mark_selected(const QView &v, const uint64_t *sel, const int64_t *sel_off, int64_t total,
                           uint8_t *flag, hipStream_t st);
hipError_t q_compact_flags(const uint8_t *flag, int64_t N, int32_t *out, int64_t *count, Scratch &sc,
                           hipStream_t st);
hipError_t q_zero_at(const int32_t *pids, int64_t N, uint32_t *cnt, hipStream_t st);
hipError_t q_rank_keys_sel(const QView &v, const uint64_t *sel, const int64_t *sel_off, int64_t total,
                           const uint32_t *cnt, uint64_t *keys, hipStream_t st);
hipError_t q_bounds(const uint64_t *best, const int64_t *best_off, const int32_t *k, const double *c, int nq,
                    int32_t *bound, int32_t *seed_kth, hipStream_t st);
// flagged indices to out1 (their number to *count1), the others to out0
hipError_t q_split_flags(const uint8_t *flag, int64_t N, int32_t *out1, int64_t *count1, int32_t *out0,
                         hipStream_t st, Scratch &sc);
// live pairs of a task set (seeds excluded), in task order; with rem_out,
// also each pair's remaining budget at rem_out[pid]
hipError_t q_survivors(const TView &t, const uint8_t *seedflag, int32_t *out, int64_t *count, Scratch &sc,
                       hipStream_t st, uint32_t *rem_out = nullptr);
// dst[s * n + i] = src[i] for s < ns (the per-split copies of a split screen)
hipError_t q_replicate_u32(const uint32_t *src, int64_t n, uint32_t *dst, int ns, hipStream_t st);
// after a screen split ns ways (ns <= 16) over item ranges: keep the pairs
// every split kept whose summed partial counts stay within the budget, with
// the budget left (sp_*: the splits' lists, [ns][ntask_pad] and [ns][cap_total])
hipError_t q_screen_merge(TaskSet &ts, int ns, const int32_t *sp_len, const int32_t *sp_pid,
                          const uint32_t *sp_rem, hipStream_t st,
                          bool one_per_task = false);
// number of tasks whose list is not empty
hipError_t q_count_live(const int32_t *len, int64_t n, unsigned long long *dev, int64_t *count, hipStream_t st);
// *scored -= (ntask - *nusers) * m, on the device
hipError_t q_scored_fix(unsigned long long *scored, int64_t ntask, const int64_t *nusers, int64_t m, hipStream_t st);
// cand_off[0..nq] = exclusive scan of qcount[q] + seeds[q]
hipError_t q_cand_offsets(const int32_t *qcount, const int32_t *seeds, int nq, int64_t *cand_off, Scratch &sc,
                          hipStream_t st);
// dense estimator candidates: pid of each selected key (segments cand_off),
// and keys (predicted log-rank, user) for the second selection
hipError_t q_est_cand_pids(const uint64_t *csel, const int64_t *coff, int nq, int64_t nc, int32_t *pids,
                           hipStream_t st);
hipError_t q_est_cand_keys(const uint64_t *csel, const float *pred, int64_t nc, uint64_t *keys, hipStream_t st);
hipError_t q_count_by_query(const int32_t *pids, int64_t N, const int32_t *pair_q, int32_t *qcount,
                            hipStream_t st);
hipError_t q_cand_keys(const QView &v, const uint64_t *sel, const int64_t *sel_off, int64_t nsel,
                       const int32_t *surv, int64_t nsurv, const int32_t *pair_u, const int32_t *pair_q,
                       const uint32_t *cnt, const int64_t *cand_off, int32_t *cursor, uint64_t *keys,
                       hipStream_t st);
hipError_t q_write_answer(const uint64_t *keys, int64_t total, int32_t *ids, int32_t *ranks, hipStream_t st);
hipError_t q_ranks_out(const uint32_t *cnt, int64_t n, int32_t *ranks, hipStream_t st);
// tasks of the n users u0 .. u0 + n - 1, one entry each (pair id = user id)
hipError_t q_tasks_one_per_user(int64_t n, int64_t ntask_pad, const PairSet &ps, int plain, TaskSet &ts,
                                hipStream_t st, int64_t u0 = 0);
hipError_t q_copy(const void *src, void *dst, int64_t bytes, hipStream_t st);
// keep[pid] = 1 for the non-seed pairs the rank table cannot rule out
// (tab_t, tab_cnt: [n][TABLE_COLS] thresholds and certain counts)
hipError_t q_table_keep(const PairSet &ps, const uint8_t *seedflag, const int32_t *bound, const double *tab_t,
                        const uint32_t *tab_cnt, uint8_t *keep, hipStream_t st,
                        const float *t_up = nullptr);
hipError_t q_round_up_f32(const double *x, int64_t n, float *out, hipStream_t st);
// the paper's table query (Sec. 4.3) for a dense batch of nq queries (pairs
// u * nq + q; keys query-major): brackets and estimates, each query's R_lo_k,
// R_hi_k and case, the step-2 classification, the answer assembly.  Keys
// carry an integer rank in their top 32 bits, or with fk = 1 the order key
// of an FP32 bound (the paper's estimated cells).
hipError_t q_tqb_bounds(int64_t n, int nq, int64_t m, const double *t64, const double *tab_t, const uint32_t *tab_cnt,
                        uint64_t *key_lo, uint64_t *key_hi, double *est, hipStream_t st);
hipError_t q_tqb_kth(int nq, const int32_t *k, const double *c, const uint64_t *sel_lo, const uint64_t *sel_hi,
                     const int64_t *sel_off, uint32_t *R_lo, uint32_t *R_hi, int32_t *first_case, hipStream_t st,
                     int fk = 0);
hipError_t q_tqb_classify(int64_t n, int nq, const double *c, const uint32_t *R_lo, const uint32_t *R_hi,
                          const int32_t *first_case, const uint64_t *key_lo, const uint64_t *key_hi, const double *est,
                          uint64_t *key_c, uint64_t *key_t, unsigned long long *nadm, hipStream_t st, int fk = 0);
hipError_t q_tqb_answer(int nq, int64_t n, int64_t total, const int64_t *off, const int32_t *first_case,
                        const int64_t *sel_off, const uint64_t *sel_hi, const int32_t *nc, const int64_t *off_c,
                        const uint64_t *sel_c, const int64_t *off_t, const uint64_t *sel_t, const double *est,
                        int32_t *ids, double *est_out, hipStream_t st, int fk = 0);

}  // namespace rkr
