// query.hip -- per-call helper kernels of the query pipeline: seed keys,
// seed marking, compaction of flagged pairs, survivor collection, the per-query
// rank bound and the answer assembly.
#include <algorithm>

#include "query.h"

namespace rkr {

static inline unsigned nblocks(int64_t n, int bs) { return (unsigned)((n + bs - 1) / bs); }

__device__ inline int seg_of(const int64_t *off, int nseg, int64_t j) {
    int lo = 0, hi = nseg;    // off[lo] <= j < off[hi]
    while (hi - lo > 1) {
        int mid = (lo + hi) >> 1;
        if (off[mid] <= j) lo = mid; else hi = mid;
    }
    return lo;
}

__device__ inline int32_t pid_of(const QView &v, int q, int64_t i) {
    return v.dense ? (int32_t)(i * v.nq + q) : v.qm_pid[v.seg_off[q] + i];
}

__global__ void k_fill_u32(uint32_t *p, uint32_t v, int64_t n) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t s = (int64_t)gridDim.x * blockDim.x;
    for (; i < n; i += s) p[i] = v;
}
__global__ void k_fill_u8(uint8_t *p, uint8_t v, int64_t n) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t s = (int64_t)gridDim.x * blockDim.x;
    for (; i < n; i += s) p[i] = v;
}
hipError_t launch_fill_u32(uint32_t *p, uint32_t v, int64_t n, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    int64_t nb = (n + 255) / 256;
    if (nb > 65536) nb = 65536;
    hipLaunchKernelGGL(k_fill_u32, dim3((unsigned)nb), dim3(256), 0, st, p, v, n);
    return hipGetLastError();
}
hipError_t launch_fill_u8(uint8_t *p, uint8_t v, int64_t n, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    int64_t nb = (n + 255) / 256;
    if (nb > 65536) nb = 65536;
    hipLaunchKernelGGL(k_fill_u8, dim3((unsigned)nb), dim3(256), 0, st, p, v, n);
    return hipGetLastError();
}

// Seed keys: smaller is more promising.  Default heuristic: -t / |u| (for an
// isotropic item set the rank is a decreasing function of the cosine of u and
// q).  With an estimator, its predicted log-rank.  Low 32 bits: position in
// the query's domain list (ascending user id), so ties go to smaller ids.
__global__ void k_seed_keys(QView v, const int32_t *pair_u, const double *t64, const double *unorm3,
                            const float *pred, int64_t total, uint64_t *keys) {
    int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= total) return;
    int q = v.dense ? (int)(j / v.n) : seg_of(v.seg_off, v.nq, j);
    int64_t i = j - v.seg_off[q];
    int32_t pid = pid_of(v, q, i);
    float h;
    if (pred) {
        h = pred[pid];
    } else {
        double nu = unorm3[3 * (int64_t)pair_u[pid] + 2];
        h = nu > 0.0 ? (float)(-t64[pid] / nu) : 0.0f;
    }
    keys[j] = ((uint64_t)f32_order_key(h) << 32) | (uint32_t)i;
}

// Dense domains: the same keys, one workgroup per tile of 64 users x 32
// queries through LDS, so the reads of the user-major pair arrays and the
// writes of the query-major keys are both coalesced.
__global__ __launch_bounds__(256) void k_seed_keys_dense(int64_t n, int nq, const double *t64,
                                                         const double *unorm3, const float *pred,
                                                         uint64_t *keys) {
    __shared__ float s_h[32][65];
    const int64_t u0 = (int64_t)blockIdx.x * 64;
    const int q0 = blockIdx.y * 32;
    const int tid = threadIdx.x;
#pragma unroll
    for (int r = 0; r < 8; ++r) {
        const int uu = r * 8 + (tid >> 5), qq = tid & 31;
        const int64_t u = u0 + uu;
        const int q = q0 + qq;
        if (u < n && q < nq) {
            const int64_t pid = u * nq + q;
            float h;
            if (pred) {
                h = pred[pid];
            } else {
                const double nu = unorm3[3 * u + 2];
                h = nu > 0.0 ? (float)(-t64[pid] / nu) : 0.0f;
            }
            s_h[qq][uu] = h;
        }
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < 8; ++r) {
        const int qq = r * 4 + (tid >> 6), uu = tid & 63;
        const int64_t u = u0 + uu;
        const int q = q0 + qq;
        if (u < n && q < nq) keys[(int64_t)q * n + u] = ((uint64_t)f32_order_key(s_h[qq][uu]) << 32) | (uint32_t)u;
    }
}

__global__ void k_mark_selected(QView v, const uint64_t *sel, const int64_t *sel_off, int64_t total,
                                uint8_t *flag) {
    int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= total) return;
    int q = seg_of(sel_off, v.nq, j);
    int64_t i = (int64_t)(uint32_t)(sel[j] & 0xFFFFFFFFu);
    flag[pid_of(v, q, i)] = 1;
}

__global__ void k_zero_at(const int32_t *pids, int64_t N, uint32_t *cnt) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < N) cnt[pids[i]] = 0;
}

// keys (rank << 32 | i) of the selected seeds of every query
__global__ void k_rank_keys_sel(QView v, const uint64_t *sel, const int64_t *sel_off, int64_t total,
                                const uint32_t *cnt, uint64_t *keys) {
    int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= total) return;
    int q = seg_of(sel_off, v.nq, j);
    uint32_t i = (uint32_t)(sel[j] & 0xFFFFFFFFu);
    int32_t pid = pid_of(v, q, i);
    keys[j] = ((uint64_t)(1u + cnt[pid]) << 32) | i;
}

// Per-query abandon bound from the k best seed ranks: B = k-th rank; the
// approximate mode (c > 1) uses floor(B / c) (see the pipeline notes).
__global__ void k_bounds(const uint64_t *best, const int64_t *best_off, const int32_t *k, const double *c,
                         int nq, int32_t *bound, int32_t *seed_kth) {
    int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= nq) return;
    uint32_t B = (uint32_t)(best[best_off[q] + k[q] - 1] >> 32);
    seed_kth[q] = (int32_t)B;
    double X = (c && c[q] > 1.0) ? floor((double)B / c[q]) : (double)B;
    bound[q] = (int32_t)X;
}

// Survivors of the screen: per task, live entries that are not seeds.
__global__ void k_surv_count(const TView t, const uint8_t *seedflag, int32_t *cnt_task) {
    int64_t ti = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (ti >= t.ntask) return;
    int c = 0;
    const int L = t.len[ti];
    const int64_t base = t.blk_base[ti >> 5] + (ti & 31);
    for (int i = 0; i < L; ++i) c += seedflag[t.ent_pid[base + (int64_t)i * 32]] ? 0 : 1;
    cnt_task[ti] = c;
}
__global__ void k_surv_write(const TView t, const uint8_t *seedflag, const int64_t *off, int32_t *out,
                             uint32_t *rem_out) {
    int64_t ti = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (ti >= t.ntask) return;
    int64_t o = off[ti];
    const int L = t.len[ti];
    const int64_t base = t.blk_base[ti >> 5] + (ti & 31);
    for (int i = 0; i < L; ++i) {
        const int64_t e = base + (int64_t)i * 32;
        int32_t pid = t.ent_pid[e];
        if (!seedflag[pid]) {
            out[o++] = pid;
            if (rem_out) rem_out[pid] = t.ent_cnt[e];
        }
    }
}

// Number of tasks with a non-empty list (one 64-bit atomic per workgroup).
__global__ void k_count_live(const int32_t *len, int64_t n, unsigned long long *out) {
    __shared__ unsigned int s;
    if (threadIdx.x == 0) s = 0;
    __syncthreads();
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const unsigned long long b = __ballot(i < n && len[i] > 0);
    if ((threadIdx.x & 63) == 0 && b) atomicAdd(&s, (unsigned int)__popcll(b));
    __syncthreads();
    if (threadIdx.x == 0 && s) atomicAdd(out, (unsigned long long)s);
}

// Answer candidates per query = its seeds + its survivors.
__global__ void k_count_by_query(const int32_t *pids, int64_t N, const int32_t *pair_q, int32_t *qcount) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < N) atomicAdd(&qcount[pair_q[pids[i]]], 1);
}
__global__ void k_cand_keys_seeds(QView v, const uint64_t *sel, const int64_t *sel_off, int64_t total,
                                  const int32_t *pair_u, const uint32_t *cnt, const int64_t *cand_off,
                                  uint64_t *keys) {
    int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= total) return;
    int q = seg_of(sel_off, v.nq, j);
    int64_t i = (int64_t)(uint32_t)(sel[j] & 0xFFFFFFFFu);
    int32_t pid = pid_of(v, q, i);
    keys[cand_off[q] + (j - sel_off[q])] = ((uint64_t)(1u + cnt[pid]) << 32) | (uint32_t)pair_u[pid];
}
__global__ void k_cand_keys_surv(const int32_t *pids, int64_t N, const int32_t *pair_u, const int32_t *pair_q,
                                 const uint32_t *cnt, const int64_t *cand_off, int32_t *cursor,
                                 uint64_t *keys) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    int32_t pid = pids[i];
    int q = pair_q[pid];
    int64_t p = cand_off[q] + atomicAdd(&cursor[q], 1);
    keys[p] = ((uint64_t)(1u + cnt[pid]) << 32) | (uint32_t)pair_u[pid];
}
__global__ void k_write_answer(const uint64_t *keys, int64_t total, int32_t *ids, int32_t *ranks) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= total) return;
    ids[i] = (int32_t)(keys[i] & 0xFFFFFFFFu);
    ranks[i] = (int32_t)(keys[i] >> 32);
}
__global__ void k_ranks_out(const uint32_t *cnt, int64_t n, int32_t *ranks) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) ranks[i] = (int32_t)(1u + cnt[i]);
}

// One entry per user (single query): task t = user u0 + t (t < n), block b's
// entries at 32 b + lane.  Built without host round trips so the whole
// single-query pipeline can be captured in a graph.
__global__ void k_tasks_one_per_user(int64_t n, int64_t ntask_pad, int64_t u0, const double *t64, int plain,
                                     int32_t *task_user, int32_t *len,
                                     int64_t *blk_base, int32_t *ent_pid, int32_t *ent_q, uint32_t *ent_cnt,
                                     float *ent_th, float *ent_tl, float *ent_tm) {
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= ntask_pad) return;
    const bool real = t < n;
    task_user[t] = real ? (int32_t)(u0 + t) : -1;
    len[t] = real ? 1 : 0;
    if ((t & 31) == 0) blk_base[t >> 5] = t;
    ent_pid[t] = real ? (int32_t)(u0 + t) : 0;
    ent_q[t] = 0;
    ent_cnt[t] = 0;
    // the FP32 values bracketing t (see k_fill_entries)
    const double tv = real ? t64[u0 + t] : 0.0;
    const float tm = (float)tv;
    ent_th[t] = real ? (plain ? tm : f32_round_up(tv)) : 0.0f;
    ent_tl[t] = real ? (plain ? tm : f32_round_down(tv)) : 0.0f;
    ent_tm[t] = real ? tm : 0.0f;
}
__global__ void k_copy_words(const uint32_t *src, uint32_t *dst, int64_t nw) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < nw) dst[i] = src[i];
}
__global__ void k_copy_bytes(const uint8_t *src, uint8_t *dst, int64_t nb) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < nb) dst[i] = src[i];
}

// ---------------------------------------------------------------------------
// Stream compaction of a 0/1 byte array (flags) into the ascending indices
// of its set (and, optionally, unset) bytes.  A block owns FC_CHUNK bytes,
// read 16 at a time per thread in FC_ITER coalesced sweeps; pass 1 counts the
// set bytes per block, an exclusive scan of the block counts gives each
// block's output offset, pass 2 re-reads the chunk and writes the indices in
// element order (sweep, thread, byte).  No per-element offsets are stored.
constexpr int FC_BS = 256, FC_ITER = 4, FC_CHUNK = FC_BS * 16 * FC_ITER;

// The lane's 16 flags at byte offset o (fewer past n; bytes past n read as 0)
__device__ inline uint4 flags16(const uint8_t *flag, int64_t n, int64_t o) {
    if (o + 16 <= n) return *(const uint4 *)(flag + o);
    uint32_t w[4] = {0u, 0u, 0u, 0u};
    for (int j = 0; j < 16; ++j)
        if (o + j < n) w[j >> 2] |= (uint32_t)flag[o + j] << (8 * (j & 3));
    return make_uint4(w[0], w[1], w[2], w[3]);
}
__device__ inline int count16(uint4 v) {
    return __popc(v.x & 0x01010101u) + __popc(v.y & 0x01010101u) + __popc(v.z & 0x01010101u) +
           __popc(v.w & 0x01010101u);
}
// block-wide exclusive prefix of v over threads, and the block total
__device__ inline int block_excl(int v, int *tot) {
    __shared__ int ws[FC_BS / 64];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    int incl = v;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const int t = __shfl_up(incl, o, 64);
        if (lane >= o) incl += t;
    }
    if (lane == 63) ws[wave] = incl;
    __syncthreads();
    int before = 0, all = 0;
#pragma unroll
    for (int w = 0; w < FC_BS / 64; ++w) {
        before += w < wave ? ws[w] : 0;
        all += ws[w];
    }
    __syncthreads();   // ws is reused by the next call
    *tot = all;
    return before + incl - v;
}

__global__ __launch_bounds__(FC_BS) void k_flag_count(const uint8_t *flag, int64_t n, int64_t *counts) {
    const int64_t base = (int64_t)blockIdx.x * FC_CHUNK;
    int c = 0;
#pragma unroll
    for (int it = 0; it < FC_ITER; ++it) c += count16(flags16(flag, n, base + it * (FC_BS * 16) + threadIdx.x * 16));
    int tot;
    (void)block_excl(c, &tot);
    if (threadIdx.x == 0) counts[blockIdx.x] = tot;
}

// out1: indices of set bytes; out0 (may be null): indices of the others
__global__ __launch_bounds__(FC_BS) void k_flag_scatter(const uint8_t *flag, int64_t n, const int64_t *offs,
                                                        int32_t *out1, int32_t *out0) {
    const int64_t base = (int64_t)blockIdx.x * FC_CHUNK;
    int64_t run1 = offs[blockIdx.x];
    int64_t run0 = base - run1;   // unset bytes before the block
    for (int it = 0; it < FC_ITER; ++it) {
        const int64_t o = base + it * (FC_BS * 16) + threadIdx.x * 16;
        const uint4 v = flags16(flag, n, o);
        const int c1 = count16(v);
        const int valid = o >= n ? 0 : (int)min<int64_t>(16, n - o);
        int tot1, tot0;
        int64_t p1 = run1 + block_excl(c1, &tot1);
        int64_t p0 = run0 + block_excl(valid - c1, &tot0);
        const uint32_t w[4] = {v.x, v.y, v.z, v.w};
        for (int j = 0; j < valid; ++j) {
            const bool set = (w[j >> 2] >> (8 * (j & 3))) & 1u;
            if (set)
                out1[p1++] = (int32_t)(o + j);
            else if (out0)
                out0[p0++] = (int32_t)(o + j);
        }
        run1 += tot1;
        run0 += tot0;
    }
}

// Rank-table filter (the paper's Lemma 1 (2) with the table of Sec. 4.2 as
// the source of lower-bound ranks): a non-seed pair (u, q) goes on to the
// screen unless some column j of u has a threshold t_{u,j} >= t(u,q) whose
// certain count is >= B[q].  Every item above t_{u,j} is above t(u,q), so
// such a pair's count reaches B[q] and its rank exceeds the bound, exactly
// what the screen would find by scanning.  Seeds (already counted) are never
// kept.
// Dense domains (nq > 0) number pairs u * nq + q, so the pair arrays are not
// read.
// The number of entries at or above s in a table row (TABLE_COLS values that
// do not increase): they form a prefix, whose length a branch-free binary
// search finds in 6 steps instead of TABLE_COLS compares (probes past the row
// count as below).  For rows in LDS; a row in global memory is cheaper to
// scan with independent loads.
__device__ inline int cols_at_or_above(const double *row, double s) {
    static_assert(TABLE_COLS <= 63, "the search's steps sum to 63");
    int L = 0;
#pragma unroll
    for (int step = 32; step > 0; step >>= 1) {
        const int j = L + step - 1;
        if (j < TABLE_COLS && row[j] >= s) L += step;
    }
    return L;
}

__global__ void k_table_keep(int64_t npairs, int nq, const int32_t *pair_u, const int32_t *pair_q,
                             const double *t64, const uint8_t *seedflag, const int32_t *bound,
                             const double *tab_t, const uint32_t *tab_cnt, uint8_t *keep) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= npairs) return;
    if (seedflag[i]) {
        keep[i] = 0;
        return;
    }
    const int64_t u = nq > 0 ? i / nq : pair_u[i];
    const int q = nq > 0 ? (int)(i - u * nq) : pair_q[i];
    const double t = t64[i];
    // the columns' thresholds do not increase: L = the number of columns
    // with t_{u,j} >= t; column L - 1 is the tightest of them (any one of
    // them gives a valid bound)
    const double *tt = tab_t + u * TABLE_COLS;
    int L = 0;
#pragma unroll
    for (int j = 0; j < TABLE_COLS; ++j) L += tt[j] >= t ? 1 : 0;
    const uint32_t best = L > 0 ? tab_cnt[u * TABLE_COLS + L - 1] : 0u;
    keep[i] = (int64_t)best >= (int64_t)bound[q] ? 0 : 1;
}

// The same filter on a dense batch (pair u * nq + q): one workgroup per
// TK_USERS users and up to 256 queries.  The pair loads are issued first, then
// the users' rows of thresholds and counts go through LDS; the number of
// columns with t_{u,j} >= t is counted directly.
constexpr int TK_USERS = 4;
__global__ __launch_bounds__(256) void k_table_keep_dense(int64_t n, int nq, const double *t64, const float *t_up,
                                                          const uint8_t *seedflag, const int32_t *bound,
                                                          const double *tab_t, const uint32_t *tab_cnt,
                                                          uint8_t *keep) {
    __shared__ double srow[TK_USERS][TABLE_COLS];
    __shared__ uint32_t scnt[TK_USERS][TABLE_COLS];
    const int64_t u0 = (int64_t)blockIdx.x * TK_USERS;
    const int q = (int)blockIdx.y * (int)blockDim.x + (int)threadIdx.x;
    double t[TK_USERS];
    uint8_t sf[TK_USERS];
#pragma unroll
    for (int k = 0; k < TK_USERS; ++k) {
        const bool ok = q < nq && u0 + k < n;
        // (an upper bound of the threshold keeps at least the pairs the
        // threshold itself keeps: the columns at or above it can only be fewer)
        t[k] = ok ? (t_up ? (double)t_up[(u0 + k) * nq + q] : t64[(u0 + k) * nq + q]) : 0.0;
        sf[k] = ok ? seedflag[(u0 + k) * nq + q] : (uint8_t)1;
    }
    const int32_t B = q < nq ? bound[q] : 0;
    if (threadIdx.x < TK_USERS * TABLE_COLS) {
        const int k = threadIdx.x / TABLE_COLS, j = threadIdx.x % TABLE_COLS;
        if (u0 + k < n) {
            srow[k][j] = tab_t[(u0 + k) * TABLE_COLS + j];
            scnt[k][j] = tab_cnt[(u0 + k) * TABLE_COLS + j];
        }
    }
    __syncthreads();
    if (q >= nq) return;
#pragma unroll
    for (int k = 0; k < TK_USERS; ++k) {
        if (u0 + k >= n) break;
        const int64_t i = (u0 + k) * nq + q;
        if (sf[k]) {
            keep[i] = 0;
            continue;
        }
        const int L = cols_at_or_above(srow[k], t[k]);
        const uint32_t best = L > 0 ? scnt[k][L - 1] : 0u;
        keep[i] = (int64_t)best >= (int64_t)B ? 0 : 1;
    }
}

// ---------------------------------------------------------------------------
// The paper's table query (Sec. 4.3, steps 1-3) for a dense batch of
// queries.  Step 1, per (user, query): L = the number of the user's columns
// (descending thresholds) at or above u.q; the rank lies between r_lo = 1 +
// cnt[L - 1] (1 when L = 0) and r_hi = 1 + cnt[L] (1 + m when L =
// TABLE_COLS); step 3's estimate is linear in u.q between the two columns
// (r_lo at either end of the row or between equal thresholds).  Keys
// (r << 32 | u) order users by bound, then id.
// ---------------------------------------------------------------------------
__device__ inline void tq_bracket(const double *tt, const uint32_t *cc, double s, int64_t m, uint32_t &rlo,
                                  uint32_t &rhi, double &e) {
    const int L = cols_at_or_above(tt, s);
    rlo = L > 0 ? 1u + cc[L - 1] : 1u;
    rhi = L < TABLE_COLS ? 1u + cc[L] : (uint32_t)(1 + m);
    e = (double)rlo;
    if (L > 0 && L < TABLE_COLS) {
        const double tA = tt[L - 1], tB = tt[L];
        if (tA > tB) e = (double)rlo + (double)(rhi - rlo) * ((tA - s) / (tA - tB));
    }
}

// Brackets and estimates of the pairs u * nq + q go to query-major arrays
// [q * n + u] (one segment per query for the selections) through an LDS tile
// of TQB_U users x 32 queries, so the reads of t64 and the writes of the
// keys both coalesce.  A workgroup takes TQB_U users and a run of qt_per such
// query tiles, so the users' table rows, read into LDS once, serve all of
// them.  32 users keep the LDS at 35 KB, four workgroups per CU.
constexpr int TQB_U = 32;
__global__ __launch_bounds__(256) void k_tqb_bounds(int64_t n, int nq, int64_t m, const double *t64,
                                                    const double *tab_t, const uint32_t *tab_cnt, uint64_t *key_lo,
                                                    uint64_t *key_hi, double *est, int qt_per) {
    __shared__ uint32_t s_lo[32][TQB_U + 1], s_hi[32][TQB_U + 1];
    __shared__ double s_e[32][TQB_U + 1];
    __shared__ double s_t[TQB_U][TABLE_COLS];
    __shared__ uint32_t s_c[TQB_U][TABLE_COLS];
    const int64_t u0 = (int64_t)blockIdx.x * TQB_U;
    const int tid = threadIdx.x;
    for (int e = tid; e < TQB_U * TABLE_COLS; e += 256) {
        const int uu = e / TABLE_COLS, j = e - uu * TABLE_COLS;
        if (u0 + uu < n) {
            s_t[uu][j] = tab_t[(u0 + uu) * TABLE_COLS + j];
            s_c[uu][j] = tab_cnt[(u0 + uu) * TABLE_COLS + j];
        }
    }
    __syncthreads();
    const int qt_end = min((nq + 31) / 32, (int)(blockIdx.y + 1) * qt_per);
    for (int qt = blockIdx.y * qt_per; qt < qt_end; ++qt) {
        const int q0 = qt * 32;
#pragma unroll
        for (int r = 0; r < TQB_U / 8; ++r) {
            const int uu = r * 8 + (tid >> 5), qq = tid & 31;
            const int64_t u = u0 + uu;
            const int q = q0 + qq;
            if (u < n && q < nq) {
                uint32_t rlo, rhi;
                double e;
                tq_bracket(s_t[uu], s_c[uu], t64[u * nq + q], m, rlo, rhi, e);
                s_lo[qq][uu] = rlo;
                s_hi[qq][uu] = rhi;
                s_e[qq][uu] = e;
            }
        }
        __syncthreads();
#pragma unroll
        for (int r = 0; r < 32 * TQB_U / 256; ++r) {
            const int qq = r * (256 / TQB_U) + tid / TQB_U, uu = tid % TQB_U;
            const int64_t u = u0 + uu;
            const int q = q0 + qq;
            if (u < n && q < nq) {
                const int64_t j = (int64_t)q * n + u;
                key_lo[j] = ((uint64_t)s_lo[qq][uu] << 32) | (uint64_t)u;
                key_hi[j] = ((uint64_t)s_hi[qq][uu] << 32) | (uint64_t)u;
                est[j] = s_e[qq][uu];
            }
        }
        __syncthreads();    // the next query tile rewrites this one's LDS
    }
}

// The bound a key's top 32 bits carry: an integer rank (the exact-cell table)
// or, with fk, the order key of an FP32 bound (the paper's estimated cells).
__device__ inline double key_bound(uint32_t top, int fk) {
    if (!fk) return (double)top;
    const uint32_t b = (top & 0x80000000u) ? (top & 0x7FFFFFFFu) : ~top;
    return (double)__uint_as_float(b);
}

// Per query: R_lo_k, R_hi_k from the k smallest keys of each kind, and
// which case of step 2 applies (1: c R_lo_k >= R_hi_k).
__global__ void k_tqb_kth(int nq, const int32_t *k, const double *c, const uint64_t *sel_lo, const uint64_t *sel_hi,
                          const int64_t *sel_off, uint32_t *R_lo, uint32_t *R_hi, int32_t *first_case, int fk) {
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= nq) return;
    const int64_t i = sel_off[q] + k[q] - 1;
    const uint32_t lo = (uint32_t)(sel_lo[i] >> 32), hi = (uint32_t)(sel_hi[i] >> 32);
    R_lo[q] = lo;
    R_hi[q] = hi;
    first_case[q] = c[q] * key_bound(lo, fk) >= key_bound(hi, fk) ? 1 : 0;
}

// Step 2 when c R_lo_k < R_hi_k, per (query, user): the admitted users
// (r_hi <= c R_lo_k) keep their (r_hi, u) key in key_c, the users still open
// (not admitted, r_lo <= R_hi_k, Lemma 1 (2)) get (fl32(estimate), u) in
// key_t for step 3; every other key is the largest value.  nadm[q] counts
// the query's admitted users.  Queries in the first case get no keys.
__global__ void k_tqb_classify(int64_t n, const double *c, const uint32_t *R_lo, const uint32_t *R_hi,
                               const int32_t *first_case, const uint64_t *key_lo, const uint64_t *key_hi,
                               const double *est, uint64_t *key_c, uint64_t *key_t, unsigned long long *nadm,
                               int fk) {
    const int q = blockIdx.y;
    const int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    bool admit = false;
    if (u < n) {
        const int64_t j = (int64_t)q * n + u;
        bool open = false;
        const uint64_t kh = key_hi[j];
        if (!first_case[q]) {
            const uint32_t rhi = (uint32_t)(kh >> 32), rlo = (uint32_t)(key_lo[j] >> 32);
            admit = key_bound(rhi, fk) <= c[q] * key_bound(R_lo[q], fk);
            open = !admit && rlo <= R_hi[q];
        }
        key_c[j] = admit ? kh : ~0ull;
        key_t[j] = open ? (((uint64_t)f32_order_key((float)est[j]) << 32) | (uint64_t)u) : ~0ull;
    }
    const unsigned long long b = __ballot(admit);
    if ((threadIdx.x & 63) == 0 && b) atomicAdd(&nadm[q], (unsigned long long)__popcll(b));
}

// Answer slot j (queries concatenated, query q from off[q]): the first case
// takes the k smallest (r_hi, u) keys, the second its nc admitted keys then
// the step-3 keys.
__global__ void k_tqb_answer(int nq, int64_t n, const int64_t *off, const int32_t *first_case, const int64_t *sel_off,
                             const uint64_t *sel_hi, const int32_t *nc, const int64_t *off_c, const uint64_t *sel_c,
                             const int64_t *off_t, const uint64_t *sel_t, const double *est, int32_t *ids,
                             double *est_out, int fk) {
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= off[nq]) return;
    const int q = seg_of(off, nq, j);
    const int64_t i = j - off[q];
    uint64_t key;
    double e;
    if (first_case[q]) {
        key = sel_hi[sel_off[q] + i];
        e = key_bound((uint32_t)(key >> 32), fk);
    } else if (i < nc[q]) {
        key = sel_c[off_c[q] + i];
        e = key_bound((uint32_t)(key >> 32), fk);
    } else {
        key = sel_t[off_t[q] + i - nc[q]];
        e = est[(int64_t)q * n + (int64_t)(key & 0xFFFFFFFFu)];
    }
    ids[j] = (int32_t)(key & 0xFFFFFFFFu);
    est_out[j] = e;
}

// out[i] = the smallest float >= x[i]
__global__ void k_round_up_f32(const double *x, int64_t n, float *out) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] = f32_round_up(x[i]);
}

#define LAUNCH1D(kern, N, ...)                                                              \
    do {                                                                                   \
        if ((N) > 0) hipLaunchKernelGGL(kern, dim3(nblocks((N), 256)), dim3(256), 0, st, __VA_ARGS__); \
    } while (0)

hipError_t q_seed_keys(const QView &v, const int32_t *pair_u, const double *t64, const double *unorm3,
                       const float *pred, int64_t total, uint64_t *keys, hipStream_t st) {
    if (v.dense) {
        if (v.n > 0 && v.nq > 0)
            hipLaunchKernelGGL(k_seed_keys_dense, dim3((unsigned)((v.n + 63) / 64), (unsigned)((v.nq + 31) / 32)),
                               dim3(256), 0, st, v.n, v.nq, t64, unorm3, pred, keys);
        return hipGetLastError();
    }
    LAUNCH1D(k_seed_keys, total, v, pair_u, t64, unorm3, pred, total, keys);
    return hipGetLastError();
}
hipError_t q_mark_selected(const QView &v, const uint64_t *sel, const int64_t *sel_off, int64_t total,
                           uint8_t *flag, hipStream_t st) {
    LAUNCH1D(k_mark_selected, total, v, sel, sel_off, total, flag);
    return hipGetLastError();
}
// flags -> ascending indices of the set bytes (out1, *count1) and, when out0
// is not null, of the unset ones
static hipError_t flag_compact(const uint8_t *flag, int64_t N, int32_t *out1, int64_t *count1, int32_t *out0,
                               Scratch &sc, hipStream_t st) {
    if (N <= 0) {
        if (count1) *count1 = 0;
        return hipSuccess;
    }
    const int64_t nb = (N + FC_CHUNK - 1) / FC_CHUNK;
    int64_t *counts = (int64_t *)sc.take(nb * 8 + 8);
    int64_t *offs = (int64_t *)sc.take(nb * 8 + 8);
    int64_t *dtot = (int64_t *)sc.take(16);
    if (!counts || !offs || !dtot) return hipErrorOutOfMemory;
    hipLaunchKernelGGL(k_flag_count, dim3((unsigned)nb), dim3(FC_BS), 0, st, flag, N, counts);
    hipError_t e = scan_i64(counts, nb, offs, dtot, sc, st);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_flag_scatter, dim3((unsigned)nb), dim3(FC_BS), 0, st, flag, N, (const int64_t *)offs, out1,
                       out0);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if (!count1) return hipSuccess;   // the caller knows the count
    if ((e = hipMemcpyAsync(count1, dtot, 8, hipMemcpyDeviceToHost, st)) != hipSuccess) return e;
    return hipStreamSynchronize(st);
}
hipError_t q_compact_flags(const uint8_t *flag, int64_t N, int32_t *out, int64_t *count, Scratch &sc,
                           hipStream_t st) {
    return flag_compact(flag, N, out, count, nullptr, sc, st);
}
hipError_t q_split_flags(const uint8_t *flag, int64_t N, int32_t *out1, int64_t *count1, int32_t *out0,
                         hipStream_t st, Scratch &sc) {
    return flag_compact(flag, N, out1, count1, out0, sc, st);
}
hipError_t q_zero_at(const int32_t *pids, int64_t N, uint32_t *cnt, hipStream_t st) {
    LAUNCH1D(k_zero_at, N, pids, N, cnt);
    return hipGetLastError();
}
hipError_t q_rank_keys_sel(const QView &v, const uint64_t *sel, const int64_t *sel_off, int64_t total,
                           const uint32_t *cnt, uint64_t *keys, hipStream_t st) {
    LAUNCH1D(k_rank_keys_sel, total, v, sel, sel_off, total, cnt, keys);
    return hipGetLastError();
}
hipError_t q_bounds(const uint64_t *best, const int64_t *best_off, const int32_t *k, const double *c, int nq,
                    int32_t *bound, int32_t *seed_kth, hipStream_t st) {
    LAUNCH1D(k_bounds, (int64_t)nq, best, best_off, k, c, nq, bound, seed_kth);
    return hipGetLastError();
}
hipError_t q_survivors(const TView &t, const uint8_t *seedflag, int32_t *out, int64_t *count, Scratch &sc,
                       hipStream_t st, uint32_t *rem_out) {
    *count = 0;
    if (t.ntask <= 0) return hipSuccess;
    int32_t *ct = (int32_t *)sc.take(t.ntask * 4);
    int64_t *off = (int64_t *)sc.take(t.ntask * 8 + 8);
    int64_t *dtot = (int64_t *)sc.take(16);
    if (!ct || !off || !dtot) return hipErrorOutOfMemory;
    LAUNCH1D(k_surv_count, t.ntask, t, seedflag, ct);
    hipError_t e = scan_i32(ct, t.ntask, off, dtot, sc, st);
    if (e != hipSuccess) return e;
    if ((e = hipMemcpyAsync(count, dtot, 8, hipMemcpyDeviceToHost, st)) != hipSuccess) return e;
    if ((e = hipStreamSynchronize(st)) != hipSuccess) return e;
    LAUNCH1D(k_surv_write, t.ntask, t, seedflag, off, out, rem_out);
    return hipGetLastError();
}
// dst[s * n + i] = src[i] for s < ns
__global__ void k_replicate_u32(const uint32_t *src, int64_t n, uint32_t *dst, int ns) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const uint32_t v = src[i];
    for (int s = 0; s < ns; ++s) dst[(int64_t)s * n + i] = v;
}

// Merge of a split screen, one thread per task.  Every split started from the
// task's list (pid, th, rem0) and kept, in order, the entries its own items
// did not rule out, with rem_s = rem0 - (its partial count).  A pair lives on
// iff every split kept it and rem0 - (sum of the partial counts) =
// sum_s rem_s - (ns - 1) rem0 is not negative; the live entries are written
// back, in order, over the task's list with that remaining budget.
constexpr int MERGE_MAX_SPLITS = 16;
__global__ void k_screen_merge(int64_t ntask, const int64_t *blk_base, int64_t cap_total, int64_t len_stride,
                               int ns, int32_t *len, int32_t *pid, float *th, uint32_t *rem,
                               const int32_t *sp_len, const int32_t *sp_pid, const uint32_t *sp_rem) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= ntask) return;
    const int L = len[t];
    if (L == 0) return;
    const int64_t base = blk_base[t >> 5] + (t & 31);
    int ptr[MERGE_MAX_SPLITS], lsz[MERGE_MAX_SPLITS];
#pragma unroll
    for (int s = 0; s < MERGE_MAX_SPLITS; ++s) {
        ptr[s] = 0;
        lsz[s] = s < ns ? sp_len[(int64_t)s * len_stride + t] : 0;
    }
    int w = 0;
    for (int i = 0; i < L; ++i) {
        const int64_t e = base + (int64_t)i * 32;
        const int32_t p = pid[e];
        const int64_t rem0 = (int32_t)rem[e];
        const float h = th[e];
        bool alive = true;
        int64_t sum = 0;
#pragma unroll
        for (int s = 0; s < MERGE_MAX_SPLITS; ++s) {
            if (s < ns) {
                const int64_t es = (int64_t)s * cap_total + base + (int64_t)ptr[s] * 32;
                if (ptr[s] < lsz[s] && sp_pid[es] == p) {
                    sum += (int32_t)sp_rem[es];
                    ++ptr[s];
                } else {
                    alive = false;
                }
            }
        }
        const int64_t r = sum - (int64_t)(ns - 1) * rem0;
        if (alive && r >= 0) {
            const int64_t ew = base + (int64_t)w * 32;
            pid[ew] = p;
            th[ew] = h;
            rem[ew] = (uint32_t)r;
            ++w;
        }
    }
    len[t] = w;
}

// The same merge for lists of one entry per task, any number of splits.
__global__ void k_screen_merge1(int64_t ntask, const int64_t *blk_base, int64_t cap_total, int64_t len_stride,
                                int ns, int32_t *len, uint32_t *rem, const int32_t *sp_len, const uint32_t *sp_rem) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= ntask || len[t] == 0) return;
    const int64_t e = blk_base[t >> 5] + (t & 31);
    const int64_t rem0 = (int32_t)rem[e];
    int64_t sum = 0;
    bool alive = true;
    for (int s = 0; s < ns; ++s) {
        if (sp_len[(int64_t)s * len_stride + t] == 0) alive = false;
        else sum += (int32_t)sp_rem[(int64_t)s * cap_total + e];
    }
    const int64_t r = sum - (int64_t)(ns - 1) * rem0;
    if (alive && r >= 0) {
        rem[e] = (uint32_t)r;
    } else {
        len[t] = 0;
    }
}

hipError_t q_replicate_u32(const uint32_t *src, int64_t n, uint32_t *dst, int ns, hipStream_t st) {
    LAUNCH1D(k_replicate_u32, n, src, n, dst, ns);
    return hipGetLastError();
}
hipError_t q_screen_merge(TaskSet &ts, int ns, const int32_t *sp_len, const int32_t *sp_pid,
                          const uint32_t *sp_rem, hipStream_t st, bool one_per_task) {
    if (one_per_task) {
        if (ns < 1) return hipErrorInvalidValue;
        LAUNCH1D(k_screen_merge1, ts.ntask, ts.ntask, ts.blk_base, ts.cap_total, ts.ntask_pad, ns, ts.len,
                 ts.ent_cnt, sp_len, sp_rem);
        return hipGetLastError();
    }
    if (ns < 1 || ns > MERGE_MAX_SPLITS) return hipErrorInvalidValue;
    LAUNCH1D(k_screen_merge, ts.ntask, ts.ntask, ts.blk_base, ts.cap_total, ts.ntask_pad, ns, ts.len, ts.ent_pid,
             ts.ent_th, ts.ent_cnt, sp_len, sp_pid, sp_rem);
    return hipGetLastError();
}

hipError_t q_count_live(const int32_t *len, int64_t n, unsigned long long *dev, int64_t *count, hipStream_t st) {
    *count = 0;
    hipError_t e = launch_fill_u32((uint32_t *)dev, 0, 2, st);
    if (e != hipSuccess) return e;
    LAUNCH1D(k_count_live, n, len, n, dev);
    unsigned long long c = 0;
    if ((e = hipMemcpyAsync(&c, dev, 8, hipMemcpyDeviceToHost, st)) != hipSuccess) return e;
    if ((e = hipStreamSynchronize(st)) != hipSuccess) return e;
    *count = (int64_t)c;
    return hipSuccess;
}
// *scored -= (ntask - *nusers) * m: a user with several tasks was scored
// once per task; the algorithmic-work counter counts its scores once
__global__ void k_scored_fix(unsigned long long *scored, int64_t ntask, const int64_t *nusers, int64_t m) {
    if (threadIdx.x == 0 && blockIdx.x == 0) *scored -= (unsigned long long)(ntask - *nusers) * (unsigned long long)m;
}
hipError_t q_scored_fix(unsigned long long *scored, int64_t ntask, const int64_t *nusers, int64_t m, hipStream_t st) {
    hipLaunchKernelGGL(k_scored_fix, dim3(1), dim3(64), 0, st, scored, ntask, nusers, m);
    return hipGetLastError();
}
// candidate counts per query (its seeds and its survivors) -> offsets
__global__ void k_cand_sizes(const int32_t *qcount, const int32_t *seeds, int nq, int32_t *sizes) {
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q < nq) sizes[q] = qcount[q] + seeds[q];
}
hipError_t q_cand_offsets(const int32_t *qcount, const int32_t *seeds, int nq, int64_t *cand_off, Scratch &sc,
                          hipStream_t st) {
    int32_t *sizes = (int32_t *)sc.take((int64_t)nq * 4);
    if (!sizes) return hipErrorOutOfMemory;
    LAUNCH1D(k_cand_sizes, (int64_t)nq, qcount, seeds, nq, sizes);
    return scan_i32(sizes, nq, cand_off, cand_off + nq, sc, st);
}
// Estimator candidates of a dense batch: the pair of each selected key
// (low half: the user) and, from the predicted log-ranks, their keys.
__global__ void k_est_cand_pids(const uint64_t *csel, const int64_t *coff, int nq, int64_t nc, int32_t *pids) {
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= nc) return;
    int lo = 0, hi = nq - 1;   // the query: the segment holding j
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (coff[mid] <= j) lo = mid; else hi = mid - 1;
    }
    pids[j] = (int32_t)((int64_t)(uint32_t)csel[j] * nq + lo);
}
__global__ void k_est_cand_keys(const uint64_t *csel, const float *pred, int64_t nc, uint64_t *keys) {
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j < nc) keys[j] = ((uint64_t)f32_order_key(pred[j]) << 32) | (csel[j] & 0xFFFFFFFFull);
}
hipError_t q_est_cand_pids(const uint64_t *csel, const int64_t *coff, int nq, int64_t nc, int32_t *pids,
                           hipStream_t st) {
    LAUNCH1D(k_est_cand_pids, nc, csel, coff, nq, nc, pids);
    return hipGetLastError();
}
hipError_t q_est_cand_keys(const uint64_t *csel, const float *pred, int64_t nc, uint64_t *keys, hipStream_t st) {
    LAUNCH1D(k_est_cand_keys, nc, csel, pred, nc, keys);
    return hipGetLastError();
}
hipError_t q_count_by_query(const int32_t *pids, int64_t N, const int32_t *pair_q, int32_t *qcount,
                            hipStream_t st) {
    LAUNCH1D(k_count_by_query, N, pids, N, pair_q, qcount);
    return hipGetLastError();
}
hipError_t q_cand_keys(const QView &v, const uint64_t *sel, const int64_t *sel_off, int64_t nsel,
                       const int32_t *surv, int64_t nsurv, const int32_t *pair_u, const int32_t *pair_q,
                       const uint32_t *cnt, const int64_t *cand_off, int32_t *cursor, uint64_t *keys,
                       hipStream_t st) {
    LAUNCH1D(k_cand_keys_seeds, nsel, v, sel, sel_off, nsel, pair_u, cnt, cand_off, keys);
    LAUNCH1D(k_cand_keys_surv, nsurv, surv, nsurv, pair_u, pair_q, cnt, cand_off, cursor, keys);
    return hipGetLastError();
}
hipError_t q_write_answer(const uint64_t *keys, int64_t total, int32_t *ids, int32_t *ranks, hipStream_t st) {
    LAUNCH1D(k_write_answer, total, keys, total, ids, ranks);
    return hipGetLastError();
}
hipError_t q_tasks_one_per_user(int64_t n, int64_t ntask_pad, const PairSet &ps, int plain, TaskSet &ts,
                                hipStream_t st, int64_t u0) {
    LAUNCH1D(k_tasks_one_per_user, ntask_pad, n, ntask_pad, u0, ps.t64, plain, ts.task_user, ts.len,
             ts.blk_base, ts.ent_pid, ts.ent_q, ts.ent_cnt, ts.ent_th, ts.ent_tl, ts.ent_tm);
    return hipGetLastError();
}
hipError_t q_copy(const void *src, void *dst, int64_t bytes, hipStream_t st) {
    if (bytes % 4 == 0 && ((uintptr_t)src % 4) == 0 && ((uintptr_t)dst % 4) == 0) {
        LAUNCH1D(k_copy_words, bytes / 4, (const uint32_t *)src, (uint32_t *)dst, bytes / 4);
    } else {
        LAUNCH1D(k_copy_bytes, bytes, (const uint8_t *)src, (uint8_t *)dst, bytes);
    }
    return hipGetLastError();
}
hipError_t q_ranks_out(const uint32_t *cnt, int64_t n, int32_t *ranks, hipStream_t st) {
    LAUNCH1D(k_ranks_out, n, cnt, n, ranks);
    return hipGetLastError();
}

hipError_t q_table_keep(const PairSet &ps, const uint8_t *seedflag, const int32_t *bound, const double *tab_t,
                        const uint32_t *tab_cnt, uint8_t *keep, hipStream_t st, const float *t_up) {
    if (t_up && !ps.dense) return hipErrorInvalidValue;
    if (ps.dense && ps.nq > 0) {
        const int64_t n = ps.npairs / ps.nq;
        // at least TK_USERS * TABLE_COLS threads: they stage the rows
        static_assert(TK_USERS * TABLE_COLS <= 256, "rows staged by one thread per cell");
        const int bs = (ps.nq >= 192 || TK_USERS * TABLE_COLS > 128) ? 256 : 128;
        if (n > 0)
            hipLaunchKernelGGL(k_table_keep_dense, dim3((unsigned)((n + TK_USERS - 1) / TK_USERS),
                                                        (unsigned)((ps.nq + bs - 1) / bs)),
                               dim3(bs), 0, st, n, ps.nq, ps.t64, t_up, seedflag, bound, tab_t, tab_cnt, keep);
        return hipGetLastError();
    }
    LAUNCH1D(k_table_keep, ps.npairs, ps.npairs, 0, ps.pair_u, ps.pair_q, ps.t64, seedflag, bound, tab_t, tab_cnt,
             keep);
    return hipGetLastError();
}
hipError_t q_tqb_bounds(int64_t n, int nq, int64_t m, const double *t64, const double *tab_t, const uint32_t *tab_cnt,
                        uint64_t *key_lo, uint64_t *key_hi, double *est, hipStream_t st) {
    if (n <= 0 || nq <= 0) return hipSuccess;
    // enough workgroups to fill the chip (about 2048), each with as many
    // query tiles as that allows
    const int64_t gx = (n + TQB_U - 1) / TQB_U, ntile = (nq + 31) / 32;
    const int64_t gy_want = std::max<int64_t>(1, std::min<int64_t>(ntile, (2048 + gx - 1) / gx));
    const int qt_per = (int)((ntile + gy_want - 1) / gy_want);
    const unsigned gy = (unsigned)((ntile + qt_per - 1) / qt_per);
    hipLaunchKernelGGL(k_tqb_bounds, dim3((unsigned)gx, gy), dim3(256), 0, st, n, nq, m, t64, tab_t, tab_cnt, key_lo,
                       key_hi, est, qt_per);
    return hipGetLastError();
}
hipError_t q_tqb_kth(int nq, const int32_t *k, const double *c, const uint64_t *sel_lo, const uint64_t *sel_hi,
                     const int64_t *sel_off, uint32_t *R_lo, uint32_t *R_hi, int32_t *first_case, hipStream_t st,
                     int fk) {
    LAUNCH1D(k_tqb_kth, nq, nq, k, c, sel_lo, sel_hi, sel_off, R_lo, R_hi, first_case, fk);
    return hipGetLastError();
}
hipError_t q_tqb_classify(int64_t n, int nq, const double *c, const uint32_t *R_lo, const uint32_t *R_hi,
                          const int32_t *first_case, const uint64_t *key_lo, const uint64_t *key_hi, const double *est,
                          uint64_t *key_c, uint64_t *key_t, unsigned long long *nadm, hipStream_t st, int fk) {
    if (n <= 0 || nq <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_tqb_classify, dim3((unsigned)((n + 255) / 256), (unsigned)nq), dim3(256), 0, st, n, c, R_lo,
                       R_hi, first_case, key_lo, key_hi, est, key_c, key_t, nadm, fk);
    return hipGetLastError();
}
hipError_t q_tqb_answer(int nq, int64_t n, int64_t total, const int64_t *off, const int32_t *first_case,
                        const int64_t *sel_off, const uint64_t *sel_hi, const int32_t *nc, const int64_t *off_c,
                        const uint64_t *sel_c, const int64_t *off_t, const uint64_t *sel_t, const double *est,
                        int32_t *ids, double *est_out, hipStream_t st, int fk) {
    LAUNCH1D(k_tqb_answer, total, nq, n, off, first_case, sel_off, sel_hi, nc, off_c, sel_c, off_t, sel_t, est, ids,
             est_out, fk);
    return hipGetLastError();
}
hipError_t q_round_up_f32(const double *x, int64_t n, float *out, hipStream_t st) {
    LAUNCH1D(k_round_up_f32, n, x, n, out);
    return hipGetLastError();
}

}  // namespace rkr
