// kernels.h -- host-side helpers shared by the runtime and the launchers.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <vector>

#include "rkr_internal.h"

namespace rkr {

// Growable device buffer.
struct DBuf {
    void *p = nullptr;
    size_t cap = 0;
    hipError_t ensure(size_t bytes) {
        if (bytes <= cap) return hipSuccess;
        if (p) { (void)hipFree(p); p = nullptr; cap = 0; }
        size_t want = bytes < 256 ? 256 : bytes;
        hipError_t e = hipMalloc(&p, want);
        if (e != hipSuccess) { p = nullptr; return e; }
        cap = want;
        return hipSuccess;
    }
    void release() { if (p) (void)hipFree(p); p = nullptr; cap = 0; }
    template <typename T> T *as() const { return (T *)p; }
};

// Bump allocator over persistent device blocks; reset() rewinds between calls.
struct Scratch {
    struct Block { void *p; size_t size, used; };
    std::vector<Block> blocks;
    void reset() { for (auto &b : blocks) b.used = 0; }
    void *take(int64_t bytes) {
        if (bytes <= 0) bytes = 256;
        size_t need = ((size_t)bytes + 255) & ~(size_t)255;
        for (auto &b : blocks)
            if (b.size - b.used >= need) { void *r = (char *)b.p + b.used; b.used += need; return r; }
        size_t sz = need > ((size_t)256 << 20) ? need : ((size_t)256 << 20);
        void *p = nullptr;
        if (hipMalloc(&p, sz) != hipSuccess) return nullptr;
        blocks.push_back({p, sz, need});
        return p;
    }
    void release() { for (auto &b : blocks) (void)hipFree(b.p); blocks.clear(); }
};

// The (user, query) pairs of one call, numbered user-major:
//   pairs of user u are pids [pair_off[u], pair_off[u+1]).
struct PairSet {
    int64_t npairs = 0;
    int nq = 0;
    int dense = 1;              // 1: every user x every query, pid = u * nq + q
    int32_t *pair_u = nullptr, *pair_q = nullptr;
    int64_t *pair_off = nullptr;    // CSR only: [n + 1]
    int32_t *qm_pid = nullptr;      // CSR only: pid of query-major candidate j
    double *t64 = nullptr;   // FP64 threshold per pair
};

// Entry lists of a set of tasks (one task = one user and its live pairs).
struct TaskSet {
    int64_t ntask = 0, ntask_pad = 0, cap_total = 0;
    int64_t nusers = 0;   // distinct users of the tasks (a user may hold several tasks)
    const int64_t *d_nusers = nullptr;   // single-pair task sets: the same count, left on the device
    DBuf b_user, b_len, b_base, b_pid, b_q, b_cnt, b_th, b_tl, b_tm;
    int32_t *task_user = nullptr, *len = nullptr;
    int64_t *blk_base = nullptr;
    int32_t *ent_pid = nullptr, *ent_q = nullptr;
    uint32_t *ent_cnt = nullptr;
    float *ent_th = nullptr, *ent_tl = nullptr, *ent_tm = nullptr;
    hipError_t reserve(int64_t ntask_pad, int64_t nblk) {
        hipError_t e;
        if ((e = b_user.ensure(ntask_pad * 4)) != hipSuccess) return e;
        if ((e = b_len.ensure(ntask_pad * 4)) != hipSuccess) return e;
        if ((e = b_base.ensure((nblk + 1) * 8)) != hipSuccess) return e;
        task_user = b_user.as<int32_t>();
        len = b_len.as<int32_t>();
        blk_base = b_base.as<int64_t>();
        return hipSuccess;
    }
    hipError_t reserve_entries(int64_t cap, int nsplit = 1) {
        hipError_t e;
        if (nsplit < 1) nsplit = 1;
        if ((e = b_pid.ensure(cap * 4)) != hipSuccess) return e;
        if ((e = b_q.ensure(cap * 4)) != hipSuccess) return e;
        if ((e = b_cnt.ensure(cap * 4 * nsplit)) != hipSuccess) return e;
        if ((e = b_th.ensure(cap * 4)) != hipSuccess) return e;
        if ((e = b_tl.ensure(cap * 4)) != hipSuccess) return e;
        if ((e = b_tm.ensure(cap * 4)) != hipSuccess) return e;
        ent_pid = b_pid.as<int32_t>();
        ent_q = b_q.as<int32_t>();
        ent_cnt = b_cnt.as<uint32_t>();
        ent_th = b_th.as<float>();
        ent_tl = b_tl.as<float>();
        ent_tm = b_tm.as<float>();
        return hipSuccess;
    }
    void release() {
        b_user.release(); b_len.release(); b_base.release(); b_pid.release(); b_q.release();
        b_cnt.release(); b_th.release(); b_tl.release(); b_tm.release();
    }
};

// prep.hip
hipError_t launch_check_values(const void *X, int64_t count, int mk, int *flags, hipStream_t st);
hipError_t launch_spec_norm(const void *X, int64_t rows, int d, int mk, double *out, hipStream_t st);
size_t norm_sort_scratch_bytes(int64_t m);
hipError_t launch_norm_sort(const double *norms, int64_t m, void *scratch, int32_t *order, hipStream_t st);
hipError_t launch_gather_rows(const void *src, const int32_t *order, int64_t rows, int d, int mk, void *dst,
                              hipStream_t st);
// split: 0 = one low-precision value per dimension; 1 / 2 = split BF16 rows
// [hi | hi | lo] (users) / [hi | lo | hi] (items) over 3d of the dpad positions
hipError_t launch_lowprec(const void *X, int64_t rows, int d, int mk, int sk, int dpad, int frag, int split,
                          uint8_t *out, double *norm3, int8_t *exps, hipStream_t st);
hipError_t launch_block_coef(const double *pnorm3, int64_t m, int64_t nblk, double g32, double g64, double cz,
                             double eabs, double *coef, hipStream_t st);
// per 64-item step of the norm-sorted items: an upper bound of |p| from that
// step on (pn: spec norms by item id, order: sorted position -> id)
hipError_t launch_step_znorm(const double *pn, const int32_t *order, int64_t m, int64_t nsteps, double *out,
                             hipStream_t st);
hipError_t launch_step_coef(const double *coef, int64_t nblk, int nib, int64_t nsteps, double *out,
                            hipStream_t st);
// Bounded FP32 thresholds of a dense batch from the BF16 copies (t_up >= the
// FP64 threshold, user-major [u * nq + q]) and the default seed keys
// (query-major), for the rank-table filter; qxyz from launch_query_xyz.
hipError_t launch_query_xyz(const double *qnorm3, int nq, double g32, double g64, float4 *out, hipStream_t st);
hipError_t launch_thresh_approx(const uint8_t *ulp, int64_t n, int dpad, int nks, const double *unorm3,
                                const uint8_t *qlp, int nq, const float4 *qxyz, float *t_up, uint32_t *keys,
                                int num_cus, hipStream_t st);
// (keys: the 32-bit order keys of -t^ / |u|, query-major [q * n + u]; the user
// is the position, for launch_select32)
// FP64 thresholds t64[p] of the listed pairs p = pids[0..N)
hipError_t launch_thresh_list(const int32_t *pids, int64_t N, const int32_t *pair_u, const int32_t *pair_q,
                              const void *Um, const void *Qm, int d, int mk, double *t64, hipStream_t st);
hipError_t launch_thresh(const int32_t *pair_u, const int32_t *pair_q, int64_t npairs, const void *Um,
                         const void *Qm, int d, int mk, double *t64, hipStream_t st);
// with keys (and unorm3), also the default seed keys, query-major [nq][n]
hipError_t launch_thresh_dense(const void *Um, int64_t n, const void *Qm, int nq, int d, int mk, double *t64,
                               hipStream_t st, const double *unorm3 = nullptr, uint64_t *keys = nullptr);
hipError_t launch_recheck_dev(const int2 *rec, const unsigned long long *count, int64_t cap, const int32_t *pair_u,
                              const double *t64, const void *Um, const void *Pm, int d, int mk, uint32_t *cnt,
                              unsigned long long *flips, hipStream_t st);
hipError_t launch_recheck(const int2 *rec, int64_t nrec, const int32_t *pair_u, const double *t64, const void *Um,
                          const void *Pm, int d, int mk, uint32_t *cnt, unsigned long long *flips,
                          hipStream_t st);

// select.hip
hipError_t scan_i32(const int32_t *in, int64_t n, int64_t *out, int64_t *total, Scratch &sc, hipStream_t st);
hipError_t scan_i64(const int64_t *in, int64_t n, int64_t *out, int64_t *total, Scratch &sc, hipStream_t st);
hipError_t launch_select(const uint64_t *keys, const int64_t *seg_off, const int32_t *kk, int64_t nseg,
                         const int64_t *out_off, uint64_t *out, hipStream_t st);
// the same over 32-bit keys whose id is their position in the segment (output
// keys (key << 32 | position), as launch_select's)
hipError_t launch_select32(const uint32_t *keys, const int64_t *seg_off, const int32_t *kk, int64_t nseg,
                           const int64_t *out_off, uint64_t *out, hipStream_t st);
// Tasks of the pairs pids[0..N) (ascending, so each user's pairs are a run):
// one task per user, or, with max_len > 0, one per max_len pairs of a user.
hipError_t build_tasks(const int32_t *pids, int64_t N, const PairSet &ps, int plain, const int32_t *bound,
                       TaskSet &ts, Scratch &sc, hipStream_t st,
                       const uint32_t *rem_init = nullptr, int max_len = 0);
hipError_t launch_iota(int32_t *out, int64_t n, hipStream_t st);
hipError_t launch_dense_pairs(int64_t n, int nq, int32_t *pair_u, int32_t *pair_q, hipStream_t st);
hipError_t build_csr_pairs(const int32_t *cand_ids, const int64_t *cand_off_dev, int nq, int64_t total, int64_t n,
                           PairSet &ps, int *dflags, Scratch &sc, hipStream_t st);

// query.hip (per-call orchestration kernels)
hipError_t launch_fill_u32(uint32_t *p, uint32_t v, int64_t n, hipStream_t st);
hipError_t launch_fill_u8(uint8_t *p, uint8_t v, int64_t n, hipStream_t st);

// count.hip
int max_nks(int sk);
int nks_bucket(int sk, int nks);
int nub_of(int sk, int nks, int variant);
int nib_of(int sk, int nks, int variant);
int num_variants(int sk, int nks);

}  // namespace rkr
