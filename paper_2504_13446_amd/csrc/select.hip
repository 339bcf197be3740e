// select.hip -- segmented k-smallest selection (radix select + bitonic sort in
// LDS), device-wide exclusive scan, and the builders that turn lists of
// (user, query) pairs into the count kernel's block-interleaved entry lists.
#include "rkr_internal.h"
#include "kernels.h"
#include "query.h"

namespace rkr {

static inline unsigned nblocks(int64_t n, int bs) { return (unsigned)((n + bs - 1) / bs); }

// ---------------------------------------------------------------------------
// Exclusive scan (int32 or int64 input -> int64 output), three phases.
// ---------------------------------------------------------------------------
constexpr int SCAN_BS = 256, SCAN_PER = 8, SCAN_TILE = SCAN_BS * SCAN_PER;

template <typename In>
__global__ __launch_bounds__(SCAN_BS) void k_scan_reduce(const In *in, int64_t n, int64_t *sums) {
    __shared__ int64_t s[SCAN_BS];
    int64_t base = (int64_t)blockIdx.x * SCAN_TILE;
    int64_t acc = 0;
    for (int j = 0; j < SCAN_PER; ++j) {
        int64_t i = base + (int64_t)j * SCAN_BS + threadIdx.x;
        if (i < n) acc += (int64_t)in[i];
    }
    s[threadIdx.x] = acc;
    __syncthreads();
    for (int o = SCAN_BS / 2; o > 0; o >>= 1) {
        if (threadIdx.x < o) s[threadIdx.x] += s[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) sums[blockIdx.x] = s[0];
}

// Scan of one tile per block with a carried-in offset per block.
template <typename In>
__global__ __launch_bounds__(SCAN_BS) void k_scan_tile(const In *in, int64_t n, const int64_t *offs,
                                                       int64_t *out) {
    __shared__ int64_t s[SCAN_BS];
    int64_t base = (int64_t)blockIdx.x * SCAN_TILE + (int64_t)threadIdx.x * SCAN_PER;
    int64_t v[SCAN_PER];
    int64_t tot = 0;
    for (int j = 0; j < SCAN_PER; ++j) {
        int64_t i = base + j;
        v[j] = (i < n) ? (int64_t)in[i] : 0;
        tot += v[j];
    }
    s[threadIdx.x] = tot;
    __syncthreads();
    for (int o = 1; o < SCAN_BS; o <<= 1) {
        int64_t t = (threadIdx.x >= o) ? s[threadIdx.x - o] : 0;
        __syncthreads();
        s[threadIdx.x] += t;
        __syncthreads();
    }
    int64_t run = s[threadIdx.x] - tot + (offs ? offs[blockIdx.x] : 0);
    for (int j = 0; j < SCAN_PER; ++j) {
        int64_t i = base + j;
        if (i < n) out[i] = run;
        run += v[j];
    }
}

template <typename In>
__global__ void k_scan_total(const In *in, const int64_t *out, int64_t n, int64_t *total);

template <typename In>
static hipError_t scan_impl(const In *in, int64_t n, int64_t *out, int64_t *total, Scratch &sc,
                            hipStream_t st) {
    if (n <= 0) {
        if (total) { int64_t z = 0; return hipMemcpyAsync(total, &z, 8, hipMemcpyHostToDevice, st); }
        return hipSuccess;
    }
    int64_t nb = (n + SCAN_TILE - 1) / SCAN_TILE;
    if (nb == 1) {
        hipLaunchKernelGGL((k_scan_tile<In>), dim3(1), dim3(SCAN_BS), 0, st, in, n, (const int64_t *)nullptr, out);
    } else {
        int64_t *sums = (int64_t *)sc.take((nb + 1) * 8);
        int64_t *soffs = (int64_t *)sc.take((nb + 1) * 8);
        if (!sums || !soffs) return hipErrorOutOfMemory;
        hipLaunchKernelGGL((k_scan_reduce<In>), dim3((unsigned)nb), dim3(SCAN_BS), 0, st, in, n, sums);
        hipError_t e = scan_impl<int64_t>(sums, nb, soffs, nullptr, sc, st);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL((k_scan_tile<In>), dim3((unsigned)nb), dim3(SCAN_BS), 0, st, in, n,
                           (const int64_t *)soffs, out);
    }
    if (total) {
        // total = out[n-1] + in[n-1]
        hipLaunchKernelGGL(k_scan_total<In>, dim3(1), dim3(1), 0, st, in, out, n, total);
    }
    return hipGetLastError();
}

template <typename In>
__global__ void k_scan_total(const In *in, const int64_t *out, int64_t n, int64_t *total) {
    *total = out[n - 1] + (int64_t)in[n - 1];
}

hipError_t scan_i32(const int32_t *in, int64_t n, int64_t *out, int64_t *total, Scratch &sc, hipStream_t st) {
    return scan_impl<int32_t>(in, n, out, total, sc, st);
}
hipError_t scan_i64(const int64_t *in, int64_t n, int64_t *out, int64_t *total, Scratch &sc, hipStream_t st) {
    return scan_impl<int64_t>(in, n, out, total, sc, st);
}

// ---------------------------------------------------------------------------
// Segmented selection of the K smallest 64-bit keys (keys unique within a
// segment; K <= SEL_MAX, which every caller's limit on k guarantees).  One
// workgroup per segment: radix passes over the segment narrow a bucket
// until the keys at or below it fit in LDS, one more pass gathers them, and a
// bitonic sort orders them; output sorted ascending.  K32: the segment holds
// 32-bit keys whose id is their position in the segment, and the key of
// position i is (key << 32 | i) (the dense seed keys: half the bytes read).
// ---------------------------------------------------------------------------
constexpr int SEL_BS = 1024;
constexpr int SEL_MAX = 4096;
constexpr int SEL_UNROLL = 8;
constexpr int SEL_HIST = 16 * 256;     // histogram counters in LDS

__device__ inline void lds_bitonic_sort(uint64_t *s, int npow2) {
    for (int k = 2; k <= npow2; k <<= 1) {
        for (int j = k >> 1; j > 0; j >>= 1) {
            for (int i = threadIdx.x; i < npow2; i += SEL_BS) {
                int l = i ^ j;
                if (l > i) {
                    uint64_t a = s[i], b = s[l];
                    bool up = (i & k) == 0;
                    if (up ? (a > b) : (a < b)) { s[i] = b; s[l] = a; }
                }
            }
            __syncthreads();
        }
    }
}

template <bool K32>
__global__ __launch_bounds__(SEL_BS) void k_select(const void *keys, const int64_t *seg_off,
                                                   const int32_t *kk, const int64_t *out_off,
                                                   uint64_t *out) {
    __shared__ uint64_t s[SEL_MAX];
    __shared__ uint32_t hist[16][256];
    __shared__ uint32_t sh_cnt;
    __shared__ uint64_t sh_prefix, sh_mask;
    __shared__ int64_t sh_need;
    __shared__ int sh_done, sh_bin;
    __shared__ int64_t sh_cum;
    __shared__ uint32_t sh_wsum[SEL_BS / 64];
    const int seg = blockIdx.x;
    const int64_t b = seg_off[seg], len = seg_off[seg + 1] - b;
    int64_t K = kk[seg];
    if (K > len) K = len;
    const int64_t ob = out_off[seg];
    if (K <= 0) return;
    // loads in flight per thread: twice as many 4-byte keys, so that as many
    // bytes are in flight (the passes are bound by that)
    constexpr int UNR = K32 ? 2 * SEL_UNROLL : SEL_UNROLL;
    const uint64_t *x = (const uint64_t *)keys + b;
    const uint32_t *x32 = (const uint32_t *)keys + b;
    // UNR keys from positions i0 + r * SEL_BS (those past the end are never
    // used): all loads are issued before any key is put together, so that
    // they are in flight at once
    auto load_keys = [&](int64_t i0, uint64_t *v) {
        if constexpr (K32) {
            uint32_t w[UNR];
#pragma unroll
            for (int r = 0; r < UNR; ++r) {
                const int64_t i = i0 + (int64_t)r * SEL_BS;
                w[r] = i < len ? x32[i] : 0u;
            }
#pragma unroll
            for (int r = 0; r < UNR; ++r)
                v[r] = ((uint64_t)w[r] << 32) | (uint64_t)(uint32_t)(i0 + (int64_t)r * SEL_BS);
        } else {
#pragma unroll
            for (int r = 0; r < UNR; ++r) {
                const int64_t i = i0 + (int64_t)r * SEL_BS;
                v[r] = i < len ? x[i] : 0ull;
            }
        }
    };
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;

    uint64_t T;   // select keys <= T
    if (len <= SEL_MAX) {
        T = ~0ull;
    } else {
        if (tid == 0) { sh_prefix = 0; sh_mask = 0; sh_need = K; sh_done = 0; }
        __syncthreads();
        uint32_t *hf = &hist[0][0];
        // Digits: bits 63..53 first (an order key's sign, exponent and two
        // mantissa bits, so one segment's keys spread over many bins), then
        // 8-bit digits, the last of 5 bits.
        int width = 11, shift = 53;
        for (;;) {
            const int nbins = 1 << width;
            const int ncopy = min(16, SEL_HIST / nbins);    // copies of the histogram, shared by waves
            const uint64_t dmask = (uint64_t)(nbins - 1);
            for (int i = tid; i < SEL_HIST; i += SEL_BS) hf[i] = 0;
            if (tid == 0) { sh_bin = 0; sh_cum = 0; }
            __syncthreads();
            const uint64_t pre = sh_prefix, msk = sh_mask;
            uint32_t *hw = hf + (wave % ncopy) * nbins;
            // UNR independent loads in flight per thread
            for (int64_t i0 = tid; i0 < len; i0 += (int64_t)SEL_BS * UNR) {
                uint64_t v[UNR];
                load_keys(i0, v);
#pragma unroll
                for (int r = 0; r < UNR; ++r) {
                    // lanes in the first valid lane's bin add their count in
                    // one atomic (keys that pile into one bin would otherwise
                    // serialise on it); the others add one each
                    const bool valid = i0 + (int64_t)r * SEL_BS < len && (v[r] & msk) == pre;
                    const uint32_t bin = (uint32_t)((v[r] >> shift) & dmask);
                    const uint64_t act = __ballot(valid);
                    if (act == 0) continue;
                    const int lead = __ffsll((long long)act) - 1;
                    const uint32_t b0 = __shfl(bin, lead, 64);
                    const uint64_t same = __ballot(valid && bin == b0);
                    if (valid) {
                        if (bin != b0) atomicAdd(&hw[bin], 1u);
                        else if (lane == lead) atomicAdd(&hw[b0], (uint32_t)__popcll(same));
                    }
                }
            }
            __syncthreads();
            for (int i = tid; i < nbins; i += SEL_BS) {
                uint32_t t = hf[i];
                for (int c = 1; c < ncopy; ++c) t += hf[c * nbins + i];
                hf[i] = t;
            }
            __syncthreads();
            // The bin holding the need-th key: each thread sums a run of
            // `per` bins, and a block-wide prefix sum of the runs names the
            // one run (and then the bin) the need-th key falls in.
            const int per = nbins > SEL_BS ? nbins / SEL_BS : 1;
            const int64_t need = sh_need;
            uint32_t mine = 0;
            if (tid * per < nbins)
                for (int j = 0; j < per; ++j) mine += hf[tid * per + j];
            uint32_t incl = mine;
            for (int o = 1; o < 64; o <<= 1) {
                const uint32_t y = __shfl_up(incl, o, 64);
                if (lane >= o) incl += y;
            }
            if (lane == 63) sh_wsum[wave] = incl;
            __syncthreads();
            uint32_t wpre = 0;
            for (int w = 0; w < wave; ++w) wpre += sh_wsum[w];
            const int64_t before = (int64_t)wpre + incl - mine;    // keys in the bins ahead of this run
            if (mine > 0 && before < need && need <= before + (int64_t)mine) {
                int64_t cum = before;
                int v = tid * per;
                while (cum + (int64_t)hf[v] < need) { cum += hf[v]; ++v; }
                sh_bin = v;
                sh_cum = cum;
            }
            __syncthreads();
            if (tid == 0) {
                const int v = sh_bin;
                const int64_t cum = sh_cum;
                sh_need = need - cum;
                sh_prefix = pre | ((uint64_t)v << shift);
                sh_mask = msk | (dmask << shift);
                // Keys at or below the bucket's upper end: K - (need - cum)
                // below the bucket plus the bucket itself.  They hold the K
                // smallest, so once they fit in LDS the sort finishes the job
                // (no further pass over the segment).
                const int64_t at_or_below = K - (need - cum) + (int64_t)hf[v];
                if ((int64_t)hf[v] == need - cum || at_or_below <= SEL_MAX) sh_done = 1;
            }
            __syncthreads();
            if (sh_done || shift == 0) break;
            width = shift < 8 ? shift : 8;
            shift -= width;
        }
        T = sh_prefix | ~sh_mask;
    }
    if (tid == 0) sh_cnt = 0;
    __syncthreads();
    for (int64_t i0 = tid; i0 < len; i0 += (int64_t)SEL_BS * UNR) {
        uint64_t v[UNR];
        load_keys(i0, v);
#pragma unroll
        for (int r = 0; r < UNR; ++r) {
            if (i0 + (int64_t)r * SEL_BS < len && v[r] <= T) {
                uint32_t p = atomicAdd(&sh_cnt, 1u);
                if (p < SEL_MAX) s[p] = v[r];
            }
        }
    }
    __syncthreads();
    int cnt = (int)min((uint32_t)SEL_MAX, sh_cnt);
    int np2 = 1;
    while (np2 < cnt) np2 <<= 1;
    for (int i = cnt + tid; i < np2; i += SEL_BS) s[i] = ~0ull;
    __syncthreads();
    lds_bitonic_sort(s, np2);
    for (int64_t i = tid; i < K; i += SEL_BS) out[ob + i] = s[i];
}

hipError_t launch_select(const uint64_t *keys, const int64_t *seg_off, const int32_t *kk, int64_t nseg,
                         const int64_t *out_off, uint64_t *out, hipStream_t st) {
    if (nseg <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_select<false>, dim3((unsigned)nseg), dim3(SEL_BS), 0, st, keys, seg_off, kk, out_off, out);
    return hipGetLastError();
}
hipError_t launch_select32(const uint32_t *keys, const int64_t *seg_off, const int32_t *kk, int64_t nseg,
                           const int64_t *out_off, uint64_t *out, hipStream_t st) {
    if (nseg <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_select<true>, dim3((unsigned)nseg), dim3(SEL_BS), 0, st, keys, seg_off, kk, out_off, out);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Task-set builder.  Input: pids[N], ascending (hence grouped by user, since
// pairs are numbered user-major).  Output (TaskSet): one task per distinct
// user, its entry list in block-interleaved layout.  Screening tasks stay in
// user order; exact tasks are grouped by list length (see k_task_permute).
// ---------------------------------------------------------------------------
__global__ void k_user_change(const int32_t *pids, int64_t N, const int32_t *pair_u, int32_t *flag) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    flag[i] = (i == 0 || pair_u[pids[i]] != pair_u[pids[i - 1]]) ? 1 : 0;
}

// excl[i] = number of task starts before i; element i belongs to task
// excl[i] + flag[i] - 1.
__global__ void k_task_starts(const int32_t *pids, int64_t N, const int32_t *pair_u, const int32_t *flag,
                              const int64_t *excl, int64_t *task_start, int32_t *task_user) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N || !flag[i]) return;
    int64_t t = excl[i];
    task_start[t] = i;
    task_user[t] = pair_u[pids[i]];
}

__global__ void k_task_len(const int64_t *task_start, int64_t ntask, int64_t N, int64_t ntask_pad,
                           int32_t *task_user, int32_t *len) {
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= ntask_pad) return;
    if (t < ntask) {
        int64_t e = (t + 1 < ntask) ? task_start[t + 1] : N;
        len[t] = (int32_t)(e - task_start[t]);
    } else {
        len[t] = 0;
        task_user[t] = -1;
    }
}

// Exact passes: tasks with several entries first, then the single-entry
// tasks, each group in user order.  A wave scans as long as its longest list and the waves of a
// workgroup meet at every step's barrier, so a few users with several pairs
// spread over many waves would hold all of them back.
__global__ void k_multi_flag(const int32_t *len, int64_t ntask, int32_t *multi) {
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= ntask) return;
    multi[t] = len[t] > 1 ? 1 : 0;
}

__global__ void k_task_permute(const int64_t *start_in, const int32_t *user_in, const int32_t *len_in,
                               const int32_t *multi, const int64_t *mex, const int64_t *nmulti, int64_t ntask,
                               int64_t *start_out, int32_t *user_out, int32_t *len_out) {
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= ntask) return;
    const int64_t pos = multi[t] ? mex[t] : nmulti[0] + t - mex[t];
    start_out[pos] = start_in[t];
    user_out[pos] = user_in[t];
    len_out[pos] = len_in[t];
}

// Tasks of one pair each: task t holds pair t of the list; blocks of 32
// tasks have one entry slot per task, empty blocks none.
__global__ void k_single_tasks(const int32_t *pids, int64_t N, const int32_t *pair_u, int64_t ntask_pad, int64_t nblk,
                               int64_t nb_used, int64_t *task_start, int32_t *task_user, int32_t *len,
                               int64_t *blk_base) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < ntask_pad) {
        task_user[t] = t < N ? pair_u[pids[t]] : -1;
        len[t] = t < N ? 1 : 0;
    }
    if (t <= N) task_start[t] = t;
    if (t <= nblk) blk_base[t] = 32 * (t < nb_used ? t : nb_used);
}

__global__ void k_block_cap(const int32_t *len, int64_t nblk, int64_t *cap32) {
    int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= nblk) return;
    int32_t mx = 0;
    for (int i = 0; i < 32; ++i) mx = max(mx, len[b * 32 + i]);
    cap32[b] = 32 * (int64_t)mx;
}

// Entry fill, one workgroup per block of 32 tasks, 64 slots per pass through
// an LDS tile: reads run along a task's pairs (consecutive), writes along the
// 32 lanes of a slot (consecutive), so both sides coalesce.  Screening entries
// get (pid, upper edge, remaining budget B[q] - 1); exact entries (pid, both
// edges, fl32(t)) -- their counts start at 0 in the kernel itself.
template <bool SCREEN>
__global__ __launch_bounds__(256) void k_fill_entries(const int32_t *pids, const int64_t *task_start,
                                                      const int32_t *len, int64_t ntask, const int64_t *blk_base,
                                                      int64_t nblk, int64_t cap_total,
                                                      const int32_t *pair_q, const double *t64, int plain,
                                                      const int32_t *bound,
                                                      const uint32_t *rem_init, int32_t *ent_pid,
                                                      uint32_t *ent_cnt, float *ent_th,
                                                      float *ent_tl, float *ent_tm) {
    constexpr int JT = 64;
    __shared__ int32_t s_pid[32][JT + 1];
    __shared__ float s_a[32][JT + 1], s_b[32][JT + 1], s_c[32][JT + 1];
    const int64_t b = blockIdx.x;
    const int tid = threadIdx.x;
    const int64_t base = blk_base[b];
    const int64_t cap = ((b + 1 < nblk ? blk_base[b + 1] : cap_total) - base) / 32;
    for (int64_t j0 = 0; j0 < cap; j0 += JT) {
#pragma unroll
        for (int r = 0; r < 8; ++r) {
            const int l = r * 4 + (tid >> 6), jj = tid & 63;
            const int64_t t = b * 32 + l, j = j0 + jj;
            if (t < ntask && j < len[t]) {
                const int32_t pid = pids[task_start[t] + j];
                s_pid[l][jj] = pid;
                // the FP32 values bracketing t: the smallest float >= t, the
                // largest <= t, and fl32(t); plain mode compares the score
                // with fl32(t) itself (both edges = fl32(t))
                const double tv = t64[pid];
                const float tm = (float)tv;
                s_a[l][jj] = plain ? tm : f32_round_up(tv);
                if constexpr (SCREEN) {
                    // a fresh pair starts with B[q] - 1, a carried one with its remaining budget
                    s_b[l][jj] = __uint_as_float(rem_init ? rem_init[pid] : (uint32_t)(bound[pair_q[pid]] - 1));
                } else {
                    s_b[l][jj] = plain ? tm : f32_round_down(tv);
                    s_c[l][jj] = tm;
                }
            }
        }
        __syncthreads();
#pragma unroll
        for (int r = 0; r < 8; ++r) {
            const int jj = r * 8 + (tid >> 5), l = tid & 31;
            const int64_t t = b * 32 + l, j = j0 + jj;
            if (t < ntask && j < len[t]) {
                const int64_t e = base + j * 32 + l;
                ent_pid[e] = s_pid[l][jj];
                ent_th[e] = s_a[l][jj];
                if constexpr (SCREEN) {
                    ent_cnt[e] = __float_as_uint(s_b[l][jj]);
                } else {
                    ent_tl[e] = s_b[l][jj];
                    ent_tm[e] = s_c[l][jj];
                }
            }
        }
        __syncthreads();
    }
}

// Task starts of a run of one user's pairs cut every max_len pairs: pair i
// (of run excl[i] + flag[i] - 1, which starts at run_start[...]) starts a task
// when its position in the run is a multiple of max_len.
__global__ void k_split_runs(int64_t N, const int32_t *flag, const int64_t *excl, const int64_t *run_start,
                             int max_len, int32_t *flag_out) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    const int64_t pos = i - run_start[excl[i] + flag[i] - 1];
    flag_out[i] = (pos % max_len) == 0 ? 1 : 0;
}

hipError_t build_tasks(const int32_t *pids, int64_t N, const PairSet &ps, int plain, const int32_t *bound,
                       TaskSet &ts, Scratch &sc, hipStream_t st, const uint32_t *rem_init, int max_len) {
    ts.ntask = 0;
    ts.ntask_pad = 0;
    ts.cap_total = 0;
    ts.nusers = 0;
    ts.d_nusers = nullptr;
    if (N <= 0) return hipSuccess;
    hipError_t e;
    int32_t *flag = (int32_t *)sc.take(N * 4);
    int64_t *excl = (int64_t *)sc.take(N * 8);
    int64_t *dtot = (int64_t *)sc.take(16);
    if (!flag || !excl || !dtot) return hipErrorOutOfMemory;
    hipLaunchKernelGGL(k_user_change, dim3(nblocks(N, 256)), dim3(256), 0, st, pids, N, ps.pair_u, flag);
    if ((e = scan_i32(flag, N, excl, dtot, sc, st)) != hipSuccess) return e;
    if (max_len == 1) {
        // every pair is a task of its own: the sizes follow from N, so the
        // lists are laid out with nothing read back (the distinct-user count
        // stays on the device)
        const int64_t ntask = N, ntask_pad = (N + 511) / 512 * 512, nblk = ntask_pad / 32;
        const int64_t nb_used = (N + 31) / 32, cap_total = nb_used * 32;
        if ((e = ts.reserve(ntask_pad, nblk)) != hipSuccess) return e;
        int64_t *task_start = (int64_t *)sc.take((ntask + 1) * 8);
        if (!task_start) return hipErrorOutOfMemory;
        hipLaunchKernelGGL(k_single_tasks, dim3(nblocks(ntask_pad + 1, 256)), dim3(256), 0, st, pids, N, ps.pair_u,
                           ntask_pad, nblk, nb_used, task_start, ts.task_user, ts.len, ts.blk_base);
        if ((e = ts.reserve_entries(cap_total)) != hipSuccess) return e;
        if (bound)
            hipLaunchKernelGGL(k_fill_entries<true>, dim3((unsigned)nblk), dim3(256), 0, st, pids, task_start, ts.len,
                               ntask, ts.blk_base, nblk, cap_total, ps.pair_q, ps.t64, plain, bound,
                               rem_init, ts.ent_pid, ts.ent_cnt, ts.ent_th, ts.ent_tl, ts.ent_tm);
        else
            hipLaunchKernelGGL(k_fill_entries<false>, dim3((unsigned)nblk), dim3(256), 0, st, pids, task_start, ts.len,
                               ntask, ts.blk_base, nblk, cap_total, ps.pair_q, ps.t64, plain, bound,
                               rem_init, ts.ent_pid, ts.ent_cnt, ts.ent_th, ts.ent_tl, ts.ent_tm);
        ts.ntask = ntask;
        ts.ntask_pad = ntask_pad;
        ts.cap_total = cap_total;
        ts.nusers = -1;
        ts.d_nusers = dtot;
        return hipGetLastError();
    }
    int64_t ntask = 0;
    if ((e = hipMemcpyAsync(&ntask, dtot, 8, hipMemcpyDeviceToHost, st)) != hipSuccess) return e;
    if ((e = hipStreamSynchronize(st)) != hipSuccess) return e;
    ts.nusers = ntask;
    if (max_len > 0 && ntask < N) {
        // runs of one user become tasks of at most max_len pairs
        int64_t *run_start = (int64_t *)sc.take((ntask + 1) * 8);
        int32_t *run_user = (int32_t *)sc.take(ntask * 4);
        int32_t *flag2 = (int32_t *)sc.take(N * 4);
        int64_t *excl2 = (int64_t *)sc.take(N * 8);
        if (!run_start || !run_user || !flag2 || !excl2) return hipErrorOutOfMemory;
        hipLaunchKernelGGL(k_task_starts, dim3(nblocks(N, 256)), dim3(256), 0, st, pids, N, ps.pair_u, flag, excl,
                           run_start, run_user);
        hipLaunchKernelGGL(k_split_runs, dim3(nblocks(N, 256)), dim3(256), 0, st, N, flag, excl, run_start, max_len,
                           flag2);
        if ((e = scan_i32(flag2, N, excl2, dtot, sc, st)) != hipSuccess) return e;
        if ((e = hipMemcpyAsync(&ntask, dtot, 8, hipMemcpyDeviceToHost, st)) != hipSuccess) return e;
        if ((e = hipStreamSynchronize(st)) != hipSuccess) return e;
        flag = flag2;
        excl = excl2;
    }
    const int64_t ntask_pad = (ntask + 511) / 512 * 512;
    const int64_t nblk = ntask_pad / 32;
    if ((e = ts.reserve(ntask_pad, nblk)) != hipSuccess) return e;
    int64_t *task_start = (int64_t *)sc.take((ntask + 1) * 8);
    int64_t *cap32 = (int64_t *)sc.take(nblk * 8);
    if (!task_start || !cap32) return hipErrorOutOfMemory;
    hipLaunchKernelGGL(k_task_starts, dim3(nblocks(N, 256)), dim3(256), 0, st, pids, N, ps.pair_u, flag, excl,
                       task_start, ts.task_user);
    hipLaunchKernelGGL(k_task_len, dim3(nblocks(ntask_pad, 256)), dim3(256), 0, st, task_start, ntask, N,
                       ntask_pad, ts.task_user, ts.len);
    if (!bound && ntask > 32) {
        int32_t *multi = (int32_t *)sc.take(ntask * 4);
        int64_t *mex = (int64_t *)sc.take(ntask * 8);
        int64_t *nmulti = (int64_t *)sc.take(16);
        int64_t *start2 = (int64_t *)sc.take((ntask + 1) * 8);
        int32_t *user0 = (int32_t *)sc.take(ntask * 4);
        int32_t *len0 = (int32_t *)sc.take(ntask * 4);
        if (!multi || !mex || !nmulti || !start2 || !user0 || !len0) return hipErrorOutOfMemory;
        hipLaunchKernelGGL(k_multi_flag, dim3(nblocks(ntask, 256)), dim3(256), 0, st, ts.len, ntask, multi);
        if ((e = scan_i32(multi, ntask, mex, nmulti, sc, st)) != hipSuccess) return e;
        if ((e = hipMemcpyAsync(user0, ts.task_user, ntask * 4, hipMemcpyDeviceToDevice, st)) != hipSuccess) return e;
        if ((e = hipMemcpyAsync(len0, ts.len, ntask * 4, hipMemcpyDeviceToDevice, st)) != hipSuccess) return e;
        hipLaunchKernelGGL(k_task_permute, dim3(nblocks(ntask, 256)), dim3(256), 0, st, task_start, user0, len0,
                           multi, mex, nmulti, ntask, start2, ts.task_user, ts.len);
        task_start = start2;
    }
    hipLaunchKernelGGL(k_block_cap, dim3(nblocks(nblk, 256)), dim3(256), 0, st, ts.len, nblk, cap32);
    if ((e = scan_i64(cap32, nblk, ts.blk_base, dtot, sc, st)) != hipSuccess) return e;
    int64_t cap_total = 0;
    if ((e = hipMemcpyAsync(&cap_total, dtot, 8, hipMemcpyDeviceToHost, st)) != hipSuccess) return e;
    if ((e = hipStreamSynchronize(st)) != hipSuccess) return e;
    if ((e = ts.reserve_entries(cap_total)) != hipSuccess) return e;
    if (bound)
        hipLaunchKernelGGL(k_fill_entries<true>, dim3((unsigned)nblk), dim3(256), 0, st, pids, task_start, ts.len,
                           ntask, ts.blk_base, nblk, cap_total, ps.pair_q, ps.t64, plain, bound,
                           rem_init, ts.ent_pid, ts.ent_cnt, ts.ent_th, ts.ent_tl, ts.ent_tm);
    else
        hipLaunchKernelGGL(k_fill_entries<false>, dim3((unsigned)nblk), dim3(256), 0, st, pids, task_start, ts.len,
                           ntask, ts.blk_base, nblk, cap_total, ps.pair_q, ps.t64, plain, bound,
                           rem_init, ts.ent_pid, ts.ent_cnt, ts.ent_th, ts.ent_tl, ts.ent_tm);
    ts.ntask = ntask;
    ts.ntask_pad = ntask_pad;
    ts.cap_total = cap_total;
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Small element-wise helpers.
// ---------------------------------------------------------------------------
__global__ void k_iota(int32_t *out, int64_t n) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] = (int32_t)i;
}
hipError_t launch_iota(int32_t *out, int64_t n, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_iota, dim3(nblocks(n, 256)), dim3(256), 0, st, out, n);
    return hipGetLastError();
}

// Dense domain pairs: pid = u * nq + q.
__global__ void k_dense_pairs(int64_t n, int nq, int32_t *pair_u, int32_t *pair_q) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n * nq) return;
    pair_u[i] = (int32_t)(i / nq);
    pair_q[i] = (int32_t)(i % nq);
}
hipError_t launch_dense_pairs(int64_t n, int nq, int32_t *pair_u, int32_t *pair_q, hipStream_t st) {
    int64_t N = n * nq;
    if (N <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_dense_pairs, dim3(nblocks(N, 256)), dim3(256), 0, st, n, nq, pair_u, pair_q);
    return hipGetLastError();
}

// CSR (query-major candidate lists) -> user-major pairs.
// 1) per-user counts, 2) scan -> pair_off, 3) scatter with a cursor, 4) sort
// each user's pairs by query (insertion sort; lists are short) so the layout
// is deterministic.  qm_pid[j] = pid of the j-th query-major candidate.
__global__ void k_csr_count(const int32_t *cand_ids, int64_t total, int32_t *ucount) {
    int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j < total) atomicAdd(&ucount[cand_ids[j]], 1);
}
__global__ void k_csr_scatter(const int32_t *cand_ids, const int64_t *cand_off, int nq, int64_t total,
                              const int64_t *pair_off, int32_t *cursor, int32_t *pair_u, int32_t *pair_q) {
    int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= total) return;
    // query of position j: binary search in cand_off
    int lo = 0, hi = nq;   // cand_off[lo] <= j < cand_off[hi]
    while (hi - lo > 1) {
        int mid = (lo + hi) >> 1;
        if (cand_off[mid] <= j) lo = mid; else hi = mid;
    }
    int u = cand_ids[j];
    int64_t p = pair_off[u] + atomicAdd(&cursor[u], 1);
    pair_u[p] = u;
    pair_q[p] = lo;
}
__global__ void k_csr_sort_users(const int64_t *pair_off, int64_t n, int32_t *pair_q) {
    int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (u >= n) return;
    int64_t b = pair_off[u], e = pair_off[u + 1];
    for (int64_t i = b + 1; i < e; ++i) {
        int32_t v = pair_q[i];
        int64_t j = i - 1;
        while (j >= b && pair_q[j] > v) { pair_q[j + 1] = pair_q[j]; --j; }
        pair_q[j + 1] = v;
    }
}
// qm_pid: for query q's candidate list position j, find pid by binary search
// of q within user u's (sorted) pair_q segment.
__global__ void k_csr_qm_pid(const int32_t *cand_ids, const int64_t *cand_off, int nq, int64_t total,
                             const int64_t *pair_off, const int32_t *pair_q, int32_t *qm_pid) {
    int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= total) return;
    int lo = 0, hi = nq;
    while (hi - lo > 1) {
        int mid = (lo + hi) >> 1;
        if (cand_off[mid] <= j) lo = mid; else hi = mid;
    }
    int u = cand_ids[j];
    int64_t b = pair_off[u], e = pair_off[u + 1];
    while (e - b > 1) {
        int64_t mid = (b + e) >> 1;
        if (pair_q[mid] <= lo) b = mid; else e = mid;
    }
    qm_pid[j] = (int32_t)b;
}
// duplicate / range validation of candidate lists: bit 1 = id out of range,
// bit 2 = duplicate within a list (lists need not be sorted).
__global__ void k_csr_validate(const int32_t *cand_ids, int64_t total, int64_t n, int *flags) {
    int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= total) return;
    int u = cand_ids[j];
    if (u < 0 || u >= n) atomicOr(flags, 1);
}
__global__ void k_csr_dupcheck(const int64_t *pair_off, int64_t n, const int32_t *pair_q, int *flags) {
    int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (u >= n) return;
    for (int64_t i = pair_off[u] + 1; i < pair_off[u + 1]; ++i)
        if (pair_q[i] == pair_q[i - 1]) { atomicOr(flags, 2); return; }
}

hipError_t build_csr_pairs(const int32_t *cand_ids, const int64_t *cand_off_dev, int nq, int64_t total,
                           int64_t n, PairSet &ps, int *dflags, Scratch &sc, hipStream_t st) {
    hipError_t e;
    int32_t *ucount = (int32_t *)sc.take(n * 4);
    int32_t *cursor = (int32_t *)sc.take(n * 4);
    int64_t *dtot = (int64_t *)sc.take(16);
    if (!ucount || !cursor || !dtot) return hipErrorOutOfMemory;
    if ((e = hipMemsetAsync(ucount, 0, n * 4, st)) != hipSuccess) return e;
    if ((e = hipMemsetAsync(cursor, 0, n * 4, st)) != hipSuccess) return e;
    hipLaunchKernelGGL(k_csr_validate, dim3(nblocks(total, 256)), dim3(256), 0, st, cand_ids, total, n, dflags);
    int flags = 0;
    if ((e = hipMemcpyAsync(&flags, dflags, 4, hipMemcpyDeviceToHost, st)) != hipSuccess) return e;
    if ((e = hipStreamSynchronize(st)) != hipSuccess) return e;
    if (flags) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_csr_count, dim3(nblocks(total, 256)), dim3(256), 0, st, cand_ids, total, ucount);
    if ((e = scan_i32(ucount, n, ps.pair_off, dtot, sc, st)) != hipSuccess) return e;
    // pair_off[n] = total
    if ((e = hipMemcpyAsync(ps.pair_off + n, &total, 8, hipMemcpyHostToDevice, st)) != hipSuccess) return e;
    hipLaunchKernelGGL(k_csr_scatter, dim3(nblocks(total, 256)), dim3(256), 0, st, cand_ids, cand_off_dev, nq,
                       total, ps.pair_off, cursor, ps.pair_u, ps.pair_q);
    hipLaunchKernelGGL(k_csr_sort_users, dim3(nblocks(n, 256)), dim3(256), 0, st, ps.pair_off, n, ps.pair_q);
    hipLaunchKernelGGL(k_csr_dupcheck, dim3(nblocks(n, 256)), dim3(256), 0, st, ps.pair_off, n, ps.pair_q, dflags);
    hipLaunchKernelGGL(k_csr_qm_pid, dim3(nblocks(total, 256)), dim3(256), 0, st, cand_ids, cand_off_dev, nq,
                       total, ps.pair_off, ps.pair_q, ps.qm_pid);
    if ((e = hipMemcpyAsync(&flags, dflags, 4, hipMemcpyDeviceToHost, st)) != hipSuccess) return e;
    if ((e = hipStreamSynchronize(st)) != hipSuccess) return e;
    if (flags) return hipErrorInvalidValue;
    return hipGetLastError();
}

}  // namespace rkr
