// count.hip -- fused low-precision score + rank count (the O(nmd) scan of
// Def. 1, Sec. 2, done as a tiled U.P^T on the matrix cores).
//
// One workgroup = 8 wave64.  A wave owns NUB blocks of 32 users; the users'
// low-precision vectors stay in registers for the whole scan (B operand).
// Items stream through LDS in steps of NIB blocks of 32 items, stored in
// global memory already in MFMA fragment order so that both the global->LDS
// copy and the LDS->register fragment reads are linear.  A 32x32 MFMA output
// block leaves, in lane l, the scores of user (l % 32) against 16 items; the
// lane pair (l, l+32) covers all 32 items of the block.
//
// Each (user, query) pair of the wave's users is an "entry" (block-interleaved
// SoA arrays, see CountArgs).  For every step the lane loops over its user's
// live entries and compares each of its scores with the pair's band edges:
//   hi = next_up(th + eps),  lo = next_down(tl - eps)
// where th >= t64 >= tl bracket the FP64 threshold and eps bounds
// |score - s64(u,p)| for every item of the step (error-bound coefficients per
// item block; P is sorted by norm so the per-block maxima are tight).
//   score >  hi  => s64(u,p) > t64   (certainly above: counted)
//   score <  lo  => s64(u,p) < t64   (certainly not above)
//   otherwise       near tie: exact mode emits (pair, item) for the FP64 recheck.
// Screen mode counts only certain-above scores and drops a pair as soon as
// 1 + count exceeds the query's bound B[q] (a proven upper bound on the k-th
// smallest rank): its rank is then > B >= R_k, so it cannot be in the answer
// (Def. 2), the counts only grow.  A screen split over item ranges (blockIdx.y)
// gives every split its own copy of the lists; a split's partial count above
// the budget already proves the pair out, and the host merges the splits'
// lists after the launch.  This is the paper's Lemma 1 (2) filter
// applied to exact partial counts.  A screen entry holds (pid, th, rem) with
// rem = B[q] - 1 - count: the pair dies when rem turns negative; survivors are
// compacted to the front of the user's list every step.  With enough live
// entries the screen compares 7-bit monotone codes of the scores instead of
// the scores (a lower bound of the certain count, four compares per dword).
// Table mode builds the rank table's cells (Sec. 4.2): every user carries its
// TABLE_COLS thresholds in registers and counts, for each, the scores
// certainly above it over all of P; near ties are left uncounted (the cells
// are lower bounds of the exact counts) and nothing is emitted.
#include "rkr_internal.h"
#include "tile_common.h"

#include <algorithm>
#include <cstdlib>

namespace rkr {


// Screening compares scores as 7-bit codes once some lane of the wave holds
// this many live entries (below it, quantising costs more than it saves).
constexpr int SWAR_MIN_ENTRIES = 4;

// Bucketed counting for screens with many live entries per user: the step's
// codes of a user (both lanes of its pair) go into a 128-bin LDS histogram,
// turned into suffix sums, so an entry's count of codes above its
// threshold's code is one byte read instead of a compare over every code.
// 128 one-byte bins per user (a byte never overflows: at most 128 codes per
// pair), at a stride of 33 words so that the 32 users of a wave that update
// the same bin do so in different LDS banks.
constexpr int HIST_STRIDE = 132;
template <int MODE, int NUB>
constexpr int hist_bytes() {
    return MODE == CM_SCREEN ? WAVES_PER_WG * NUB * USER_BLOCK * HIST_STRIDE : 0;
}

// acc += median(a, b, c) for unsigned integers: two VALU instructions (the
// compiler only forms the median from min/max when it can order the bounds
// itself, and left to itself it keeps every median of a step live before
// summing them).
__device__ inline void add_med3_u32(uint32_t &acc, uint32_t a, uint32_t b, uint32_t c) {
    uint32_t t;
    asm("v_med3_u32 %1, %2, %3, %4\n\tv_add_u32 %0, %0, %1" : "+v"(acc), "=&v"(t) : "v"(a), "v"(b), "v"(c));
}

// LDS stages of P: the exact and table passes (little work per step) keep up
// to five stages, screening (long steps) double-buffers.  150 KB of LDS at most.
// Exact passes also keep a near-tie record buffer per wave in LDS (REC_PER_WAVE).
template <int MODE>
constexpr int record_bytes() {
    return MODE == CM_EXACT ? WAVES_PER_WG * REC_PER_WAVE * 8 : 0;
}
template <int MODE>
constexpr int stage_buffers(int step_bytes) {
    if (MODE == CM_SCREEN) return 2;
    const int nb = (153600 - record_bytes<MODE>()) / step_bytes;
    return nb < 2 ? 2 : (nb > 5 ? 5 : nb);
}
// Staging loads the last wave of a workgroup issues per step (the fewest of
// any wave): a lower bound on the vector-memory operations a step's staging
// adds to every wave's counter.
constexpr int stage_loads_min(int step_bytes) {
    int c = 0;
    for (int j = 0; j < 64; ++j)
        if ((j * 512 + (WAVES_PER_WG - 1) * 64) * 16 < step_bytes) ++c;
    return c;
}
template <int SK, int MODE, int NKS, int NUB, int NIB>
__device__ inline void count_tile(const CountArgs &a, const int64_t tile, uint8_t *lds, uint64_t &ncmp,
                                  uint64_t &nslot, uint64_t &nstep, uint64_t &nscored) {
    using FT = typename FragT<SK>::T;
    constexpr int FB = frag_fb(SK);
    constexpr int KS = frag_ks(SK);
    constexpr int ES = elem_size(SK);
    constexpr int TASKS_PER_WG = WAVES_PER_WG * NUB * USER_BLOCK;
    constexpr int STEP_BYTES_MAX = NIB * NKS * 64 * FB;
    constexpr int LOADS_MAX = (STEP_BYTES_MAX + 512 * 16 - 1) / (512 * 16);

    constexpr int step_bytes = STEP_BYTES_MAX;
    constexpr int STAGE = STEP_BYTES_MAX + 32;     // P tile + the step's coefficients
    constexpr int NBUF = stage_buffers<MODE>(STAGE);
    // Screening stages the next step and meets at a barrier after every step.
    // Exact and table passes with four or more stages stage PF = NBUF - 2
    // steps ahead and meet after every second step: step st writes the stage
    // of step st - 2, which every wave has left by then (a barrier follows
    // st - 2 or st - 1), and at a barrier the next two steps have landed.
    constexpr bool SYNC2 = MODE != CM_SCREEN && NBUF >= 4;
    constexpr int PF = SYNC2 ? NBUF - 2 : NBUF - 1;
    // at a barrier, the staging of at most this many later operations may
    // still be in flight (each step adds >= stage_loads_min per wave)
    constexpr int WAIT_N = (SYNC2 ? PF - 2 : PF - 1) * stage_loads_min(STEP_BYTES_MAX);
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;
    const int l32 = lane & 31;
    const int half = lane >> 5;
    const int split = blockIdx.y;

    int64_t s_begin = a.step0 + (int64_t)split * a.steps_per_split;
    int64_t s_end = s_begin + a.steps_per_split;
    if (s_end > a.step_end) s_end = a.step_end;

    // ---- this lane's users, their register-stationary fragments and entries
    int uid[NUB];
    int64_t tix[NUB];
    int len[NUB];
    int64_t ebase[NUB];
    double un_hat[NUB], un_del[NUB], un_full[NUB];
    int uscale[NUB];
    float fth[NUB];   // bound check: the folded threshold (0 without)
    FT bfrag[NUB][NKS];
#pragma unroll
    for (int ub = 0; ub < NUB; ++ub) {
        int64_t t = tile * TASKS_PER_WG + (wave * NUB + ub) * USER_BLOCK + l32;
        tix[ub] = t;
        int u;
        if constexpr (MODE == CM_TABLE || MODE == CM_BOUND) {
            u = (t < a.ntask) ? (int)t : -1;
            len[ub] = (u >= 0) ? (MODE == CM_TABLE ? TABLE_COLS : 1) : 0;
            ebase[ub] = 0;
        } else {
            u = (t < a.ntask) ? a.task_user[t] : -1;
            len[ub] = (u >= 0) ? a.ent_len[split * a.len_stride + t] : 0;
            ebase[ub] = a.blk_base[t >> 5] + l32;
            // a split screen works on its own copy of the lists
            if constexpr (MODE == CM_SCREEN) ebase[ub] += (int64_t)split * a.cap_total;
        }
        uid[ub] = u;
        fth[ub] = (MODE == CM_BOUND && a.fold_th && u >= 0) ? a.fold_th[u] : 0.0f;
        un_hat[ub] = un_del[ub] = un_full[ub] = 0.0;
        uscale[ub] = 127;
        if (u >= 0) {
            un_hat[ub] = a.unorm3[3 * (int64_t)u + 0];
            un_del[ub] = a.unorm3[3 * (int64_t)u + 1];
            un_full[ub] = a.unorm3[3 * (int64_t)u + 2];
            if constexpr (SK == SK_FP8) uscale[ub] = 127 + (int)a.uexp[u];
        }
        const uint8_t *urow = a.ulp + ((int64_t)(u >= 0 ? u : 0) * a.dpad + half * (KS / 2)) * ES;
#pragma unroll
        for (int s = 0; s < NKS; ++s) {
            FT v{};
            if (u >= 0) v = *(const FT *)(urow + (int64_t)s * KS * ES);
            bfrag[ub][s] = v;
        }
    }

    // Screening pass over the live entries of user block ub for the current
    // step: count(hi) returns the lane's number of scores certainly above hi
    // (a lower bound of the exact count); entries whose remaining budget turns
    // negative are dropped, the others are compacted to the front.
    // Entry fields are addressed by 32-bit byte offsets from the array bases
    // (the host keeps every entry array below 4 GiB).
    uint32_t ebyte[NUB];
#pragma unroll
    for (int ub = 0; ub < NUB; ++ub) ebyte[ub] = (uint32_t)ebase[ub] * 4u;
    auto ld_i32 = [](const void *base, uint32_t off) { return *(const int32_t *)((const uint8_t *)base + off); };
    auto ld_f32 = [](const void *base, uint32_t off) { return *(const float *)((const uint8_t *)base + off); };
    auto st_u32 = [](void *base, uint32_t off, uint32_t v) { *(uint32_t *)((uint8_t *)base + off) = v; };

    // The fields of a group of ED entries load while the previous group is
    // counted; a step's first group is requested before its scores are
    // computed, so the matrix-core work hides that latency.
    //
    // The loop over entries runs nit (the wave's longest list, uniform)
    // iterations; every lane loads slot i (slots below nit exist for every
    // lane of the block: a block's lists were laid out for its longest initial
    // list).  A live entry is written back only if it moves down to slot w < i
    // (all fields) or stays and its budget changed (the budget); a dead entry,
    // or a lane past its own list, writes nothing, since the list ends at w.
    // The two lanes of a pair write identical values.
    constexpr int ED = 4;
    int g0_pid[NUB][ED], g0_rem[NUB][ED];
    float g0_th[NUB][ED];
    int nit[NUB];
    auto wave_max = [](int v) {
#pragma unroll
        for (int o = 32; o >= 1; o >>= 1) v = max(v, __shfl_xor(v, o, 64));
        return __builtin_amdgcn_readfirstlane(v);
    };
    auto fetch_into = [&](int ub, int i0, int *pid, int *rem, float *th) {
#pragma unroll
        for (int k = 0; k < ED; ++k) {
            const int i = i0 + k;
            if (i < nit[ub]) {
                const uint32_t o = ebyte[ub] + (uint32_t)i * 128u;
                pid[k] = ld_i32(a.ent_pid, o);
                th[k] = ld_f32(a.ent_th, o);
                rem[k] = ld_i32(a.ent_cnt, o);
            }
        }
    };
    // first group of the current lists (sets nit)
    auto fetch_first = [&](int ub) {
        nit[ub] = wave_max(len[ub]);
        fetch_into(ub, 0, g0_pid[ub], g0_rem[ub], g0_th[ub]);
    };

    // Screening pass over the live entries of user block ub for the current
    // step: count(hi) returns the lane's number of scores certainly above hi
    // (a lower bound of the exact count); entries whose remaining budget turns
    // negative are dropped, the others are compacted to the front.
    auto screen_entries = [&](int ub, float eps, auto count, bool paired) {
        int w = 0;
        const int mylen = len[ub];
        const int lim = nit[ub];
        int pid_n[ED], rem_n[ED];
        float th_n[ED];
#pragma unroll
        for (int k = 0; k < ED; ++k) {
            pid_n[k] = g0_pid[ub][k];
            rem_n[k] = g0_rem[ub][k];
            th_n[k] = g0_th[ub][k];
        }
        for (int i0 = 0; i0 < lim; i0 += ED) {
            // take the group's fields before the next group's loads overwrite them
            int pid_c[ED], rem_c[ED];
            float th_c[ED];
#pragma unroll
            for (int k = 0; k < ED; ++k) {
                pid_c[k] = pid_n[k];
                rem_c[k] = rem_n[k];
                th_c[k] = th_n[k];
            }
            fetch_into(ub, i0 + ED, pid_n, rem_n, th_n);
#pragma unroll
            for (int k = 0; k < ED; ++k) {
                const int i = i0 + k;
                if (i < lim) {
                    const bool act = i < mylen;
                    const float hb = f32_next_up(th_c[k] + eps);
                    const float hi = a.plain ? th_c[k] : hb;
                    // paired: count gives the pair's total, else the lane's
                    const uint32_t c = paired ? count(hi) : pair_sum(count(hi));
                    // remaining budget: the pair dies when more than bound - 1 items are certainly above
                    const int rem = rem_c[k] - (int)c;
                    const bool alive = act && rem >= 0;
                    // only what changes is written: an entry that moves down
                    // to slot w, or the budget of one that stays; slots from w
                    // on are past the list and never read
                    if (alive) {
                        const uint32_t ow = ebyte[ub] + (uint32_t)w * 128u;
                        if (w != i) {
                            st_u32(a.ent_cnt, ow, (uint32_t)rem);
                            st_u32(a.ent_pid, ow, (uint32_t)pid_c[k]);
                            st_u32(a.ent_th, ow, __float_as_uint(th_c[k]));
                        } else if (c != 0) {
                            st_u32(a.ent_cnt, ow, (uint32_t)rem);
                        }
                    }
                    w += alive ? 1 : 0;
                }
            }
        }
        len[ub] = w;
        ncmp += (uint64_t)mylen * (NIB * 16);
        nslot += (uint64_t)lim * (NIB * 16);
    };

    // Exact passes: this wave's near-tie record buffer (LDS, after the P
    // stages) and its fill count (uniform); flushed when full and at the end.
    int2 *const recbuf = (int2 *)(lds + NBUF * STAGE) + wave * REC_PER_WAVE;
    int rb_n = 0;
    auto flush_records = [&]() {
        if (rb_n == 0) return;
        unsigned long long base = 0;
        if (lane == 0) base = atomicAdd(a.emit_count, (unsigned long long)rb_n);
        base = __shfl(base, 0, 64);
        for (int i = lane; i < rb_n; i += 64)
            if (base + (unsigned long long)i < a.emit_cap) a.emit[base + i] = recbuf[i];
        rb_n = 0;
    };

    // Exact passes: the first EC entries of each lane's list stay in registers
    // (fields and running count) for the whole scan; most lists of the seed,
    // refine and all-ranks passes hold one or two pairs.
    constexpr int EC = MODE == CM_EXACT ? 2 : 0;
    int rpid[NUB][EC > 0 ? EC : 1];
    float rth[NUB][EC > 0 ? EC : 1], rtl[NUB][EC > 0 ? EC : 1], rtm[NUB][EC > 0 ? EC : 1];
    uint32_t rcnt[NUB][EC > 0 ? EC : 1];
#pragma unroll
    for (int ub = 0; ub < NUB; ++ub)
#pragma unroll
        for (int k = 0; k < EC; ++k) {
            rcnt[ub][k] = 0;
            rpid[ub][k] = 0;
            rth[ub][k] = rtl[ub][k] = rtm[ub][k] = 0.0f;
            if (k < len[ub]) {
                const int64_t e = ebase[ub] + (int64_t)k * 32;
                rpid[ub][k] = a.ent_pid[e];
                rth[ub][k] = a.ent_th[e];
                rtl[ub][k] = a.ent_tl[e];
                rtm[ub][k] = a.ent_tm[e];
            }
        }

    // Table passes: the user's TABLE_COLS thresholds and running counts stay
    // in registers for the whole scan.
    constexpr int TC = MODE == CM_TABLE ? TABLE_COLS : 1;
    float tth[NUB][TC];
    uint32_t tcnt[NUB][TC];
#pragma unroll
    for (int ub = 0; ub < NUB; ++ub)
#pragma unroll
        for (int j = 0; j < TC; ++j) {
            tcnt[ub][j] = 0;
            tth[ub][j] = 0.0f;
            if constexpr (MODE == CM_TABLE)
                if (uid[ub] >= 0) tth[ub][j] = a.ent_th[(int64_t)uid[ub] * TABLE_COLS + j];
        }

    double bound_max = 0.0;     // bound check only
    uint32_t bound_over = 0;
    int any_live = 0;
#pragma unroll
    for (int ub = 0; ub < NUB; ++ub) any_live |= (len[ub] > 0);
    if (!__syncthreads_or(any_live) || s_begin >= s_end) return;

    // ---- prologue: stage the first PF steps (direct global -> LDS, 16 bytes
    // per lane); wait for the first (the first two with SYNC2)
    const int64_t npro = std::min<int64_t>(PF, s_end - s_begin);
    for (int64_t k = 0; k < npro; ++k)
        stage_step<LOADS_MAX>(a.plp + (s_begin + k) * (int64_t)step_bytes, lds + k * STAGE, step_bytes, tid,
                              a.step_coef + 4 * (s_begin + k));
    if (npro == PF)
        wait_vm<WAIT_N>();
    else
        wait_vm<0>();
    // "any list still live" flags of the step-end barrier: one slot per step,
    // three in rotation; the slot of step k - 1 is cleared after the barrier
    // of step k (every read of it precedes that barrier) and reused at step
    // k + 2 (whose writes follow the barrier of step k + 1)
    __shared__ int wg_live[3];
    if (tid < 3) wg_live[tid] = 0;
    int lslot = 0;
    __syncthreads();
    int cbuf = 0;   // LDS stage holding step st

    // Screening, second half of the workgroup: its waves count a step's codes
    // at the start of the next step, before their matrix-core work, so that on
    // a SIMD one wave's MFMA overlaps the other wave's compare loop.
    constexpr int QW = NIB * 4;
    uint32_t qd_p[NUB][QW];
    float mn_p[NUB], sc_p[NUB], eps_p[NUB];
    bool hist_p[NUB];
#pragma unroll
    for (int ub = 0; ub < NUB; ++ub) hist_p[ub] = false;
    bool have_prev = false;
    const bool late = MODE == CM_SCREEN && wave >= WAVES_PER_WG / 2;
    // this lane pair's histogram of user block ub (screening only)
    uint8_t *const hist_lds = lds + NBUF * STAGE + record_bytes<MODE>();
    auto hist_of = [&](int ub) { return hist_lds + ((wave * NUB + ub) * USER_BLOCK + l32) * HIST_STRIDE; };
    // The pair's codes into the histogram (bin b = code - 128), then in place
    // the suffix counts SS[b] = #{codes of the pair with bin > b}.  Only this
    // wave touches its histograms and its LDS operations run in order, so a
    // wavefront fence (no workgroup barrier) orders the phases.
    auto build_hist = [&](int ub, const uint32_t *qd) {
        uint32_t *hw = (uint32_t *)hist_of(ub);
#pragma unroll
        for (int k = 0; k < 16; ++k) hw[half * 16 + k] = 0u;
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
#pragma unroll
        for (int j = 0; j < QW; ++j)
#pragma unroll
            for (int b = 0; b < 4; ++b) {
                const uint32_t bin = ((qd[j] >> (8 * b)) & 0xFFu) - 128u;
                __hip_atomic_fetch_add(hw + (bin >> 2), 1u << (8 * (bin & 3u)), __ATOMIC_RELAXED,
                                       __HIP_MEMORY_SCOPE_WORKGROUP);
            }
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        // each lane of the pair turns its half (16 words, 64 bins) into suffix
        // counts; the lower half adds the upper half's total
        uint32_t x[16];
#pragma unroll
        for (int k = 0; k < 16; ++k) x[k] = hw[half * 16 + k];
        uint32_t tot = 0;
#pragma unroll
        for (int k = 0; k < 16; ++k) tot += (x[k] * 0x01010101u) >> 24;
        // the swap hands each lane its partner's total in one of the two
        // results and keeps its own in the other: their sum minus its own is
        // the partner's
        auto sw = __builtin_amdgcn_permlane32_swap(tot, tot, false, false);
        uint32_t carry = half == 0 ? sw[0] + sw[1] - tot : 0u;
#pragma unroll
        for (int k = 15; k >= 0; --k) {
            // byte j of t: the bins above j within the word
            uint32_t t = x[k] >> 8;
            t += t >> 8;
            t += t >> 16;
            const uint32_t wsum = (x[k] * 0x01010101u) >> 24;
            x[k] = t + carry * 0x01010101u;
            carry += wsum;
        }
#pragma unroll
        for (int k = 0; k < 16; ++k) hw[half * 16 + k] = x[k];
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    };
    // the pair's count of codes above F(hi): the same number code_count and
    // a sum over the pair give
    auto hist_count = [&](int ub, float mn, float sc, float hi) -> uint32_t {
        const float v = __builtin_amdgcn_fmed3f(fmaf(hi - mn, sc, 128.0f), 128.0f, 255.0f);
        const uint32_t g = __builtin_amdgcn_cvt_pk_u8_f32(v, 0, 0u) & 0xFFu;
        return (uint32_t)hist_of(ub)[g - 128u];
    };
    // the code compare against threshold hi (see the compare section)
    auto code_count = [](const uint32_t *qd, float mn, float sc, float hi) -> uint32_t {
        const float v = __builtin_amdgcn_fmed3f(fmaf(hi - mn, sc, 128.0f), 128.0f, 255.0f);
        // g = F(hi) in [128, 255]; byte (code - (g - 127)) has its top bit
        // set iff code > g, and never borrows (code >= 128 >= g - 127)
        const uint32_t g = __builtin_amdgcn_cvt_pk_u8_f32(v, 0, 0u);
        const uint32_t H = __builtin_amdgcn_perm(0u, g, 0u) - 0x7F7F7F7Fu;
        uint32_t c = 0;
#pragma unroll
        for (int j = 0; j < QW; ++j) c = __builtin_popcount((qd[j] - H) & 0x80808080u) + c;
        return c;
    };

    for (int64_t st = s_begin; st < s_end; ++st) {
        ++nstep;
        {
            // (user, item) scores this step owes to users with a live pair
            // (both lanes of a pair hold the same user and list length)
            uint32_t lanes = 0;
#pragma unroll
            for (int ub = 0; ub < NUB; ++ub) lanes += (uint32_t)__popcll(__ballot(len[ub] > 0));
            const int64_t rest = a.m - st * (NIB * 32);
            nscored += (uint64_t)(lanes / 2) * (uint64_t)(rest < NIB * 32 ? rest : NIB * 32);
        }
        const uint8_t *tile = lds + cbuf * STAGE;
        // prefetch step st + NBUF - 1 straight into its LDS stage; that stage was
        // last read in the previous step, before the barrier that ended it
        if constexpr (MODE == CM_SCREEN) {
#pragma unroll
            for (int ub = 0; ub < NUB; ++ub) fetch_first(ub);
        }
        if (st + PF < s_end) {
            const int pb = cbuf + PF >= NBUF ? cbuf + PF - NBUF : cbuf + PF;
            stage_step<LOADS_MAX>(a.plp + (st + PF) * (int64_t)step_bytes, lds + pb * STAGE, step_bytes,
                                  tid, a.step_coef + 4 * (st + PF));
        }
        if constexpr (MODE == CM_SCREEN) {
            if (late && have_prev) {
#pragma unroll
                for (int ub = 0; ub < NUB; ++ub) {
                    if (hist_p[ub])
                        screen_entries(ub, eps_p[ub], [&](float hi) { return hist_count(ub, mn_p[ub], sc_p[ub], hi); },
                                       true);
                    else
                        screen_entries(ub, eps_p[ub],
                                       [&](float hi) { return code_count(qd_p[ub], mn_p[ub], sc_p[ub], hi); }, false);
                }
            }
        }

        // ---- scores of NIB x 32 items against NUB x 32 users
        f32x16 acc[NIB][NUB];
#pragma unroll
        for (int ib = 0; ib < NIB; ++ib)
#pragma unroll
            for (int ub = 0; ub < NUB; ++ub)
#pragma unroll
                for (int r = 0; r < 16; ++r) acc[ib][ub][r] = MODE == CM_BOUND ? -fth[ub] : 0.0f;
        int pscale[NIB];
#pragma unroll
        for (int ib = 0; ib < NIB; ++ib) {
            pscale[ib] = 127;
            if constexpr (SK == SK_FP8) {
                int64_t item = st * (NIB * 32) + ib * 32 + l32;
                pscale[ib] = 127 + (item < a.m ? (int)a.pexp[item] : 0);
            }
        }
        // every k-step is real (the layouts are padded to NKS), so this is one
        // straight-line block the scheduler can pipeline LDS reads through
#pragma unroll
        for (int s = 0; s < NKS; ++s) {
#pragma unroll
            for (int ib = 0; ib < NIB; ++ib) {
                FT af = *(const FT *)(tile + ((ib * NKS + s) * 64 + lane) * FB);
#pragma unroll
                for (int ub = 0; ub < NUB; ++ub)
                    acc[ib][ub] = mfma_step<SK>(acc[ib][ub], af, bfrag[ub][s], pscale[ib], uscale[ub]);
            }
        }
        {
            // Issue order of the block above: PIPE fragment reads in flight
            // ahead of the matrix-core instructions that consume them (left
            // alone, the scheduler waits for every read right before its use).
            constexpr int NRD = NKS * NIB;
            constexpr int RPF = sizeof(FT) >= 16 ? (int)sizeof(FT) / 16 : 1;   // LDS reads per fragment
            constexpr int PIPE = NRD < 4 ? NRD : 4;
            __builtin_amdgcn_sched_group_barrier(0x100, PIPE * RPF, 0);
#pragma unroll
            for (int i = 0; i < NRD - PIPE; ++i) {
                __builtin_amdgcn_sched_group_barrier(0x008, NUB, 0);
                __builtin_amdgcn_sched_group_barrier(0x100, RPF, 0);
            }
            __builtin_amdgcn_sched_group_barrier(0x008, PIPE * NUB, 0);
        }
        // items past the end never count: make their scores -inf
        const int64_t item0 = st * (NIB * 32);
        if (item0 + NIB * 32 > a.m) {
            // item - item0 is a constant per register plus 4 * half: compare
            // the constant part with one per-lane limit
            const int lim = (int)(a.m - item0) - 4 * half;
#pragma unroll
            for (int ib = 0; ib < NIB; ++ib)
#pragma unroll
                for (int r = 0; r < 16; ++r) {
                    if (ib * 32 + 8 * (r >> 2) + (r & 3) >= lim) {
#pragma unroll
                        for (int ub = 0; ub < NUB; ++ub) acc[ib][ub][r] = -__builtin_inff();
                    }
                }
        }

        // ---- error bound of this step for each of the lane's users
        const double *cs = (const double *)(tile + STEP_BYTES_MAX);   // staged with the tile
        const double ca = cs[0], cb = cs[1], cc = cs[2], cabs = cs[3];

        // ---- compare and count
        // Screening only needs a lower bound of each pair's count.  With enough
        // live entries, the lane's scores are first mapped to 7-bit codes by a
        // monotone function F, and an entry counts the codes above F(hi):
        // code(s) > F(hi) implies s > hi.  Four codes share a dword, so one
        // subtract, mask and bit count compare four scores with an entry.
        //   F(x) = cvt_u8(med3(fma(x - mn, sc, 128), 128, 255)),  sc = 126 / (mx - mn)
        // with [mn, mx] the range of the lane's scores in the step (of both
        // lanes of the pair for bucketed counting)
        // For a score x in [mn, mx], (x - mn) * sc <= 126 (1 + 2^-22), so the fma
        // lies in [128, 254.01] (med3 is the identity there): every code byte keeps
        // its top bit.  A flat or tiny range gives sc = 0: all codes 128, nothing
        // counted (still a lower bound).  Past-the-end items (a partial last step)
        // take the code of mn, 128, which is never counted either.
        // With pair, the range is the user's over both lanes of its pair, so
        // the two lanes code with one map (the pair's histogram merges their
        // codes); the per-entry code compare keeps each lane's own, finer range.
        auto pair_min_max = [](float &mn, float &mx) {
            // each lane gets its partner's value in one of the two results
            // and keeps its own in the other
            auto a = __builtin_amdgcn_permlane32_swap(__float_as_uint(mn), __float_as_uint(mn), false, false);
            auto b = __builtin_amdgcn_permlane32_swap(__float_as_uint(mx), __float_as_uint(mx), false, false);
            mn = fminf(__uint_as_float(a[0]), __uint_as_float(a[1]));
            mx = fmaxf(__uint_as_float(b[0]), __uint_as_float(b[1]));
        };
        auto quantize = [&](int ub, bool full, uint32_t *qd, float &mn_o, float &sc_o, bool pair) {
            float mn, mx;
            if (full) {
                mn = acc[0][ub][0];
                mx = mn;
#pragma unroll
                for (int ib = 0; ib < NIB; ++ib)
#pragma unroll
                    for (int r = 0; r < 16; ++r) {
                        mn = fminf(mn, acc[ib][ub][r]);
                        mx = fmaxf(mx, acc[ib][ub][r]);
                    }
                if (pair) pair_min_max(mn, mx);
            } else {
                mn = __builtin_inff();
                mx = -__builtin_inff();
#pragma unroll
                for (int ib = 0; ib < NIB; ++ib)
#pragma unroll
                    for (int r = 0; r < 16; ++r) {
                        const float v = acc[ib][ub][r];
                        if (v != -__builtin_inff()) {
                            mn = fminf(mn, v);
                            mx = fmaxf(mx, v);
                        }
                    }
                if (pair) pair_min_max(mn, mx);
                if (!(mn <= mx)) mn = mx = 0.0f;
#pragma unroll
                for (int ib = 0; ib < NIB; ++ib)
#pragma unroll
                    for (int r = 0; r < 16; ++r)
                        if (acc[ib][ub][r] == -__builtin_inff()) acc[ib][ub][r] = mn;
            }
            const float rg = mx - mn;
            const float sc = rg > 1e-30f ? 126.0f * __builtin_amdgcn_rcpf(rg) : 0.0f;
#pragma unroll
            for (int ib = 0; ib < NIB; ++ib)
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    uint32_t wd = 0;
#pragma unroll
                    for (int b = 0; b < 4; ++b)
                        wd = __builtin_amdgcn_cvt_pk_u8_f32(fmaf(acc[ib][ub][4 * j + b] - mn, sc, 128.0f), b, wd);
                    qd[ib * 4 + j] = wd;
                }
            mn_o = mn;
            sc_o = sc;
        };
#pragma unroll
        for (int ub = 0; ub < NUB; ++ub) {
            double E = un_hat[ub] * ca + un_del[ub] * cb + un_full[ub] * cc + cabs;
            const float eps = f32_round_up(E * (1.0 + 1e-9));
            if constexpr (MODE == CM_SCREEN) {
                const bool full = item0 + NIB * 32 <= a.m;
                const bool many = a.hist_min > 0 && __ballot(len[ub] >= a.hist_min) != 0ull;
                if (late) {
                    quantize(ub, full, qd_p[ub], mn_p[ub], sc_p[ub], many);
                    eps_p[ub] = eps;
                    hist_p[ub] = many;
                    if (many) build_hist(ub, qd_p[ub]);
                } else if (full && many) {
                    uint32_t qd[QW];
                    float mn, sc;
                    quantize(ub, true, qd, mn, sc, true);
                    build_hist(ub, qd);
                    screen_entries(ub, eps, [&](float hi) { return hist_count(ub, mn, sc, hi); }, true);
                } else if (full && __ballot(len[ub] >= SWAR_MIN_ENTRIES) != 0ull) {
                    uint32_t qd[QW];
                    float mn, sc;
                    quantize(ub, true, qd, mn, sc, false);
                    screen_entries(ub, eps, [&](float hi) { return code_count(qd, mn, sc, hi); }, false);
                } else {
                    screen_entries(ub, eps, [&](float hi) -> uint32_t {
                        uint32_t c = 0;
#pragma unroll
                        for (int ib = 0; ib < NIB; ++ib)
#pragma unroll
                            for (int r = 0; r < 16; ++r) c += (acc[ib][ub][r] > hi) ? 1u : 0u;
                        return c;
                    }, false);
                }
                continue;
            }
            if constexpr (MODE == CM_BOUND) {
                // the lane's largest |score - s64| / eps over its real items,
                // and the number of scores beyond eps (there should be none);
                // folded: |acc - (s64 - th)| against the folded bound
                const double fold = (double)fth[ub];
                const double efold = a.fold_th ? f32_round_up((E * (1.0 + 1.0 / (double)a.dpad) +
                                                               2.0 * (double)(a.dpad + 1) * 0x1p-23 * fabs(fold)) *
                                                              (1.0 + 1e-9))
                                               : (double)eps;
                if (uid[ub] >= 0) {
                    const int64_t urow = (int64_t)uid[ub] * a.d_master;
#pragma unroll
                    for (int ib = 0; ib < NIB; ++ib)
#pragma unroll
                        for (int r = 0; r < 16; ++r) {
                            const int64_t item = item0 + ib * 32 + 8 * (r >> 2) + 4 * half + (r & 3);
                            if (item < a.m) {
                                double s64 = 0.0;
                                for (int k = 0; k < a.d_master; ++k)
                                    s64 = fma(master_elem(a.um_master, a.mk_master, urow + k),
                                              master_elem(a.pm_master, a.mk_master, item * a.d_master + k), s64);
                                const double ratio = fabs((double)acc[ib][ub][r] - (s64 - fold)) / efold;
                                bound_max = fmax(bound_max, ratio);
                                bound_over += ratio > 1.0 ? 1u : 0u;
                            }
                        }
                }
                continue;
            }
            if constexpr (MODE == CM_TABLE) {
                // s > hi as an integer median: with order keys (ks, kh) of the
                // scores and of hi (zeros made +0, so the key order is the
                // float order), med3(ks, kh, kh + 1) - kh is 1 iff ks > kh,
                // else 0.  The kh terms are taken out once per step (exact
                // modulo 2^32); no compare masks are kept live.
                uint32_t ks[NIB * 16];
#pragma unroll
                for (int ib = 0; ib < NIB; ++ib)
#pragma unroll
                    for (int r = 0; r < 16; ++r) ks[ib * 16 + r] = f32_order_key(acc[ib][ub][r] + 0.0f);
#pragma unroll
                for (int j = 0; j < TC; ++j) {
                    const uint32_t kh = f32_order_key(f32_next_up(tth[ub][j] + eps) + 0.0f);
                    uint32_t c = 0u - (uint32_t)(NIB * 16) * kh;
                    const uint32_t kh1 = kh + 1u;   // no wrap: kh is the key of a finite float
#pragma unroll
                    for (int i = 0; i < NIB * 16; ++i) add_med3_u32(c, ks[i], kh, kh1);
                    tcnt[ub][j] += c;
                }
                continue;
            }
            const int mylen = len[ub];
            // band count of one entry against the step's scores: certainly-above
            // scores add to cnt, near ties are emitted for the FP64 recheck
            auto exact_entry = [&](bool act, int pid, float th, float tl, float tmv, uint32_t &cnt) {
                const float hi = a.plain ? th : f32_next_up(th + eps);
                const float lo = a.plain ? f32_next_up(hi) : f32_next_down(tl - eps);
                // two counts per score: c of scores above hi (certainly above
                // the threshold), cl of scores at or above lo; every score above
                // hi is at or above lo, so near ties (lo <= score <= hi) exist
                // exactly when cl > c.  Plain mode has lo = next_up(hi): none.
                uint32_t c = 0, cl = 0;
#pragma unroll
                for (int ib = 0; ib < NIB; ++ib)
#pragma unroll
                    for (int r = 0; r < 16; ++r) {
                        const float sv = acc[ib][ub][r];
                        c += (sv > hi) ? 1u : 0u;
                        cl += (sv >= lo) ? 1u : 0u;
                    }
                if (__ballot(act && cl != c) != 0ull) {
                    // rare: the masks of this entry's near ties and of their
                    // plain FP32 verdicts (score > fl32(t))
                    uint32_t umask = 0, pmask = 0;
#pragma unroll
                    for (int ib = 0; ib < NIB; ++ib)
#pragma unroll
                        for (int r = 0; r < 16; ++r) {
                            const float sv = acc[ib][ub][r];
                            umask |= (sv >= lo && !(sv > hi)) ? (1u << (ib * 16 + r)) : 0u;
                            pmask |= (sv > tmv) ? (1u << (ib * 16 + r)) : 0u;
                        }
                    if (!act) umask = 0;
                    const uint32_t nu = __popc(umask);
                    // record offsets: with at most one record per lane (the
                    // usual case) they are the lane's rank among the lanes
                    // that have one; otherwise a prefix sum over the wave
                    uint32_t incl, total;
                    const uint64_t has = __ballot(nu != 0);
                    if (__ballot(nu > 1) == 0ull) {
                        incl = __builtin_amdgcn_mbcnt_hi((uint32_t)(has >> 32),
                                                         __builtin_amdgcn_mbcnt_lo((uint32_t)has, 0u)) + nu;
                        total = (uint32_t)__popcll(has);
                    } else {
                        incl = wave_incl_scan(nu, lane);
                        total = __shfl(incl, 63, 64);
                    }
                    if (rb_n + (int)total > REC_PER_WAVE) flush_records();
                    auto put = [&](auto &&store) {
                        uint32_t mm = umask;
                        while (mm) {
                            const int bit = __ffs(mm) - 1;
                            mm &= mm - 1;
                            const int ib = bit >> 4, r = bit & 15;
                            const int64_t item = item0 + ib * 32 + 8 * (r >> 2) + 4 * half + (r & 3);
                            const int plainbit = ((pmask >> bit) & 1u) ? (int)0x80000000 : 0;
                            store(make_int2(pid, (int)item | plainbit));
                        }
                    };
                    if ((int)total <= REC_PER_WAVE) {
                        // into this wave's LDS buffer
                        int pos = rb_n + (int)(incl - nu);
                        put([&](int2 rec) { recbuf[pos++] = rec; });
                        rb_n += (int)total;
                    } else {
                        // more than a buffer's worth at once: straight to the output
                        unsigned long long base = 0;
                        if (lane == 0) base = atomicAdd(a.emit_count, (unsigned long long)total);
                        unsigned long long pos = __shfl(base, 0, 64) + (incl - nu);
                        put([&](int2 rec) {
                            if (pos < a.emit_cap) a.emit[pos] = rec;
                            ++pos;
                        });
                    }
                }
                cnt += pair_sum(c);
            };
            // the first EC entries live in registers for the whole scan
#pragma unroll
            for (int k = 0; k < EC; ++k)
                if (__ballot(k < mylen) != 0ull)
                    exact_entry(k < mylen, rpid[ub][k], rth[ub][k], rtl[ub][k], rtm[ub][k], rcnt[ub][k]);
            // the rest: fields from memory (the fields of entry i + 1 load while
            // entry i is counted), the partial count kept per split
            int pid_n = 0;
            float th_n = 0.0f, tl_n = 0.0f, tm_n = 0.0f;
            uint32_t cnt_n = 0;
            auto fetch = [&](int i) {
                const int64_t e = ebase[ub] + (int64_t)i * 32;
                pid_n = a.ent_pid[e];
                th_n = a.ent_th[e];
                tl_n = a.ent_tl[e];
                tm_n = a.ent_tm[e];
                cnt_n = (st == s_begin) ? 0u : a.ent_cnt[(int64_t)split * a.cap_total + e];
            };
            if (mylen > EC) fetch(EC);
            for (int i = EC; __ballot(i < mylen) != 0ull; ++i) {
                const bool act = i < mylen;
                const int64_t e = ebase[ub] + (int64_t)i * 32;
                // take every field of entry i before the prefetch overwrites them
                const int pid = pid_n;
                const float th = th_n;
                const float tl = tl_n, tmv = tm_n;
                uint32_t cnt = cnt_n;
                if (i + 1 < mylen) fetch(i + 1);
                exact_entry(act, pid, th, tl, tmv, cnt);
                if (act && half == 0) a.ent_cnt[(int64_t)split * a.cap_total + e] = cnt;
            }
            // exact lists never change during a pass: the statistics are
            // added once per tile, after the scan
        }

        have_prev = late;
        cbuf = cbuf + 1 == NBUF ? 0 : cbuf + 1;
        if (SYNC2 && ((st - s_begin) & 1) == 0) continue;
        // step st + 1 (with SYNC2, st + 2 too) has landed (same-wave entry
        // stores stay ordered before the next step's loads of the same slots)
        if (st + PF < s_end)
            wait_vm<WAIT_N>();
        else
            wait_vm<0>();
        int live = 0;
#pragma unroll
        for (int ub = 0; ub < NUB; ++ub) live |= (len[ub] > 0);
        const bool wave_live = __ballot(live) != 0ull;    // every lane takes part
        if (lane == 0 && wave_live) atomicOr(&wg_live[lslot], 1);
        __syncthreads();
        const int any = wg_live[lslot];
        if (tid == 0) wg_live[lslot == 0 ? 2 : lslot - 1] = 0;
        lslot = lslot == 2 ? 0 : lslot + 1;
        if (!any) break;
    }

    if constexpr (MODE == CM_SCREEN) {
        if (late && have_prev) {
#pragma unroll
            for (int ub = 0; ub < NUB; ++ub) {
                fetch_first(ub);
                if (hist_p[ub])
                    screen_entries(ub, eps_p[ub], [&](float hi) { return hist_count(ub, mn_p[ub], sc_p[ub], hi); },
                                   true);
                else
                    screen_entries(ub, eps_p[ub], [&](float hi) { return code_count(qd_p[ub], mn_p[ub], sc_p[ub], hi); },
                                   false);
            }
        }
    }

    if constexpr (MODE == CM_EXACT) {
        flush_records();
        const uint64_t nsc = (uint64_t)(s_end - s_begin);
#pragma unroll
        for (int ub = 0; ub < NUB; ++ub) {
            ncmp += nsc * (uint64_t)len[ub] * (NIB * 16);
            nslot += nsc * (uint64_t)wave_max(len[ub]) * (NIB * 16);
        }
    }
    // ---- write back
    if constexpr (MODE == CM_BOUND) {
        if (bound_max > 0.0) atomicMax(&a.cnt_out[0], __float_as_uint(f32_round_up(bound_max)));
        if (bound_over) atomicAdd(&a.cnt_out[1], bound_over);
        return;
    }
#pragma unroll
    for (int ub = 0; ub < NUB; ++ub) {
        if (uid[ub] < 0) continue;
        if constexpr (MODE == CM_SCREEN) {
            if (half == 0) a.ent_len[split * a.len_stride + tix[ub]] = len[ub];
        } else if constexpr (MODE == CM_TABLE) {
            // both lanes of a pair hold the same user: sum their halves
#pragma unroll
            for (int j = 0; j < TC; ++j) {
                const uint32_t c = pair_sum(tcnt[ub][j]);
                if (half == 0) atomicAdd(&a.cnt_out[(int64_t)uid[ub] * TABLE_COLS + j], c);
            }
        } else {
            if (half == 0) {
#pragma unroll
                for (int k = 0; k < EC; ++k)
                    if (k < len[ub]) atomicAdd(&a.cnt_out[rpid[ub][k]], rcnt[ub][k]);
                for (int i = EC; i < len[ub]; ++i) {
                    const int64_t e = ebase[ub] + (int64_t)i * 32;
                    atomicAdd(&a.cnt_out[a.ent_pid[e]], a.ent_cnt[(int64_t)split * a.cap_total + e]);
                }
            }
        }
    }
}

// One workgroup per tile of users (grid launch), or, with a tile counter, a
// persistent grid whose workgroups take tiles from the counter until none is
// left (every workgroup exits once the counter passes the last tile).
template <int SK, int MODE, int NKS, int NUB, int NIB, bool PERSIST>
__global__ __launch_bounds__(512) void k_count(CountArgs a) {
    extern __shared__ __attribute__((aligned(16))) uint8_t lds[];
    const int lane = threadIdx.x & 63;
    uint64_t ncmp = 0, nslot = 0, nstep = 0, nscored = 0;
    if constexpr (!PERSIST) {
        count_tile<SK, MODE, NKS, NUB, NIB>(a, (int64_t)blockIdx.x, lds, ncmp, nslot, nstep, nscored);
    } else {
        __shared__ int64_t sh_tile;
        for (;;) {
            if (threadIdx.x == 0) sh_tile = (int64_t)atomicAdd(a.tile_counter, 1ull);
            __syncthreads();
            const int64_t t = sh_tile;
            __syncthreads();
            if (t >= a.ntiles) break;
            count_tile<SK, MODE, NKS, NUB, NIB>(a, t, lds, ncmp, nslot, nstep, nscored);
            __syncthreads();   // the next tile reuses the LDS buffers
        }
    }
    // executed compares (both lanes of a pair count their own items)
    uint64_t tot = ncmp, tslot = nslot;
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) {
        tot += __shfl_xor(tot, o, 64);
        tslot += __shfl_xor(tslot, o, 64);
    }
    if (lane == 0 && a.stat) {
        atomicAdd(a.stat, (unsigned long long)tot);
        atomicAdd(a.stat + 2, (unsigned long long)tslot);   // lane slots, active or not
        atomicAdd(a.stat + 6, (unsigned long long)nscored); // per wave: its users' scores
    }
    // executed matrix-core flop: every step of a workgroup multiplies its
    // 8 x NUB x 32 users by NIB x 32 items over the padded dimension
    constexpr unsigned long long FLOP_PER_STEP =
        2ull * WAVES_PER_WG * NUB * USER_BLOCK * NIB * 32 * NKS * frag_ks(SK);
    if (threadIdx.x == 0 && a.stat) atomicAdd(a.stat + 4, (unsigned long long)nstep * FLOP_PER_STEP);
}

template <int SK, int MODE, int NKS, int NUB, int NIB>
static hipError_t launch_one(const CountArgs &a, int nsplit, hipStream_t st) {
    constexpr int TASKS_PER_WG = WAVES_PER_WG * NUB * USER_BLOCK;
    constexpr int STEP_BYTES_MAX = NIB * NKS * 64 * frag_fb(SK);
    constexpr int STAGE = STEP_BYTES_MAX + 32;
    const size_t lds = (size_t)stage_buffers<MODE>(STAGE) * STAGE + record_bytes<MODE>() + hist_bytes<MODE, NUB>();
    if (a.nks != NKS) return hipErrorInvalidValue;   // layouts are padded to a supported k-step count
    const int64_t ntiles = (a.ntask + TASKS_PER_WG - 1) / TASKS_PER_WG;
    if (ntiles == 0) return hipSuccess;
    CountArgs b = a;
    b.ntiles = ntiles;
    if constexpr (MODE == CM_SCREEN) {
        if (b.tile_counter) {
            auto kern = k_count<SK, MODE, NKS, NUB, NIB, true>;
            hipError_t e = hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize,
                                               (int)lds);
            if (e != hipSuccess) return e;
            dim3 grid((unsigned)std::min<int64_t>(ntiles, std::max(1, b.persistent_ctas)), 1);
            hipLaunchKernelGGL(kern, grid, dim3(512), lds, st, b);
            return hipGetLastError();
        }
    }
    b.tile_counter = nullptr;
    auto kern = k_count<SK, MODE, NKS, NUB, NIB, false>;
    hipError_t e = hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    dim3 grid((unsigned)ntiles, (unsigned)nsplit);
    hipLaunchKernelGGL(kern, grid, dim3(512), lds, st, b);
    return hipGetLastError();
}

// Tile variants of the count kernel (user blocks x item blocks per wave):
// v0 = 2 x 2, v1 = 1 x 4, v2 = 1 x 2.  v1 halves the entry iterations per
// compared score at the cost of no reuse of an LDS A fragment across user
// blocks; v2 is the low-register tile of the exact passes (their near-tie
// masks hold 64 items per step).
template <int SK, int MODE>
static hipError_t dispatch_nks(const CountArgs &a, int nsplit, int variant, hipStream_t st) {
    const int nks = a.nks;
    if constexpr (SK == SK_BF16) {
        if (variant == 2) {
            if (nks <= 4) return launch_one<SK, MODE, 4, 1, 2>(a, nsplit, st);
            if (nks <= 8) return launch_one<SK, MODE, 8, 1, 2>(a, nsplit, st);
            if (nks <= 13) return launch_one<SK, MODE, 13, 1, 2>(a, nsplit, st);
            if (nks <= 20) return launch_one<SK, MODE, 20, 1, 2>(a, nsplit, st);
        }
        if constexpr (MODE == CM_SCREEN) {
            if (nks <= 4) return variant ? launch_one<SK, MODE, 4, 1, 4>(a, nsplit, st) : launch_one<SK, MODE, 4, 2, 2>(a, nsplit, st);
            if (nks <= 8) return variant ? launch_one<SK, MODE, 8, 1, 4>(a, nsplit, st) : launch_one<SK, MODE, 8, 2, 2>(a, nsplit, st);
            if (nks <= 13) return variant ? launch_one<SK, MODE, 13, 1, 4>(a, nsplit, st) : launch_one<SK, MODE, 13, 2, 2>(a, nsplit, st);
            if (nks <= 20) return launch_one<SK, MODE, 20, 1, 2>(a, nsplit, st);
        }
    } else if constexpr (SK == SK_F32) {
        if (nks <= 32) return launch_one<SK, MODE, 32, 1, 1>(a, nsplit, st);
        if (nks <= 64) return launch_one<SK, MODE, 64, 1, 1>(a, nsplit, st);
        if (nks <= 100) return launch_one<SK, MODE, 100, 1, 1>(a, nsplit, st);
        if (nks <= 160) return launch_one<SK, MODE, 160, 1, 1>(a, nsplit, st);
    } else {
        if (variant == 2) {
            if (nks <= 2) return launch_one<SK, MODE, 2, 1, 2>(a, nsplit, st);
            if (nks <= 4) return launch_one<SK, MODE, 4, 1, 2>(a, nsplit, st);
            if (nks <= 8) return launch_one<SK, MODE, 8, 1, 2>(a, nsplit, st);
        }
        if constexpr (MODE == CM_SCREEN) {
            if (nks <= 2) return variant ? launch_one<SK, MODE, 2, 1, 4>(a, nsplit, st) : launch_one<SK, MODE, 2, 2, 2>(a, nsplit, st);
            if (nks <= 4) return variant ? launch_one<SK, MODE, 4, 1, 4>(a, nsplit, st) : launch_one<SK, MODE, 4, 2, 2>(a, nsplit, st);
            if (nks <= 8) return launch_one<SK, MODE, 8, 1, 2>(a, nsplit, st);
        }
    }
    return hipErrorInvalidValue;
}

template <int SK>
static hipError_t dispatch_mode(int mode, const CountArgs &a, int nsplit, int variant, hipStream_t st) {
    if (mode == CM_SCREEN) return dispatch_nks<SK, CM_SCREEN>(a, nsplit, variant, st);
    if (mode == CM_EXACT) return dispatch_nks<SK, CM_EXACT>(a, nsplit, variant, st);
    if (mode == CM_TABLE) return dispatch_nks<SK, CM_TABLE>(a, nsplit, variant, st);
    if (mode == CM_BOUND) return dispatch_nks<SK, CM_BOUND>(a, nsplit, variant, st);
    return hipErrorInvalidValue;
}

hipError_t launch_count(int sk, int mode, const CountArgs &a, int nsplit, int variant, hipStream_t st) {
    if (sk == SK_BF16 && mode == CM_EXACT && variant == 2) {
        static const bool generic = [] {
            const char *v = getenv("RKR_EXACT_GENERIC");
            return v && *v == '1';
        }();
        if (!generic) return launch_exact_bf16(a, nsplit, st);
    }
    if (sk == SK_BF16) return dispatch_mode<SK_BF16>(mode, a, nsplit, variant, st);
    if (sk == SK_F32) return dispatch_mode<SK_F32>(mode, a, nsplit, variant, st);
    if (sk == SK_FP8) return dispatch_mode<SK_FP8>(mode, a, nsplit, variant, st);
    return hipErrorInvalidValue;
}

// The k-step count an index pads its low-precision layouts to: the smallest
// count a kernel is instantiated for that holds nks k-steps (0 if none).
int nks_bucket(int sk, int nks) {
    static const int bf16[] = {4, 8, 13, 20}, f32[] = {32, 64, 100, 160}, fp8[] = {2, 4, 8};
    const int *b = sk == SK_BF16 ? bf16 : (sk == SK_F32 ? f32 : fp8);
    const int nb = sk == SK_FP8 ? 3 : 4;
    for (int i = 0; i < nb; ++i)
        if (nks <= b[i]) return b[i];
    return 0;
}

// Largest supported k-step count per score kind (d <= KS * max).
int max_nks(int sk) { return sk == SK_BF16 ? 20 : (sk == SK_F32 ? 160 : 8); }
int nub_of(int sk, int nks, int variant) {
    if (sk == SK_F32 || variant != 0) return 1;
    if (sk == SK_BF16) return nks <= 13 ? 2 : 1;
    return nks <= 4 ? 2 : 1;
}
int nib_of(int sk, int nks, int variant) {
    if (sk == SK_F32) return 1;
    if (variant != 1) return 2;
    if (sk == SK_BF16) return nks <= 13 ? 4 : 2;
    return nks <= 4 ? 4 : 2;
}
int num_variants(int sk, int nks) {
    if (sk == SK_BF16) return nks <= 13 ? 3 : 1;
    if (sk == SK_FP8) return nks <= 4 ? 3 : 1;
    return 1;
}

}  // namespace rkr
