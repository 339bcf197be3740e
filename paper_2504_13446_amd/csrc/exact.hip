// exact.hip -- the exact passes of the fused score + count (Def. 1, Sec. 2)
// for BF16 scores: for every (user, query) pair of a task list, the number of
// items certainly above the pair's FP64 threshold, every near tie emitted for
// the FP64 recheck.
//
// Operands, entry lists, band edges, records and outputs are those of the
// count kernel's exact mode (count.hip).  What differs is the schedule, made
// for what these passes look like -- one or two pairs per user, so a few
// compares per score against a 13-MFMA score tile -- where a wave that
// computes a step's scores and then compares them leaves the matrix cores
// idle through every compare and waits on its own last MFMA before it:
//
//  * The loop over item steps is software-pipelined.  While a wave compares
//    the scores of step st (accumulators `cur`) it computes those of step
//    st + 1 (accumulators `nxt`); the two are one basic block, and scheduling
//    groups interleave them: one LDS fragment read and one MFMA, then a few
//    compare instructions, and so on.  The compare of step st never waits for
//    an MFMA of step st + 1.
//  * Per step a lane counts its 32 scores above the first pair's upper edge
//    and at or above its lower edge; the counts stay per lane (the pair sum is
//    taken once, at the end); a near tie shows as a difference of the two and
//    takes the rare path that writes records, after the block.
//  * Items stream through NBUF LDS stages (direct global -> LDS copies);
//    the workgroup meets at one barrier per SP steps.  Step st + D is staged
//    at step st; at a barrier before step st0, the stages of steps up to
//    st0 + SP have landed (each wave waits until at most the copies of later
//    steps are in flight), and a stage is overwritten only after a barrier
//    has followed every read of it.  SP = 2, D = 4 with five stages.
//  * The users' fragments, the pairs of each lane and their counts live in
//    registers for the whole scan: a task holds at most two pairs (the task
//    builder gives a user with more pairs several tasks; the all-ranks passes
//    have one pair per user), so no list is read inside the loop.
#include "rkr_internal.h"
#include "tile_common.h"

#include <algorithm>

namespace rkr {

namespace {

#ifndef EX_PIPE
#define EX_PIPE 4
#endif
constexpr int EX_NIB = 2;          // item blocks of 32 per step: 64 items
constexpr int EX_LDS = 153600;     // LDS for the item stages and the record buffers

template <int NKS>
struct ExactGeom {
    static constexpr int FB = frag_fb(SK_BF16);
    static constexpr int STEP_BYTES = EX_NIB * NKS * 64 * FB;
    static constexpr int STAGE = STEP_BYTES + 32;   // item tile + the step's four error-bound coefficients
    static constexpr int REC_BYTES = WAVES_PER_WG * REC_PER_WAVE * 8;
    static constexpr int NBUF_FIT = (EX_LDS - REC_BYTES) / STAGE;
    static constexpr int NBUF = NBUF_FIT > 5 ? 5 : NBUF_FIT;
    static_assert(NBUF >= 3, "the pipeline needs three LDS stages");
    // barrier period and staging distance: D >= SP + 1 (steps st0 + 1 .. st0
    // + SP are staged before the barrier at st0) and D <= NBUF - SP + 1 (the
    // stage step st + D overwrites was last read before the previous barrier)
    static constexpr int SP = NBUF >= 5 ? 2 : 1;
    static constexpr int D = NBUF - SP + 1;
    static constexpr int LOADS = (STEP_BYTES + 8191) / 8192;
    static constexpr int LDS_BYTES = NBUF * STAGE;   // dynamic LDS (the record buffers are a static array)
};

// One item step (STEP_BYTES, then the step's 32 bytes of error-bound
// coefficients) from global memory into an LDS stage, 16 bytes per lane, as
// buffer loads that write LDS directly (M0 = the wave's LDS base).
//
// The copies are issued from inline assembly so that the compiler's wait
// model does not see them: it would otherwise either wait for every copy in
// flight before the next read of any stage (the buffer form) or count LDS
// reads as out of order while a copy is in flight and wait for all of them
// each time it needs one (the global form).  The kernel orders the copies
// itself (vmcnt waits per wave, then a barrier, before a stage is read; a
// barrier after every read of a stage before it is refilled).  Waits the
// compiler inserts for its own memory operations stay correct: it can only
// under-count the operations issued after them, which makes a wait stricter.
template <int STEP_BYTES, int LOADS>
struct StageCopy {
    uint32_t voff[LOADS];   // this lane's byte offsets in the step (loop invariant)
    uint32_t lds_off[LOADS + 1];   // the wave's LDS offsets in a stage, then the coefficients'
    int nload;              // copies this wave issues per step (wave-uniform)
    __device__ StageCopy(int wave, int lane) {
        nload = 0;
#pragma unroll
        for (int j = 0; j < LOADS; ++j) {
            const int wbase = (j * 512 + wave * 64) * 16;
            voff[j] = (uint32_t)(wbase + lane * 16);
            lds_off[j] = (uint32_t)wbase;
            nload += wbase < STEP_BYTES ? 1 : 0;
        }
        lds_off[LOADS] = STEP_BYTES;
        nload += wave == 0 ? 1 : 0;
    }
    static __device__ i32x4 rsrc(const void *base, uint32_t bytes) {
        const uint64_t b = (uint64_t)base;
        // word 1: base bits 32..47, stride 0; word 3: 32-bit data format, no swizzle
        return i32x4{__builtin_amdgcn_readfirstlane((int)(uint32_t)b),
                     __builtin_amdgcn_readfirstlane((int)((uint32_t)(b >> 32) & 0xFFFFu)), (int)bytes, 0x00020000};
    }
    static __device__ void copy16(i32x4 r, uint32_t m0v, uint32_t voff) {
        asm volatile("s_mov_b32 m0, %0\n\ts_nop 0\n\tbuffer_load_dwordx4 %1, %2, 0 offen lds"
                     :
                     : "s"(m0v), "v"(voff), "s"(r)
                     : "memory");
    }
    // copy step src (and its coefficients) into the stage at LDS offset stage_off
    __device__ void operator()(const uint8_t *src, uint32_t stage_off, int wave, int lane, const double *coef) const {
        const i32x4 rp = rsrc(src, STEP_BYTES);
#pragma unroll
        for (int j = 0; j < LOADS; ++j)
            if ((int)lds_off[j] < STEP_BYTES) copy16(rp, __builtin_amdgcn_readfirstlane(stage_off + lds_off[j]), voff[j]);
        if (wave == 0 && lane < 2)
            copy16(rsrc(coef, 32), __builtin_amdgcn_readfirstlane(stage_off + lds_off[LOADS]), (uint32_t)(lane * 16));
    }
};

// s_waitcnt vmcnt(n) for a wave-uniform n (values above 24 wait for 24).
__device__ inline void wait_vm_n(int n) {
    switch (n) {
    case 0: wait_vm<0>(); break;
    case 1: wait_vm<1>(); break;
    case 2: wait_vm<2>(); break;
    case 3: wait_vm<3>(); break;
    case 4: wait_vm<4>(); break;
    case 5: wait_vm<5>(); break;
    case 6: wait_vm<6>(); break;
    case 7: wait_vm<7>(); break;
    case 8: wait_vm<8>(); break;
    case 9: wait_vm<9>(); break;
    case 10: wait_vm<10>(); break;
    case 11: wait_vm<11>(); break;
    case 12: wait_vm<12>(); break;
    case 13: wait_vm<13>(); break;
    case 14: wait_vm<14>(); break;
    case 15: wait_vm<15>(); break;
    case 16: wait_vm<16>(); break;
    case 17: wait_vm<17>(); break;
    case 18: wait_vm<18>(); break;
    case 19: wait_vm<19>(); break;
    case 20: wait_vm<20>(); break;
    case 21: wait_vm<21>(); break;
    case 22: wait_vm<22>(); break;
    case 23: wait_vm<23>(); break;
    default: wait_vm<24>(); break;
    }
}

template <int NKS>
__device__ inline void exact_tile(const CountArgs &a, const int64_t tile, uint8_t *lds, int2 *recs, uint64_t &ncmp,
                                  uint64_t &nslot, uint64_t &nstep, uint64_t &nscored) {
    using G = ExactGeom<NKS>;
    using FT = typename FragT<SK_BF16>::T;
    constexpr int NIB = EX_NIB;
    constexpr int FB = G::FB, STEP_BYTES = G::STEP_BYTES, STAGE = G::STAGE, NBUF = G::NBUF;
    constexpr int SP = G::SP, D = G::D, LOADS = G::LOADS;
    constexpr int KS = frag_ks(SK_BF16), ES = elem_size(SK_BF16);
    constexpr int NSC = NIB * 16;    // scores per lane per step

    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;
    const int wave_u = __builtin_amdgcn_readfirstlane(wave);   // the same, known to be uniform
    const int l32 = lane & 31;
    const int half = lane >> 5;
    const int split = blockIdx.y;
    const int64_t s_begin = a.step0 + (int64_t)split * a.steps_per_split;
    const int64_t s_end = std::min<int64_t>(s_begin + a.steps_per_split, a.step_end);

    // ---- the lane's user: register-stationary fragments, norms, first pairs
    const int64_t t = tile * (WAVES_PER_WG * USER_BLOCK) + wave * USER_BLOCK + l32;
    const int u = t < a.ntask ? a.task_user[t] : -1;
    const int len = u >= 0 ? a.ent_len[split * a.len_stride + t] : 0;
    const int64_t ebase = u >= 0 ? a.blk_base[t >> 5] + l32 : 0;
    double un_hat = 0.0, un_del = 0.0, un_full = 0.0;
    if (u >= 0) {
        un_hat = a.unorm3[3 * (int64_t)u + 0];
        un_del = a.unorm3[3 * (int64_t)u + 1];
        un_full = a.unorm3[3 * (int64_t)u + 2];
    }
    FT bfrag[NKS];
    {
        const uint8_t *urow = a.ulp + ((int64_t)(u >= 0 ? u : 0) * a.dpad + half * (KS / 2)) * ES;
#pragma unroll
        for (int s = 0; s < NKS; ++s) {
            FT v{};
            if (u >= 0) v = *(const FT *)(urow + (int64_t)s * KS * ES);
            bfrag[s] = v;
        }
    }
    int pid0 = 0, pid1 = 0;
    float th0 = 0.0f, tl0 = 0.0f, tm0 = 0.0f, th1 = 0.0f, tl1 = 0.0f, tm1 = 0.0f;
    if (len > 0) {
        pid0 = a.ent_pid[ebase];
        th0 = a.ent_th[ebase];
        tl0 = a.ent_tl[ebase];
        tm0 = a.ent_tm[ebase];
    }
    if (len > 1) {
        pid1 = a.ent_pid[ebase + 32];
        th1 = a.ent_th[ebase + 32];
        tl1 = a.ent_tl[ebase + 32];
        tm1 = a.ent_tm[ebase + 32];
    }
    uint32_t cnt0 = 0, cnt1 = 0;   // per-lane certain counts of the two register pairs
    int wlen = len;   // at most 2 (see the top of the file)
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) wlen = max(wlen, __shfl_xor(wlen, o, 64));
    wlen = __builtin_amdgcn_readfirstlane(wlen);
    if (!__syncthreads_or(len > 0) || s_begin >= s_end) return;

    // ---- near-tie records: a per-wave LDS buffer, flushed with one global
    // atomic when full and at the end.  It is an array of its own, apart from
    // the item stages, so that the compiler can tell that writing a record
    // does not touch a stage an LDS copy is still filling (it would otherwise
    // wait for every copy in flight before each record write).
    int2 *const recbuf = recs + wave * REC_PER_WAVE;
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

    // band edges of a pair for a step's bound eps
    auto edges = [&](float th, float tl, float eps, float &hi, float &lo) {
        hi = a.plain ? th : f32_next_up(th + eps);
        lo = a.plain ? f32_next_up(hi) : f32_next_down(tl - eps);
    };
    // the step's bound for this lane's user from the coefficients staged with its tile
    auto step_eps = [&](const uint8_t *tile) -> float {
        const double *cs = (const double *)(tile + STEP_BYTES);
        const double E = un_hat * cs[0] + un_del * cs[1] + un_full * cs[2] + cs[3];
        return f32_round_up(E * (1.0 + 1e-9));
    };
    // item of score r of block ib in this lane, for a step starting at item0
    auto item_of = [&](int64_t item0, int ib, int r) -> int64_t {
        return item0 + ib * 32 + 8 * (r >> 2) + 4 * half + (r & 3);
    };
    // near ties of one pair in one step (scores in [lo, hi]) to the record
    // buffer, each with the plain FP32 verdict (score > fl32(t)) in its top bit
    auto emit_ties = [&](const f32x16 *acc, bool act, int pid, float hi, float lo, float tm, int64_t item0) {
        // bit ib * 16 + r of each mask is score r of block ib (shifted in
        // from the top, so that no per-bit constants are needed)
        uint32_t umask = 0, pmask = 0;
#pragma unroll
        for (int ib = NIB - 1; ib >= 0; --ib)
#pragma unroll
            for (int r = 15; r >= 0; --r) {
                const float sv = acc[ib][r];
                umask = (umask << 1) | ((sv >= lo && !(sv > hi)) ? 1u : 0u);
                pmask = (pmask << 1) | ((sv > tm) ? 1u : 0u);
            }
        if (!act) umask = 0;
        const uint32_t nu = __popc(umask);
        // record offsets: with at most one record per lane (the usual case)
        // the lane's rank among the lanes that have one, else a prefix sum
        uint32_t incl, total;
        const uint64_t has = __ballot(nu != 0);
        if (__ballot(nu > 1) == 0ull) {
            incl = __builtin_amdgcn_mbcnt_hi((uint32_t)(has >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)has, 0u)) + nu;
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
                const int64_t item = item_of(item0, bit >> 4, bit & 15);
                const int plainbit = ((pmask >> bit) & 1u) ? (int)0x80000000 : 0;
                store(make_int2(pid, (int)item | plainbit));
            }
        };
        if ((int)total <= REC_PER_WAVE) {
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
    };
    // count of one pair over one step (per lane), and whether it has near ties
    auto count_pair = [&](const f32x16 *acc, float hi, float lo, uint32_t &c, uint32_t &cl) {
        c = 0;
        cl = 0;
#pragma unroll
        for (int ib = 0; ib < NIB; ++ib)
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                const float sv = acc[ib][r];
                c += (sv > hi) ? 1u : 0u;
                cl += (sv >= lo) ? 1u : 0u;
            }
    };
    // the second pair of the lane (rare: waves whose tasks hold two)
    auto second_pair = [&](const f32x16 *acc, float eps, int64_t item0) {
        float hi, lo;
        edges(th1, tl1, eps, hi, lo);
        uint32_t c, cl;
        count_pair(acc, hi, lo, c, cl);
        const bool act = len > 1;
        cnt1 += c;
        if (__ballot(act && cl != c) != 0ull) emit_ties(acc, act, pid1, hi, lo, tm1, item0);
    };
    // scores of items past the end never count
    auto mask_tail = [&](f32x16 *acc, int64_t item0) {
        if (item0 + NIB * 32 <= a.m) return;
        const int lim = (int)(a.m - item0) - 4 * half;
#pragma unroll
        for (int ib = 0; ib < NIB; ++ib)
#pragma unroll
            for (int r = 0; r < 16; ++r)
                if (ib * 32 + 8 * (r >> 2) + (r & 3) >= lim) acc[ib][r] = -__builtin_inff();
    };
    // the scores of a step (MFMA block only)
    auto scores = [&](const uint8_t *tile, f32x16 *acc) {
#pragma unroll
        for (int ib = 0; ib < NIB; ++ib)
#pragma unroll
            for (int r = 0; r < 16; ++r) acc[ib][r] = 0.0f;
#pragma unroll
        for (int s = 0; s < NKS; ++s)
#pragma unroll
            for (int ib = 0; ib < NIB; ++ib) {
                const FT af = *(const FT *)(tile + ((ib * NKS + s) * 64 + lane) * FB);
                acc[ib] = mfma_step<SK_BF16>(acc[ib], af, bfrag[s], 127, 127);
            }
    };

    // The scores of the next step (nxt, from the stage at tn) and the count
    // of the first pair over the current step (cur) in one block, in a fixed
    // order: chunk i reads fragment i + PIPE, issues MFMA i and compares the
    // next share of the current scores; a scheduling fence closes each chunk,
    // so every MFMA has PIPE fragment reads in flight ahead of it and compare
    // instructions between it and the next one.
    auto score_and_count = [&](const uint8_t *tn, f32x16 *nxt, const f32x16 *cur, float hi, float lo,
                               uint32_t &c, uint32_t &cl) {
        constexpr int NRD = NKS * NIB;
        constexpr int PIPE = NRD < EX_PIPE ? NRD : EX_PIPE;
        auto frag = [&](int i) { return *(const FT *)(tn + (((i % NIB) * NKS + i / NIB) * 64 + lane) * FB); };
#pragma unroll
        for (int ib = 0; ib < NIB; ++ib)
#pragma unroll
            for (int r = 0; r < 16; ++r) nxt[ib][r] = 0.0f;
        FT fr[PIPE];
#pragma unroll
        for (int i = 0; i < PIPE; ++i) fr[i] = frag(i);
        c = 0;
        cl = 0;
#pragma unroll
        for (int i = 0; i < NRD; ++i) {
            const FT f = fr[i % PIPE];
            if (i + PIPE < NRD) fr[i % PIPE] = frag(i + PIPE);
            nxt[i % NIB] = mfma_step<SK_BF16>(nxt[i % NIB], f, bfrag[i / NIB], 127, 127);
#pragma unroll
            for (int k = i * NSC / NRD; k < (i + 1) * NSC / NRD; ++k) {
                const float sv = cur[k / 16][k % 16];
                c += (sv > hi) ? 1u : 0u;
                cl += (sv >= lo) ? 1u : 0u;
            }
            __builtin_amdgcn_sched_barrier(0);
        }
    };

    // ---- prologue: stage steps s_begin .. s_begin + D - 1; the first lands
    const StageCopy<STEP_BYTES, LOADS> stage(wave_u, lane);
    const int nload = stage.nload;
    // the LDS offset of the stages (M0 takes LDS offsets, not generic addresses)
    const uint32_t lds_base = (uint32_t)(uintptr_t)(const __attribute__((address_space(3))) uint8_t *)lds;
    const int64_t npro = std::min<int64_t>(D, s_end - s_begin);
    for (int64_t k = 0; k < npro; ++k)
        stage(a.plp + (s_begin + k) * (int64_t)STEP_BYTES, lds_base + k * STAGE, wave_u, lane,
              a.step_coef + 4 * (s_begin + k));
    // before the barrier at step st0: steps up to st0 + SP have landed; the
    // copies of later steps (staged up to step st0 - 1 + D) may be in flight
    auto barrier_before = [&](int64_t st0) {
        const int64_t last = std::min<int64_t>(st0 - 1 + D, s_end - 1);
        const int64_t later = std::max<int64_t>(0, last - (st0 + SP));
        wait_vm_n((int)later * nload);
        __syncthreads();
    };
    wait_vm_n((int)(npro - 1) * nload);
    __syncthreads();

    f32x16 accA[NIB], accB[NIB];
    scores(lds, accA);
    float eps_cur = step_eps(lds);
    mask_tail(accA, s_begin * (NIB * 32));
    barrier_before(s_begin);

    int slot_nxt = 1 % NBUF;      // stage of step st + 1
    int slot_stg = D % NBUF;      // stage of step st + D
    // One step: stage st + D, compare st (cur) while scoring st + 1 (nxt).
    // The last step of a tile scores a stale stage too (its result is never
    // used): the block then has no branch, and the compare stays in it.
    auto body = [&](f32x16 *cur, f32x16 *nxt, int64_t st) {
        if (st + D < s_end)
            stage(a.plp + (st + D) * (int64_t)STEP_BYTES, lds_base + slot_stg * STAGE, wave_u, lane,
                  a.step_coef + 4 * (st + D));
        const int64_t item0 = st * (NIB * 32);
        float hi0, lo0;
        edges(th0, tl0, eps_cur, hi0, lo0);
        const uint8_t *tn = lds + slot_nxt * STAGE;
        uint32_t c0, cl0;
        score_and_count(tn, nxt, cur, hi0, lo0, c0, cl0);
        const float eps_nxt = step_eps(tn);
        cnt0 += c0;
        if (__ballot(len > 0 && cl0 != c0) != 0ull) emit_ties(cur, len > 0, pid0, hi0, lo0, tm0, item0);
        if (wlen > 1) second_pair(cur, eps_cur, item0);
        mask_tail(nxt, item0 + NIB * 32);
        eps_cur = eps_nxt;
        slot_nxt = slot_nxt + 1 == NBUF ? 0 : slot_nxt + 1;
        slot_stg = slot_stg + 1 == NBUF ? 0 : slot_stg + 1;
        ++nstep;
    };

    for (int64_t st = s_begin;;) {
        body(accA, accB, st);
        if (++st >= s_end) break;
        if (SP == 1) barrier_before(st);
        body(accB, accA, st);
        if (++st >= s_end) break;
        barrier_before(st);
    }
    flush_records();

    // ---- statistics and write-back (exact lists never change in a pass)
    const uint64_t nsc = (uint64_t)(s_end - s_begin);
    ncmp += nsc * (uint64_t)len * NSC;
    nslot += nsc * (uint64_t)wlen * NSC;
    {
        const uint32_t lanes = (uint32_t)__popcll(__ballot(len > 0));
        const int64_t first = s_begin * (NIB * 32);
        const int64_t last = std::min<int64_t>(s_end * (NIB * 32), a.m);
        if (last > first) nscored += (uint64_t)(lanes / 2) * (uint64_t)(last - first);
    }
    const uint32_t tot0 = pair_sum(cnt0), tot1 = pair_sum(cnt1);
    if (u >= 0 && half == 0) {
        if (len > 0) atomicAdd(&a.cnt_out[pid0], tot0);
        if (len > 1) atomicAdd(&a.cnt_out[pid1], tot1);
    }
}

template <int NKS>
__global__ __launch_bounds__(512) void k_exact(CountArgs a) {
    extern __shared__ __attribute__((aligned(16))) uint8_t lds[];
    __shared__ int2 recs[WAVES_PER_WG * REC_PER_WAVE];
    const int lane = threadIdx.x & 63;
    uint64_t ncmp = 0, nslot = 0, nstep = 0, nscored = 0;
    exact_tile<NKS>(a, (int64_t)blockIdx.x, lds, recs, ncmp, nslot, nstep, nscored);
    uint64_t tot = ncmp, tslot = nslot;
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) {
        tot += __shfl_xor(tot, o, 64);
        tslot += __shfl_xor(tslot, o, 64);
    }
    if (lane == 0 && a.stat) {
        atomicAdd(a.stat, (unsigned long long)tot);
        atomicAdd(a.stat + 2, (unsigned long long)tslot);
        atomicAdd(a.stat + 6, (unsigned long long)nscored);
    }
    // executed matrix-core flop: 8 x 32 users by 64 items over the padded dimension per step
    // (a tile runs one score block more than it has steps: the prologue's)
    constexpr unsigned long long FLOP_PER_STEP = 2ull * WAVES_PER_WG * USER_BLOCK * EX_NIB * 32 * NKS * frag_ks(SK_BF16);
    if (threadIdx.x == 0 && a.stat && nstep) atomicAdd(a.stat + 4, (unsigned long long)(nstep + 1) * FLOP_PER_STEP);
}

template <int NKS>
hipError_t launch_exact_nks(const CountArgs &a, int nsplit, hipStream_t st) {
    using G = ExactGeom<NKS>;
    if (a.nks != NKS) return hipErrorInvalidValue;
    constexpr int TASKS_PER_WG = WAVES_PER_WG * USER_BLOCK;
    const int64_t ntiles = (a.ntask + TASKS_PER_WG - 1) / TASKS_PER_WG;
    if (ntiles == 0) return hipSuccess;
    CountArgs b = a;
    b.ntiles = ntiles;
    b.tile_counter = nullptr;
    auto kern = k_exact<NKS>;
    hipError_t e = hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize, G::LDS_BYTES);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(kern, dim3((unsigned)ntiles, (unsigned)nsplit), dim3(512), G::LDS_BYTES, st, b);
    return hipGetLastError();
}

}  // namespace

// Exact pass with BF16 scores (item steps of 64, one workgroup of 8 waves per
// 256 tasks and item split); the layouts are padded to nks k-steps, and no
// task holds more than two pairs.
hipError_t launch_exact_bf16(const CountArgs &a, int nsplit, hipStream_t st) {
    const int nks = a.nks;
    if (nks <= 4) return launch_exact_nks<4>(a, nsplit, st);
    if (nks <= 8) return launch_exact_nks<8>(a, nsplit, st);
    if (nks <= 13) return launch_exact_nks<13>(a, nsplit, st);
    if (nks <= 20) return launch_exact_nks<20>(a, nsplit, st);
    return hipErrorInvalidValue;
}

}  // namespace rkr
