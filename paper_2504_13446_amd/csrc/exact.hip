// exact.hip -- the exact passes of the fused score + count (Def. 1, Sec. 2)
// for BF16 scores: for every (user, query) pair of a task list, the number of
// items certainly above the pair's FP64 threshold, every near tie emitted for
// the FP64 recheck.
//
// Same operands, entry lists, records and outputs as the count kernel's
// exact mode (count.hip), with a schedule and a compare made for these
// passes: one pair per task (the task builder gives a user with several
// pairs a task for each; the all-ranks passes have one pair per user).
//
//  * Threshold in the accumulator.  The first MFMA of a step starts from
//    C = -tf instead of 0 (tf = th, the FP32 value >= the FP64 threshold t64;
//    in plain mode tf = fl32(t64)), so the step ends with acc = score - tf.
//    The error bound of the count kernels covers this with one more term in
//    the FP32 accumulation: |acc - (u^.p^ - th)| <= gamma(dpad + 1) (|u^||p^| +
//    |th|) <= E_old (1 + 1/dpad) + gamma(dpad + 1) |th|, where E_old is the
//    usual per-step bound (its FP32 term is gamma(dpad) |u^||p^|, the other
//    terms are positive) and gamma(n) = 2 n 2^-23.  With E that sum:
//      acc > E             => s64 > th >= t64          (certainly above)
//      acc < -(E + th - tl) => s64 < tl <= t64          (certainly not above)
//    and anything in between is a near tie.  A score then costs one compare
//    (against ehi = E rounded up) and half a v_min3: a near tie is possible
//    only where min |acc| <= elo = E + th - tl, which sends the wave to the
//    rare path that writes records (exact masks there).
//  * The loop over item steps is software-pipelined.  While a wave counts
//    step st (accumulators `cur`) it computes step st + 1 (`nxt`); the two
//    are one basic block, in fixed chunks (one LDS fragment read, one MFMA,
//    a share of the compares; a scheduling fence after each), so the compare
//    of step st never waits for an MFMA of step st + 1 and the matrix cores
//    are fed between compares.  Counts stay per lane; the pair sum is taken
//    once, at the end.
//  * Items stream through NBUF LDS stages (buffer loads that write LDS);
//    the workgroup meets at one barrier per SP steps.  Step st + D is staged
//    at step st; at a barrier before step st0, the stages of steps up to
//    st0 + SP have landed (each wave waits until at most the copies of later
//    steps are in flight), and a stage is overwritten only after a barrier
//    has followed every read of it.
//  * Shape.  A step holds 32 items (one MFMA block) and a workgroup 12 waves
//    of 32 users: at about 160 VGPRs three waves share a SIMD, so a wave
//    waiting on LDS or the barrier leaves two to feed the matrix core (the
//    64-item, 8-wave shape needs 229 VGPRs: two waves per SIMD).  Nine
//    stages of 13 KB, SP = 4, D = 6.  The band of a step is computed in FP32
//    from per-step coefficients rounded up to FP32 (five FMAs instead of a
//    dozen FP64 operations and two conversions); see band_of32.
#include "rkr_internal.h"
#include "tile_common.h"

#include <algorithm>

namespace rkr {

namespace {

#ifndef EX_PIPE
#define EX_PIPE 4
#endif
constexpr int EX_LDS = 153600;     // LDS for the item stages and the record buffers

// A pass shape: NIB item blocks of 32 per step (64 or 32 items), NW waves per
// workgroup (32 users each), B32: the band of a step computed in FP32 from
// coefficients rounded up, instead of FP64.
template <int NKS, int NIB, int NW, bool B32>
struct ExactGeom {
    static constexpr int FB = frag_fb(SK_BF16);
    static constexpr int STEP_BYTES = NIB * NKS * 64 * FB;
    static constexpr int STAGE = STEP_BYTES + 32;   // item tile + the step's four error-bound coefficients
    static constexpr int COEF_LANES = B32 ? 1 : 2;  // 16-byte copies of the coefficients
    static constexpr int REC_BYTES = NW * REC_PER_WAVE * 8;
    static constexpr int NBUF_FIT = (EX_LDS - REC_BYTES) / STAGE;
    static constexpr int NBUF_MAX = NIB == 1 ? 9 : 5;
    static constexpr int NBUF = NBUF_FIT > NBUF_MAX ? NBUF_MAX : NBUF_FIT;
    static_assert(NBUF >= 3, "the pipeline needs three LDS stages");
    // barrier period and staging distance: D >= SP + 1 (steps st0 + 1 .. st0
    // + SP are staged before the barrier at st0) and D <= NBUF - SP + 1 (the
    // stage step st + D overwrites was last read before the previous barrier)
    static constexpr int SP = NBUF >= 9 ? 4 : (NBUF >= 5 ? 2 : 1);
    static constexpr int D = NBUF - SP + 1;
    static_assert(D >= SP + 1, "staging distance");
    static constexpr int LOADS = (STEP_BYTES + NW * 1024 - 1) / (NW * 1024);
    static constexpr int LDS_BYTES = NBUF * STAGE;   // dynamic LDS (the record buffers are a static array)
    static constexpr int SR = 2 / NIB;               // kernel steps per 64-item step of the host's ranges
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
template <int STEP_BYTES, int LOADS, int NW, int COEF_LANES>
struct StageCopy {
    uint32_t voff[LOADS];   // this lane's byte offsets in the step (loop invariant)
    uint32_t lds_off[LOADS + 1];   // the wave's LDS offsets in a stage, then the coefficients'
    int nload;              // copies this wave issues per step (wave-uniform)
    __device__ StageCopy(int wave, int lane) {
        nload = 0;
#pragma unroll
        for (int j = 0; j < LOADS; ++j) {
            const int wbase = (j * NW * 64 + wave * 64) * 16;
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
    __device__ void operator()(const uint8_t *src, uint32_t stage_off, int wave, int lane, const void *coef) const {
        const i32x4 rp = rsrc(src, STEP_BYTES);
#pragma unroll
        for (int j = 0; j < LOADS; ++j)
            if ((int)lds_off[j] < STEP_BYTES) copy16(rp, __builtin_amdgcn_readfirstlane(stage_off + lds_off[j]), voff[j]);
        if (wave == 0 && lane < COEF_LANES)
            copy16(rsrc(coef, COEF_LANES * 16), __builtin_amdgcn_readfirstlane(stage_off + lds_off[LOADS]),
                   (uint32_t)(lane * 16));
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

template <int NKS, bool SCREEN, int NIB, int NW, bool B32>
__device__ inline void pass_tile(const CountArgs &a, const int64_t tile, const int split, uint8_t *lds, int2 *recs,
                                 int *wg_live, uint64_t &ncmp, uint64_t &nslot, uint64_t &nstep, uint64_t &nscored) {
    using G = ExactGeom<NKS, NIB, NW, B32>;
    using FT = typename FragT<SK_BF16>::T;
    constexpr int FB = G::FB, STEP_BYTES = G::STEP_BYTES, STAGE = G::STAGE, NBUF = G::NBUF;
    constexpr int SP = G::SP, D = G::D, LOADS = G::LOADS, SR = G::SR;
    constexpr int KS = frag_ks(SK_BF16), ES = elem_size(SK_BF16);
    constexpr int NSC = NIB * 16;    // scores per lane per step

    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;
    const int wave_u = __builtin_amdgcn_readfirstlane(wave);   // the same, known to be uniform
    const int l32 = lane & 31;
    const int half = lane >> 5;
    // the host's ranges are in 64-item steps; this pass's steps hold NIB * 32 items
    const int64_t r_begin = a.step0 + (int64_t)split * a.steps_per_split;
    const int64_t s_begin = r_begin * SR;
    const int64_t s_end = std::min<int64_t>(std::min<int64_t>(r_begin + a.steps_per_split, a.step_end) * SR,
                                            (a.m + NIB * 32 - 1) / (NIB * 32));
    // the loop's step numbers in 32 bits, so that its tests are scalar
    // compares (item numbers are 32-bit in the records, so steps fit)
    const int sb32 = (int)s_begin, se32 = (int)s_end;
    const int s_full = (int)(a.m / (NIB * 32));   // steps with no item past the end
    // the step's error-bound coefficients (FP64, or FP32 rounded up)
    const void *coef_base = B32 ? (const void *)(NIB == 1 ? a.step_coef32_half : a.step_coef32)
                                : (const void *)(NIB == 1 ? a.step_coef_half : a.step_coef);
    auto coef_of = [&](int64_t st) -> const void * {
        return (const uint8_t *)coef_base + st * (B32 ? 16 : 32);
    };

    // ---- the lane's user: register-stationary fragments, norms, its pair
    const int64_t t = tile * (NW * USER_BLOCK) + wave * USER_BLOCK + l32;
    const int u = t < a.ntask ? a.task_user[t] : -1;
    bool live = u >= 0 && a.ent_len[split * a.len_stride + t] > 0;
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
    // The pair: pid, the FP32 values th >= t64 >= tl bracketing its FP64
    // threshold and tm = fl32(t64).  The accumulators start from -tf (tf = th,
    // or tm in plain mode), so they end at score - tf (see the top of the file).
    // A screening pair carries its remaining budget rem instead (it dies when
    // rem turns negative), and its lists are the split's own copy.
    int pid = 0, rem = 0;
    float th = 0.0f, tl = 0.0f, tm = 0.0f;
    // (a tile may reach past the padded task list: its entries are never read)
    const int64_t e_pair = (t < a.ntask ? a.blk_base[t >> 5] : 0) + l32 + (SCREEN ? (int64_t)split * a.cap_total : 0);
    if (live) {
        pid = a.ent_pid[e_pair];
        th = a.ent_th[e_pair];
        if constexpr (SCREEN) {
            rem = (int)a.ent_cnt[e_pair];
        } else {
            tl = a.ent_tl[e_pair];
            tm = a.ent_tm[e_pair];
        }
    }
    // (screening entries of plain mode already hold fl32(t) in th)
    const float tf = (!SCREEN && a.plain) ? tm : th;
    f32x16 negt;
#pragma unroll
    for (int r = 0; r < 16; ++r) negt[r] = -tf;
    // the threshold's share of the error bound, gamma(dpad + 1) |tf|, and the
    // bracket width th - tl (exact: both are FP32 values one ulp apart at most)
    const double gam1 = 2.0 * (double)(a.dpad + 1) * 0x1p-23;
    const double th_term = gam1 * fabs((double)tf);
    // (a lane without a live pair gets an empty near-tie band, elo = -inf,
    // so that the per-step near-tie test is a bare compare)
    const double bracket = live ? (double)th - (double)tl : -(double)__builtin_inff();
    const double inflate = 1.0 + 1.0 / (double)a.dpad;
    // the FP32 form of the band: every input rounded up; each of the five
    // FP32 operations on these non-negative values loses at most a relative
    // 2^-24 (plus 2^-150 if the result is subnormal), so a final factor 1 +
    // 2^-20 and an added 2^-126 keep it above the FP64 value.  Plain mode
    // (no near ties, acc > 0 counts) comes out of the same instructions: a
    // zero factor, threshold term and 2^-126 give ehi = 0, and a bracket of
    // -inf gives elo = -inf.
    const float uh32 = f32_round_up(un_hat), ud32 = f32_round_up(un_del), uf32 = f32_round_up(un_full);
    const float infl32 = a.plain ? 0.0f : f32_round_up(inflate), tt32 = a.plain ? 0.0f : f32_round_up(th_term);
    const float br32 = a.plain ? -__builtin_inff() : f32_round_up(bracket);   // -inf without a live pair too
    const float tiny32 = a.plain ? 0.0f : 0x1p-126f;
    // plain verdict of a near tie: score > tm, i.e. acc > tm - th (exact)
    const float pd = tm - th;
    uint32_t cnt = 0;   // per-lane certain count of the pair
    uint32_t nlive = 0;   // screening: steps scored with a live pair
    // Cauchy-Schwarz settle of the exact passes (Lemma 1 over the
    // norm-sorted items): |s64(u,p)| <= |u||p| (1 + gamma64) and |p| <= Z[st]
    // from step st on, so from the first step s_set with |u| Z[st] (1 +
    // 2^-30) < L the pair's verdict is the same for every later item: with
    // L = tl <= t64 nothing is above; with L = -th everything is.  The
    // workgroup scores up to the last settle step of its live pairs, and a
    // pair settled above adds the items it did not score.  (s_set is found
    // after the first copies are issued, so that its loads overlap them.)
    int64_t s_set = INT64_MAX;
    bool set_above = false;
    auto znorm = [&](int64_t st) { return a.step_znorm[st / SR]; };
    auto find_settle = [&]() {
        // (screening passes stop on their budgets; they do not settle)
        if constexpr (SCREEN) return;
        if (!(live && a.step_znorm && !a.plain)) return;
        const float lpos = tl;
        const double L = fmax((double)lpos, -(double)th);
        if (!(L > 0.0)) return;
        const double nu = un_full * (1.0 + 0x1p-30);
        // the range's smallest bound first: most pairs never settle in it
        if (!(nu * znorm(s_end - 1) < L)) return;
        int64_t lo = s_begin, hi = s_end - 1;
        while (lo < hi) {
            const int64_t mid = (lo + hi) >> 1;
            if (nu * znorm(mid) < L) hi = mid; else lo = mid + 1;
        }
        s_set = lo;
        set_above = th < 0.0f;
    };
    // items of the pass's range from step st on (real items only)
    auto items_from = [&](int64_t st) -> int64_t {
        return std::max<int64_t>(0, std::min<int64_t>(s_end * (NIB * 32), a.m) - st * (NIB * 32));
    };
    // the pass ends before step stop (s_end: it ran to the end)
    auto settle_rest = [&](int64_t stop) {
        if (!(live && set_above && stop < s_end)) return;
        const int64_t rest = items_from(stop);
        if constexpr (SCREEN) {
            rem -= (int)rest;
            live = rem >= 0;
        } else if (half == 0) {
            cnt += (uint32_t)rest;
        }
    };
    if (!__syncthreads_or(live) || s_begin >= s_end) return;

    // ---- near-tie records: a per-wave LDS buffer, flushed with one global
    // atomic when full and at the end.  It is an array of its own, apart from
    // the item stages, so that the compiler can tell that writing a record
    // does not touch a stage an LDS copy is still filling.
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

    // The band of a step in accumulator units (acc = score - tf): certainly
    // above when acc > ehi, certainly not above when acc < -elo, a near tie in
    // between.  From the step's coefficients (staged with its tile).
    auto band_of = [&](double ca, double cb, double cc, double cabs, float &ehi, float &elo) {
        if (a.plain) {
            ehi = 0.0f;                  // acc > 0: the plain FP32 verdict, no near ties
            elo = -__builtin_inff();
            return;
        }
        const double E = (un_hat * ca + un_del * cb + un_full * cc + cabs) * inflate + th_term;
        ehi = f32_round_up(E * (1.0 + 1e-9));
        elo = f32_round_up((E + bracket) * (1.0 + 1e-9));
    };
    // (no branch: plain mode's edges come from the set-up values above; the
    // coefficients are finite, so e is 0 there)
    auto band_of32 = [&](float ca, float cb, float cc, float cabs, float &ehi, float &elo) {
        const float e = __builtin_fmaf(__builtin_fmaf(uh32, ca, __builtin_fmaf(ud32, cb, __builtin_fmaf(uf32, cc, cabs))),
                                       infl32, tt32);
        ehi = __builtin_fmaf(e, 1.0f + 0x1p-20f, tiny32);
        elo = __builtin_fmaf(e + br32, 1.0f + 0x1p-20f, tiny32);
    };
    auto band_of_tile = [&](const uint8_t *tile, float &ehi, float &elo) {
        if constexpr (B32) {
            const float *cs = (const float *)(tile + STEP_BYTES);
            band_of32(cs[0], cs[1], cs[2], cs[3], ehi, elo);
        } else {
            const double *cs = (const double *)(tile + STEP_BYTES);
            band_of(cs[0], cs[1], cs[2], cs[3], ehi, elo);
        }
    };
    // item of score r of block ib in this lane, for a step starting at item0
    auto item_of = [&](int64_t item0, int ib, int r) -> int64_t {
        return item0 + ib * 32 + 8 * (r >> 2) + 4 * half + (r & 3);
    };
    // near ties of the pair in one step to the record buffer, each with the
    // plain FP32 verdict in its top bit.  32-item steps (NIB = 1): one score
    // position at a time, a wave ballot of the lanes whose score there is a
    // near tie, skipped (a uniform branch) when there is none, which is nearly
    // always: a step that gets here usually holds one or two near ties in all
    // of its 64 lanes.  A position adds at most 64 records, so one flush makes
    // room.  64-item steps (NIB = 2, the shape for 20 k-steps, where near ties
    // are many): per-lane bit masks of all 32 positions and one pass over the
    // set bits (32 ballots cost more there).
    static_assert(REC_PER_WAVE >= 64, "a score position's records must fit the buffer");
    auto emit_by_position = [&](const f32x16 *acc, float ehi, float elo, int64_t item0) {
#pragma unroll
        for (int ib = 0; ib < NIB; ++ib)
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                const float v = acc[ib][r];
                const bool tie = live & (v >= -elo) & !(v > ehi);
                const uint64_t m = __ballot(tie);
                if (m == 0ull) continue;
                const int n = (int)__popcll(m);
                if (rb_n + n > REC_PER_WAVE) flush_records();
                if (tie) {
                    const int pos =
                        rb_n + (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32),
                                                              __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
                    const int plainbit = (v > pd) ? (int)0x80000000 : 0;
                    recbuf[pos] = make_int2(pid, (int)item_of(item0, ib, r) | plainbit);
                }
                rb_n += n;
            }
    };
    auto emit_by_masks = [&](const f32x16 *acc, float ehi, float elo, int64_t item0) {
        // bit ib * 16 + r of each mask is score r of block ib (shifted in
        // from the top, so that no per-bit constants are needed)
        uint32_t umask = 0, pmask = 0;
#pragma unroll
        for (int ib = NIB - 1; ib >= 0; --ib)
#pragma unroll
            for (int r = 15; r >= 0; --r) {
                const float v = acc[ib][r];
                umask = (umask << 1) | ((v >= -elo && !(v > ehi)) ? 1u : 0u);
                pmask = (pmask << 1) | ((v > pd) ? 1u : 0u);
            }
        if (!live) umask = 0;
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
    auto emit_ties = [&](const f32x16 *acc, float ehi, float elo, int64_t item0) {
        if constexpr (NIB == 1)
            emit_by_position(acc, ehi, elo, item0);
        else
            emit_by_masks(acc, ehi, elo, item0);
    };
    // scores of items past the end never count
    auto mask_tail = [&](f32x16 *acc, int s) {
        if (s < s_full) return;
        const int64_t item0 = (int64_t)s * (NIB * 32);
        const int lim = (int)(a.m - item0) - 4 * half;
#pragma unroll
        for (int ib = 0; ib < NIB; ++ib)
#pragma unroll
            for (int r = 0; r < 16; ++r)
                if (ib * 32 + 8 * (r >> 2) + (r & 3) >= lim) acc[ib][r] = -__builtin_inff();
    };
    // the accumulators of a step (MFMA block only): score - tf
    auto scores = [&](const uint8_t *tile, f32x16 *acc) {
#pragma unroll
        for (int s = 0; s < NKS; ++s)
#pragma unroll
            for (int ib = 0; ib < NIB; ++ib) {
                const FT af = *(const FT *)(tile + ((ib * NKS + s) * 64 + lane) * FB);
                acc[ib] = mfma_step<SK_BF16>(s == 0 ? negt : acc[ib], af, bfrag[s], 127, 127);
            }
    };
    // The accumulators of the next step (nxt, from the stage at tn) and the
    // count of the current step (cur) in one block, in a fixed order: chunk i
    // reads fragment i + PIPE, issues MFMA i and handles the next share of the
    // current scores (one compare and half a min3 each); a scheduling fence
    // closes each chunk, so every MFMA has PIPE fragment reads in flight ahead
    // of it and compare instructions between it and the next one.  side(i)
    // adds other work of the step to chunk i.  dmin is the smallest |acc| of
    // the lane: a near tie is possible only if dmin <= elo.
    auto score_and_count = [&](const uint8_t *tn, f32x16 *nxt, const f32x16 *cur, float ehi, uint32_t &c,
                               float &dmin, auto &&side) {
        constexpr int NRD = NKS * NIB;
        constexpr int PIPE = NRD < EX_PIPE ? NRD : EX_PIPE;
        auto frag = [&](int i) { return *(const FT *)(tn + (((i % NIB) * NKS + i / NIB) * 64 + lane) * FB); };
        FT fr[PIPE];
#pragma unroll
        for (int i = 0; i < PIPE; ++i) fr[i] = frag(i);
        if constexpr (SCREEN) dmin = 0.0f;   // (unused)
#pragma unroll
        for (int i = 0; i < NRD; ++i) {
            const FT f = fr[i % PIPE];
            if (i + PIPE < NRD) fr[i % PIPE] = frag(i + PIPE);
            nxt[i % NIB] = mfma_step<SK_BF16>(i < NIB ? negt : nxt[i % NIB], f, bfrag[i / NIB], 127, 127);
            // scores in pairs (one min3 each), 32 over the NRD chunks
            const int k0 = (i * NSC / NRD) & ~1, k1 = ((i + 1) * NSC / NRD) & ~1;
            for (int k = k0; k < k1; k += 2) {
                const float v0 = cur[k / 16][k % 16], v1 = cur[(k + 1) / 16][(k + 1) % 16];
                const uint32_t b = ((v0 > ehi) ? 1u : 0u) + ((v1 > ehi) ? 1u : 0u);
                // min(dmin, |v0|, |v1|) in one instruction (fminf would
                // quieten its operands first; the scores are never NaN);
                // screening has no near ties to look for.  The first pair
                // starts both (no constants to move in).
                if (k == 0) {
                    c = b;
                    if constexpr (!SCREEN) asm("v_min_f32 %0, |%1|, |%2|" : "=v"(dmin) : "v"(v0), "v"(v1));
                } else {
                    c += b;
                    if constexpr (!SCREEN)
                        asm("v_min3_f32 %0, %1, |%2|, |%3|" : "=v"(dmin) : "v"(dmin), "v"(v0), "v"(v1));
                }
            }
            // keep this chunk's share here: the compiler would otherwise
            // sink it out of the block to where the count is used
            if (k1 > 0) {
                if constexpr (SCREEN)
                    asm volatile("" : "+v"(c));
                else
                    asm volatile("" : "+v"(c), "+v"(dmin));
            }
            side(i);
            __builtin_amdgcn_sched_barrier(0);
        }
    };

    // ---- prologue: stage steps s_begin .. s_begin + D - 1; the first lands
    const StageCopy<STEP_BYTES, LOADS, NW, G::COEF_LANES> stage(wave_u, lane);
    const int nload = stage.nload;
    // the LDS offset of the stages (M0 takes LDS offsets, not generic addresses)
    const uint32_t lds_base = (uint32_t)(uintptr_t)(const __attribute__((address_space(3))) uint8_t *)lds;
    const int64_t npro = std::min<int64_t>(D, s_end - s_begin);
    for (int64_t k = 0; k < npro; ++k)
        stage(a.plp + (s_begin + k) * (int64_t)STEP_BYTES, lds_base + k * STAGE, wave_u, lane, coef_of(s_begin + k));
    // before the barrier at step st0: steps up to st0 + SP have landed; the
    // copies of later steps (staged up to step st0 - 1 + D) may be in flight
    find_settle();
    // Exact: the workgroup scores the steps up to the last settle step of its
    // live pairs (a maximum taken once; wg_live[0] holds it, in steps past
    // s_begin).  Screening: it stops at a barrier once none of its pairs
    // needs the steps from there on (dead or settled), with "any needs"
    // flags, one slot per barrier, three in rotation: the slot of barrier
    // b - 1 is cleared after barrier b (every read of it came before) and
    // written again only after barrier b + 1.
    if constexpr (!SCREEN) {
        int need = live ? (int)(std::min<int64_t>(s_set, s_end) - s_begin) : 0;
#pragma unroll
        for (int o = 32; o >= 1; o >>= 1) need = std::max(need, __shfl_xor(need, o, 64));
        if (lane == 0) atomicMax(&wg_live[0], need);
    }
    wait_vm_n((int)(npro - 1) * nload);
    __syncthreads();
    const int s_run = SCREEN ? se32 : sb32 + __builtin_amdgcn_readfirstlane(wg_live[0]);
    int lslot = 0;
    auto barrier_before = [&](int st0) -> bool {
        // copies of steps past s_run issued before it was known only make
        // this wait stricter
        const int last = std::min(st0 - 1 + D, s_run - 1);
        const int later = std::max(0, last - (st0 + SP));
        wait_vm_n(later * nload);
        if constexpr (!SCREEN) {
            __syncthreads();
            return true;
        } else {
            // (the ballot runs on every lane, outside the lane-0 branch)
            const bool wave_needs = __ballot(live && st0 < s_set) != 0ull;
            if (lane == 0 && wave_needs) atomicOr(&wg_live[lslot], 1);
            __syncthreads();
            const int any = wg_live[lslot];
            if (tid == 0) wg_live[lslot == 0 ? 2 : lslot - 1] = 0;
            lslot = lslot == 2 ? 0 : lslot + 1;
            return any != 0;
        }
    };

    f32x16 accA[NIB], accB[NIB];
    float ehi = 0.0f, elo = 0.0f;   // the band of the current step
    bool go = false;
    if (s_run > sb32) {
        scores(lds, accA);
        band_of_tile(lds, ehi, elo);
        mask_tail(accA, sb32);
        go = barrier_before(sb32);
    }

    int slot_nxt = 1 % NBUF;      // stage of step st + 1
    int slot_stg = D % NBUF;      // stage of step st + D
    // One step: stage st + D, count st (cur) while scoring st + 1 (nxt).
    // The last step of a tile scores a stale stage too (its result is never
    // used): the block then has no branch, and the compare stays in it.
    auto body = [&](f32x16 *cur, f32x16 *nxt, int st) {
        if (st + D < s_run)
            stage(a.plp + (int64_t)(st + D) * STEP_BYTES, lds_base + slot_stg * STAGE, wave_u, lane, coef_of(st + D));
        const int64_t item0 = (int64_t)st * (NIB * 32);
        const uint8_t *tn = lds + slot_nxt * STAGE;
        uint32_t c;
        float dmin;
        // inside the block: the next step's band (coefficients read first,
        // used half way)
        constexpr int NRD = NKS * NIB;
        using CT = typename std::conditional<B32, float, double>::type;
        const CT *csp = (const CT *)(tn + STEP_BYTES);
        CT cs0 = 0, cs1 = 0, cs2 = 0, cs3 = 0;
        float ehi_n = 0.0f, elo_n = 0.0f;
        score_and_count(tn, nxt, cur, ehi, c, dmin, [&](int i) {
            if (i == 0) {
                cs0 = csp[0];
                cs1 = csp[1];
                cs2 = csp[2];
                cs3 = csp[3];
            }
            if (i == NRD / 2) {
                if constexpr (B32)
                    band_of32(cs0, cs1, cs2, cs3, ehi_n, elo_n);
                else
                    band_of(cs0, cs1, cs2, cs3, ehi_n, elo_n);
            }
        });
        if constexpr (SCREEN) {
            // the budget left after this step's certainly-above items
            nscored += (uint64_t)(__popcll(__ballot(live)) / 2) *
                       (uint64_t)(st < s_full ? NIB * 32 : (int)(a.m - item0));
            nlive += live ? 1u : 0u;
            rem -= (int)pair_sum(c);   // both halves of the step's items (lanes l and l + 32)
            live = live && rem >= 0;
        } else {
            cnt += c;
            if (__ballot(dmin <= elo) != 0ull) emit_ties(cur, ehi, elo, item0);   // (elo = -inf: no live pair)
        }
        mask_tail(nxt, st + 1);
        ehi = ehi_n;
        elo = elo_n;
        slot_nxt = slot_nxt + 1 == NBUF ? 0 : slot_nxt + 1;
        slot_stg = slot_stg + 1 == NBUF ? 0 : slot_stg + 1;
        ++nstep;
    };

    int st = sb32;
    if (go)
        for (;;) {
            body(accA, accB, st);
            if (++st >= s_run) break;
            if (SP == 1 && !barrier_before(st)) break;
            body(accB, accA, st);
            if (++st >= s_run) break;
            if ((SP == 2 || ((st - sb32) & (SP - 1)) == 0) && !barrier_before(st)) break;
        }
    // the pass scored steps s_begin .. stop - 1; a workgroup that stops
    // early may still have copies in flight into its LDS: they land before
    // it ends
    const int64_t stop = go ? st : s_begin;
    if (stop < s_end) wait_vm<0>();
    settle_rest(stop);
    if constexpr (SCREEN) {
        if (u >= 0 && half == 0) {
            a.ent_len[split * a.len_stride + t] = live ? 1 : 0;
            if (live) a.ent_cnt[e_pair] = (uint32_t)rem;
        }
        ncmp += (uint64_t)nlive * NSC;
        nslot += ncmp;
        return;
    }
    flush_records();

    // ---- statistics and write-back (exact lists never change in a pass)
    const uint64_t nsc = (uint64_t)(stop - s_begin);
    const uint32_t lanes = (uint32_t)__popcll(__ballot(live));
    ncmp += nsc * (live ? 1u : 0u) * NSC;
    nslot += nsc * (lanes ? 1u : 0u) * NSC;
    {
        const int64_t first = s_begin * (NIB * 32);
        const int64_t last = std::min<int64_t>(stop * (NIB * 32), a.m);
        if (last > first) nscored += (uint64_t)(lanes / 2) * (uint64_t)(last - first);
    }
    const uint32_t tot = pair_sum(cnt);
    if (live && half == 0) atomicAdd(&a.cnt_out[pid], tot);
}

template <int NKS, bool SCREEN, int NIB, int NW, bool B32>
__global__ __launch_bounds__(NW * 64) void k_pass(CountArgs a) {
    extern __shared__ __attribute__((aligned(16))) uint8_t lds[];
    __shared__ int2 recs[SCREEN ? 1 : NW * REC_PER_WAVE];
    __shared__ int wg_live[3];
    const int lane = threadIdx.x & 63;
    if (threadIdx.x < 3) wg_live[threadIdx.x] = 0;   // read after the tile's first barrier
    uint64_t ncmp = 0, nslot = 0, nstep = 0, nscored = 0;
    // one workgroup per (tile, item split); a mapping that gave each XCD
    // consecutive tiles of one split (shared items in its L2) measured slower
    const int split = (int)blockIdx.y;
    const int64_t tile = blockIdx.x;
    pass_tile<NKS, SCREEN, NIB, NW, B32>(a, tile, split, lds, recs, wg_live, ncmp, nslot, nstep, nscored);
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
    // executed matrix-core flop: NW x 32 users by NIB x 32 items over the padded dimension per step
    // (a tile runs one score block more than it has steps: the prologue's)
    constexpr unsigned long long FLOP_PER_STEP = 2ull * NW * USER_BLOCK * NIB * 32 * NKS * frag_ks(SK_BF16);
    if (threadIdx.x == 0 && a.stat && nstep) atomicAdd(a.stat + 4, (unsigned long long)(nstep + 1) * FLOP_PER_STEP);
}

template <int NKS, bool SCREEN, int NIB, int NW, bool B32>
hipError_t launch_pass_nks(const CountArgs &a, int nsplit, hipStream_t st) {
    using G = ExactGeom<NKS, NIB, NW, B32>;
    if (a.nks != NKS) return hipErrorInvalidValue;
    constexpr int TASKS_PER_WG = NW * USER_BLOCK;
    const int64_t ntiles = (a.ntask + TASKS_PER_WG - 1) / TASKS_PER_WG;
    if (ntiles == 0) return hipSuccess;
    CountArgs b = a;
    b.ntiles = ntiles;
    b.tile_counter = nullptr;
    auto kern = k_pass<NKS, SCREEN, NIB, NW, B32>;
    hipError_t e = hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize, G::LDS_BYTES);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(kern, dim3((unsigned)ntiles, (unsigned)nsplit), dim3(NW * 64), G::LDS_BYTES, st, b);
    return hipGetLastError();
}

// The pass shape: 0 = 64-item steps, 8 waves, FP64 band; 1 = the same with
// the FP32 band; 2 = 32-item steps, 12 waves (three per SIMD), FP32 band.
// Shape 2 up to 13 k-steps (d <= 208 in BF16); with 20 its registers would
// spill, so shape 1.  RKR_PASS_SHAPE overrides the choice (for measurements).
int pass_shape(int nks) {
    const char *v = getenv("RKR_PASS_SHAPE");   // read per launch, so that a process can compare shapes
    const int forced = v ? atoi(v) : -1;
    if (forced >= 0 && forced <= 2) return forced;
    return nks <= 13 ? 2 : 1;
}

template <bool SCREEN, int NIB, int NW, bool B32>
hipError_t launch_pass_shape(const CountArgs &a, int nsplit, hipStream_t st) {
    const int nks = a.nks;
    if (nks <= 4) return launch_pass_nks<4, SCREEN, NIB, NW, B32>(a, nsplit, st);
    if (nks <= 8) return launch_pass_nks<8, SCREEN, NIB, NW, B32>(a, nsplit, st);
    if (nks <= 13) return launch_pass_nks<13, SCREEN, NIB, NW, B32>(a, nsplit, st);
    if (nks <= 20) return launch_pass_nks<20, SCREEN, NIB, NW, B32>(a, nsplit, st);
    return hipErrorInvalidValue;
}

template <bool SCREEN>
hipError_t launch_pass(const CountArgs &a, int nsplit, hipStream_t st) {
    switch (pass_shape(a.nks)) {
    case 1: return launch_pass_shape<SCREEN, 2, 8, true>(a, nsplit, st);
    case 0: return launch_pass_shape<SCREEN, 2, 8, false>(a, nsplit, st);
    default: return launch_pass_shape<SCREEN, 1, 12, true>(a, nsplit, st);
    }
}

}  // namespace

// Tasks per workgroup of the pipelined passes (users per tile).
int pass_tasks_per_wg(int nks) { return (pass_shape(nks) == 2 ? 12 : 8) * USER_BLOCK; }

// Exact pass with BF16 scores (item steps of 64, one workgroup of 8 waves per
// 256 tasks and item split); the layouts are padded to nks k-steps, and every
// task holds one pair.
hipError_t launch_exact_bf16(const CountArgs &a, int nsplit, hipStream_t st) { return launch_pass<false>(a, nsplit, st); }

// Screening pass with BF16 scores, one pair per task: a pair's remaining
// budget loses its certainly-above items; it dies (list length 0) when the
// budget turns negative, and a workgroup stops once all its pairs are dead.
// Items and splits as for the screening mode of the count kernel.
hipError_t launch_screen1_bf16(const CountArgs &a, int nsplit, hipStream_t st) { return launch_pass<true>(a, nsplit, st); }

}  // namespace rkr
