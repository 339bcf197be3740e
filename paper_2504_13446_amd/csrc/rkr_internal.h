// rkr_internal.h -- declarations shared by the host runtime and the HIP kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace rkr {

enum ScoreKind { SK_F32 = 0, SK_BF16 = 1, SK_FP8 = 2 };
enum MasterKind { MK_F32 = 0, MK_BF16 = 1 };

// 32x32 MFMA geometry per score kind.
//   KS: dimensions consumed by one MFMA k-step.
//   FB: bytes one lane contributes to one operand fragment.
//   ES: bytes per element of the low-precision copy.
__host__ __device__ constexpr int frag_ks(int sk) { return sk == SK_BF16 ? 16 : (sk == SK_FP8 ? 64 : 2); }
__host__ __device__ constexpr int frag_fb(int sk) { return sk == SK_BF16 ? 16 : (sk == SK_FP8 ? 32 : 4); }
__host__ __device__ constexpr int elem_size(int sk) { return sk == SK_BF16 ? 2 : (sk == SK_FP8 ? 1 : 4); }

constexpr int ITEM_BLOCK = 32;      // items per MFMA output block (rows)
constexpr int STEP_ITEMS = 64;      // items per pipeline step of the count kernel
constexpr int USER_BLOCK = 32;      // users per MFMA output block (columns)
constexpr int WAVES_PER_WG = 8;     // count kernel workgroup = 8 wave64

// ---------------------------------------------------------------------------
// Exactly-rounded float helpers (finite inputs).
// ---------------------------------------------------------------------------
__host__ __device__ inline float f32_next_up(float x) {
    union { float f; int32_t i; } v{x};
    if (v.i == (int32_t)0x80000000) { v.i = 1; return v.f; }   // -0 -> smallest positive
    v.i += (v.i >= 0) ? 1 : -1;
    return v.f;
}
__host__ __device__ inline float f32_next_down(float x) { return -f32_next_up(-x); }

// Largest float <= x and smallest float >= x.
__host__ __device__ inline float f32_round_down(double x) {
    float f = (float)x;
    if ((double)f > x) f = f32_next_down(f);
    return f;
}
__host__ __device__ inline float f32_round_up(double x) {
    float f = (float)x;
    if ((double)f < x) f = f32_next_up(f);
    return f;
}

// Monotone map float -> uint32 (a < b  <=>  key(a) < key(b)), for finite values.
__host__ __device__ inline uint32_t f32_order_key(float x) {
    union { float f; uint32_t u; } v{x};
    return (v.u & 0x80000000u) ? ~v.u : (v.u | 0x80000000u);
}

// Widen a master element to double (exact).
__device__ inline double master_elem(const void *base, int mk, int64_t i) {
    if (mk == MK_BF16) {
        uint32_t b = (uint32_t)((const uint16_t *)base)[i] << 16;
        return (double)__uint_as_float(b);
    }
    return (double)((const float *)base)[i];
}

// ---------------------------------------------------------------------------
// Count kernel arguments.
// ---------------------------------------------------------------------------
struct CountArgs {
    // items, sorted by norm, low precision, fragment-major:
    //   [item block b][k-step s][lane 0..63][FB bytes]
    const uint8_t *plp;
    int64_t m;
    int nks;                      // k-steps per vector
    const double *step_coef;      // [nsteps][4]: a, b, c, abs   (error-bound coefficients)
    const double *step_coef_half; // the same per 32-item block (pipelined passes with 32-item steps)
    const float *step_coef32;     // pipelined passes: step_coef rounded up to FP32, per 64 items
    const float *step_coef32_half;//   and per 32 items
    const int8_t *pexp;           // FP8: per-item power-of-two scale exponent (sorted order)
    // users, low precision, row-major [n][dpad]
    const uint8_t *ulp;
    int dpad;
    const double *unorm3;         // [n][3]: |u_hat|, |delta u|, |u|
    const int8_t *uexp;           // FP8: per-user exponent
    // tasks: 32 tasks form a block; block tb's entries sit at blk_base[tb] + i*32 + (t%32)
    const int32_t *task_user;     // [ntask_pad] user id, -1 for padding
    int64_t ntask;                // real tasks (ntask_pad is a multiple of 512)
    const int64_t *blk_base;
    int32_t *ent_len;             // [ntask_pad]; split screens: [nsplit][len_stride]
    int64_t len_stride;           // split screens: each split's own lists (0: one copy)
    int32_t *ent_pid;
    int32_t *ent_q;
    uint32_t *ent_cnt;            // exact: [nsplit][cap_total] counts; screen: remaining budget
                                  // (split screens: pid, th and cnt are [nsplit][cap_total] too)
    float *ent_th;                // FP32 value >= the FP64 threshold
    float *ent_tl;                // FP32 value <= the FP64 threshold
    const float *ent_tm;          // fl32 of the FP64 threshold (plain verdict of near ties)
    int64_t cap_total;
    const int32_t *bound;         // [nq] abandon bound (screen mode), INT32_MAX = none
    int nq;
    // P range: steps [step0 + split * steps_per_split, ...) of nsteps, cut at step_end
    int64_t nsteps;
    int64_t steps_per_split;
    int64_t step0;
    int64_t step_end;
    // exact mode outputs
    uint32_t *cnt_out;            // [npairs] += certain-above count
    int2 *emit;                   // near-tie records (pid, item)
    unsigned long long *emit_count;
    unsigned long long emit_cap;
    unsigned long long *stat;     // [0]: executed compares, [2]: compare lane slots, [4]: matrix-core flop,
                                  // [6]: (user, item) scores of users with a live pair
    const double *step_znorm;     // pipelined passes: per 64-item step, an upper bound of |p| from
                                  // that step on (Cauchy-Schwarz settle), or null
    int plain;                    // 1: compare the score with fl32(t) only (no band, no recheck)
    int hist_min;                 // screening: bucketed counting once some lane of a wave holds
                                  // this many live entries (0: never)
    const float *fold_th;         // bound check only: per-user FP32 threshold folded into the
                                  // accumulators (the form of the pipelined passes), or null
    const void *um_master;        // bound check only: master user rows [n][d]
    const void *pm_master;        // bound check only: master item rows in norm order [m][d]
    int d_master, mk_master;
    // persistent launch: workgroups take tiles from *tile_counter (zeroed before
    // the launch) until it passes ntiles; null = one workgroup per tile
    unsigned long long *tile_counter;
    int64_t ntiles;
    int persistent_ctas;
};

// CM_TABLE: the rank table's cells.  Task t is user t (ntask = n, no entry
// lists); user u's TABLE_COLS thresholds, rounded up to FP32, are read from
// ent_th[u * TABLE_COLS + j], and cnt_out[u * TABLE_COLS + j] += the count of
// items certainly above column j (a lower bound of the exact count).
// CM_BOUND: a check of the error bound.  Task t is user t (ntask = n); for
// every score of a real item the FP64 spec dot is recomputed from the master
// values (um_master, pm_master: user rows, items in norm order) and the
// largest |score - s64| / eps (eps: the bound the other modes use for that
// user and step) goes to cnt_out[0] (FP32 bits, rounded up), the number of
// scores with ratio above 1 to cnt_out[1].  With fold_th, the accumulators
// start from -th (th = fold_th[u]) as in the pipelined passes, and the check is
// |acc - (s64 - th)| against their bound E (1 + 1/dpad) + gamma(dpad + 1) |th|.
enum CountMode { CM_SCREEN = 0, CM_EXACT = 1, CM_TABLE = 2, CM_BOUND = 3 };
constexpr int TABLE_COLS = 48;

struct DeviceIndex;

// launchers (count.hip)
hipError_t launch_count(int sk, int mode, const CountArgs &a, int nsplit, int variant, hipStream_t st);
// the software-pipelined exact pass for BF16 scores (exact.hip); its tasks
// hold one pair each
hipError_t launch_exact_bf16(const CountArgs &a, int nsplit, hipStream_t st);
// tasks per workgroup of the pipelined passes for nks k-steps (their tile of users)
int pass_tasks_per_wg(int nks);
// the same kernel as a screening pass, one pair per task
hipError_t launch_screen1_bf16(const CountArgs &a, int nsplit, hipStream_t st);

}  // namespace rkr
