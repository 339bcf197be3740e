// tile_common.h -- device helpers shared by the count kernels: MFMA operand
// types and the 32x32 matrix-core step per score kind, lane-pair and wave
// reductions, and the direct global -> LDS staging of an item step.
#pragma once
#include "rkr_internal.h"

namespace rkr {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef int i32x8 __attribute__((ext_vector_type(8)));
typedef int i32x4 __attribute__((ext_vector_type(4)));

template <int SK> struct FragT;
template <> struct FragT<SK_BF16> { using T = i32x4; };
template <> struct FragT<SK_F32> { using T = float; };
template <> struct FragT<SK_FP8> { using T = i32x8; };

template <int SK>
__device__ inline f32x16 mfma_step(f32x16 acc, typename FragT<SK>::T a, typename FragT<SK>::T b,
                                   int sa, int sb) {
    if constexpr (SK == SK_BF16) {
        return __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8, a),
                                                       __builtin_bit_cast(bf16x8, b), acc, 0, 0, 0);
    } else if constexpr (SK == SK_F32) {
        return __builtin_amdgcn_mfma_f32_32x32x2f32(a, b, acc, 0, 0, 0);
    } else {
        // A and B in FP8 e4m3 (format code 0); per-lane E8M0 scales (127 = 1.0)
        return __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(a, b, acc, 0, 0, 0, sa, 0, sb);
    }
}

// Sum of a value over the lane pair (l, l + 32).
__device__ inline uint32_t pair_sum(uint32_t v) {
    auto r = __builtin_amdgcn_permlane32_swap(v, v, false, false);
    return r[0] + r[1];
}

// Inclusive prefix sum over the 64 lanes.
__device__ inline uint32_t wave_incl_scan(uint32_t v, int lane) {
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        uint32_t t = __shfl_up(v, o, 64);
        if (lane >= o) v += t;
    }
    return v;
}

// Copy step_bytes from global memory to LDS with global_load_lds_dwordx4: the
// 64 lanes of a wave fill 1 KB of LDS starting at the (wave-uniform) base.
// The step's four error-bound coefficients (32 bytes) follow its P tile in
// the same LDS stage: two lanes of wave 0 copy them, so they arrive with the
// tile instead of costing a memory round trip when the step needs them.
template <int LOADS>
__device__ inline void stage_step(const uint8_t *src, uint8_t *dst, int step_bytes, int tid, const double *coef) {
    const int wave = tid >> 6;
#pragma unroll
    for (int j = 0; j < LOADS; ++j) {
        const int wbase = (j * 512 + wave * 64) * 16;
        const int off = wbase + (tid & 63) * 16;
        if (off < step_bytes)
            __builtin_amdgcn_global_load_lds((const void *)(src + off),
                                             (__attribute__((address_space(3))) void *)(dst + wbase), 16, 0, 0);
    }
    if (wave == 0 && (tid & 63) < 2)
        __builtin_amdgcn_global_load_lds((const void *)(coef + 2 * (tid & 63)),
                                         (__attribute__((address_space(3))) void *)(dst + step_bytes), 16, 0, 0);
}

// s_waitcnt for at most N outstanding vector-memory operations (the other
// counters left free).
template <int N>
__device__ inline void wait_vm() {
    static_assert(N >= 0 && N < 64, "vmcnt is six bits");
    __builtin_amdgcn_s_waitcnt((N & 15) | ((N >> 4) << 14) | (7 << 4) | (15 << 8));
}

// Exact passes keep a near-tie record buffer per wave in LDS: records are
// appended there and copied out with one global atomic per flush.
constexpr int REC_PER_WAVE = 256;

}  // namespace rkr
