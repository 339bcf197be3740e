// mlp.h -- the learned rank estimator: per-user score sketch, features, and
// an 18 -> 64 -> 64 -> 1 MLP trained and run by this library's kernels.
#pragma once
#include "kernels.h"
#include "rkr.h"

#include <algorithm>
#include <cmath>

namespace rkr {

constexpr int SKETCH_LEVELS = 16;
constexpr int MLP_IN = 18, MLP_H = 64;
constexpr int MLP_NPARAM = MLP_H * MLP_IN + MLP_H + MLP_H * MLP_H + MLP_H + MLP_H + 1;   // 5441

struct Estimator {
    bool has_sketch = false;
    bool trained = false;
    int samples = 0;
    double last_loss = 0.0;
    DBuf sketch;        // [n][16] float
    DBuf params, grads, adam_m, adam_v;   // [MLP_NPARAM] float
    DBuf pred;          // [nq][n] float
    DBuf feat, targ, work;
};

rkr_status est_build_sketch(Estimator &e, const void *Um, int64_t n, const void *Pm_sorted, int64_t m, int d, int mk,
                            const double *unorm3, int samples, Scratch &sc, hipStream_t st);
// For each user: the spec scores against min(samples, 4096, m) norm-stratified
// items (the middle item of each of S equal buckets of the norm-sorted P),
// sorted descending and read at `levels` (2..64) positions spaced
// geometrically from 1 to S, ceil(S^(j / (levels - 1))).  sketch_out[u][j] =
// fl32(score / |u|), raw_out[u][j] = the FP64 score; either may be null.
// RKR_E_INVALID if m = 0, samples <= 0 or levels is out of range.
rkr_status sample_levels(const void *Um, int64_t n, const void *Pm_sorted, int64_t m, int d, int mk, int samples,
                         int levels, float *sketch_out, double *raw_out, Scratch &sc, hipStream_t st);
hipError_t est_features(const int32_t *pids, int64_t N, const int32_t *pair_u, const double *t64,
                        const double *unorm3, const float *sketch, const uint32_t *cnt, float *X, float *z,
                        hipStream_t st);
hipError_t est_fwd_bwd(Estimator &e, const float *X, const float *z, const int64_t *order, int64_t N, int64_t off,
                       int64_t nb, float scale, float *grad, double *loss_dev, Scratch &sc, hipStream_t st);
hipError_t est_adam(Estimator &e, float lr, int t, hipStream_t st);
hipError_t est_infer(Estimator &e, const float *X, const int32_t *pids, int64_t N, const int32_t *pair_u,
                     const double *t64, const double *unorm3, float *out, int qmajor_nq, int64_t qmajor_n,
                     hipStream_t st);
hipError_t est_init(Estimator &e, const float *z, int64_t N, uint64_t seed, Scratch &sc, hipStream_t st);
hipError_t est_perm(int64_t *order, int64_t N, int64_t a, int64_t b, hipStream_t st);
hipError_t est_mark_strided(int nq, int64_t n, int per, uint64_t seed, uint8_t *flag, hipStream_t st);
void est_release(Estimator &e);

}  // namespace rkr
