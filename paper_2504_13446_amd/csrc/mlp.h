// mlp.h -- the learned rank estimator: per-user score sketch, features, and
// an 18 -> 64 -> 64 -> 1 MLP trained and run by this library's kernels.
#pragma once
#include "kernels.h"
#include "rkr.h"

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
rkr_status est_predict_for_query(Estimator &e, int nq, const void *Qm, const void *Um, int64_t n, int d, int mk,
                                 const double *unorm3, const float **pred_out, hipStream_t st);
void est_release(Estimator &e);

}  // namespace rkr
