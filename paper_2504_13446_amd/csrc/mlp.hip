// mlp.hip -- learned rank estimator (sketch, features, MLP training and inference).
#include "mlp.h"

namespace rkr {

rkr_status est_build_sketch(Estimator &, const void *, int64_t, const void *, int64_t, int, int, const double *,
                            int, Scratch &, hipStream_t) {
    return RKR_E_UNSUPPORTED;
}
rkr_status est_predict_for_query(Estimator &, int, const void *, const void *, int64_t, int, int, const double *,
                                 const float **, hipStream_t) {
    return RKR_E_STATE;
}
void est_release(Estimator &e) {
    e.sketch.release(); e.params.release(); e.grads.release(); e.adam_m.release(); e.adam_v.release();
    e.pred.release(); e.feat.release(); e.targ.release(); e.work.release();
}

}  // namespace rkr
