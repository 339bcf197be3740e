// paper_table.h -- the paper's rank table (Alg. 1, Sec. 4.2) and query
// step 1 on it (Sec. 4.3).
#pragma once
#include "kernels.h"

namespace rkr {

// Cells of users u0 .. u0 + nu - 1 from their sample scores S [nu][ns]
// (bucket l's samples at soff[l] .. soff[l + 1], bsize[l] = |P_l|), the spec
// norms unorm [n] and the largest item norm *pmax; writes fmin [n], step [n]
// and cells [n][tau] (FP32).  hipErrorInvalidValue for tau outside
// [2, paper_table_tau_max()].
hipError_t launch_ptab_cells(int64_t u0, int64_t nu, const double *S, int ns, int omega, const int32_t *soff,
                             const int64_t *bsize, int tau, const double *unorm, const double *pmax, double *fmin,
                             double *step, float *cells, hipStream_t st);
// Query step 1 for every (user, query) of a dense batch: t64 user-major
// [u * nq + q]; keys and estimates query-major [q * n + u].
hipError_t launch_ptq_bounds(int64_t n, int nq, int64_t m, int tau, const double *t64, const double *fmin,
                             const double *step, const float *cells, uint64_t *key_lo, uint64_t *key_hi, double *est,
                             hipStream_t st);
int paper_table_tau_max();

}  // namespace rkr
