// paper_table.hip -- the paper's own method: the rank table of Alg. 1
// (Sec. 4.2) with cells estimated from samples per norm bucket, and query
// step 1 (Sec. 4.3) on it.
//
// Table build, per user u (one wave per user):
//   f_max = |u| max|p| (the footnote's domain value, Cauchy-Schwarz), f_min =
//   -f_max; tau uniform thresholds t_j = f_min + j step, step = (f_max -
//   f_min) / (tau - 1), ascending.  For bucket l of the norm-sorted items,
//   A_l[j] = #{sampled p of bucket l : s(u,p) > t_j}; the cell is
//   T_j = 1 + sum_l (A_l[j] |P_l|) / s_l, added in bucket order in FP64 and
//   kept in FP32.  A sample above thresholds 0 .. L-1 only (L = #{j : t_j <
//   s(u,p)}) adds to A_l[0 .. L-1], so A_l is the suffix sum of a histogram
//   of L over the bucket's samples: one LDS histogram per bucket, one wave
//   scan, no per-threshold loop over samples.
// The sample scores s(u,p) are spec dots (FP64 sequential fma), computed by
// the register-tiled threshold kernel before this one.
#include "paper_table.h"

namespace rkr {

// Number of thresholds t_j = fmin + j step (j < tau) that satisfy t_j < x
// (strict = false: t_j <= x).  The t_j do not decrease in j (a product and a
// sum, each rounded monotonically), so the count is where they pass x; the
// quotient gives a first guess and direct comparisons settle it.
__device__ inline int ptab_count_below(double f0, double step, int tau, double x, bool strict) {
    auto below = [&](int j) {
        const double t = f0 + (double)j * step;
        return strict ? t < x : t <= x;
    };
    int g;
    if (step > 0.0) {
        double q = floor((x - f0) / step) + 1.0;
        q = fmin(fmax(q, 0.0), (double)tau);
        g = (int)q;
    } else {
        g = below(0) ? tau : 0;
    }
    while (g > 0 && !below(g - 1)) --g;
    while (g < tau && below(g)) ++g;
    return g;
}

// at most 32 columns per lane: tau + 1 histogram slots over 64 lanes
constexpr int PT_PER_LANE = 32;
constexpr int PT_TAU_MAX = 64 * PT_PER_LANE - 1;

// One wave per user of the chunk [u0, u0 + nu).  S: the chunk's sample scores
// [nu][ns] (bucket l's at soff[l] .. soff[l + 1]); bsize[l] = |P_l|.
__global__ __launch_bounds__(64) void k_ptab_cells(int64_t u0, int64_t nu, const double *S, int ns, int omega,
                                                   const int32_t *soff, const int64_t *bsize, int tau,
                                                   const double *unorm, const double *pmax, double *fmin_out,
                                                   double *step_out, float *cells) {
    __shared__ uint32_t H[PT_TAU_MAX + 1];
    const int64_t ul = blockIdx.x;
    if (ul >= nu) return;
    const int64_t u = u0 + ul;
    const int lane = threadIdx.x;
    const double fmax_u = unorm[u] * pmax[0];
    const double fmin_u = -fmax_u;
    const double step = (fmax_u - fmin_u) / (double)(tau - 1);
    // lane owns columns j = lane * per .. lane * per + per - 1
    const int per = (tau + 1 + 63) / 64;
    double T[PT_PER_LANE];
#pragma unroll
    for (int i = 0; i < PT_PER_LANE; ++i) T[i] = 1.0;
    const double *Su = S + ul * ns;
    // per <= PT_PER_LANE since tau <= PT_TAU_MAX
    for (int l = 0; l < omega; ++l) {
        const int b0 = soff[l], sl = soff[l + 1] - b0;
        if (sl == 0) continue;
        for (int j = lane; j <= tau; j += 64) H[j] = 0u;
        __syncthreads();
        for (int i = lane; i < sl; i += 64)
            atomicAdd(&H[ptab_count_below(fmin_u, step, tau, Su[b0 + i], true)], 1u);
        __syncthreads();
        // A[j] = sum of H[L] over L > j: the lane's own range first (from its
        // top down), then the sums of the lanes above it
        uint32_t part = 0;
        for (int i = 0; i < per; ++i) {
            const int L = lane * per + i;
            if (L <= tau) part += H[L];
        }
        uint32_t above = 0;   // sum of the parts of lanes > lane
        {
            uint32_t v = part;
#pragma unroll
            for (int o = 1; o < 64; o <<= 1) {
                const uint32_t t = __shfl_down(v, o, 64);
                if (lane + o < 64) v += t;
            }
            above = v - part;     // inclusive suffix minus own part
        }
        const double wsz = (double)bsize[l];
        const double ws = (double)sl;
        uint32_t acc = above;
#pragma unroll
        for (int i = PT_PER_LANE - 1; i >= 0; --i) {
            if (i < per) {
                const int j = lane * per + i;
                if (j < tau) {
                    // acc holds the sum of H[L] over L > j
                    T[i] = T[i] + ((double)acc * wsz) / ws;
                }
                if (j <= tau) acc += H[j];
            }
        }
        __syncthreads();      // the next bucket clears H
    }
#pragma unroll
    for (int i = 0; i < PT_PER_LANE; ++i) {
        const int j = lane * per + i;
        if (i < per && j < tau) cells[u * tau + j] = (float)T[i];
    }
    if (lane == 0) {
        fmin_out[u] = fmin_u;
        step_out[u] = step;
    }
}

// Query step 1 on the paper's table, per pair (u, q) (t64 user-major
// [u * nq + q]): L = #{j : t_j <= u.q}; r_lo = T[L] (1 when L = tau), r_hi =
// T[L-1] (m + 1 when L = 0); the estimate of step 3 interpolates linearly in
// u.q between (t[L-1], r_hi) and (t[L], r_lo), r_lo at either end or between
// equal thresholds.  Outputs are query-major [q * n + u]: keys (order key of
// the FP32 bound) << 32 | u, and the FP64 estimate; the transposition goes
// through an LDS tile of 32 users x 32 queries so that reads and writes
// coalesce.
__global__ __launch_bounds__(256) void k_ptq_bounds(int64_t n, int nq, int64_t m, int tau, const double *t64,
                                                    const double *fmin, const double *step, const float *cells,
                                                    uint64_t *key_lo, uint64_t *key_hi, double *est, int qt_per) {
    __shared__ uint32_t s_lo[32][33], s_hi[32][33];
    __shared__ double s_e[32][33];
    const int64_t u0 = (int64_t)blockIdx.x * 32;
    const int tid = threadIdx.x;
    const int qt_end = min((nq + 31) / 32, (int)(blockIdx.y + 1) * qt_per);
    for (int qt = blockIdx.y * qt_per; qt < qt_end; ++qt) {
        const int q0 = qt * 32;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int uu = r * 8 + (tid >> 5), qq = tid & 31;
            const int64_t u = u0 + uu;
            const int q = q0 + qq;
            if (u < n && q < nq) {
                const double x = t64[u * nq + q];
                const double f0 = fmin[u], st = step[u];
                const int L = ptab_count_below(f0, st, tau, x, false);
                const float *row = cells + u * tau;
                const float rlo = L == tau ? 1.0f : row[L];
                const float rhi = L == 0 ? (float)(m + 1) : row[L - 1];
                double e = (double)rlo;
                if (L > 0 && L < tau) {
                    const double tA = f0 + (double)(L - 1) * st, tB = f0 + (double)L * st;
                    if (tB > tA) e = (double)rhi + ((double)rlo - (double)rhi) * ((x - tA) / (tB - tA));
                }
                s_lo[qq][uu] = f32_order_key(rlo);
                s_hi[qq][uu] = f32_order_key(rhi);
                s_e[qq][uu] = e;
            }
        }
        __syncthreads();
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int qq = r * 8 + tid / 32, uu = tid % 32;
            const int64_t u = u0 + uu;
            const int q = q0 + qq;
            if (u < n && q < nq) {
                const int64_t j = (int64_t)q * n + u;
                key_lo[j] = ((uint64_t)s_lo[qq][uu] << 32) | (uint64_t)u;
                key_hi[j] = ((uint64_t)s_hi[qq][uu] << 32) | (uint64_t)u;
                est[j] = s_e[qq][uu];
            }
        }
        __syncthreads();
    }
}

hipError_t launch_ptab_cells(int64_t u0, int64_t nu, const double *S, int ns, int omega, const int32_t *soff,
                             const int64_t *bsize, int tau, const double *unorm, const double *pmax, double *fmin,
                             double *step, float *cells, hipStream_t st) {
    if (nu <= 0) return hipSuccess;
    if (tau < 2 || tau > PT_TAU_MAX) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_ptab_cells, dim3((unsigned)nu), dim3(64), 0, st, u0, nu, S, ns, omega, soff, bsize, tau,
                       unorm, pmax, fmin, step, cells);
    return hipGetLastError();
}

hipError_t launch_ptq_bounds(int64_t n, int nq, int64_t m, int tau, const double *t64, const double *fmin,
                             const double *step, const float *cells, uint64_t *key_lo, uint64_t *key_hi, double *est,
                             hipStream_t st) {
    if (n <= 0 || nq <= 0) return hipSuccess;
    const int64_t gx = (n + 31) / 32;
    const int qtiles = (nq + 31) / 32;
    int gy = (int)std::max<int64_t>(1, std::min<int64_t>(qtiles, 4096 / std::max<int64_t>(1, gx)));
    const int qt_per = (qtiles + gy - 1) / gy;
    gy = (qtiles + qt_per - 1) / qt_per;
    hipLaunchKernelGGL(k_ptq_bounds, dim3((unsigned)gx, (unsigned)gy), dim3(256), 0, st, n, nq, m, tau, t64, fmin,
                       step, cells, key_lo, key_hi, est, qt_per);
    return hipGetLastError();
}

int paper_table_tau_max() { return PT_TAU_MAX; }

}  // namespace rkr
