/*
 * rkr_oracle.c -- plain, slow CPU reference for exact reverse k-ranks.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
 * calls this file; only the test suite, the smoke check and the CPU-baseline
 * leg of the benchmark use it.  It shares no code, header or constant with the
 * GPU path.
 *
 * Every routine below is the textbook definition written out:
 *   - rank (paper Sec. 2, Def. 1): r(q,u,P) = 1 + #{p in P : u.p > u.q},
 *     strict ">" so equal scores are not counted;
 *   - the inner product is fixed to ONE floating-point evaluation, the
 *     "spec dot": acc = +0.0, then acc = fma(x[k], y[k], acc) for
 *     k = 0, 1, ..., d-1 in order, on the master values widened exactly to
 *     double.  The paper does not state a precision (Sec. 5 only says C++);
 *     the spec dot is the reading used throughout.
 *
 * Inputs are double arrays (row-major [rows][d]); the Python wrapper widens
 * FP32 / BF16 masters to double, which is exact.  Build without -ffast-math
 * and with -ffp-contract=off so that no expression is re-associated or fused
 * beyond the explicit fma() calls.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* Spec dot: sequential fused multiply-add in dimension order. */
static double spec_dot(const double *x, const double *y, int d)
{
    double acc = 0.0;
    for (int k = 0; k < d; ++k)
        acc = fma(x[k], y[k], acc);
    return acc;
}

static void set_threads(int nthreads)
{
#ifdef _OPENMP
    if (nthreads > 0)
        omp_set_num_threads(nthreads);
#else
    (void)nthreads;
#endif
}

int orc_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Spec inner products of every (x_i, y_j): out[i*ny + j]. */
void orc_dots(const double *X, int64_t nx, const double *Y, int64_t ny, int d,
              double *out)
{
    for (int64_t i = 0; i < nx; ++i)
        for (int64_t j = 0; j < ny; ++j)
            out[i * ny + j] = spec_dot(X + i * d, Y + j * d, d);
}

/* Euclidean norms: sqrt of the spec dot of a vector with itself. */
void orc_norms(const double *X, int64_t nx, int d, double *out)
{
    for (int64_t i = 0; i < nx; ++i)
        out[i] = sqrt(spec_dot(X + i * d, X + i * d, d));
}

/*
 * Def. 1 ranks.  For each listed user u (uids[j], or user j when uids is
 * NULL, j < nu) and each query q_i (i < nq):
 *     ranks[i*nu + j] = 1 + #{p in P : s(u,p) > s(u,q_i)}.
 * The item scores s(u,p) do not depend on the query, so each is evaluated
 * once per user and compared against every query threshold of that user.
 */
void orc_ranks(const double *U, int64_t n, const double *P, int64_t m,
               const double *Qv, int64_t nq, int d,
               const int64_t *uids, int64_t nu, int32_t *ranks, int nthreads)
{
    (void)n;
    set_threads(nthreads);
#pragma omp parallel
    {
        double *t = (double *)malloc(sizeof(double) * (size_t)(nq > 0 ? nq : 1));
        int64_t *cnt = (int64_t *)malloc(sizeof(int64_t) * (size_t)(nq > 0 ? nq : 1));
#pragma omp for schedule(dynamic, 4)
        for (int64_t j = 0; j < nu; ++j) {
            const double *u = U + (uids ? uids[j] : j) * d;
            for (int64_t i = 0; i < nq; ++i) {
                t[i] = spec_dot(u, Qv + i * d, d);
                cnt[i] = 0;
            }
            for (int64_t p = 0; p < m; ++p) {
                double s = spec_dot(u, P + p * d, d);
                for (int64_t i = 0; i < nq; ++i)
                    if (s > t[i])
                        cnt[i] += 1;
            }
            for (int64_t i = 0; i < nq; ++i)
                ranks[i * nu + j] = (int32_t)(1 + cnt[i]);
        }
        free(t);
        free(cnt);
    }
}

/*
 * Certify a claimed answer of one reverse k-ranks query (Def. 2 with the
 * tie-break "rank ascending, then user id ascending").
 *
 *   ids[0..k-1], ranks[0..k-1]: the claim, sorted by (rank, id).
 *   check[0..nc-1]: users to examine (all users, or a sample of them).
 *
 * For every claimed user the full rank is recomputed; a mismatch is counted
 * in out[0].  Let R be the worst claimed rank and W the largest claimed id
 * whose rank is R.  Any other examined user u must satisfy
 * r(u) > R, or r(u) == R and u > W; otherwise the claim left out a better
 * user and out[1] is incremented.  Counting for such a user stops as soon
 * as 1 + count exceeds R, which cannot change the verdict because counts
 * only grow.  out[2] receives the number of examined users.
 */
void orc_certify(const double *U, int64_t n, const double *P, int64_t m,
                 const double *q, int d, int k, const int64_t *ids,
                 const int32_t *ranks, const int64_t *check, int64_t nc,
                 int64_t *out, int nthreads)
{
    set_threads(nthreads);
    int64_t bad_rank = 0, bad_set = 0;
    int32_t R = 0;
    int64_t W = -1;
    for (int i = 0; i < k; ++i)
        if (ranks[i] > R)
            R = ranks[i];
    for (int i = 0; i < k; ++i)
        if (ranks[i] == R && ids[i] > W)
            W = ids[i];
    char *claimed = (char *)calloc((size_t)n, 1);
    for (int i = 0; i < k; ++i)
        claimed[ids[i]] = 1;

#pragma omp parallel for schedule(dynamic, 1) reduction(+ : bad_rank)
    for (int i = 0; i < k; ++i) {
        const double *u = U + ids[i] * d;
        double t = spec_dot(u, q, d);
        int64_t c = 0;
        for (int64_t p = 0; p < m; ++p)
            if (spec_dot(u, P + p * d, d) > t)
                c += 1;
        if (1 + c != (int64_t)ranks[i])
            bad_rank += 1;
    }

#pragma omp parallel for schedule(dynamic, 64) reduction(+ : bad_set)
    for (int64_t j = 0; j < nc; ++j) {
        int64_t uid = check[j];
        if (claimed[uid])
            continue;
        const double *u = U + uid * d;
        double t = spec_dot(u, q, d);
        int64_t c = 0;
        for (int64_t p = 0; p < m && 1 + c <= R; ++p)
            if (spec_dot(u, P + p * d, d) > t)
                c += 1;
        if (1 + c < R || (1 + c == R && uid < W))
            bad_set += 1;
    }
    free(claimed);
    out[0] = bad_rank;
    out[1] = bad_set;
    out[2] = nc;
}

/*
 * Order of P by norm, descending, ties by item id ascending (the sort of
 * the paper's pre-processing step 1, Sec. 4.2, with a deterministic
 * tie-break).  norms[] are the spec norms; out[r] = id of the r-th item.
 */
static const double *g_sort_norms;
static int cmp_desc(const void *a, const void *b)
{
    int64_t i = *(const int64_t *)a, j = *(const int64_t *)b;
    double x = g_sort_norms[i], y = g_sort_norms[j];
    if (x > y) return -1;
    if (x < y) return 1;
    return (i > j) - (i < j);
}

void orc_norm_order(const double *norms, int64_t m, int64_t *out)
{
    for (int64_t i = 0; i < m; ++i)
        out[i] = i;
    g_sort_norms = norms;
    qsort(out, (size_t)m, sizeof(int64_t), cmp_desc);
}

/*
 * Per-user score sketch: for each user u and the sample items S (rows of
 * the item matrix listed in sample[0..ns-1]), sort the spec scores s(u,p)
 * in descending order and take the entries at the 1-based positions
 * pos[0..np-1]; each is divided by the user's spec norm (a user with zero
 * norm gets zeros).  out[u*np + j].
 */
static int cmp_dbl_desc(const void *a, const void *b)
{
    double x = *(const double *)a, y = *(const double *)b;
    return (x < y) - (x > y);
}

void orc_sketch(const double *U, int64_t n, const double *P,
                const int64_t *sample, int64_t ns, int d, const int32_t *pos,
                int np, double *out, int nthreads)
{
    set_threads(nthreads);
#pragma omp parallel
    {
        double *s = (double *)malloc(sizeof(double) * (size_t)ns);
#pragma omp for schedule(dynamic, 16)
        for (int64_t i = 0; i < n; ++i) {
            const double *u = U + i * d;
            double nu = sqrt(spec_dot(u, u, d));
            for (int64_t j = 0; j < ns; ++j)
                s[j] = spec_dot(u, P + sample[j] * d, d);
            qsort(s, (size_t)ns, sizeof(double), cmp_dbl_desc);
            for (int j = 0; j < np; ++j)
                out[i * np + j] = nu > 0.0 ? s[pos[j] - 1] / nu : 0.0;
        }
        free(s);
    }
}

/*
 * Rank table (paper Sec. 4.2, steps 2 and 3), with exact cells.
 * Columns: for each user, its spec scores against the sample items (rows of
 * P listed in sample[0..ns-1]), sorted in descending order and read at the
 * 1-based positions pos[0..np-1] give the thresholds t_out[u*np + j].  Cells:
 * cnt_out[u*np + j] = #{p in P : s(u,p) > t_out[u*np + j]}, the paper's cell
 * T_{i,j} = 1 + sum_p I[u_i.p > t_{i,j}] without its leading 1, counted over
 * all of P (the paper estimates it from samples instead).
 */
void orc_rank_table(const double *U, int64_t n, const double *P, int64_t m,
                    const int64_t *sample, int64_t ns, int d, const int32_t *pos,
                    int np, double *t_out, int64_t *cnt_out, int nthreads)
{
    set_threads(nthreads);
#pragma omp parallel
    {
        double *s = (double *)malloc(sizeof(double) * (size_t)(ns > 0 ? ns : 1));
        double *all = (double *)malloc(sizeof(double) * (size_t)(m > 0 ? m : 1));
#pragma omp for schedule(dynamic, 4)
        for (int64_t i = 0; i < n; ++i) {
            const double *u = U + i * d;
            for (int64_t j = 0; j < ns; ++j)
                s[j] = spec_dot(u, P + sample[j] * d, d);
            qsort(s, (size_t)ns, sizeof(double), cmp_dbl_desc);
            for (int64_t p = 0; p < m; ++p)
                all[p] = spec_dot(u, P + p * d, d);
            for (int j = 0; j < np; ++j) {
                const double t = s[pos[j] - 1];
                int64_t c = 0;
                for (int64_t p = 0; p < m; ++p)
                    if (all[p] > t)
                        ++c;
                t_out[i * np + j] = t;
                cnt_out[i * np + j] = c;
            }
        }
        free(all);
        free(s);
    }
}
