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
 *   order[0..m-1]: the order in which items are visited (NULL: 0..m-1); the
 *   norm order of Sec. 4.2 step 1 lets the early stop below come sooner.
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
                 const int64_t *order, int64_t *out, int nthreads)
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
            if (spec_dot(u, P + (order ? order[p] : p) * d, d) > t)
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

/*
 * Four spec dots of one vector x against four others: each result is the
 * spec dot above (its own accumulator, dimensions in order, one fma each);
 * the four chains only run side by side so that one waits less on the
 * latency of the previous fma.
 */
static void spec_dot4(const double *x, const double *y0, const double *y1, const double *y2,
                      const double *y3, int d, double out[4])
{
    double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
    for (int k = 0; k < d; ++k) {
        a0 = fma(x[k], y0[k], a0);
        a1 = fma(x[k], y1[k], a1);
        a2 = fma(x[k], y2[k], a2);
        a3 = fma(x[k], y3[k], a3);
    }
    out[0] = a0;
    out[1] = a1;
    out[2] = a2;
    out[3] = a3;
}

/*
 * Partial Def. 1 count of one user: the items P[order[0]], P[order[1]], ...
 * are visited in that order and c counts those with s(u,p) > t.  The scan
 * stops once ((1 + c) << 32 | uid) exceeds *stop (read atomically, it may
 * shrink while the scan runs), or after the last item.  Returns c; *done is 1
 * when every item was visited (then 1 + c is the exact rank), and *seen the
 * number of items visited.
 */
static int64_t scan_user(const double *u, int64_t uid, double t, const double *P,
                         const int64_t *order, int64_t m, int d, const uint64_t *stop,
                         int *done, int64_t *seen)
{
    int64_t c = 0, j = 0;
    double s[4];
    while (j < m) {
        if (j + 4 <= m) {
            spec_dot4(u, P + order[j] * d, P + order[j + 1] * d, P + order[j + 2] * d,
                      P + order[j + 3] * d, d, s);
            c += (s[0] > t) + (s[1] > t) + (s[2] > t) + (s[3] > t);
            j += 4;
        } else {
            c += spec_dot(u, P + order[j] * d, d) > t;
            j += 1;
        }
        uint64_t key = ((uint64_t)(1 + c) << 32) | (uint64_t)uid;
        if (stop && key > __atomic_load_n(stop, __ATOMIC_RELAXED))
            break;
    }
    *done = j == m;
    *seen = j;
    return c;
}

/* Max-heap of (rank << 32 | uid) keys. */
static void heap_down(uint64_t *h, int n, int i)
{
    for (;;) {
        int l = 2 * i + 1, r = l + 1, b = i;
        if (l < n && h[l] > h[b]) b = l;
        if (r < n && h[r] > h[b]) b = r;
        if (b == i) return;
        uint64_t x = h[i]; h[i] = h[b]; h[b] = x;
        i = b;
    }
}

static int cmp_u64(const void *a, const void *b)
{
    uint64_t x = *(const uint64_t *)a, y = *(const uint64_t *)b;
    return (x > y) - (x < y);
}

/* visit order of the users: larger t/|u| first (|u| = 0: first), ties by id */
struct visit { double key, t; int64_t uid; };
static int cmp_visit(const void *a, const void *b)
{
    const struct visit *x = (const struct visit *)a, *y = (const struct visit *)b;
    if (x->key > y->key) return -1;
    if (x->key < y->key) return 1;
    return (x->uid > y->uid) - (x->uid < y->uid);
}

/*
 * Exact reverse k-ranks answer of one query by early abandon (Def. 2, ties on
 * rank broken by user id; the abandon rule is Lemma 1 (2), Sec. 4, applied to
 * exact partial counts).  Domain: the users uids[0..nu-1] (all n users when
 * uids is NULL).  Items are visited in the order order[0..m-1] (a permutation
 * of 0..m-1; the norm order of Sec. 4.2 step 1 makes abandoning early likely).
 *
 *   1. t_u = s(u,q) for every user of the domain;
 *   2. the users are visited by t_u / |u| descending (|u| = 0 first; such a
 *      user has rank 1), ties by id;
 *   3. the first k of them are counted over every item: their (rank, id)
 *      keys fill a max-heap;
 *   4. every other user scans the items and is abandoned once
 *      (1 + partial count, id) exceeds the heap's largest key, since counts
 *      only grow; a user that reaches the end with a smaller key than the
 *      heap's largest replaces it;
 *   5. the answer is the heap by (rank, id) ascending.
 * Step 4 runs in parallel over users; the heap changes under a lock and its
 * largest key is published with an atomic store (a stale, larger value only
 * delays an abandon).  ids_out[k], ranks_out[k]; stats[0] = items visited
 * over all users, stats[1] = users that visited every item.
 */
void orc_topk_abandon(const double *U, int64_t n, const double *P, int64_t m,
                      const int64_t *order, const double *q, int d, int k,
                      const int64_t *uids, int64_t nu, int64_t *ids_out, int32_t *ranks_out,
                      int64_t *stats, int nthreads)
{
    set_threads(nthreads);
    if (!uids)
        nu = n;
    struct visit *vis = (struct visit *)malloc(sizeof(struct visit) * (size_t)(nu > 0 ? nu : 1));
#pragma omp parallel for schedule(static)
    for (int64_t j = 0; j < nu; ++j) {
        const int64_t u = uids ? uids[j] : j;
        const double *uv = U + u * d;
        const double t = spec_dot(uv, q, d);
        const double nrm = sqrt(spec_dot(uv, uv, d));
        vis[j].key = nrm > 0.0 ? t / nrm : INFINITY;
        vis[j].t = t;
        vis[j].uid = u;
    }
    qsort(vis, (size_t)nu, sizeof(struct visit), cmp_visit);

    const int kk = (int)(k < nu ? k : nu);
    uint64_t *heap = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)(kk > 0 ? kk : 1));
    int64_t visited = 0, full = 0;
    /* step 3: the first kk users, counted over every item */
#pragma omp parallel for schedule(dynamic, 1) reduction(+ : visited, full)
    for (int j = 0; j < kk; ++j) {
        int done = 0;
        int64_t seen = 0;
        const int64_t c = scan_user(U + vis[j].uid * d, vis[j].uid, vis[j].t, P, order, m, d,
                                    NULL, &done, &seen);
        heap[j] = ((uint64_t)(1 + c) << 32) | (uint64_t)vis[j].uid;
        visited += seen;
        full += 1;
    }
    for (int i = kk / 2 - 1; i >= 0; --i)
        heap_down(heap, kk, i);
    uint64_t worst = kk > 0 ? heap[0] : 0;
    /* step 4 */
#pragma omp parallel for schedule(dynamic, 16) reduction(+ : visited, full)
    for (int64_t j = kk; j < nu; ++j) {
        int done = 0;
        int64_t seen = 0;
        const int64_t uid = vis[j].uid;
        const int64_t c = scan_user(U + uid * d, uid, vis[j].t, P, order, m, d, &worst, &done,
                                    &seen);
        visited += seen;
        if (!done)
            continue;
        full += 1;
        const uint64_t key = ((uint64_t)(1 + c) << 32) | (uint64_t)uid;
#pragma omp critical(orc_heap)
        {
            if (key < heap[0]) {
                heap[0] = key;
                heap_down(heap, kk, 0);
                __atomic_store_n(&worst, heap[0], __ATOMIC_RELAXED);
            }
        }
    }
    /* step 5 */
    qsort(heap, (size_t)kk, sizeof(uint64_t), cmp_u64);
    for (int i = 0; i < kk; ++i) {
        ids_out[i] = (int64_t)(heap[i] & 0xffffffffu);
        ranks_out[i] = (int32_t)(heap[i] >> 32);
    }
    if (stats) {
        stats[0] = visited;
        stats[1] = full;
    }
    free(heap);
    free(vis);
}

/*
 * The paper's rank table (Sec. 4.2, Alg. 1), with estimated cells.
 *   Step 1: the items in norm order (order[0..m-1], descending norm) are cut
 *     into omega equally sized buckets: bucket l holds the positions
 *     [floor(l m / omega), floor((l + 1) m / omega)).
 *   Sampling: bucket l's samples are the items at the positions
 *     sample_pos[l * s + i] of that bucket, i < s_l = min(s, |P_l|) (the
 *     random draws are inputs).
 *   Step 2: tau uniform thresholds between f_min and f_max, here the
 *     footnote's domain values: f_max = |u| max_p |p| (Cauchy-Schwarz),
 *     f_min = -f_max, with |x| the spec norm; t_j = f_min + j * step for
 *     j = 0..tau-1 (ascending), step = (f_max - f_min) / (tau - 1).
 *   Step 3: every cell starts at 1 and each bucket adds, in bucket order,
 *     (A_l[j] |P_l|) / s_l with A_l[j] = #{sampled p of bucket l : s(u,p) >
 *     t_j} (eq. of the cell estimator; with s_l = |P_l| the cell is exactly
 *     1 + #{p : s(u,p) > t_j}).  The cell is kept in FP32 (round to nearest).
 * Outputs per user: fmin_out[u], step_out[u], T_out[u * tau + j].
 */
void orc_paper_table(const double *U, int64_t n, const double *P, int64_t m,
                     const int64_t *order, int d, int tau, int omega, int s,
                     const int32_t *sample_pos, double *fmin_out, double *step_out,
                     float *T_out, int nthreads)
{
    set_threads(nthreads);
    double pmax = 0.0;
    for (int64_t i = 0; i < m; ++i) {
        double x = sqrt(spec_dot(P + i * d, P + i * d, d));
        if (x > pmax)
            pmax = x;
    }
#pragma omp parallel
    {
        double *T = (double *)malloc(sizeof(double) * (size_t)tau);
        double *t = (double *)malloc(sizeof(double) * (size_t)tau);
        int64_t *A = (int64_t *)malloc(sizeof(int64_t) * (size_t)tau);
#pragma omp for schedule(dynamic, 16)
        for (int64_t ui = 0; ui < n; ++ui) {
            const double *u = U + ui * d;
            const double fmax = sqrt(spec_dot(u, u, d)) * pmax;
            const double fmin = -fmax;
            const double step = (fmax - fmin) / (double)(tau - 1);
            for (int j = 0; j < tau; ++j) {
                t[j] = fmin + (double)j * step;
                T[j] = 1.0;
            }
            for (int l = 0; l < omega; ++l) {
                const int64_t b0 = (int64_t)l * m / omega, b1 = (int64_t)(l + 1) * m / omega;
                const int64_t size = b1 - b0;
                const int64_t sl = size < s ? size : s;
                if (sl == 0)
                    continue;
                for (int j = 0; j < tau; ++j)
                    A[j] = 0;
                /* each sample adds 1 to A[j] for every threshold it is above;
                   the thresholds ascend, so the first one it is not above
                   ends its walk */
                for (int64_t i = 0; i < sl; ++i) {
                    const double *p = P + order[b0 + sample_pos[(int64_t)l * s + i]] * d;
                    const double sc = spec_dot(u, p, d);
                    for (int j = 0; j < tau; ++j) {
                        if (sc > t[j])
                            A[j] += 1;
                        else
                            break;
                    }
                }
                for (int j = 0; j < tau; ++j)
                    T[j] = T[j] + ((double)A[j] * (double)size) / (double)sl;
            }
            fmin_out[ui] = fmin;
            step_out[ui] = step;
            for (int j = 0; j < tau; ++j)
                T_out[ui * tau + j] = (float)T[j];
        }
        free(A);
        free(t);
        free(T);
    }
}
