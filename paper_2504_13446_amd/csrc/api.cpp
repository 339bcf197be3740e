// api.cpp -- the C ABI of librkr: validation, index construction and the
// query pipeline.  Every step of the computation runs in the HIP kernels of
// this library; this file only plans, allocates and launches.
//
// Query pipeline (exact, Def. 2; approximate, Def. 3):
//   1. pairs      the (user, query) pairs of the domain, numbered user-major
//   2. thresholds t(u,q) = spec dot in FP64 (the paper's query step 1, Sec. 4.3)
//   3. seeds      per query the S = seed_mult*k most promising users
//   4. exact count of the seed pairs (screen + FP64 near-tie recheck)
//   5. bound      B_q = k-th smallest seed rank >= R_k (the k-th smallest rank
//                 over all users); X_q = B_q (exact) or floor(B_q / c) (approx.)
//   5b. table     with a rank table (Sec. 4.2), pairs whose table lower bound
//                 already exceeds X_q are dropped without a scan
//   6. screen     every pair is scanned against norm-sorted P and dropped once
//                 1 + certain count > X_q (the paper's Lemma 1 (2))
//   7. refine     exact count of the pairs still live after the screen
//   8. answer     per query the k best (rank, id) among seeds and survivors
// Exactness: a dropped pair has rank > X_q = B_q >= the k-th rank of the
// returned set (the count kernel only drops a pair once its certain count,
// a lower bound of the exact one, shows it), so it is strictly worse than
// every returned user; every user that can be in the answer is counted
// exactly.  Approximate mode: a dropped pair has rank > floor(B_q / c), so
// c * rank > B_q >= a_i for every i <= k (a_i: the i-th rank of the returned
// set); the i-th smallest rank over all users either belongs to a counted user,
// and then a_i is at most it, or to a dropped one, and then a_i < c times it:
// Def. 3 holds either way.
#include <math.h>
#include <string.h>

#include <stdio.h>
#include <stdlib.h>
#include <sys/stat.h>

#include <algorithm>
#include <chrono>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "kernels.h"
#include "query.h"
#include "rkr.h"
#include "mlp.h"
#include "paper_table.h"

using namespace rkr;

static thread_local std::string g_err;

static rkr_status fail(rkr_status s, const std::string &msg) {
    g_err = msg;
    return s;
}
static rkr_status fail_hip(hipError_t e, const char *what) {
    if (e == hipErrorOutOfMemory) return fail(RKR_E_NOMEM, std::string("out of device memory in ") + what);
    return fail(RKR_E_DEVICE, std::string(what) + ": " + hipGetErrorString(e));
}
#define HIPCK(x)                                             \
    do {                                                     \
        hipError_t _e = (x);                                 \
        if (_e != hipSuccess) return fail_hip(_e, #x);       \
    } while (0)

static double now_ms() {
    return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

// Online autotuner of the screening kernel's launch (tile variant x grid or
// persistent).  For each shape key the first calls run the candidates in turn
// and record their HIP-event times; later calls use the fastest.  Decisions
// persist in a text cache (RKR_AUTOTUNE_CACHE, default
// $HOME/.cache/rkr/autotune.txt, "off" to disable), one "key candidate" line
// each, read at index build.  RKR_SCREEN_CANDIDATE forces a candidate.
struct Tuner {
    std::map<std::string, int> best;
    std::map<std::string, std::vector<double>> trials;
    std::string path;
    void load() {
        const char *env = getenv("RKR_AUTOTUNE_CACHE");
        const char *home = getenv("HOME");
        if (env && *env) path = env;
        else if (home && *home) path = std::string(home) + "/.cache/rkr/autotune.txt";
        if (path.empty() || path == "off") return;
        FILE *f = fopen(path.c_str(), "r");
        if (!f) return;
        char k[512];
        int v;
        while (fscanf(f, "%511s %d", k, &v) == 2) best[k] = v;
        fclose(f);
    }
    void save(const std::string &key, int v) {
        if (path.empty() || path == "off") return;
        std::string dir = path.substr(0, path.find_last_of('/'));
        if (!dir.empty()) {
            std::string cur;
            for (size_t i = 0; i < dir.size(); ++i) {
                cur += dir[i];
                if (dir[i] == '/' && i > 0) mkdir(cur.c_str(), 0755);
            }
            mkdir(dir.c_str(), 0755);
        }
        FILE *f = fopen(path.c_str(), "a");
        if (!f) return;
        fprintf(f, "%s %d\n", key.c_str(), v);
        fclose(f);
    }
    int pick(const std::string &key, int nvar) {
        if (nvar <= 1) return 0;
        const char *force = getenv("RKR_SCREEN_CANDIDATE");   // fixed choice, e.g. for profiling
        if (force && *force) {
            int v = atoi(force);
            if (v >= 0 && v < nvar) return v;
        }
        auto it = best.find(key);
        if (it != best.end() && it->second < nvar) return it->second;
        const auto &t = trials[key];
        return (int)t.size() < nvar ? (int)t.size() : 0;
    }
    void record(const std::string &key, int variant, double ms, int nvar) {
        if (nvar <= 1 || best.count(key)) return;
        auto &t = trials[key];
        if ((int)t.size() != variant) return;
        t.push_back(ms);
        if ((int)t.size() == nvar) {
            int b = (int)(std::min_element(t.begin(), t.end()) - t.begin());
            best[key] = b;
            save(key, b);
        }
    }
};

// The single-query all-ranks pipeline captured in a hipGraph: every size is
// fixed by n, so thresholds -> one-entry-per-user tasks -> exact count ->
// FP64 recheck (record count read on the device) -> ranks replay as one
// graph launch.  The graph owns its buffers, so eager calls that grow the
// index's buffers never touch memory the graph refers to.
struct RanksGraph {
    bool valid = false;
    hipStream_t cs = nullptr;
    hipGraph_t g = nullptr;
    hipGraphExec_t ge = nullptr;
    DBuf qbuf, rbuf, pair_u, pair_q, t64, cnt, ctr, emit;
    TaskSet ts;
    int64_t emit_cap = 0;
    void destroy() {
        if (ge) (void)hipGraphExecDestroy(ge);
        if (g) (void)hipGraphDestroy(g);
        ge = nullptr;
        g = nullptr;
        valid = false;
    }
    void release() {
        destroy();
        if (cs) (void)hipStreamDestroy(cs);
        cs = nullptr;
        DBuf *b[] = {&qbuf, &rbuf, &pair_u, &pair_q, &t64, &cnt, &ctr, &emit};
        for (DBuf *x : b) x->release();
        ts.release();
    }
};

struct rkr_index {
    int64_t n = 0, m = 0;
    int d = 0, dpad = 0, nks = 0, mk = 0, sk = 0, recheck = 1;
    int split = 0;                    // 1: split BF16 scores (sk is SK_BF16, rows of 3d terms)
    double g32 = 0.0, g64 = 0.0;      // the error bound's FP32 (matrix-core sums) and FP64 factors
    int64_t nblk32 = 0, nblk = 0;     // item blocks of 32 (real, allocated: a multiple of 4)
    int num_cus = 256;
    int dev = 0;                      // device the index was built on
    hipStream_t st = nullptr;
    // index data
    DBuf Um, Pm, perm, ulp, plp, unorm3, pnorm3, uexp, pexp, coef;
    DBuf coef_step[3];    // per-step coefficient maxima for steps of 1, 2, 4 blocks
    DBuf coef32_step[2];  // the same for steps of 1 and 2 blocks, rounded up to FP32
    DBuf tup, qlp, qnorm3, qxyz;   // bounded FP32 thresholds of a dense batch and the queries' BF16 copies
    // pair_u / pair_q currently hold the dense layout of (dp_n users, dp_nq
    // queries) at these addresses (-1: something else)
    int64_t dp_n = -1;
    int dp_nq = -1;
    const void *dp_u = nullptr, *dp_q = nullptr;
    size_t dp_ucap = 0, dp_qcap = 0;   // (a buffer that grew was allocated anew)
    DBuf step_znorm;      // per 64-item step: an upper bound of |p| from that step on
    // per-call buffers
    Scratch sc;
    DBuf pair_u, pair_q, pair_off, qm_pid, t64, cnt, seedflag, keys, sel, selrank, best, cand,
        candkeys, ans, seedpid, surv, emit, ctr, bound, seedkth, kdev, sdev, cdev, segoff, seloff, bestoff,
        candoff, cursor, qcount, flags, allpid, keep;
    TaskSet ts_screen, ts_screen2, ts_exact;
    DBuf sp_len, sp_pid, sp_th, sp_cnt;   // per-split lists of a split screen phase
    // rank table (Sec. 4.2): [n][TABLE_COLS] FP64 thresholds, their FP32
    // round-ups, and certain counts over all of P
    DBuf tab_t, tab_th, tab_cnt;
    bool has_table = false;
    // the paper's own rank table (Alg. 1, Sec. 4.2): per user f_min and the
    // threshold step (FP64), and [n][ptab_tau] estimated cells (FP32)
    DBuf ptab_fmin, ptab_step, ptab_cells;
    int ptab_tau = 0;
    bool has_ptab = false;
    int64_t emit_cap = 0;
    // events: 0..3 an exact pass and its recheck; 4..9 the stage boundaries of
    // a batch; 10..41 its screening phases
    hipEvent_t ev[42] = {};
    rkr_query_opts qo{};
    rkr_query_stats stats{};
    Tuner tuner;
    RanksGraph rg;
    // estimator
    Estimator est;
};

// ---------------------------------------------------------------------------
// build
// ---------------------------------------------------------------------------
static_assert(TABLE_COLS == RKR_TABLE_COLS, "the kernels' table width is the ABI's");
static rkr_status build_rank_table(rkr_index *x, int samples);
static rkr_status scratch_address(int dev, uint8_t **out);

extern "C" rkr_status rkr_build(const void *U, int64_t n, const void *P, int64_t m, int32_t d, rkr_dtype dt,
                                const rkr_build_opts *opts, rkr_index **out) {
    g_err.clear();
    if (!out) return fail(RKR_E_INVALID, "out is NULL");
    *out = nullptr;
    if (n <= 0) return fail(RKR_E_INVALID, "n must be positive");
    if (m < 0) return fail(RKR_E_INVALID, "m must be non-negative");
    if (d <= 0 || d > 4096) return fail(RKR_E_INVALID, "d must be in 1..4096");
    if (dt != RKR_F32 && dt != RKR_BF16) return fail(RKR_E_INVALID, "unknown master dtype");
    if (!U || (m > 0 && !P)) return fail(RKR_E_INVALID, "U or P is NULL");
    if (n >= (1ll << 31) || m >= (1ll << 31)) return fail(RKR_E_UNSUPPORTED, "n and m must be below 2^31");
    int sk = SK_BF16, recheck = 1, sketch = 0, table = 0;
    hipStream_t st = nullptr;
    if (opts) {
        sk = opts->score;
        recheck = opts->recheck ? 1 : 0;
        sketch = opts->sketch_samples;
        table = opts->rank_table;
        st = (hipStream_t)opts->stream;
    }
    if (sk != SK_F32 && sk != SK_BF16 && sk != SK_FP8 && sk != RKR_SCORE_BF16X3)
        return fail(RKR_E_INVALID, "unknown score kind");
    if (sketch < 0) return fail(RKR_E_INVALID, "sketch_samples must be >= 0");
    if (table < 0) return fail(RKR_E_INVALID, "rank_table must be >= 0");
    // split BF16 runs the BF16 kernels on rows of 3d terms
    const int split = sk == RKR_SCORE_BF16X3 ? 1 : 0;
    if (split) sk = SK_BF16;
    const int KS = frag_ks(sk);
    const int terms = split ? 3 * d : d;
    // pad to a k-step count the count kernels are instantiated for (zero padding)
    const int nks = nks_bucket(sk, (terms + KS - 1) / KS);
    if (nks == 0)
        return fail(RKR_E_UNSUPPORTED, "d too large for this score kind (max " +
                                           std::to_string(max_nks(sk) * KS / (split ? 3 : 1)) + ")");
    const int dpad = nks * KS;

    rkr_index *x = new (std::nothrow) rkr_index();
    if (!x) return fail(RKR_E_NOMEM, "host allocation failed");
    x->n = n; x->m = m; x->d = d; x->dpad = dpad; x->nks = nks; x->sk = sk; x->split = split; x->recheck = recheck;
    x->mk = dt == RKR_BF16 ? MK_BF16 : MK_F32;
    x->st = st;
    x->qo.seed_mult = 0;   // chosen per call (see run_batch)
    x->tuner.load();
    {
        int dev = 0, cus = 0;
        if (hipGetDevice(&dev) == hipSuccess) x->dev = dev;
        if (hipGetDevice(&dev) == hipSuccess &&
            hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && cus > 0)
            x->num_cus = cus;
    }
    const int mes = dt == RKR_BF16 ? 2 : 4;
    const int es = elem_size(sk);
    x->nblk32 = (m + 31) / 32;
    x->nblk = (x->nblk32 + 3) / 4 * 4;
    rkr_status rs = RKR_OK;
    auto body = [&]() -> rkr_status {
        HIPCK(x->Um.ensure((size_t)n * d * mes));
        HIPCK(x->Pm.ensure((size_t)std::max<int64_t>(m, 1) * d * mes));
        HIPCK(x->perm.ensure((size_t)std::max<int64_t>(m, 1) * 4));
        HIPCK(x->ulp.ensure((size_t)n * dpad * es));
        HIPCK(x->plp.ensure((size_t)std::max<int64_t>(x->nblk, 1) * 32 * dpad * es));
        HIPCK(x->unorm3.ensure((size_t)n * 3 * 8));
        HIPCK(x->pnorm3.ensure((size_t)std::max<int64_t>(m, 1) * 3 * 8));
        HIPCK(x->uexp.ensure((size_t)n));
        HIPCK(x->pexp.ensure((size_t)std::max<int64_t>(m, 1)));
        HIPCK(x->coef.ensure((size_t)std::max<int64_t>(x->nblk, 1) * 4 * 8));
        HIPCK(x->flags.ensure(16));
        HIPCK(launch_fill_u32(x->flags.as<uint32_t>(), 0, 4, st));
        HIPCK(hipMemcpyAsync(x->Um.p, U, (size_t)n * d * mes, hipMemcpyDeviceToDevice, st));
        HIPCK(launch_check_values(x->Um.p, n * d, x->mk, x->flags.as<int>(), st));
        if (m > 0) {
            HIPCK(launch_check_values(P, m * d, x->mk, x->flags.as<int>(), st));
            // P in norm order (descending, ties by id)
            double *pn = (double *)x->sc.take(m * 8);
            void *srt = x->sc.take((int64_t)norm_sort_scratch_bytes(m));
            if (!pn || !srt) return fail(RKR_E_NOMEM, "sort scratch");
            HIPCK(launch_spec_norm(P, m, d, x->mk, pn, st));
            HIPCK(launch_norm_sort(pn, m, srt, x->perm.as<int32_t>(), st));
            HIPCK(launch_gather_rows(P, x->perm.as<int32_t>(), m, d, x->mk, x->Pm.p, st));
            const int64_t ns64 = (m + 63) / 64;
            HIPCK(x->step_znorm.ensure((size_t)ns64 * 8));
            HIPCK(launch_step_znorm(pn, x->perm.as<int32_t>(), m, ns64, x->step_znorm.as<double>(), st));
        }
        HIPCK(launch_fill_u8(x->plp.as<uint8_t>(), 0, (int64_t)x->nblk * 32 * dpad * es, st));
        HIPCK(launch_lowprec(x->Um.p, n, d, x->mk, sk, dpad, 0, split, x->ulp.as<uint8_t>(),
                             x->unorm3.as<double>(), x->uexp.as<int8_t>(), st));
        HIPCK(launch_lowprec(x->Pm.p, m, d, x->mk, sk, dpad, 1, split ? 2 : 0, x->plp.as<uint8_t>(),
                             x->pnorm3.as<double>(), x->pexp.as<int8_t>(), st));
        const double u = ldexp(1.0, -23);
        double g32 = sk == SK_F32 ? 2.0 * (dpad + 2) * u : 2.0 * dpad * u;
        // split BF16: the products summed, |hi.hi| + |hi.lo| + |lo.hi|, stay
        // below (1 + 2^-5) |u_hat| |p_hat|, and the lo.lo product left out is
        // below 1.02 * 2^-16 |u| |p| (|lo| <= 2^-8 (1 + 2^-8) |x| per element)
        if (split) g32 *= 1.0 + 0x1p-5;
        const double cz = split ? 0x1.06p-16 : 0.0;
        const double u64 = ldexp(1.0, -53);
        const double g64 = d * u64 / (1.0 - d * u64) * 1.01;
        const double eabs = dpad * ldexp(1.0, -100);
        x->g32 = g32;
        x->g64 = g64;
        HIPCK(launch_block_coef(x->pnorm3.as<double>(), m, x->nblk, g32, g64, cz, eabs, x->coef.as<double>(), st));
        for (int k = 0; k < 3; ++k) {
            const int nib = 1 << k;
            const int64_t ns = (x->nblk32 + nib - 1) / nib;
            HIPCK(x->coef_step[k].ensure((size_t)std::max<int64_t>(ns, 1) * 4 * 8));
            HIPCK(launch_step_coef(x->coef.as<double>(), x->nblk, nib, ns, x->coef_step[k].as<double>(), st));
            if (k < 2) {
                HIPCK(x->coef32_step[k].ensure((size_t)std::max<int64_t>(ns, 1) * 4 * 4));
                HIPCK(q_round_up_f32(x->coef_step[k].as<double>(), ns * 4, x->coef32_step[k].as<float>(), st));
            }
        }
        int flags = 0;
        HIPCK(hipMemcpyAsync(&flags, x->flags.p, 4, hipMemcpyDeviceToHost, st));
        HIPCK(hipStreamSynchronize(st));
        if (flags & 1) return fail(RKR_E_INVALID, "U or P holds a non-finite value");
        if (flags & 2) return fail(RKR_E_INVALID, "U or P holds a value with magnitude above 2^50");
        if (sketch > 0) {
            rkr_status s2 = est_build_sketch(x->est, x->Um.p, n, x->Pm.p, m, d, x->mk, x->unorm3.as<double>(),
                                             sketch, x->sc, st);
            if (s2 != RKR_OK) return s2;
        }
        x->sc.reset();
        if (table > 0 && m > 0) {
            rkr_status s3 = build_rank_table(x, table);
            if (s3 != RKR_OK) return s3;
        }
        x->sc.reset();
        return RKR_OK;
    };
    rs = body();
    if (rs != RKR_OK) {
        rkr_destroy(x);
        return rs;
    }
    // set-up of rkr_ranks_noalloc on this device: taking the address of its
    // static array makes the runtime place the array now, not in that call
    // (a failure here surfaces there)
    uint8_t *na = nullptr;
    (void)scratch_address(x->dev, &na);
    g_err.clear();
    *out = x;
    return RKR_OK;
}

extern "C" void rkr_destroy(rkr_index *x) {
    if (!x) return;
    (void)hipStreamSynchronize(x->st);
    DBuf *bufs[] = {&x->keep, &x->tab_t, &x->tab_th, &x->tab_cnt, &x->ptab_fmin, &x->ptab_step, &x->ptab_cells,
                    &x->Um, &x->Pm, &x->perm, &x->ulp, &x->plp, &x->unorm3, &x->pnorm3, &x->uexp, &x->pexp,
                    &x->coef, &x->coef_step[0], &x->coef_step[1], &x->coef_step[2], &x->coef32_step[0],
                    &x->coef32_step[1], &x->tup, &x->qlp, &x->qnorm3, &x->qxyz, &x->pair_u, &x->pair_q,
                    &x->pair_off, &x->qm_pid, &x->t64,
                    &x->cnt, &x->seedflag, &x->keys, &x->sel, &x->selrank, &x->best, &x->cand,
                    &x->candkeys, &x->ans, &x->seedpid, &x->surv, &x->emit, &x->ctr, &x->bound, &x->seedkth,
                    &x->kdev, &x->sdev, &x->cdev, &x->segoff, &x->seloff, &x->bestoff, &x->candoff, &x->cursor,
                    &x->qcount, &x->flags, &x->allpid, &x->sp_len, &x->sp_pid, &x->sp_th, &x->sp_cnt};
    for (DBuf *b : bufs) b->release();
    x->ts_screen.release();
    x->ts_screen2.release();
    x->ts_exact.release();
    x->rg.release();
    for (auto &e : x->ev)
        if (e) (void)hipEventDestroy(e);
    x->sc.release();
    est_release(x->est);
    delete x;
}

extern "C" rkr_status rkr_configure(rkr_index *x, const rkr_query_opts *o) {
    g_err.clear();
    if (!x || !o) return fail(RKR_E_INVALID, "NULL argument");
    if (o->seed_mult < 0 || o->prune_mult < 0) return fail(RKR_E_INVALID, "negative option");
    if (o->reserved0 != 0) return fail(RKR_E_INVALID, "reserved0 must be 0");
    if (o->use_estimator && !x->est.trained) return fail(RKR_E_STATE, "estimator not trained");
    rkr_query_opts q = *o;
    x->qo = q;
    return RKR_OK;
}

extern "C" rkr_status rkr_rank_table(const rkr_index *x, double *t_out, uint32_t *cnt_out) {
    g_err.clear();
    if (!x || !t_out || !cnt_out) return fail(RKR_E_INVALID, "NULL argument");
    if (!x->has_table) return fail(RKR_E_STATE, "index built without a rank table");
    const int64_t cells = x->n * TABLE_COLS;
    HIPCK(hipMemcpyAsync(t_out, x->tab_t.p, cells * 8, hipMemcpyDeviceToDevice, x->st));
    HIPCK(hipMemcpyAsync(cnt_out, x->tab_cnt.p, cells * 4, hipMemcpyDeviceToDevice, x->st));
    HIPCK(hipStreamSynchronize(x->st));
    return RKR_OK;
}
extern "C" rkr_status rkr_stats(const rkr_index *x, rkr_query_stats *out) {
    g_err.clear();
    if (!x || !out) return fail(RKR_E_INVALID, "NULL argument");
    *out = x->stats;
    return RKR_OK;
}

extern "C" const char *rkr_last_error(void) { return g_err.c_str(); }

// ---------------------------------------------------------------------------
// counting passes
// ---------------------------------------------------------------------------
static hipError_t ensure_events(rkr_index *x) {
    for (auto &e : x->ev)
        if (!e) {
            hipError_t r = hipEventCreate(&e);
            if (r != hipSuccess) return r;
        }
    return hipSuccess;
}
// Elapsed milliseconds between two recorded events (after a stream sync).
static double event_ms(hipEvent_t a, hipEvent_t b) {
    float ms = 0.0f;
    if (hipEventElapsedTime(&ms, a, b) != hipSuccess) {
        (void)hipGetLastError();   // a timing left out is no error of the call
        return 0.0;
    }
    return (double)ms;
}
static std::string tune_key(const rkr_index *x, int nq, int64_t npairs) {
    char b[256];
    snprintf(b, sizeof b, "gfx950/screen2/sk%d/nks%d/n%lld/m%lld/nq%d/pairs%lld", x->sk, x->nks, (long long)x->n,
             (long long)x->m, nq, (long long)npairs);
    return b;
}

// An exact pass's splits share nothing but the count they add to: few user
// tiles (the refine of a batch's survivors) spread over more of them.
static constexpr int64_t kMaxExactSplits = 64;

// Splits of the item range for a pass over gx user tiles (one workgroup per
// CU): the count in 1..max_split that minimises rounds x (split length + a
// workgroup's fixed cost), ceil(gx * ns / cus) * (nsteps / ns + overhead)
// (smallest such count on ties).

static int64_t pick_nsplit(int64_t gx, int64_t nsteps, int cus, int64_t max_split = 16) {
    const int64_t maxs = std::max<int64_t>(1, std::min<int64_t>(max_split, nsteps));
    const int64_t c = std::max(1, cus);
    int64_t best = 1;
    double best_cost = 1e300;
    // a workgroup's fixed cost (staging ahead, the first barrier, the final
    // flush) is worth about kSplitOverhead steps of its range
    constexpr double kSplitOverhead = 24.0;
    for (int64_t ns = 1; ns <= maxs; ++ns) {
        const double cost = (double)((gx * ns + c - 1) / c) * ((double)nsteps / (double)ns + kSplitOverhead);
        if (cost < best_cost - 1e-12) {
            best_cost = cost;
            best = ns;
        }
    }
    return best;
}

// Tile of the exact passes: v2, 1 x 2 blocks per wave (the low-register
// tile; FP32 scores have one tile, v0 = 1 x 1).
static int exact_variant(const rkr_index *x) { return x->sk == SK_F32 ? 0 : 2; }

// The pairs of a dense batch (pid = u * nq + q) depend on (n, nq) only: the
// lists are written again only when the shape or the buffers change.
static hipError_t dense_pairs(rkr_index *x, int64_t n, int nq, hipStream_t st) {
    if (x->dp_n == n && x->dp_nq == nq && x->dp_u == x->pair_u.p && x->dp_q == x->pair_q.p &&
        x->dp_ucap == x->pair_u.cap && x->dp_qcap == x->pair_q.cap)
        return hipSuccess;
    x->dp_n = -1;
    hipError_t e = launch_dense_pairs(n, nq, x->pair_u.as<int32_t>(), x->pair_q.as<int32_t>(), st);
    if (e != hipSuccess) return e;
    x->dp_n = n;
    x->dp_nq = nq;
    x->dp_u = x->pair_u.p;
    x->dp_q = x->pair_q.p;
    x->dp_ucap = x->pair_u.cap;
    x->dp_qcap = x->pair_q.cap;
    return hipSuccess;
}

// The screen's phase ends, in 64ths of the item scan (the last is 64); a
// list such as "4,8,12,..,64" in RKR_SCREEN_PHASES replaces them (tuning).
static constexpr int kMaxPhases = 16;
static const std::vector<int> &screen_phases() {
    static const std::vector<int> ends = [] {
        std::vector<int> v;
        if (const char *e = getenv("RKR_SCREEN_PHASES")) {
            int prev = 0;
            for (const char *p = e; *p;) {
                char *q = nullptr;
                const long x = strtol(p, &q, 10);
                if (q == p) break;
                if (x > prev && x <= 64 && (int)v.size() < kMaxPhases) {
                    v.push_back((int)x);
                    prev = (int)x;
                }
                p = *q ? q + 1 : q;
            }
        }
        if (v.empty() || v.back() != 64) v = {2, 5, 10, 20, 36, 64};
        return v;
    }();
    return ends;
}

// Users per workgroup of an exact pass (the pipelined pass for BF16 scores,
// else the count kernel's tile); it sets the item splits of a launch.
static int exact_tasks_per_wg(const rkr_index *x, int xv) {
    if (x->sk == SK_BF16 && xv == 2) return pass_tasks_per_wg(x->nks);
    return WAVES_PER_WG * nub_of(x->sk, x->nks, xv) * USER_BLOCK;
}

// An environment switch that is on when set to "1" (read once).
static bool env_flag(const char *name) {
    const char *v = getenv(name);
    return v && v[0] == '1' && v[1] == 0;
}

// Live entries per lane from which the screen counts by histogram (bucketed
// counting) instead of comparing codes one entry at a time (RKR_SCREEN_HIST
// overrides it; 0: never).  Both count lower bounds of the certain counts.
static int screen_hist_min() {
    const char *v = getenv("RKR_SCREEN_HIST");
    if (v && *v) return std::max(0, atoi(v));
    return 12;
}

static CountArgs count_args(rkr_index *x, const PairSet &ps, TaskSet &ts, int variant) {
    CountArgs a{};
    const int nib = nib_of(x->sk, x->nks, variant);
    a.plp = x->plp.as<uint8_t>();
    a.m = x->m;
    a.nks = x->nks;
    a.step_coef = x->coef_step[nib == 1 ? 0 : (nib == 2 ? 1 : 2)].as<double>();
    a.step_coef_half = x->coef_step[0].as<double>();
    a.step_coef32 = x->coef32_step[1].as<float>();
    a.step_coef32_half = x->coef32_step[0].as<float>();
    a.pexp = x->pexp.as<int8_t>();
    a.ulp = x->ulp.as<uint8_t>();
    a.dpad = x->dpad;
    a.unorm3 = x->unorm3.as<double>();
    a.uexp = x->uexp.as<int8_t>();
    a.task_user = ts.task_user;
    a.ntask = ts.ntask;
    a.blk_base = ts.blk_base;
    a.ent_len = ts.len;
    a.ent_pid = ts.ent_pid;
    a.ent_q = ts.ent_q;
    a.ent_cnt = ts.ent_cnt;
    a.ent_th = ts.ent_th;
    a.ent_tl = ts.ent_tl;
    a.ent_tm = ts.ent_tm;
    a.cap_total = ts.cap_total;
    a.bound = x->bound.as<int32_t>();
    a.nq = ps.nq;
    a.nsteps = (x->nblk32 + nib - 1) / nib;
    a.steps_per_split = a.nsteps;
    a.step0 = 0;
    a.step_end = a.nsteps;
    a.cnt_out = x->cnt.as<uint32_t>();
    a.emit = x->emit.as<int2>();
    a.emit_count = x->ctr.as<unsigned long long>();
    a.emit_cap = (unsigned long long)x->emit_cap;
    a.stat = x->ctr.as<unsigned long long>() + 1;
    a.plain = x->recheck ? 0 : 1;
    a.hist_min = screen_hist_min();
    // the pipelined passes' steps are 64 items (two blocks)
    a.step_znorm = (nib == 2 && x->m > 0 && !env_flag("RKR_NO_SETTLE")) ? x->step_znorm.as<double>() : nullptr;
    return a;
}

// Largest near-tie record buffer an exact pass may grow to: half of the
// device memory free beyond the current buffer (at least 2^24 records).
static int64_t max_emit_records(const rkr_index *x) {
    size_t freeb = 0, totalb = 0;
    if (hipMemGetInfo(&freeb, &totalb) != hipSuccess) return (int64_t)1 << 24;
    const int64_t have = (int64_t)x->emit_cap;
    return std::max<int64_t>((int64_t)1 << 24, have + (int64_t)(freeb / 2 / 8));
}

// Exact counts (certain-above + FP64 recheck of near ties) of the pairs
// pids[0..N) (ascending); adds into cnt[pid] after zeroing it.
static rkr_status exact_count(rkr_index *x, const PairSet &ps, const int32_t *pids, int64_t N) {
    if (N <= 0) return RKR_OK;
    hipStream_t st = x->st;
    HIPCK(ensure_events(x));
    TaskSet &ts = x->ts_exact;
    // one pair per task: the exact kernel folds the pair's threshold into its
    // accumulators (a user with several pairs gets a task for each)
    hipError_t e = build_tasks(pids, N, ps, x->recheck ? 0 : 1, nullptr, ts, x->sc, st, nullptr, 1);
    if (e != hipSuccess) return fail_hip(e, "build_tasks (exact)");
    const int xv = exact_variant(x);
    const int tpw = exact_tasks_per_wg(x, xv);
    const int64_t gx = (ts.ntask + tpw - 1) / tpw;
    CountArgs a = count_args(x, ps, ts, xv);
    const int64_t nsteps = a.nsteps;
    int64_t nsplit = pick_nsplit(gx, nsteps, x->num_cus, kMaxExactSplits);
    HIPCK(ts.reserve_entries(ts.cap_total, (int)nsplit));
    a.ent_cnt = ts.ent_cnt;
    a.steps_per_split = (nsteps + nsplit - 1) / nsplit;
    nsplit = std::max<int64_t>(1, (nsteps + a.steps_per_split - 1) / std::max<int64_t>(a.steps_per_split, 1));
    if (x->emit_cap == 0) {
        x->emit_cap = 1 << 22;
        HIPCK(x->emit.ensure((size_t)x->emit_cap * 8));
    }
    unsigned long long *ctr = x->ctr.as<unsigned long long>();
    for (int attempt = 0; attempt < 4; ++attempt) {
        a.emit = x->emit.as<int2>();
        a.emit_cap = (unsigned long long)x->emit_cap;
        // the work counters as they were, for a retry (slots 8..15)
        HIPCK(hipMemcpyAsync(ctr + 8, ctr, 64, hipMemcpyDeviceToDevice, st));
        HIPCK(q_zero_at(pids, N, x->cnt.as<uint32_t>(), st));
        HIPCK(launch_fill_u32(x->ctr.as<uint32_t>(), 0, 2, st));   // emit counter (64-bit)
        HIPCK(hipEventRecord(x->ev[0], st));
        HIPCK(launch_count(x->sk, CM_EXACT, a, (int)nsplit, xv, st));
        HIPCK(hipEventRecord(x->ev[1], st));
        // users with several tasks were scored once per task: count their
        // (user, item) scores once in the algorithmic-work counter
        if (ts.d_nusers)
            HIPCK(q_scored_fix(ctr + 7, ts.ntask, ts.d_nusers, x->m, st));
        // the recheck reads the record count on the device (at most the
        // buffer's size); one read-back then tells whether the buffer held them all
        HIPCK(hipEventRecord(x->ev[2], st));
        HIPCK(launch_recheck_dev(x->emit.as<int2>(), ctr, (int64_t)x->emit_cap, ps.pair_u, ps.t64, x->Um.p, x->Pm.p,
                                 x->d, x->mk, x->cnt.as<uint32_t>(), ctr + 2, st));
        HIPCK(hipEventRecord(x->ev[3], st));
        unsigned long long ne = 0;
        HIPCK(hipMemcpyAsync(&ne, ctr, 8, hipMemcpyDeviceToHost, st));
        HIPCK(hipStreamSynchronize(st));
        x->stats.ms_exact_kernel += event_ms(x->ev[0], x->ev[1]);
        if (ne <= (unsigned long long)x->emit_cap) {
            if (!ts.d_nusers && ts.ntask > ts.nusers) {
                unsigned long long scored = 0;
                HIPCK(hipMemcpyAsync(&scored, ctr + 7, 8, hipMemcpyDeviceToHost, st));
                HIPCK(hipStreamSynchronize(st));
                scored -= (unsigned long long)(ts.ntask - ts.nusers) * (unsigned long long)x->m;
                HIPCK(hipMemcpyAsync(ctr + 7, &scored, 8, hipMemcpyHostToDevice, st));
            }
            x->stats.uncertain += (int64_t)ne;
            x->stats.ms_recheck_kernel += event_ms(x->ev[2], x->ev[3]);
            return RKR_OK;
        }
        // the buffer overflowed: the counts are incomplete; the counters go
        // back to where they were and the pass runs again
        HIPCK(hipMemcpyAsync(ctr + 1, ctr + 9, 56, hipMemcpyDeviceToDevice, st));
        x->stats.emit_retries += 1;
        const int64_t max_emit = max_emit_records(x);
        if ((int64_t)ne + (int64_t)(ne / 4) > max_emit && N > 1) {
            // more near ties than the device has room for (wide bands, e.g.
            // FP8 scores): count the pairs in parts, each sized for about
            // half of that room if the ties spread evenly (a part that still
            // overflows splits again; a single pair emits at most m records)
            const int64_t parts = std::min<int64_t>(N, ((int64_t)ne + max_emit / 2 - 1) / (max_emit / 2));
            const int64_t chunk = (N + parts - 1) / parts;
            for (int64_t p0 = 0; p0 < N; p0 += chunk) {
                rkr_status r = exact_count(x, ps, pids + p0, std::min<int64_t>(chunk, N - p0));
                if (r != RKR_OK) return r;
            }
            return RKR_OK;
        }
        x->emit_cap = std::min<int64_t>((int64_t)(ne + ne / 4 + 1024), std::max<int64_t>(max_emit, x->m + 1024));
        HIPCK(x->emit.ensure((size_t)x->emit_cap * 8));
    }
    return fail(RKR_E_DEVICE, "near-tie buffer kept overflowing");
}

// The rank table (Sec. 4.2).  Thresholds (step 2): the user's spec scores
// against S norm-stratified sample items, read at TABLE_COLS geometrically
// spaced positions of their descending order (the paper spaces them
// uniformly between the extreme scores).  Cells (step 3): counted over all of
// P by the count kernel's table mode, as certain counts (lower bounds of the
// exact counts) in place of the paper's sampled estimates, so that they can
// rule pairs out without losing exactness.
static rkr_status build_rank_table(rkr_index *x, int samples) {
    const int64_t n = x->n, cells = n * TABLE_COLS;
    hipStream_t st = x->st;
    x->has_table = false;
    HIPCK(x->tab_t.ensure(cells * 8));
    HIPCK(x->tab_th.ensure(cells * 4));
    HIPCK(x->tab_cnt.ensure(cells * 4));
    rkr_status rs = sample_levels(x->Um.p, n, x->Pm.p, x->m, x->d, x->mk, samples, TABLE_COLS, nullptr,
                                  x->tab_t.as<double>(), x->sc, st);
    if (rs != RKR_OK) return fail(rs, "rank table: sample scores");
    HIPCK(q_round_up_f32(x->tab_t.as<double>(), cells, x->tab_th.as<float>(), st));
    HIPCK(launch_fill_u32(x->tab_cnt.as<uint32_t>(), 0, cells, st));
    PairSet ps;     // table mode reads neither pairs nor entry lists
    TaskSet ts;
    const int xv = x->sk == SK_F32 ? 0 : 2;
    CountArgs a = count_args(x, ps, ts, xv);
    a.ntask = n;
    a.ent_th = x->tab_th.as<float>();
    a.cnt_out = x->tab_cnt.as<uint32_t>();
    a.stat = nullptr;
    a.emit = nullptr;
    a.emit_count = nullptr;
    a.emit_cap = 0;
    const int tpw = WAVES_PER_WG * nub_of(x->sk, x->nks, xv) * USER_BLOCK;
    const int64_t gx = (n + tpw - 1) / tpw;
    int64_t nsplit = pick_nsplit(gx, a.nsteps, x->num_cus);
    a.steps_per_split = (a.nsteps + nsplit - 1) / nsplit;
    nsplit = (a.nsteps + a.steps_per_split - 1) / a.steps_per_split;
    HIPCK(launch_count(x->sk, CM_TABLE, a, (int)nsplit, xv, st));
    HIPCK(hipStreamSynchronize(st));
    x->has_table = true;
    return RKR_OK;
}

// ---------------------------------------------------------------------------
// check of the error bound (every user x every item)
// ---------------------------------------------------------------------------
extern "C" rkr_status rkr_score_error(rkr_index *x, double *max_ratio_out, int64_t *over_out) {
    g_err.clear();
    if (!x || !max_ratio_out || !over_out) return fail(RKR_E_INVALID, "NULL argument");
    hipStream_t st = x->st;
    x->sc.reset();
    uint32_t *out = (uint32_t *)x->sc.take(8);
    if (!out) return fail(RKR_E_NOMEM, "scratch");
    HIPCK(launch_fill_u32(out, 0, 2, st));
    if (x->m > 0) {
        PairSet ps;
        TaskSet ts;
        const int xv = x->sk == SK_F32 ? 0 : 2;
        CountArgs a = count_args(x, ps, ts, xv);
        a.ntask = x->n;
        a.cnt_out = out;
        a.stat = nullptr;
        a.emit = nullptr;
        a.emit_count = nullptr;
        a.emit_cap = 0;
        a.um_master = x->Um.p;
        a.pm_master = x->Pm.p;
        a.d_master = x->d;
        a.mk_master = x->mk;
        const int tpw = WAVES_PER_WG * nub_of(x->sk, x->nks, xv) * USER_BLOCK;
        int64_t nsplit = pick_nsplit((x->n + tpw - 1) / tpw, a.nsteps, x->num_cus);
        a.steps_per_split = (a.nsteps + nsplit - 1) / nsplit;
        nsplit = (a.nsteps + a.steps_per_split - 1) / a.steps_per_split;
        HIPCK(launch_count(x->sk, CM_BOUND, a, (int)nsplit, xv, st));
    }
    uint32_t h[2] = {0, 0};
    HIPCK(hipMemcpyAsync(h, out, 8, hipMemcpyDeviceToHost, st));
    HIPCK(hipStreamSynchronize(st));
    float r;
    memcpy(&r, &h[0], 4);
    *max_ratio_out = (double)r;
    *over_out = (int64_t)h[1];
    return RKR_OK;
}

// The same check in the form of the pipelined passes (BF16 scores): the
// thresholds th = the FP32 values above s64(u, q) folded into the
// accumulators, checked against their bound.
extern "C" rkr_status rkr_score_error_at(rkr_index *x, const void *q, double *max_ratio_out, int64_t *over_out) {
    g_err.clear();
    if (!x || !q || !max_ratio_out || !over_out) return fail(RKR_E_INVALID, "NULL argument");
    if (x->sk != SK_BF16) return fail(RKR_E_UNSUPPORTED, "the folded form is the BF16 passes'");
    hipStream_t st = x->st;
    x->sc.reset();
    HIPCK(launch_fill_u32(x->flags.as<uint32_t>(), 0, 4, st));
    HIPCK(launch_check_values(q, x->d, x->mk, x->flags.as<int>(), st));
    int flags = 0;
    HIPCK(hipMemcpyAsync(&flags, x->flags.p, 4, hipMemcpyDeviceToHost, st));
    HIPCK(hipStreamSynchronize(st));
    if (flags) return fail(RKR_E_INVALID, "the query holds a non-finite value or one above 2^50");
    uint32_t *out = (uint32_t *)x->sc.take(8);
    double *t64 = (double *)x->sc.take(x->n * 8);
    float *th = (float *)x->sc.take(x->n * 4);
    if (!out || !t64 || !th) return fail(RKR_E_NOMEM, "scratch");
    HIPCK(launch_thresh_dense(x->Um.p, x->n, q, 1, x->d, x->mk, t64, st));
    HIPCK(q_round_up_f32(t64, x->n, th, st));
    HIPCK(launch_fill_u32(out, 0, 2, st));
    if (x->m > 0) {
        PairSet ps;
        TaskSet ts;
        const int xv = 2;
        CountArgs a = count_args(x, ps, ts, xv);
        a.ntask = x->n;
        a.cnt_out = out;
        a.stat = nullptr;
        a.emit = nullptr;
        a.emit_count = nullptr;
        a.emit_cap = 0;
        a.um_master = x->Um.p;
        a.pm_master = x->Pm.p;
        a.d_master = x->d;
        a.mk_master = x->mk;
        a.fold_th = th;
        const int tpw = WAVES_PER_WG * nub_of(x->sk, x->nks, xv) * USER_BLOCK;
        int64_t nsplit = pick_nsplit((x->n + tpw - 1) / tpw, a.nsteps, x->num_cus);
        a.steps_per_split = (a.nsteps + nsplit - 1) / nsplit;
        nsplit = (a.nsteps + a.steps_per_split - 1) / a.steps_per_split;
        HIPCK(launch_count(x->sk, CM_BOUND, a, (int)nsplit, xv, st));
    }
    uint32_t h[2] = {0, 0};
    HIPCK(hipMemcpyAsync(h, out, 8, hipMemcpyDeviceToHost, st));
    HIPCK(hipStreamSynchronize(st));
    float r;
    memcpy(&r, &h[0], 4);
    *max_ratio_out = (double)r;
    *over_out = (int64_t)h[1];
    return RKR_OK;
}

// ---------------------------------------------------------------------------
// batch queries
// ---------------------------------------------------------------------------
static rkr_status run_batch(rkr_index *x, int32_t nq, const void *Qm, const int32_t *k, const double *c,
                            const int64_t *cand_off, const int32_t *cand_ids, int32_t *ids_out, int32_t *ranks_out) {
    g_err.clear();
    if (!x) return fail(RKR_E_INVALID, "index is NULL");
    if (nq < 1) return fail(RKR_E_INVALID, "nq must be positive");
    if (nq > 65535) return fail(RKR_E_UNSUPPORTED, "nq above 65535");
    if (!Qm || !k || !ids_out || !ranks_out) return fail(RKR_E_INVALID, "NULL argument");
    const int64_t n = x->n;
    const bool dense = cand_off == nullptr;
    if (!dense && !cand_ids) return fail(RKR_E_INVALID, "cand_ids is NULL");
    std::vector<int64_t> dom(nq), S(nq);
    if (!dense) {
        if (cand_off[0] != 0) return fail(RKR_E_INVALID, "cand_off[0] must be 0");
        for (int q = 0; q < nq; ++q)
            if (cand_off[q + 1] < cand_off[q]) return fail(RKR_E_INVALID, "cand_off must be non-decreasing");
    }
    int64_t ksum = 0;
    for (int q = 0; q < nq; ++q) {
        dom[q] = dense ? n : cand_off[q + 1] - cand_off[q];
        if (!dense && dom[q] > n) return fail(RKR_E_INVALID, "candidate list longer than n");
        if (k[q] < 1 || k[q] > dom[q]) return fail(RKR_E_INVALID, "k out of range for query " + std::to_string(q));
        if (k[q] > 4096) return fail(RKR_E_UNSUPPORTED, "k above 4096");
        if (c && (!(c[q] >= 1.0))) return fail(RKR_E_INVALID, "c must be >= 1 (query " + std::to_string(q) + ")");
        ksum += k[q];
    }
    hipStream_t st = x->st;
    const double t0 = now_ms();
    x->stats = rkr_query_stats{};
    x->stats.queries = nq;
    x->sc.reset();
    const int d = x->d;
    // stage boundaries as events (read once, at the end): thresholds, seeds,
    // screen, refine, answer
    HIPCK(ensure_events(x));
    hipEvent_t *sev = x->ev + 4, *pev = x->ev + 10;
    HIPCK(hipEventRecord(sev[0], st));
    // query values
    HIPCK(launch_fill_u32(x->flags.as<uint32_t>(), 0, 4, st));
    HIPCK(launch_check_values(Qm, (int64_t)nq * d, x->mk, x->flags.as<int>(), st));

    // ---- 1. pairs
    PairSet ps;
    ps.nq = nq;
    ps.dense = dense ? 1 : 0;
    const int64_t npairs = dense ? n * nq : cand_off[nq];
    // pair ids are 32-bit
    if (npairs >= ((int64_t)1 << 31)) return fail(RKR_E_UNSUPPORTED, "2^31 or more (user, query) pairs: split the batch");
    ps.npairs = npairs;
    x->stats.pairs = npairs;
    HIPCK(x->pair_u.ensure(npairs * 4));
    HIPCK(x->pair_q.ensure(npairs * 4));
    ps.pair_u = x->pair_u.as<int32_t>();
    ps.pair_q = x->pair_q.as<int32_t>();
    std::vector<int64_t> segoff(nq + 1);
    for (int q = 0; q <= nq; ++q) segoff[q] = dense ? (int64_t)q * n : cand_off[q];
    HIPCK(x->segoff.ensure((nq + 1) * 8));
    HIPCK(hipMemcpyAsync(x->segoff.p, segoff.data(), (nq + 1) * 8, hipMemcpyHostToDevice, st));
    if (dense) {
        HIPCK(dense_pairs(x, n, nq, st));
    } else {
        HIPCK(x->pair_off.ensure((n + 1) * 8));
        HIPCK(x->qm_pid.ensure(npairs * 4));
        ps.pair_off = x->pair_off.as<int64_t>();
        ps.qm_pid = x->qm_pid.as<int32_t>();
        x->dp_n = -1;   // the CSR layout overwrites the pair lists
        hipError_t e = build_csr_pairs(cand_ids, x->segoff.as<int64_t>(), nq, npairs, n, ps, x->flags.as<int>() + 1,
                                       x->sc, st);
        if (e == hipErrorInvalidValue)
            return fail(RKR_E_INVALID, "candidate ids out of range or duplicated within a list");
        if (e != hipSuccess) return fail_hip(e, "build_csr_pairs");
    }
    // ---- 2. thresholds (dense batches without the estimator: with the
    // default seed keys written from the same register tile)
    HIPCK(x->t64.ensure(npairs * 8));
    HIPCK(x->keys.ensure(npairs * 8));
    ps.t64 = x->t64.as<double>();
    // dense batches: the default seed keys come out of the threshold kernel
    // (with the estimator they pick its candidates)
    const bool keys_fused = dense;
    // Dense batches filtered by the rank table: every pair needs its
    // threshold only for the filter and the seed order, so those get bounded
    // FP32 values from the matrix cores (t_up >= the FP64 threshold); the FP64
    // thresholds are computed for the pairs that are counted (seeds, then the
    // pairs the filter keeps).
    const bool approx_t = keys_fused && x->has_table && !x->qo.no_table && x->sk == SK_BF16 && !x->split &&
                          !env_flag("RKR_FP64_THRESHOLDS");
    if (approx_t) {
        HIPCK(x->qlp.ensure((size_t)nq * x->dpad * 2));
        HIPCK(x->qnorm3.ensure((size_t)nq * 3 * 8));
        HIPCK(x->qxyz.ensure((size_t)nq * 16));
        HIPCK(x->tup.ensure(npairs * 4));
        HIPCK(launch_lowprec(Qm, nq, d, x->mk, SK_BF16, x->dpad, 0, 0, x->qlp.as<uint8_t>(), x->qnorm3.as<double>(),
                             nullptr, st));
        HIPCK(launch_query_xyz(x->qnorm3.as<double>(), nq, x->g32, x->g64, x->qxyz.as<float4>(), st));
        HIPCK(launch_thresh_approx(x->ulp.as<uint8_t>(), n, x->dpad, x->nks, x->unorm3.as<double>(),
                                   x->qlp.as<uint8_t>(), nq, x->qxyz.as<float4>(), x->tup.as<float>(),
                                   x->keys.as<uint32_t>(), x->num_cus, st));
    } else if (dense)
        HIPCK(launch_thresh_dense(x->Um.p, n, Qm, nq, d, x->mk, ps.t64, st, keys_fused ? x->unorm3.as<double>() : nullptr,
                                  keys_fused ? x->keys.as<uint64_t>() : nullptr));
    else
        HIPCK(launch_thresh(ps.pair_u, ps.pair_q, npairs, x->Um.p, Qm, d, x->mk, ps.t64, st));
    {
        int flags = 0;
        HIPCK(hipMemcpyAsync(&flags, x->flags.p, 4, hipMemcpyDeviceToHost, st));
        HIPCK(hipStreamSynchronize(st));
        if (flags & 1) return fail(RKR_E_INVALID, "a query holds a non-finite value");
        if (flags & 2) return fail(RKR_E_INVALID, "a query holds a value with magnitude above 2^50");
    }
    HIPCK(hipEventRecord(sev[1], st));

    // ---- 3. seeds
    std::vector<int64_t> seloff(nq + 1, 0), bestoff(nq + 1, 0);
    std::vector<int32_t> Sv(nq);
    const bool use_est = x->qo.use_estimator != 0;
    if (use_est && !x->est.trained) return fail(RKR_E_STATE, "estimator not trained");
    // approximate mode with pruning: the candidates are the prune_mult * k
    // users of best predicted rank (estimator) or best t/|u| (heuristic),
    // counted exactly; no screen, so Def. 3 is not guaranteed
    const bool pruned = c && x->qo.prune_mult > 0;
    const float *pred = nullptr;
    if (use_est && !dense) {
        HIPCK(x->est.pred.ensure(npairs * 4));
        HIPCK(est_infer(x->est, nullptr, nullptr, npairs, ps.pair_u, ps.t64, x->unorm3.as<double>(),
                        x->est.pred.as<float>(), 0, 0, st));
        pred = x->est.pred.as<float>();
    }
    // default seeds: 2k per query, or k when the rank table prunes (then a
    // seed missed by the heuristic costs one screened and refined pair, less
    // than counting a second k of seeds exactly)
    const bool table_on = x->has_table && !x->qo.no_table;
    const int seed_mult = x->qo.seed_mult > 0 ? x->qo.seed_mult : (table_on ? 1 : 2);
    const int64_t mult = pruned ? std::max(1, x->qo.prune_mult) : seed_mult;
    for (int q = 0; q < nq; ++q) {
        S[q] = std::min<int64_t>(dom[q], std::min<int64_t>(4096, std::max<int64_t>(k[q], mult * k[q])));
        Sv[q] = (int32_t)S[q];
        seloff[q + 1] = seloff[q] + S[q];
        bestoff[q + 1] = bestoff[q] + k[q];
    }
    const int64_t nsel = seloff[nq];
    QView v{ps.dense, nq, n, x->segoff.as<int64_t>(), ps.qm_pid};
    HIPCK(x->keys.ensure(npairs * 8));
    HIPCK(x->sel.ensure(nsel * 8));
    HIPCK(x->selrank.ensure(nsel * 8));
    HIPCK(x->seloff.ensure((nq + 1) * 8));
    HIPCK(x->bestoff.ensure((nq + 1) * 8));
    HIPCK(x->sdev.ensure(nq * 4));
    HIPCK(x->kdev.ensure(nq * 4));
    HIPCK(x->best.ensure(ksum * 8));
    HIPCK(hipMemcpyAsync(x->seloff.p, seloff.data(), (nq + 1) * 8, hipMemcpyHostToDevice, st));
    HIPCK(hipMemcpyAsync(x->bestoff.p, bestoff.data(), (nq + 1) * 8, hipMemcpyHostToDevice, st));
    HIPCK(hipMemcpyAsync(x->sdev.p, Sv.data(), nq * 4, hipMemcpyHostToDevice, st));
    HIPCK(hipMemcpyAsync(x->kdev.p, k, nq * 4, hipMemcpyHostToDevice, st));
    if (c) {
        HIPCK(x->cdev.ensure(nq * 8));
        HIPCK(hipMemcpyAsync(x->cdev.p, c, nq * 8, hipMemcpyHostToDevice, st));
    }
    if (!keys_fused)
        HIPCK(q_seed_keys(v, ps.pair_u, ps.t64, x->unorm3.as<double>(), pred, npairs, x->keys.as<uint64_t>(), st));
    if (use_est && dense) {
        // The estimator orders the kEstCand * S users of best t/|u| per query
        // (their FP64 thresholds are its input) and the seeds are the S of
        // best predicted rank among them: inference over every (user, query)
        // pair would cost more than the seed pass it is meant to shorten.
        constexpr int64_t kEstCand = 16;
        std::vector<int64_t> coff(nq + 1, 0);
        std::vector<int32_t> Cv(nq);
        for (int q = 0; q < nq; ++q) {
            Cv[q] = (int32_t)std::min<int64_t>(dom[q], std::min<int64_t>(4096, std::max<int64_t>(S[q], kEstCand * S[q])));
            coff[q + 1] = coff[q] + Cv[q];
        }
        const int64_t nc = coff[nq];
        HIPCK(x->est.pred.ensure(nc * 4));
        int64_t *d_coff = (int64_t *)x->sc.take((nq + 1) * 8);
        int32_t *d_C = (int32_t *)x->sc.take(nq * 4);
        uint64_t *csel = (uint64_t *)x->sc.take(nc * 8);
        uint64_t *ckeys = (uint64_t *)x->sc.take(nc * 8);
        int32_t *cpid = (int32_t *)x->sc.take(nc * 4);
        if (!d_coff || !d_C || !csel || !ckeys || !cpid) return fail(RKR_E_NOMEM, "estimator candidates");
        HIPCK(hipMemcpyAsync(d_coff, coff.data(), (nq + 1) * 8, hipMemcpyHostToDevice, st));
        HIPCK(hipMemcpyAsync(d_C, Cv.data(), nq * 4, hipMemcpyHostToDevice, st));
        // (with bounded thresholds the seed keys are 32 bits, the user being
        // the position in the query's row)
        if (approx_t)
            HIPCK(launch_select32(x->keys.as<uint32_t>(), x->segoff.as<int64_t>(), d_C, nq, d_coff, csel, st));
        else
            HIPCK(launch_select(x->keys.as<uint64_t>(), x->segoff.as<int64_t>(), d_C, nq, d_coff, csel, st));
        HIPCK(q_est_cand_pids(csel, d_coff, nq, nc, cpid, st));
        if (approx_t)
            HIPCK(launch_thresh_list(cpid, nc, ps.pair_u, ps.pair_q, x->Um.p, Qm, d, x->mk, ps.t64, st));
        HIPCK(est_infer(x->est, nullptr, cpid, nc, ps.pair_u, ps.t64, x->unorm3.as<double>(),
                        x->est.pred.as<float>(), 0, 0, st));
        HIPCK(q_est_cand_keys(csel, x->est.pred.as<float>(), nc, ckeys, st));
        HIPCK(launch_select(ckeys, d_coff, x->sdev.as<int32_t>(), nq, x->seloff.as<int64_t>(),
                            x->sel.as<uint64_t>(), st));
    } else if (approx_t) {
        HIPCK(launch_select32(x->keys.as<uint32_t>(), x->segoff.as<int64_t>(), x->sdev.as<int32_t>(), nq,
                              x->seloff.as<int64_t>(), x->sel.as<uint64_t>(), st));
    } else {
        HIPCK(launch_select(x->keys.as<uint64_t>(), x->segoff.as<int64_t>(), x->sdev.as<int32_t>(), nq,
                            x->seloff.as<int64_t>(), x->sel.as<uint64_t>(), st));
    }
    HIPCK(x->seedflag.ensure(npairs));
    HIPCK(launch_fill_u8(x->seedflag.as<uint8_t>(), 0, npairs, st));
    HIPCK(q_mark_selected(v, x->sel.as<uint64_t>(), x->seloff.as<int64_t>(), nsel, x->seedflag.as<uint8_t>(), st));
    HIPCK(x->seedpid.ensure(nsel * 4));
    HIPCK(x->allpid.ensure(npairs * 4));
    // seeds (counted exactly below) and the other pairs (the ones to screen;
    // with a rank table the filter lists them instead); every query selects
    // S[q] distinct pairs of its own, so there are nsel seeds
    const int64_t nseed = nsel;
    HIPCK(q_split_flags(x->seedflag.as<uint8_t>(), npairs, x->seedpid.as<int32_t>(), nullptr,
                        table_on ? nullptr : x->allpid.as<int32_t>(), st, x->sc));
    if (approx_t)
        HIPCK(launch_thresh_list(x->seedpid.as<int32_t>(), nseed, ps.pair_u, ps.pair_q, x->Um.p, Qm, d, x->mk, ps.t64,
                                 st));
    x->stats.seed_pairs = nseed;
    // ---- 4. exact count of the seeds
    HIPCK(x->cnt.ensure(npairs * 4));
    HIPCK(x->ctr.ensure(256));
    HIPCK(launch_fill_u32(x->ctr.as<uint32_t>(), 0, 64, st));
    unsigned long long *ctr_d = x->ctr.as<unsigned long long>();
    rkr_status rs = exact_count(x, ps, x->seedpid.as<int32_t>(), nseed);
    if (rs != RKR_OK) return rs;
    x->stats.ms_seed_kernel = x->stats.ms_exact_kernel;
    // the work counter after the seeds (slot 16), read with the others at the end
    HIPCK(hipMemcpyAsync(ctr_d + 16, ctr_d + 7, 8, hipMemcpyDeviceToDevice, st));
    // ---- 5. per-query bound
    HIPCK(q_rank_keys_sel(v, x->sel.as<uint64_t>(), x->seloff.as<int64_t>(), nsel, x->cnt.as<uint32_t>(),
                          x->selrank.as<uint64_t>(), st));
    HIPCK(launch_select(x->selrank.as<uint64_t>(), x->seloff.as<int64_t>(), x->kdev.as<int32_t>(), nq,
                        x->bestoff.as<int64_t>(), x->best.as<uint64_t>(), st));
    HIPCK(x->bound.ensure(nq * 4));
    HIPCK(x->seedkth.ensure(nq * 4));
    HIPCK(q_bounds(x->best.as<uint64_t>(), x->bestoff.as<int64_t>(), x->kdev.as<int32_t>(),
                   c ? x->cdev.as<double>() : nullptr, nq, x->bound.as<int32_t>(), x->seedkth.as<int32_t>(), st));
    HIPCK(hipEventRecord(sev[2], st));

    // ---- 6. screen every pair against its bound
    bool need_screen = false;
    for (int q = 0; q < nq; ++q) need_screen |= dom[q] > S[q];
    if (pruned) need_screen = false;
    int64_t nsurv = 0;
    HIPCK(x->surv.ensure(npairs * 4));
    int64_t nscreen = npairs - nseed;   // the seeds' ranks are known: they are not screened
    const bool table_used = need_screen && nscreen > 0 && x->has_table && !x->qo.no_table;
    if (table_used) {
        // the rank table rules out pairs the screen would drop (Lemma 1 (2))
        HIPCK(x->keep.ensure(npairs));
        HIPCK(q_table_keep(ps, x->seedflag.as<uint8_t>(), x->bound.as<int32_t>(), x->tab_t.as<double>(),
                           x->tab_cnt.as<uint32_t>(), x->keep.as<uint8_t>(), st,
                           approx_t ? x->tup.as<float>() : nullptr));
        int64_t nk = 0;
        HIPCK(q_compact_flags(x->keep.as<uint8_t>(), npairs, x->allpid.as<int32_t>(), &nk, x->sc, st));
        if (approx_t)
            HIPCK(launch_thresh_list(x->allpid.as<int32_t>(), nk, ps.pair_u, ps.pair_q, x->Um.p, Qm, d, x->mk, ps.t64,
                                     st));
        x->stats.table_pruned = nscreen - nk;
        nscreen = nk;
    }
    if (need_screen && nscreen > 0) {
        // After the rank table about one pair per user is left: BF16 screens
        // then run the pipelined single-pair kernel (one pair per task; a
        // user with several gets a task for each).  Dense screens (many pairs
        // per user) run the count kernel's screening mode.
        const bool single = table_used && x->sk == SK_BF16 && !env_flag("RKR_SCREEN_GENERIC");
        const int max_len = single ? 1 : 0;
        hipError_t e = build_tasks(x->allpid.as<int32_t>(), nscreen, ps, x->recheck ? 0 : 1, x->bound.as<int32_t>(),
                                   x->ts_screen, x->sc, st, nullptr, max_len);
        if (e != hipSuccess) return fail_hip(e, "build_tasks (screen)");
        // the screening kernel addresses entries with 32-bit byte offsets
        if (x->ts_screen.cap_total >= ((int64_t)1 << 30))
            return fail(RKR_E_UNSUPPORTED, "more than 2^30 screening entries: split the batch");
        // candidates: each tile variant, launched as a grid or as a persistent grid
        // a table-pruned screen sees far fewer pairs: tuned on its own
        const std::string key = tune_key(x, nq, npairs) + (table_used ? "/table" : "");
        const int ntv = num_variants(x->sk, x->nks);
        const int cand = single ? 0 : x->tuner.pick(key, 2 * ntv);
        const int variant = single ? exact_variant(x) : cand % ntv;
        const bool persistent = !single && cand >= ntv;
        // The scan runs in phases.  Without the rank table every user stays
        // live through the first quarter or so of P, then users die fast;
        // after the table most pairs die within the first tenth.  After a
        // phase whose end leaves fewer than half of the current tasks live,
        // the live pairs are compacted, with their remaining budgets, into a
        // new dense task set, so that later steps run only tiles of live
        // users.  A phase with fewer tiles than compute units is split over
        // item ranges.
        const std::vector<int> &phase_end = screen_phases();   // in 64ths of the scan
        HIPCK(ensure_events(x));
        TaskSet *cur = &x->ts_screen, *nxt = &x->ts_screen2;
        const int tpw = single ? pass_tasks_per_wg(x->nks) : WAVES_PER_WG * nub_of(x->sk, x->nks, variant) * USER_BLOCK;
        const int64_t nsteps = count_args(x, ps, *cur, variant).nsteps;
        int64_t s0 = 0;
        bool ph_timed[kMaxPhases] = {};
        double ms_kernel = 0.0;
        x->stats.screen_ctas = 0;
        for (int ph = 0; ph < (int)phase_end.size() && s0 < nsteps; ++ph) {
            const int64_t s1 = phase_end[ph] == 64 ? nsteps : nsteps * phase_end[ph] / 64;
            if (s1 <= s0) continue;
            CountArgs a = count_args(x, ps, *cur, variant);
            a.step0 = s0;
            a.step_end = s1;
            a.steps_per_split = s1 - s0;
            const int64_t tiles = (cur->ntask + tpw - 1) / tpw;
            // Too few tiles of live users to fill the device: split the phase
            // over item ranges (a grid launch, whatever the candidate), each
            // split on its own copy of the lists (entry offsets stay 32-bit),
            // and merge the copies afterwards.
            const bool pers_phase = persistent && tiles >= x->num_cus;
            int64_t nsplit = 1;
            if (tiles < x->num_cus) {
                // (lists of one pair per task merge with any number of splits)
                const int64_t max_split = single ? kMaxExactSplits : 16;
                nsplit = std::min<int64_t>(pick_nsplit(tiles, s1 - s0, x->num_cus, max_split), max_split);
                while (nsplit > 1 && cur->cap_total * nsplit >= ((int64_t)1 << 30)) --nsplit;
                if (nsplit > 1) {
                    a.steps_per_split = (s1 - s0 + nsplit - 1) / nsplit;
                    nsplit = (s1 - s0 + a.steps_per_split - 1) / a.steps_per_split;
                }
            }
            if (nsplit > 1) {
                const int64_t cap = cur->cap_total, ntp = cur->ntask_pad;
                HIPCK(x->sp_len.ensure(ntp * nsplit * 4));
                HIPCK(x->sp_pid.ensure(cap * nsplit * 4));
                HIPCK(x->sp_th.ensure(cap * nsplit * 4));
                HIPCK(x->sp_cnt.ensure(cap * nsplit * 4));
                HIPCK(q_replicate_u32((const uint32_t *)cur->len, ntp, x->sp_len.as<uint32_t>(), (int)nsplit, st));
                HIPCK(q_replicate_u32((const uint32_t *)cur->ent_pid, cap, x->sp_pid.as<uint32_t>(), (int)nsplit, st));
                HIPCK(q_replicate_u32((const uint32_t *)cur->ent_th, cap, x->sp_th.as<uint32_t>(), (int)nsplit, st));
                HIPCK(q_replicate_u32(cur->ent_cnt, cap, x->sp_cnt.as<uint32_t>(), (int)nsplit, st));
                a.ent_len = x->sp_len.as<int32_t>();
                a.len_stride = ntp;
                a.ent_pid = x->sp_pid.as<int32_t>();
                a.ent_th = x->sp_th.as<float>();
                a.ent_cnt = x->sp_cnt.as<uint32_t>();
            }
            if (pers_phase) {
                x->stats.persistent_phases += 1;
                HIPCK(launch_fill_u32(x->ctr.as<uint32_t>() + 8, 0, 2, st));
                a.tile_counter = x->ctr.as<unsigned long long>() + 4;
                a.persistent_ctas = x->num_cus;
            }
            HIPCK(hipEventRecord(pev[2 * ph], st));
            if (single)
                HIPCK(launch_screen1_bf16(a, (int)nsplit, st));
            else
                HIPCK(launch_count(x->sk, CM_SCREEN, a, (int)nsplit, variant, st));
            HIPCK(hipEventRecord(pev[2 * ph + 1], st));
            ph_timed[ph] = true;
            if (nsplit > 1)
                HIPCK(q_screen_merge(*cur, (int)nsplit, x->sp_len.as<int32_t>(), x->sp_pid.as<int32_t>(),
                                     x->sp_cnt.as<uint32_t>(), st, single));
            x->stats.screen_ctas = std::max<int64_t>(x->stats.screen_ctas,
                                                     pers_phase ? std::min<int64_t>(x->num_cus, tiles) : tiles * nsplit);
            s0 = s1;
            if (s0 >= nsteps) break;
            if (single) {
                // one pair per task: compact after every phase (one read-back,
                // the count of live pairs), budgets at cnt[pid]
                TView tv{cur->ntask, cur->len, cur->blk_base, cur->ent_pid, cur->ent_cnt};
                int64_t npl = 0;
                HIPCK(q_survivors(tv, x->seedflag.as<uint8_t>(), x->surv.as<int32_t>(), &npl, x->sc, st,
                                  x->cnt.as<uint32_t>()));
                if (npl == 0) {                          // every screened pair is dead
                    cur->ntask = 0;
                    break;
                }
                e = build_tasks(x->surv.as<int32_t>(), npl, ps, x->recheck ? 0 : 1, x->bound.as<int32_t>(), *nxt,
                                x->sc, st, x->cnt.as<uint32_t>(), max_len);
                if (e != hipSuccess) return fail_hip(e, "build_tasks (screen compaction)");
                std::swap(cur, nxt);
                continue;
            }
            HIPCK(hipStreamSynchronize(st));
            int64_t nlive = 0;
            HIPCK(q_count_live(cur->len, cur->ntask, x->ctr.as<unsigned long long>() + 6, &nlive, st));
            if (nlive == 0) break;                       // every screened pair is dead
            if (2 * nlive >= cur->ntask) continue;       // still dense: keep the tiles
            // compact: live pairs in task order (grouped by user), budgets at cnt[pid]
            TView tv{cur->ntask, cur->len, cur->blk_base, cur->ent_pid, cur->ent_cnt};
            int64_t npl = 0;
            HIPCK(q_survivors(tv, x->seedflag.as<uint8_t>(), x->surv.as<int32_t>(), &npl, x->sc, st,
                              x->cnt.as<uint32_t>()));
            e = build_tasks(x->surv.as<int32_t>(), npl, ps, x->recheck ? 0 : 1, x->bound.as<int32_t>(), *nxt, x->sc,
                            st, x->cnt.as<uint32_t>(), max_len);
            if (e != hipSuccess) return fail_hip(e, "build_tasks (screen compaction)");
            std::swap(cur, nxt);
        }
        TView tv{cur->ntask, cur->len, cur->blk_base, cur->ent_pid, cur->ent_cnt};
        HIPCK(q_survivors(tv, x->seedflag.as<uint8_t>(), x->surv.as<int32_t>(), &nsurv, x->sc, st));
        // (q_survivors read its count back: every phase has ended)
        for (int ph = 0; ph < kMaxPhases; ++ph)
            if (ph_timed[ph]) ms_kernel += event_ms(pev[2 * ph], pev[2 * ph + 1]);
        x->stats.ms_screen_kernel = ms_kernel;
        if (!single) x->tuner.record(key, cand, ms_kernel, 2 * ntv);
        x->stats.screen_variant = single ? -1 : cand;
    }
    // the work counter before the refine (slot 17)
    HIPCK(hipMemcpyAsync(ctr_d + 17, ctr_d + 7, 8, hipMemcpyDeviceToDevice, st));
    HIPCK(hipEventRecord(sev[3], st));
    x->stats.survivors = nsurv;
    // ---- 7. refine the survivors
    rs = exact_count(x, ps, x->surv.as<int32_t>(), nsurv);
    if (rs != RKR_OK) return rs;
    x->stats.refined_pairs = nsurv;
    HIPCK(hipEventRecord(sev[4], st));

    // ---- 8. answer: k best (rank, id) among seeds and survivors; the
    // candidate lists per query (its seeds, then its survivors) are laid out
    // on the device
    HIPCK(x->qcount.ensure(nq * 4));
    HIPCK(launch_fill_u32(x->qcount.as<uint32_t>(), 0, nq, st));
    HIPCK(q_count_by_query(x->surv.as<int32_t>(), nsurv, ps.pair_q, x->qcount.as<int32_t>(), st));
    HIPCK(x->candoff.ensure((nq + 1) * 8));
    HIPCK(x->cursor.ensure(nq * 4));
    HIPCK(x->candkeys.ensure((nsel + nsurv) * 8));
    HIPCK(x->ans.ensure(ksum * 8));
    HIPCK(q_cand_offsets(x->qcount.as<int32_t>(), x->sdev.as<int32_t>(), nq, x->candoff.as<int64_t>(), x->sc, st));
    HIPCK(hipMemcpyAsync(x->cursor.p, x->sdev.p, nq * 4, hipMemcpyDeviceToDevice, st));
    HIPCK(q_cand_keys(v, x->sel.as<uint64_t>(), x->seloff.as<int64_t>(), nsel, x->surv.as<int32_t>(), nsurv,
                      ps.pair_u, ps.pair_q, x->cnt.as<uint32_t>(), x->candoff.as<int64_t>(), x->cursor.as<int32_t>(),
                      x->candkeys.as<uint64_t>(), st));
    HIPCK(launch_select(x->candkeys.as<uint64_t>(), x->candoff.as<int64_t>(), x->kdev.as<int32_t>(), nq,
                        x->bestoff.as<int64_t>(), x->ans.as<uint64_t>(), st));
    HIPCK(q_write_answer(x->ans.as<uint64_t>(), ksum, ids_out, ranks_out, st));
    HIPCK(hipEventRecord(sev[5], st));
    // one read-back of the counters and the survivors per query
    unsigned long long ctr[32] = {};
    std::vector<int32_t> hq(nq, 0);
    HIPCK(hipMemcpyAsync(ctr, x->ctr.p, sizeof ctr, hipMemcpyDeviceToHost, st));
    HIPCK(hipMemcpyAsync(hq.data(), x->qcount.p, nq * 4, hipMemcpyDeviceToHost, st));
    HIPCK(hipStreamSynchronize(st));
    x->stats.compares = (int64_t)ctr[1];
    x->stats.flips = (int64_t)ctr[2];
    x->stats.compare_slots = (int64_t)ctr[3];
    x->stats.mfma_flop = (int64_t)ctr[5];
    x->stats.scored_pairs = (int64_t)ctr[7];
    x->stats.scored_seed = (int64_t)ctr[16];
    x->stats.scored_exact = (int64_t)ctr[16] + (int64_t)(ctr[7] - ctr[17]);
    x->stats.ms_thresh = event_ms(sev[0], sev[1]);
    x->stats.ms_seed = event_ms(sev[1], sev[2]);
    x->stats.ms_screen = event_ms(sev[2], sev[3]);
    x->stats.ms_refine = event_ms(sev[3], sev[4]);
    x->stats.ms_select = event_ms(sev[4], sev[5]);
    x->stats.ms_total = now_ms() - t0;
    if (c) {
        int64_t settled = 0;
        for (int q = 0; q < nq; ++q) settled += (hq[q] == 0);
        x->stats.approx_settled = settled;
    }
    return RKR_OK;
}

extern "C" rkr_status rkr_query_batch(rkr_index *x, int32_t nq, const void *Qm, const int32_t *k, const double *c,
                                      const int64_t *cand_off, const int32_t *cand_ids, int32_t *ids_out,
                                      int32_t *ranks_out) {
    return run_batch(x, nq, Qm, k, c, cand_off, cand_ids, ids_out, ranks_out);
}

extern "C" rkr_status rkr_query_exact(rkr_index *x, const void *q, int32_t k, int32_t *ids_out, int32_t *ranks_out) {
    return rkr_query_batch(x, 1, q, &k, nullptr, nullptr, nullptr, ids_out, ranks_out);
}

extern "C" rkr_status rkr_query_approx(rkr_index *x, const void *q, int32_t k, double c, int32_t *ids_out,
                                       int32_t *rank_ub_out) {
    if (!(c >= 1.0)) return fail(RKR_E_INVALID, "c must be >= 1");
    return rkr_query_batch(x, 1, q, &k, &c, nullptr, nullptr, ids_out, rank_ub_out);
}

static rkr_status ranks_eager(rkr_index *x, const void *q, int32_t *ranks_out) {
    hipStream_t st = x->st;
    const int64_t n = x->n;
    const double t0 = now_ms();
    x->stats = rkr_query_stats{};
    x->stats.queries = 1;
    x->sc.reset();
    PairSet ps;
    ps.nq = 1;
    ps.dense = 1;
    ps.npairs = n;
    x->stats.pairs = n;
    HIPCK(x->pair_u.ensure(n * 4));
    HIPCK(x->pair_q.ensure(n * 4));
    HIPCK(x->t64.ensure(n * 8));
    HIPCK(x->cnt.ensure(n * 4));
    HIPCK(x->allpid.ensure(n * 4));
    HIPCK(x->ctr.ensure(256));
    ps.pair_u = x->pair_u.as<int32_t>();
    ps.pair_q = x->pair_q.as<int32_t>();
    ps.t64 = x->t64.as<double>();
    HIPCK(launch_fill_u32(x->flags.as<uint32_t>(), 0, 4, st));
    HIPCK(launch_check_values(q, x->d, x->mk, x->flags.as<int>(), st));
    HIPCK(dense_pairs(x, n, 1, st));
    HIPCK(launch_thresh_dense(x->Um.p, n, q, 1, x->d, x->mk, ps.t64, st));
    int flags = 0;
    HIPCK(hipMemcpyAsync(&flags, x->flags.p, 4, hipMemcpyDeviceToHost, st));
    HIPCK(hipStreamSynchronize(st));
    if (flags) return fail(RKR_E_INVALID, "the query holds a non-finite value or one above 2^50");
    HIPCK(launch_fill_u32(x->ctr.as<uint32_t>(), 0, 16, st));
    HIPCK(launch_iota(x->allpid.as<int32_t>(), n, st));
    rkr_status rs = exact_count(x, ps, x->allpid.as<int32_t>(), n);
    if (rs != RKR_OK) return rs;
    HIPCK(q_ranks_out(x->cnt.as<uint32_t>(), n, ranks_out, st));
    unsigned long long ctr[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    HIPCK(hipMemcpyAsync(ctr, x->ctr.p, 64, hipMemcpyDeviceToHost, st));
    HIPCK(hipStreamSynchronize(st));
    x->stats.compares = (int64_t)ctr[1];
    x->stats.flips = (int64_t)ctr[2];
    x->stats.mfma_flop = (int64_t)ctr[5];
    x->stats.scored_pairs = (int64_t)ctr[7];
    x->stats.scored_exact = (int64_t)ctr[7];
    x->stats.refined_pairs = n;
    x->stats.ms_total = now_ms() - t0;
    return RKR_OK;
}

static rkr_status capture_ranks_graph(rkr_index *x) {
    RanksGraph &g = x->rg;
    const int64_t n = x->n;
    const int mes = x->mk == MK_BF16 ? 2 : 4;
    const int xv = exact_variant(x);
    const int tpw = exact_tasks_per_wg(x, xv);
    const int64_t ntask_pad = (n + 511) / 512 * 512;
    g.emit_cap = std::max<int64_t>(1 << 20, 2 * x->stats.uncertain + 65536);
    if (!g.cs) HIPCK(hipStreamCreateWithFlags(&g.cs, hipStreamNonBlocking));
    HIPCK(g.qbuf.ensure((size_t)x->d * mes));
    HIPCK(g.rbuf.ensure(n * 4));
    HIPCK(g.pair_u.ensure(n * 4));
    HIPCK(g.pair_q.ensure(n * 4));
    HIPCK(g.t64.ensure(n * 8));
    HIPCK(g.cnt.ensure(n * 4));
    HIPCK(g.ctr.ensure(64));
    HIPCK(g.emit.ensure((size_t)g.emit_cap * 8));
    HIPCK(g.ts.reserve(ntask_pad, ntask_pad / 32));
    PairSet ps;
    ps.nq = 1;
    ps.dense = 1;
    ps.npairs = n;
    ps.pair_u = g.pair_u.as<int32_t>();
    ps.pair_q = g.pair_q.as<int32_t>();
    ps.t64 = g.t64.as<double>();
    g.ts.ntask = n;
    g.ts.ntask_pad = ntask_pad;
    g.ts.cap_total = ntask_pad;
    CountArgs a = count_args(x, ps, g.ts, xv);
    const int64_t nsteps = a.nsteps;
    const int64_t gx = (n + tpw - 1) / tpw;
    int64_t nsplit = pick_nsplit(gx, nsteps, x->num_cus);
    HIPCK(g.ts.reserve_entries(ntask_pad, (int)nsplit));
    a = count_args(x, ps, g.ts, xv);
    a.steps_per_split = (nsteps + nsplit - 1) / nsplit;
    nsplit = std::max<int64_t>(1, (nsteps + a.steps_per_split - 1) / std::max<int64_t>(a.steps_per_split, 1));
    a.cnt_out = g.cnt.as<uint32_t>();
    a.emit = g.emit.as<int2>();
    a.emit_count = g.ctr.as<unsigned long long>();
    a.emit_cap = (unsigned long long)g.emit_cap;
    a.stat = g.ctr.as<unsigned long long>() + 1;
    hipStream_t cs = g.cs;
    HIPCK(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
    // kernels only (fills instead of memsets), so every replay starts clean
    hipError_t e = launch_fill_u32(g.ctr.as<uint32_t>(), 0, 16, cs);
    if (e == hipSuccess) e = launch_dense_pairs(n, 1, ps.pair_u, ps.pair_q, cs);
    if (e == hipSuccess)
        e = launch_thresh_dense(x->Um.p, n, g.qbuf.p, 1, x->d, x->mk, ps.t64, cs);
    if (e == hipSuccess) e = q_tasks_one_per_user(n, ntask_pad, ps, x->recheck ? 0 : 1, g.ts, cs);
    if (e == hipSuccess) e = launch_fill_u32(g.cnt.as<uint32_t>(), 0, n, cs);
    if (e == hipSuccess) e = launch_count(x->sk, CM_EXACT, a, (int)nsplit, xv, cs);
    if (e == hipSuccess)
        e = launch_recheck_dev(g.emit.as<int2>(), g.ctr.as<unsigned long long>(), g.emit_cap, ps.pair_u, ps.t64,
                               x->Um.p, x->Pm.p, x->d, x->mk, g.cnt.as<uint32_t>(),
                               g.ctr.as<unsigned long long>() + 2, cs);
    if (e == hipSuccess) e = q_ranks_out(g.cnt.as<uint32_t>(), n, g.rbuf.as<int32_t>(), cs);
    hipGraph_t graph = nullptr;
    hipError_t e2 = hipStreamEndCapture(cs, &graph);
    if (e != hipSuccess || e2 != hipSuccess) {
        if (graph) (void)hipGraphDestroy(graph);
        return fail_hip(e != hipSuccess ? e : e2, "graph capture of the ranks pipeline");
    }
    g.g = graph;
    HIPCK(hipGraphInstantiate(&g.ge, g.g, nullptr, nullptr, 0));
    g.valid = true;
    return RKR_OK;
}

extern "C" rkr_status rkr_ranks(rkr_index *x, const void *q, int32_t *ranks_out) {
    g_err.clear();
    if (!x || !q || !ranks_out) return fail(RKR_E_INVALID, "NULL argument");
    if (!x->qo.graph) return ranks_eager(x, q, ranks_out);
    RanksGraph &g = x->rg;
    if (!g.valid) {
        // first call: run eagerly (sizes the near-tie buffer), then capture
        rkr_status rs = ranks_eager(x, q, ranks_out);
        if (rs != RKR_OK) return rs;
        return capture_ranks_graph(x);
    }
    hipStream_t st = x->st;
    const double t0 = now_ms();
    const int mes = x->mk == MK_BF16 ? 2 : 4;
    HIPCK(launch_fill_u32(x->flags.as<uint32_t>(), 0, 4, st));
    HIPCK(launch_check_values(q, x->d, x->mk, x->flags.as<int>(), st));
    HIPCK(q_copy(q, g.qbuf.p, (int64_t)x->d * mes, st));
    HIPCK(hipGraphLaunch(g.ge, st));
    unsigned long long ctr[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    int flags = 0;
    HIPCK(hipMemcpyAsync(ctr, g.ctr.p, 64, hipMemcpyDeviceToHost, st));
    HIPCK(hipMemcpyAsync(&flags, x->flags.p, 4, hipMemcpyDeviceToHost, st));
    HIPCK(hipStreamSynchronize(st));
    if (flags) return fail(RKR_E_INVALID, "the query holds a non-finite value or one above 2^50");
    if (ctr[0] > (unsigned long long)g.emit_cap) {
        // more near ties than the captured buffer holds: answer eagerly, recapture next time
        g.destroy();
        return ranks_eager(x, q, ranks_out);
    }
    HIPCK(q_copy(g.rbuf.p, ranks_out, x->n * 4, st));
    HIPCK(hipStreamSynchronize(st));
    x->stats = rkr_query_stats{};
    x->stats.queries = 1;
    x->stats.pairs = x->n;
    x->stats.refined_pairs = x->n;
    x->stats.uncertain = (int64_t)ctr[0];
    x->stats.compares = (int64_t)ctr[1];
    x->stats.flips = (int64_t)ctr[2];
    x->stats.mfma_flop = (int64_t)ctr[5];
    x->stats.scored_pairs = (int64_t)ctr[7];
    x->stats.scored_exact = (int64_t)ctr[7];
    x->stats.ms_total = now_ms() - t0;
    x->stats.graph_replays = 1;
    return RKR_OK;
}

// ---------------------------------------------------------------------------
// All ranks without allocating (rkr_ranks_noalloc)
// ---------------------------------------------------------------------------
// The per-call device memory of rkr_ranks_noalloc is one static array per
// device (every device the library runs on holds it until the process ends).
// In host code `scratch` only names the array: its device address is taken
// once per device with hipGetSymbolAddress (that device current) and only
// that address reaches kernels.  Calls on one device share the array, so
// calls that overlap on one device race; each call clears what must start at
// zero.
static constexpr size_t kNoAllocBytes = (size_t)64 << 20;        // 64 MiB
static constexpr int64_t kNoAllocMaxUsers = (int64_t)1 << 20;
static constexpr int64_t kNoAllocMaxItems = (int64_t)1 << 22;
static __device__ __align__(256) uint8_t scratch[kNoAllocBytes];
static constexpr int kMaxDevices = 64;
static uint8_t *g_scratch_dev[kMaxDevices];
static std::mutex g_scratch_mu;

static rkr_status scratch_address(int dev, uint8_t **out) {
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (dev < 0 || dev >= kMaxDevices) return fail(RKR_E_UNSUPPORTED, "device ordinal above 63");
    if (!g_scratch_dev[dev]) {
        int cur = 0;
        HIPCK(hipGetDevice(&cur));
        if (cur != dev) HIPCK(hipSetDevice(dev));
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (cur != dev) (void)hipSetDevice(cur);
        if (e != hipSuccess) return fail_hip(e, "hipGetSymbolAddress(scratch)");
        g_scratch_dev[dev] = (uint8_t *)p;
    }
    *out = g_scratch_dev[dev];
    return RKR_OK;
}

// Bump placement inside the scratch array (256-byte aligned pieces).
struct Carve {
    uint8_t *base;
    size_t used = 0;
    template <typename T> T *take(int64_t count) {
        T *p = (T *)(base + used);
        used += ((size_t)count * sizeof(T) + 255) & ~(size_t)255;
        return p;
    }
};

// The sequence of the captured all-ranks graph (thresholds -> one entry per
// user -> exact count -> FP64 recheck -> ranks), on users in chunks whose
// entry lists and near-tie records fit the scratch array; a chunk whose near
// ties overflow is counted again in smaller chunks (a single user emits at
// most m records, which always fit).
extern "C" rkr_status rkr_ranks_noalloc(rkr_index *x, const void *q, int32_t *ranks_out) {
    g_err.clear();
    if (!x || !q || !ranks_out) return fail(RKR_E_INVALID, "NULL argument");
    const int64_t n = x->n, m = x->m;
    if (n > kNoAllocMaxUsers) return fail(RKR_E_UNSUPPORTED, "rkr_ranks_noalloc: more than 2^20 users");
    if (m > kNoAllocMaxItems) return fail(RKR_E_UNSUPPORTED, "rkr_ranks_noalloc: more than 2^22 items");
    uint8_t *base = nullptr;
    rkr_status rs = scratch_address(x->dev, &base);
    if (rs != RKR_OK) return rs;
    hipStream_t st = x->st;
    const double t0 = now_ms();
    // pieces for every user
    Carve cv{base};
    double *t64 = cv.take<double>(n);
    int32_t *pair_u = cv.take<int32_t>(n);
    int32_t *pair_q = cv.take<int32_t>(n);
    uint32_t *cnt = cv.take<uint32_t>(n);
    unsigned long long *ctr = cv.take<unsigned long long>(8);
    int *flags = cv.take<int>(4);
    const size_t fixed = cv.used;
    PairSet ps;
    ps.nq = 1;
    ps.dense = 1;
    ps.npairs = n;
    ps.pair_u = pair_u;
    ps.pair_q = pair_q;
    ps.t64 = t64;
    HIPCK(launch_fill_u32((uint32_t *)flags, 0, 4, st));
    HIPCK(launch_check_values(q, x->d, x->mk, flags, st));
    HIPCK(launch_dense_pairs(n, 1, pair_u, pair_q, st));
    HIPCK(launch_thresh_dense(x->Um.p, n, q, 1, x->d, x->mk, t64, st));
    int hflags = 0;
    HIPCK(hipMemcpyAsync(&hflags, flags, 4, hipMemcpyDeviceToHost, st));
    HIPCK(hipStreamSynchronize(st));
    if (hflags) return fail(RKR_E_INVALID, "the query holds a non-finite value or one above 2^50");

    x->stats = rkr_query_stats{};
    x->stats.queries = 1;
    x->stats.pairs = n;
    const int xv = exact_variant(x);
    const int tpw = exact_tasks_per_wg(x, xv);
    // first chunk: every user, or as many as leave half of the array to records
    const size_t per_task_max = 36 + 4 * 16;   // entry lists with up to 16 item splits
    int64_t chunk = std::min<int64_t>(n, (int64_t)((kNoAllocBytes - fixed) / 2 / per_task_max));
    chunk = std::max<int64_t>(chunk, 1);
    int64_t u0 = 0;
    while (u0 < n) {
        const int64_t C = std::min<int64_t>(chunk, n - u0);
        const int64_t ntp = (C + 511) / 512 * 512;
        Carve cc{base, fixed};
        TaskSet ts;
        ts.task_user = cc.take<int32_t>(ntp);
        ts.len = cc.take<int32_t>(ntp);
        ts.blk_base = cc.take<int64_t>(ntp / 32 + 1);
        ts.ent_pid = cc.take<int32_t>(ntp);
        ts.ent_q = cc.take<int32_t>(ntp);
        ts.ent_th = cc.take<float>(ntp);
        ts.ent_tl = cc.take<float>(ntp);
        ts.ent_tm = cc.take<float>(ntp);
        ts.ntask = C;
        ts.ntask_pad = ntp;
        ts.cap_total = ntp;
        CountArgs a = count_args(x, ps, ts, xv);
        const int64_t nsteps = a.nsteps;
        int64_t nsplit = pick_nsplit((C + tpw - 1) / tpw, nsteps, x->num_cus);
        a.steps_per_split = (nsteps + nsplit - 1) / nsplit;
        nsplit = std::max<int64_t>(1, (nsteps + a.steps_per_split - 1) / std::max<int64_t>(a.steps_per_split, 1));
        ts.ent_cnt = cc.take<uint32_t>(ntp * nsplit);
        a.ent_cnt = ts.ent_cnt;
        if (cc.used + 8 * 1024 > kNoAllocBytes) return fail(RKR_E_DEVICE, "rkr_ranks_noalloc: scratch layout");
        int2 *emit = (int2 *)(base + cc.used);
        const int64_t emit_cap = (int64_t)((kNoAllocBytes - cc.used) / sizeof(int2));
        a.cnt_out = cnt;
        a.emit = emit;
        a.emit_count = ctr;
        a.emit_cap = (unsigned long long)emit_cap;
        a.stat = ctr + 1;
        HIPCK(launch_fill_u32((uint32_t *)ctr, 0, 16, st));
        HIPCK(q_tasks_one_per_user(C, ntp, ps, x->recheck ? 0 : 1, ts, st, u0));
        HIPCK(launch_fill_u32(cnt + u0, 0, C, st));
        HIPCK(launch_count(x->sk, CM_EXACT, a, (int)nsplit, xv, st));
        unsigned long long c8[8] = {0, 0, 0, 0, 0, 0, 0, 0};
        HIPCK(hipMemcpyAsync(c8, ctr, 64, hipMemcpyDeviceToHost, st));
        HIPCK(hipStreamSynchronize(st));
        const unsigned long long ne = c8[0];
        if (ne > (unsigned long long)emit_cap) {
            if (C == 1) return fail(RKR_E_DEVICE, "rkr_ranks_noalloc: near ties of one user exceed the scratch array");
            // too many near ties for this chunk: count it again in smaller chunks
            x->stats.emit_retries += 1;
            const double shrink = 0.8 * (double)emit_cap / (double)ne;
            chunk = std::max<int64_t>(1, std::min<int64_t>(C / 2, (int64_t)((double)C * shrink)));
            continue;
        }
        HIPCK(launch_recheck(emit, (int64_t)ne, pair_u, t64, x->Um.p, x->Pm.p, x->d, x->mk, cnt, ctr + 2, st));
        HIPCK(q_ranks_out(cnt + u0, C, ranks_out + u0, st));
        unsigned long long flips = 0;
        HIPCK(hipMemcpyAsync(&flips, ctr + 2, 8, hipMemcpyDeviceToHost, st));
        HIPCK(hipStreamSynchronize(st));
        x->stats.uncertain += (int64_t)ne;
        x->stats.compares += (int64_t)c8[1];
        x->stats.flips += (int64_t)flips;
        x->stats.mfma_flop += (int64_t)c8[5];
        x->stats.scored_pairs += (int64_t)c8[7];
        u0 += C;
    }
    x->stats.refined_pairs = n;
    x->stats.scored_exact = x->stats.scored_pairs;
    x->stats.ms_total = now_ms() - t0;
    return RKR_OK;
}

// ---------------------------------------------------------------------------
// the paper's table query (Sec. 4.3, steps 1-3) on the index's rank table
// ---------------------------------------------------------------------------
// The query of Sec. 4.3 on a rank table: the exact-cell table built with the
// index (paper = false) or the paper's estimated table of Alg. 1 (paper =
// true, whose bounds are FP32 values: the keys carry their order keys).
static rkr_status table_query_batch(rkr_index *x, int32_t nq, const void *Qm, const int32_t *k, const double *c,
                                    int32_t *ids_out, double *est_out, bool paper) {
    g_err.clear();
    if (!x || !Qm || !k || !c || !ids_out || !est_out) return fail(RKR_E_INVALID, "NULL argument");
    if (!paper && !x->has_table) return fail(RKR_E_STATE, "index built without a rank table");
    if (paper && !x->has_ptab) return fail(RKR_E_STATE, "no paper rank table (rkr_paper_table_build)");
    const int fk = paper ? 1 : 0;
    if (nq < 1 || nq > 65535) return fail(RKR_E_INVALID, "nq must be in [1, 65535]");
    const int64_t n = x->n;
    if (n * (int64_t)nq >= ((int64_t)1 << 31)) return fail(RKR_E_UNSUPPORTED, "n * nq must stay below 2^31");
    std::vector<int64_t> off(nq + 1, 0), segoff(nq + 1, 0);
    for (int q = 0; q < nq; ++q) {
        if (k[q] < 1 || (int64_t)k[q] > n) return fail(RKR_E_INVALID, "k must be in [1, n]");
        if (k[q] > 4096) return fail(RKR_E_UNSUPPORTED, "k above 4096");
        if (!(c[q] >= 1.0) || c[q] == HUGE_VAL) return fail(RKR_E_INVALID, "c must be finite and at least 1");
        off[q + 1] = off[q] + k[q];
        segoff[q + 1] = segoff[q] + n;
    }
    hipStream_t st = x->st;
    const double t0 = now_ms();
    const int64_t np = n * nq, total = off[nq];
    x->stats = rkr_query_stats{};
    x->stats.queries = nq;
    x->stats.pairs = np;
    x->sc.reset();
    HIPCK(x->t64.ensure(np * 8));
    HIPCK(x->flags.ensure(16));
    auto take = [&](int64_t bytes) { return x->sc.take(bytes); };
    uint64_t *key_lo = (uint64_t *)take(np * 8), *key_hi = (uint64_t *)take(np * 8);
    uint64_t *key_c = (uint64_t *)take(np * 8), *key_t = (uint64_t *)take(np * 8);
    double *est = (double *)take(np * 8);
    uint64_t *sel_lo = (uint64_t *)take(total * 8), *sel_hi = (uint64_t *)take(total * 8);
    uint64_t *sel_c = (uint64_t *)take(total * 8), *sel_t = (uint64_t *)take(total * 8);
    int64_t *d_off = (int64_t *)take((nq + 1) * 8), *d_seg = (int64_t *)take((nq + 1) * 8);
    int64_t *d_offc = (int64_t *)take((nq + 1) * 8), *d_offt = (int64_t *)take((nq + 1) * 8);
    int32_t *d_k = (int32_t *)take(nq * 4), *d_nc = (int32_t *)take(nq * 4), *d_nt = (int32_t *)take(nq * 4);
    int32_t *d_first = (int32_t *)take(nq * 4);
    double *d_c = (double *)take(nq * 8);
    uint32_t *d_Rlo = (uint32_t *)take(nq * 4), *d_Rhi = (uint32_t *)take(nq * 4);
    unsigned long long *d_nadm = (unsigned long long *)take(nq * 8);
    if (!key_lo || !key_hi || !key_c || !key_t || !est || !sel_lo || !sel_hi || !sel_c || !sel_t || !d_off ||
        !d_seg || !d_offc || !d_offt || !d_k || !d_nc || !d_nt || !d_first || !d_c || !d_Rlo || !d_Rhi || !d_nadm)
        return fail(RKR_E_NOMEM, "out of device memory (table query)");
    HIPCK(hipMemcpyAsync(d_off, off.data(), (nq + 1) * 8, hipMemcpyHostToDevice, st));
    HIPCK(hipMemcpyAsync(d_seg, segoff.data(), (nq + 1) * 8, hipMemcpyHostToDevice, st));
    HIPCK(hipMemcpyAsync(d_k, k, nq * 4, hipMemcpyHostToDevice, st));
    HIPCK(hipMemcpyAsync(d_c, c, nq * 8, hipMemcpyHostToDevice, st));
    // step 1: u.q for every (user, query) (spec FP64 dots), brackets, estimates
    HIPCK(launch_fill_u32(x->flags.as<uint32_t>(), 0, 4, st));
    HIPCK(launch_check_values(Qm, (int64_t)nq * x->d, x->mk, x->flags.as<int>(), st));
    HIPCK(launch_thresh_dense(x->Um.p, n, Qm, nq, x->d, x->mk, x->t64.as<double>(), st));
    if (paper)
        HIPCK(launch_ptq_bounds(n, nq, x->m, x->ptab_tau, x->t64.as<double>(), x->ptab_fmin.as<double>(),
                                x->ptab_step.as<double>(), x->ptab_cells.as<float>(), key_lo, key_hi, est, st));
    else
        HIPCK(q_tqb_bounds(n, nq, x->m, x->t64.as<double>(), x->tab_t.as<double>(), x->tab_cnt.as<uint32_t>(),
                           key_lo, key_hi, est, st));
    // R_lo_k, R_hi_k per query and the case of step 2
    HIPCK(launch_select(key_lo, d_seg, d_k, nq, d_off, sel_lo, st));
    HIPCK(launch_select(key_hi, d_seg, d_k, nq, d_off, sel_hi, st));
    HIPCK(q_tqb_kth(nq, d_k, d_c, sel_lo, sel_hi, d_off, d_Rlo, d_Rhi, d_first, st, fk));
    // step 2, second case: admitted users and the users left open
    HIPCK(launch_fill_u32((uint32_t *)d_nadm, 0, 2 * (int64_t)nq, st));
    HIPCK(q_tqb_classify(n, nq, d_c, d_Rlo, d_Rhi, d_first, key_lo, key_hi, est, key_c, key_t, d_nadm, st, fk));
    std::vector<unsigned long long> nadm(nq);
    std::vector<int32_t> first(nq), nc(nq), nt(nq);
    int flags = 0;
    HIPCK(hipMemcpyAsync(nadm.data(), d_nadm, nq * 8, hipMemcpyDeviceToHost, st));
    HIPCK(hipMemcpyAsync(first.data(), d_first, nq * 4, hipMemcpyDeviceToHost, st));
    HIPCK(hipMemcpyAsync(&flags, x->flags.p, 4, hipMemcpyDeviceToHost, st));
    HIPCK(hipStreamSynchronize(st));
    if (flags) return fail(RKR_E_INVALID, "a query holds a non-finite value or one above 2^50");
    // fewer than k users have r_hi < R_hi_k, and at least k have r_lo <= R_hi_k
    std::vector<int64_t> offc(nq + 1, 0), offt(nq + 1, 0);
    int64_t admitted = 0;
    for (int q = 0; q < nq; ++q) {
        nc[q] = first[q] ? 0 : (int32_t)std::min<unsigned long long>(nadm[q], (unsigned long long)k[q]);
        nt[q] = first[q] ? 0 : k[q] - nc[q];
        offc[q + 1] = offc[q] + nc[q];
        offt[q + 1] = offt[q] + nt[q];
        admitted += (int64_t)nadm[q];
    }
    HIPCK(hipMemcpyAsync(d_nc, nc.data(), nq * 4, hipMemcpyHostToDevice, st));
    HIPCK(hipMemcpyAsync(d_nt, nt.data(), nq * 4, hipMemcpyHostToDevice, st));
    HIPCK(hipMemcpyAsync(d_offc, offc.data(), (nq + 1) * 8, hipMemcpyHostToDevice, st));
    HIPCK(hipMemcpyAsync(d_offt, offt.data(), (nq + 1) * 8, hipMemcpyHostToDevice, st));
    // step 2's admitted users by (r_hi, id); step 3's fill by (fl32(estimate), id)
    HIPCK(launch_select(key_c, d_seg, d_nc, nq, d_offc, sel_c, st));
    HIPCK(launch_select(key_t, d_seg, d_nt, nq, d_offt, sel_t, st));
    HIPCK(q_tqb_answer(nq, n, total, d_off, d_first, d_off, sel_hi, d_nc, d_offc, sel_c, d_offt, sel_t, est, ids_out,
                       est_out, st, fk));
    HIPCK(hipStreamSynchronize(st));
    x->stats.survivors = admitted;
    x->stats.ms_total = now_ms() - t0;
    return RKR_OK;
}

extern "C" rkr_status rkr_query_table_batch(rkr_index *x, int32_t nq, const void *Qm, const int32_t *k,
                                            const double *c, int32_t *ids_out, double *est_out) {
    return table_query_batch(x, nq, Qm, k, c, ids_out, est_out, false);
}

extern "C" rkr_status rkr_query_table(rkr_index *x, const void *q, int32_t k, double c, int32_t *ids_out,
                                      double *est_out) {
    return rkr_query_table_batch(x, 1, q, &k, &c, ids_out, est_out);
}

// ---------------------------------------------------------------------------
// the paper's own rank table (Alg. 1, Sec. 4.2) and its query (Sec. 4.3)
// ---------------------------------------------------------------------------
extern "C" rkr_status rkr_paper_table_build(rkr_index *x, int32_t tau, int32_t omega, int32_t s,
                                            const int32_t *sample_pos) {
    g_err.clear();
    if (!x || !sample_pos) return fail(RKR_E_INVALID, "NULL argument");
    if (tau < 2) return fail(RKR_E_INVALID, "tau must be at least 2");
    if (tau > paper_table_tau_max())
        return fail(RKR_E_UNSUPPORTED, "tau above " + std::to_string(paper_table_tau_max()));
    if (omega < 1 || s < 1) return fail(RKR_E_INVALID, "omega and s must be positive");
    if ((int64_t)omega * s > ((int64_t)1 << 22)) return fail(RKR_E_UNSUPPORTED, "omega * s above 2^22");
    const int64_t n = x->n, m = x->m;
    const int d = x->d;
    hipStream_t st = x->st;
    // buckets of the norm-sorted items and the positions of their samples
    std::vector<int32_t> soff(omega + 1, 0), idx;
    std::vector<int64_t> bsize(omega, 0);
    for (int l = 0; l < omega; ++l) {
        const int64_t b0 = (int64_t)l * m / omega, b1 = (int64_t)(l + 1) * m / omega;
        const int64_t size = b1 - b0, sl = std::min<int64_t>(s, size);
        bsize[l] = size;
        std::vector<int32_t> seen(sample_pos + (int64_t)l * s, sample_pos + (int64_t)l * s + sl);
        for (int32_t v : seen)
            if (v < 0 || v >= size)
                return fail(RKR_E_INVALID, "sample position out of its bucket (bucket " + std::to_string(l) + ")");
        std::sort(seen.begin(), seen.end());
        if (std::adjacent_find(seen.begin(), seen.end()) != seen.end())
            return fail(RKR_E_INVALID, "sample positions repeat within bucket " + std::to_string(l));
        for (int64_t i = 0; i < sl; ++i) idx.push_back((int32_t)(b0 + sample_pos[(int64_t)l * s + i]));
        soff[l + 1] = soff[l] + (int32_t)sl;
    }
    const int ns = soff[omega];
    const int mes = x->mk == MK_BF16 ? 2 : 4;
    x->has_ptab = false;
    x->sc.reset();
    HIPCK(x->ptab_fmin.ensure(n * 8));
    HIPCK(x->ptab_step.ensure(n * 8));
    HIPCK(x->ptab_cells.ensure(n * (int64_t)tau * 4));
    double *unorm = (double *)x->sc.take(n * 8);
    double *pmax = (double *)x->sc.take(8);
    int32_t *d_soff = (int32_t *)x->sc.take((omega + 1) * 4);
    int64_t *d_bsize = (int64_t *)x->sc.take(omega * 8);
    int32_t *d_idx = (int32_t *)x->sc.take(std::max(ns, 1) * 4);
    void *Sm = x->sc.take((int64_t)std::max(ns, 1) * d * mes);
    // sample scores of a chunk of users: at most 2^28 doubles
    const int64_t chunk = std::max<int64_t>(64, (((int64_t)1 << 28) / std::max(ns, 1)) / 64 * 64);
    const int64_t cu = std::min<int64_t>(n, chunk);
    double *S = (double *)x->sc.take(cu * std::max(ns, 1) * 8);
    if (!unorm || !pmax || !d_soff || !d_bsize || !d_idx || !Sm || !S)
        return fail(RKR_E_NOMEM, "out of device memory (paper rank table)");
    HIPCK(hipMemcpyAsync(d_soff, soff.data(), (omega + 1) * 4, hipMemcpyHostToDevice, st));
    HIPCK(hipMemcpyAsync(d_bsize, bsize.data(), omega * 8, hipMemcpyHostToDevice, st));
    if (ns > 0) {
        HIPCK(hipMemcpyAsync(d_idx, idx.data(), (size_t)ns * 4, hipMemcpyHostToDevice, st));
        HIPCK(launch_gather_rows(x->Pm.p, d_idx, ns, d, x->mk, Sm, st));
    }
    HIPCK(launch_spec_norm(x->Um.p, n, d, x->mk, unorm, st));
    // the items are in norm order: the first has the largest spec norm
    if (m > 0)
        HIPCK(launch_spec_norm(x->Pm.p, 1, d, x->mk, pmax, st));
    else
        HIPCK(launch_fill_u32((uint32_t *)pmax, 0, 2, st));
    for (int64_t u0 = 0; u0 < n; u0 += cu) {
        const int64_t nu = std::min<int64_t>(cu, n - u0);
        if (ns > 0)
            HIPCK(launch_thresh_dense((const uint8_t *)x->Um.p + u0 * d * mes, nu, Sm, ns, d, x->mk, S, st));
        HIPCK(launch_ptab_cells(u0, nu, S, ns, omega, d_soff, d_bsize, tau, unorm, pmax, x->ptab_fmin.as<double>(),
                                x->ptab_step.as<double>(), x->ptab_cells.as<float>(), st));
    }
    HIPCK(hipStreamSynchronize(st));
    x->sc.reset();
    x->ptab_tau = tau;
    x->has_ptab = true;
    return RKR_OK;
}

extern "C" rkr_status rkr_paper_table(const rkr_index *x, double *fmin_out, double *step_out, float *cells_out) {
    g_err.clear();
    if (!x || !fmin_out || !step_out || !cells_out) return fail(RKR_E_INVALID, "NULL argument");
    if (!x->has_ptab) return fail(RKR_E_STATE, "no paper rank table (rkr_paper_table_build)");
    HIPCK(hipMemcpyAsync(fmin_out, x->ptab_fmin.p, x->n * 8, hipMemcpyDeviceToDevice, x->st));
    HIPCK(hipMemcpyAsync(step_out, x->ptab_step.p, x->n * 8, hipMemcpyDeviceToDevice, x->st));
    HIPCK(hipMemcpyAsync(cells_out, x->ptab_cells.p, x->n * (int64_t)x->ptab_tau * 4, hipMemcpyDeviceToDevice, x->st));
    HIPCK(hipStreamSynchronize(x->st));
    return RKR_OK;
}

extern "C" rkr_status rkr_query_paper_table_batch(rkr_index *x, int32_t nq, const void *Qm, const int32_t *k,
                                                  const double *c, int32_t *ids_out, double *val_out) {
    return table_query_batch(x, nq, Qm, k, c, ids_out, val_out, true);
}

extern "C" rkr_status rkr_query_paper_table(rkr_index *x, const void *q, int32_t k, double c, int32_t *ids_out,
                                            double *val_out) {
    return rkr_query_paper_table_batch(x, 1, q, &k, &c, ids_out, val_out);
}

// ---------------------------------------------------------------------------
// learned rank estimator
// ---------------------------------------------------------------------------
static rkr_status ensure_params(rkr_index *x) {
    HIPCK(x->est.params.ensure(MLP_NPARAM * 4));
    HIPCK(x->est.grads.ensure(MLP_NPARAM * 4));
    HIPCK(x->est.adam_m.ensure(MLP_NPARAM * 4));
    HIPCK(x->est.adam_v.ensure(MLP_NPARAM * 4));
    return RKR_OK;
}

// Training data: for each training query, the pairs_per_query / 2 users of
// best t/|u| plus pairs_per_query / 2 users spread uniformly over the user
// ids (stratified, random offset per query); their exact ranks come from the
// exact counting path.  Then E epochs of minibatch Adam on ln r.
extern "C" rkr_status rkr_train(rkr_index *x, int32_t nq, const void *Qm, int32_t pairs_per_query, int32_t epochs,
                                int32_t batch, float lr, uint64_t seed) {
    g_err.clear();
    if (!x) return fail(RKR_E_INVALID, "index is NULL");
    if (!x->est.has_sketch) return fail(RKR_E_STATE, "index built without a sketch (sketch_samples = 0)");
    if (nq < 1 || nq > 65535 || !Qm) return fail(RKR_E_INVALID, "nq must be in 1..65535 and Qm non-NULL");
    if (pairs_per_query < 2 || epochs < 1 || batch < 1 || !(lr > 0.0f))
        return fail(RKR_E_INVALID, "pairs_per_query >= 2, epochs >= 1, batch >= 1 and lr > 0 required");
    hipStream_t st = x->st;
    const int64_t n = x->n;
    const int d = x->d;
    const double t0 = now_ms();
    x->sc.reset();
    PairSet ps;
    ps.nq = nq;
    ps.dense = 1;
    const int64_t npairs = n * nq;
    if (npairs >= ((int64_t)1 << 31)) return fail(RKR_E_UNSUPPORTED, "2^31 or more (user, query) pairs: fewer queries");
    ps.npairs = npairs;
    HIPCK(x->pair_u.ensure(npairs * 4));
    HIPCK(x->pair_q.ensure(npairs * 4));
    HIPCK(x->t64.ensure(npairs * 8));
    HIPCK(x->cnt.ensure(npairs * 4));
    HIPCK(x->ctr.ensure(256));
    ps.pair_u = x->pair_u.as<int32_t>();
    ps.pair_q = x->pair_q.as<int32_t>();
    ps.t64 = x->t64.as<double>();
    HIPCK(launch_fill_u32(x->flags.as<uint32_t>(), 0, 4, st));
    HIPCK(launch_check_values(Qm, (int64_t)nq * d, x->mk, x->flags.as<int>(), st));
    HIPCK(dense_pairs(x, n, nq, st));
    HIPCK(launch_thresh_dense(x->Um.p, n, Qm, nq, d, x->mk, ps.t64, st));
    // best users by t/|u| (select) + stratified users, marked in a pair flag array
    const int top = (int)std::min<int64_t>(std::min<int64_t>(pairs_per_query / 2, 4096), n);
    const int strat = (int)std::min<int64_t>(pairs_per_query - pairs_per_query / 2, n);
    std::vector<int64_t> segoff(nq + 1), seloff(nq + 1);
    std::vector<int32_t> Sv(nq, top);
    for (int q = 0; q <= nq; ++q) { segoff[q] = (int64_t)q * n; seloff[q] = (int64_t)q * top; }
    HIPCK(x->segoff.ensure((nq + 1) * 8));
    HIPCK(x->seloff.ensure((nq + 1) * 8));
    HIPCK(x->sdev.ensure(nq * 4));
    HIPCK(x->keys.ensure(npairs * 8));
    HIPCK(x->sel.ensure((int64_t)nq * top * 8 + 8));
    HIPCK(x->seedflag.ensure(npairs));
    HIPCK(hipMemcpyAsync(x->segoff.p, segoff.data(), (nq + 1) * 8, hipMemcpyHostToDevice, st));
    HIPCK(hipMemcpyAsync(x->seloff.p, seloff.data(), (nq + 1) * 8, hipMemcpyHostToDevice, st));
    HIPCK(hipMemcpyAsync(x->sdev.p, Sv.data(), nq * 4, hipMemcpyHostToDevice, st));
    QView v{1, nq, n, x->segoff.as<int64_t>(), nullptr};
    HIPCK(q_seed_keys(v, ps.pair_u, ps.t64, x->unorm3.as<double>(), nullptr, npairs, x->keys.as<uint64_t>(), st));
    HIPCK(launch_select(x->keys.as<uint64_t>(), x->segoff.as<int64_t>(), x->sdev.as<int32_t>(), nq,
                        x->seloff.as<int64_t>(), x->sel.as<uint64_t>(), st));
    HIPCK(launch_fill_u8(x->seedflag.as<uint8_t>(), 0, npairs, st));
    HIPCK(q_mark_selected(v, x->sel.as<uint64_t>(), x->seloff.as<int64_t>(), (int64_t)nq * top,
                          x->seedflag.as<uint8_t>(), st));
    HIPCK(est_mark_strided(nq, n, strat, seed, x->seedflag.as<uint8_t>(), st));
    HIPCK(x->seedpid.ensure(npairs * 4));
    int64_t N = 0;
    HIPCK(q_compact_flags(x->seedflag.as<uint8_t>(), npairs, x->seedpid.as<int32_t>(), &N, x->sc, st));
    HIPCK(launch_fill_u32(x->ctr.as<uint32_t>(), 0, 16, st));
    rkr_status rs = exact_count(x, ps, x->seedpid.as<int32_t>(), N);
    if (rs != RKR_OK) return rs;
    // features and targets
    HIPCK(x->est.feat.ensure(N * MLP_IN * 4));
    HIPCK(x->est.targ.ensure(N * 4));
    HIPCK(x->est.work.ensure(N * 8));
    float *X = x->est.feat.as<float>();
    float *z = x->est.targ.as<float>();
    HIPCK(est_features(x->seedpid.as<int32_t>(), N, ps.pair_u, ps.t64, x->unorm3.as<double>(),
                       x->est.sketch.as<float>(), x->cnt.as<uint32_t>(), X, z, st));
    rs = ensure_params(x);
    if (rs != RKR_OK) return rs;
    HIPCK(launch_fill_u32(x->est.adam_m.as<uint32_t>(), 0, MLP_NPARAM, st));
    HIPCK(launch_fill_u32(x->est.adam_v.as<uint32_t>(), 0, MLP_NPARAM, st));
    HIPCK(est_init(x->est, z, N, seed, x->sc, st));
    // minibatch Adam; epoch e visits the samples in the order (a_e i + b_e) mod N
    int64_t *order = x->est.work.as<int64_t>();
    double *lossd = (double *)x->sc.take(8);
    if (!lossd) return fail(RKR_E_NOMEM, "scratch");
    const int64_t B = std::min<int64_t>(batch, N);
    int step = 0;
    double last = 0.0;
    static const int64_t primes[] = {1000003, 999983, 1299709, 1686049, 2750159, 3497861, 4256233, 5800079};
    for (int e = 0; e < epochs; ++e) {
        int64_t a = primes[e % 8];
        while (N > 1 && std::__gcd(a, N) != 1) ++a;
        HIPCK(est_perm(order, N, a % std::max<int64_t>(N, 1), (int64_t)(seed + 7919 * e) % std::max<int64_t>(N, 1), st));
        double esum = 0.0;
        for (int64_t off = 0; off < N; off += B) {
            const int64_t nb = std::min<int64_t>(B, N - off);
            HIPCK(est_fwd_bwd(x->est, X, z, order, N, off, nb, 1.0f / (float)nb, x->est.grads.as<float>(), lossd,
                              x->sc, st));
            HIPCK(est_adam(x->est, lr, ++step, st));
            if (e == epochs - 1) {
                double l = 0.0;
                HIPCK(hipMemcpyAsync(&l, lossd, 8, hipMemcpyDeviceToHost, st));
                HIPCK(hipStreamSynchronize(st));
                esum += l;
            }
        }
        if (e == epochs - 1) last = esum / (double)N;
    }
    HIPCK(hipStreamSynchronize(st));
    x->est.trained = true;
    x->est.last_loss = last;
    x->stats = rkr_query_stats{};
    x->stats.pairs = N;
    x->stats.mlp_loss = last;
    x->stats.ms_total = now_ms() - t0;
    return RKR_OK;
}

extern "C" rkr_status rkr_predict(rkr_index *x, int32_t nq, const void *Qm, float *out) {
    g_err.clear();
    if (!x || !Qm || !out) return fail(RKR_E_INVALID, "NULL argument");
    if (!x->est.trained) return fail(RKR_E_STATE, "estimator not trained");
    if (nq < 1 || nq > 65535) return fail(RKR_E_INVALID, "nq must be in 1..65535");
    hipStream_t st = x->st;
    const int64_t n = x->n, npairs = n * nq;
    if (npairs >= ((int64_t)1 << 31)) return fail(RKR_E_UNSUPPORTED, "2^31 or more (user, query) pairs: fewer queries");
    x->sc.reset();
    HIPCK(x->pair_u.ensure(npairs * 4));
    HIPCK(x->pair_q.ensure(npairs * 4));
    HIPCK(x->t64.ensure(npairs * 8));
    HIPCK(dense_pairs(x, n, nq, st));
    HIPCK(launch_thresh_dense(x->Um.p, n, Qm, nq, x->d, x->mk, x->t64.as<double>(), st));
    HIPCK(est_infer(x->est, nullptr, nullptr, npairs, x->pair_u.as<int32_t>(), x->t64.as<double>(),
                    x->unorm3.as<double>(), out, nq, n, st));
    HIPCK(hipStreamSynchronize(st));
    return RKR_OK;
}

extern "C" rkr_status rkr_mlp_get(rkr_index *x, float *p) {
    g_err.clear();
    if (!x || !p) return fail(RKR_E_INVALID, "NULL argument");
    if (!x->est.trained) return fail(RKR_E_STATE, "estimator has no parameters");
    HIPCK(hipMemcpyAsync(p, x->est.params.p, MLP_NPARAM * 4, hipMemcpyDeviceToHost, x->st));
    HIPCK(hipStreamSynchronize(x->st));
    return RKR_OK;
}

extern "C" rkr_status rkr_mlp_set(rkr_index *x, const float *p) {
    g_err.clear();
    if (!x || !p) return fail(RKR_E_INVALID, "NULL argument");
    if (!x->est.has_sketch) return fail(RKR_E_STATE, "index built without a sketch (sketch_samples = 0)");
    rkr_status rs = ensure_params(x);
    if (rs != RKR_OK) return rs;
    HIPCK(hipMemcpyAsync(x->est.params.p, p, MLP_NPARAM * 4, hipMemcpyHostToDevice, x->st));
    HIPCK(hipStreamSynchronize(x->st));
    x->est.trained = true;
    return RKR_OK;
}

extern "C" rkr_status rkr_mlp_grad(rkr_index *x, const float *X, const float *z, int32_t N, float *g, double *loss) {
    g_err.clear();
    if (!x || !X || !z || !g || !loss) return fail(RKR_E_INVALID, "NULL argument");
    if (N < 1) return fail(RKR_E_INVALID, "N must be positive");
    if (!x->est.trained) return fail(RKR_E_STATE, "estimator has no parameters");
    x->sc.reset();
    double *ld = (double *)x->sc.take(8);
    if (!ld) return fail(RKR_E_NOMEM, "scratch");
    HIPCK(est_fwd_bwd(x->est, X, z, nullptr, N, 0, N, 1.0f / (float)N, g, ld, x->sc, x->st));
    double l = 0.0;
    HIPCK(hipMemcpyAsync(&l, ld, 8, hipMemcpyDeviceToHost, x->st));
    HIPCK(hipStreamSynchronize(x->st));
    *loss = l / (double)N;
    return RKR_OK;
}

extern "C" rkr_status rkr_mlp_adam(rkr_index *x, const float *grad, float lr, int32_t step, int32_t reset) {
    g_err.clear();
    if (!x || !grad) return fail(RKR_E_INVALID, "NULL argument");
    if (step < 1 || !(lr > 0.0f)) return fail(RKR_E_INVALID, "step >= 1 and lr > 0 required");
    if (!x->est.trained) return fail(RKR_E_STATE, "estimator has no parameters");
    hipStream_t st = x->st;
    if (reset) {
        HIPCK(launch_fill_u32(x->est.adam_m.as<uint32_t>(), 0, MLP_NPARAM, st));
        HIPCK(launch_fill_u32(x->est.adam_v.as<uint32_t>(), 0, MLP_NPARAM, st));
    }
    HIPCK(hipMemcpyAsync(x->est.grads.p, grad, MLP_NPARAM * 4, hipMemcpyDeviceToDevice, st));
    HIPCK(est_adam(x->est, lr, step, st));
    HIPCK(hipStreamSynchronize(st));
    return RKR_OK;
}

extern "C" rkr_status rkr_sketch(rkr_index *x, float *out) {
    g_err.clear();
    if (!x || !out) return fail(RKR_E_INVALID, "NULL argument");
    if (!x->est.has_sketch) return fail(RKR_E_STATE, "index built without a sketch");
    HIPCK(hipMemcpyAsync(out, x->est.sketch.p, (size_t)x->n * SKETCH_LEVELS * 4, hipMemcpyDeviceToDevice, x->st));
    HIPCK(hipStreamSynchronize(x->st));
    return RKR_OK;
}
