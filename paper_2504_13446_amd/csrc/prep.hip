// prep.hip -- index construction (norms, norm order, low-precision copies,
// error-bound coefficients), FP64 thresholds and the FP64 near-tie recheck.
#include "rkr_internal.h"
#include "kernels.h"
#include "tile_common.h"

namespace rkr {

// ---------------------------------------------------------------------------
// Input validation: bit 1 = non-finite value, bit 2 = |value| > 2^50.
// ---------------------------------------------------------------------------
__global__ void k_check_values(const void *X, int64_t count, int mk, int *flags) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t stride = (int64_t)gridDim.x * blockDim.x;
    int f = 0;
    for (; i < count; i += stride) {
        double v = master_elem(X, mk, i);
        if (!isfinite(v)) f |= 1;
        else if (fabs(v) > 0x1p50) f |= 2;
    }
    if (f) atomicOr(flags, f);
}

// ---------------------------------------------------------------------------
// Spec norm: sqrt of the sequential-fma sum of squares, one thread per row.
// ---------------------------------------------------------------------------
__global__ void k_spec_norm(const void *X, int64_t rows, int d, int mk, double *out) {
    int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= rows) return;
    double acc = 0.0;
    for (int k = 0; k < d; ++k) {
        double v = master_elem(X, mk, r * d + k);
        acc = fma(v, v, acc);
    }
    out[r] = sqrt(acc);
}

// ---------------------------------------------------------------------------
// Bitonic sort of (key, id) records: norm descending, id ascending.
// Padding records carry key = -inf and id = INT64_MAX so they sort last.
// ---------------------------------------------------------------------------
struct NormRec { double key; int64_t id; };

__device__ inline bool rec_before(const NormRec &a, const NormRec &b) {
    return (a.key > b.key) || (a.key == b.key && a.id < b.id);
}

__global__ void k_sort_init(const double *norms, int64_t m, int64_t mpow2, NormRec *recs) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= mpow2) return;
    recs[i] = (i < m) ? NormRec{norms[i], i} : NormRec{-__builtin_inf(), INT64_MAX};
}

__global__ void k_bitonic_global(NormRec *recs, int64_t mpow2, int64_t j, int64_t k) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= mpow2) return;
    int64_t l = i ^ j;
    if (l <= i) return;
    NormRec a = recs[i], b = recs[l];
    bool up = (i & k) == 0;
    bool swap = up ? rec_before(b, a) : rec_before(a, b);
    if (swap) { recs[i] = b; recs[l] = a; }
}

// All stages with j < 1024 inside LDS (2048-record tiles).
__global__ __launch_bounds__(1024) void k_bitonic_local(NormRec *recs, int64_t mpow2, int64_t k_lo,
                                                         int64_t k_hi) {
    __shared__ NormRec s[2048];
    int64_t base = (int64_t)blockIdx.x * 2048;
    int t = threadIdx.x;
    s[t] = recs[base + t];
    s[t + 1024] = recs[base + t + 1024];
    __syncthreads();
    for (int64_t k = k_lo; k <= k_hi; k <<= 1) {
        for (int64_t j = (k_lo == k_hi ? 1024 : k >> 1); j >= 1; j >>= 1) {
            if (j > 1024) continue;
            for (int r = 0; r < 2; ++r) {
                int i = t + r * 1024;
                int l = i ^ (int)j;
                if (l > i) {
                    int64_t gi = base + i;
                    bool up = (gi & k) == 0;
                    NormRec a = s[i], b = s[l];
                    bool swap = up ? rec_before(b, a) : rec_before(a, b);
                    if (swap) { s[i] = b; s[l] = a; }
                }
            }
            __syncthreads();
        }
    }
    recs[base + t] = s[t];
    recs[base + t + 1024] = s[t + 1024];
}

__global__ void k_sort_extract(const NormRec *recs, int64_t m, int32_t *order) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < m) order[i] = (int32_t)recs[i].id;
}

// Gather master rows into norm order.
__global__ void k_gather_rows(const void *src, const int32_t *order, int64_t rows, int d, int mk,
                              void *dst) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t total = rows * d;
    int64_t stride = (int64_t)gridDim.x * blockDim.x;
    size_t es = mk == MK_BF16 ? 2 : 4;
    for (; i < total; i += stride) {
        int64_t r = i / d, k = i - r * d;
        int64_t s = (int64_t)order[r] * d + k;
        if (es == 2) ((uint16_t *)dst)[i] = ((const uint16_t *)src)[s];
        else ((float *)dst)[i] = ((const float *)src)[s];
    }
}

// ---------------------------------------------------------------------------
// Low-precision copies.
// ---------------------------------------------------------------------------
__device__ inline uint16_t bf16_rne(float x) {
    uint32_t b = __float_as_uint(x);
    b = b + 0x7FFFu + ((b >> 16) & 1u);
    return (uint16_t)(b >> 16);
}

// FP8 e4m3 (finite-only variant: max 448) of |v| <= 448, round to nearest
// even; values below the smallest normal 2^-6 become 0.  Returns the byte
// and writes the decoded value.
__device__ inline uint8_t fp8_e4m3_rne(float v, float *dec) {
    float a = fabsf(v);
    uint8_t sign = v < 0.0f ? 0x80 : 0;
    if (!(a >= 0x1p-6f)) { *dec = 0.0f; return 0; }
    int e;
    frexpf(a, &e);              // a = f * 2^e, f in [0.5, 1)
    int E = e - 1;              // a in [2^E, 2^(E+1))
    float ulp = ldexpf(1.0f, E - 3);
    float qv = rintf(a / ulp) * ulp;   // a / ulp is exact (power of two); rintf ties to even
    if (qv >= ldexpf(1.0f, E + 1)) E += 1;
    if (qv > 448.0f) qv = 448.0f;
    int mant = (int)rintf(qv / ldexpf(1.0f, E - 3)) - 8;   // 0..7
    *dec = v < 0.0f ? -qv : qv;
    return (uint8_t)(sign | ((E + 7) << 3) | (mant & 7));
}

// One thread per row.  Writes the low-precision row, the exact residual norms
// (|x_hat|, |x - x_hat|, |x|), and (FP8) the row's scale exponent.
// Layout: row-major [rows][dpad] if frag == 0, else fragment order
//   [row / 32][k-step][lane][FB bytes] with lane = row % 32 + 32 * half.
// Split BF16 (split != 0): each value is hi = bf16(x) plus lo = bf16(x - hi),
// x_hat = hi + lo, and the row holds three copies of the d dimensions back to
// back, [hi | hi | lo] for split == 1 and [hi | lo | hi] for split == 2, so
// that one dot product of a split-1 row with a split-2 row over 3d terms is
// hi.hi + hi.lo + lo.hi.
__global__ void k_lowprec(const void *X, int64_t rows, int d, int mk, int sk, int dpad, int frag, int split,
                          uint8_t *out, double *norm3, int8_t *exps) {
    int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= rows) return;
    const int KS = frag_ks(sk), FB = frag_fb(sk), ES = elem_size(sk);
    const int nks = dpad / KS;
    int scale_e = 0;
    if (sk == SK_FP8) {
        double mx = 0.0;
        for (int k = 0; k < d; ++k) mx = fmax(mx, fabs(master_elem(X, mk, r * d + k)));
        if (mx > 0.0) {
            int e;
            frexp(mx / 448.0, &e);          // mx/448 in [2^(e-1), 2^e)
            scale_e = e;                    // mx * 2^-e <= 448 * 2^0 ... adjust below
            if (ldexp(mx, -(scale_e - 1)) <= 448.0) scale_e -= 1;
            if (scale_e < -100) scale_e = -100;
            if (scale_e > 100) scale_e = 100;
        }
        exps[r] = (int8_t)scale_e;
    }
    double nh = 0.0, nd = 0.0, nf = 0.0;
    for (int k = 0; k < dpad; ++k) {
        // position k holds dimension src of copy seg (seg 3 and above: padding)
        const int seg = split ? k / d : (k < d ? 0 : 3);
        const int src = split ? k - seg * d : k;
        double x = seg < 3 ? master_elem(X, mk, r * d + src) : 0.0;
        double xh;
        uint8_t bytes[4];
        if (sk == SK_BF16) {
            float xf = (fabs(x) < 0x1p-50) ? 0.0f : (float)x;
            uint16_t b = bf16_rne(xf);
            xh = (double)__uint_as_float((uint32_t)b << 16);
            if (split) {
                // xf - hi is exact in FP32 (the rounding error of hi)
                const uint16_t bl = bf16_rne((float)((double)xf - xh));
                const double xl = (double)__uint_as_float((uint32_t)bl << 16);
                if (seg == (split == 1 ? 2 : 1)) b = bl;
                xh += xl;            // x_hat = hi + lo, exact in FP64
            }
            bytes[0] = b & 0xFF; bytes[1] = b >> 8;
        } else if (sk == SK_F32) {
            float xf = (fabs(x) < 0x1p-50) ? 0.0f : (float)x;
            xh = (double)xf;
            uint32_t b = __float_as_uint(xf);
            bytes[0] = b & 0xFF; bytes[1] = (b >> 8) & 0xFF; bytes[2] = (b >> 16) & 0xFF; bytes[3] = b >> 24;
        } else {
            float dec;
            uint8_t b = fp8_e4m3_rne((float)ldexp(x, -scale_e), &dec);
            xh = ldexp((double)dec, scale_e);
            bytes[0] = b;
        }
        if (seg == 0) {          // each dimension once
            double dl = x - xh;  // exact: both are FP32-representable, same scale
            nh = fma(xh, xh, nh);
            nd = fma(dl, dl, nd);
            nf = fma(x, x, nf);
        }
        int64_t off;
        if (!frag) {
            off = (r * dpad + k) * ES;
        } else {
            int s = k / KS, kk = k % KS;
            int half = kk / (KS / 2), e = kk % (KS / 2);
            int64_t blk = r / 32;
            int lane = (int)(r % 32) + 32 * half;
            off = ((blk * nks + s) * 64 + lane) * (int64_t)FB + e * ES;
        }
        for (int b = 0; b < ES; ++b) out[off + b] = bytes[b];
    }
    const double infl = 1.0 + 0x1p-40;
    norm3[3 * r + 0] = sqrt(nh) * infl;
    norm3[3 * r + 1] = sqrt(nd) * infl;
    norm3[3 * r + 2] = sqrt(nf) * infl;
}

// Error-bound coefficients per 32-item block (items sorted by norm):
//   a = g32 * X + Y,  b = X + Y,  c = (g64 + cz) * Z,  abs
// with X = max |p_hat|, Y = max |delta p|, Z = max |p| over the block, so that
//   |score - s64(u,p)| <= |u_hat| a + |delta u| b + |u| c + abs.
// cz is the relative bound of a product the score leaves out (split BF16:
// lo.lo), 0 otherwise.
__global__ void k_block_coef(const double *pnorm3, int64_t m, int64_t nblk, double g32, double g64,
                             double cz, double eabs, double *coef) {
    int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= nblk) return;
    double X = 0, Y = 0, Z = 0;
    for (int64_t i = b * 32; i < b * 32 + 32 && i < m; ++i) {
        X = fmax(X, pnorm3[3 * i + 0]);
        Y = fmax(Y, pnorm3[3 * i + 1]);
        Z = fmax(Z, pnorm3[3 * i + 2]);
    }
    const double infl = 1.0 + 0x1p-40;
    coef[4 * b + 0] = (g32 * X + Y) * infl;
    coef[4 * b + 1] = (X + Y) * infl;
    coef[4 * b + 2] = (g64 + cz) * Z * infl;
    coef[4 * b + 3] = eabs;
}

// Per step of 64 items in norm order: an upper bound of |p| over the step's
// items and every later one, the spec norm of the step's first item inflated
// by 1 + 2^-40 (the norms are sorted, non-increasing, and the FP64 sum of
// squares and its square root are within 2^-41 of |p|^2 and |p| for d <= 4096).
__global__ void k_step_znorm(const double *pn, const int32_t *order, int64_t m, int64_t nsteps, double *out) {
    int64_t st = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (st >= nsteps) return;
    const int64_t i = st * 64;
    out[st] = i < m ? pn[order[i]] * (1.0 + 0x1p-40) : 0.0;
}

// Per step of nib consecutive blocks: the maxima of the blocks' coefficients
// (a step's error bound covers all of its items).
__global__ void k_step_coef(const double *coef, int64_t nblk, int nib, int64_t nsteps, double *out) {
    int64_t st = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (st >= nsteps) return;
    double c[4] = {0.0, 0.0, 0.0, 0.0};
    for (int ib = 0; ib < nib; ++ib) {
        const int64_t b = st * nib + ib;
        if (b < nblk)
            for (int k = 0; k < 4; ++k) c[k] = fmax(c[k], coef[4 * b + k]);
    }
    for (int k = 0; k < 4; ++k) out[4 * st + k] = c[k];
}

// ---------------------------------------------------------------------------
// FP64 thresholds t(u,q) = spec dot (the FP32 values bracketing it are
// derived where the count kernel's entries are filled).
// ---------------------------------------------------------------------------
__global__ void k_thresh(const int32_t *pair_u, const int32_t *pair_q, int64_t npairs,
                         const void *Um, const void *Qm, int d, int mk, double *t64) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= npairs) return;
    const int64_t u = pair_u[i], q = pair_q[i];
    double acc = 0.0;
    for (int k = 0; k < d; ++k)
        acc = fma(master_elem(Um, mk, u * d + k), master_elem(Qm, mk, q * d + k), acc);
    t64[i] = acc;
}

// Dense thresholds, register-tiled: a block computes 64 users x 64 queries
// (4 x 4 per thread) with both operands staged in LDS as doubles, 32
// dimensions at a time; every dot still runs its fma chain in dimension
// order, so the values equal the per-pair kernel's.  pid = u * nq + q.
// With keys, each pair's default seed key is written too (query-major, as
// the seed-key kernel writes it: (order key of fl32(-t / |u|)) << 32 | u).
__global__ __launch_bounds__(256) void k_thresh_dense(const void *Um, int64_t n, const void *Qm, int nq, int d, int mk,
                                                      double *t64, const double *unorm3, uint64_t *keys) {
    // rows of 66 doubles: 16-byte aligned, so each adjacent operand pair of a
    // thread is one 16-byte LDS read
    __shared__ __attribute__((aligned(16))) double su[32][66];
    __shared__ __attribute__((aligned(16))) double sq[32][66];
    const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
    const int64_t ub = (int64_t)blockIdx.y * 64;
    const int qb = blockIdx.x * 64;
    double acc[4][4];
    for (int a = 0; a < 4; ++a)
        for (int b = 0; b < 4; ++b) acc[a][b] = 0.0;
    // BF16 rows of d % 8 == 0 at 16-byte aligned bases: a thread stages eight
    // consecutive elements of one user row and one query row per chunk from
    // one 16-byte load each
    const bool wide = mk == MK_BF16 && (d & 7) == 0 && (((uintptr_t)Um | (uintptr_t)Qm) & 15) == 0;
    for (int k0 = 0; k0 < d; k0 += 32) {
        if (wide && k0 + 32 <= d) {
            const int r = threadIdx.x >> 2, g = threadIdx.x & 3;
            const int64_t u = ub + r;
            const int q = qb + r;
            const uint4 zero = make_uint4(0u, 0u, 0u, 0u);
            const uint4 wu = u < n ? *(const uint4 *)((const uint16_t *)Um + u * d + k0 + g * 8) : zero;
            const uint4 wq = q < nq ? *(const uint4 *)((const uint16_t *)Qm + (int64_t)q * d + k0 + g * 8) : zero;
            const uint32_t au[4] = {wu.x, wu.y, wu.z, wu.w}, aq[4] = {wq.x, wq.y, wq.z, wq.w};
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                // element 2j is the low half of word j, element 2j + 1 the high half
                su[g * 8 + 2 * j][r] = (double)__uint_as_float(au[j] << 16);
                su[g * 8 + 2 * j + 1][r] = (double)__uint_as_float(au[j] & 0xFFFF0000u);
                sq[g * 8 + 2 * j][r] = (double)__uint_as_float(aq[j] << 16);
                sq[g * 8 + 2 * j + 1][r] = (double)__uint_as_float(aq[j] & 0xFFFF0000u);
            }
        } else {
            for (int e = threadIdx.x; e < 64 * 32; e += 256) {
                const int r = e >> 5, kk = e & 31;
                const int64_t u = ub + r;
                const int q = qb + r;
                su[kk][r] = (k0 + kk < d && u < n) ? master_elem(Um, mk, u * d + k0 + kk) : 0.0;
                sq[kk][r] = (k0 + kk < d && q < nq) ? master_elem(Qm, mk, (int64_t)q * d + k0 + kk) : 0.0;
            }
        }
        __syncthreads();
        const int kmax = min(32, d - k0);
        for (int kk = 0; kk < kmax; ++kk) {
            // a thread's users (queries) are tile columns 2t, 2t + 1, 32 + 2t,
            // 33 + 2t: sixteen lanes read 256 contiguous bytes per 16-byte
            // read, one per LDS bank
            const double2 a01 = *(const double2 *)&su[kk][ty * 2], a23 = *(const double2 *)&su[kk][32 + ty * 2];
            const double2 b01 = *(const double2 *)&sq[kk][tx * 2], b23 = *(const double2 *)&sq[kk][32 + tx * 2];
            const double a[4] = {a01.x, a01.y, a23.x, a23.y}, b[4] = {b01.x, b01.y, b23.x, b23.y};
            for (int x = 0; x < 4; ++x)
                for (int y = 0; y < 4; ++y) acc[x][y] = fma(a[x], b[y], acc[x][y]);
        }
        __syncthreads();
    }
    // tile columns of x (users) and y (queries): 0, 1 -> 2t, 2t + 1; 2, 3 -> 32 + 2t, 33 + 2t
    const int64_t ua = ub + ty * 2, uc = ub + 32 + ty * 2;
    const int qa = qb + tx * 2, qc = qb + 32 + tx * 2;
    if (uc + 1 < n && qc + 1 < nq && ((n | nq) & 1) == 0) {
        // full tile, even sizes: a thread's queries come in adjacent pairs in
        // t64 and its users in adjacent pairs in the query-major keys, so
        // both go out as 16-byte stores (the indices below are even)
        for (int x = 0; x < 4; ++x) {
            const int64_t u = (x < 2 ? ua : uc) + (x & 1);
            *(double2 *)&t64[u * nq + qa] = make_double2(acc[x][0], acc[x][1]);
            *(double2 *)&t64[u * nq + qc] = make_double2(acc[x][2], acc[x][3]);
        }
        if (keys) {
            uint64_t key[4][4];
            for (int x = 0; x < 4; ++x) {
                const int64_t u = (x < 2 ? ua : uc) + (x & 1);
                const double nu = unorm3[3 * u + 2];
                for (int y = 0; y < 4; ++y) {
                    const float h = nu > 0.0 ? (float)(-acc[x][y] / nu) : 0.0f;
                    key[y][x] = ((uint64_t)f32_order_key(h) << 32) | (uint32_t)u;
                }
            }
            for (int y = 0; y < 4; ++y) {
                const int64_t q = (y < 2 ? qa : qc) + (y & 1);
                *(ulonglong2 *)&keys[q * n + ua] = make_ulonglong2(key[y][0], key[y][1]);
                *(ulonglong2 *)&keys[q * n + uc] = make_ulonglong2(key[y][2], key[y][3]);
            }
        }
        return;
    }
    for (int x = 0; x < 4; ++x) {
        const int64_t u = (x < 2 ? ua : uc) + (x & 1);
        if (u >= n) continue;
        for (int y = 0; y < 4; ++y) {
            const int q = (y < 2 ? qa : qc) + (y & 1);
            if (q >= nq) continue;
            t64[u * nq + q] = acc[x][y];
            if (keys) {
                const double nu = unorm3[3 * u + 2];
                const float h = nu > 0.0 ? (float)(-acc[x][y] / nu) : 0.0f;
                keys[(int64_t)q * n + u] = ((uint64_t)f32_order_key(h) << 32) | (uint32_t)u;
            }
        }
    }
}

// ---------------------------------------------------------------------------
// FP64 recheck of near ties: one thread per emitted (pair, item) record.
// The item id is in sorted order; its master row sits in Pm_sorted.
// Bit 31 of the item field carries the plain FP32 verdict (score > fl32(t)).
// ---------------------------------------------------------------------------
// The spec inner product of master rows a and b: one FP64 fma chain in
// dimension order.  Rows are read 16 bytes at a time when both are 16-byte
// aligned; the chain (and so the result) is the same either way.
__device__ inline double spec_dot_rows(const void *A, int64_t ra, const void *B, int64_t rb, int d, int mk) {
    double acc = 0.0;
    if (mk == MK_BF16) {
        const uint16_t *a = (const uint16_t *)A + ra * d, *b = (const uint16_t *)B + rb * d;
        int k = 0;
        if ((((uintptr_t)a | (uintptr_t)b) & 15) == 0) {
            for (; k + 8 <= d; k += 8) {
                const uint4 va = *(const uint4 *)(a + k), vb = *(const uint4 *)(b + k);
                const uint32_t wa[4] = {va.x, va.y, va.z, va.w}, wb[4] = {vb.x, vb.y, vb.z, vb.w};
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    // element 2j is the low half of word j, element 2j + 1 the high half
                    acc = fma((double)__uint_as_float(wa[j] << 16), (double)__uint_as_float(wb[j] << 16), acc);
                    acc = fma((double)__uint_as_float(wa[j] & 0xFFFF0000u),
                              (double)__uint_as_float(wb[j] & 0xFFFF0000u), acc);
                }
            }
        }
        for (; k < d; ++k)
            acc = fma((double)__uint_as_float((uint32_t)a[k] << 16), (double)__uint_as_float((uint32_t)b[k] << 16),
                      acc);
        return acc;
    }
    const float *a = (const float *)A + ra * d, *b = (const float *)B + rb * d;
    int k = 0;
    if ((((uintptr_t)a | (uintptr_t)b) & 15) == 0) {
        for (; k + 4 <= d; k += 4) {
            const float4 va = *(const float4 *)(a + k), vb = *(const float4 *)(b + k);
            acc = fma((double)va.x, (double)vb.x, acc);
            acc = fma((double)va.y, (double)vb.y, acc);
            acc = fma((double)va.z, (double)vb.z, acc);
            acc = fma((double)va.w, (double)vb.w, acc);
        }
    }
    for (; k < d; ++k) acc = fma((double)a[k], (double)b[k], acc);
    return acc;
}

// A grid of at most 2^16 workgroups strides over the records (a launch's
// work-items must stay below 2^32; wide bands can emit more records).
__global__ void k_recheck(const int2 *rec, int64_t nrec, const int32_t *pair_u, const double *t64,
                          const void *Um, const void *Pm, int d, int mk, uint32_t *cnt,
                          unsigned long long *flips) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    const int64_t i0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    // every wave runs the same number of iterations (the ballot needs them all)
    const int64_t iters = (nrec + stride - 1) / stride;
    unsigned long long nflip = 0;
    for (int64_t it = 0; it < iters; ++it) {
        const int64_t i = i0 + it * stride;
        bool flip = false;
        if (i < nrec) {
            const int2 r = rec[i];
            const int pid = r.x;
            const int64_t item = r.y & 0x7FFFFFFF;
            const bool plain = (r.y >> 31) & 1;
            const int64_t u = pair_u[pid];
            const double acc = spec_dot_rows(Um, u, Pm, item, d, mk);
            const bool above = acc > t64[pid];
            if (above) atomicAdd(&cnt[pid], 1u);
            flip = above != plain;
        }
        nflip += (unsigned long long)__popcll(__ballot(flip));
    }
    if ((threadIdx.x & 63) == 0 && nflip) atomicAdd(flips, nflip);
}

// The same with the record count read from device memory (graph replays):
// a fixed grid strides over min(*count, cap) records.
__global__ void k_recheck_dev(const int2 *rec, const unsigned long long *count, int64_t cap, const int32_t *pair_u,
                              const double *t64, const void *Um, const void *Pm, int d, int mk, uint32_t *cnt,
                              unsigned long long *flips) {
    const int64_t nrec = (int64_t)min((unsigned long long)cap, *count);
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    uint32_t nflip = 0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nrec; i += stride) {
        const int2 r = rec[i];
        const int pid = r.x;
        const int64_t item = r.y & 0x7FFFFFFF;
        const bool plain = (r.y >> 31) & 1;
        const int64_t u = pair_u[pid];
        const double acc = spec_dot_rows(Um, u, Pm, item, d, mk);
        const bool above = acc > t64[pid];
        if (above) atomicAdd(&cnt[pid], 1u);
        nflip += (above != plain) ? 1u : 0u;
    }
    if (nflip) atomicAdd(flips, (unsigned long long)nflip);
}

// ---------------------------------------------------------------------------
// Bounded thresholds of a dense batch, for the rank-table filter and the seed
// order (the FP64 thresholds are then computed only for the pairs that are
// counted).  t^ = u^.q^ on the matrix cores (BF16 copies, products exact,
// FP32 sums); its distance to the FP64 threshold s64(u, q) is at most
//   gamma32 |u^||q^| + |du||q^| + |u^||dq| + |du||dq| + gamma64 |u||q|
//   = a_u X_q + b_u Y_q + c_u Z_q
// with a = |x^|, b = |x - x^|, c = |x| and X_q = gamma32 a_q + b_q, Y_q =
// a_q + b_q, Z_q = gamma64 c_q, all rounded up (the same terms as the error
// bound of the scores, with q in place of p).  Out: t_up >= t^ + that bound
// (FP32, rounded up; user-major [u * nq + q]) and the default seed keys
// (query-major [q * n + u]): the 32-bit order keys of -t^ / |u|, the user
// being the position in the query's row.
// ---------------------------------------------------------------------------
__global__ void k_query_xyz(const double *qnorm3, int nq, double g32, double g64, float4 *out) {
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= nq) return;
    const double a = qnorm3[3 * q], b = qnorm3[3 * q + 1], c = qnorm3[3 * q + 2];
    const double sl = 1.0 + 0x1p-40;   // the FP64 products' own rounding
    out[q] = make_float4(f32_round_up((g32 * a + b) * sl), f32_round_up((a + b) * sl), f32_round_up(g64 * c * sl),
                         0.0f);
}

// One workgroup of 8 waves per query tile of 256 and a stride of 32-user
// blocks; wave w holds queries 32w .. 32w + 31 of the tile as register-
// stationary A operands, the block's users are the B operands (one
// 32x32x16 MFMA per k-step).  A lane's outputs are one user (its column) and
// 16 queries (rows): keys go out along the users (128 contiguous bytes per
// query row); t_up goes through LDS so that each user's row of queries is
// written contiguously.
template <int NKS>
__global__ __launch_bounds__(512) void k_thresh_approx(const uint8_t *ulp, int64_t n, int dpad, const double *unorm3,
                                                       const uint8_t *qlp, int nq, const float4 *qxyz, float *t_up,
                                                       uint32_t *keys) {
    using FT = typename FragT<SK_BF16>::T;
    constexpr int KS = 16;
    __shared__ float4 sq[256];
    __shared__ float stile[32][257];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, l32 = lane & 31, half = lane >> 5;
    const int q0 = blockIdx.y * 256;
    const int nqt = min(256, nq - q0);
    FT afr[NKS];
    {
        const int q = q0 + wave * 32 + l32;
#pragma unroll
        for (int s = 0; s < NKS; ++s) {
            FT v{};
            if (q < nq) v = *(const FT *)(qlp + ((int64_t)q * dpad + s * KS + half * 8) * 2);
            afr[s] = v;
        }
    }
    if (threadIdx.x < 256) sq[threadIdx.x] = threadIdx.x < nqt ? qxyz[q0 + threadIdx.x] : make_float4(0, 0, 0, 0);
    __syncthreads();
    const int64_t nblk = (n + 31) / 32;
    for (int64_t bk = blockIdx.x; bk < nblk; bk += gridDim.x) {
        const int64_t ub = bk * 32;
        const int64_t u = ub + l32;
        f32x16 acc{};
        const uint8_t *urow = ulp + ((u < n ? u : 0) * dpad + half * 8) * 2;
#pragma unroll
        for (int s = 0; s < NKS; ++s) {
            FT bf{};
            if (u < n) bf = *(const FT *)(urow + s * KS * 2);
            acc = mfma_step<SK_BF16>(acc, afr[s], bf, 127, 127);
        }
        float au = 0.0f, bu = 0.0f, cu = 0.0f, inv = 0.0f;
        if (u < n) {
            au = f32_round_up(unorm3[3 * u]);
            bu = f32_round_up(unorm3[3 * u + 1]);
            cu = f32_round_up(unorm3[3 * u + 2]);
            const double nu = unorm3[3 * u + 2];
            inv = nu > 0.0 ? (float)(1.0 / nu) : 0.0f;
        }
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            const int ql = wave * 32 + 8 * (r >> 2) + 4 * half + (r & 3);   // query within the tile
            const float4 z = sq[ql];
            const float th = acc[r];
            const float dd = __builtin_fmaf(au, z.x, __builtin_fmaf(bu, z.y, cu * z.z));
            const float sm = th + __builtin_fmaf(dd, 0x1p-20f, dd);
            stile[l32][ql] = sm + __builtin_fmaf(__builtin_fabsf(sm), 0x1p-22f, 0x1p-126f);
            if (u < n && ql < nqt)
                keys[(int64_t)(q0 + ql) * n + u] = f32_order_key(-th * inv);   // (the user is the position)
        }
        __syncthreads();
        for (int idx = threadIdx.x; idx < 32 * 256; idx += 512) {
            const int i = idx >> 8, j = idx & 255;
            if (j < nqt && ub + i < n) t_up[(ub + i) * nq + q0 + j] = stile[i][j];
        }
        __syncthreads();
    }
}

// FP64 thresholds of the listed pairs only (sequential fma, as in k_thresh).
__global__ void k_thresh_list(const int32_t *pids, int64_t N, const int32_t *pair_u, const int32_t *pair_q,
                              const void *Um, const void *Qm, int d, int mk, double *t64) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    const int32_t p = pids[i];
    t64[p] = spec_dot_rows(Um, pair_u[p], Qm, pair_q[p], d, mk);
}

// The recheck with the rows staged through LDS: a workgroup takes 256
// records at a time and walks the dimension in chunks of RC_K elements; for
// each chunk the records' item-row segments and their distinct user-row
// segments are loaded into LDS with coalesced 16-byte loads (eight lanes per
// 128-byte segment of FP32, four of BF16), then each thread extends its own
// record's FP64 chain over the chunk (k ascending, the same sequence of fma as
// spec_dot_rows, so the same double).  A pass emits the near ties of one user
// together, so a run of records sharing a user loads its row once.
constexpr int RC_REC = 256, RC_K = 32;
template <int MK>
__device__ inline void rc_load_rows(const void *X, const int64_t *rows, int nrows, int d, int k0, int kn,
                                    float (*dst)[RC_K + 1], int tid) {
    constexpr int EPL = MK == MK_BF16 ? 8 : 4;   // elements per 16-byte lane load
    constexpr int LPR = RC_K / EPL;              // lanes per row segment
    for (int idx = tid; idx < nrows * LPR; idx += 256) {
        const int row = idx / LPR, c = (idx % LPR) * EPL;
        const int64_t rr = rows[row];
        float *o = &dst[row][c];
        if constexpr (MK == MK_BF16) {
            const uint16_t *src = (const uint16_t *)X + rr * d + k0 + c;
            if (rr >= 0 && c + 8 <= kn && ((((uintptr_t)src) & 15) == 0)) {
                const uint4 v = *(const uint4 *)src;
                const uint32_t w[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    o[2 * e] = __uint_as_float(w[e] << 16);
                    o[2 * e + 1] = __uint_as_float(w[e] & 0xFFFF0000u);
                }
            } else {
#pragma unroll
                for (int e = 0; e < 8; ++e) o[e] = (rr >= 0 && c + e < kn) ? __uint_as_float((uint32_t)src[e] << 16) : 0.0f;
            }
        } else {
            const float *src = (const float *)X + rr * d + k0 + c;
            if (rr >= 0 && c + 4 <= kn && ((((uintptr_t)src) & 15) == 0)) {
                const float4 v = *(const float4 *)src;
                o[0] = v.x;
                o[1] = v.y;
                o[2] = v.z;
                o[3] = v.w;
            } else {
#pragma unroll
                for (int e = 0; e < 4; ++e) o[e] = (rr >= 0 && c + e < kn) ? src[e] : 0.0f;
            }
        }
    }
}
template <int MK>
__global__ __launch_bounds__(256) void k_recheck_coop(const int2 *rec, const unsigned long long *count, int64_t cap,
                                                      const int32_t *pair_u, const double *t64, const void *Um,
                                                      const void *Pm, int d, uint32_t *cnt,
                                                      unsigned long long *flips) {
    __shared__ float su[RC_REC][RC_K + 1], sp[RC_REC][RC_K + 1];
    __shared__ int64_t ru[RC_REC], rp[RC_REC], uu[RC_REC];
    __shared__ int wsum[4];
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int64_t nrec = (int64_t)min((unsigned long long)cap, *count);
    const int64_t nblk = (nrec + RC_REC - 1) / RC_REC;
    unsigned long long nflip = 0;
    for (int64_t b = blockIdx.x; b < nblk; b += gridDim.x) {
        const int64_t i = b * RC_REC + tid;
        int pid = 0;
        bool plain = false;
        const bool real = i < nrec;
        if (real) {
            const int2 r = rec[i];
            pid = r.x;
            plain = (r.y >> 31) & 1;
            ru[tid] = pair_u[pid];
            rp[tid] = r.y & 0x7FFFFFFF;
        } else {
            ru[tid] = -1;
            rp[tid] = -1;
        }
        __syncthreads();
        // distinct user rows: a record opens a slot when its user differs
        // from the previous record's (real records are a prefix of the block)
        const bool open = real && (tid == 0 || ru[tid] != ru[tid - 1]);
        const uint64_t bal = __ballot(open);
        const uint64_t upto = lane == 63 ? ~0ull : ((2ull << lane) - 1);
        if (lane == 0) wsum[wv] = __popcll(bal);
        __syncthreads();
        int slot = __popcll(bal & upto) - 1;
        for (int k = 0; k < wv; ++k) slot += wsum[k];
        const int nu = wsum[0] + wsum[1] + wsum[2] + wsum[3];
        if (open) uu[slot] = ru[tid];
        __syncthreads();
        double acc = 0.0;
        for (int k0 = 0; k0 < d; k0 += RC_K) {
            const int kn = min(RC_K, d - k0);
            rc_load_rows<MK>(Pm, rp, RC_REC, d, k0, kn, sp, tid);
            rc_load_rows<MK>(Um, uu, nu, d, k0, kn, su, tid);
            __syncthreads();
            if (real)
                for (int k = 0; k < kn; ++k) acc = fma((double)su[slot][k], (double)sp[tid][k], acc);
            __syncthreads();
        }
        bool flip = false;
        if (real) {
            const bool above = acc > t64[pid];
            if (above) atomicAdd(&cnt[pid], 1u);
            flip = above != plain;
        }
        nflip += (unsigned long long)__popcll(__ballot(flip));
    }
    if ((threadIdx.x & 63) == 0 && nflip) atomicAdd(flips, nflip);
}

// ---------------------------------------------------------------------------
// host launchers
// ---------------------------------------------------------------------------
static inline unsigned nblocks(int64_t n, int bs) { return (unsigned)((n + bs - 1) / bs); }

hipError_t launch_check_values(const void *X, int64_t count, int mk, int *flags, hipStream_t st) {
    if (count <= 0) return hipSuccess;
    int64_t nb = (count + 255) / 256;
    if (nb > 65536) nb = 65536;
    hipLaunchKernelGGL(k_check_values, dim3((unsigned)nb), dim3(256), 0, st, X, count, mk, flags);
    return hipGetLastError();
}

hipError_t launch_spec_norm(const void *X, int64_t rows, int d, int mk, double *out, hipStream_t st) {
    if (rows <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_spec_norm, dim3(nblocks(rows, 256)), dim3(256), 0, st, X, rows, d, mk, out);
    return hipGetLastError();
}

hipError_t launch_norm_sort(const double *norms, int64_t m, void *scratch, int32_t *order,
                            hipStream_t st) {
    if (m <= 0) return hipSuccess;
    int64_t mp = 2048;
    while (mp < m) mp <<= 1;
    NormRec *recs = (NormRec *)scratch;
    hipLaunchKernelGGL(k_sort_init, dim3(nblocks(mp, 256)), dim3(256), 0, st, norms, m, mp, recs);
    // stages k = 2 .. 2048 entirely in LDS
    hipLaunchKernelGGL(k_bitonic_local, dim3((unsigned)(mp / 2048)), dim3(1024), 0, st, recs, mp,
                       (int64_t)2, (int64_t)2048);
    for (int64_t k = 4096; k <= mp; k <<= 1) {
        for (int64_t j = k >> 1; j > 1024; j >>= 1)
            hipLaunchKernelGGL(k_bitonic_global, dim3(nblocks(mp, 256)), dim3(256), 0, st, recs, mp, j, k);
        hipLaunchKernelGGL(k_bitonic_local, dim3((unsigned)(mp / 2048)), dim3(1024), 0, st, recs, mp, k, k);
    }
    hipLaunchKernelGGL(k_sort_extract, dim3(nblocks(m, 256)), dim3(256), 0, st, recs, m, order);
    return hipGetLastError();
}

size_t norm_sort_scratch_bytes(int64_t m) {
    int64_t mp = 2048;
    while (mp < m) mp <<= 1;
    return (size_t)mp * sizeof(NormRec);
}

hipError_t launch_gather_rows(const void *src, const int32_t *order, int64_t rows, int d, int mk,
                              void *dst, hipStream_t st) {
    int64_t total = rows * d;
    if (total <= 0) return hipSuccess;
    int64_t nb = (total + 255) / 256;
    if (nb > 262144) nb = 262144;
    hipLaunchKernelGGL(k_gather_rows, dim3((unsigned)nb), dim3(256), 0, st, src, order, rows, d, mk, dst);
    return hipGetLastError();
}

hipError_t launch_lowprec(const void *X, int64_t rows, int d, int mk, int sk, int dpad, int frag, int split,
                          uint8_t *out, double *norm3, int8_t *exps, hipStream_t st) {
    if (rows <= 0) return hipSuccess;
    if (split && (sk != SK_BF16 || 3 * d > dpad)) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_lowprec, dim3(nblocks(rows, 128)), dim3(128), 0, st, X, rows, d, mk, sk, dpad,
                       frag, split, out, norm3, exps);
    return hipGetLastError();
}

hipError_t launch_block_coef(const double *pnorm3, int64_t m, int64_t nblk, double g32, double g64,
                             double cz, double eabs, double *coef, hipStream_t st) {
    if (nblk <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_block_coef, dim3(nblocks(nblk, 256)), dim3(256), 0, st, pnorm3, m, nblk, g32,
                       g64, cz, eabs, coef);
    return hipGetLastError();
}

hipError_t launch_step_znorm(const double *pn, const int32_t *order, int64_t m, int64_t nsteps, double *out,
                             hipStream_t st) {
    if (nsteps <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_step_znorm, dim3(nblocks(nsteps, 256)), dim3(256), 0, st, pn, order, m, nsteps, out);
    return hipGetLastError();
}

hipError_t launch_step_coef(const double *coef, int64_t nblk, int nib, int64_t nsteps, double *out,
                            hipStream_t st) {
    if (nsteps <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_step_coef, dim3(nblocks(nsteps, 256)), dim3(256), 0, st, coef, nblk, nib, nsteps, out);
    return hipGetLastError();
}

hipError_t launch_thresh(const int32_t *pair_u, const int32_t *pair_q, int64_t npairs, const void *Um,
                         const void *Qm, int d, int mk, double *t64, hipStream_t st) {
    if (npairs <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_thresh, dim3(nblocks(npairs, 256)), dim3(256), 0, st, pair_u, pair_q, npairs,
                       Um, Qm, d, mk, t64);
    return hipGetLastError();
}

hipError_t launch_thresh_dense(const void *Um, int64_t n, const void *Qm, int nq, int d, int mk, double *t64,
                               hipStream_t st, const double *unorm3, uint64_t *keys) {
    if (n <= 0 || nq <= 0) return hipSuccess;
    dim3 g((unsigned)((nq + 63) / 64), (unsigned)((n + 63) / 64));
    hipLaunchKernelGGL(k_thresh_dense, g, dim3(256), 0, st, Um, n, Qm, nq, d, mk, t64, unorm3, keys);
    return hipGetLastError();
}

static bool env_flag_rc(const char *name) {
    const char *v = getenv(name);
    return v && v[0] == '1' && v[1] == 0;
}

hipError_t launch_recheck_dev(const int2 *rec, const unsigned long long *count, int64_t cap, const int32_t *pair_u,
                              const double *t64, const void *Um, const void *Pm, int d, int mk, uint32_t *cnt,
                              unsigned long long *flips, hipStream_t st) {
    // FP32 master rows of d >= 192 (1.2 KB at d = 300) through LDS in full
    // lines; BF16 rows and short FP32 rows (d = 100: 35.6 against 28.3 ms
    // for the single-query workload) measured faster one thread per record
    if (mk == MK_BF16 || (d < 192 && !env_flag_rc("RKR_RECHECK_COOP")) || env_flag_rc("RKR_RECHECK_THREAD"))
        hipLaunchKernelGGL(k_recheck_dev, dim3(2048), dim3(256), 0, st, rec, count, cap, pair_u, t64, Um, Pm, d, mk,
                           cnt, flips);
    else
        hipLaunchKernelGGL(k_recheck_coop<MK_F32>, dim3(1024), dim3(256), 0, st, rec, count, cap, pair_u, t64, Um, Pm,
                           d, cnt, flips);
    return hipGetLastError();
}

hipError_t launch_recheck(const int2 *rec, int64_t nrec, const int32_t *pair_u, const double *t64,
                          const void *Um, const void *Pm, int d, int mk, uint32_t *cnt,
                          unsigned long long *flips, hipStream_t st) {
    if (nrec <= 0) return hipSuccess;
    const unsigned nb = nblocks(std::min<int64_t>(nrec, (int64_t)65536 * 256), 256);
    hipLaunchKernelGGL(k_recheck, dim3(nb), dim3(256), 0, st, rec, nrec, pair_u, t64, Um, Pm, d, mk, cnt, flips);
    return hipGetLastError();
}

hipError_t launch_query_xyz(const double *qnorm3, int nq, double g32, double g64, float4 *out, hipStream_t st) {
    if (nq <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_query_xyz, dim3(nblocks(nq, 256)), dim3(256), 0, st, qnorm3, nq, g32, g64, out);
    return hipGetLastError();
}

hipError_t launch_thresh_approx(const uint8_t *ulp, int64_t n, int dpad, int nks, const double *unorm3,
                                const uint8_t *qlp, int nq, const float4 *qxyz, float *t_up, uint32_t *keys,
                                int num_cus, hipStream_t st) {
    if (n <= 0 || nq <= 0) return hipSuccess;
    const int64_t nblk = (n + 31) / 32;
    const dim3 g((unsigned)std::min<int64_t>(nblk, (int64_t)num_cus * 4), (unsigned)((nq + 255) / 256));
    switch (nks) {
    case 4: hipLaunchKernelGGL(k_thresh_approx<4>, g, dim3(512), 0, st, ulp, n, dpad, unorm3, qlp, nq, qxyz, t_up, keys); break;
    case 8: hipLaunchKernelGGL(k_thresh_approx<8>, g, dim3(512), 0, st, ulp, n, dpad, unorm3, qlp, nq, qxyz, t_up, keys); break;
    case 13: hipLaunchKernelGGL(k_thresh_approx<13>, g, dim3(512), 0, st, ulp, n, dpad, unorm3, qlp, nq, qxyz, t_up, keys); break;
    case 20: hipLaunchKernelGGL(k_thresh_approx<20>, g, dim3(512), 0, st, ulp, n, dpad, unorm3, qlp, nq, qxyz, t_up, keys); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_thresh_list(const int32_t *pids, int64_t N, const int32_t *pair_u, const int32_t *pair_q,
                              const void *Um, const void *Qm, int d, int mk, double *t64, hipStream_t st) {
    if (N <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_thresh_list, dim3(nblocks(N, 256)), dim3(256), 0, st, pids, N, pair_u, pair_q, Um, Qm, d, mk,
                       t64);
    return hipGetLastError();
}

}  // namespace rkr
