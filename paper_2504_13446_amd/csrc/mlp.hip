// mlp.hip -- the learned rank estimator.
//
// Sketch.  For each user u: the spec scores s64(u,p) against S items taken
// from the middle of S equal buckets of the norm-sorted item set (the paper's
// norm-stratified sampling, Sec. 4.2 step 3, with one sample per bucket),
// sorted descending, read at 16 positions spaced geometrically from 1 to S,
// divided by the spec norm of u.  FP64 throughout, so the values equal the
// reference's to the bit (then rounded to FP32).
//
// Network.  x = [t(u,q)/|u|, |u|, sketch(u)] (18) -> 64 -> 64 -> 1 with ReLU,
// predicting ln r(q,u,P); it plays the part of the paper's rank table plus
// interpolation (Sec. 4.1, Sec. 4.3 step 3).  Training runs in FP32 with
// hand-written forward/backward kernels (deterministic two-stage gradient
// reduction) and Adam; inference runs on the matrix cores in BF16 with FP32
// accumulation, chaining the layers in registers.
#include "mlp.h"

namespace rkr {

static inline unsigned nblocks(int64_t n, int bs) { return (unsigned)((n + bs - 1) / bs); }

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef short s16x8 __attribute__((ext_vector_type(8)));

// parameter offsets in the flat vector: W1[64x18], b1[64], W2[64x64], b2[64], w3[64], b3[1]
constexpr int OFF_W1 = 0;
constexpr int OFF_B1 = OFF_W1 + MLP_H * MLP_IN;
constexpr int OFF_W2 = OFF_B1 + MLP_H;
constexpr int OFF_B2 = OFF_W2 + MLP_H * MLP_H;
constexpr int OFF_W3 = OFF_B2 + MLP_H;
constexpr int OFF_B3 = OFF_W3 + MLP_H;

// ---------------------------------------------------------------------------
// Sketch
// ---------------------------------------------------------------------------
// scores[i][j] = s64(U[u0 + i], Pm_sorted[sample_j]) for a batch of users; FP64,
// tile 64 users x 64 samples per 256 threads (4 x 4 per thread), the k loop
// runs in order 0..d-1 so every dot is the sequential fma chain.
__global__ __launch_bounds__(256) void k_sketch_scores(const void *Um, int64_t u0, int64_t nb, const void *Pm,
                                                       int64_t m, int S, int d, int mk, double *scores) {
    __shared__ double su[32][65];
    __shared__ double sp[32][65];
    const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
    const int64_t ub = u0 + (int64_t)blockIdx.y * 64;
    const int jb = blockIdx.x * 64;
    double acc[4][4];
    for (int a = 0; a < 4; ++a)
        for (int b = 0; b < 4; ++b) acc[a][b] = 0.0;
    for (int k0 = 0; k0 < d; k0 += 32) {
        for (int e = threadIdx.x; e < 64 * 32; e += 256) {
            int r = e / 32, kk = e % 32;
            int64_t u = ub + r;
            int j = jb + r;
            double vu = 0.0, vp = 0.0;
            if (k0 + kk < d && u < u0 + nb) vu = master_elem(Um, mk, u * d + k0 + kk);
            if (k0 + kk < d && j < S) {
                int64_t item = ((2 * (int64_t)j + 1) * m) / (2 * (int64_t)S);
                vp = master_elem(Pm, mk, item * d + k0 + kk);
            }
            su[kk][r] = vu;
            sp[kk][r] = vp;
        }
        __syncthreads();
        const int kmax = min(32, d - k0);
        for (int kk = 0; kk < kmax; ++kk) {
            double a[4], b[4];
            for (int t = 0; t < 4; ++t) { a[t] = su[kk][ty * 4 + t]; b[t] = sp[kk][tx * 4 + t]; }
            for (int x = 0; x < 4; ++x)
                for (int y = 0; y < 4; ++y) acc[x][y] = fma(a[x], b[y], acc[x][y]);
        }
        __syncthreads();
    }
    for (int x = 0; x < 4; ++x)
        for (int y = 0; y < 4; ++y) {
            int64_t i = (int64_t)blockIdx.y * 64 + ty * 4 + x;
            int j = jb + tx * 4 + y;
            if (ub + ty * 4 + x < u0 + nb && j < S) scores[i * S + j] = acc[x][y];
        }
}

// One workgroup per user: bitonic sort (descending) of the S scores in LDS,
// then out[u][j] = fl32(score at 1-based position pos[j] / |u|) and raw[u][j]
// = that score itself, for j < levels (either output may be null).
__global__ __launch_bounds__(1024) void k_sketch_select(const void *Um, int64_t u0, int64_t nb, const double *scores,
                                                        int S, int d, int mk, const int *pos, int levels,
                                                        float *out, double *raw) {
    __shared__ double s[4096];
    __shared__ double nrm;
    const int64_t i = blockIdx.x;
    if (i >= nb) return;
    const int64_t u = u0 + i;
    int np2 = 1;
    while (np2 < S) np2 <<= 1;
    for (int j = threadIdx.x; j < np2; j += 1024) s[j] = (j < S) ? scores[i * S + j] : -__builtin_inf();
    if (threadIdx.x == 0) {
        double acc = 0.0;
        for (int k = 0; k < d; ++k) {
            double v = master_elem(Um, mk, u * d + k);
            acc = fma(v, v, acc);
        }
        nrm = sqrt(acc);
    }
    __syncthreads();
    for (int k = 2; k <= np2; k <<= 1)
        for (int j = k >> 1; j > 0; j >>= 1) {
            for (int t = threadIdx.x; t < np2; t += 1024) {
                int l = t ^ j;
                if (l > t) {
                    double a = s[t], b = s[l];
                    bool desc = (t & k) == 0;
                    if (desc ? (a < b) : (a > b)) { s[t] = b; s[l] = a; }
                }
            }
            __syncthreads();
        }
    if ((int)threadIdx.x < levels) {
        const double sv = s[pos[threadIdx.x] - 1];
        if (out) out[u * levels + threadIdx.x] = (float)(nrm > 0.0 ? sv / nrm : 0.0);
        if (raw) raw[u * levels + threadIdx.x] = sv;
    }
}

// ---------------------------------------------------------------------------
// Features and targets
// ---------------------------------------------------------------------------
__device__ inline float feat_of(int f, float tn, float un, const float *sk) {
    return f == 0 ? tn : (f == 1 ? un : sk[f - 2]);
}

// X[i] = [t/|u|, |u|, sketch(u)], z[i] = ln(1 + cnt)  (cnt may be null)
__global__ void k_features(const int32_t *pids, int64_t N, const int32_t *pair_u, const double *t64,
                           const double *unorm3, const float *sketch, const uint32_t *cnt, float *X, float *z) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    int32_t pid = pids ? pids[i] : (int32_t)i;
    int64_t u = pair_u[pid];
    double nu = unorm3[3 * u + 2];
    X[i * MLP_IN + 0] = nu > 0.0 ? (float)(t64[pid] / nu) : 0.0f;
    X[i * MLP_IN + 1] = (float)nu;
    for (int j = 0; j < SKETCH_LEVELS; ++j) X[i * MLP_IN + 2 + j] = sketch[u * SKETCH_LEVELS + j];
    if (z && cnt) z[i] = logf(1.0f + (float)cnt[pid]);
}

// ---------------------------------------------------------------------------
// FP32 training: forward + backward of 128 samples per workgroup; the block's
// gradient is written to its own slot (partial[block][NPARAM]) and summed in a
// fixed order afterwards, so results do not depend on scheduling.
// ---------------------------------------------------------------------------
constexpr int TB = 64;

__global__ __launch_bounds__(256) void k_mlp_fwd_bwd(const float *P, const float *X, const float *z,
                                                     const int64_t *order, int64_t N, int64_t off, float scale,
                                                     float *partial, double *loss_part) {
    __shared__ float sW1[MLP_H * MLP_IN];
    __shared__ float sW2[MLP_H * MLP_H];
    __shared__ float sX[TB][MLP_IN];
    __shared__ float sA1[TB][MLP_H];   // a1, later da1
    __shared__ float sA2[TB][MLP_H];   // a2, later da2
    __shared__ float sdy[TB];
    __shared__ double sloss[256];
    const int tid = threadIdx.x;
    const int64_t base = off + (int64_t)blockIdx.x * TB;
    for (int i = tid; i < MLP_H * MLP_IN; i += 256) sW1[i] = P[OFF_W1 + i];
    for (int i = tid; i < MLP_H * MLP_H; i += 256) sW2[i] = P[OFF_W2 + i];
    for (int e = tid; e < TB * MLP_IN; e += 256) {
        int r = e / MLP_IN, f = e % MLP_IN;
        int64_t gi = base + r;
        float v = 0.0f;
        if (gi < N) v = X[(order ? order[gi] : gi) * MLP_IN + f];
        sX[r][f] = v;
    }
    __syncthreads();
    // layer 1
    for (int e = tid; e < TB * MLP_H; e += 256) {
        int r = e / MLP_H, j = e % MLP_H;
        float a = P[OFF_B1 + j];
        for (int k = 0; k < MLP_IN; ++k) a = fmaf(sW1[j * MLP_IN + k], sX[r][k], a);
        sA1[r][j] = a;
    }
    __syncthreads();
    // layer 2
    for (int e = tid; e < TB * MLP_H; e += 256) {
        int r = e / MLP_H, j = e % MLP_H;
        float a = P[OFF_B2 + j];
        for (int k = 0; k < MLP_H; ++k) a = fmaf(sW2[j * MLP_H + k], fmaxf(sA1[r][k], 0.0f), a);
        sA2[r][j] = a;
    }
    __syncthreads();
    // output, residual, dL/dy = scale * 2 (y - z)   (scale = 1 / batch size)
    double lsum = 0.0;
    if (tid < TB) {
        int64_t gi = base + tid;
        float dy = 0.0f;
        if (gi < N) {
            float y = P[OFF_B3];
            for (int j = 0; j < MLP_H; ++j) y = fmaf(P[OFF_W3 + j], fmaxf(sA2[tid][j], 0.0f), y);
            float r = y - z[order ? order[gi] : gi];
            lsum = (double)r * (double)r;
            dy = scale * 2.0f * r;
        }
        sdy[tid] = dy;
    }
    sloss[tid] = lsum;
    __syncthreads();
    float *G = partial + (int64_t)blockIdx.x * MLP_NPARAM;
    // dw3, db2-prep: da2 = dy * w3 * [a2 > 0]
    if (tid < MLP_H) {
        float g = 0.0f;
        for (int r = 0; r < TB; ++r) g = fmaf(sdy[r], fmaxf(sA2[r][tid], 0.0f), g);
        G[OFF_W3 + tid] = g;
    }
    if (tid == 64) {
        float g = 0.0f;
        for (int r = 0; r < TB; ++r) g += sdy[r];
        G[OFF_B3] = g;
    }
    __syncthreads();
    for (int e = tid; e < TB * MLP_H; e += 256) {
        int r = e / MLP_H, j = e % MLP_H;
        sA2[r][j] = sA2[r][j] > 0.0f ? sdy[r] * P[OFF_W3 + j] : 0.0f;
    }
    __syncthreads();
    // dW2 = da2^T h1, db2 = sum da2
    for (int e = tid; e < MLP_H * MLP_H; e += 256) {
        int j = e / MLP_H, k = e % MLP_H;
        float g = 0.0f;
        for (int r = 0; r < TB; ++r) g = fmaf(sA2[r][j], fmaxf(sA1[r][k], 0.0f), g);
        G[OFF_W2 + e] = g;
    }
    if (tid < MLP_H) {
        float g = 0.0f;
        for (int r = 0; r < TB; ++r) g += sA2[r][tid];
        G[OFF_B2 + tid] = g;
    }
    __syncthreads();
    // da1 = (da2 W2) * [a1 > 0]   (overwrites a1 after dW2 has used h1)
    float da1[TB * MLP_H / 256];
    for (int c = 0; c < TB * MLP_H / 256; ++c) {
        int e = tid + c * 256;
        int r = e / MLP_H, k = e % MLP_H;
        float g = 0.0f;
        for (int j = 0; j < MLP_H; ++j) g = fmaf(sA2[r][j], sW2[j * MLP_H + k], g);
        da1[c] = sA1[r][k] > 0.0f ? g : 0.0f;
    }
    __syncthreads();
    for (int c = 0; c < TB * MLP_H / 256; ++c) {
        int e = tid + c * 256;
        sA1[e / MLP_H][e % MLP_H] = da1[c];
    }
    __syncthreads();
    // dW1 = da1^T X, db1 = sum da1
    for (int e = tid; e < MLP_H * MLP_IN; e += 256) {
        int j = e / MLP_IN, k = e % MLP_IN;
        float g = 0.0f;
        for (int r = 0; r < TB; ++r) g = fmaf(sA1[r][j], sX[r][k], g);
        G[OFF_W1 + e] = g;
    }
    if (tid < MLP_H) {
        float g = 0.0f;
        for (int r = 0; r < TB; ++r) g += sA1[r][tid];
        G[OFF_B1 + tid] = g;
    }
    // loss of the block (fixed-order tree)
    for (int o = 128; o > 0; o >>= 1) {
        __syncthreads();
        if (tid < o) sloss[tid] += sloss[tid + o];
    }
    if (tid == 0) loss_part[blockIdx.x] = sloss[0];
}

__global__ void k_grad_reduce(const float *partial, int nblk, float *grad) {
    int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= MLP_NPARAM) return;
    float g = 0.0f;
    for (int b = 0; b < nblk; ++b) g += partial[(int64_t)b * MLP_NPARAM + p];
    grad[p] = g;
}

__global__ void k_loss_reduce(const double *part, int nblk, double *out) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    double s = 0.0;
    for (int b = 0; b < nblk; ++b) s += part[b];
    *out = s;
}

// Adam (Kingma & Ba): bias-corrected first and second moments.
__global__ void k_adam(float *P, const float *g, float *m, float *v, float lr, float b1, float b2, float eps,
                       float c1, float c2) {
    int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= MLP_NPARAM) return;
    float gi = g[p];
    float mi = b1 * m[p] + (1.0f - b1) * gi;
    float vi = b2 * v[p] + (1.0f - b2) * gi * gi;
    m[p] = mi;
    v[p] = vi;
    float mh = mi / c1, vh = vi / c2;
    P[p] -= lr * mh / (sqrtf(vh) + eps);
}

// ---------------------------------------------------------------------------
// BF16 inference on the matrix cores.
//
// Per wave, 32 pairs at a time.  Layer l computes H_l^T = W_l H_{l-1}^T: the
// weights are the A operand (rows = output units), the activations the B
// operand (columns = pairs), so each lane ends with one pair's column.  The
// 32x32 output block leaves lane l with rows {0-3, 8-11, ...} (l < 32) or
// {4-7, 12-15, ...} (l >= 32); one permlane32 swap per register pair turns
// that into the B layout of the next layer (8 consecutive units per lane).
// ---------------------------------------------------------------------------
__device__ inline uint16_t to_bf16_bits(float x) {
    uint32_t b = __float_as_uint(x);
    b = b + 0x7FFFu + ((b >> 16) & 1u);
    return (uint16_t)(b >> 16);
}
__device__ inline bf16x8 pack8(const float *v) {
    s16x8 r;
    for (int i = 0; i < 8; ++i) r[i] = (short)to_bf16_bits(v[i]);
    return __builtin_bit_cast(bf16x8, r);
}
__device__ inline float swap_half(float a, float b, bool keep_a) {
    // returns, per lane, the element of the swapped pair this lane keeps
    auto r = __builtin_amdgcn_permlane32_swap(__float_as_uint(a), __float_as_uint(b), false, false);
    return __uint_as_float(keep_a ? r[0] : r[1]);
}

// Convert a 32x32 output block (16 regs) of one 32-row unit block into two
// B fragments (k-steps of 16 units): frag[s][0..7] for s = 0, 1.
__device__ inline void block_to_b(const f32x16 &D, float (&out)[2][8]) {
    for (int s = 0; s < 2; ++s) {
        for (int r = 0; r < 4; ++r) {
            const float a = D[8 * s + r], b = D[8 * s + 4 + r];
            auto w = __builtin_amdgcn_permlane32_swap(__float_as_uint(a), __float_as_uint(b), false, false);
            out[s][r] = __uint_as_float(w[0]);
            out[s][4 + r] = __uint_as_float(w[1]);
        }
    }
}

__global__ __launch_bounds__(256) void k_mlp_infer(const float *P, const float *X, const int32_t *pids, int64_t N,
                                                   const int32_t *pair_u, const double *t64, const double *unorm3,
                                                   const float *sketch, float *out, int qmajor_nq, int64_t qmajor_n) {
    __shared__ float sb1[MLP_H], sb2[MLP_H], sw3[MLP_H];
    const int lane = threadIdx.x & 63, half = lane >> 5, l32 = lane & 31;
    for (int i = threadIdx.x; i < MLP_H; i += blockDim.x) {
        sb1[i] = P[OFF_B1 + i];
        sb2[i] = P[OFF_B2 + i];
        sw3[i] = P[OFF_W3 + i];
    }
    __syncthreads();
    const float b3 = P[OFF_B3];
    // weight fragments: A[i = unit][k]: lane holds row (l32 + 32 hb), k = 16 s + 8 half .. + 7
    bf16x8 w1f[2][2], w2f[2][4];
    for (int hb = 0; hb < 2; ++hb) {
        for (int s = 0; s < 2; ++s) {
            float v[8];
            for (int e = 0; e < 8; ++e) {
                int k = 16 * s + 8 * half + e;
                v[e] = k < MLP_IN ? P[OFF_W1 + (32 * hb + l32) * MLP_IN + k] : 0.0f;
            }
            w1f[hb][s] = pack8(v);
        }
        for (int s = 0; s < 4; ++s) {
            float v[8];
            for (int e = 0; e < 8; ++e) v[e] = P[OFF_W2 + (32 * hb + l32) * MLP_H + 16 * s + 8 * half + e];
            w2f[hb][s] = pack8(v);
        }
    }
    const int64_t wave_id = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) >> 6;
    for (int64_t c0 = wave_id * 32; c0 < N; c0 += nwaves * 32) {
        const int64_t i = c0 + l32;
        const bool valid = i < N;
        // B operand of layer 1: features k = 16 s + 8 half .. + 7 of pair i
        float xf[2][8];
        if (X) {
            for (int s = 0; s < 2; ++s)
                for (int e = 0; e < 8; ++e) {
                    int k = 16 * s + 8 * half + e;
                    xf[s][e] = (valid && k < MLP_IN) ? X[i * MLP_IN + k] : 0.0f;
                }
        } else {
            float tn = 0.0f, un = 0.0f;
            const float *sk = sketch;
            if (valid) {
                int32_t pid = pids ? pids[i] : (int32_t)i;
                int64_t u = pair_u[pid];
                double nu = unorm3[3 * u + 2];
                tn = nu > 0.0 ? (float)(t64[pid] / nu) : 0.0f;
                un = (float)nu;
                sk = sketch + u * SKETCH_LEVELS;
            }
            for (int s = 0; s < 2; ++s)
                for (int e = 0; e < 8; ++e) {
                    int k = 16 * s + 8 * half + e;
                    xf[s][e] = (valid && k < MLP_IN) ? feat_of(k, tn, un, sk) : 0.0f;
                }
        }
        bf16x8 xb[2] = {pack8(xf[0]), pack8(xf[1])};
        // layer 1
        float h1[2][2][8];   // [unit block][k-step][8]
        for (int hb = 0; hb < 2; ++hb) {
            f32x16 D = {};
            for (int s = 0; s < 2; ++s) D = __builtin_amdgcn_mfma_f32_32x32x16_bf16(w1f[hb][s], xb[s], D, 0, 0, 0);
            for (int r = 0; r < 16; ++r) {
                int row = 32 * hb + 8 * (r >> 2) + 4 * half + (r & 3);
                D[r] = fmaxf(D[r] + sb1[row], 0.0f);
            }
            block_to_b(D, h1[hb]);
        }
        bf16x8 hb1[4] = {pack8(h1[0][0]), pack8(h1[0][1]), pack8(h1[1][0]), pack8(h1[1][1])};
        // layer 2 and the output unit
        float y = 0.0f;
        for (int hb = 0; hb < 2; ++hb) {
            f32x16 D = {};
            for (int s = 0; s < 4; ++s) D = __builtin_amdgcn_mfma_f32_32x32x16_bf16(w2f[hb][s], hb1[s], D, 0, 0, 0);
            for (int r = 0; r < 16; ++r) {
                int row = 32 * hb + 8 * (r >> 2) + 4 * half + (r & 3);
                y = fmaf(sw3[row], fmaxf(D[r] + sb2[row], 0.0f), y);
            }
        }
        auto yy = __builtin_amdgcn_permlane32_swap(__float_as_uint(y), __float_as_uint(y), false, false);
        y = __uint_as_float(yy[0]) + __uint_as_float(yy[1]) + b3;
        if (valid && half == 0) {
            if (qmajor_nq > 0) out[(i % qmajor_nq) * qmajor_n + i / qmajor_nq] = y;
            else out[i] = y;
        }
    }
}

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------
rkr_status est_build_sketch(Estimator &e, const void *Um, int64_t n, const void *Pm_sorted, int64_t m, int d, int mk,
                            const double *unorm3, int samples, Scratch &sc, hipStream_t st) {
    (void)unorm3;
    if (samples <= 0) return RKR_OK;
    if (samples > 4096) samples = 4096;
    int S = (int)std::min<int64_t>((int64_t)samples, m);
    e.samples = S;
    if (e.sketch.ensure((size_t)n * SKETCH_LEVELS * 4) != hipSuccess) return RKR_E_NOMEM;
    if (S <= 0) {
        // no items: every sketch value is 0
        if (launch_fill_u32((uint32_t *)e.sketch.p, 0, n * SKETCH_LEVELS, st) != hipSuccess) return RKR_E_DEVICE;
        e.has_sketch = true;
        return RKR_OK;
    }
    rkr_status rs = sample_levels(Um, n, Pm_sorted, m, d, mk, S, SKETCH_LEVELS, e.sketch.as<float>(), nullptr, sc,
                                  st);
    if (rs != RKR_OK) return rs;
    e.has_sketch = true;
    return RKR_OK;
}

rkr_status sample_levels(const void *Um, int64_t n, const void *Pm_sorted, int64_t m, int d, int mk, int samples,
                         int levels, float *sketch_out, double *raw_out, Scratch &sc, hipStream_t st) {
    const int S = (int)std::min<int64_t>((int64_t)std::min(samples, 4096), m);
    if (S <= 0 || levels < 2 || levels > 64) return RKR_E_INVALID;
    int pos[64] = {};
    for (int j = 0; j < levels; ++j) {
        double v = std::ceil(std::pow((double)S, (double)j / (levels - 1)) - 1e-9);
        int p = (int)v;
        pos[j] = p < 1 ? 1 : (p > S ? S : p);
    }
    int *dpos = (int *)sc.take(sizeof(pos));
    const int64_t nbmax = std::max<int64_t>(64, std::min<int64_t>(n, ((int64_t)1 << 31) / ((int64_t)S * 8)));
    double *scr = (double *)sc.take(nbmax * S * 8);
    if (!dpos || !scr) return RKR_E_NOMEM;
    if (hipMemcpyAsync(dpos, pos, sizeof(pos), hipMemcpyHostToDevice, st) != hipSuccess) return RKR_E_DEVICE;
    for (int64_t u0 = 0; u0 < n; u0 += nbmax) {
        int64_t nb = std::min<int64_t>(nbmax, n - u0);
        dim3 g1(nblocks(S, 64), nblocks(nb, 64));
        hipLaunchKernelGGL(k_sketch_scores, g1, dim3(256), 0, st, Um, u0, nb, Pm_sorted, m, S, d, mk, scr);
        hipLaunchKernelGGL(k_sketch_select, dim3((unsigned)nb), dim3(1024), 0, st, Um, u0, nb, (const double *)scr, S,
                           d, mk, (const int *)dpos, levels, sketch_out, raw_out);
        if (hipGetLastError() != hipSuccess) return RKR_E_DEVICE;
    }
    if (hipStreamSynchronize(st) != hipSuccess) return RKR_E_DEVICE;
    return RKR_OK;
}

hipError_t est_features(const int32_t *pids, int64_t N, const int32_t *pair_u, const double *t64,
                        const double *unorm3, const float *sketch, const uint32_t *cnt, float *X, float *z,
                        hipStream_t st) {
    if (N <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_features, dim3(nblocks(N, 256)), dim3(256), 0, st, pids, N, pair_u, t64, unorm3, sketch, cnt,
                       X, z);
    return hipGetLastError();
}

// One pass of forward + backward over samples [off, off + nb) (in `order`);
// grad = sum over the samples of scale * dL_i/dtheta; loss = sum (y - z)^2.
hipError_t est_fwd_bwd(Estimator &e, const float *X, const float *z, const int64_t *order, int64_t N, int64_t off,
                       int64_t nb, float scale, float *grad, double *loss_dev, Scratch &sc, hipStream_t st) {
    const int nblk = (int)((nb + TB - 1) / TB);
    float *partial = (float *)sc.take((int64_t)nblk * MLP_NPARAM * 4);
    double *lp = (double *)sc.take((int64_t)nblk * 8);
    if (!partial || !lp) return hipErrorOutOfMemory;
    const int64_t end = std::min<int64_t>(N, off + nb);
    hipLaunchKernelGGL(k_mlp_fwd_bwd, dim3(nblk), dim3(256), 0, st, e.params.as<float>(), X, z, order, end, off, scale,
                       partial, lp);
    hipLaunchKernelGGL(k_grad_reduce, dim3(nblocks(MLP_NPARAM, 256)), dim3(256), 0, st, (const float *)partial, nblk,
                       grad);
    hipLaunchKernelGGL(k_loss_reduce, dim3(1), dim3(64), 0, st, (const double *)lp, nblk, loss_dev);
    return hipGetLastError();
}

hipError_t est_adam(Estimator &e, float lr, int t, hipStream_t st) {
    const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
    const float c1 = 1.0f - powf(b1, (float)t), c2 = 1.0f - powf(b2, (float)t);
    hipLaunchKernelGGL(k_adam, dim3(nblocks(MLP_NPARAM, 256)), dim3(256), 0, st, e.params.as<float>(),
                       (const float *)e.grads.as<float>(), e.adam_m.as<float>(), e.adam_v.as<float>(), lr, b1, b2,
                       eps, c1, c2);
    return hipGetLastError();
}

hipError_t est_infer(Estimator &e, const float *X, const int32_t *pids, int64_t N, const int32_t *pair_u,
                     const double *t64, const double *unorm3, float *out, int qmajor_nq, int64_t qmajor_n,
                     hipStream_t st) {
    if (N <= 0) return hipSuccess;
    int64_t waves = (N + 31) / 32;
    int64_t blocks = std::min<int64_t>((waves + 3) / 4, 4096);
    hipLaunchKernelGGL(k_mlp_infer, dim3((unsigned)blocks), dim3(256), 0, st, e.params.as<float>(), X, pids, N, pair_u,
                       t64, unorm3, (const float *)e.sketch.as<float>(), out, qmajor_nq, qmajor_n);
    return hipGetLastError();
}

// Deterministic initialisation: uniform(-a, a) with a = sqrt(6 / (fan_in + fan_out))
// per weight matrix (Glorot), from a counter-based hash (splitmix64) of
// (seed, index); biases 0 and b3 = mean target.
__device__ inline uint64_t splitmix64(uint64_t x) {
    x += 0x9E3779B97F4A7C15ull;
    x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ull;
    x = (x ^ (x >> 27)) * 0x94D049BB133111EBull;
    return x ^ (x >> 31);
}
__device__ inline float hash_uniform(uint64_t seed, uint64_t i) {
    return (float)((splitmix64(seed * 0x100000001B3ull + i) >> 40) * (1.0 / 16777216.0)) * 2.0f - 1.0f;
}
__global__ void k_init_params(float *P, uint64_t seed) {
    int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= MLP_NPARAM) return;
    float v = 0.0f;
    if (p < OFF_B1) v = hash_uniform(seed, p) * sqrtf(6.0f / (MLP_IN + MLP_H));
    else if (p >= OFF_W2 && p < OFF_B2) v = hash_uniform(seed, p) * sqrtf(6.0f / (MLP_H + MLP_H));
    else if (p >= OFF_W3 && p < OFF_B3) v = hash_uniform(seed, p) * sqrtf(6.0f / (MLP_H + 1));
    P[p] = v;
}
__global__ void k_sum_f32(const float *z, int64_t N, double *out) {
    __shared__ double s[256];
    double a = 0.0;
    for (int64_t i = threadIdx.x; i < N; i += 256) a += (double)z[i];
    s[threadIdx.x] = a;
    for (int o = 128; o > 0; o >>= 1) {
        __syncthreads();
        if (threadIdx.x < o) s[threadIdx.x] += s[threadIdx.x + o];
    }
    if (threadIdx.x == 0) *out = s[0];
}
__global__ void k_set_b3(float *P, const double *sum, int64_t N) { P[OFF_B3] = N > 0 ? (float)(*sum / N) : 0.0f; }
// order[i] = (a i + b) mod N: a permutation when gcd(a, N) = 1
__global__ void k_affine_perm(int64_t *order, int64_t N, int64_t a, int64_t b) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < N) order[i] = (int64_t)(((__int128)a * i + b) % N);
}
// stratified users of query q: u_j = floor((j + f_q) n / per), f_q in [0, 1) from a hash
__global__ void k_mark_strided(int nq, int64_t n, int per, uint64_t seed, uint8_t *flag) {
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (int64_t)nq * per) return;
    int q = (int)(t / per), j = (int)(t % per);
    double f = (splitmix64(seed ^ (0xA5A5ull + q)) >> 11) * (1.0 / 9007199254740992.0);
    int64_t u = (int64_t)(((double)j + f) * (double)n / (double)per);
    if (u >= n) u = n - 1;
    flag[u * nq + q] = 1;
}

hipError_t est_init(Estimator &e, const float *z, int64_t N, uint64_t seed, Scratch &sc, hipStream_t st) {
    hipLaunchKernelGGL(k_init_params, dim3(nblocks(MLP_NPARAM, 256)), dim3(256), 0, st, e.params.as<float>(), seed);
    double *sum = (double *)sc.take(8);
    if (!sum) return hipErrorOutOfMemory;
    hipLaunchKernelGGL(k_sum_f32, dim3(1), dim3(256), 0, st, z, N, sum);
    hipLaunchKernelGGL(k_set_b3, dim3(1), dim3(1), 0, st, e.params.as<float>(), (const double *)sum, N);
    return hipGetLastError();
}
hipError_t est_perm(int64_t *order, int64_t N, int64_t a, int64_t b, hipStream_t st) {
    if (N <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_affine_perm, dim3(nblocks(N, 256)), dim3(256), 0, st, order, N, a, b);
    return hipGetLastError();
}
hipError_t est_mark_strided(int nq, int64_t n, int per, uint64_t seed, uint8_t *flag, hipStream_t st) {
    int64_t T = (int64_t)nq * per;
    if (T <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_mark_strided, dim3(nblocks(T, 256)), dim3(256), 0, st, nq, n, per, seed, flag);
    return hipGetLastError();
}

void est_release(Estimator &e) {
    e.sketch.release(); e.params.release(); e.grads.release(); e.adam_m.release(); e.adam_v.release();
    e.pred.release(); e.feat.release(); e.targ.release(); e.work.release();
}

}  // namespace rkr
