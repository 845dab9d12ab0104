// hs_learned.hpp -- learned splitters and the multiway partition pass.
//
// The paper partitions around one pivot per pass (Sec. III-B, Alg. 3).  This
// front end replaces sampled pivots by a learned model of the key
// distribution that places 255 splitters at once, and partitions the keys
// into the resulting buckets in one pass (histogram + scatter); each bucket
// then continues through the paper's method (partition levels, on-chip sort,
// bitonic network).  The steps:
//
//   sample      m keys drawn with splitmix64 (output k of splitmix64(seed),
//               scaled to [0, n) by a 64x64 high multiply), sorted by the
//               library's own sort;
//   model       an fp32 MLP 1-32-32-1 (tanh, tanh, sigmoid) fitted to the
//               sample's empirical CDF: input z = (asinh(x / s) - mu) / sd over
//               the sample (s: the sample's 1% order statistic when it is
//               positive there and spans more than three decades, likewise
//               for negative samples, else its standard deviation), targets
//               (rank + 0.5) / m at 4096 evenly spaced order statistics of the
//               sorted sample, mean squared error, Adam; forward, backward
//               and update are this file's kernels (one launch per step);
//   splitters   for j = 1..255 the smallest key of the sorted sample with
//               F >= j/256, by a 64-ary search over the sample's ranks (one
//               wave per splitter; a run of equal sample keys then becomes a
//               single splitter, which gives it an equality bucket), then
//               running maximum and de-duplication;
//   judge       the model's bucket imbalance (largest non-equality bucket over
//               the ideal n/256) on a held-out sample is compared with that of
//               the sample's order statistics (the sampled-pivot fallback);
//               the model is used unless its imbalance exceeds 1.25 times the
//               fallback's;
//   multiway    distinct splitters d_0 < ... < d_{k-1} define 2k+1 buckets: key
//               x with r = #{d_i < x} goes to bucket 2r+1 if d_r == x (an
//               equality bucket, final) and to bucket 2r otherwise; every
//               comparison is an exact comparison of order words, so the
//               learned model never changes the integer arithmetic of the sort.
#pragma once

#include "hs_kernels.hpp"

namespace hs {

constexpr int MLP_H = 32;
constexpr int MLP_NP = 1153;
constexpr int MLP_PS = 1156;  // stride of the per-workgroup partial gradients (16-byte rows)
constexpr int MLP_W1 = 0, MLP_B1 = 32, MLP_W2 = 64, MLP_B2 = 64 + 1024, MLP_W3 = 64 + 1024 + 32,
              MLP_B3 = 64 + 1024 + 64;
constexpr int NBUCKET = 256;           // buckets the splitters aim for
constexpr int NSPLIT = NBUCKET - 1;    // splitters
constexpr int NB_MAX = 2 * NSPLIT + 1; // buckets including the equality buckets
constexpr int MW_NT = 1024;            // threads of a multiway workgroup
constexpr int MW_TILE = 8192;          // keys per multiway tile (longer runs per bucket: 2048 to 8192
                                       // took the 2^28 float64 pass from 2.66 to 2.08 ms)

__device__ __host__ __forceinline__ uint64_t splitmix64_at(uint64_t seed, uint64_t k)
{
    uint64_t z = seed + (k + 1) * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

// The model's view of a key: the searched word S (the key's order word, or
// its key half for key/value words) and the real value fed to the model.
template <int F> struct LearnKey;
template <> struct LearnKey<FMT_F64> {
    using K = uint64_t;
    using S = uint64_t;
    static __device__ __forceinline__ S search(K k) { return k; }
    static __device__ __forceinline__ K word(S s) { return s; }
    // Non-finite values are fed to the model as the largest finite value of
    // their sign, which keeps the feature finite and in totalOrder order.
    static __device__ __forceinline__ double value(S s)
    {
        const double x = __longlong_as_double((long long)dec_f64(s));
        if (__builtin_isfinite(x)) return x;
        return (s >> 63) ? 1.7976931348623157e308 : -1.7976931348623157e308;
    }
};
template <> struct LearnKey<FMT_I32> {
    using K = uint32_t;
    using S = uint32_t;
    static __device__ __forceinline__ S search(K k) { return k; }
    static __device__ __forceinline__ K word(S s) { return s; }
    static __device__ __forceinline__ double value(S s) { return (double)(int32_t)dec_i32(s); }
};
template <> struct LearnKey<FMT_U32> {
    using K = uint32_t;
    using S = uint32_t;
    static __device__ __forceinline__ S search(K k) { return k; }
    static __device__ __forceinline__ K word(S s) { return s; }
    static __device__ __forceinline__ double value(S s) { return (double)s; }
};
template <> struct LearnKey<FMT_I64> {
    using K = uint64_t;
    using S = uint64_t;
    static __device__ __forceinline__ S search(K k) { return k; }
    static __device__ __forceinline__ K word(S s) { return s; }
    static __device__ __forceinline__ double value(S s) { return (double)(long long)dec_i64(s); }
};
template <> struct LearnKey<FMT_KV> {
    using K = uint64_t;
    using S = uint32_t;
    static __device__ __forceinline__ S search(K k) { return (S)(k >> 32); }
    static __device__ __forceinline__ K word(S s) { return (K)s << 32; }  // smallest word with that key
    static __device__ __forceinline__ double value(S s) { return (double)(int32_t)dec_i32(s); }
};
template <> struct LearnKey<FMT_KV_F64> {
    using K = u128;
    using S = uint64_t;
    static __device__ __forceinline__ S search(K k) { return (S)(k >> 64); }
    static __device__ __forceinline__ K word(S s) { return (K)s << 64; }  // smallest word with that key
    static __device__ __forceinline__ double value(S s) { return LearnKey<FMT_F64>::value(s); }
};

constexpr uint32_t LEARN_NTRAIN = 4096;  // training points: evenly spaced order statistics of the sample

// Scalars of the learned front end, in device memory.
// Barrier of the persistent training kernel: arrivals, generation, and an
// error word set when a wait runs out (the workgroups were not all
// resident); each on a line of its own.
struct LearnBar {
    alignas(256) uint32_t arrive;
    alignas(256) uint32_t gen;
    alignas(256) uint32_t err;
};

struct LearnCtl {
    double scale;                 // the feature is asinh(x / scale)
    double mu, sd;                // feature normalisation
    unsigned long long smin, smax;  // searched words of the sample's extremes
    uint32_t k;                   // distinct splitters in use
    uint32_t use_model;           // 1: the model's splitters, 0: the sample's order statistics
    float model_imb, sample_imb;  // imbalance of both splitter sets on the held-out sample
    uint32_t reserved[2];
    LearnBar bar;                 // training barrier (zeroed with the rest)
};

// ---------------------------------------------------------------- sampling

template <int F>
__global__ void k_ls_sample(Raw raw, uint32_t n, uint64_t seed, uint32_t m, Raw out)
{
    const uint32_t k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= m) return;
    const uint32_t i = (uint32_t)__umul64hi(splitmix64_at(seed, k), (uint64_t)n);
    if constexpr (raw_key_bytes<F>() == 8) ((uint64_t *)out.keys)[k] = ((const uint64_t *)raw.keys)[i];
    else ((uint32_t *)out.keys)[k] = ((const uint32_t *)raw.keys)[i];
    if constexpr (has_vals<F>()) out.vals[k] = raw.vals[i];
}

// Held-out sample as order words.
template <int F>
__global__ void k_ls_holdout(Raw raw, uint32_t n, uint64_t seed, uint32_t h, typename KeyOf<F>::type *out)
{
    const uint32_t k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= h) return;
    const uint32_t i = (uint32_t)__umul64hi(splitmix64_at(seed, k), (uint64_t)n);
    out[k] = raw_load<F>(raw, i);
}

// ---------------------------------------------------------------- features

__device__ __forceinline__ double block_sum(double v, double *red)
{
    const int tid = threadIdx.x, lane = lane_id(), wave = tid / WAVE, nw = blockDim.x / WAVE;
    for (int d = 1; d < WAVE; d <<= 1) v += __shfl_xor(v, d);
    __syncthreads();
    if (lane == 0) red[wave] = v;
    __syncthreads();
    double s = 0.0;
    for (int w = 0; w < nw; ++w) s += red[w];  // fixed order: deterministic
    return s;
}

// asinh(x / s), the quotient clamped to the finite doubles.
__device__ __forceinline__ double feat(double x, double s)
{
    double t = x / s;
    t = t > 1.7976931348623157e308 ? 1.7976931348623157e308 : t;
    t = t < -1.7976931348623157e308 ? -1.7976931348623157e308 : t;
    return asinh(t);
}

// Training points: ntrain = min(LEARN_NTRAIN, m) evenly spaced ranks of the
// sorted sample.
__device__ __host__ __forceinline__ uint32_t ntrain_of(uint32_t m) { return m < LEARN_NTRAIN ? m : LEARN_NTRAIN; }
__device__ __forceinline__ uint32_t train_rank(uint32_t k, uint32_t m)
{
    const uint32_t nt = ntrain_of(m);
    return (uint32_t)(((uint64_t)k * m) / nt) + m / (2 * nt);
}

// One workgroup over the sorted sample: the feature's scale and statistics,
// inputs z and targets y of the training points, the order-statistic
// splitters (the fallback) and the extremes.
template <int F>
__global__ __launch_bounds__(1024) void k_ls_prep(Raw sorted, uint32_t m, float *z, float *y,
                                                   typename KeyOf<F>::type *fallback, LearnCtl *lc, double *fbuf)
{
    using LK = LearnKey<F>;
    __shared__ double red[16];
    const uint32_t tid = threadIdx.x;
    auto val = [&](uint32_t k) { return LK::value(LK::search(raw_load<F>(sorted, k))); };
    // scale: the 1% order statistic of a positive sample spanning more than
    // three decades (or minus the 99% one of such a negative sample), else
    // the sample's standard deviation
    const double a = val((uint32_t)(0.01 * (double)m)), b = val((uint32_t)(0.99 * (double)m));
    double sc;
    if (a > 0.0 && b / a > 1000.0) {
        sc = a;
    } else if (b < 0.0 && a / b > 1000.0) {
        sc = -b;
    } else {
        double s0 = 0.0;
        for (uint32_t k = tid; k < m; k += blockDim.x) s0 += val(k);
        const double mean = block_sum(s0, red) / (double)m;
        double v0 = 0.0;
        for (uint32_t k = tid; k < m; k += blockDim.x) {
            const double d = val(k) - mean;
            v0 += d * d;
        }
        sc = sqrt(block_sum(v0, red) / (double)m);
        if (!(sc > 0.0 && sc <= 1.7976931348623157e308)) sc = 1.0;
    }
    // each sample's feature once (kept in fbuf by the thread that reads it back)
    double s = 0.0;
    for (uint32_t k = tid; k < m; k += blockDim.x) {
        const double f = feat(val(k), sc);
        fbuf[k] = f;
        s += f;
    }
    const double mu = block_sum(s, red) / (double)m;
    double v = 0.0;
    for (uint32_t k = tid; k < m; k += blockDim.x) {
        const double d = fbuf[k] - mu;
        v += d * d;
    }
    double sd = sqrt(block_sum(v, red) / (double)m);
    if (!(sd > 0.0)) sd = 1.0;
    __syncthreads();  // fbuf of every sample written (the training points are other threads')
    for (uint32_t k = tid; k < ntrain_of(m); k += blockDim.x) {
        const uint32_t r = train_rank(k, m);
        z[k] = (float)((fbuf[r] - mu) / sd);
        y[k] = (float)(((double)r + 0.5) / (double)m);
    }
    for (uint32_t j = tid; j < (uint32_t)NSPLIT; j += blockDim.x)
        fallback[j] = raw_load<F>(sorted, (uint32_t)(((uint64_t)(j + 1) * m) / NBUCKET));
    if (tid == 0) {
        lc->scale = sc;
        lc->mu = mu;
        lc->sd = sd;
        lc->smin = LK::search(raw_load<F>(sorted, 0));
        lc->smax = LK::search(raw_load<F>(sorted, m - 1));
    }
}

// ---------------------------------------------------------------- the model

// Xavier-uniform initialisation from splitmix64 (53-bit uniforms): W1 takes
// draws 0..31, W2 draws 32..1055, w3 draws 1056..1087; biases are zero.
__global__ void k_mlp_init(float *p, float *mom, float *vel, uint64_t seed, uint32_t *done)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i == 0 && done) *done = 0u;  // the step counter of k_mlp_step
    if (i >= MLP_NP) return;
    mom[i] = 0.f;
    vel[i] = 0.f;
    double a = 0.0;
    int64_t draw = -1;
    if (i < MLP_B1) {
        a = sqrt(6.0 / (1 + MLP_H));
        draw = i;
    } else if (i >= MLP_W2 && i < MLP_B2) {
        a = sqrt(6.0 / (MLP_H + MLP_H));
        draw = MLP_H + (i - MLP_W2);
    } else if (i >= MLP_W3 && i < MLP_B3) {
        a = sqrt(6.0 / (MLP_H + 1));
        draw = MLP_H + MLP_H * MLP_H + (i - MLP_W3);
    }
    if (draw < 0) {
        p[i] = 0.f;
        return;
    }
    const double u = (double)(splitmix64_at(seed, (uint64_t)draw) >> 11) * (1.0 / 9007199254740992.0);
    p[i] = (float)((2.0 * u - 1.0) * a);
}

// tanh(v) = 1 - 2 / (1 + e^(2v)) with the hardware exponential and
// reciprocal: exact limits of +-1 for large |v|, absolute error a few fp32
// ulps.
__device__ __forceinline__ float tanh_fast(float v)
{
    return fmaf(-2.f, __builtin_amdgcn_rcpf(1.f + __expf(2.f * v)), 1.f);
}

// Forward pass of one input with the parameters in LDS.
__device__ __forceinline__ float mlp_forward1(const float *sp, float zf, float *h1, float *h2)
{
#pragma unroll
    for (int i = 0; i < MLP_H; ++i) h1[i] = tanh_fast(fmaf(sp[MLP_W1 + i], zf, sp[MLP_B1 + i]));
#pragma unroll
    for (int o = 0; o < MLP_H; ++o) {
        float s = sp[MLP_B2 + o];
#pragma unroll
        for (int i = 0; i < MLP_H; ++i) s = fmaf(sp[MLP_W2 + o * MLP_H + i], h1[i], s);
        h2[o] = tanh_fast(s);
    }
    float s = sp[MLP_B3];
#pragma unroll
    for (int i = 0; i < MLP_H; ++i) s = fmaf(sp[MLP_W3 + i], h2[i], s);
    return 1.f / (1.f + __expf(-s));
}

__global__ __launch_bounds__(256) void k_mlp_forward(const float *p, const float *z, uint32_t m, float *out)
{
    __shared__ float sp[MLP_NP];
    for (int i = threadIdx.x; i < MLP_NP; i += blockDim.x) sp[i] = p[i];
    __syncthreads();
    const uint32_t k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= m) return;
    float h1[MLP_H], h2[MLP_H];
    out[k] = mlp_forward1(sp, z[k], h1, h2);
}

// Gradient of the mean squared error over samples [0, m) of (z, y) for the
// 256 samples of workgroup g: their gradient sum goes to part[g * MLP_PS ...]
// and their squared error to loss_blk[g].  Each wave takes 64 samples and
// runs the three products of a step on the matrix cores (fp32 MFMA 16x16x4:
// lane l holds A[l%16][l/16] and B[l/16][l%16], and register r of the
// result holds D[4(l/16)+r][l%16]):
//   forward      A2 = H1 W2^T (64x32x32), H1 = tanh(z W1 + b1) computed in
//                the operand layout, H2 = tanh(A2 + b2), F = sigmoid(H2 w3 + b3)
//                (the sum over the 32 outputs of a sample runs over the 16
//                lanes of a row and the two output blocks);
//   weights      dW2 = D2^T H1 (32x32 over the wave's 64 samples) with
//                D2 = ds3 w3 (1 - H2^2), ds3 = 2 (F - y) / m F (1 - F);
//                D2 is already in the operand layout this product needs;
//   layer 1      dH1 = D2 W2 (64x32x32; D2 goes through LDS to change
//                layout), ds1 = dH1 (1 - H1^2);
// and the vector terms (b2, W1, b1, w3, b3, the loss) are sums over lanes.
// The four waves' partials are added in a fixed order, so the result is
// deterministic.
typedef float mlp_v4f __attribute__((ext_vector_type(4)));

__device__ __forceinline__ mlp_v4f mfma4(float a, float b, mlp_v4f c)
{
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

// Sum over the 16 lanes of a row (lanes with equal lane / 16), in every one.
__device__ __forceinline__ float row16_sum(float v)
{
    v += __shfl_xor(v, 1);
    v += __shfl_xor(v, 2);
    v += __shfl_xor(v, 4);
    v += __shfl_xor(v, 8);
    return v;
}

// Sum over lanes l, l ^ 16, l ^ 32, l ^ 48 (the four rows), in every one.
__device__ __forceinline__ float rows4_sum(float v)
{
    v += __shfl_xor(v, 16);
    v += __shfl_xor(v, 32);
    return v;
}

__device__ __forceinline__ void mlp_grad_block(const float *sp, const float *z, const float *y, uint32_t m,
                                               float *part, float *loss_blk)
{
    constexpr int NT = 256, NW = NT / WAVE, DS = 33;  // DS: row stride of the D2 rows in LDS
    __shared__ float sz[NT], sy[NT], sv[NT];
    __shared__ float sd2[NW][WAVE * DS];
    __shared__ float sw2[NW][MLP_H * MLP_H];
    __shared__ float svec[NW][4][MLP_H];
    __shared__ float sscal[NW][2];
    const int tid = threadIdx.x, lane = lane_id(), wv = tid / WAVE;
    const int g = lane >> 4, c = lane & 15;
    const uint32_t k = blockIdx.x * NT + tid;
    const bool valid = k < m;
    sz[tid] = valid ? z[k] : 0.f;
    sy[tid] = valid ? y[k] : 0.f;
    sv[tid] = valid ? 1.f : 0.f;
    __syncthreads();
    const float *wz = sz + wv * WAVE, *wy = sy + wv * WAVE, *wvl = sv + wv * WAVE;

    // ---- forward: A2 = H1 W2^T; B operand W2^T[4ku + g][16ob + c]
    float bw[2][8];
#pragma unroll
    for (int ob = 0; ob < 2; ++ob)
#pragma unroll
        for (int ku = 0; ku < 8; ++ku) bw[ob][ku] = sp[MLP_W2 + (16 * ob + c) * MLP_H + 4 * ku + g];
    mlp_v4f acc[4][2];
#pragma unroll
    for (int sb = 0; sb < 4; ++sb) {
        acc[sb][0] = mlp_v4f{0.f, 0.f, 0.f, 0.f};
        acc[sb][1] = mlp_v4f{0.f, 0.f, 0.f, 0.f};
        const float zs = wz[sb * 16 + c];  // A operand: sample sb*16 + c, unit 4ku + g
#pragma unroll
        for (int ku = 0; ku < 8; ++ku) {
            const int u = 4 * ku + g;
            const float a = tanh_fast(fmaf(sp[MLP_W1 + u], zs, sp[MLP_B1 + u]));
            acc[sb][0] = mfma4(a, bw[0][ku], acc[sb][0]);
            acc[sb][1] = mfma4(a, bw[1][ku], acc[sb][1]);
        }
    }
    // result: acc[sb][ob][r] = A2[sb*16 + 4g + r][16ob + c]
    float d2v[4][2][4];
    float dw3p[2] = {0.f, 0.f}, db3p = 0.f, lossp = 0.f;
#pragma unroll
    for (int sb = 0; sb < 4; ++sb)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int s = sb * 16 + 4 * g + r;
            float h2[2], a3p = 0.f;
#pragma unroll
            for (int ob = 0; ob < 2; ++ob) {
                h2[ob] = tanh_fast(acc[sb][ob][r] + sp[MLP_B2 + 16 * ob + c]);
                a3p = fmaf(h2[ob], sp[MLP_W3 + 16 * ob + c], a3p);
            }
            const float f = 1.f / (1.f + __expf(-(row16_sum(a3p) + sp[MLP_B3])));
            const float e = wvl[s] * (f - wy[s]);
            const float ds3 = 2.f * e / (float)m * f * (1.f - f);
#pragma unroll
            for (int ob = 0; ob < 2; ++ob) {
                d2v[sb][ob][r] = ds3 * sp[MLP_W3 + 16 * ob + c] * (1.f - h2[ob] * h2[ob]);
                dw3p[ob] = fmaf(ds3, h2[ob], dw3p[ob]);
            }
            if (c == 0) {  // one lane per sample
                db3p += ds3;
                lossp = fmaf(e, e, lossp);
            }
        }

    // ---- dW2 = D2^T H1: A operand D2[s][16ob + c], B operand H1[s][16ub + c],
    // s = sb*16 + 4g + r over the 16 steps (sb, r)
    float h1d[4][4][2];
    mlp_v4f acc2[2][2];
#pragma unroll
    for (int ob = 0; ob < 2; ++ob)
#pragma unroll
        for (int ub = 0; ub < 2; ++ub) acc2[ob][ub] = mlp_v4f{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int sb = 0; sb < 4; ++sb)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const float zs = wz[sb * 16 + 4 * g + r];
#pragma unroll
            for (int ub = 0; ub < 2; ++ub)
                h1d[sb][r][ub] = tanh_fast(fmaf(sp[MLP_W1 + 16 * ub + c], zs, sp[MLP_B1 + 16 * ub + c]));
#pragma unroll
            for (int ob = 0; ob < 2; ++ob)
#pragma unroll
                for (int ub = 0; ub < 2; ++ub) acc2[ob][ub] = mfma4(d2v[sb][ob][r], h1d[sb][r][ub], acc2[ob][ub]);
        }

    // ---- dH1 = D2 W2: A operand D2[sb*16 + c][4ko + g] (through LDS), B operand W2[4ko + g][16ub + c]
    float *wd2 = sd2[wv];
#pragma unroll
    for (int sb = 0; sb < 4; ++sb)
#pragma unroll
        for (int ob = 0; ob < 2; ++ob)
#pragma unroll
            for (int r = 0; r < 4; ++r) wd2[(sb * 16 + 4 * g + r) * DS + 16 * ob + c] = d2v[sb][ob][r];
    __syncthreads();
    float bw2[2][8];
#pragma unroll
    for (int ub = 0; ub < 2; ++ub)
#pragma unroll
        for (int ko = 0; ko < 8; ++ko) bw2[ub][ko] = sp[MLP_W2 + (4 * ko + g) * MLP_H + 16 * ub + c];
    float dw1p[2] = {0.f, 0.f}, db1p[2] = {0.f, 0.f};
#pragma unroll
    for (int sb = 0; sb < 4; ++sb) {
        mlp_v4f acc3[2] = {mlp_v4f{0.f, 0.f, 0.f, 0.f}, mlp_v4f{0.f, 0.f, 0.f, 0.f}};
#pragma unroll
        for (int ko = 0; ko < 8; ++ko) {
            const float a = wd2[(sb * 16 + c) * DS + 4 * ko + g];
            acc3[0] = mfma4(a, bw2[0][ko], acc3[0]);
            acc3[1] = mfma4(a, bw2[1][ko], acc3[1]);
        }
        // acc3[ub][r] = dH1[sb*16 + 4g + r][16ub + c], the layout of h1d
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const float zs = wz[sb * 16 + 4 * g + r];
#pragma unroll
            for (int ub = 0; ub < 2; ++ub) {
                const float h = h1d[sb][r][ub];
                const float ds1 = acc3[ub][r] * (1.f - h * h);
                dw1p[ub] = fmaf(ds1, zs, dw1p[ub]);
                db1p[ub] += ds1;
            }
        }
    }

    // ---- the wave's partials to LDS, then the sum over the waves
    float *w2 = sw2[wv];
#pragma unroll
    for (int ob = 0; ob < 2; ++ob)
#pragma unroll
        for (int ub = 0; ub < 2; ++ub)
#pragma unroll
            for (int r = 0; r < 4; ++r) w2[(16 * ob + 4 * g + r) * MLP_H + 16 * ub + c] = acc2[ob][ub][r];
    float db2p[2] = {0.f, 0.f};
#pragma unroll
    for (int ob = 0; ob < 2; ++ob)
#pragma unroll
        for (int sb = 0; sb < 4; ++sb)
#pragma unroll
            for (int r = 0; r < 4; ++r) db2p[ob] += d2v[sb][ob][r];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        const float b2s = rows4_sum(db2p[h]), w1s = rows4_sum(dw1p[h]), b1s = rows4_sum(db1p[h]);
        const float w3s = rows4_sum(dw3p[h]);
        if (g == 0) {
            svec[wv][0][16 * h + c] = b2s;
            svec[wv][1][16 * h + c] = w1s;
            svec[wv][2][16 * h + c] = b1s;
            svec[wv][3][16 * h + c] = w3s;
        }
    }
    const float b3s = rows4_sum(db3p), ls = rows4_sum(lossp);
    if (lane == 0) {
        sscal[wv][0] = b3s;
        sscal[wv][1] = ls;
    }
    __syncthreads();
    float *gout = part + (size_t)blockIdx.x * MLP_PS;
    for (int i = tid; i < MLP_H * MLP_H; i += NT)
        gout[MLP_W2 + i] = ((sw2[0][i] + sw2[1][i]) + sw2[2][i]) + sw2[3][i];
    if (tid < 4 * MLP_H) {
        const int v = tid / MLP_H, j = tid % MLP_H;
        const float t = ((svec[0][v][j] + svec[1][v][j]) + svec[2][v][j]) + svec[3][v][j];
        const int off = v == 0 ? MLP_B2 : v == 1 ? MLP_W1 : v == 2 ? MLP_B1 : MLP_W3;
        gout[off + j] = t;
    }
    if (tid == 0) gout[MLP_B3] = ((sscal[0][0] + sscal[1][0]) + sscal[2][0]) + sscal[3][0];
    if (tid == 1 && loss_blk) loss_blk[blockIdx.x] = ((sscal[0][1] + sscal[1][1]) + sscal[2][1]) + sscal[3][1];
    __syncthreads();  // the caller may overwrite the parameters in LDS next
}

__global__ __launch_bounds__(256) void k_mlp_grad(const float *p, const float *z, const float *y, uint32_t m,
                                                  float *part, float *loss_blk)
{
    __shared__ float sp[MLP_NP];
    for (int i = threadIdx.x; i < MLP_NP; i += blockDim.x) sp[i] = p[i];
    __syncthreads();
    mlp_grad_block(sp, z, y, m, part, loss_blk);
}

// One Adam step of parameter i (beta1 0.9, beta2 0.999, eps 1e-8, bias
// correction) with gradient g at step t.
__device__ __forceinline__ void adam_update(float *p, float *mom, float *vel, uint32_t i, float g, int t, float lr)
{
    const float b1c = 0.9f, b2c = 0.999f, eps = 1e-8f;
    const float c1 = 1.f - powf(b1c, (float)t), c2 = 1.f - powf(b2c, (float)t);
    const float mo = b1c * mom[i] + (1.f - b1c) * g;
    const float ve = b2c * vel[i] + (1.f - b2c) * g * g;
    mom[i] = mo;
    vel[i] = ve;
    p[i] -= lr * (mo / c1) / (sqrtf(ve / c2) + eps);
}

// One training step in one launch, for a few workgroups: each workgroup
// writes the gradient sum of its 256 samples (as k_mlp_grad) and counts
// itself done; the last one to finish sums the partial gradients of every
// parameter over the workgroups in a fixed order (so a step gives the same
// bits every time) and applies Adam.  The agent-scope fences make the
// partials of every workgroup visible to the last one; every workgroup has
// read the parameters before it counts itself done, so the update cannot
// race with a reader.  `done` is zero on entry and left zero.  With `loss`
// set the last workgroup also writes the step's mean squared error (the loss
// before the update).
__global__ __launch_bounds__(256) void k_mlp_step(float *p, float *mom, float *vel, const float *z, const float *y,
                                                  uint32_t m, float *part, float *loss_blk, uint32_t *done, int t,
                                                  float lr, float *loss)
{
    __shared__ uint32_t s_last;
    __shared__ float sp[MLP_NP];
    for (int i = threadIdx.x; i < MLP_NP; i += blockDim.x) sp[i] = p[i];
    __syncthreads();
    mlp_grad_block(sp, z, y, m, part, loss_blk);
    __threadfence();
    __syncthreads();
    if (threadIdx.x == 0) s_last = atomicAdd(done, 1u) == gridDim.x - 1 ? 1u : 0u;
    __syncthreads();
    if (!s_last) return;
    __threadfence();
    const uint32_t G = gridDim.x;
    for (uint32_t i = threadIdx.x; i < (uint32_t)MLP_NP; i += blockDim.x) {
        float g = 0.f;
        for (uint32_t b0 = 0; b0 < G; b0 += 16) {
            float v[16];
#pragma unroll
            for (uint32_t u = 0; u < 16; ++u) v[u] = b0 + u < G ? part[(size_t)(b0 + u) * MLP_PS + i] : 0.f;
#pragma unroll
            for (uint32_t u = 0; u < 16; ++u) g += v[u];
        }
        adam_update(p, mom, vel, i, g, t, lr);
    }
    if (loss && threadIdx.x < WAVE) {
        float l = 0.f;
        for (uint32_t b = threadIdx.x; b < G; b += WAVE) l += loss_blk[b];
        for (int d = 1; d < WAVE; d <<= 1) l += __shfl_xor(l, d);
        if (threadIdx.x == 0) *loss = l / (float)m;
    }
    if (threadIdx.x == 0) *done = 0u;
}

// The fused step sums all partials in one workgroup: for at most this many
// workgroups (larger batches take k_mlp_grad + k_mlp_update).
constexpr uint32_t MLP_STEP_MAX_G = 64;

// Barrier over the G workgroups of k_mlp_train: arrival is one device-scope
// atomic per workgroup, the last arrival resets the count and bumps the
// generation, the others poll it with a bounded spin; the agent-scope fences
// make the partial gradients written before the barrier visible after it.  A
// wait that runs out sets bar->err and every workgroup leaves.
constexpr uint32_t LEARN_SPIN_LIMIT = 1u << 22;

__device__ __forceinline__ bool learn_barrier(LearnBar *bar, uint32_t &gen)
{
    __shared__ uint32_t s_ok;
    __syncthreads();
    if (threadIdx.x == 0) {
        bool ok = true;
        __threadfence();
        if (__hip_atomic_load(&bar->err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) {
            ok = false;
        } else if (atomicAdd(&bar->arrive, 1u) == gridDim.x - 1) {
            atomicExch(&bar->arrive, 0u);
            __threadfence();
            atomicAdd(&bar->gen, 1u);
        } else {
            uint32_t spins = 0;
            while (__hip_atomic_load(&bar->gen, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) == gen) {
                if (__hip_atomic_load(&bar->err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) ||
                    ++spins > LEARN_SPIN_LIMIT) {
                    atomicOr(&bar->err, 1u);
                    ok = false;
                    break;
                }
                __builtin_amdgcn_s_sleep(2);
            }
        }
        __threadfence();
        ++gen;
        s_ok = ok ? 1u : 0u;
    }
    __syncthreads();
    return s_ok != 0;
}

// Every training step in one launch of G workgroups (all resident): each
// keeps the parameters and Adam's moments in LDS; per step it writes the
// gradient sum of its 256 samples to the step's half of `part` (the halves
// alternate, so a workgroup that runs ahead never overwrites partials that
// another one still reads), meets the others at the barrier, then sums the
// G partials of every parameter in a fixed order and applies Adam itself.
// Every workgroup does the same arithmetic in the same order, so all hold
// the same parameters, and no second barrier is needed.  Workgroup 0 writes
// the final parameters to p (which holds the initial ones on entry) and the
// mean squared error of the last step (before its update) to *loss.  If the
// barrier fails (bar->err set), the kernel stops; the caller then must not
// use p.
__global__ __launch_bounds__(256) void k_mlp_train(float *p, const float *z, const float *y, uint32_t m, int steps,
                                                   float lr, float *part, float *loss_blk, LearnBar *bar,
                                                   float *loss)
{
    __shared__ float sp[MLP_NP], smo[MLP_NP], sve[MLP_NP];
    const uint32_t G = gridDim.x;
    for (int i = threadIdx.x; i < MLP_NP; i += blockDim.x) {
        sp[i] = p[i];
        smo[i] = 0.f;
        sve[i] = 0.f;
    }
    __syncthreads();
    uint32_t gen = 0;
    for (int t = 1; t <= steps; ++t) {
        float *pt = part + (size_t)(t & 1) * G * MLP_PS;
        float *lt = loss_blk + (size_t)(t & 1) * G;
        mlp_grad_block(sp, z, y, m, pt, lt);
        if (!learn_barrier(bar, gen)) return;
        for (uint32_t i = threadIdx.x; i < (uint32_t)MLP_NP; i += blockDim.x) {
            // the partials of parameter i: sixteen loads in flight, summed in
            // workgroup order
            float g = 0.f;
            for (uint32_t b0 = 0; b0 < G; b0 += 16) {
                float v[16];
#pragma unroll
                for (uint32_t u = 0; u < 16; ++u) v[u] = b0 + u < G ? pt[(size_t)(b0 + u) * MLP_PS + i] : 0.f;
#pragma unroll
                for (uint32_t u = 0; u < 16; ++u) g += v[u];
            }
            adam_update(sp, smo, sve, i, g, t, lr);
        }
        if (t == steps && blockIdx.x == 0 && loss && threadIdx.x < WAVE) {
            float l = 0.f;
            for (uint32_t b = threadIdx.x; b < G; b += WAVE) l += lt[b];
            for (int d = 1; d < WAVE; d <<= 1) l += __shfl_xor(l, d);
            if (threadIdx.x == 0) *loss = l / (float)m;
        }
        __syncthreads();
    }
    if (blockIdx.x == 0)
        for (int i = threadIdx.x; i < MLP_NP; i += blockDim.x) p[i] = sp[i];
}

// Second half: sum the G partial gradients of every parameter in a fixed
// order (so a step gives the same bits every time), then either apply one
// Adam step (beta1 0.9, beta2 0.999, eps 1e-8, bias correction) to p, mom
// and vel, or write the gradient to grad_out.  Workgroup w owns parameters
// 64w .. 64w+63; its four waves sum a quarter of the partials each.  With
// `loss` set, workgroup 0 also writes the mean squared error of the step
// (the loss before the update).
__global__ __launch_bounds__(256) void k_mlp_update(float *p, float *mom, float *vel, const float *part, uint32_t G,
                                                    int t, float lr, float *grad_out, const float *loss_blk,
                                                    float *loss, uint32_t m)
{
    __shared__ float acc[4][WAVE];
    const int lane = lane_id(), q = threadIdx.x / WAVE;
    const uint32_t i = blockIdx.x * WAVE + lane;
    const uint32_t b0 = (uint32_t)(((uint64_t)G * q) / 4), b1 = (uint32_t)(((uint64_t)G * (q + 1)) / 4);
    float g = 0.f;
    if (i < (uint32_t)MLP_NP) {
        uint32_t b = b0;
        for (; b + 8 <= b1; b += 8) {
            float v[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) v[u] = part[(size_t)(b + u) * MLP_PS + i];
#pragma unroll
            for (int u = 0; u < 8; ++u) g += v[u];
        }
        for (; b < b1; ++b) g += part[(size_t)b * MLP_PS + i];
    }
    acc[q][lane] = g;
    if (blockIdx.x == 0 && q == 1 && loss && loss_blk) {  // the step's loss, one wave, fixed order
        float l = 0.f;
        for (uint32_t b = (uint32_t)lane; b < G; b += WAVE) l += loss_blk[b];
        for (int d = 1; d < WAVE; d <<= 1) l += __shfl_xor(l, d);
        if (lane == 0) *loss = l / (float)m;
    }
    __syncthreads();
    if (q != 0 || i >= (uint32_t)MLP_NP) return;
    g = ((acc[0][lane] + acc[1][lane]) + acc[2][lane]) + acc[3][lane];
    if (grad_out) {
        grad_out[i] = g;
        return;
    }
    adam_update(p, mom, vel, i, g, t, lr);
}

constexpr int MLP_UPDATE_GRID = (MLP_NP + WAVE - 1) / WAVE;

// ---------------------------------------------------------------- splitters

// One wave per splitter j: the smallest key t of the sorted sample with
// F(value(t)) >= (j+1)/256 (the largest sample key when there is none), by a
// 64-ary search over the sample's ranks: lane l probes rank
// lo + floor(span * l / 63), so lane 0 probes lo and lane 63 probes hi; a
// ballot finds the first probe at or above the target and the range shrinks
// to (previous probe, that probe].  Three rounds cover 2^16 ranks.  The
// splitter is the smallest word with that key.  (The model is not monotone
// in general; the search then returns one crossing, and the running maximum
// of the judge restores the order.)
template <int F>
__global__ __launch_bounds__(256) void k_ls_invert(const float *p, const LearnCtl *lc, Raw sorted, uint32_t m,
                                                   typename KeyOf<F>::type *split)
{
    using LK = LearnKey<F>;
    __shared__ float sp[MLP_NP];
    for (int i = threadIdx.x; i < MLP_NP; i += blockDim.x) sp[i] = p[i];
    __syncthreads();
    const int lane = lane_id();
    const uint32_t j = (blockIdx.x * blockDim.x + threadIdx.x) / WAVE;
    if (j >= (uint32_t)NSPLIT) return;
    const float q = (float)(j + 1) / (float)NBUCKET;
    const double sc = lc->scale, mu = lc->mu, sd = lc->sd;
    uint32_t lo = 0, hi = m - 1;
    float h1[MLP_H], h2[MLP_H];
    while (lo < hi) {
        const uint32_t span = hi - lo;
        const uint32_t probe = lo + (uint32_t)(((uint64_t)span * (uint32_t)lane) / (WAVE - 1));
        const double x = LK::value(LK::search(raw_load<F>(sorted, probe)));
        const float zf = (float)((feat(x, sc) - mu) / sd);
        const bool ge = mlp_forward1(sp, zf, h1, h2) >= q;
        const uint64_t bal = __ballot(ge);
        if (bal == 0) {  // F < q up to hi, which is then the last rank: answer it
            lo = hi;
            break;
        }
        const int first = __builtin_ctzll(bal);
        const uint32_t at = lane_bcast(probe, first);
        if (first == 0) {
            hi = lo;
            break;
        }
        lo = lane_bcast(probe, first - 1) + 1;
        hi = at;
    }
    if (lane == 0) split[j] = LK::word(LK::search(raw_load<F>(sorted, lo)));
}

// One workgroup: running maximum and de-duplication of the model's
// splitters, de-duplication of the order statistics, bucket imbalance of
// both on the held-out sample, and the choice.  Writes the chosen distinct
// splitters to `chosen` and their count to lc->k.  mode: JUDGE_AUTO, or
// JUDGE_MODEL / JUDGE_SAMPLE to force one set (JUDGE_SAMPLE does not read
// the model's splitters and reports a model imbalance of -1; a training run
// that could not finish forces it too).  counts_out (optional, 2 * NB_MAX
// words) receives the held-out bucket counts of both sets, the model's
// first (2k + 1 used entries each, the rest zero).
constexpr int JUDGE_AUTO = 0, JUDGE_MODEL = 1, JUDGE_SAMPLE = 2;

template <int F>
__global__ __launch_bounds__(256) void k_ls_judge(const typename KeyOf<F>::type *model_split,
                                                  const typename KeyOf<F>::type *sample_split,
                                                  const typename KeyOf<F>::type *holdout, uint32_t h,
                                                  typename KeyOf<F>::type *chosen, LearnCtl *lc, int mode,
                                                  uint32_t *counts_out)
{
    using K = typename KeyOf<F>::type;
    __shared__ K sn[NSPLIT], so[NSPLIT], dm[NSPLIT], ds[NSPLIT];
    __shared__ uint32_t cm[NB_MAX], cs[NB_MAX];
    __shared__ uint32_t km_s, ks_s, um_s;
    const int tid = threadIdx.x;
    // a training run that could not finish leaves no model: the sample's
    // order statistics are used
    if (mode != JUDGE_SAMPLE && __hip_atomic_load(&lc->bar.err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))
        mode = JUDGE_SAMPLE;
    // both splitter lists into LDS (the loop below runs on one thread)
    for (int j = tid; j < NSPLIT; j += blockDim.x) {
        if (mode != JUDGE_SAMPLE) sn[j] = model_split[j];
        so[j] = sample_split[j];
    }
    __syncthreads();
    if (tid == 0) {
        uint32_t km = 0, ks = 0;
        K run = 0;
        for (int j = 0; j < NSPLIT; ++j) {
            if (mode != JUDGE_SAMPLE) {
                const K v = j == 0 ? sn[0] : (sn[j] > run ? sn[j] : run);
                run = v;
                if (km == 0 || dm[km - 1] != v) dm[km++] = v;
            }
            const K w = so[j];
            if (ks == 0 || ds[ks - 1] != w) ds[ks++] = w;
        }
        km_s = km;
        ks_s = ks;
    }
    for (int i = tid; i < NB_MAX; i += blockDim.x) cm[i] = cs[i] = 0;
    __syncthreads();
    const uint32_t km = km_s, ks = ks_s;
    auto bucket = [](const K *d, uint32_t k, K x) {
        uint32_t lo = 0, hi = k;
        while (lo < hi) {
            const uint32_t mid = (lo + hi) >> 1;
            if (d[mid] < x) lo = mid + 1; else hi = mid;
        }
        return (lo < k && d[lo] == x) ? 2 * lo + 1 : 2 * lo;
    };
    for (uint32_t i = tid; i < h; i += blockDim.x) {
        const K x = holdout[i];
        atomicAdd(&cm[bucket(dm, km, x)], 1u);
        atomicAdd(&cs[bucket(ds, ks, x)], 1u);
    }
    __syncthreads();
    if (tid == 0) {
        uint32_t mm = 0, ms = 0;
        for (uint32_t b = 0; b <= 2 * km; b += 2) mm = max(mm, cm[b]);
        for (uint32_t b = 0; b <= 2 * ks; b += 2) ms = max(ms, cs[b]);
        const float ideal = (float)h / (float)NBUCKET;
        const float im = mode == JUDGE_SAMPLE ? -1.f : (float)mm / ideal, is = (float)ms / ideal;
        const bool use_model = mode == JUDGE_MODEL || (mode == JUDGE_AUTO && im <= 1.25f * is);
        lc->model_imb = im;
        lc->sample_imb = is;
        lc->use_model = use_model ? 1u : 0u;
        lc->k = use_model ? km : ks;
        um_s = use_model ? 1u : 0u;
    }
    __syncthreads();
    const bool um = um_s != 0;
    const uint32_t k = um ? km : ks;
    for (uint32_t i = tid; i < k; i += blockDim.x) chosen[i] = um ? dm[i] : ds[i];
    if (counts_out)
        for (int i = tid; i < NB_MAX; i += blockDim.x) {
            counts_out[i] = cm[i];
            counts_out[NB_MAX + i] = cs[i];
        }
}

// ---------------------------------------------------------------- multiway partition

// Workgroup w owns keys [w*chunk, (w+1)*chunk).  The splitters sit in LDS
// padded to 256 entries with the largest word, which is never below a key,
// so r = #{splitters < x} takes eight fixed steps with no branches; every
// thread keeps several keys in flight.
template <typename K>
__device__ __forceinline__ void mw_load_splitters(K *sd, const K *dsplit, uint32_t k)
{
    for (uint32_t i = threadIdx.x; i < (uint32_t)NBUCKET; i += blockDim.x) sd[i] = i < k ? dsplit[i] : key_max<K>();
}

template <typename K>
__device__ __forceinline__ uint32_t mw_bucket(const K *sd, uint32_t k, K x)
{
    uint32_t r = 0;
#pragma unroll
    for (uint32_t step = NBUCKET / 2; step; step >>= 1)
        if (sd[r + step - 1] < x) r += step;
    return (r < k && sd[r] == x) ? 2 * r + 1 : 2 * r;
}

constexpr int MW_ITEMS = 8;  // keys per thread per round of the histogram pass

// Load the keys p0 + j*MW_NT + threadIdx.x (j < ITEMS) of the range
// [p0, p0 + cnt) as order words, with bounds-checked buffer loads (a lane
// past the end reads zero and moves no data): straight-line code, so the
// next round's loads can be in flight while this round is processed.
template <int F, bool SRC_IS_RAW, int ITEMS>
__device__ __forceinline__ void mw_load(Raw raw, const typename KeyOf<F>::type *src, uint32_t p0, uint32_t cnt,
                                        typename KeyOf<F>::type (&x)[ITEMS])
{
    using K = typename KeyOf<F>::type;
    p0 = (uint32_t)__builtin_amdgcn_readfirstlane((int)p0);
    cnt = (uint32_t)__builtin_amdgcn_readfirstlane((int)cnt);
    if constexpr (SRC_IS_RAW && F == FMT_KV) {
        const auto rk = tile_rsrc((const uint32_t *)raw.keys + p0, cnt * 4u);
        const auto rv = tile_rsrc((const uint32_t *)raw.vals + p0, cnt * 4u);
#pragma unroll
        for (int j = 0; j < ITEMS; ++j) {
            const uint32_t off = (uint32_t)(j * MW_NT + threadIdx.x) * 4u;
            x[j] = enc_kv(rsrc_load32(rk, off), rsrc_load32(rv, off));
        }
    } else if constexpr (SRC_IS_RAW && F == FMT_KV_F64) {
        const auto rk = tile_rsrc((const uint64_t *)raw.keys + p0, cnt * 8u);
        const auto rv = tile_rsrc((const uint32_t *)raw.vals + p0, cnt * 4u);
#pragma unroll
        for (int j = 0; j < ITEMS; ++j) {
            const uint32_t i = (uint32_t)(j * MW_NT + threadIdx.x);
            x[j] = enc_kv_f64(rsrc_load64(rk, i * 8u), rsrc_load32(rv, i * 4u));
        }
    } else if constexpr (sizeof(K) == 16) {
        const auto r = tile_rsrc(src + p0, cnt * 16u);
#pragma unroll
        for (int j = 0; j < ITEMS; ++j) x[j] = rsrc_load128(r, (uint32_t)(j * MW_NT + threadIdx.x) * 16u);
    } else if constexpr (sizeof(K) == 4) {
        const auto r = tile_rsrc((SRC_IS_RAW ? (const K *)raw.keys : src) + p0, cnt * 4u);
#pragma unroll
        for (int j = 0; j < ITEMS; ++j) {
            const uint32_t v = rsrc_load32(r, (uint32_t)(j * MW_NT + threadIdx.x) * 4u);
            x[j] = SRC_IS_RAW ? enc_word<F>((K)v) : (K)v;
        }
    } else {
        const auto r = tile_rsrc((SRC_IS_RAW ? (const K *)raw.keys : src) + p0, cnt * 8u);
#pragma unroll
        for (int j = 0; j < ITEMS; ++j) {
            const uint64_t v = rsrc_load64(r, (uint32_t)(j * MW_NT + threadIdx.x) * 8u);
            x[j] = SRC_IS_RAW ? enc_word<F>((K)v) : (K)v;
        }
    }
}

// Pass 1: bucket sizes of every workgroup's chunk, bucket-major:
// hist[b * G + w].
template <int F, bool SRC_IS_RAW>
__global__ __launch_bounds__(MW_NT) void k_mw_hist(Raw raw, const typename KeyOf<F>::type *src, uint32_t n,
                                                   uint32_t chunk, const typename KeyOf<F>::type *dsplit,
                                                   const LearnCtl *lc, uint32_t *hist)
{
    using K = typename KeyOf<F>::type;
    __shared__ K sd[NBUCKET];
    __shared__ uint32_t cnt[NB_MAX];
    const uint32_t k = lc->k, nb = 2 * k + 1;
    mw_load_splitters(sd, dsplit, k);
    for (uint32_t i = threadIdx.x; i < nb; i += MW_NT) cnt[i] = 0;
    __syncthreads();
    const uint32_t b0 = blockIdx.x * chunk, b1 = min(n, b0 + chunk);
    constexpr uint32_t STEP = MW_NT * MW_ITEMS;
    K x[MW_ITEMS];
    if (b0 < b1) mw_load<F, SRC_IS_RAW, MW_ITEMS>(raw, src, b0, min(STEP, b1 - b0), x);
    for (uint32_t base = b0; base < b1; base += STEP) {
        // the next round's loads first (an empty range after the last round)
        K xn[MW_ITEMS];
        const uint32_t nbase = base + STEP;
        mw_load<F, SRC_IS_RAW, MW_ITEMS>(raw, src, nbase < b1 ? nbase : base, nbase < b1 ? min(STEP, b1 - nbase) : 0u,
                                        xn);
#pragma unroll
        for (int j = 0; j < MW_ITEMS; ++j) {
            const uint32_t i = base + j * MW_NT + threadIdx.x;
            const uint32_t bk = mw_bucket(sd, k, x[j]);
            if (i < b1) atomicAdd(&cnt[bk], 1u);
        }
#pragma unroll
        for (int j = 0; j < MW_ITEMS; ++j) x[j] = xn[j];
    }
    __syncthreads();
    for (uint32_t b = threadIdx.x; b < nb; b += MW_NT) hist[(size_t)b * gridDim.x + blockIdx.x] = cnt[b];
}

// Pass 2a: one workgroup per bucket scans its G workgroup counts
// (exclusive, in place) and writes the bucket's total.
__global__ __launch_bounds__(1024) void k_mw_scan_cols(uint32_t *hist, uint32_t G, const LearnCtl *lc,
                                                       uint32_t *total)
{
    __shared__ uint32_t wsum[16];
    const uint32_t b = blockIdx.x;
    if (b >= 2 * lc->k + 1) return;
    uint32_t *col = hist + (size_t)b * G;
    const int tid = threadIdx.x, lane = lane_id(), wave = tid / WAVE, nw = blockDim.x / WAVE;
    uint32_t carry = 0;
    for (uint32_t base = 0; base < G; base += blockDim.x) {
        const uint32_t i = base + tid;
        const uint32_t v = i < G ? col[i] : 0u;
        const uint32_t incl = wave_incl_scan(v);
        if (lane == WAVE - 1) wsum[wave] = incl;
        __syncthreads();
        uint32_t pre = 0, tot = 0;
        for (int w = 0; w < nw; ++w) {
            if (w < wave) pre += wsum[w];
            tot += wsum[w];
        }
        if (i < G) col[i] = carry + pre + incl - v;
        carry += tot;
        __syncthreads();
    }
    if (tid == 0) total[b] = carry;
}

// Pass 2b: bucket starts (exclusive scan of the totals, one workgroup).
__global__ __launch_bounds__(1024) void k_mw_scan_starts(const uint32_t *total, const LearnCtl *lc,
                                                         uint32_t *start)
{
    __shared__ uint32_t wsum[16];
    const uint32_t nb = 2 * lc->k + 1;
    const int tid = threadIdx.x, lane = lane_id(), wave = tid / WAVE, nw = blockDim.x / WAVE;
    const uint32_t v = (uint32_t)tid < nb ? total[tid] : 0u;
    const uint32_t incl = wave_incl_scan(v);
    if (lane == WAVE - 1) wsum[wave] = incl;
    __syncthreads();
    uint32_t pre = 0;
    for (int w = 0; w < nw; ++w)
        if (w < wave) pre += wsum[w];
    if ((uint32_t)tid <= nb) start[tid] = pre + incl - v;  // start[nb] = n
}

// Pass 3: every workgroup re-reads its chunk tile by tile, groups each tile
// by bucket in LDS (LDS atomics give each key its rank in its bucket) and
// writes every bucket's run at the workgroup's running offset for that
// bucket, consecutive lanes on consecutive addresses.  DST_IS_RAW writes
// the caller's format to `out` instead of order words to `dst`.
template <int F, bool SRC_IS_RAW, bool DST_IS_RAW>
__global__ __launch_bounds__(MW_NT) void k_mw_scatter(Raw raw, const typename KeyOf<F>::type *src, uint32_t n,
                                                      uint32_t chunk, const typename KeyOf<F>::type *dsplit,
                                                      const LearnCtl *lc, const uint32_t *hist,
                                                      const uint32_t *start, typename KeyOf<F>::type *dst, Raw out)
{
    using K = typename KeyOf<F>::type;
    constexpr int ITEMS = MW_TILE / MW_NT;
    constexpr int STORES = ITEMS * ((DST_IS_RAW && has_vals<F>()) ? 2 : 1);
    __shared__ K sd[NBUCKET];
    __shared__ uint32_t cnt[NB_MAX], tbase[NB_MAX], run[NB_MAX];
    __shared__ K stage[MW_TILE];
    __shared__ uint16_t sbk[MW_TILE];
    __shared__ uint32_t wsum[MW_NT / WAVE];
    const uint32_t k = lc->k, nb = 2 * k + 1;
    const int tid = threadIdx.x, lane = lane_id(), wave = tid / WAVE;
    mw_load_splitters(sd, dsplit, k);
    for (uint32_t b = tid; b < nb; b += MW_NT) {
        run[b] = start[b] + hist[(size_t)b * gridDim.x + blockIdx.x];
        cnt[b] = 0;
    }
    const uint32_t c0 = blockIdx.x * chunk, c1 = min(n, c0 + chunk);
    K x[ITEMS];
    if (c0 < c1) mw_load<F, SRC_IS_RAW, ITEMS>(raw, src, c0, min((uint32_t)MW_TILE, c1 - c0), x);
    wait_vmcnt<0>();  // both edges into the loop arrive with the tile loaded
    __syncthreads();
    for (uint32_t t0 = c0; t0 < c1; t0 += MW_TILE) {
        const uint32_t cnt_t = min((uint32_t)MW_TILE, c1 - t0);
        uint32_t bk[ITEMS], rk[ITEMS];
#pragma unroll
        for (int j = 0; j < ITEMS; ++j) {
            const uint32_t i = (uint32_t)(j * MW_NT + tid);
            bk[j] = mw_bucket(sd, k, x[j]);
            rk[j] = 0;
            if (i < cnt_t) rk[j] = atomicAdd(&cnt[bk[j]], 1u);
        }
        // the next tile's loads (an empty range after the last tile)
        K xn[ITEMS];
        const uint32_t nt0 = t0 + MW_TILE;
        mw_load<F, SRC_IS_RAW, ITEMS>(raw, src, nt0 < c1 ? nt0 : t0, nt0 < c1 ? min((uint32_t)MW_TILE, c1 - nt0) : 0u,
                                      xn);
        __syncthreads();
        {  // exclusive scan of the tile's bucket counts: thread t owns buckets 2t, 2t+1
            const uint32_t c0v = (uint32_t)(2 * tid) < nb ? cnt[2 * tid] : 0u;
            const uint32_t c1v = (uint32_t)(2 * tid + 1) < nb ? cnt[2 * tid + 1] : 0u;
            const uint32_t v = c0v + c1v;
            const uint32_t incl = wave_incl_scan(v);
            if (lane == WAVE - 1) wsum[wave] = incl;
            __syncthreads();
            uint32_t pre = 0;
#pragma unroll
            for (int w = 0; w < MW_NT / WAVE; ++w)
                if (w < wave) pre += wsum[w];
            const uint32_t base = pre + incl - v;
            if ((uint32_t)(2 * tid) < nb) tbase[2 * tid] = base;
            if ((uint32_t)(2 * tid + 1) < nb) tbase[2 * tid + 1] = base + c0v;
        }
        __syncthreads();
#pragma unroll
        for (int j = 0; j < ITEMS; ++j) {
            const uint32_t i = (uint32_t)(j * MW_NT + tid);
            if (i < cnt_t) {
                const uint32_t pos = tbase[bk[j]] + rk[j];
                stage[pos] = x[j];
                sbk[pos] = (uint16_t)bk[j];
            }
        }
        __syncthreads();
        // Lanes past the end of a partial tile store the tile's last key
        // again at its own slot: a fixed number of stores, no branch.
#pragma unroll
        for (int j = 0; j < ITEMS; ++j) {
            const uint32_t i = min((uint32_t)(j * MW_NT + tid), cnt_t - 1);
            const uint32_t b = sbk[i];
            if constexpr (DST_IS_RAW) raw_store<F>(out, run[b] + (i - tbase[b]), stage[i]);
            else dst[run[b] + (i - tbase[b])] = stage[i];
        }
        __syncthreads();
        for (uint32_t b = tid; b < nb; b += MW_NT) {
            run[b] += cnt[b];
            cnt[b] = 0;
        }
        __syncthreads();
        wait_vmcnt<STORES>();  // the next tile's loads (older than the stores) are in
#pragma unroll
        for (int j = 0; j < ITEMS; ++j) x[j] = xn[j];
    }
}

// Splitter count of a caller-supplied splitter set.
__global__ void k_ls_set_k(LearnCtl *lc, uint32_t k)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) lc->k = k;
}

// Route every bucket: equality buckets become fill tasks (split into chunks
// so that one wave never fills more than FILL_CHUNK keys), open buckets of at
// most T keys become local tasks, larger ones the first partition level's
// segments.  One lane per bucket, wave-batched emission.
template <int F>
__global__ __launch_bounds__(256) void k_mw_route(Ctl *ctl, const LearnCtl *lc, const uint32_t *start,
                                                  const typename KeyOf<F>::type *dsplit,
                                                  const typename KeyOf<F>::type *buf, uint32_t buf_id,
                                                  Seg<typename KeyOf<F>::type> *cand, unsigned long long *cur,
                                                  Task<typename KeyOf<F>::type> *tasks,
                                                  uint32_t T, uint32_t leaf, int rule, uint32_t cand_cap,
                                                  uint32_t task_cap)
{
    using K = typename KeyOf<F>::type;
    const int lane = lane_id();
    const uint32_t nb = 2 * lc->k + 1;
    const uint32_t b = (blockIdx.x * blockDim.x + threadIdx.x);
    const bool valid = b < nb;
    const uint32_t s0 = valid ? start[b] : 0u, s1 = valid ? start[b + 1] : 0u, m = s1 - s0;
    const bool eq = valid && (b & 1u) && m > 0;
    const bool is_local = valid && !(b & 1u) && m >= 1 && m <= T;
    const bool big = valid && !(b & 1u) && m > T;
    // fills, chunked
    const uint32_t nchunk = eq ? (m + FILL_CHUNK - 1) / FILL_CHUNK : 0u;
    uint32_t maxc = nchunk;
    for (int d = 1; d < WAVE; d <<= 1) maxc = max(maxc, (uint32_t)__shfl_xor((int)maxc, d));
    for (uint32_t c = 0; c < maxc; ++c) {
        Task<K> t;
        t.b = s0 + c * FILL_CHUNK;
        t.e = min(s1, t.b + FILL_CHUNK);
        t.src = buf_id;
        t.kind = TASK_FILL;
        t.fill = eq ? dsplit[(b - 1) / 2] : K(0);
        wave_flush_task(t, c < nchunk, true, tasks, task_cap, ctl);
    }
    {
        Task<K> t;
        t.b = s0;
        t.e = s1;
        t.src = buf_id;
        t.kind = TASK_LOCAL;
        t.fill = 0;
        wave_flush_task(t, is_local, m <= leaf, tasks, task_cap, ctl);
    }
    const unsigned long long lk = wave_sum64(is_local ? (unsigned long long)m : 0ull);
    const unsigned long long fk = wave_sum64(eq ? (unsigned long long)m : 0ull);
    if (lane == 0) {
        if (lk) atomicAdd(&ctl->local_keys, lk);
        if (fk) atomicAdd(&ctl->fill_keys, fk);
    }
    Seg<K> sg;
    sg.b = s0;
    sg.e = s1;
    sg.tile0 = 0;
    sg.flags = 0;
    sg.ub = 0;
    sg.piv = 0;
    SrcReader<F> rd{buf, Raw{nullptr, nullptr}, false};
    for (uint64_t bb = __ballot(big); bb; bb &= bb - 1) {
        const int src = __builtin_ctzll(bb);
        const uint32_t x0 = (uint32_t)__builtin_amdgcn_readlane((int)s0, src);
        const uint32_t x1 = (uint32_t)__builtin_amdgcn_readlane((int)s1, src);
        const K pv = wave_pick_pivot<K>(rd, x0, x1, rule, lane);
        if (lane == src) sg.piv = pv;
    }
    wave_emit_segs(sg, big, cand, cur, &ctl->lev[1], cand_cap, ctl);
}

}  // namespace hs
