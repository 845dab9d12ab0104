/*
 * learned_oracle.c -- TEST INFRASTRUCTURE ONLY (part of the CPU oracle).
 *
 * Plain fp64 reference of the learned-splitter front end that replaces
 * sampled pivots by a multiway split: a sample of the keys, a 1-32-32-1 MLP
 * fitted to the sample's empirical CDF, splitters read off the model by
 * bisection, and the exact bucket histogram those splitters induce.  None of
 * this is in the paper (which partitions around one pivot at a time); the
 * readings are listed in the repository's design notes:
 *   - sample: m indices i_k = floor(r_k * n / 2^64) where r_k is the k-th
 *     output of splitmix64 seeded with `seed` (Steele, Lea, Flood 2014);
 *   - feature z = (asinh(x / s) - mu) / sd with mu, sd the mean and
 *     (population) standard deviation of asinh(x / s) over the sample; the
 *     scale s comes from the sorted sample: with a = its order statistic of
 *     rank floor(0.01 m) and b that of rank floor(0.99 m), s = a when the
 *     sample is positive there and spans more than three decades (a > 0 and
 *     b / a > 1000), s = -b when it is negative there and spans more than
 *     three decades (b < 0 and a / b > 1000), else the sample's population
 *     standard deviation (1 if that is not a positive finite number); a
 *     quotient x / s beyond the largest double is clamped to it;
 *   - training set: the ntrain = min(4096, m) sample keys of rank
 *     floor(k m / ntrain) + floor(m / (2 ntrain)), k = 0 .. ntrain - 1 (evenly
 *     spaced order statistics); target of the sample key of rank j (0-based,
 *     ascending) is (j + 0.5) / m;
 *   - model: h1 = tanh(W1 z + b1), h2 = tanh(W2 h1 + b2),
 *     F(z) = sigmoid(w3 . h2 + b3); 1153 parameters laid out as
 *     [W1(32) b1(32) W2(32x32, row = output unit) b2(32) w3(32) b3(1)];
 *   - loss: mean squared error over the batch; optimizer: Adam with
 *     beta1 = 0.9, beta2 = 0.999, eps = 1e-8 and bias correction (Kingma & Ba);
 *   - init: Xavier-uniform weights U(-a, a), a = sqrt(6 / (fan_in + fan_out)),
 *     from splitmix64 (53-bit uniforms), biases zero;
 *   - splitter j (1 <= j < nb): the smallest key t of the sorted sample with
 *     F(value(t)) >= j / nb (the largest sample key when there is none), by
 *     bisection over the sample's ranks; then a running maximum and
 *     de-duplication give distinct splitters d_0 < ... < d_{k-1} (a run of
 *     equal sample keys yields one splitter, and so an equality bucket);
 *   - buckets: a key x with r = #{d_i < x} falls in bucket 2r + 1 if
 *     d_r == x (an equality bucket: every key in it is equal) and in bucket
 *     2r otherwise; 2k + 1 buckets.
 * Keys are given as the same unsigned order words the rest of the oracle
 * uses (float64: IEEE totalOrder key).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define H 32
#define NPARAM (H + H + H * H + H + H + 1)
#define OFF_W1 0
#define OFF_B1 (OFF_W1 + H)
#define OFF_W2 (OFF_B1 + H)
#define OFF_B2 (OFF_W2 + H * H)
#define OFF_W3 (OFF_B2 + H)
#define OFF_B3 (OFF_W3 + H)

/* ---- splitmix64 --------------------------------------------------------- */

/* Output k (0-based) of splitmix64 seeded with `seed`: the state advances by
 * the golden-ratio increment before each output, so output k is the mix of
 * seed + (k + 1) * increment. */
uint64_t oracle_splitmix64_at(uint64_t seed, uint64_t k)
{
    uint64_t z = seed + (k + 1) * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

void oracle_sample_indices(uint64_t seed, int64_t n, int64_t m, int64_t *idx)
{
    for (int64_t k = 0; k < m; ++k) {
        unsigned __int128 r = (unsigned __int128)oracle_splitmix64_at(seed, (uint64_t)k) * (uint64_t)n;
        idx[k] = (int64_t)(uint64_t)(r >> 64);
    }
}

/* ---- the model ---------------------------------------------------------- */

int64_t oracle_mlp_nparam(void) { return NPARAM; }

static double uniform01(uint64_t seed, uint64_t k)
{
    return (double)(oracle_splitmix64_at(seed, k) >> 11) * (1.0 / 9007199254740992.0);
}

void oracle_mlp_init(uint64_t seed, double *p)
{
    memset(p, 0, sizeof(double) * NPARAM);
    uint64_t k = 0;
    const double a1 = sqrt(6.0 / (1 + H)), a2 = sqrt(6.0 / (H + H)), a3 = sqrt(6.0 / (H + 1));
    for (int i = 0; i < H; ++i) p[OFF_W1 + i] = (2.0 * uniform01(seed, k++) - 1.0) * a1;
    for (int i = 0; i < H * H; ++i) p[OFF_W2 + i] = (2.0 * uniform01(seed, k++) - 1.0) * a2;
    for (int i = 0; i < H; ++i) p[OFF_W3 + i] = (2.0 * uniform01(seed, k++) - 1.0) * a3;
}

static double sigmoid(double v) { return 1.0 / (1.0 + exp(-v)); }

/* Forward pass of one input; fills the hidden activations if asked. */
static double forward1(const double *p, double z, double *h1, double *h2)
{
    double a[H], b[H];
    for (int i = 0; i < H; ++i) a[i] = tanh(p[OFF_W1 + i] * z + p[OFF_B1 + i]);
    for (int o = 0; o < H; ++o) {
        double s = p[OFF_B2 + o];
        for (int i = 0; i < H; ++i) s += p[OFF_W2 + o * H + i] * a[i];
        b[o] = tanh(s);
    }
    double s = p[OFF_B3];
    for (int i = 0; i < H; ++i) s += p[OFF_W3 + i] * b[i];
    if (h1) memcpy(h1, a, sizeof a);
    if (h2) memcpy(h2, b, sizeof b);
    return sigmoid(s);
}

void oracle_mlp_forward(const double *p, const double *z, int64_t m, double *out)
{
    for (int64_t k = 0; k < m; ++k) out[k] = forward1(p, z[k], NULL, NULL);
}

/* Loss = mean over the batch of (F(z_k) - y_k)^2; grad receives dLoss/dp. */
double oracle_mlp_loss_grad(const double *p, const double *z, const double *y, int64_t m, double *grad)
{
    memset(grad, 0, sizeof(double) * NPARAM);
    double loss = 0.0;
    for (int64_t k = 0; k < m; ++k) {
        double h1[H], h2[H];
        const double f = forward1(p, z[k], h1, h2);
        const double e = f - y[k];
        loss += e * e;
        /* chain rule, output first */
        const double dout = 2.0 * e / (double)m;  /* dLoss/dF */
        const double ds3 = dout * f * (1.0 - f); /* through the sigmoid */
        grad[OFF_B3] += ds3;
        double dh2[H];
        for (int i = 0; i < H; ++i) {
            grad[OFF_W3 + i] += ds3 * h2[i];
            dh2[i] = ds3 * p[OFF_W3 + i];
        }
        double ds2[H];
        for (int o = 0; o < H; ++o) ds2[o] = dh2[o] * (1.0 - h2[o] * h2[o]); /* through tanh */
        double dh1[H] = {0};
        for (int o = 0; o < H; ++o) {
            grad[OFF_B2 + o] += ds2[o];
            for (int i = 0; i < H; ++i) {
                grad[OFF_W2 + o * H + i] += ds2[o] * h1[i];
                dh1[i] += ds2[o] * p[OFF_W2 + o * H + i];
            }
        }
        for (int i = 0; i < H; ++i) {
            const double ds1 = dh1[i] * (1.0 - h1[i] * h1[i]);
            grad[OFF_B1 + i] += ds1;
            grad[OFF_W1 + i] += ds1 * z[k];
        }
    }
    return loss / (double)m;
}

/* One Adam step (t = 1 for the first step). */
void oracle_adam_step(double *p, double *mom, double *vel, const double *grad, int64_t t, double lr)
{
    const double b1 = 0.9, b2 = 0.999, eps = 1e-8;
    const double c1 = 1.0 - pow(b1, (double)t), c2 = 1.0 - pow(b2, (double)t);
    for (int i = 0; i < NPARAM; ++i) {
        mom[i] = b1 * mom[i] + (1.0 - b1) * grad[i];
        vel[i] = b2 * vel[i] + (1.0 - b2) * grad[i] * grad[i];
        p[i] -= lr * (mom[i] / c1) / (sqrt(vel[i] / c2) + eps);
    }
}

/* asinh(x / s), the quotient clamped to the finite doubles. */
static double feat(double x, double s)
{
    double t = x / s;
    if (t > 1.7976931348623157e308) t = 1.7976931348623157e308;
    if (t < -1.7976931348623157e308) t = -1.7976931348623157e308;
    return asinh(t);
}

/* Scale s of the feature from the sorted sample xs[0..m) (see above). */
double oracle_feature_scale(const double *xs, int64_t m)
{
    const double a = xs[(int64_t)(0.01 * (double)m)], b = xs[(int64_t)(0.99 * (double)m)];
    if (a > 0.0 && b / a > 1000.0) return a;
    if (b < 0.0 && a / b > 1000.0) return -b;
    double s = 0.0;
    for (int64_t k = 0; k < m; ++k) s += xs[k];
    const double mean = s / (double)m;
    double v = 0.0;
    for (int64_t k = 0; k < m; ++k) v += (xs[k] - mean) * (xs[k] - mean);
    const double sd = sqrt(v / (double)m);
    return (sd > 0.0 && sd <= 1.7976931348623157e308) ? sd : 1.0;
}

/* Mean and population standard deviation of asinh(x / s) over the sample. */
void oracle_feature_stats(const double *x, int64_t m, double s, double *mu, double *sd)
{
    double sum = 0.0;
    for (int64_t k = 0; k < m; ++k) sum += feat(x[k], s);
    const double mean = sum / (double)m;
    double v = 0.0;
    for (int64_t k = 0; k < m; ++k) {
        const double d = feat(x[k], s) - mean;
        v += d * d;
    }
    *mu = mean;
    *sd = sqrt(v / (double)m);
}

/* Ranks of the training set in a sorted sample of m keys (see above). */
int64_t oracle_training_points(int64_t m, int64_t *rank)
{
    const int64_t nt = m < 4096 ? m : 4096;
    for (int64_t k = 0; k < nt; ++k) rank[k] = (k * m) / nt + m / (2 * nt);
    return nt;
}

/* Full-batch training from `seed`-initialised weights: `steps` Adam steps on
 * (z, y).  Writes the final parameters and each step's loss. */
void oracle_mlp_train(uint64_t seed, const double *z, const double *y, int64_t m, int64_t steps, double lr,
                      double *p, double *losses)
{
    double *mom = (double *)calloc(NPARAM, sizeof(double));
    double *vel = (double *)calloc(NPARAM, sizeof(double));
    double *g = (double *)malloc(sizeof(double) * NPARAM);
    oracle_mlp_init(seed, p);
    for (int64_t t = 1; t <= steps; ++t) {
        losses[t - 1] = oracle_mlp_loss_grad(p, z, y, m, g);
        oracle_adam_step(p, mom, vel, g, t, lr);
    }
    free(mom);
    free(vel);
    free(g);
}

/* ---- splitters ---------------------------------------------------------- */

uint64_t oracle_key_f64(uint64_t bits);

/* Order words of an array of float64 bit patterns. */
void oracle_keys_f64(const uint64_t *bits, int64_t n, uint64_t *out)
{
    for (int64_t i = 0; i < n; ++i) out[i] = oracle_key_f64(bits[i]);
}

static double value_of_f64_key(uint64_t key)
{
    uint64_t bits = (key >> 63) ? (key & 0x7fffffffffffffffull) : ~key;
    double x;
    memcpy(&x, &bits, sizeof x);
    return x;
}

static double model_at(const double *p, double sc, double mu, double sd, uint64_t key)
{
    return forward1(p, (feat(value_of_f64_key(key), sc) - mu) / sd, NULL, NULL);
}

/* The rank of the smallest key of the sorted sample (order words) with
 * F >= q, by bisection over the ranks (the last rank when there is none); for
 * a model that is not monotone, one rank where F crosses q. */
int64_t oracle_invert_one_f64(const double *p, double sc, double mu, double sd, const uint64_t *sorted, int64_t m,
                              double q)
{
    int64_t lo = 0, hi = m - 1;
    while (lo < hi) {
        const int64_t mid = lo + (hi - lo) / 2;
        if (model_at(p, sc, mu, sd, sorted[mid]) >= q)
            hi = mid;
        else
            lo = mid + 1;
    }
    return lo;
}

/* Splitters for nb buckets: nb - 1 bisections over the sorted sample (m
 * order words), then the running maximum; returns them in split[0 .. nb-2]. */
void oracle_invert_f64(const double *p, double sc, double mu, double sd, const uint64_t *sorted, int64_t m, int nb,
                       uint64_t *split)
{
    for (int j = 1; j < nb; ++j)
        split[j - 1] = sorted[oracle_invert_one_f64(p, sc, mu, sd, sorted, m, (double)j / (double)nb)];
    for (int j = 1; j < nb - 1; ++j)
        if (split[j] < split[j - 1]) split[j] = split[j - 1];
}

/* Distinct values of a non-decreasing list; returns their count. */
int64_t oracle_dedupe(const uint64_t *s, int64_t k, uint64_t *d)
{
    int64_t c = 0;
    for (int64_t i = 0; i < k; ++i)
        if (c == 0 || s[i] != d[c - 1]) d[c++] = s[i];
    return c;
}

/* Bucket sizes induced by distinct splitters d[0..k-1] (2k + 1 buckets). */
void oracle_bucket_hist(const uint64_t *keys, int64_t n, const uint64_t *d, int64_t k, int64_t *counts)
{
    memset(counts, 0, sizeof(int64_t) * (size_t)(2 * k + 1));
    for (int64_t i = 0; i < n; ++i) {
        const uint64_t x = keys[i];
        int64_t lo = 0, hi = k; /* r = number of splitters < x */
        while (lo < hi) {
            const int64_t mid = (lo + hi) / 2;
            if (d[mid] < x)
                lo = mid + 1;
            else
                hi = mid;
        }
        const int64_t r = lo;
        counts[(r < k && d[r] == x) ? 2 * r + 1 : 2 * r] += 1;
    }
}
