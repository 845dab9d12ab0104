/*
 * hsort.h -- C ABI of the MI355X (gfx950) hybrid quicksort + bitonic sort.
 *
 * The method is the hybrid sort of Bramas, "A Novel Hybrid Quicksort
 * Algorithm Vectorized using AVX-512 on Intel Skylake" (arXiv 1704.08579):
 * quicksort partitioning around a pivot (Sec. III-B, Algorithm 3; Sec. III-C,
 * Algorithm 4) with partitions below a bound sorted by a branch-free bitonic
 * network (Sec. III-A, Algorithms 1 and 2), for int32, uint32, int64 and
 * float64 keys and key/value pairs with int32 or float64 keys and int32
 * values (Sec. III-D).
 *
 * Conventions shared by every entry point:
 *   - Every array pointer is a DEVICE pointer (hipMalloc memory, or e.g. a
 *     torch tensor's data_ptr()).  `stream` is a hipStream_t; NULL means the
 *     null stream.  Work is enqueued on `stream`.  The sorts read their
 *     control block back at the end (and, with the host-driven level loop,
 *     after each batch of levels) to report errors raised inside kernels,
 *     so a sort returns once its work on `stream` has completed; while the
 *     stream is being captured into a graph nothing is read back (see the
 *     plan entry points).  A whole-array sort that is a single on-chip task
 *     (at most the on-chip limit, 8192 keys by default, 4096 float64
 *     key/value pairs) cannot fail and reads nothing back: it returns as
 *     soon as it is enqueued (after it completed when statistics are asked
 *     for).  Up to 1024 keys (512 float64 key/value pairs; fewer when
 *     hs_opts.local_T or hs_opts.leaf is set lower) it is one wave's
 *     bitonic network in a single kernel.  hs_partition_i32
 *     and the learned method's kernel entry points return as soon as their
 *     work is enqueued.
 *   - Sorts are in place, ascending and not stable: the paper's partition
 *     and bitonic network are not stable (Sec. II-A).  Equal keys of the
 *     key/value sorts come out ordered by value (a valid, deterministic
 *     choice among the permutations the method allows).
 *   - The caller owns every array and the stream; the library keeps no
 *     pointer once the call's work on `stream` has completed.  Scratch
 *     memory ("workspace") is owned by the library, cached per device and
 *     grown on demand, unless the caller passes one in hs_opts.
 *   - Errors are reported by return code only (hs_status); nothing is
 *     thrown across the ABI.  Argument errors are detected before any
 *     launch.  hs_last_error() returns a thread-local message describing
 *     the last non-OK return of the calling thread.  With HSORT_LOG=1 in the
 *     environment every sort call prints one line to stderr (operation,
 *     size, options, result and, when statistics are asked for, levels and
 *     times).
 *   - Limits: 0 <= n < 2^31 elements per call (positions fit 32 bits inside
 *     the kernels; byte offsets are 64-bit).
 */
#ifndef HSORT_H
#define HSORT_H

#include <stddef.h>
#include <stdint.h>

#if defined(__GNUC__) || defined(__clang__)
#define HS_API __attribute__((visibility("default")))
#else
#define HS_API
#endif

#ifdef __cplusplus
extern "C" {
#endif

typedef enum hs_status {
    HS_OK = 0,
    HS_EINVAL = -1,       /* bad argument (null pointer, n out of range, overlap, ...) */
    HS_ENOMEM = -2,       /* device allocation of the workspace failed */
    HS_EHIP = -3,         /* a HIP runtime call failed; see hs_last_error() */
    HS_EWORKSPACE = -4,   /* caller-provided workspace is too small */
    HS_EUNSUPPORTED = -5, /* device is not gfx950, or an option is not supported */
    HS_EINTERNAL = -6     /* a kernel reported a broken invariant */
} hs_status;

/* Operation codes for hs_workspace_size(), plans and the autotuner. */
enum { HS_OP_SORT_I32 = 0, HS_OP_SORT_F64 = 1, HS_OP_SORT_KV_I32 = 2,
       HS_OP_PARTITION_I32 = 3, HS_OP_SORT_SEGMENTED_I32 = 4,
       HS_OP_SORT_U32 = 5, HS_OP_SORT_I64 = 6, HS_OP_SORT_KV_F64 = 7, HS_OP_SORT_SEGMENTED_F64 = 8 };

/* Pivot rules (hs_opts.pivot_rule). */
enum { HS_PIVOT_AUTO = 0,     /* the tuned default */
       HS_PIVOT_MEDIAN3 = 1,  /* median of first, middle, last (Sec. IV-A) */
       HS_PIVOT_NINTHER = 2,  /* median of three medians of three */
       HS_PIVOT_SAMPLE = 3 }; /* global levels: lower median of 64 evenly spaced keys
                                 (ninther below 256 keys); on chip every rule but
                                 MEDIAN3 takes the lower median of 32 evenly spaced
                                 keys */

/* Sort methods (hs_opts.method). */
enum { HS_METHOD_PLAIN = 0,     /* the paper's method: one pivot per partition */
       HS_METHOD_LEARNED = 1 }; /* a 256-way split by learned splitters first (see below) */

/* Level drivers (hs_opts.driver).  In both, the segment list of the next
 * level is built on the device by the kernels that finalize a level.
 * PERSISTENT runs every partition level in one launch whose workgroups meet
 * at grid barriers: no host round trip, so the call can be captured into a
 * graph.  HOST launches the levels in batches of fixed-grid kernels and
 * reads the control block back after each batch; on this chip a kernel
 * boundary costs less than a grid barrier, so it is the faster one.  AUTO
 * (0) takes HOST, or PERSISTENT while the stream is being captured. */
enum { HS_DRIVER_AUTO = 0, HS_DRIVER_HOST = 1, HS_DRIVER_PERSISTENT = 2 };

/* Flags of the learned method (hs_opts.learn_flags). */
enum { HS_LEARN_FORCE_MODEL = 1,    /* use the model's splitters whatever the judge says */
       HS_LEARN_FORCE_SAMPLE = 2 }; /* use the sample's order statistics (skip the model) */

/* Optional per-call statistics (host memory).  Filling it costs one extra
 * stream synchronisation. */
typedef struct hs_stats {
    int64_t passes;        /* global partition levels run */
    int64_t bytes_alg;     /* algorithmic HBM bytes: 2*s per key per pass and per local sort */
    int64_t keys_partitioned; /* sum over levels of the keys in partitioned segments */
    int64_t tasks;         /* on-chip (local sort / fill) tasks */
    int64_t max_depth;     /* deepest global level that partitioned */
    int32_t fallback_used; /* learned method: 1 if the judge chose the sample's order statistics */
    int32_t splitters;     /* learned method: distinct splitters used */
    double bucket_imbalance; /* learned method: imbalance of the splitters used (held-out sample) */
    /* Kernel times measured with HIP events on `stream` around each launch
     * (filled only when stats are requested). */
    double partition_ms;   /* sum over the partition-pass launches */
    double local_ms;       /* the on-chip sort launches (both, when levels outlasted the first batch) */
    int64_t partition_launches;
    /* learned method only */
    double model_imbalance;  /* largest non-equality bucket / (n/256), model splitters, held-out sample */
    double sample_imbalance; /* the same for the sample's order statistics */
    double learn_ms;         /* sampling, sample sort, training, inversion and judge */
    double multiway_ms;      /* the multiway partition pass */
    double final_loss;       /* training loss after the last step */
} hs_stats;

/* Optional tuning knobs.  A NULL hs_opts*, or 0 in a field, selects the
 * tuned default. */
typedef struct hs_opts {
    int32_t pivot_rule;   /* HS_PIVOT_* */
    int32_t local_T;      /* on-chip segment limit in keys (ranges up to it are sorted on chip; larger ones
                           * are partitioned again); capped at 8192 (4096 for float64 key/value) */
    int32_t method;       /* HS_METHOD_* */
    int32_t learn_flags;  /* HS_LEARN_* */
    int32_t train_steps;  /* learned method: Adam steps (default 100) */
    int32_t sample_log2;  /* learned method: log2 of the training sample (default 16, range 10..20) */
    float learning_rate;  /* learned method: Adam learning rate (default 3e-2) */
    int32_t driver;       /* HS_DRIVER_*: how the partition levels are driven */
    int32_t spin_limit;   /* testing: cap on the polls of one grid-barrier wait (0: about 4M); a wait that
                           * runs out fails the call with HS_EINTERNAL */
    int32_t leaf;         /* largest range one wave sorts with the bitonic network alone: a power of two in
                           * 64..1024, capped at the type's network (1024 int32, 512 float64 and
                           * key/value, 256 float64 key/value; the default); larger ranges go to the
                           * workgroup on-chip sort */
    int32_t autotune;     /* 1: use (or first measure and remember) the tuned knobs for this operation and
                           * size class; see hs_autotune */
    int32_t inplace;      /* 1: partition levels in place in the caller's arrays (no second copy of the keys
                           * in the workspace: one bit per key and 4 bytes per 64 keys instead); host-driven
                           * levels only (not with HS_DRIVER_PERSISTENT, a plan, the autotuner or the learned
                           * method, which return HS_EINVAL).  Output identical, slower per level */
    uint64_t seed;        /* learned method: seed of the sample draws and the initial weights */
    void *workspace;      /* caller-owned device scratch, or NULL */
    size_t workspace_bytes;
} hs_opts;

/* Sort n int32 keys in place (Algorithm 4 on int32). */
HS_API int hs_sort_i32(int32_t *keys, int64_t n, const hs_opts *opts, hs_stats *stats, void *stream);

/* Sort n float64 keys in place by IEEE 754-2008 totalOrder:
 * -NaN < -inf < ... < -0 < +0 < ... < +inf < +NaN.  Output bits are the input
 * bits, permuted. */
HS_API int hs_sort_f64(double *keys, int64_t n, const hs_opts *opts, hs_stats *stats, void *stream);

/* Sort n uint32 keys in place (unsigned order; the same kernels as int32). */
HS_API int hs_sort_u32(uint32_t *keys, int64_t n, const hs_opts *opts, hs_stats *stats, void *stream);

/* Sort n int64 keys in place (two's-complement order; the same kernels as
 * float64, with the sign bit flipped instead of the totalOrder map). */
HS_API int hs_sort_i64(int64_t *keys, int64_t n, const hs_opts *opts, hs_stats *stats, void *stream);

/* Stable argsort of n int32 keys: keys_out receives the keys in ascending
 * order and idx_out[i] the position in `keys` of keys_out[i]; equal keys keep
 * their input order.  It is the key/value sort (Sec. III-D) with the indices
 * 0..n-1 as values: the (key, value) order word orders equal keys by index,
 * so the output is unique.  keys_out may be `keys` (in place) or a separate
 * array; idx_out must not overlap either.  All three are DEVICE pointers. */
HS_API int hs_argsort_i32(const int32_t *keys, int32_t *keys_out, int32_t *idx_out, int64_t n,
                          const hs_opts *opts, hs_stats *stats, void *stream);

/* Stable argsort of n float64 keys by IEEE 754-2008 totalOrder: keys_out
 * receives the keys in order (bits unchanged) and idx_out[i] the position in
 * `keys` of keys_out[i]; keys with equal bits keep their input order.  It is
 * the key/value sort of Sec. III-D on float64 keys with the indices 0..n-1
 * as values (the value breaks ties, so the order is unique).  keys_out may
 * be `keys` or a separate array; idx_out must not overlap either (DEVICE
 * pointers; HS_EINVAL otherwise, before any launch). */
HS_API int hs_argsort_f64(const double *keys, double *keys_out, int32_t *idx_out, int64_t n,
                          const hs_opts *opts, hs_stats *stats, void *stream);

/* Sort n (key, value) pairs held as two separate arrays (Sec. III-D) by key,
 * in place; every value moves with its key.  keys and vals must not
 * overlap. */
HS_API int hs_sort_kv_i32(int32_t *keys, int32_t *vals, int64_t n, const hs_opts *opts,
                   hs_stats *stats, void *stream);

/* Sort n (float64 key, int32 value) pairs held as two separate arrays
 * (Sec. III-D) by the key's IEEE 754-2008 totalOrder, in place; every value
 * moves with its key, and equal keys (equal bits) are ordered by their
 * values' bits as unsigned 32-bit integers, so the output is unique.  A pair
 * travels as one 128-bit order word (the key's totalOrder word above the
 * value), on the same kernels as the other formats with half as many keys
 * per on-chip task.  keys and vals must not overlap (DEVICE pointers).  With
 * the learned method the model sees the keys (its splitters are the
 * smallest words of their keys). */
HS_API int hs_sort_kv_f64(double *keys, int32_t *vals, int64_t n, const hs_opts *opts, hs_stats *stats,
                          void *stream);

/* Partition n int32 keys in place around `pivot` (Algorithm 3's contract):
 * afterwards keys[0,k) <= pivot < keys[k,n), with k = #{x <= pivot} written
 * to the DEVICE int64 *d_count_le.  The order inside each side is
 * unspecified.  By default the keys are staged in the workspace and
 * partitioned back (one read and one write of each key after the copy);
 * with opts->inplace set they never leave the array (classify, count the
 * misplaced keys, exchange them pairwise), and the workspace holds one bit
 * per key and 4 bytes per 64 keys instead of a copy.  The call returns once
 * its work is enqueued, so errors found by its kernels cannot be returned:
 * if one flags an inconsistency (the misplaced-key counts of the in-place
 * exchange do not match), *d_count_le is set to -1 and the keys are left
 * partly partitioned.  n = 0 writes 0 without touching keys.  Every clear
 * is a kernel (no memset), so the call can be captured into a graph. */
HS_API int hs_partition_i32(int32_t *keys, int64_t n, int32_t pivot, int64_t *d_count_le,
                     const hs_opts *opts, void *stream);

/* hs_sort_i32 for callers that cannot allocate memory: code being captured
 * into a HIP graph, tight serving loops, harnesses that forbid hipMalloc.
 * Same result as hs_sort_i32 with default options (it runs the same
 * kernels), but its scratch memory is a static device array of the library
 * (20 MiB per GPU, reserved when the library's code is loaded on the device
 * and held until the process ends) instead of the cached workspace; the
 * call makes no hipMalloc, hipFree or other allocating call (the first call
 * on a device looks up the array's address there).  Limits and errors:
 * n <= 2^22 keys (HS_EINVAL above), NULL keys with n > 0 (HS_EINVAL), not a
 * gfx950 device (HS_EUNSUPPORTED), a kernel-reported error (HS_EINTERNAL).
 * Every call on one GPU shares that GPU's array and starts by clearing what
 * must start at zero; calls whose work overlaps on one GPU (other streams,
 * other threads, or a graph replayed while a call runs) race on it and must
 * be ordered by the caller.  While `stream` is being captured the sort runs
 * its persistent level driver and nothing is read back (kernel-reported
 * errors cannot be returned then). */
HS_API int hs_sort_i32_noalloc(int32_t *keys, int64_t n, void *stream);

/* Sort nseg independent int32 segments in place: segment i is
 * keys[off[i], off[i+1]) with the DEVICE array off[nseg+1], off[0] = 0,
 * non-decreasing, off[nseg] = n_total (the caller states n_total so that no
 * read-back is needed). */
HS_API int hs_sort_segmented_i32(int32_t *keys, int64_t n_total, const int64_t *d_offsets,
                          int64_t nseg, const hs_opts *opts, hs_stats *stats, void *stream);

/* The same for float64 segments: every segment is sorted by Algorithm 4 on
 * its own (IEEE 754-2008 totalOrder; output bits = input bits permuted within
 * each segment).  Offsets as for hs_sort_segmented_i32; malformed offsets
 * found by the kernels return HS_EINTERNAL. */
HS_API int hs_sort_segmented_f64(double *keys, int64_t n_total, const int64_t *d_offsets,
                                 int64_t nseg, const hs_opts *opts, hs_stats *stats, void *stream);

/* ---- The learned-splitter method (HS_METHOD_LEARNED) -------------------
 *
 * Not in the paper, which partitions around one pivot at a time (Sec. III-B,
 * Algorithm 3).  A sample of 2^sample_log2 keys (drawn with splitmix64) is
 * sorted; an fp32 MLP 1-32-32-1 (tanh, tanh, sigmoid) is trained on the GPU
 * by these kernels to the sample's empirical CDF (input
 * (asinh(x / s) - mu) / sd, with s the sample's 1% order statistic when the
 * sample is positive there and spans more than three decades, likewise for
 * negative samples, else its standard deviation; targets (rank + 0.5)/m at
 * 4096 evenly spaced order statistics of the sorted sample; mean squared
 * error; full-batch Adam, 100 steps at lr 3e-2 by default, all in one
 * launch); 255 splitters are read off the model (for j = 1..255 the smallest
 * sample key with F >= j/256), and a judge compares the model's bucket
 * imbalance on a held-out sample with that of the sample's order statistics
 * (the sampled-pivot fallback), keeping the model unless it is more than
 * 1.25 times worse.  One multiway pass then splits the keys into 2k+1
 * buckets (k distinct splitters; keys equal to a splitter form a final
 * bucket) by exact comparisons, and every bucket continues through the
 * plain method.  The output is the same as the plain method's.
 * sort_i32, sort_f64 and sort_kv_i32 accept it; the segmented sort does not.
 *
 * The model parameters are 1153 fp32 values laid out as
 * [W1(32) b1(32) W2(32x32, row = output unit) b2(32) w3(32) b3(1)];
 * F(z) = sigmoid(w3 . tanh(W2 tanh(W1 z + b1) + b2) + b3).  The calls below
 * expose the model's kernels and the multiway pass on their own (device
 * pointers; asynchronous on `stream`). */

/* out[i] = F(z[i]) for i < m. */
HS_API int hs_mlp_forward_f32(const float *d_params, const float *d_z, int64_t m, float *d_out, void *stream);

/* Gradient of the mean squared error (1/m) sum_i (F(z_i) - y_i)^2 with
 * respect to the 1153 parameters, summed over samples in a fixed order (so
 * repeated calls give identical bits); m <= 2^20. */
HS_API int hs_mlp_grad_f32(const float *d_params, const float *d_z, const float *d_y, int64_t m, float *d_grad,
                           void *stream);

/* Xavier-uniform initialisation from `seed` (splitmix64 draws) followed by
 * `steps` full-batch Adam steps at learning rate `lr`; the trained
 * parameters go to d_params (1153 floats); d_loss (optional, `steps` floats)
 * receives the loss before each step.  m <= 2^20. */
HS_API int hs_mlp_train_f32(const float *d_z, const float *d_y, int64_t m, int32_t steps, float lr, uint64_t seed,
                            float *d_params, float *d_loss, void *stream);

/* Split n float64 keys (IEEE totalOrder) in place into the 2k+1 buckets of
 * k distinct, increasing splitters given as totalOrder keys (the unsigned
 * word bits ^ (sign ? ~0 : 1 << 63)) in device memory (k <= 255): bucket 2r
 * holds the keys strictly between splitters r-1 and r, bucket 2r+1 the keys
 * equal to splitter r.  d_start (2k+2 uint32) receives the bucket starts
 * (d_start[2k+1] = n).  The order inside a bucket is unspecified. */
HS_API int hs_multiway_partition_f64(double *keys, int64_t n, const uint64_t *d_splitters, int32_t k,
                                     uint32_t *d_start, void *stream);

/* The learned front end of a float64 sort on its own, for inspection (keys
 * are read, not changed): the training sample of 2^sample_log2 keys
 * (splitmix64(seed), with replacement) sorted by the plain method, the
 * held-out sample of 2^14 keys (splitmix64(seed + 1)), the model trained on
 * the sample's empirical CDF, its 255 splitters (for j = 1..255 the smallest
 * key of the sorted sample with F >= j/256, found by a 64-ary search over
 * the sample's ranks in fp32, before the running maximum), the sample's
 * order statistics (the key of rank floor(j * m / 256) of the sorted sample,
 * j = 1..255), and the judge: running maximum and de-duplication of the
 * model's splitters,
 * de-duplication of the order statistics, the bucket counts of both sets on
 * the held-out sample, their imbalance (largest non-equality bucket over
 * h/256) and the choice (the model unless its imbalance exceeds 1.25 times
 * the order statistics').  Same options and results as the learned sort's
 * front end (hs_opts.method is taken as HS_METHOD_LEARNED).
 * Outputs (device memory, caller-owned; totalOrder keys as uint64 words):
 *   d_params       1153 floats, the trained parameters;
 *   d_model_split  255 words, the model's splitters;
 *   d_sample_split 255 words, the order statistics;
 *   d_chosen       255 words, the first report->k are the chosen distinct
 *                  splitters;
 *   d_holdout      2^14 words, the held-out sample in draw order;
 *   d_train_sorted 2^sample_log2 doubles, the sorted training sample;
 *   d_counts       2 * 511 words: the held-out bucket counts of the model's
 *                  distinct splitters (bucket 2r: keys strictly between
 *                  splitters r-1 and r, 2r+1: keys equal to splitter r),
 *                  then those of the order statistics; unused entries 0;
 *   report         (host) feature normalisation mu and sd, the sample's
 *                  extreme keys, sizes, the judge's imbalances and choice,
 *                  and the loss after the last training step.
 * With HS_LEARN_FORCE_SAMPLE the model is not trained: d_params and
 * d_model_split are copied from uninitialised workspace and carry no
 * meaning, and the model imbalance is -1.  Returns once the work is done
 * (it reads the report back).  HS_EINVAL for n < 1 or a NULL pointer. */
typedef struct hs_learn_report {
    double scale;            /* the feature's scale s */
    double mu, sd;           /* the model's input is (asinh(x / s) - mu) / sd */
    uint64_t smin, smax;     /* totalOrder keys of the sample's smallest and largest key */
    int32_t m, h;            /* training and held-out sample sizes */
    int32_t k;               /* distinct splitters chosen */
    int32_t use_model;       /* 1: the model's splitters, 0: the order statistics */
    float model_imbalance, sample_imbalance, final_loss;
    int32_t reserved;
} hs_learn_report;
HS_API int hs_learn_debug_f64(const double *keys, int64_t n, const hs_opts *opts, float *d_params,
                              uint64_t *d_model_split, uint64_t *d_sample_split, uint64_t *d_chosen,
                              uint64_t *d_holdout, double *d_train_sorted, uint32_t *d_counts,
                              hs_learn_report *report, void *stream);

/* ---- Plans: one sort captured into a HIP graph -------------------------
 *
 * hs_plan_create prepares a sort of a fixed shape (op HS_OP_SORT_I32, _U32,
 * _I64, _F64, _KV_I32, _KV_F64, _SORT_SEGMENTED_I32 or _SORT_SEGMENTED_F64;
 * n keys; nseg segments for the segmented ops, ignored otherwise) and
 * allocates the plan's own workspace; it takes no buffers.  hs_plan_exec
 * sorts the caller's buffers (keys; vals only for key/value, d_offsets only
 * for segmented; each of the plan's shape) with the plan: the partition
 * levels run in the persistent driver and every clear is a kernel, so the
 * whole sort is one HIP graph launched on `stream`.  The graph is recorded
 * by the first hs_plan_exec and recorded again, and updated in place, when
 * a later call passes other buffers than the call before it; a replay on
 * the same buffers is only hipGraphLaunch.  The first call also tunes the
 * knobs when opts->autotune is set (hs_autotune on those buffers, persistent
 * driver) and, for segmented sorts, reads the offsets once to size the
 * recorded levels; it synchronizes `stream` for that.  Any later offsets
 * are correct too (the persistent driver finishes whatever levels remain).
 * Replays of one plan must not overlap (they share its workspace), and calls
 * on one plan must not run concurrently from several threads.
 * Errors: HS_EINVAL for a bad op, size or pointer, for in-place levels, the
 * host-driven level loop or a caller workspace in opts, and for a stream of
 * another device than the plan's; HS_ENOMEM if the workspace cannot be
 * allocated; HS_EHIP if recording or launching the graph fails. */
typedef struct hs_plan hs_plan;
HS_API int hs_plan_create(int op, int64_t n, int64_t nseg, const hs_opts *opts, hs_plan **plan);
HS_API int hs_plan_exec(hs_plan *plan, void *keys, int32_t *vals, const int64_t *d_offsets, void *stream);
/* Waits for the plan's last replay on `stream` and reports the error word
 * its kernels left (HS_EINTERNAL if set). */
HS_API int hs_plan_check(hs_plan *plan, void *stream);
HS_API void hs_plan_destroy(hs_plan *plan);

/* ---- Autotuner ---------------------------------------------------------
 *
 * Measures the sort of the given input (left unchanged: the tuner sorts a
 * copy) under every combination of on-chip limit local_T (2048, 4096, 8192,
 * up to the type's limit), one-wave bitonic bound leaf (the type's network
 * size L, L/2, L/4: 1024, 512, 256 for int32; 256, 128, 64 for float64
 * key/value; 512, 256, 128 otherwise) and global pivot rule
 * (ninther, sample median of 64), for the driver base->driver selects, with
 * HIP events (one warm-up and two timed runs each, fastest kept).  Every
 * candidate's output is compared on the device with the first candidate's:
 * all must be identical.  The best knobs go to *best (a copy of base with
 * them filled in) and are remembered per device, operation, method, driver
 * and size class (n and nseg rounded up to powers of two); a later call or a
 * sort with opts->autotune set reuses them.  Allocates a copy of the input. */
typedef struct hs_tune_report {
    int32_t candidates;      /* configurations measured (0: taken from the cache) */
    int32_t outputs_equal;   /* 1 if every candidate produced the same bytes */
    double best_ms;          /* fastest sort */
    double default_ms;       /* the sort with the default knobs */
    int32_t local_T, leaf, pivot_rule, reserved;
} hs_tune_report;
HS_API int hs_autotune(int op, void *keys, int32_t *vals, int64_t n, const int64_t *d_offsets, int64_t nseg,
                       const hs_opts *base, hs_opts *best, hs_tune_report *report, void *stream);

/* Bytes of workspace that operation `op` needs for n keys (and nseg
 * segments) with the given options.  With HSORT_GUARD=1 in the environment
 * (a debugging aid), every region of the workspace is followed by 256 guard
 * bytes that a sort fills before it runs and checks after it (a sort that
 * finds them changed returns HS_EINTERNAL); the size then includes them. */
HS_API int hs_workspace_size(int op, int64_t n, int64_t nseg, const hs_opts *opts, size_t *bytes);

/* Thread-local description of the last non-OK return ("" if none). */
HS_API const char *hs_last_error(void);

/* Library version, major*10000 + minor*100 + patch. */
HS_API int hs_version(void);

#ifdef __cplusplus
}
#endif

#endif /* HSORT_H */
