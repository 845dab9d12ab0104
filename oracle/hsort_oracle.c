/*
 * hsort_oracle.c -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, scalar CPU reference of the hybrid quicksort of Bramas,
 * "A Novel Hybrid Quicksort Algorithm Vectorized using AVX-512 on Intel
 * Skylake" (arXiv 1704.08579).  Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg may load this library.  It shares no code,
 * header, table or helper with the GPU library, and the GPU library never
 * links it.
 *
 * What is computed, and from where in the paper:
 *   - hybrid sort: quicksort on partitions larger than a bound, bitonic
 *     sorting network below it (Sec. III-C, Algorithm 4; Sec. III-A);
 *   - the bitonic network in its same-direction form (Sec. II-A, Fig. 2
 *     caption: every switch exchanges in the same direction; first the
 *     "extremities to the centre" boxes, then the linear boxes);
 *   - padding of a partial network with the greatest key (Sec. III-A,
 *     "Sorting Small Arrays");
 *   - partition with "<= pivot" on the left and the boundary as the result
 *     (Sec. III-B, Algorithm 3's contract);
 *   - key/value pairs moved together with their keys (Sec. III-D).
 *
 * Readings taken where the paper is silent or ambiguous (all listed in the
 * design notes of the repository):
 *   - Pivot = median of the first, middle and last element (Sec. IV-A names a
 *     3-value median "similar to the STL" without positions).
 *   - Equal keys: a three-way (<, ==, >) split, so runs of equal keys end the
 *     recursion.  On distinct keys this is the paper's two-way split with the
 *     pivot placed in its final slot; the two-way recursion of Algorithm 4
 *     shrinks an all-equal run by one element per level.
 *   - float64 keys are ordered by IEEE 754-2008 totalOrder (Sec. 5.10 of the
 *     standard) through the bit key K defined in oracle_key_f64().
 *   - Sort bound: partitions of at most `leaf` elements (256 by default, the
 *     paper's 16 vectors of 16 int32) go to the bitonic network.
 *
 * Element model: every key is mapped to an unsigned 64-bit "order key" whose
 * unsigned order is the key order (int32: sign bit flipped; float64: the
 * totalOrder key).  Comparisons act on that order key only; a value, when
 * present, travels with its key and never takes part in a comparison.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
    uint64_t key; /* order key */
    int32_t val;  /* payload (key/value sorts only) */
} elem_t;

/* ---- key maps ---------------------------------------------------------- */

/* int32 -> order key: flipping the sign bit maps two's-complement order onto
 * unsigned order (INT32_MIN -> 0, -1 -> 0x7fffffff, 0 -> 0x80000000). */
static uint64_t key_i32(int32_t x) { return (uint64_t)((uint32_t)x ^ 0x80000000u); }
static int32_t unkey_i32(uint64_t k) { return (int32_t)((uint32_t)k ^ 0x80000000u); }

/* uint32 -> order key: the value itself.  int64 -> order key: the sign bit
 * flipped, as for int32 (INT64_MIN -> 0, 0 -> 2^63). */
static uint64_t key_u32(uint32_t x) { return (uint64_t)x; }
static uint32_t unkey_u32(uint64_t k) { return (uint32_t)k; }
static uint64_t key_i64(int64_t x) { return (uint64_t)x ^ 0x8000000000000000ull; }
static int64_t unkey_i64(uint64_t k) { return (int64_t)(k ^ 0x8000000000000000ull); }

/* float64 bits -> totalOrder key.  Negative numbers (sign bit set) have all
 * bits inverted, so a larger magnitude gives a smaller key and -NaN lands
 * below -inf; non-negative numbers get the sign bit set, so they sit above
 * every negative number and keep their bit order (+0 < denormals < normals <
 * +inf < +NaN). */
uint64_t oracle_key_f64(uint64_t bits)
{
    if (bits >> 63) return ~bits;
    return bits | 0x8000000000000000ull;
}

uint64_t oracle_unkey_f64(uint64_t key)
{
    if (key >> 63) return key & 0x7fffffffffffffffull;
    return ~key;
}

/* ---- bitonic network (Sec. II-A, Sec. III-A) ---------------------------- */

static void cmp_swap(elem_t *a, int64_t i, int64_t j)
{
    /* i < j; the lower index receives the smaller key.  Swap only when the
     * keys are strictly out of order, so equal keys keep their slots. */
    if (a[i].key > a[j].key) {
        elem_t t = a[i];
        a[i] = a[j];
        a[j] = t;
    }
}

/* Same-direction bitonic network over N = 2^logn elements.  Stage s merges
 * sorted runs of length 2^(s-1) into runs of 2^s: first every i with bit
 * (s-1) clear meets its mirror image i ^ (2^s - 1) inside the run
 * ("extremities to the centre"), then half-cleaners at distance 2^(s-2),
 * ..., 1 ("linear progression"). */
static void bitonic_network(elem_t *a, int logn)
{
    int64_t n = (int64_t)1 << logn;
    for (int s = 1; s <= logn; ++s) {
        int64_t m = ((int64_t)1 << s) - 1;
        for (int64_t i = 0; i < n; ++i)
            if (!(i & ((int64_t)1 << (s - 1)))) cmp_swap(a, i, i ^ m);
        for (int t = s - 2; t >= 0; --t) {
            int64_t d = (int64_t)1 << t;
            for (int64_t i = 0; i < n; ++i)
                if (!(i & d)) cmp_swap(a, i, i | d);
        }
    }
}

/* The network for a partial array: copy into a power-of-two buffer padded
 * with the greatest key, run the network, copy the first n back. */
static void bitonic_small(elem_t *a, int64_t n)
{
    if (n <= 1) return;
    int logn = 0;
    while (((int64_t)1 << logn) < n) ++logn;
    int64_t big = (int64_t)1 << logn;
    elem_t *buf = (elem_t *)malloc((size_t)big * sizeof(elem_t));
    memcpy(buf, a, (size_t)n * sizeof(elem_t));
    for (int64_t i = n; i < big; ++i) {
        buf[i].key = UINT64_MAX;
        buf[i].val = 0;
    }
    bitonic_network(buf, logn);
    memcpy(a, buf, (size_t)n * sizeof(elem_t));
    free(buf);
}

/* ---- hybrid quicksort (Sec. III-C, Algorithm 4) ------------------------- */

static uint64_t median3(uint64_t x, uint64_t y, uint64_t z)
{
    if (x > y) { uint64_t t = x; x = y; y = t; }
    if (y > z) { uint64_t t = y; y = z; z = t; }
    if (x > y) { uint64_t t = x; x = y; y = t; }
    return y;
}

static void swap_el(elem_t *a, int64_t i, int64_t j)
{
    elem_t t = a[i];
    a[i] = a[j];
    a[j] = t;
}

typedef struct {
    int64_t leaf;       /* partitions of <= leaf elements are bitonic-sorted */
    int64_t max_depth;  /* deepest partition level reached */
    int64_t partitions; /* number of partition calls */
} qs_ctx;

/* Sort a[lo..hi] (inclusive).  Partition while the range holds more than
 * `leaf` elements, then hand it to the bitonic network.  The larger side is
 * handled by the loop and the smaller by recursion, so the stack stays
 * logarithmic. */
static void hybrid(elem_t *a, int64_t lo, int64_t hi, int64_t depth, qs_ctx *c)
{
    while (hi - lo + 1 > c->leaf) {
        if (depth + 1 > c->max_depth) c->max_depth = depth + 1;
        c->partitions++;
        uint64_t p = median3(a[lo].key, a[lo + (hi - lo) / 2].key, a[hi].key);
        /* three-way split: [lo, lt) < p, [lt, gt] == p, (gt, hi] > p */
        int64_t lt = lo, i = lo, gt = hi;
        while (i <= gt) {
            if (a[i].key < p)
                swap_el(a, lt++, i++);
            else if (a[i].key > p)
                swap_el(a, i, gt--);
            else
                ++i;
        }
        ++depth;
        if (lt - lo < hi - gt) {
            hybrid(a, lo, lt - 1, depth, c);
            lo = gt + 1;
        } else {
            hybrid(a, gt + 1, hi, depth, c);
            hi = lt - 1;
        }
    }
    if (hi > lo) bitonic_small(a + lo, hi - lo + 1);
}

static int64_t sort_elems(elem_t *a, int64_t n, int64_t leaf)
{
    qs_ctx c = {leaf < 1 ? 1 : leaf, 0, 0};
    if (n > 1) hybrid(a, 0, n - 1, 0, &c);
    return c.max_depth;
}

/* ---- public entry points ------------------------------------------------ */

/* Each returns the number of partition levels on the deepest path (0 when
 * the whole array went straight to the network), or -1 on allocation
 * failure.  `leaf` is the sort bound: ranges of at most `leaf` elements are
 * handed to the bitonic network (256 reproduces the paper's bound). */

int64_t oracle_sort_i32(int32_t *keys, int64_t n, int64_t leaf)
{
    elem_t *a = (elem_t *)malloc((size_t)(n > 0 ? n : 1) * sizeof(elem_t));
    if (!a) return -1;
    for (int64_t i = 0; i < n; ++i) {
        a[i].key = key_i32(keys[i]);
        a[i].val = 0;
    }
    int64_t d = sort_elems(a, n, leaf);
    for (int64_t i = 0; i < n; ++i) keys[i] = unkey_i32(a[i].key);
    free(a);
    return d;
}

int64_t oracle_sort_f64(uint64_t *bits, int64_t n, int64_t leaf)
{
    elem_t *a = (elem_t *)malloc((size_t)(n > 0 ? n : 1) * sizeof(elem_t));
    if (!a) return -1;
    for (int64_t i = 0; i < n; ++i) {
        a[i].key = oracle_key_f64(bits[i]);
        a[i].val = 0;
    }
    int64_t d = sort_elems(a, n, leaf);
    for (int64_t i = 0; i < n; ++i) bits[i] = oracle_unkey_f64(a[i].key);
    free(a);
    return d;
}

int64_t oracle_sort_u32(uint32_t *keys, int64_t n, int64_t leaf)
{
    elem_t *a = (elem_t *)malloc((size_t)(n > 0 ? n : 1) * sizeof(elem_t));
    if (!a) return -1;
    for (int64_t i = 0; i < n; ++i) {
        a[i].key = key_u32(keys[i]);
        a[i].val = 0;
    }
    int64_t d = sort_elems(a, n, leaf);
    for (int64_t i = 0; i < n; ++i) keys[i] = unkey_u32(a[i].key);
    free(a);
    return d;
}

int64_t oracle_sort_i64(int64_t *keys, int64_t n, int64_t leaf)
{
    elem_t *a = (elem_t *)malloc((size_t)(n > 0 ? n : 1) * sizeof(elem_t));
    if (!a) return -1;
    for (int64_t i = 0; i < n; ++i) {
        a[i].key = key_i64(keys[i]);
        a[i].val = 0;
    }
    int64_t d = sort_elems(a, n, leaf);
    for (int64_t i = 0; i < n; ++i) keys[i] = unkey_i64(a[i].key);
    free(a);
    return d;
}

/* Stable argsort by definition: sort the pairs (key, position) -- as one
 * order key, the int32 key's order word above the position -- and read the
 * positions back.  n < 2^31. */
int64_t oracle_argsort_i32(int32_t *keys, int32_t *idx, int64_t n, int64_t leaf)
{
    elem_t *a = (elem_t *)malloc((size_t)(n > 0 ? n : 1) * sizeof(elem_t));
    if (!a) return -1;
    for (int64_t i = 0; i < n; ++i) {
        a[i].key = (key_i32(keys[i]) << 32) | (uint64_t)i;
        a[i].val = 0;
    }
    int64_t d = sort_elems(a, n, leaf);
    for (int64_t i = 0; i < n; ++i) {
        keys[i] = unkey_i32(a[i].key >> 32);
        idx[i] = (int32_t)(uint32_t)a[i].key;
    }
    free(a);
    return d;
}

int64_t oracle_sort_kv_i32(int32_t *keys, int32_t *vals, int64_t n, int64_t leaf)
{
    elem_t *a = (elem_t *)malloc((size_t)(n > 0 ? n : 1) * sizeof(elem_t));
    if (!a) return -1;
    for (int64_t i = 0; i < n; ++i) {
        a[i].key = key_i32(keys[i]);
        a[i].val = vals[i];
    }
    int64_t d = sort_elems(a, n, leaf);
    for (int64_t i = 0; i < n; ++i) {
        keys[i] = unkey_i32(a[i].key);
        vals[i] = a[i].val;
    }
    free(a);
    return d;
}

/* Key/value pairs with float64 keys (Sec. III-D): the value travels with
 * the key's totalOrder key and never takes part in a comparison, so equal
 * keys leave their values in whatever order the method produced. */
int64_t oracle_sort_kv_f64(uint64_t *bits, int32_t *vals, int64_t n, int64_t leaf)
{
    elem_t *a = (elem_t *)malloc((size_t)(n > 0 ? n : 1) * sizeof(elem_t));
    if (!a) return -1;
    for (int64_t i = 0; i < n; ++i) {
        a[i].key = oracle_key_f64(bits[i]);
        a[i].val = vals[i];
    }
    int64_t d = sort_elems(a, n, leaf);
    for (int64_t i = 0; i < n; ++i) {
        bits[i] = oracle_unkey_f64(a[i].key);
        vals[i] = a[i].val;
    }
    free(a);
    return d;
}

/* Stable argsort of float64 keys by definition: the pairs (key, position)
 * in lexicographic order.  The key/value sort above (Sec. III-D) orders the
 * keys; every run of equal keys (equal bits) then has its positions put in
 * ascending order (insertion sort over the run). */
int64_t oracle_argsort_f64(uint64_t *bits, int32_t *idx, int64_t n, int64_t leaf)
{
    for (int64_t i = 0; i < n; ++i) idx[i] = (int32_t)i;
    int64_t d = oracle_sort_kv_f64(bits, idx, n, leaf);
    if (d < 0) return d;
    for (int64_t lo = 0; lo < n;) {
        int64_t hi = lo + 1;
        while (hi < n && bits[hi] == bits[lo]) ++hi;
        for (int64_t i = lo + 1; i < hi; ++i) {
            const int32_t v = idx[i];
            int64_t j = i - 1;
            while (j >= lo && idx[j] > v) {
                idx[j + 1] = idx[j];
                --j;
            }
            idx[j + 1] = v;
        }
        lo = hi;
    }
    return d;
}

/* Segmented sort: every [off[i], off[i+1]) is sorted on its own. */
int64_t oracle_sort_segmented_i32(int32_t *keys, const int64_t *off, int64_t nseg,
                                  int64_t leaf)
{
    int64_t dmax = 0;
    for (int64_t s = 0; s < nseg; ++s) {
        int64_t d = oracle_sort_i32(keys + off[s], off[s + 1] - off[s], leaf);
        if (d < 0) return -1;
        if (d > dmax) dmax = d;
    }
    return dmax;
}

int64_t oracle_sort_segmented_f64(uint64_t *bits, const int64_t *off, int64_t nseg, int64_t leaf)
{
    int64_t dmax = 0;
    for (int64_t s = 0; s < nseg; ++s) {
        int64_t d = oracle_sort_f64(bits + off[s], off[s + 1] - off[s], leaf);
        if (d < 0) return -1;
        if (d > dmax) dmax = d;
    }
    return dmax;
}

/* Partition contract of Algorithm 3: afterwards keys[0,k) <= pivot < keys[k,n)
 * and k is returned.  One pass with a read cursor and a write cursor. */
int64_t oracle_partition_le_i32(int32_t *keys, int64_t n, int32_t pivot)
{
    int64_t w = 0;
    for (int64_t r = 0; r < n; ++r) {
        if (keys[r] <= pivot) {
            int32_t t = keys[w];
            keys[w] = keys[r];
            keys[r] = t;
            ++w;
        }
    }
    return w;
}

/* ---- network checks (0-1 principle) ------------------------------------- */

/* Apply the same-direction network to N = 2^logn order keys (and values). */
void oracle_bitonic_apply(uint64_t *keys, int32_t *vals, int logn)
{
    int64_t n = (int64_t)1 << logn;
    elem_t *a = (elem_t *)malloc((size_t)n * sizeof(elem_t));
    for (int64_t i = 0; i < n; ++i) {
        a[i].key = keys[i];
        a[i].val = vals ? vals[i] : 0;
    }
    bitonic_network(a, logn);
    for (int64_t i = 0; i < n; ++i) {
        keys[i] = a[i].key;
        if (vals) vals[i] = a[i].val;
    }
    free(a);
}

/* 0-1 check of the last stage alone (the merger of two sorted halves): all
 * (N/2+1)^2 inputs made of an ascending 0-1 lower half with z0 zeros and an
 * ascending 0-1 upper half with z1 zeros.  Counts unsorted outputs. */
int64_t oracle_bitonic_merger_failures(int logn)
{
    if (logn < 1 || logn > 24) return -1;
    int64_t n = (int64_t)1 << logn, h = n / 2;
    elem_t *a = (elem_t *)malloc((size_t)n * sizeof(elem_t));
    int64_t fails = 0;
    int s = logn;
    int64_t m = n - 1;
    for (int64_t z0 = 0; z0 <= h; ++z0) {
        for (int64_t z1 = 0; z1 <= h; ++z1) {
            for (int64_t i = 0; i < h; ++i) a[i].key = i < z0 ? 0 : 1;
            for (int64_t i = 0; i < h; ++i) a[h + i].key = i < z1 ? 0 : 1;
            for (int64_t i = 0; i < n; ++i)
                if (!(i & ((int64_t)1 << (s - 1)))) cmp_swap(a, i, i ^ m);
            for (int t = s - 2; t >= 0; --t) {
                int64_t d = (int64_t)1 << t;
                for (int64_t i = 0; i < n; ++i)
                    if (!(i & d)) cmp_swap(a, i, i | d);
            }
            for (int64_t i = 1; i < n; ++i)
                if (a[i - 1].key > a[i].key) {
                    ++fails;
                    break;
                }
        }
    }
    free(a);
    return fails;
}

/* Run the network on every 0-1 input of N = 2^logn lines, logn in [0, 4]
 * (all 2^N inputs) and count outputs that are not sorted.  By the 0-1
 * principle a comparator network sorts every input iff it sorts every 0-1
 * input. */
int64_t oracle_bitonic_exhaustive_failures(int logn)
{
    if (logn < 0 || logn > 4) return -1;
    int64_t n = (int64_t)1 << logn;
    elem_t a[16];
    int64_t fails = 0;
    for (uint64_t m = 0; m < ((uint64_t)1 << n); ++m) {
        for (int64_t i = 0; i < n; ++i) {
            a[i].key = (m >> i) & 1;
            a[i].val = 0;
        }
        bitonic_network(a, logn);
        for (int64_t i = 1; i < n; ++i)
            if (a[i - 1].key > a[i].key) {
                ++fails;
                break;
            }
    }
    return fails;
}
