// hs_kernels.hpp -- HIP kernels of the gfx950 hybrid quicksort.
//
// The method (Sec. III-C, Algorithm 4) partitions every range larger than a
// bound around a pivot (Sec. III-B, Algorithm 3) and sorts small ranges with
// a bitonic network (Sec. III-A).  On the GPU the recursion is laid out in
// two tiers:
//
//   global levels   every segment larger than the on-chip limit T is
//                   partitioned out of place, tile by tile, into the other
//                   half of a ping-pong pair of buffers (k_partition); each
//                   tile plays the role of one of Algorithm 3's vector steps:
//                   a wavefront ballot/prefix-sum replaces the compress-store,
//                   and one 64-bit atomic per tile reserves the tile's slots
//                   from the segment's front (<= pivot) and back (> pivot)
//                   write cursors, like Algorithm 3's left_w / right_w;
//   on-chip tier    segments of at most T keys are sorted by one workgroup
//                   in LDS (k_local): three-way partition levels over all
//                   live sub-ranges at once, then the bitonic network in
//                   VGPRs for every sub-range of at most LEAF keys.
//
// All kernels compare unsigned order words (see hs_device.hpp); the caller's
// format is decoded on the first read and re-encoded on the final store.
#pragma once

#include "hs_device.hpp"

namespace hs {

// ---------------------------------------------------------------- shared types

constexpr uint32_t SEG_STRICT = 1u;  // partition with "<" (the ">=" side is all == pivot)
constexpr uint32_t SEG_UB = 2u;      // ub holds an upper bound of every key in the segment

constexpr uint32_t TASK_LOCAL = 0u;  // sort the range on chip
constexpr uint32_t TASK_FILL = 1u;   // every key of the range equals `fill`

constexpr uint32_t SRC_BUF0 = 0u, SRC_BUF1 = 1u, SRC_RAW = 2u;

constexpr uint32_t ERR_CURSOR = 1u;    // a segment's cursors do not add up
constexpr uint32_t ERR_CAND_CAP = 2u;  // segment list overflow
constexpr uint32_t ERR_TASK_CAP = 4u;  // task list overflow
constexpr uint32_t ERR_OFFSETS = 8u;   // segment offsets outside [0, n_total] or decreasing

constexpr int PIVOT_MEDIAN3 = 1, PIVOT_NINTHER = 2, PIVOT_SAMPLE = 3;

template <typename K> struct Seg {
    uint32_t b, e;    // element range [b, e)
    uint32_t tile0;   // first tile of this segment in the level's tile space
    uint32_t flags;   // SEG_*
    K piv, ub;
};

template <typename K> struct Task {
    uint32_t b, e;
    uint32_t src;   // SRC_*: where the keys of the range are now
    uint32_t kind;  // TASK_*
    K fill;
};

// Control block of one call, in device memory.
struct Ctl {
    uint32_t nseg;       // segments in the current level list
    uint32_t ntiles;     // tiles of the current level
    uint32_t ncand;      // segments written for the next level
    uint32_t ntask;      // tasks written
    uint32_t task_next;  // dynamic task counter of k_local
    uint32_t err;        // ERR_* bits
    unsigned long long level_keys;  // keys in the current level's segments
    unsigned long long local_keys;  // keys handed to local tasks
    unsigned long long fill_keys;   // keys handed to fill tasks
    unsigned long long pad[2];
};

// ---------------------------------------------------------------- tile geometry

template <typename K> struct PartCfg;
template <> struct PartCfg<uint32_t> { static constexpr int NT = 256, TILE = 4096; };
template <> struct PartCfg<uint64_t> { static constexpr int NT = 256, TILE = 2048; };

// Tiles are aligned to absolute multiples of TILE, so the interior tiles of a
// segment are full and 16-byte aligned (for 16-byte-aligned buffers).
template <typename K>
__device__ __host__ __forceinline__ uint32_t seg_tiles(uint32_t b, uint32_t e)
{
    constexpr uint32_t TILE = PartCfg<K>::TILE;
    return (e + TILE - 1) / TILE - b / TILE;
}

// ---------------------------------------------------------------- pivot choice

// Key readers: an internal buffer of order words, or the caller's arrays.
template <int F> struct SrcReader {
    using K = typename KeyOf<F>::type;
    const K *buf;
    Raw raw;
    bool is_raw;
    __device__ __forceinline__ K operator()(uint32_t i) const { return is_raw ? raw_load<F>(raw, i) : buf[i]; }
};

template <typename K> __device__ __forceinline__ K med3(K a, K b, K c)
{
    if (a > b) { K t = a; a = b; b = t; }
    if (b > c) { K t = b; b = c; c = t; }
    if (a > b) { K t = a; a = b; b = t; }
    return b;
}

// Pivot of [b, e) (e - b >= 2).  MEDIAN3 takes the first, middle and last
// key (the 3-value median of Sec. IV-A at the positions of Appendix A's
// middle rule); NINTHER the median of three such medians over nine evenly
// spaced keys; SAMPLE the median of 31 evenly spaced keys.  The choice only
// changes how many levels run, never the output.
template <typename K, typename Rd>
__device__ K pick_pivot(const Rd &rd, uint32_t b, uint32_t e, int rule)
{
    const uint32_t m = e - b;
    if (rule == PIVOT_MEDIAN3 || m < 64) return med3<K>(rd(b), rd(b + (m - 1) / 2), rd(e - 1));
    if (rule == PIVOT_NINTHER) {
        K v[9];
#pragma unroll
        for (int i = 0; i < 9; ++i) v[i] = rd(b + (uint32_t)(((uint64_t)(m - 1) * i) / 8));
        return med3<K>(med3<K>(v[0], v[1], v[2]), med3<K>(v[3], v[4], v[5]), med3<K>(v[6], v[7], v[8]));
    }
    constexpr int NS = 31;
    K v[NS];
    for (int i = 0; i < NS; ++i) v[i] = rd(b + (uint32_t)(((uint64_t)(m - 1) * i) / (NS - 1)));
    for (int i = 1; i < NS; ++i) {  // insertion sort of the sample
        K x = v[i];
        int j = i - 1;
        while (j >= 0 && v[j] > x) {
            v[j + 1] = v[j];
            --j;
        }
        v[j + 1] = x;
    }
    return v[NS / 2];
}

// ---------------------------------------------------------------- init

// One array: the whole range becomes a level-0 segment, or a single local
// task when it fits on chip.
template <int F>
__global__ void k_init_single(Ctl *ctl, Seg<typename KeyOf<F>::type> *cand, Task<typename KeyOf<F>::type> *tasks,
                              Raw raw, uint32_t n, uint32_t T, int rule, int has_pivot,
                              typename KeyOf<F>::type user_pivot)
{
    using K = typename KeyOf<F>::type;
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    if (n <= T && !has_pivot) {
        if (n >= 2) {
            Task<K> t;
            t.b = 0;
            t.e = n;
            t.src = SRC_RAW;
            t.kind = TASK_LOCAL;
            t.fill = 0;
            tasks[0] = t;
            ctl->ntask = 1;
            ctl->local_keys = n;
        }
        return;
    }
    Seg<K> s;
    s.b = 0;
    s.e = n;
    s.tile0 = 0;
    s.flags = 0;
    s.ub = 0;
    if (has_pivot) {
        s.piv = user_pivot;
    } else {
        SrcReader<F> rd{nullptr, raw, true};
        s.piv = pick_pivot<K>(rd, 0, n, rule);
    }
    cand[0] = s;
    ctl->ncand = 1;
}

// Many arrays: thread i routes segment i [off[i], off[i+1]).
template <int F>
__global__ void k_init_segmented(Ctl *ctl, Seg<typename KeyOf<F>::type> *cand,
                                 Task<typename KeyOf<F>::type> *tasks, Raw raw, const int64_t *off,
                                 uint32_t nseg, uint32_t n_total, uint32_t T, int rule, uint32_t cand_cap,
                                 uint32_t task_cap)
{
    using K = typename KeyOf<F>::type;
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nseg) return;
    const int64_t b64 = off[i], e64 = off[i + 1];
    if (b64 < 0 || e64 > (int64_t)n_total || e64 < b64) {  // malformed offsets: skip and flag
        atomicOr(&ctl->err, ERR_OFFSETS);
        return;
    }
    const uint32_t b = (uint32_t)b64, e = (uint32_t)e64;
    if (e <= b + 1) return;  // empty or single key: already in place
    const uint32_t m = e - b;
    if (m <= T) {
        const uint32_t k = atomicAdd(&ctl->ntask, 1u);
        if (k >= task_cap) {
            atomicOr(&ctl->err, ERR_TASK_CAP);
            return;
        }
        Task<K> t;
        t.b = b;
        t.e = e;
        t.src = SRC_RAW;
        t.kind = TASK_LOCAL;
        t.fill = 0;
        tasks[k] = t;
        atomicAdd(&ctl->local_keys, (unsigned long long)m);
        return;
    }
    Seg<K> s;
    s.b = b;
    s.e = e;
    s.tile0 = 0;
    s.flags = 0;
    s.ub = 0;
    SrcReader<F> rd{nullptr, raw, true};
    s.piv = pick_pivot<K>(rd, b, e, rule);
    const uint32_t k = atomicAdd(&ctl->ncand, 1u);
    if (k >= cand_cap) {
        atomicOr(&ctl->err, ERR_CAND_CAP);
        return;
    }
    cand[k] = s;
}

// ---------------------------------------------------------------- plan

// One workgroup: turn the candidate list into the level list (exclusive scan
// of tile counts), zero the write cursors, publish the level's sizes.
template <typename K>
__global__ __launch_bounds__(1024) void k_plan(Ctl *ctl, Seg<K> *segs, unsigned long long *cur, uint32_t cap)
{
    __shared__ uint32_t wsum[16];
    __shared__ unsigned long long wkeys[16];
    const uint32_t n = min(ctl->ncand, cap);  // an overflow is flagged in err; never read past the list
    const int tid = threadIdx.x, lane = lane_id(), wave = tid / WAVE;
    const int nw = blockDim.x / WAVE;
    uint32_t carry = 0;
    unsigned long long keys = 0;
    for (uint32_t base = 0; base < n; base += blockDim.x) {
        const uint32_t i = base + tid;
        uint32_t nt = 0, sz = 0;
        if (i < n) {
            nt = seg_tiles<K>(segs[i].b, segs[i].e);
            sz = segs[i].e - segs[i].b;
        }
        const uint32_t incl = wave_incl_scan(nt);
        unsigned long long ks = sz;
        for (int d = 1; d < WAVE; d <<= 1) ks += __shfl_xor(ks, d);
        if (lane == WAVE - 1) wsum[wave] = incl;
        if (lane == 0) wkeys[wave] = ks;
        __syncthreads();
        uint32_t pre = 0, tot = 0;
        unsigned long long ksum = 0;
        for (int w = 0; w < nw; ++w) {
            if (w < wave) pre += wsum[w];
            tot += wsum[w];
            ksum += wkeys[w];
        }
        if (i < n) {
            segs[i].tile0 = carry + pre + incl - nt;
            cur[i] = 0ull;
        }
        carry += tot;
        keys += ksum;
        __syncthreads();
    }
    if (tid == 0) {
        ctl->nseg = n;
        ctl->ntiles = carry;
        ctl->ncand = 0;
        ctl->level_keys = keys;
    }
}

// ---------------------------------------------------------------- partition pass

// One level of out-of-place partitioning.  Workgroup g owns a contiguous run
// of the level's tiles.  Per tile: load (16 B per lane per load, coalesced),
// compare with the segment's pivot, count the <= side and the > side per
// thread, scan the counts across the workgroup, reserve both slot runs with
// one 64-bit atomic on the segment's cursor word (low half: front cursor,
// high half: back cursor), compact the tile in LDS (<= keys first), and
// write both runs out with consecutive lanes on consecutive addresses.
template <int F, bool SRC_IS_RAW, bool DST_IS_RAW>
__global__ __launch_bounds__(256) void k_partition(const Ctl *ctl, const Seg<typename KeyOf<F>::type> *segs,
                                                   unsigned long long *cur, const typename KeyOf<F>::type *src,
                                                   Raw raw, typename KeyOf<F>::type *dst, Raw raw_dst,
                                                   int aligned)
{
    using K = typename KeyOf<F>::type;
    constexpr int NT = PartCfg<K>::NT, TILE = PartCfg<K>::TILE, ITEMS = TILE / NT;
    constexpr int NW = NT / WAVE;
    static_assert(ITEMS <= 32, "item masks are 32-bit");
    __shared__ K stage[TILE];
    __shared__ uint32_t wsum[NW];
    __shared__ uint32_t sbase[2];

    const uint32_t ntiles = ctl->ntiles, nseg = ctl->nseg;
    const uint32_t per = (ntiles + gridDim.x - 1) / gridDim.x;
    uint32_t t = blockIdx.x * per;
    const uint32_t tend = min(ntiles, t + per);
    if (t >= tend) return;
    const int tid = threadIdx.x, lane = lane_id(), wave = tid / WAVE;

    uint32_t lo = 0, hi = nseg;
    while (hi - lo > 1) {
        const uint32_t mid = (lo + hi) >> 1;
        if (segs[mid].tile0 <= t) lo = mid; else hi = mid;
    }
    uint32_t s = lo;
    Seg<K> sg = segs[s];
    uint32_t next0 = (s + 1 < nseg) ? segs[s + 1].tile0 : ntiles;

    for (; t < tend; ++t) {
        while (t >= next0) {
            ++s;
            sg = segs[s];
            next0 = (s + 1 < nseg) ? segs[s + 1].tile0 : ntiles;
        }
        const uint32_t a = sg.b / TILE + (t - sg.tile0);
        const uint32_t p0 = max(sg.b, a * TILE);
        const uint32_t cnt = min(sg.e, (a + 1) * TILE) - p0;
        const bool full = aligned && cnt == (uint32_t)TILE;

        K x[ITEMS];
        if (full) {
            if constexpr (F == FMT_KV && SRC_IS_RAW) {
                const uint4 *kp = (const uint4 *)((const uint32_t *)raw.keys + p0);
                const uint4 *vp = (const uint4 *)((const uint32_t *)raw.vals + p0);
#pragma unroll
                for (int j = 0; j < ITEMS / 4; ++j) {
                    const uint4 kk = kp[j * NT + tid], vv = vp[j * NT + tid];
                    x[4 * j + 0] = enc_kv(kk.x, vv.x);
                    x[4 * j + 1] = enc_kv(kk.y, vv.y);
                    x[4 * j + 2] = enc_kv(kk.z, vv.z);
                    x[4 * j + 3] = enc_kv(kk.w, vv.w);
                }
            } else if constexpr (sizeof(K) == 4) {
                const uint4 *pp = (const uint4 *)((SRC_IS_RAW ? (const K *)raw.keys : src) + p0);
#pragma unroll
                for (int j = 0; j < ITEMS / 4; ++j) {
                    const uint4 v = pp[j * NT + tid];
                    x[4 * j + 0] = v.x;
                    x[4 * j + 1] = v.y;
                    x[4 * j + 2] = v.z;
                    x[4 * j + 3] = v.w;
                }
                if constexpr (SRC_IS_RAW) {
#pragma unroll
                    for (int j = 0; j < ITEMS; ++j) x[j] = (K)enc_i32((uint32_t)x[j]);
                }
            } else {
                const ulonglong2 *pp = (const ulonglong2 *)((SRC_IS_RAW ? (const K *)raw.keys : src) + p0);
#pragma unroll
                for (int j = 0; j < ITEMS / 2; ++j) {
                    const ulonglong2 v = pp[j * NT + tid];
                    x[2 * j + 0] = v.x;
                    x[2 * j + 1] = v.y;
                }
                if constexpr (SRC_IS_RAW) {
#pragma unroll
                    for (int j = 0; j < ITEMS; ++j) x[j] = (K)enc_f64((uint64_t)x[j]);
                }
            }
        } else {
#pragma unroll
            for (int j = 0; j < ITEMS; ++j) {
                const uint32_t i = (uint32_t)(j * NT + tid);
                if (i < cnt) {
                    if constexpr (SRC_IS_RAW) x[j] = raw_load<F>(raw, p0 + i);
                    else x[j] = src[p0 + i];
                } else {
                    x[j] = 0;
                }
            }
        }

        const bool strict = (sg.flags & SEG_STRICT) != 0;
        const K piv = sg.piv;
        uint32_t lemask = 0, cle = 0, cgt = 0;
#pragma unroll
        for (int j = 0; j < ITEMS; ++j) {
            const bool valid = full || (uint32_t)(j * NT + tid) < cnt;
            const bool le = strict ? (x[j] < piv) : (x[j] <= piv);
            if (valid) {
                if (le) {
                    lemask |= 1u << j;
                    ++cle;
                } else {
                    ++cgt;
                }
            }
        }
        const uint32_t code = cle | (cgt << 16);
        const uint32_t incl = wave_incl_scan(code);
        if (lane == WAVE - 1) wsum[wave] = incl;
        __syncthreads();
        uint32_t pre = 0, tot = 0;
#pragma unroll
        for (int w = 0; w < NW; ++w) {
            const uint32_t v = wsum[w];
            if (w < wave) pre += v;
            tot += v;
        }
        const uint32_t excl = pre + incl - code;
        const uint32_t tot_le = tot & 0xFFFFu, tot_gt = tot >> 16;
        if (tid == 0) {
            const unsigned long long old =
                atomicAdd(&cur[s], (unsigned long long)tot_le | ((unsigned long long)tot_gt << 32));
            sbase[0] = sg.b + (uint32_t)old;
            sbase[1] = sg.e - (uint32_t)(old >> 32) - tot_gt;
        }
        uint32_t lp = excl & 0xFFFFu, gp = tot_le + (excl >> 16);
#pragma unroll
        for (int j = 0; j < ITEMS; ++j) {
            const bool valid = full || (uint32_t)(j * NT + tid) < cnt;
            if (valid) {
                if (lemask & (1u << j)) stage[lp++] = x[j];
                else stage[gp++] = x[j];
            }
        }
        __syncthreads();
        const uint32_t lt_base = sbase[0], gt_base = sbase[1];
        for (uint32_t i = tid; i < cnt; i += NT) {
            const K v = stage[i];
            const uint32_t pos = i < tot_le ? lt_base + i : gt_base + (i - tot_le);
            if constexpr (DST_IS_RAW) raw_store<F>(raw_dst, pos, v);
            else dst[pos] = v;
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------- finalize

// One thread per segment of the level: split it at its front cursor (the
// count of the <= side, Algorithm 3's left_w) and route both children.  A
// child larger than T becomes a segment of the next level with its own
// pivot; a smaller child becomes a local task; the ">=" child of a strict
// split holds only keys equal to the pivot and becomes a fill task.
//
// Equal keys: a left child inherits its parent's pivot as an upper bound.
// When a segment's pivot equals that bound, the segment is split with "<"
// instead of "<=", which moves every copy of the bound into a final range.
// This keeps runs of equal keys from being re-partitioned level after level.
template <int F>
__global__ __launch_bounds__(256) void k_finalize(Ctl *ctl, const Seg<typename KeyOf<F>::type> *segs,
                                                  const unsigned long long *cur,
                                                  Seg<typename KeyOf<F>::type> *cand,
                                                  Task<typename KeyOf<F>::type> *tasks,
                                                  const typename KeyOf<F>::type *out, uint32_t out_id,
                                                  uint32_t T, int rule, uint32_t cand_cap, uint32_t task_cap)
{
    using K = typename KeyOf<F>::type;
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= ctl->nseg) return;
    const Seg<K> sg = segs[i];
    const unsigned long long c = cur[i];
    const uint32_t nle = (uint32_t)c, ngt = (uint32_t)(c >> 32);
    if (nle + ngt != sg.e - sg.b) {
        atomicOr(&ctl->err, ERR_CURSOR);
        return;
    }
    const uint32_t mid = sg.b + nle;
    const bool strict = (sg.flags & SEG_STRICT) != 0;
    SrcReader<F> rd{out, Raw{nullptr, nullptr}, false};

    auto emit_task = [&](uint32_t b, uint32_t e, uint32_t kind, K fill) {
        const uint32_t k = atomicAdd(&ctl->ntask, 1u);
        if (k >= task_cap) {
            atomicOr(&ctl->err, ERR_TASK_CAP);
            return;
        }
        Task<K> t;
        t.b = b;
        t.e = e;
        t.src = out_id;
        t.kind = kind;
        t.fill = fill;
        tasks[k] = t;
        atomicAdd(kind == TASK_FILL ? &ctl->fill_keys : &ctl->local_keys, (unsigned long long)(e - b));
    };
    auto emit_child = [&](uint32_t b, uint32_t e, uint32_t flags, K ub) {
        const uint32_t m = e - b;
        if (m == 0) return;
        if (m <= T) {
            emit_task(b, e, TASK_LOCAL, 0);
            return;
        }
        Seg<K> ch;
        ch.b = b;
        ch.e = e;
        ch.tile0 = 0;
        ch.ub = ub;
        ch.piv = pick_pivot<K>(rd, b, e, rule);
        ch.flags = flags;
        if ((flags & SEG_UB) && ch.piv == ub) ch.flags |= SEG_STRICT;
        const uint32_t k = atomicAdd(&ctl->ncand, 1u);
        if (k >= cand_cap) {
            atomicOr(&ctl->err, ERR_CAND_CAP);
            return;
        }
        cand[k] = ch;
    };

    if (strict) {
        emit_child(sg.b, mid, 0u, 0);                        // keys < pivot
        if (sg.e > mid) emit_task(mid, sg.e, TASK_FILL, sg.piv);  // keys == pivot
    } else {
        emit_child(sg.b, mid, SEG_UB, sg.piv);               // keys <= pivot
        emit_child(mid, sg.e, sg.flags & SEG_UB, sg.ub);     // keys > pivot
    }
}

// Count of the <= side after a single-segment pass (partition entry point).
__global__ void k_write_count(const unsigned long long *cur, int64_t *d_count)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) *d_count = (int64_t)(uint32_t)cur[0];
}

// ---------------------------------------------------------------- on-chip sort

template <typename K> struct LocalCfg;
template <> struct LocalCfg<uint32_t> { static constexpr int T = 16384, NT = 1024, KPT = 16, LEAF = 256; };
template <> struct LocalCfg<uint64_t> { static constexpr int T = 8192, NT = 1024, KPT = 8, LEAF = 256; };

// Sort the keys of one wave's registers (any load order) with the smallest
// network that holds `sz` keys, and hand back key i of the sorted order to
// (lane i / KPL, register i % KPL).
template <int KPL, typename K, typename Ld, typename St>
__device__ __forceinline__ void wave_sort_n(uint32_t sz, int lane, const Ld &ld, const St &st)
{
    K x[KPL];
#pragma unroll
    for (int j = 0; j < KPL; ++j) {
        const uint32_t p = (uint32_t)(j * WAVE + lane);
        x[j] = p < sz ? ld(p) : key_max<K>();
    }
    bitonic_wave<KPL>(x, lane);
#pragma unroll
    for (int j = 0; j < KPL; ++j) {
        const uint32_t i = (uint32_t)(lane * KPL + j);
        if (i < sz) st(i, x[j]);
    }
}

template <typename K, typename Ld, typename St>
__device__ __forceinline__ void wave_sort(uint32_t sz, int lane, const Ld &ld, const St &st)
{
    if (sz <= 64) wave_sort_n<1, K>(sz, lane, ld, st);
    else if (sz <= 128) wave_sort_n<2, K>(sz, lane, ld, st);
    else wave_sort_n<4, K>(sz, lane, ld, st);
}

// One workgroup per task (claimed dynamically).  The task's keys are loaded
// into LDS; every level partitions all live sub-ranges at once, three ways
// (< pivot, == pivot, > pivot), with positions from one workgroup-wide scan
// of packed (lt, eq) counts; thread t owns the contiguous chunk
// [t*KPT, (t+1)*KPT) and LDS keeps one pad slot per chunk so chunk reads are
// free of bank conflicts.  Sub-ranges of at most LEAF keys go to the bitonic
// network (one wave each) as soon as they appear; runs equal to a pivot are
// final.  The sorted range is stored back in the caller's format.
template <int F>
__global__ __launch_bounds__(1024, 8) void k_local(Ctl *ctl, const Task<typename KeyOf<F>::type> *tasks,
                                                   typename KeyOf<F>::type *buf0,
                                                   typename KeyOf<F>::type *buf1, Raw raw, int rule,
                                                   uint32_t task_cap)
{
    using K = typename KeyOf<F>::type;
    using C = LocalCfg<K>;
    static_assert(C::NT * C::KPT == C::T, "one chunk of KPT keys per thread");
    constexpr int T = C::T, NT = C::NT, KPT = C::KPT, LEAF = C::LEAF;
    constexpr int NW = NT / WAVE;
    constexpr int MAXACT = T / (LEAF + 1) + 1;
    constexpr int MAXLEAF = 2 * MAXACT;
    static_assert(MAXACT <= WAVE, "one wave builds the range list");
    static_assert(KPT <= 32, "per-key masks are 32-bit");

    __shared__ K sk[T + T / KPT];
    __shared__ uint32_t act_b[2][MAXACT], act_e[2][MAXACT];
    __shared__ K act_p[2][MAXACT];
    __shared__ uint32_t SB[MAXACT], SE[MAXACT];
    __shared__ uint32_t leaf_b[MAXLEAF], leaf_e[MAXLEAF];
    __shared__ uint32_t wsum[NW];
    __shared__ uint32_t s_nact, s_nleaf, s_list, s_task;

    const int tid = threadIdx.x, lane = lane_id(), wave = tid / WAVE;
    const uint32_t ntask = min(ctl->ntask, task_cap);
    auto E = [](uint32_t p) { return p + p / KPT; };

    for (;;) {
        if (tid == 0) s_task = atomicAdd(&ctl->task_next, 1u);
        __syncthreads();
        const uint32_t ti = s_task;
        __syncthreads();
        if (ti >= ntask) break;
        const Task<K> tk = tasks[ti];
        const uint32_t b = tk.b, m = tk.e - tk.b;

        if (tk.kind == TASK_FILL) {
            for (uint32_t i = tid; i < m; i += NT) raw_store<F>(raw, b + i, tk.fill);
            continue;
        }
        const K *sbuf = tk.src == SRC_BUF0 ? buf0 : buf1;
        const bool sraw = tk.src == SRC_RAW;
        auto gload = [&](uint32_t i) -> K { return sraw ? raw_load<F>(raw, i) : sbuf[i]; };

        if (m <= (uint32_t)LEAF) {
            if (wave == 0) {
                wave_sort<K>(m, lane, [&](uint32_t p) { return gload(b + p); },
                             [&](uint32_t i, K v) { raw_store<F>(raw, b + i, v); });
            }
            continue;
        }

        for (uint32_t i = tid; i < m; i += NT) sk[E(i)] = gload(b + i);
        __syncthreads();
        if (tid == 0) {
            act_b[0][0] = 0;
            act_e[0][0] = m;
            auto rd = [&](uint32_t p) { return sk[E(p)]; };
            act_p[0][0] = pick_pivot<K>(rd, 0, m, rule);
            s_nact = 1;
            s_list = 0;
        }
        __syncthreads();

        for (;;) {
            const uint32_t na = s_nact, L = s_list;
            if (na == 0) break;
            // ---- load my chunk and classify against my sub-range's pivot
            const uint32_t t0 = (uint32_t)tid * KPT;
            K x[KPT];
#pragma unroll
            for (int j = 0; j < KPT; ++j) x[j] = (t0 + j < m) ? sk[t0 + j + tid] : K(0);
            int s0 = -1;
            {
                int lo = 0, hi = (int)na;  // largest s with act_b[s] <= t0
                while (lo < hi) {
                    const int md = (lo + hi) >> 1;
                    if (act_b[L][md] <= t0) lo = md + 1; else hi = md;
                }
                s0 = lo - 1;
            }
            uint32_t ltm = 0, eqm = 0, inm = 0, cl = 0, ce = 0;
            {
                int s = s0;
                uint32_t se = s >= 0 ? act_e[L][s] : 0u;
                K sp = s >= 0 ? act_p[L][s] : K(0);
                uint32_t nb = (s + 1 < (int)na) ? act_b[L][s + 1] : 0xFFFFFFFFu;
#pragma unroll
                for (int j = 0; j < KPT; ++j) {
                    const uint32_t p = t0 + j;
                    if (p >= nb) {
                        ++s;
                        se = act_e[L][s];
                        sp = act_p[L][s];
                        nb = (s + 1 < (int)na) ? act_b[L][s + 1] : 0xFFFFFFFFu;
                    }
                    if (s >= 0 && p < se) {
                        inm |= 1u << j;
                        if (x[j] < sp) {
                            ltm |= 1u << j;
                            ++cl;
                        } else if (x[j] == sp) {
                            eqm |= 1u << j;
                            ++ce;
                        }
                    }
                }
            }
            const uint32_t code = cl | (ce << 16);
            const uint32_t incl = wave_incl_scan(code);
            if (lane == WAVE - 1) wsum[wave] = incl;
            __syncthreads();
            uint32_t pre = 0;
            for (int w = 0; w < wave; ++w) pre += wsum[w];
            const uint32_t excl = pre + incl - code;
            // ---- sub-range boundary prefixes
            {
                int s = s0;
                uint32_t sb = s >= 0 ? act_b[L][s] : 0u, se = s >= 0 ? act_e[L][s] : 0u;
                uint32_t nb = (s + 1 < (int)na) ? act_b[L][s + 1] : 0xFFFFFFFFu;
                uint32_t run = excl;
#pragma unroll
                for (int j = 0; j < KPT; ++j) {
                    const uint32_t p = t0 + j;
                    if (p >= nb) {
                        ++s;
                        sb = act_b[L][s];
                        se = act_e[L][s];
                        nb = (s + 1 < (int)na) ? act_b[L][s + 1] : 0xFFFFFFFFu;
                    }
                    if (inm & (1u << j)) {
                        if (p == sb) SB[s] = run;
                        run += (ltm >> j & 1u) | ((eqm >> j & 1u) << 16);
                        if (p + 1 == se) SE[s] = run;
                    }
                }
            }
            __syncthreads();
            // ---- scatter to the new positions (every key of the pass is in registers)
            {
                int s = s0;
                uint32_t sb = s >= 0 ? act_b[L][s] : 0u, sbp = s >= 0 ? SB[s] : 0u;
                uint32_t tl = s >= 0 ? SE[s] - SB[s] : 0u;
                uint32_t nb = (s + 1 < (int)na) ? act_b[L][s + 1] : 0xFFFFFFFFu;
                uint32_t run = excl;
#pragma unroll
                for (int j = 0; j < KPT; ++j) {
                    const uint32_t p = t0 + j;
                    if (p >= nb) {
                        ++s;
                        sb = act_b[L][s];
                        sbp = SB[s];
                        tl = SE[s] - SB[s];
                        nb = (s + 1 < (int)na) ? act_b[L][s + 1] : 0xFFFFFFFFu;
                    }
                    if (inm & (1u << j)) {
                        const uint32_t r = run - sbp;
                        const uint32_t rl = r & 0xFFFFu, re = r >> 16;
                        const uint32_t nl = tl & 0xFFFFu, ne = tl >> 16;
                        uint32_t np;
                        if (ltm & (1u << j)) np = sb + rl;
                        else if (eqm & (1u << j)) np = sb + nl + re;
                        else np = sb + nl + ne + (p - sb - rl - re);
                        sk[E(np)] = x[j];
                        run += (ltm >> j & 1u) | ((eqm >> j & 1u) << 16);
                    }
                }
            }
            __syncthreads();
            // ---- next list: children larger than LEAF stay live, 2..LEAF become leaves
            if (wave == 0) {
                const uint32_t s = (uint32_t)lane;
                uint32_t lb = 0, le = 0, rb = 0, re = 0;
                if (s < na) {
                    const uint32_t b0 = act_b[L][s], e0 = act_e[L][s];
                    const uint32_t tl = SE[s] - SB[s];
                    const uint32_t nl = tl & 0xFFFFu, ne = tl >> 16;
                    lb = b0;
                    le = b0 + nl;
                    rb = b0 + nl + ne;
                    re = e0;
                }
                const bool aL = le - lb > (uint32_t)LEAF, aR = re - rb > (uint32_t)LEAF;
                const bool fL = le - lb >= 2 && !aL, fR = re - rb >= 2 && !aR;
                const uint32_t na_me = (uint32_t)aL + (uint32_t)aR, nf_me = (uint32_t)fL + (uint32_t)fR;
                const uint32_t ai = wave_incl_scan(na_me), fi = wave_incl_scan(nf_me);
                uint32_t ap = ai - na_me, fp = fi - nf_me;
                const uint32_t N = 1u - L;
                auto rd = [&](uint32_t p) { return sk[E(p)]; };
                if (aL) {
                    act_b[N][ap] = lb;
                    act_e[N][ap] = le;
                    act_p[N][ap] = pick_pivot<K>(rd, lb, le, rule);
                    ++ap;
                }
                if (aR) {
                    act_b[N][ap] = rb;
                    act_e[N][ap] = re;
                    act_p[N][ap] = pick_pivot<K>(rd, rb, re, rule);
                }
                if (fL) {
                    leaf_b[fp] = lb;
                    leaf_e[fp] = le;
                    ++fp;
                }
                if (fR) {
                    leaf_b[fp] = rb;
                    leaf_e[fp] = re;
                }
                if (lane == WAVE - 1) {
                    s_nact = ai;
                    s_nleaf = fi;
                    s_list = N;
                }
            }
            __syncthreads();
            // ---- bitonic network on this level's leaves, one wave per leaf
            const uint32_t nleaf = s_nleaf;
            for (uint32_t li = (uint32_t)wave; li < nleaf; li += NW) {
                const uint32_t fb = leaf_b[li], fe = leaf_e[li];
                wave_sort<K>(fe - fb, lane, [&](uint32_t p) { return sk[E(fb + p)]; },
                             [&](uint32_t i, K v) { sk[E(fb + i)] = v; });
            }
            __syncthreads();
        }
        for (uint32_t i = tid; i < m; i += NT) raw_store<F>(raw, b + i, sk[E(i)]);
        __syncthreads();
    }
}

}  // namespace hs
