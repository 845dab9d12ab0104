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
//   on-chip tier    segments of at most T keys are sorted on chip
//                   (hs_local.hpp).
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
constexpr uint32_t ERR_LEVELS = 16u;   // more partition levels than the driver allows
constexpr uint32_t ERR_BARRIER = 32u;  // a grid barrier timed out (workgroups not co-resident)

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

// The segment list of one partition level, built while the level before it
// is finalized.  Level L uses list, cursor array and counters number L & 1.
struct alignas(256) LevelCounts {
    unsigned long long segs_tiles;  // low half: segments in the list, high half: their tiles
    alignas(256) unsigned long long keys;  // keys in those segments (its own line: see wave_emit_segs2)
    uint32_t max_seg;                      // the largest of them
};

// Control block of one call, in device memory.  Every counter that many
// waves update atomically sits on a 256-byte line of its own: atomics on one
// line serialize.
struct Ctl {
    LevelCounts lev[2];
    alignas(256) uint32_t ntask;     // tasks for k_local, written from the front of the task list
    alignas(256) uint32_t nsmall;    // tasks for k_small, written from the back of the task list
    alignas(256) uint32_t task_next; // dynamic task counter of k_local
    alignas(256) uint32_t err;       // ERR_* bits
    alignas(256) unsigned long long local_keys;  // keys handed to local tasks
    unsigned long long fill_keys;                // keys handed to fill tasks
    alignas(256) uint32_t bar_arrive;  // grid barrier of the persistent level driver
    alignas(256) uint32_t bar_gen;
    alignas(256) uint32_t levels;      // levels that had at least one segment (one writer)
    unsigned long long part_keys;      // keys in the segments of every level run
};

// Items a wave emits over a batch of up to 64 steps are parked one or two per
// lane (lane k keeps what step k emitted) and appended to a device list with
// a single atomic per wave.
template <typename T>
__device__ __forceinline__ void wave_flush2(const T &a, bool ha, const T &b, bool hb, uint32_t *counter, T *list,
                                            uint32_t cap, Ctl *ctl, uint32_t errbit, bool from_back)
{
    const uint32_t cnt = (ha ? 1u : 0u) + (hb ? 1u : 0u);
    if (__ballot(cnt != 0) == 0) return;
    const uint32_t incl = wave_incl_scan(cnt);
    const uint32_t total = (uint32_t)__builtin_amdgcn_readlane((int)incl, WAVE - 1);
    uint32_t base = 0;
    if (lane_id() == 0) base = atomicAdd(counter, total);
    base = (uint32_t)__builtin_amdgcn_readfirstlane((int)base);
    uint32_t k = base + incl - cnt;
    auto put = [&](const T &item) {
        if (k < cap) list[from_back ? cap - 1 - k : k] = item;
        else atomicOr(&ctl->err, errbit);
        ++k;
    };
    if (ha) put(a);
    if (hb) put(b);
}

template <typename T>
__device__ __forceinline__ void wave_flush(const T &item, bool has, uint32_t *counter, T *list, uint32_t cap,
                                           Ctl *ctl, uint32_t errbit, bool from_back = false)
{
    const uint64_t m = __ballot(has);
    if (m == 0) return;
    const uint32_t total = (uint32_t)__popcll(m);
    uint32_t base = 0;
    if (lane_id() == 0) base = atomicAdd(counter, total);
    base = (uint32_t)__builtin_amdgcn_readfirstlane((int)base);
    const uint32_t k = base + mask_below(m);
    if (has) {
        if (k < cap) list[from_back ? cap - 1 - k : k] = item;
        else atomicOr(&ctl->err, errbit);
    }
}

// The task list holds on-chip tasks (sorted by k_local, one workgroup each)
// from the front and small tasks (at most LEAF keys, or fills: one wave each
// in k_small) from the back.  The two counts together never exceed its
// capacity; an overflow sets ERR_TASK_CAP.
template <typename T>
__device__ __forceinline__ void wave_flush_task(const T &item, bool has, bool small, T *list, uint32_t cap,
                                                Ctl *ctl)
{
    wave_flush(item, has && !small, &ctl->ntask, list, cap, ctl, ERR_TASK_CAP, false);
    wave_flush(item, has && small, &ctl->nsmall, list, cap, ctl, ERR_TASK_CAP, true);
}

// Two items per lane, one atomic per list.
template <typename T>
__device__ __forceinline__ void wave_flush_task2(const T &a, bool ha, bool sa, const T &b, bool hb, bool sb,
                                                 T *list, uint32_t cap, Ctl *ctl)
{
    wave_flush2(a, ha && !sa, b, hb && !sb, &ctl->ntask, list, cap, ctl, ERR_TASK_CAP, false);
    wave_flush2(a, ha && sa, b, hb && sb, &ctl->nsmall, list, cap, ctl, ERR_TASK_CAP, true);
}

__device__ __forceinline__ unsigned long long wave_sum64(unsigned long long v)
{
    for (int d = 1; d < WAVE; d <<= 1) v += __shfl_xor(v, d);
    return v;
}

// ---------------------------------------------------------------- tile geometry

template <typename K> struct PartCfg;
// Measured on MI355X (f64 and int32 at 2^27..2^28): 1024-thread workgroups
// with 8 keys (8-byte words) or 16 keys (int32) per thread keep the most
// bytes in flight; 256/512-thread shapes and 1-workgroup-per-CU tiles were
// up to 6% slower end to end.
template <> struct PartCfg<uint32_t> { static constexpr int NT = 1024, TILE = 16384; };
template <> struct PartCfg<uint64_t> { static constexpr int NT = 1024, TILE = 8192; };
// 16-byte words: the same 128 KB of keys in flight per workgroup pair.
template <> struct PartCfg<u128> { static constexpr int NT = 1024, TILE = 4096; };

// Write-cursor words of different segments sit 256 bytes apart: atomics on
// one cache line serialize, so neighbouring segments must not share one.
constexpr uint32_t CUR_STRIDE = 32;

// Tiles of a segment.  4-byte words: the tiles start at the segment's first
// key, tile k holding keys [b + k*TILE, min(b + (k+1)*TILE, e)), so every
// tile but the last is full and the deep levels, whose segments span one to
// a few tiles, get fewer and fuller tiles (int32 2^28: 6.65 -> 6.54 ms of
// partition passes).  Wider words: the tiles sit at absolute multiples of
// TILE, partial at both ends of a segment; measured, segment-aligned tiles
// cost them 3% (float64 2^28: 12.37 -> 12.78 ms).  Every load and store of
// the passes is per key, so either layout is valid for every word size.
template <typename K>
__device__ __host__ __forceinline__ uint32_t seg_tiles(uint32_t b, uint32_t e)
{
    constexpr uint32_t TILE = PartCfg<K>::TILE;
    if constexpr (sizeof(K) == 4) return (e - b + TILE - 1) / TILE;
    else return (e + TILE - 1) / TILE - b / TILE;
}

// Tile t of a segment [b, e) whose first tile is tile0: its first key and
// key count.
template <typename K>
__device__ __forceinline__ void seg_tile_range(uint32_t b, uint32_t e, uint32_t tile0, uint32_t t, uint32_t &p0,
                                               uint32_t &cnt)
{
    constexpr uint32_t TILE = PartCfg<K>::TILE;
    if constexpr (sizeof(K) == 4) {
        p0 = b + (t - tile0) * TILE;
        cnt = min(e - p0, TILE);
    } else {
        const uint32_t a = b / TILE + (t - tile0);
        p0 = max(b, a * TILE);
        cnt = min(e, (a + 1) * TILE) - p0;
    }
}

// Append the segments a wave holds (lane k: up to two, a before b) to the
// next level's list.  One 64-bit atomic reserves both the list slots (low
// half) and the segments' tiles (high half), so tile0 grows with the slot
// index and a tile finds its segment by binary search.  The cursor word of
// each new slot is cleared here.  The list's key count and largest segment
// are only read after the level, so the caller accumulates them per lane
// (keys, mx) and adds them once at its end: the slot/tile atomic is the only
// one that every batch of every wave makes on that line.
template <typename K>
__device__ __forceinline__ void wave_emit_segs2(Seg<K> a, bool ha, Seg<K> b, bool hb, Seg<K> *list,
                                                unsigned long long *curs, LevelCounts *lc, uint32_t cap, Ctl *ctl,
                                                unsigned long long &keys, uint32_t &mx)
{
    const uint32_t cnt = (ha ? 1u : 0u) + (hb ? 1u : 0u);
    if (__ballot(cnt != 0) == 0) return;
    const uint32_t nta = ha ? seg_tiles<K>(a.b, a.e) : 0u, ntb = hb ? seg_tiles<K>(b.b, b.e) : 0u;
    const uint32_t nt = nta + ntb;
    const uint32_t ic = wave_incl_scan(cnt), it = wave_incl_scan(nt);
    const uint32_t tc = (uint32_t)__builtin_amdgcn_readlane((int)ic, WAVE - 1);
    const uint32_t tt = (uint32_t)__builtin_amdgcn_readlane((int)it, WAVE - 1);
    unsigned long long base = 0;
    if (lane_id() == 0) base = atomicAdd(&lc->segs_tiles, ((unsigned long long)tt << 32) | (unsigned long long)tc);
    const uint32_t slot0 = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)base);
    const uint32_t tile_base = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)(base >> 32));
    uint32_t k = slot0 + ic - cnt, t0 = tile_base + it - nt;
    auto put = [&](Seg<K> item, uint32_t ntiles) {
        if (k < cap) {
            item.tile0 = t0;
            list[k] = item;
            curs[(size_t)k * CUR_STRIDE] = 0ull;
        } else {
            atomicOr(&ctl->err, ERR_CAND_CAP);
        }
        ++k;
        t0 += ntiles;
        keys += item.e - item.b;
        mx = max(mx, item.e - item.b);
    };
    if (ha) put(a, nta);
    if (hb) put(b, ntb);
}

// Add a wave's accumulated key count and largest segment to a level list.
__device__ __forceinline__ void wave_emit_totals(LevelCounts *lc, unsigned long long keys, uint32_t mx)
{
    keys = wave_sum64(keys);
    for (int d = 1; d < WAVE; d <<= 1) mx = max(mx, (uint32_t)__shfl_xor((int)mx, d));
    if (lane_id() == 0 && keys) {
        atomicAdd(&lc->keys, keys);
        atomicMax(&lc->max_seg, mx);
    }
}

// One segment per lane.
template <typename K>
__device__ __forceinline__ void wave_emit_segs(Seg<K> item, bool has, Seg<K> *list, unsigned long long *curs,
                                               LevelCounts *lc, uint32_t cap, Ctl *ctl)
{
    unsigned long long keys = 0;
    uint32_t mx = 0;
    wave_emit_segs2(item, has, item, false, list, curs, lc, cap, ctl, keys, mx);
    wave_emit_totals(lc, keys, mx);
}

// Number of segments of a level list that may be read (an overflow is
// flagged in err; never read past the list).
__device__ __forceinline__ uint32_t level_segs(unsigned long long st, uint32_t cap)
{
    return min((uint32_t)st, cap);
}

// ---------------------------------------------------------------- grid barrier

// Barrier over every workgroup of a persistent launch (all of them resident:
// the grid never exceeds what the occupancy calculator reports).  Arrival is
// one device-scope atomic per workgroup; the last arrival resets the count
// and bumps the generation, which the others poll with a bounded spin.  The
// agent-scope fences on both sides make every write before the barrier
// visible to every read after it, across the chip's L2 slices.  A spin that
// runs out sets ERR_BARRIER; every workgroup then leaves the driver.
constexpr uint32_t BARRIER_SPIN_LIMIT = 1u << 22;

__device__ __forceinline__ bool grid_barrier(Ctl *ctl, uint32_t &gen, uint32_t spin_limit)
{
    __shared__ uint32_t s_ok;
    __syncthreads();
    if (threadIdx.x == 0) {
        bool ok = true;
        __threadfence();
        if (__hip_atomic_load(&ctl->err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) & ERR_BARRIER) {
            ok = false;  // another workgroup gave up: leave without arriving
        } else if (atomicAdd(&ctl->bar_arrive, 1u) == gridDim.x - 1) {
            atomicExch(&ctl->bar_arrive, 0u);
            __threadfence();
            atomicAdd(&ctl->bar_gen, 1u);
        } else {
            uint32_t spins = 0;
            while (__hip_atomic_load(&ctl->bar_gen, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) == gen) {
                if (__hip_atomic_load(&ctl->err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) & ERR_BARRIER) {
                    ok = false;
                    break;
                }
                if (++spins > spin_limit) {
                    atomicOr(&ctl->err, ERR_BARRIER);
                    ok = false;
                    break;
                }
                __builtin_amdgcn_s_sleep(8);
            }
        }
        __threadfence();
        ++gen;
        s_ok = ok ? 1u : 0u;
    }
    __syncthreads();
    return s_ok != 0;
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

// Pivot of [b, e) (e - b >= 2) computed by one thread.  MEDIAN3 takes the
// first, middle and last key (the 3-value median of Sec. IV-A at the
// positions of Appendix A's middle rule); any other rule takes the ninther,
// the median of three such medians over nine evenly spaced keys.  The
// choice only changes how many levels run, never the output.
template <typename K, typename Rd>
__device__ K pick_pivot(const Rd &rd, uint32_t b, uint32_t e, int rule)
{
    const uint32_t m = e - b;
    if (rule == PIVOT_MEDIAN3 || m < 64) return med3<K>(rd(b), rd(b + (m - 1) / 2), rd(e - 1));
    K v[9];
#pragma unroll
    for (int i = 0; i < 9; ++i) v[i] = rd(b + (uint32_t)(((uint64_t)(m - 1) * i) / 8));
    return med3<K>(med3<K>(v[0], v[1], v[2]), med3<K>(v[3], v[4], v[5]), med3<K>(v[6], v[7], v[8]));
}

// Pivot of [b, e) computed by a whole wave (every lane gets the result).
// SAMPLE: lane i reads the key at b + i*(m-1)/63, the 64 samples are sorted
// with the in-register bitonic network and the lower median is taken.
template <typename K, typename Rd>
__device__ K wave_pick_pivot(const Rd &rd, uint32_t b, uint32_t e, int rule, int lane)
{
    const uint32_t m = e - b;
    if (rule != PIVOT_SAMPLE || m < 256) return pick_pivot<K>(rd, b, e, rule);
    K x[1];
    x[0] = rd(b + (uint32_t)(((uint64_t)(m - 1) * (uint32_t)lane) / (WAVE - 1)));
    bitonic_wave<1>(x, lane);
    return lane_bcast(x[0], WAVE / 2 - 1);
}

// Pivots of two ranges at once (the children of one segment): the sample
// loads of both are issued before either network runs, so the two load
// latencies overlap.  has0 / has1: whether the range needs a pivot.
template <typename K, typename Rd>
__device__ void wave_pick_pivot2(const Rd &rd, uint32_t b0, uint32_t e0, bool has0, uint32_t b1, uint32_t e1,
                                 bool has1, int rule, int lane, K &p0, K &p1)
{
    const uint32_t m0 = e0 - b0, m1 = e1 - b1;
    const bool s0 = has0 && rule == PIVOT_SAMPLE && m0 >= 256, s1 = has1 && rule == PIVOT_SAMPLE && m1 >= 256;
    K x0[1], x1[1];
    if (s0) x0[0] = rd(b0 + (uint32_t)(((uint64_t)(m0 - 1) * (uint32_t)lane) / (WAVE - 1)));
    if (s1) x1[0] = rd(b1 + (uint32_t)(((uint64_t)(m1 - 1) * (uint32_t)lane) / (WAVE - 1)));
    if (s0) {
        bitonic_wave<1>(x0, lane);
        p0 = lane_bcast(x0[0], WAVE / 2 - 1);
    } else if (has0) {
        p0 = pick_pivot<K>(rd, b0, e0, rule);
    }
    if (s1) {
        bitonic_wave<1>(x1, lane);
        p1 = lane_bcast(x1[0], WAVE / 2 - 1);
    } else if (has1) {
        p1 = pick_pivot<K>(rd, b1, e1, rule);
    }
}

// ---------------------------------------------------------------- init

// One array: the whole range becomes a level-0 segment, or a single local
// task when it fits on chip.
template <int F>
__global__ void k_init_single(Ctl *ctl, Seg<typename KeyOf<F>::type> *cand, unsigned long long *cur,
                              Task<typename KeyOf<F>::type> *tasks, Raw raw, uint32_t n, uint32_t T, uint32_t leaf,
                              uint32_t task_cap, int rule, int has_pivot, typename KeyOf<F>::type user_pivot)
{
    using K = typename KeyOf<F>::type;
    if (blockIdx.x != 0 || threadIdx.x >= WAVE) return;
    const int lane = lane_id();
    if (n <= T && !has_pivot) {
        if (n >= 2 && lane == 0) {
            Task<K> t;
            t.b = 0;
            t.e = n;
            t.src = SRC_RAW;
            t.kind = TASK_LOCAL;
            t.fill = 0;
            if (n > leaf) {
                tasks[0] = t;
                ctl->ntask = 1;
            } else {
                tasks[task_cap - 1] = t;
                ctl->nsmall = 1;
            }
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
        s.piv = wave_pick_pivot<K>(rd, 0, n, rule, lane);
    }
    if (lane == 0) {
        cand[0] = s;
        cur[0] = 0ull;
        ctl->lev[0].segs_tiles = ((unsigned long long)seg_tiles<K>(0, n) << 32) | 1ull;
        ctl->lev[0].keys = n;
        ctl->lev[0].max_seg = n;
    }
}

// Many arrays: each wave routes 64 consecutive segments, lane i segment
// [off[i], off[i+1]).  Segments of at most T keys become local tasks, larger
// ones level-0 segments (their pivots are picked by the whole wave, one
// segment after the other).
template <int F>
__global__ __launch_bounds__(256) void k_init_segmented(Ctl *ctl, Seg<typename KeyOf<F>::type> *cand,
                                                        unsigned long long *cur,
                                                        Task<typename KeyOf<F>::type> *tasks, Raw raw,
                                                        const int64_t *off, uint32_t nseg, uint32_t n_total,
                                                        uint32_t T, uint32_t leaf, int rule, uint32_t cand_cap,
                                                        uint32_t task_cap)
{
    using K = typename KeyOf<F>::type;
    const int lane = lane_id();
    const uint32_t w = (blockIdx.x * blockDim.x + threadIdx.x) / WAVE;
    const uint32_t i = w * WAVE + (uint32_t)lane;
    uint32_t b = 0, e = 0;
    bool bad = false;
    if (i < nseg) {
        const int64_t b64 = off[i], e64 = off[i + 1];
        bad = b64 < 0 || e64 > (int64_t)n_total || e64 < b64;  // malformed offsets: skip and flag
        if (!bad) {
            b = (uint32_t)b64;
            e = (uint32_t)e64;
        }
    }
    if (__ballot(bad) && lane == 0) atomicOr(&ctl->err, ERR_OFFSETS);
    const uint32_t m = e - b;
    const bool is_task = m >= 2 && m <= T;
    const bool is_big = m > T;
    Task<K> t;
    t.b = b;
    t.e = e;
    t.src = SRC_RAW;
    t.kind = TASK_LOCAL;
    t.fill = 0;
    wave_flush_task(t, is_task, m <= leaf, tasks, task_cap, ctl);
    const unsigned long long lk = wave_sum64(is_task ? (unsigned long long)m : 0ull);
    if (lane == 0 && lk) atomicAdd(&ctl->local_keys, lk);

    Seg<K> sg;
    sg.b = b;
    sg.e = e;
    sg.tile0 = 0;
    sg.flags = 0;
    sg.ub = 0;
    sg.piv = 0;
    SrcReader<F> rd{nullptr, raw, true};
    for (uint64_t big = __ballot(is_big); big; big &= big - 1) {
        const int src = __builtin_ctzll(big);
        const uint32_t bb = (uint32_t)__builtin_amdgcn_readlane((int)b, src);
        const uint32_t ee = (uint32_t)__builtin_amdgcn_readlane((int)e, src);
        const K p = wave_pick_pivot<K>(rd, bb, ee, rule, lane);
        if (lane == src) sg.piv = p;
    }
    wave_emit_segs(sg, is_big, cand, cur, &ctl->lev[0], cand_cap, ctl);
}

// Bookkeeping at the start of a level with list number `par`: clear the
// next level's counters (always: an empty level must leave an empty list
// behind, not the one of the level before it) and count a non-empty level.
// One thread.
__device__ __forceinline__ void level_begin(Ctl *ctl, int par)
{
    LevelCounts &nx = ctl->lev[1 - par];
    atomicExch(&nx.segs_tiles, 0ull);
    atomicExch(&nx.keys, 0ull);
    atomicExch(&nx.max_seg, 0u);
    const LevelCounts &cur = ctl->lev[par];
    if ((uint32_t)__hip_atomic_load(&cur.segs_tiles, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) {
        atomicAdd(&ctl->levels, 1u);
        atomicAdd(&ctl->part_keys, __hip_atomic_load(&cur.keys, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
    }
}

// ---------------------------------------------------------------- partition pass

// Where one tile of the level lies: segment index, first key, key count.
template <typename K> struct TileLoc {
    uint32_t s, p0, cnt;
    bool full;
};

// One level of out-of-place partitioning.  Workgroup g owns a contiguous run
// of the level's tiles and keeps the next tile's loads in flight while it
// processes the current one.  Per tile: compare with the segment's pivot,
// count the <= side and the > side per thread, scan the counts across the
// workgroup, reserve both slot runs with one 64-bit atomic on the segment's
// cursor word (low half: front cursor, high half: back cursor -- Algorithm
// 3's left_w and right_w), compact the tile in LDS (<= keys first) and write
// both runs out with consecutive lanes on consecutive addresses.
// Bounds-checked loads: a buffer resource covering one tile's keys; a lane
// past the end reads zero and moves no data, so every tile runs the same
// straight-line code.
constexpr int BUF_RSRC_WORD3 = 0x00020000;  // raw buffer, 32-bit dwords (gfx9 family)

__device__ __forceinline__ __amdgpu_buffer_rsrc_t tile_rsrc(const void *base, uint32_t bytes)
{
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(base), (short)0, (int)bytes, BUF_RSRC_WORD3);
}

__device__ __forceinline__ uint32_t rsrc_load32(__amdgpu_buffer_rsrc_t r, uint32_t byte_off)
{
    return (uint32_t)__builtin_amdgcn_raw_buffer_load_b32(r, (int)byte_off, 0, 0);
}

__device__ __forceinline__ uint64_t rsrc_load64(__amdgpu_buffer_rsrc_t r, uint32_t byte_off)
{
    const auto w = __builtin_amdgcn_raw_buffer_load_b64(r, (int)byte_off, 0, 0);
    return ((uint64_t)(uint32_t)w[1] << 32) | (uint32_t)w[0];
}

__device__ __forceinline__ u128 rsrc_load128(__amdgpu_buffer_rsrc_t r, uint32_t byte_off)
{
    const auto w = __builtin_amdgcn_raw_buffer_load_b128(r, (int)byte_off, 0, 0);
    const uint64_t lo = ((uint64_t)(uint32_t)w[1] << 32) | (uint32_t)w[0];
    const uint64_t hi = ((uint64_t)(uint32_t)w[3] << 32) | (uint32_t)w[2];
    return ((u128)hi << 64) | lo;
}

// s_waitcnt on the vector-memory counter alone: at most n operations still
// outstanding (gfx9 encoding: vmcnt bits 3:0 and 15:14; expcnt and lgkmcnt
// left at their maxima).
template <int N> __device__ __forceinline__ void wait_vmcnt()
{
    static_assert(N >= 0 && N < 64, "vmcnt is 6 bits");
    __builtin_amdgcn_s_waitcnt((N & 0xF) | ((N >> 4) << 14) | 0x70 | 0xF00);
}

// Workgroup `wg` of `nwg` takes the tiles wg, wg + nwg, wg + 2*nwg, ... of
// the level, so the workgroups running at any moment read neighbouring tiles
// and write to the few segments those tiles belong to (measured against
// contiguous runs of tiles per workgroup: int32 2^28 partition passes 6.54 ->
// 6.26 ms, float64 12.35 -> 11.93 ms; the first level, whose writes go to two
// streams either way, 388 -> 362 us).  The tile count is bounded by the
// tiles of the segments in the list (a list overflow, which is flagged,
// cannot create tiles without keys), so every tile holds at least one key.
// The LDS staging area is the caller's, so the persistent driver shares it
// between levels.
//
// Order within a tile: classify, scan, reserve (the cursor atomic), issue
// the next tile's loads, compact in LDS, write out.  Loads and stores share
// one in-order counter on this chip, so the code between the atomic and the
// use of its result, and the write-out, are straight-line with a fixed
// number of memory instructions: waiting for the atomic then waits neither
// for the next tile's loads nor for anything younger, and the next tile's
// reads overlap this tile's writes.
template <int F, bool SRC_IS_RAW, bool DST_IS_RAW>
__device__ __forceinline__ void partition_level(uint32_t ntiles, uint32_t nseg,
                                                const Seg<typename KeyOf<F>::type> *segs, unsigned long long *cur,
                                                const typename KeyOf<F>::type *src, Raw raw,
                                                typename KeyOf<F>::type *dst, Raw raw_dst, uint32_t wg, uint32_t nwg,
                                                typename KeyOf<F>::type *stage, uint32_t *wsum, uint32_t *sbase)
{
    using K = typename KeyOf<F>::type;
    constexpr int NT = PartCfg<K>::NT, TILE = PartCfg<K>::TILE, ITEMS = TILE / NT;
    constexpr int NW = NT / WAVE;
    static_assert(TILE < 65536, "per-tile counts are 16-bit");

    if (nseg == 0) return;
    {
        const Seg<K> last = segs[nseg - 1];
        ntiles = min(ntiles, last.tile0 + seg_tiles<K>(last.b, last.e));
    }
    // the tile index is uniform: keep it (and the tile loop) scalar
    uint32_t t = (uint32_t)__builtin_amdgcn_readfirstlane((int)wg);
    if (t >= ntiles) return;
    const int tid = threadIdx.x, lane = lane_id(), wave = tid / WAVE;

    // The segment of tile tt: the last one with tile0 <= tt at or after
    // segment lo (whose first tile is lo_tile0), by a 64-way search: lane l
    // probes lo + span*l/64; tile0 grows with the index, so the probes at or
    // below tt are a prefix of the lanes.  Every segment has a tile, so the
    // answer lies within tt - lo_tile0 segments of lo: two rounds of parallel
    // loads when a workgroup's next tile is nwg = 512 tiles on (two rounds of
    // one workgroup per compute unit).
    auto search = [&](uint32_t tt, uint32_t lo, uint32_t lo_tile0) -> uint32_t {
        uint32_t hi = (uint32_t)min((uint64_t)nseg, (uint64_t)lo + (tt - lo_tile0) + 1u);
        while (hi - lo > 1) {
            const uint32_t span = hi - lo;
            const uint32_t probe = lo + (uint32_t)(((uint64_t)span * (uint32_t)lane) / WAVE);
            const uint64_t m = __ballot(segs[probe].tile0 <= tt);  // lane 0 probes lo: always set
            const int last = 63 - __builtin_clzll(m);
            const uint32_t nlo = lane_bcast(probe, last);
            hi = last == WAVE - 1 ? hi : lane_bcast(probe, last + 1);
            lo = nlo;
        }
        return (uint32_t)__builtin_amdgcn_readfirstlane((int)lo);
    };
    uint32_t s_cur = search(t, 0, 0);
    Seg<K> sg_cur = segs[s_cur];

    auto locate = [&](uint32_t tt, Seg<K> &sg_out) {
        if (tt >= sg_cur.tile0 + seg_tiles<K>(sg_cur.b, sg_cur.e)) {
            s_cur = search(tt, s_cur, sg_cur.tile0);
            sg_cur = segs[s_cur];
        }
        sg_out = sg_cur;
        TileLoc<K> L;
        L.s = s_cur;
        uint32_t p0, cnt;
        seg_tile_range<K>(sg_cur.b, sg_cur.e, sg_cur.tile0, tt, p0, cnt);
        // the tile's place is the same in every lane: readfirstlane keeps it
        // (and the full-tile branch) scalar
        L.p0 = (uint32_t)__builtin_amdgcn_readfirstlane((int)p0);
        L.cnt = (uint32_t)__builtin_amdgcn_readfirstlane((int)cnt);
        L.full = L.cnt == (uint32_t)TILE;
        return L;
    };
    // lane tid takes keys j*NT + tid of the tile: consecutive lanes read
    // consecutive addresses.  The tile's place is the same in every lane;
    // readfirstlane says so, so the buffer resource lives in scalar registers.
    auto load = [&](const TileLoc<K> &Lv, K (&x)[ITEMS]) {
        TileLoc<K> L;
        L.p0 = (uint32_t)__builtin_amdgcn_readfirstlane((int)Lv.p0);
        L.cnt = (uint32_t)__builtin_amdgcn_readfirstlane((int)Lv.cnt);
        if constexpr (SRC_IS_RAW && F == FMT_KV) {
            const auto rk = tile_rsrc((const uint32_t *)raw.keys + L.p0, L.cnt * 4u);
            const auto rv = tile_rsrc((const uint32_t *)raw.vals + L.p0, L.cnt * 4u);
#pragma unroll
            for (int j = 0; j < ITEMS; ++j) {
                const uint32_t off = (uint32_t)(j * NT + tid) * 4u;
                x[j] = enc_kv(rsrc_load32(rk, off), rsrc_load32(rv, off));
            }
        } else if constexpr (SRC_IS_RAW && F == FMT_KV_F64) {
            const auto rk = tile_rsrc((const uint64_t *)raw.keys + L.p0, L.cnt * 8u);
            const auto rv = tile_rsrc((const uint32_t *)raw.vals + L.p0, L.cnt * 4u);
#pragma unroll
            for (int j = 0; j < ITEMS; ++j) {
                const uint32_t i = (uint32_t)(j * NT + tid);
                x[j] = enc_kv_f64(rsrc_load64(rk, i * 8u), rsrc_load32(rv, i * 4u));
            }
        } else if constexpr (sizeof(K) == 16) {
            const auto r = tile_rsrc(src + L.p0, L.cnt * 16u);
#pragma unroll
            for (int j = 0; j < ITEMS; ++j) x[j] = rsrc_load128(r, (uint32_t)(j * NT + tid) * 16u);
        } else if constexpr (sizeof(K) == 4) {
            const auto r = tile_rsrc((SRC_IS_RAW ? (const K *)raw.keys : src) + L.p0, L.cnt * 4u);
#pragma unroll
            for (int j = 0; j < ITEMS; ++j) {
                const uint32_t v = rsrc_load32(r, (uint32_t)(j * NT + tid) * 4u);
                x[j] = SRC_IS_RAW ? enc_word<F>((K)v) : (K)v;
            }
        } else {
            const auto r = tile_rsrc((SRC_IS_RAW ? (const K *)raw.keys : src) + L.p0, L.cnt * 8u);
#pragma unroll
            for (int j = 0; j < ITEMS; ++j) {
                const uint64_t v = rsrc_load64(r, (uint32_t)(j * NT + tid) * 8u);
                x[j] = SRC_IS_RAW ? enc_word<F>((K)v) : (K)v;
            }
        }
    };

    // Stores issued by the write-out of one tile.
    constexpr int STORES = ITEMS * ((DST_IS_RAW && has_vals<F>()) ? 2 : 1);
    static_assert(STORES < 64, "vmcnt is 6 bits");

    Seg<K> sg;
    TileLoc<K> L = locate(t, sg);
    K x[ITEMS];
    load(L, x);
    // Both edges into the loop arrive with the tile's keys loaded, so the loop
    // head waits for nothing (the back edge may still have stores in flight).
    wait_vmcnt<0>();

    for (; t < ntiles; t += nwg) {
        const bool more = t + nwg < ntiles;
        // "<= pivot" (or "< pivot" for a strict segment) as one compare against
        // the largest key still on the low side; none is when strict and the
        // pivot is the least key
        const bool strict = (sg.flags & SEG_STRICT) != 0;
        const bool none = strict && sg.piv == K(0);
        const K lim = strict ? sg.piv - K(1) : sg.piv;
        auto low = [&](K v) { return !none && v <= lim; };
        // lanes past the end of a partial tile hold no key: item j is one iff
        // tid < cnt - j*NT (a scalar bound per item)
        auto valid = [&](int j) { return (int)tid < (int)L.cnt - j * NT; };
        uint32_t cle = 0, cva = ITEMS;
        if (L.full) {
#pragma unroll
            for (int j = 0; j < ITEMS; ++j) cle += (uint32_t)low(x[j]);
        } else {
            cva = 0;
#pragma unroll
            for (int j = 0; j < ITEMS; ++j) {
                const bool v = valid(j);
                cle += (uint32_t)(v && low(x[j]));
                cva += (uint32_t)v;
            }
        }
        const uint32_t cgt = cva - cle;
        const uint32_t code = cle | (cgt << 16);
        const uint32_t incl = wave_incl_scan(code);
        if (lane == WAVE - 1) wsum[wave] = incl;
        // where the next tile lies (segment records are read before the
        // atomic below, so that its wait covers nothing else)
        Seg<K> sgn = sg;
        TileLoc<K> Ln;
        if (more) {
            Ln = locate(t + nwg, sgn);
        } else {
            Ln.s = L.s;
            Ln.p0 = L.p0;
            Ln.cnt = 0;
            Ln.full = false;
        }
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
        unsigned long long old = 0;
        if (tid == 0)
            old = atomicAdd(&cur[(size_t)L.s * CUR_STRIDE],
                            (unsigned long long)tot_le | ((unsigned long long)tot_gt << 32));
        // the next tile's loads (an empty range past the last tile)
        K xn[ITEMS];
        load(Ln, xn);
        asm volatile("" ::: "memory");  // keep the use of the atomic's result below the loads
        // compaction into the staging area: a running slot per side
        uint32_t lp = excl & 0xFFFFu, gp = tot_le + (excl >> 16);
        if (L.full) {
#pragma unroll
            for (int j = 0; j < ITEMS; ++j) {
                const bool l = low(x[j]);
                stage[l ? lp : gp] = x[j];
                lp += (uint32_t)l;
                gp += (uint32_t)!l;
            }
        } else {
#pragma unroll
            for (int j = 0; j < ITEMS; ++j) {
                const bool v = valid(j), l = low(x[j]);
                if (v) stage[l ? lp : gp] = x[j];
                lp += (uint32_t)(v && l);
                gp += (uint32_t)(v && !l);
            }
        }
        if (tid == 0) {
            sbase[0] = sg.b + (uint32_t)old;
            sbase[1] = sg.e - (uint32_t)(old >> 32) - tot_gt;
        }
        __syncthreads();
        // No barrier after the write-out: the next tile's LDS writes come
        // after its first barrier, which every wave reaches only once done here.
        // Lanes past the end of a partial tile store the tile's last key
        // again at its own slot: no branch, a fixed number of stores.
        const uint32_t lt_base = sbase[0], gt_base = sbase[1];
#pragma unroll
        for (int j = 0; j < ITEMS; ++j) {
            const uint32_t i = min((uint32_t)(j * NT + tid), L.cnt - 1);
            const K v = stage[i];
            const uint32_t pos = i < tot_le ? lt_base + i : gt_base + (i - tot_le);
            if constexpr (DST_IS_RAW) raw_store<F>(raw_dst, pos, v);
            else dst[pos] = v;
        }
        wait_vmcnt<STORES>();  // the next tile's loads (older than the stores) are in
        L = Ln;
        sg = sgn;
#pragma unroll
        for (int j = 0; j < ITEMS; ++j) x[j] = xn[j];
    }
    __syncthreads();  // the caller may reuse the staging area
}

// One partition level as a kernel of its own (the host-driven level loop and
// the partition entry point): level list number `par`.  With begin_level set
// its first thread also does the level's bookkeeping (level_begin): the
// finalize kernel that follows builds the next list on cleared counters.
template <int F, bool SRC_IS_RAW, bool DST_IS_RAW>
__global__ __launch_bounds__(PartCfg<typename KeyOf<F>::type>::NT) void k_partition(
    Ctl *ctl, int par, int begin_level, const Seg<typename KeyOf<F>::type> *segs, unsigned long long *cur,
    const typename KeyOf<F>::type *src, Raw raw, typename KeyOf<F>::type *dst, Raw raw_dst, uint32_t cap)
{
    using K = typename KeyOf<F>::type;
    __shared__ K stage[PartCfg<K>::TILE];
    __shared__ uint32_t wsum[PartCfg<K>::NT / WAVE];
    __shared__ uint32_t sbase[2];
    if (begin_level && blockIdx.x == 0 && threadIdx.x == 0) level_begin(ctl, par);
    const unsigned long long st = ctl->lev[par].segs_tiles;
    partition_level<F, SRC_IS_RAW, DST_IS_RAW>((uint32_t)(st >> 32), level_segs(st, cap), segs, cur, src, raw, dst,
                                               raw_dst, blockIdx.x, gridDim.x, stage, wsum, sbase);
}

// ---------------------------------------------------------------- block-wide appends

// What the waves of a workgroup park in one batch (lane k: up to two
// segments for the next level and up to two tasks) is appended with one
// atomic per list for the whole workgroup: the waves publish their counts in
// LDS, one thread reserves the workgroup's slots, and every wave writes its
// items at its share.  Every thread of the workgroup must call it.
struct BlockFlushLds {
    uint32_t cnt[32][4];   // per wave: segments, their tiles, on-chip tasks, small tasks
    uint32_t base[32][4];  // per wave: first slot / tile of each
};

template <typename K>
__device__ __forceinline__ void block_flush(const Seg<K> &a, bool ha, const Seg<K> &b, bool hb, const Task<K> &ta,
                                            bool hta, bool sta, const Task<K> &tb, bool htb, bool stb,
                                            Seg<K> *list, unsigned long long *curs, LevelCounts *lc, uint32_t cand_cap,
                                            Task<K> *tasks, uint32_t task_cap, Ctl *ctl, unsigned long long &keys,
                                            uint32_t &mx, BlockFlushLds &L)
{
    const int lane = lane_id(), wv = (int)(threadIdx.x / WAVE), nw = (int)(blockDim.x / WAVE);
    const uint32_t nta = ha ? seg_tiles<K>(a.b, a.e) : 0u, ntb = hb ? seg_tiles<K>(b.b, b.e) : 0u;
    const uint32_t c_s = (ha ? 1u : 0u) + (hb ? 1u : 0u), c_t = nta + ntb;
    const uint32_t c_l = (hta && !sta ? 1u : 0u) + (htb && !stb ? 1u : 0u);
    const uint32_t c_m = (hta && sta ? 1u : 0u) + (htb && stb ? 1u : 0u);
    const uint32_t i_s = wave_incl_scan(c_s), i_t = wave_incl_scan(c_t);
    const uint32_t i_l = wave_incl_scan(c_l), i_m = wave_incl_scan(c_m);
    __syncthreads();  // the previous batch has read its bases
    if (lane == WAVE - 1) {
        L.cnt[wv][0] = i_s;
        L.cnt[wv][1] = i_t;
        L.cnt[wv][2] = i_l;
        L.cnt[wv][3] = i_m;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t tot[4] = {0, 0, 0, 0};
        for (int w = 0; w < nw; ++w)
            for (int j = 0; j < 4; ++j) {
                L.base[w][j] = tot[j];
                tot[j] += L.cnt[w][j];
            }
        uint32_t g[4] = {0, 0, 0, 0};
        if (tot[0]) {
            const unsigned long long r =
                atomicAdd(&lc->segs_tiles, ((unsigned long long)tot[1] << 32) | (unsigned long long)tot[0]);
            g[0] = (uint32_t)r;
            g[1] = (uint32_t)(r >> 32);
        }
        if (tot[2]) g[2] = atomicAdd(&ctl->ntask, tot[2]);
        if (tot[3]) g[3] = atomicAdd(&ctl->nsmall, tot[3]);
        for (int w = 0; w < nw; ++w)
            for (int j = 0; j < 4; ++j) L.base[w][j] += g[j];
    }
    __syncthreads();
    uint32_t ks = L.base[wv][0] + i_s - c_s, kt = L.base[wv][1] + i_t - c_t;
    uint32_t kl = L.base[wv][2] + i_l - c_l, km = L.base[wv][3] + i_m - c_m;
    auto put_seg = [&](Seg<K> item, uint32_t ntiles) {
        if (ks < cand_cap) {
            item.tile0 = kt;
            list[ks] = item;
            curs[(size_t)ks * CUR_STRIDE] = 0ull;
        } else {
            atomicOr(&ctl->err, ERR_CAND_CAP);
        }
        ++ks;
        kt += ntiles;
        keys += item.e - item.b;
        mx = max(mx, item.e - item.b);
    };
    if (ha) put_seg(a, nta);
    if (hb) put_seg(b, ntb);
    auto put_task = [&](const Task<K> &t, bool small) {
        uint32_t &k = small ? km : kl;
        if (k < task_cap) tasks[small ? task_cap - 1 - k : k] = t;
        else atomicOr(&ctl->err, ERR_TASK_CAP);
        ++k;
    };
    if (hta) put_task(ta, sta);
    if (htb) put_task(tb, stb);
}

// The workgroup's sums of its waves' counters, added to the device with one
// atomic each: ekeys and emax are per lane (the segments each lane emitted),
// lkeys and fkeys are the same in every lane of a wave.  Every thread of the
// workgroup must call it.
__device__ __forceinline__ void block_totals(LevelCounts *lc, Ctl *ctl, unsigned long long ekeys, uint32_t emax,
                                             unsigned long long lkeys, unsigned long long fkeys, BlockFlushLds &L)
{
    const int lane = lane_id(), wv = (int)(threadIdx.x / WAVE), nw = (int)(blockDim.x / WAVE);
    __shared__ unsigned long long s_sum[32][3];
    ekeys = wave_sum64(ekeys);
    for (int d = 1; d < WAVE; d <<= 1) emax = max(emax, (uint32_t)__shfl_xor((int)emax, d));
    __syncthreads();
    if (lane == 0) {
        s_sum[wv][0] = ekeys;
        s_sum[wv][1] = lkeys;
        s_sum[wv][2] = fkeys;
        L.cnt[wv][0] = emax;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long e = 0, l = 0, f = 0;
        uint32_t m = 0;
        for (int w = 0; w < nw; ++w) {
            e += s_sum[w][0];
            l += s_sum[w][1];
            f += s_sum[w][2];
            m = max(m, L.cnt[w][0]);
        }
        if (e) {
            atomicAdd(&lc->keys, e);
            atomicMax(&lc->max_seg, m);
        }
        if (l) atomicAdd(&ctl->local_keys, l);
        if (f) atomicAdd(&ctl->fill_keys, f);
    }
}

// ---------------------------------------------------------------- finalize

// Split every segment of the level at its front cursor (the count of the <=
// side, Algorithm 3's left_w) and route both children.  A child larger than
// T becomes a segment of the next level with its own pivot; a smaller child
// becomes a local task; the ">=" child of a strict split holds only keys
// equal to the pivot and becomes a fill task.  Waves take segments in a
// grid-stride loop, 64 at a time, and a workgroup appends what its waves
// emit with one atomic per list and batch (at the deepest levels tens of
// thousands of waves append to the same few counters, and atomics on one
// address serialize).  Every thread of the workgroup must call it.
//
// Equal keys: a left child inherits its parent's pivot as an upper bound.
// When a segment's pivot equals that bound, the segment is split with "<"
// instead of "<=", which moves every copy of the bound into a final range.
// This keeps runs of equal keys from being re-partitioned level after level.
// Fill tasks are cut into chunks of at most FILL_CHUNK keys so that no wave
// writes a long run of equal keys alone.
constexpr uint32_t FILL_CHUNK = 1u << 16;

template <int F>
__device__ __forceinline__ void finalize_level(Ctl *ctl, uint32_t nseg, const Seg<typename KeyOf<F>::type> *segs,
                                               const unsigned long long *cur, Seg<typename KeyOf<F>::type> *cand,
                                               unsigned long long *ncur, LevelCounts *nlev,
                                               Task<typename KeyOf<F>::type> *tasks,
                                               const typename KeyOf<F>::type *out, uint32_t out_id, Raw raw,
                                               uint32_t T, uint32_t leaf, int rule, uint32_t cand_cap,
                                               uint32_t task_cap, uint32_t w, uint32_t nwaves)
{
    using K = typename KeyOf<F>::type;
    const int lane = lane_id();
    // the level's output: an internal buffer, or the caller's arrays (levels
    // partitioned in place)
    SrcReader<F> rd{out, raw, out_id == SRC_RAW};
    unsigned long long lkeys = 0, fkeys = 0, ekeys = 0;
    uint32_t emax = 0;

    // the record and cursor of the wave's next segment are loaded while the
    // current one is processed
    Seg<K> nx_sg{};
    unsigned long long nx_c = 0;
    if (w < nseg) {
        nx_sg = segs[w];
        nx_c = cur[(size_t)w * CUR_STRIDE];
    }
    __shared__ BlockFlushLds fl;
    // the batch loop runs as long as the workgroup's first wave has work, so
    // every wave of the workgroup takes part in every block-wide append
    const uint32_t w_first = w - (uint32_t)(threadIdx.x / WAVE);
    for (uint32_t step0 = 0; w_first + (uint64_t)step0 * nwaves < nseg; step0 += WAVE) {
        // parked items of this batch (lane k: batch step k)
        Seg<K> c0, c1;
        Task<K> t0, t1;
        bool h_c0 = false, h_c1 = false, h_t0 = false, h_t1 = false;
        c0.tile0 = c1.tile0 = 0;
        t0.kind = t1.kind = TASK_LOCAL;
        t0.b = t0.e = t1.b = t1.e = 0;
        for (uint32_t k = 0; k < (uint32_t)WAVE; ++k) {
            const uint64_t i64 = w + (uint64_t)(step0 + k) * nwaves;
            if (i64 >= nseg) break;
            const Seg<K> sg = nx_sg;
            const unsigned long long c = nx_c;
            const uint64_t n64 = i64 + nwaves;
            if (n64 < nseg) {
                nx_sg = segs[(uint32_t)n64];
                nx_c = cur[(size_t)n64 * CUR_STRIDE];
            }
            const uint32_t nle = (uint32_t)c, ngt = (uint32_t)(c >> 32);
            if (nle + ngt != sg.e - sg.b) {
                if (lane == 0) atomicOr(&ctl->err, ERR_CURSOR);
                continue;
            }
            const uint32_t mid = sg.b + nle;
            const bool strict = (sg.flags & SEG_STRICT) != 0;
            // child ranges, with the bound each inherits
            const uint32_t cb[2] = {sg.b, mid}, ce[2] = {mid, sg.e};
            const uint32_t cfl[2] = {strict ? 0u : SEG_UB, sg.flags & SEG_UB};
            const K cub[2] = {sg.piv, sg.ub};
            // children that become segments of the next level need a pivot
            bool need[2];
#pragma unroll
            for (int side = 0; side < 2; ++side)
                need[side] = ce[side] - cb[side] > T && !(side == 1 && strict);
            K piv[2] = {K(0), K(0)};
            if (need[0] || need[1])
                wave_pick_pivot2<K>(rd, cb[0], ce[0], need[0], cb[1], ce[1], need[1], rule, lane, piv[0], piv[1]);
#pragma unroll
            for (int side = 0; side < 2; ++side) {
                const uint32_t b = cb[side], e = ce[side], m = e - b;
                if (m == 0) continue;
                Task<K> t;
                t.b = b;
                t.e = e;
                t.src = out_id;
                t.fill = 0;
                bool is_task = false;
                if (side == 1 && strict) {  // keys == pivot: final
                    t.kind = TASK_FILL;
                    t.fill = sg.piv;
                    fkeys += m;
                    if (m > FILL_CHUNK) {  // a long run: chunks, one lane each
                        const uint32_t nchunk = (m + FILL_CHUNK - 1) / FILL_CHUNK;
                        for (uint32_t c0i = 0; c0i < nchunk; c0i += WAVE) {
                            const uint32_t ci = c0i + (uint32_t)lane;
                            Task<K> tc = t;
                            tc.b = b + min(ci, nchunk) * FILL_CHUNK;
                            tc.e = min(e, tc.b + FILL_CHUNK);
                            wave_flush_task(tc, ci < nchunk, true, tasks, task_cap, ctl);
                        }
                        continue;
                    }
                    is_task = true;
                } else if (m <= T) {
                    t.kind = TASK_LOCAL;
                    is_task = true;
                    lkeys += m;
                }
                if (is_task) {
                    if (lane == (int)k) {
                        if (side == 0) { t0 = t; h_t0 = true; } else { t1 = t; h_t1 = true; }
                    }
                    continue;
                }
                Seg<K> ch;
                ch.b = b;
                ch.e = e;
                ch.tile0 = 0;
                ch.ub = cub[side];
                ch.piv = piv[side];
                ch.flags = cfl[side];
                if ((ch.flags & SEG_UB) && ch.piv == ch.ub) ch.flags |= SEG_STRICT;
                if (lane == (int)k) {
                    if (side == 0) { c0 = ch; h_c0 = true; } else { c1 = ch; h_c1 = true; }
                }
            }
        }
        block_flush(c0, h_c0, c1, h_c1, t0, h_t0, t0.kind == TASK_FILL || t0.e - t0.b <= leaf, t1, h_t1,
                    t1.kind == TASK_FILL || t1.e - t1.b <= leaf, cand, ncur, nlev, cand_cap, tasks, task_cap, ctl,
                    ekeys, emax, fl);
    }
    block_totals(nlev, ctl, ekeys, emax, lkeys, fkeys, fl);
}

template <int F>
__global__ __launch_bounds__(1024) void k_finalize(Ctl *ctl, int par, const Seg<typename KeyOf<F>::type> *segs,
                                                  const unsigned long long *cur,
                                                  Seg<typename KeyOf<F>::type> *cand, unsigned long long *ncur,
                                                  Task<typename KeyOf<F>::type> *tasks,
                                                  const typename KeyOf<F>::type *out, uint32_t out_id, Raw raw,
                                                  uint32_t T, uint32_t leaf, int rule, uint32_t cand_cap,
                                                  uint32_t task_cap)
{
    const uint32_t nseg = level_segs(ctl->lev[par].segs_tiles, cand_cap);
    finalize_level<F>(ctl, nseg, segs, cur, cand, ncur, &ctl->lev[1 - par], tasks, out, out_id, raw, T, leaf, rule,
                      cand_cap, task_cap, (blockIdx.x * blockDim.x + threadIdx.x) / WAVE,
                      gridDim.x * (blockDim.x / WAVE));
}

// ---------------------------------------------------------------- persistent level driver

// Every partition level of one call in a single launch: the workgroups
// partition the level's tiles, meet at a grid barrier, finalize its segments
// (building the next level's list and the task lists), meet again, and go on
// while the next list is non-empty.  Level L reads buffer L & 1 (level 0 the
// caller's array) and writes buffer (L + 1) & 1.  Every workgroup reads the
// same list size after the same barrier, so all of them leave together; a
// barrier that times out (ERR_BARRIER) or too many levels (ERR_LEVELS) end
// the launch with the error flagged.
template <int F>
__global__ __launch_bounds__(PartCfg<typename KeyOf<F>::type>::NT) void k_levels(
    Ctl *ctl, Seg<typename KeyOf<F>::type> *seg0, Seg<typename KeyOf<F>::type> *seg1, unsigned long long *cur0,
    unsigned long long *cur1, typename KeyOf<F>::type *buf0, typename KeyOf<F>::type *buf1, Raw raw,
    Task<typename KeyOf<F>::type> *tasks, uint32_t T, uint32_t leaf, int rule, int guard, int level0, int lmax,
    uint32_t cand_cap, uint32_t task_cap, uint32_t spin_limit)
{
    using K = typename KeyOf<F>::type;
    __shared__ K stage[PartCfg<K>::TILE];
    __shared__ uint32_t wsum[PartCfg<K>::NT / WAVE];
    __shared__ uint32_t sbase[2];
    const uint32_t wave_id = (blockIdx.x * blockDim.x + threadIdx.x) / WAVE;
    const uint32_t nwaves = gridDim.x * (blockDim.x / WAVE);
    uint32_t gen = 0;
    for (int level = level0;; ++level) {
        const int p = level & 1;
        const unsigned long long st =
            __hip_atomic_load(&ctl->lev[p].segs_tiles, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        const uint32_t nseg = level_segs(st, cand_cap), ntiles = (uint32_t)(st >> 32);
        if (nseg == 0) break;
        if (level >= lmax) {
            if (blockIdx.x == 0 && threadIdx.x == 0) atomicOr(&ctl->err, ERR_LEVELS);
            break;
        }
        if (blockIdx.x == 0 && threadIdx.x == 0) level_begin(ctl, p);
        Seg<K> *segs = p ? seg1 : seg0, *next = p ? seg0 : seg1;
        unsigned long long *cur = p ? cur1 : cur0, *ncur = p ? cur0 : cur1;
        K *dst = p ? buf0 : buf1;
        if (level == 0)
            partition_level<F, true, false>(ntiles, nseg, segs, cur, nullptr, raw, dst, Raw{}, blockIdx.x, gridDim.x,
                                            stage, wsum, sbase);
        else
            partition_level<F, false, false>(ntiles, nseg, segs, cur, p ? buf1 : buf0, raw, dst, Raw{}, blockIdx.x,
                                             gridDim.x, stage, wsum, sbase);
        if (!grid_barrier(ctl, gen, spin_limit)) break;
        const int lrule = level > guard ? PIVOT_SAMPLE : rule;
        finalize_level<F>(ctl, nseg, segs, cur, next, ncur, &ctl->lev[1 - p], tasks, dst, (uint32_t)(1 - p), raw, T,
                          leaf, lrule, cand_cap, task_cap, wave_id, nwaves);
        if (!grid_barrier(ctl, gen, spin_limit)) break;
    }
}

// Clear `nwords` 32-bit words (a kernel rather than a memset, so that the
// call can be recorded into a graph).
__global__ void k_zero_words(uint32_t *p, uint32_t nwords)
{
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < nwords; i += gridDim.x * blockDim.x) p[i] = 0u;
}

// *p = v (one word of the control block, from the host's stream order).
__global__ void k_set_word(uint32_t *p, uint32_t v)
{
    if (blockIdx.x == 0 && threadIdx.x == 0) *p = v;
}

// v[i] = i (the indices an argsort carries as values).
__global__ void k_iota(int32_t *v, uint32_t n)
{
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) v[i] = (int32_t)i;
}

// Number of 32-bit words where a and b differ, added to *count (one atomic
// per wave).
__global__ void k_count_diff(const uint32_t *a, const uint32_t *b, uint64_t nwords, unsigned long long *count)
{
    unsigned long long d = 0;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nwords; i += (uint64_t)gridDim.x * blockDim.x)
        d += a[i] != b[i];
    d = wave_sum64(d);
    if (lane_id() == 0 && d) atomicAdd(count, d);
}

// Count of the <= side after a single-segment pass (partition entry point),
// or -1 when a kernel of the pass flagged an error (the keys are then only
// partly partitioned).
__global__ void k_write_count(const Ctl *ctl, const unsigned long long *cur, int64_t *d_count)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) *d_count = ctl->err ? (int64_t)-1 : (int64_t)(uint32_t)cur[0];
}

}  // namespace hs
