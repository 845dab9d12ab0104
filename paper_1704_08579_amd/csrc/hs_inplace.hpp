// hs_inplace.hpp -- partition levels in place, without the ping-pong buffers.
//
// The paper partitions in place (Sec. III-B, Algorithm 3): vectors are loaded
// from both ends of the array and written back into the space already freed
// at the left or right end, so that no second array is needed.  That scheme
// is sequential in its two write cursors.  Here every segment of a level is
// partitioned in place by many workgroups at once, in four passes that
// never wait on each other inside a kernel:
//
//   classify  every key of the level is compared with its segment's pivot
//             once; the outcome is kept as one bit per key (64-key rows of
//             the level's tiles) and the segment's count of keys on the low
//             side is added up.  That count fixes the split point `mid`;
//   rows      for every row, the keys on the wrong side of `mid` are counted:
//             high keys before `mid` ("left-misplaced") and low keys from
//             `mid` on ("right-misplaced"), with an exclusive prefix over the
//             rows of each tile;
//   scan      one workgroup turns the tiles' totals into level-wide exclusive
//             prefixes;
//   swap      the k-th left-misplaced key of a segment trades places with its
//             k-th right-misplaced key.  Both counts are equal (the low side
//             holds exactly `mid - b` slots), ranks come from the prefixes,
//             and a wave finds the partner of its first key by a 64-way
//             search over the segment's tiles and the tile's rows, then walks
//             on through the rows' masks.  Every position is read and written by
//             exactly one lane, and the passes that located it only read the
//             masks, so no key can be seen half-moved.
//
// Extra memory: one bit per key plus 32 bits per 64-key row and a few words
// per tile, against a second copy of the keys for the out-of-place levels.
// The keys stay in the caller's format between levels (order words are
// formed on each read; a swap moves the caller's bits, and its values too).
#pragma once

#include "hs_kernels.hpp"

namespace hs {

// 64-key rows per partition tile.
template <typename K> constexpr int ip_rows() { return PartCfg<K>::TILE / WAVE; }

constexpr int IP_NT = 256;  // threads per workgroup of the row and swap passes

// The level's tile count, bounded by the tiles of the segments in its list
// (as in the out-of-place pass).
template <typename K>
__device__ __forceinline__ uint32_t ip_level_tiles(const Ctl *ctl, int par, const Seg<K> *segs, uint32_t cap,
                                                   uint32_t &nseg)
{
    const unsigned long long st = ctl->lev[par].segs_tiles;
    nseg = level_segs(st, cap);
    if (nseg == 0) return 0;
    const Seg<K> last = segs[nseg - 1];
    return min((uint32_t)(st >> 32), last.tile0 + seg_tiles<K>(last.b, last.e));
}

// Tile t of a segment: its first key and key count.
template <typename K>
__device__ __forceinline__ void ip_tile_range(const Seg<K> &sg, uint32_t t, uint32_t &p0, uint32_t &cnt)
{
    seg_tile_range<K>(sg.b, sg.e, sg.tile0, t, p0, cnt);
}

// Segment holding tile t (every tile holds at least one key).
template <typename K>
__device__ __forceinline__ uint32_t ip_find_seg(const Seg<K> *segs, uint32_t nseg, uint32_t t)
{
    uint32_t lo = 0, hi = nseg;
    while (hi - lo > 1) {
        const uint32_t m = (lo + hi) >> 1;
        if (segs[m].tile0 <= t) lo = m; else hi = m;
    }
    return lo;
}

// Largest i in [lo, hi) with key(i) <= g, for a non-decreasing key with
// key(lo) <= g (lo, hi, g wave-uniform): each step probes 64 evenly spaced
// points at once, one per lane, and keeps the interval after the last probe
// that is still <= g, so 2^18 candidates take three dependent loads.
template <typename Fn>
__device__ __forceinline__ uint32_t wave_search(uint32_t lo, uint32_t hi, uint32_t g, const Fn &key, int lane)
{
    while (hi - lo > 1) {
        const uint32_t step = (hi - lo + WAVE - 1) / WAVE;
        const uint32_t i = lo + (uint32_t)lane * step;
        const uint64_t ok = ballot(i < hi && key(i) <= g);  // a prefix of the lanes, lane 0 included
        const uint32_t last = (uint32_t)(WAVE - 1 - __builtin_clzll(ok));
        lo += last * step;
        hi = min(hi, lo + step);
    }
    return lo;
}

// ip_find_seg for a whole wave at once (t wave-uniform, every lane active):
// a few rounds of 64 probes instead of log2(nseg) dependent loads.
template <typename K>
__device__ __forceinline__ uint32_t ip_find_seg_wave(const Seg<K> *segs, uint32_t nseg, uint32_t t, int lane)
{
    return wave_search(0u, nseg, t, [&](uint32_t i) { return segs[i].tile0; }, lane);
}

// Segment record i, read through the constant address space: for a list
// that no thread writes while the kernel runs, a uniform index gives scalar
// loads, which the waits on vector loads do not cover (nor the other way
// round).  The list is written by an earlier kernel (the finalize step of
// the level before); a kernel launch invalidates the scalar cache, so these
// loads see it.  Not for lists that the same kernel writes.
template <typename K> __device__ __forceinline__ Seg<K> seg_const_load(const Seg<K> *segs, uint32_t i)
{
    const auto *c = (const __attribute__((address_space(4))) Seg<K> *)segs + i;
    Seg<K> s;
    s.b = c->b;
    s.e = c->e;
    s.tile0 = c->tile0;
    s.flags = c->flags;
    s.piv = c->piv;
    s.ub = c->ub;
    return s;
}

// Local indices [0, lim) of a tile starting at p0 with cnt keys lie before mid.
__device__ __forceinline__ uint32_t ip_left_limit(uint32_t mid, uint32_t p0, uint32_t cnt)
{
    return mid > p0 ? min(mid - p0, cnt) : 0u;
}

// Position (0..63) of the k-th set bit of m (k < popcount(m)): halve the
// window while keeping the bit inside it.
__device__ __forceinline__ uint32_t select_bit(uint64_t m, uint32_t k)
{
    uint32_t pos = 0;
#pragma unroll
    for (int s = 32; s >= 1; s >>= 1) {
        const uint64_t low = m & ((1ull << s) - 1ull);
        const uint32_t c = popc(low);
        if (k >= c) {
            k -= c;
            m >>= s;
            pos += (uint32_t)s;
        } else {
            m = low;
        }
    }
    return pos;
}

// An element in the caller's format (key, and value for the key/value
// formats), split into a load and a store so that the loads of several tiles
// or exchanges can be in flight at once: nothing is computed from the loaded
// bits until raw_word is called.
template <int F> struct RawElem {
    uint64_t k;
    int32_t v;
};
template <int F> __device__ __forceinline__ RawElem<F> raw_get(const Raw &r, uint32_t i)
{
    RawElem<F> e;
    if constexpr (raw_key_bytes<F>() == 8) e.k = ((const uint64_t *)r.keys)[i];
    else e.k = ((const uint32_t *)r.keys)[i];
    if constexpr (has_vals<F>()) e.v = r.vals[i];
    else e.v = 0;
    return e;
}
template <int F> __device__ __forceinline__ void raw_put(const Raw &r, uint32_t i, const RawElem<F> &e)
{
    if constexpr (raw_key_bytes<F>() == 8) ((uint64_t *)r.keys)[i] = e.k;
    else ((uint32_t *)r.keys)[i] = (uint32_t)e.k;
    if constexpr (has_vals<F>()) r.vals[i] = e.v;
}
template <int F> __device__ __forceinline__ typename KeyOf<F>::type raw_word(const RawElem<F> &e)
{
    if constexpr (F == FMT_KV) return enc_kv((uint32_t)e.k, (uint32_t)e.v);
    else if constexpr (F == FMT_KV_F64) return enc_kv_f64(e.k, (uint32_t)e.v);
    else return enc_word<F>((typename KeyOf<F>::type)e.k);
}

// Pass 1: classify.  Workgroup wg takes a contiguous run of the level's
// tiles and walks the segment list forward along it (one search for its
// first tile, then a look-ahead copy of the next segment, read with scalar
// loads), with the loads of the next two tiles in flight while the current
// one is classified; lane `tid`
// reads keys j*NT + tid of the tile (consecutive lanes, consecutive
// addresses), so wave w's j-th ballot is row j*NT/64 + w of the tile.  One
// 64-bit atomic per tile adds (low count, high count) to the segment's cursor
// word, which the finalize step reads like that of the out-of-place pass.
// With begin_level set, the first thread also does the level's bookkeeping.
template <int F>
__global__ __launch_bounds__(PartCfg<typename KeyOf<F>::type>::NT) void k_ip_classify(
    Ctl *__restrict__ ctl, int par, int begin_level, const Seg<typename KeyOf<F>::type> *__restrict__ segs,
    unsigned long long *__restrict__ cur, Raw raw, uint64_t *__restrict__ mask, uint32_t cap)
{
    using K = typename KeyOf<F>::type;
    constexpr int NT = PartCfg<K>::NT, TILE = PartCfg<K>::TILE, ITEMS = TILE / NT, RPT = ip_rows<K>();
    constexpr int NW = NT / WAVE;
    __shared__ uint32_t s_le[2][NW];
    if (begin_level && blockIdx.x == 0 && threadIdx.x == 0) level_begin(ctl, par);
    uint32_t nseg = 0;
    const uint32_t ntiles = ip_level_tiles<K>(ctl, par, segs, cap, nseg);
    nseg = (uint32_t)__builtin_amdgcn_readfirstlane((int)nseg);
    const uint32_t per = (uint32_t)__builtin_amdgcn_readfirstlane((int)((ntiles + gridDim.x - 1) / gridDim.x));
    uint32_t t = (uint32_t)__builtin_amdgcn_readfirstlane((int)(blockIdx.x * per));
    const uint32_t tend = (uint32_t)__builtin_amdgcn_readfirstlane((int)min(ntiles, t + per));
    if (t >= tend) return;
    const int tid = threadIdx.x, lane = lane_id(), w = tid / WAVE;
    // the segment of the first tile, then a forward walk (the level's list
    // does not change while this kernel runs: scalar loads)
    uint32_t s_cur = (uint32_t)__builtin_amdgcn_readfirstlane((int)ip_find_seg<K>(segs, nseg, t));
    Seg<K> sg_cur = seg_const_load<K>(segs, s_cur);
    Seg<K> sg_after = sg_cur;
    if (s_cur + 1 < nseg) sg_after = seg_const_load<K>(segs, s_cur + 1);
    struct Tile {
        uint32_t s, p0, cnt;
        Seg<K> sg;
        RawElem<F> x[ITEMS];
    };
    // Tile tt's place and keys.  Past the run's last tile the range is empty:
    // the buffer loads are still issued (so the number of loads in flight
    // is the same on every path) and return zeros without touching memory.
    auto fetch = [&](uint32_t tt, Tile &d) {
        d.p0 = 0;
        d.cnt = 0;
        if (tt < tend) {
            while (s_cur + 1 < nseg && tt >= sg_after.tile0) {
                ++s_cur;
                sg_cur = sg_after;
                if (s_cur + 1 < nseg) sg_after = seg_const_load<K>(segs, s_cur + 1);
            }
            ip_tile_range<K>(sg_cur, tt, d.p0, d.cnt);
        }
        d.s = s_cur;
        d.sg = sg_cur;
        const uint32_t p0 = (uint32_t)__builtin_amdgcn_readfirstlane((int)d.p0);
        const uint32_t cnt = (uint32_t)__builtin_amdgcn_readfirstlane((int)d.cnt);
        if constexpr (raw_key_bytes<F>() == 8) {
            const auto rk = tile_rsrc((const uint64_t *)raw.keys + p0, cnt * 8u);
#pragma unroll
            for (int j = 0; j < ITEMS; ++j) d.x[j].k = rsrc_load64(rk, (uint32_t)(j * NT + tid) * 8u);
        } else {
            const auto rk = tile_rsrc((const uint32_t *)raw.keys + p0, cnt * 4u);
#pragma unroll
            for (int j = 0; j < ITEMS; ++j) d.x[j].k = rsrc_load32(rk, (uint32_t)(j * NT + tid) * 4u);
        }
        if constexpr (has_vals<F>()) {
            const auto rv = tile_rsrc((const uint32_t *)raw.vals + p0, cnt * 4u);
#pragma unroll
            for (int j = 0; j < ITEMS; ++j) d.x[j].v = (int32_t)rsrc_load32(rv, (uint32_t)(j * NT + tid) * 4u);
        } else {
#pragma unroll
            for (int j = 0; j < ITEMS; ++j) d.x[j].v = 0;
        }
    };
    auto classify = [&](uint32_t tt, const Tile &c) {
        const bool strict = (c.sg.flags & SEG_STRICT) != 0;
        const bool none = strict && c.sg.piv == K(0);
        const K lim = strict ? c.sg.piv - K(1) : c.sg.piv;
        uint32_t le = 0;
#pragma unroll
        for (int j = 0; j < ITEMS; ++j) {
            const bool lo = (uint32_t)(j * NT + tid) < c.cnt && !none && raw_word<F>(c.x[j]) <= lim;
            const uint64_t m = ballot(lo);
            if (lane == 0) mask[(size_t)tt * RPT + (uint32_t)(j * NW + w)] = m;
            le += (uint32_t)lo;
        }
        // the wave sums go to one of two slots by tile parity: a wave can
        // only write the slot again after the next barrier, which thread 0
        // passes once it has read this tile's sums
        const uint32_t ws = wave_sum(le);
        if (lane == 0) s_le[tt & 1][w] = ws;
        __syncthreads();
        if (tid == 0) {
            uint32_t tot = 0;
#pragma unroll
            for (int k = 0; k < NW; ++k) tot += s_le[tt & 1][k];
            atomicAdd(&cur[(size_t)c.s * CUR_STRIDE],
                      (unsigned long long)tot | ((unsigned long long)(c.cnt - tot) << 32));
        }
    };
    // Three tile buffers in turn: tile t is classified while the loads of
    // t + 1 and t + 2 are in flight.  The loop is unrolled over the buffers
    // so that no buffer is copied (a copy would wait for its loads).
    Tile ta, tb, tc;
    fetch(t, ta);
    fetch(t + 1, tb);
    for (;;) {
        fetch(t + 2, tc);
        classify(t, ta);
        if (++t >= tend) break;
        fetch(t + 2, ta);
        classify(t, tb);
        if (++t >= tend) break;
        fetch(t + 2, tb);
        classify(t, tc);
        if (++t >= tend) break;
    }
}

// Pass 2: rows.  Thread r of a workgroup takes row r of the tile; rowpre
// receives the exclusive prefix over the tile's rows of (left-misplaced |
// right-misplaced << 16) and tot the tile's two totals.
template <int F>
__global__ __launch_bounds__(IP_NT) void k_ip_rows(const Ctl *ctl, int par, const Seg<typename KeyOf<F>::type> *segs,
                                                   const unsigned long long *cur, const uint64_t *mask,
                                                   uint32_t *rowpre, uint32_t *tot, uint32_t cap)
{
    using K = typename KeyOf<F>::type;
    constexpr int RPT = ip_rows<K>();
    constexpr int NW = IP_NT / WAVE;
    static_assert(RPT <= IP_NT, "one thread per row");
    __shared__ uint32_t s_w[NW];
    uint32_t nseg = 0;
    const uint32_t ntiles = ip_level_tiles<K>(ctl, par, segs, cap, nseg);
    const int tid = threadIdx.x, lane = lane_id(), w = tid / WAVE;
    for (uint32_t t = blockIdx.x; t < ntiles; t += gridDim.x) {
        const uint32_t s = ip_find_seg_wave<K>(segs, nseg, t, lane);
        const Seg<K> sg = segs[s];
        uint32_t p0, cnt;
        ip_tile_range<K>(sg, t, p0, cnt);
        const uint32_t mid = sg.b + (uint32_t)cur[(size_t)s * CUR_STRIDE];
        const uint32_t lim = ip_left_limit(mid, p0, cnt);
        uint32_t c = 0;
        if (tid < RPT) {
            const uint32_t r0 = (uint32_t)tid * WAVE;
            const uint64_t lo = mask[(size_t)t * RPT + tid];  // no bits past the tile's keys
            const uint64_t valid = r0 < cnt ? lanes_below(cnt - r0) : 0ull;
            const uint64_t left = r0 < lim ? lanes_below(lim - r0) : 0ull;
            c = popc(~lo & valid & left) | (popc(lo & ~left) << 16);
        }
        const uint32_t incl = wave_incl_scan(c);
        if (lane == WAVE - 1) s_w[w] = incl;
        __syncthreads();
        uint32_t pre = 0, all = 0;
#pragma unroll
        for (int k = 0; k < NW; ++k) {
            const uint32_t v = s_w[k];
            if (k < w) pre += v;
            all += v;
        }
        if (tid < RPT) rowpre[(size_t)t * RPT + tid] = pre + incl - c;
        if (tid == 0) {
            tot[2 * (size_t)t] = all & 0xFFFFu;
            tot[2 * (size_t)t + 1] = all >> 16;
        }
        __syncthreads();
    }
}

// Pass 3: scan.  One workgroup: gp[2t] and gp[2t+1] receive the exclusive
// prefixes over the level's tiles of the left- and right-misplaced totals.
template <int F>
__global__ __launch_bounds__(1024) void k_ip_scan(const Ctl *ctl, int par, const Seg<typename KeyOf<F>::type> *segs,
                                                  const uint32_t *tot, uint32_t *gp, uint32_t cap)
{
    using K = typename KeyOf<F>::type;
    constexpr int NW = 1024 / WAVE;
    __shared__ uint32_t s_l[NW], s_r[NW];
    uint32_t nseg = 0;
    const uint32_t ntiles = ip_level_tiles<K>(ctl, par, segs, cap, nseg);
    const int tid = threadIdx.x, lane = lane_id(), w = tid / WAVE;
    uint32_t carry_l = 0, carry_r = 0;
    for (uint32_t base = 0; base < ntiles; base += 1024) {
        const uint32_t i = base + (uint32_t)tid;
        const uint32_t vl = i < ntiles ? tot[2 * (size_t)i] : 0u, vr = i < ntiles ? tot[2 * (size_t)i + 1] : 0u;
        const uint32_t il = wave_incl_scan(vl), ir = wave_incl_scan(vr);
        if (lane == WAVE - 1) {
            s_l[w] = il;
            s_r[w] = ir;
        }
        __syncthreads();
        uint32_t pl = 0, pr = 0, al = 0, ar = 0;
#pragma unroll
        for (int k = 0; k < NW; ++k) {
            const uint32_t a = s_l[k], b = s_r[k];
            if (k < w) {
                pl += a;
                pr += b;
            }
            al += a;
            ar += b;
        }
        if (i < ntiles) {
            gp[2 * (size_t)i] = carry_l + pl + il - vl;
            gp[2 * (size_t)i + 1] = carry_r + pr + ir - vr;
        }
        carry_l += al;
        carry_r += ar;
        __syncthreads();
    }
}

// Lane `src` (wave-uniform) of a 64-bit value.
__device__ __forceinline__ uint64_t lane_get64(uint64_t v, uint32_t src)
{
    return ((uint64_t)lane_bcast((uint32_t)(v >> 32), (int)src) << 32) | lane_bcast((uint32_t)v, (int)src);
}

// Pass 4: swap.  Workgroups take tiles with left-misplaced keys; wave w
// takes a contiguous run of the tile's rows before mid.  The partners of a
// run's left-misplaced keys are consecutive right-misplaced keys of the
// segment, so the wave finds the first one by a 64-way search (over the
// segment's tiles, then the tile's rows: wave-uniform) and then walks
// forward through the right-misplaced bits row by row, handing partners to
// its lanes in rank order.  The masks of the run's rows and of the next 64
// right rows sit one per lane (one load each), so the walk itself reads
// registers; the exchanges of SB rows are issued together, their loads all
// in flight before the first store.
template <int F>
__global__ __launch_bounds__(IP_NT) void k_ip_swap(Ctl *ctl, int par, const Seg<typename KeyOf<F>::type> *segs,
                                                   const unsigned long long *cur, const uint64_t *mask,
                                                   const uint32_t *rowpre, const uint32_t *tot, const uint32_t *gp,
                                                   Raw raw, uint32_t cap)
{
    using K = typename KeyOf<F>::type;
    constexpr int RPT = ip_rows<K>();
    constexpr int NW = IP_NT / WAVE;
    constexpr uint32_t CH = (RPT + NW - 1) / NW;  // rows per wave
    // rows whose exchanges are issued together: 4 keeps the kernel under 64
    // VGPRs, so 8 waves per SIMD stay resident to hide the walk's latencies
    // (8 rows in flight per wave, at 5 waves per SIMD, was slower)
    constexpr int SB = 4;
    static_assert(CH <= (uint32_t)WAVE && CH % SB == 0, "a wave's rows fit one mask per lane");
    // per wave: position of the r-th set bit of the current right row in slot r
    __shared__ uint32_t s_pos[NW][WAVE];
    uint32_t nseg = 0;
    const uint32_t ntiles = ip_level_tiles<K>(ctl, par, segs, cap, nseg);
    const int tid = threadIdx.x, lane = lane_id();
    const uint32_t w = (uint32_t)__builtin_amdgcn_readfirstlane(tid / WAVE);
    for (uint32_t t = blockIdx.x; t < ntiles; t += gridDim.x) {
        if (tot[2 * (size_t)t] == 0) continue;
        const uint32_t s = ip_find_seg_wave<K>(segs, nseg, t, lane);
        const Seg<K> sg = segs[s];
        uint32_t p0, cnt;
        ip_tile_range<K>(sg, t, p0, cnt);
        const uint32_t t0 = sg.tile0, tend = t0 + seg_tiles<K>(sg.b, sg.e);
        const uint32_t mid = sg.b + (uint32_t)cur[(size_t)s * CUR_STRIDE];
        const uint32_t lim = ip_left_limit(mid, p0, cnt);
        const uint32_t rbeg = w * CH, rend = min(rbeg + CH, (lim + WAVE - 1) / WAVE);
        if (rbeg >= rend) continue;
        const uint32_t pre_beg = rowpre[(size_t)t * RPT + rbeg] & 0xFFFFu;
        const uint32_t pre_end = rend < (uint32_t)RPT ? rowpre[(size_t)t * RPT + rend] & 0xFFFFu : tot[2 * (size_t)t];
        if (pre_beg == pre_end) continue;  // no left-misplaced key in this run of rows
        // the run's left-misplaced masks, row rbeg + k in lane k
        uint64_t own = 0;
        {
            const uint32_t r = rbeg + (uint32_t)lane;
            if (r < rend) {
                const uint32_t r0 = r * WAVE;
                own = ~mask[(size_t)t * RPT + r] & lanes_below(cnt - r0) & lanes_below(lim - r0);
            }
        }
        // global right index of the run's first partner
        const uint32_t g = gp[2 * (size_t)t0 + 1] + (gp[2 * (size_t)t] - gp[2 * (size_t)t0]) + pre_beg;
        uint32_t t2 = wave_search(t0, tend, g, [&](uint32_t i) { return gp[2 * (size_t)i + 1]; }, lane);
        const uint32_t q = g - gp[2 * (size_t)t2 + 1];
        uint32_t r2 = wave_search(0u, (uint32_t)RPT, q, [&](uint32_t i) { return rowpre[(size_t)t2 * RPT + i] >> 16; },
                                  lane);
        const uint32_t k2 = q - (rowpre[(size_t)t2 * RPT + r2] >> 16);
        // the walk: tile t2 (keys p02.., lim2 of them before mid), row r2, a
        // block of right-misplaced masks (row blk0 + k in lane k), and the bits
        // of row r2 not handed out yet
        uint32_t p02 = 0, cnt2 = 0, lim2 = 0, blk0 = 0;
        uint64_t blk = 0;
        auto load_block = [&]() {
            blk0 = r2;
            const uint32_t rr = r2 + (uint32_t)lane;
            blk = 0;
            if (rr < (uint32_t)RPT) {
                const uint32_t r0 = rr * WAVE;
                const uint64_t left = r0 < lim2 ? lanes_below(lim2 - r0) : 0ull;
                blk = mask[(size_t)t2 * RPT + rr] & ~left;
            }
        };
        ip_tile_range<K>(sg, t2, p02, cnt2);
        lim2 = ip_left_limit(mid, p02, cnt2);
        load_block();
        uint64_t m2 = lane_get64(blk, 0);
        bool bad = k2 >= popc(m2);
        if (!bad) m2 &= ~lanes_below(select_bit(m2, k2));  // drop the bits of earlier ranks
        for (uint32_t rb = rbeg; rb < rend && !bad; rb += SB) {
            uint32_t pl[SB], pr[SB];
            bool me[SB];
#pragma unroll
            for (int u = 0; u < SB; ++u) {
                const uint32_t r = rb + (uint32_t)u;
                me[u] = false;
                pl[u] = pr[u] = 0;
                if (r >= rend || bad) continue;
                const uint64_t mis = lane_get64(own, r - rbeg);
                const uint32_t c = popc(mis);
                if (c == 0) continue;
                const uint32_t j = mask_below(mis);
                me[u] = (mis >> lane) & 1ull;
                pl[u] = p0 + r * WAVE + (uint32_t)lane;
                uint32_t done = 0;
                while (done < c) {
                    if (m2 == 0) {  // next row of the segment
                        if (++r2 == (uint32_t)RPT) {
                            r2 = 0;
                            if (++t2 >= tend) {
                                bad = true;
                                break;
                            }
                            ip_tile_range<K>(sg, t2, p02, cnt2);
                            lim2 = ip_left_limit(mid, p02, cnt2);
                            load_block();
                        } else if (r2 - blk0 >= (uint32_t)WAVE) {
                            load_block();
                        }
                        m2 = lane_get64(blk, r2 - blk0);
                        continue;
                    }
                    const uint32_t a = popc(m2), take = min(a, c - done);
                    // the row's set bits, in rank order, to this wave's slots (LDS
                    // operations of one wave take effect in issue order)
                    if ((m2 >> lane) & 1ull) s_pos[w][mask_below(m2)] = (uint32_t)lane;
                    if (me[u] && j >= done && j < done + take) pr[u] = p02 + r2 * WAVE + s_pos[w][j - done];
                    if (take == a) {
                        m2 = 0ull;
                    } else {
                        const uint32_t cut = (uint32_t)__builtin_amdgcn_readfirstlane((int)s_pos[w][take]);
                        m2 &= ~lanes_below(cut);
                    }
                    done += take;
                }
                // the partner is a right-misplaced key of this segment; anything
                // else would mean inconsistent counts: flag it, move nothing
                if (me[u] && (bad || pr[u] < mid || pr[u] >= sg.e)) {
                    atomicOr(&ctl->err, ERR_CURSOR);
                    me[u] = false;
                }
            }
            RawElem<F> a[SB], b[SB];
#pragma unroll
            for (int u = 0; u < SB; ++u)
                if (me[u]) {
                    a[u] = raw_get<F>(raw, pl[u]);
                    b[u] = raw_get<F>(raw, pr[u]);
                }
#pragma unroll
            for (int u = 0; u < SB; ++u)
                if (me[u]) {
                    raw_put<F>(raw, pl[u], b[u]);
                    raw_put<F>(raw, pr[u], a[u]);
                }
        }
        if (bad && lane == 0) atomicOr(&ctl->err, ERR_CURSOR);
    }
}

}  // namespace hs
