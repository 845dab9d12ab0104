// hs_local.hpp -- the on-chip tier of the gfx950 hybrid quicksort.
//
// Segments of at most T keys, as left by the global partition levels
// (hs_kernels.hpp), are sorted on chip: one workgroup per task in LDS
// (k_local) -- three-way partition levels over all live sub-ranges at once
// while any is longer than a wave's span, then one wave per sub-range:
// partition levels with the keys in registers, and the bitonic network of
// the paper (Sec. III-A) in VGPRs for every sub-range of at most LW keys --
// and one wave per small task straight from global memory (k_small).
#pragma once

#include "hs_kernels.hpp"

namespace hs {

// ---------------------------------------------------------------- on-chip sort

// T: the on-chip segment limit (keys per task); NT: threads per workgroup;
// LEAF: the largest task sorted by one wave straight from global memory
// (k_small); LW: the largest range a wave of k_local hands to the bitonic
// network (larger ones are partitioned first); WPC: workgroups resident per
// CU (LDS: 160 KB per CU; WPC * NT / 256 waves per SIMD, which sets the VGPR
// budget: 8 waves, 64 VGPRs, for int32 and 8-byte words).  A wave partition
// level costs about 25 lane operations per key, the network's in-register
// layers 1 (32-bit words: a min/max pair) or 2.5 (64-bit words) per key and
// layer, so halving a range saves the network fewer operations than the
// level costs down to 512 keys for 64-bit words (measured: 512 beats 256 and
// 128), and 32-bit words go to the network from a span (1024 keys) on.
// 8-byte words: 1024-thread workgroups with spans of 512 keys (two per CU:
// the LDS of two 8192-key tasks), 5% faster than 512-thread ones.
template <typename K> struct LocalCfg;
template <> struct LocalCfg<uint32_t> { static constexpr int T = 8192, NT = 512, LEAF = 1024, LW = 1024, WPC = 4; };
template <> struct LocalCfg<uint64_t> { static constexpr int T = 8192, NT = 1024, LEAF = 512, LW = 512, WPC = 2; };
// 16-byte words: half the keys in the same LDS, eight rows per span.
template <> struct LocalCfg<u128> { static constexpr int T = 4096, NT = 512, LEAF = 256, LW = 256, WPC = 2; };
// A second shape for 8-byte words, taken when the on-chip limit is at most
// 4096 keys: half the keys per task in half the LDS (37 KB), so four
// workgroups share a CU, with eight rows of 64 keys per span and spans that
// go to the 512-key network whole.
template <typename K> struct LocalCfgHalf { static constexpr bool on = false; };
template <> struct LocalCfgHalf<uint64_t> {
    static constexpr bool on = true;
    static constexpr int T = 4096, NT = 512, LEAF = 512, LW = 512, WPC = 4;
};

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

// The paper's wrapper (Sec. III-A, "Sorting Small Arrays"): pad to the next
// network size with the greatest key and pick the network by size.
template <int LEAF, typename K, typename Ld, typename St>
__device__ __forceinline__ void wave_sort(uint32_t sz, int lane, const Ld &ld, const St &st)
{
    if (sz <= 64) wave_sort_n<1, K>(sz, lane, ld, st);
    else if (sz <= 128) wave_sort_n<2, K>(sz, lane, ld, st);
    else if (LEAF <= 256 || sz <= 256) wave_sort_n<4, K>(sz, lane, ld, st);
    else if constexpr (LEAF >= 512) {
        if (LEAF <= 512 || sz <= 512) wave_sort_n<8, K>(sz, lane, ld, st);
        else if constexpr (LEAF >= 1024) wave_sort_n<16, K>(sz, lane, ld, st);
    }
}

// Partition of one row of keys against pivot p (Sec. III-B; on chip with an
// equal class when the range calls for it): the slot of a lane's key is its
// class's running base plus the number of lanes of that class below it, and
// the bases advance by the class counts.  The class masks are the compares'
// ballots, so the bookkeeping is scalar and one ds_write per row places 64
// keys.

// Lanes of the row starting at position r0 that lie before position e.
__device__ __forceinline__ uint32_t lanes_to(uint32_t e, uint32_t r0)
{
    return e <= r0 ? 0u : min(e - r0, (uint32_t)WAVE);
}

// Class counts of the lanes of mask mk in one row against pivot p, added to
// the wave's running totals (the compares' ballots: scalar work).
template <typename K>
__device__ __forceinline__ void row_count(K x, K p, uint64_t mk, uint32_t &nl, uint32_t &nq)
{
    nl += popc(ballot(x < p) & mk);
    nq += popc(ballot(x == p) & mk);
}

// The lanes of mask mk (FULL: every lane) of one row go to their class's
// next slot: the class's base plus the number of lanes of the class below
// (mbcnt, the base riding in its accumulator); the bases then advance by
// the class counts.  THREE: classes < p, == p, > p (bases cl, ce, cg);
// otherwise < p and >= p (cl, cg).
template <bool FULL, bool THREE, typename K>
__device__ __forceinline__ void row_place(K *sk, K x, K p, uint64_t mk, uint32_t &cl, uint32_t &ce, uint32_t &cg,
                                          int lane)
{
    const uint64_t lt = ballot(x < p) & mk;
    uint32_t d;
    if constexpr (THREE) {
        const uint64_t eq = ballot(x == p) & mk, gt = mk & ~(lt | eq);
        d = lane_select(lt, mbcnt_add(lt, cl), lane_select(eq, mbcnt_add(eq, ce), mbcnt_add(gt, cg)));
        ce += popc(eq);
        cg += popc(gt);
    } else {
        const uint64_t ge = mk & ~lt;
        d = lane_select(lt, mbcnt_add(lt, cl), mbcnt_add(ge, cg));
        cg += popc(ge);
    }
    cl += popc(lt);
    if (FULL || ((mk >> lane) & 1ull)) sk[d] = x;
}

// Whether a range of m keys with nl keys below its pivot and ne equal to it
// is split three ways (< p, == p final, > p) rather than two (< p, >= p).
// Two ways is cheaper per row; it needs nl > 0 to make progress (the pivot
// is one of the range's keys, so then both sides are smaller than the
// range), and three ways retires a large run of keys equal to the pivot at
// once.
__device__ __forceinline__ bool split_three(uint32_t nl, uint32_t ne, uint32_t m)
{
    return nl == 0u || 32u * ne >= m;
}

// Per-range class counts as one 64-bit word: keys below the pivot, keys
// equal to it, and keys of the range counted (bits 0-15, 16-31, 32-47).
__device__ __forceinline__ unsigned long long pack_counts(uint32_t nl, uint32_t ne, uint32_t c)
{
    return (unsigned long long)(nl | (ne << 16)) | ((unsigned long long)c << 32);
}

// One wave sorts sk[b, e) (at most KR rows of 64 keys; the array has KR*64
// keys of slack past the task, so a row read past e stays in bounds).  A
// range longer than LW is partitioned three ways with its keys held in
// registers (row j: positions b + 64 j + lane): a first pass counts the
// classes from the compares' ballots, a second writes each key in place to
// its slot (every key of the range is in registers before the first write).
// Ranges of at most LW keys go through the bitonic network.  Pending ranges
// sit on a stack held across the lanes of one register (entry i in lane i);
// children that need the network are pushed last, so they are taken before
// any other partition, and the stack only ever holds disjoint ranges longer
// than LW, plus two.
template <int KR, int LW, typename K>
__device__ __forceinline__ void wave_qsort(K *sk, uint32_t b, uint32_t e, int rule, int lane)
{
    static_assert(LW >= WAVE && KR * WAVE / (LW + 1) + 2 <= WAVE, "the stack of pending ranges fits one register");
    uint32_t stk = 0;
    int sp = 0;
    for (;;) {
        b = (uint32_t)__builtin_amdgcn_readfirstlane((int)b);  // uniform: row masks stay scalar
        e = (uint32_t)__builtin_amdgcn_readfirstlane((int)e);
        const uint32_t s = e - b;
        if (LW >= KR * WAVE || s <= (uint32_t)LW) {
            if (s >= 2)
                wave_sort<LW, K>(s, lane, [&](uint32_t q) { return sk[b + q]; },
                                 [&](uint32_t q, K v) { sk[b + q] = v; });
        } else if constexpr (LW < KR * WAVE) {
            const K p = pick_pivot<K>([&](uint32_t i) { return sk[i]; }, b, e, rule);
            const uint32_t nf = s / WAVE, kp = s % WAVE;  // full rows; lanes of the last, partial row
            K x[KR];
            // every load first, in groups of four rows
#pragma unroll
            for (int g = 0; g < KR / 4; ++g)
                if (g == 0 || (uint32_t)(g * 4 * WAVE) < s)
#pragma unroll
                    for (int j = g * 4; j < g * 4 + 4; ++j) x[j] = sk[b + (uint32_t)(j * WAVE + lane)];
            uint32_t nl = 0, ne = 0;
#pragma unroll
            for (int j = 0; j < KR; ++j) {
                if ((uint32_t)j < nf) row_count(x[j], p, ~0ull, nl, ne);
                else if ((uint32_t)j == nf && kp) row_count(x[j], p, lanes_below(kp), nl, ne);
            }
            uint32_t cl = b, ce = b + nl, cg = b + nl + ne;
#pragma unroll
            for (int j = 0; j < KR; ++j) {
                if ((uint32_t)j < nf) row_place<true, true>(sk, x[j], p, ~0ull, cl, ce, cg, lane);
                else if ((uint32_t)j == nf && kp) row_place<false, true>(sk, x[j], p, lanes_below(kp), cl, ce, cg, lane);
            }
            const uint32_t le = b + nl, rb = le + ne;
            const uint32_t pl = b | (le << 16), pr = rb | (e << 16);
            const bool bl = nl > (uint32_t)LW, br = e - rb > (uint32_t)LW;
            auto push = [&](uint32_t v) { stk = lane == sp ? v : stk; ++sp; };
            if (bl) push(pl);
            if (br) push(pr);
            if (!bl && nl >= 2) push(pl);
            if (!br && e - rb >= 2) push(pr);
        }
        if (sp == 0) return;
        const uint32_t t = (uint32_t)__builtin_amdgcn_readlane((int)stk, --sp);
        b = t & 0xFFFFu;
        e = t >> 16;
    }
}

// One workgroup per task of LEAF+1 .. T keys, claimed dynamically (the next
// claim is issued at the start of a task so its latency hides behind it).
//
// Block levels.  Wave w owns the span [w*KW, (w+1)*KW) of the task; row j of
// the span is positions w*KW + 64 j + lane.  At each level every live range
// (longer than KW) is partitioned around its pivot, all of them at once.  A
// live range is longer than a span, so a span meets at most two: A, holding
// the span's first position, and B, starting inside the span; both are
// wave-uniform, and so is the split of each row between them.  Every wave
// takes the pivots of its A and B itself, from the same samples of the
// range (so all waves holding a range agree): the median of 32 evenly
// spaced keys, or the paper's 3-value median.  The
// compares' ballots count each class of A and B in the span; each wave
// publishes its counts and adds them to the ranges' totals (one 64-bit LDS
// atomic per range).  After one barrier every wave knows the totals and the
// counts of the waves before it, and writes its keys, still in registers, in
// place to their class's next slot: keys keep their order within a class.
// Wave 0 meanwhile builds the next level's live list and queues children of
// 2..KW keys; a second barrier ends the level.  The task's rows go to LDS as
// they are loaded and every level reads its rows from there, so one copy of
// the level's code serves all levels.
//
// Wave levels.  Waves take queued ranges one at a time and sort each with
// wave_qsort.  Should the queue fill up, it is drained before the next block
// level (queued ranges and live ranges are disjoint, so the waves need not
// wait for each other).  The sorted task is stored back in the caller's
// format.
template <int F, int NT, int T, int LW, int WPC>
__global__ __launch_bounds__(NT, WPC * NT / 256) void k_local(Ctl *ctl, const Task<typename KeyOf<F>::type> *tasks,
                                              typename KeyOf<F>::type *buf0, typename KeyOf<F>::type *buf1,
                                              Raw raw, int rule, uint32_t task_cap)
{
    using K = typename KeyOf<F>::type;
    constexpr int NW = NT / WAVE;             // waves
    constexpr int KPT = T / NT;               // rows per span
    constexpr int KW = KPT * WAVE;            // keys per span
    constexpr int MAXACT = T / (KW + 1) + 1;  // live ranges at once
    constexpr int MAXQ = 256;                 // queued ranges
    constexpr uint32_t NONE = 0xFFu;
    static_assert(NW * KW == T && 2 * MAXACT <= WAVE && NW <= 16 && T < 65536, "span layout");

    __shared__ K sk[T + KW];  // one span of slack: wave_qsort reads whole rows past its range
    __shared__ uint32_t qr[MAXQ];
    __shared__ uint32_t s_live[2][MAXACT];               // live ranges of a level (b | e << 16)
    __shared__ unsigned long long s_cnt[2][MAXACT];      // their class counts (pack_counts)
    __shared__ unsigned long long s_wc[NW][2];           // each wave's shares of its A and B
    __shared__ uint32_t s_na[2], s_nq, s_qnext, s_task[2];

    // the wave index is uniform: readfirstlane lets the compiler keep the
    // span's row masks and class bases in scalar registers
    const int tid = threadIdx.x, lane = lane_id(), w = __builtin_amdgcn_readfirstlane(tid / WAVE);
    const uint32_t sb = (uint32_t)w * KW;
    // tasks are claimed from ctl->task_next on (a second launch after more
    // partition levels starts where the first one's tasks ended); nothing is
    // sorted once a partition level has flagged an error
    const uint32_t ntask = ctl->err ? 0u : min(ctl->ntask, task_cap);

    // queued ranges [0, cnt), claimed through s_qnext, largest first when the
    // list fits a wave (every wave sorts the same claim order: (size, index)
    // words through the 64-lane network, so the k-th claim is lane 63 - k)
    auto drain = [&](uint32_t cnt) {
        const bool lpt = cnt <= (uint32_t)WAVE;
        uint32_t ord[1] = {0u};
        if (lpt) {
            if ((uint32_t)lane < cnt) {
                const uint32_t t = qr[lane];
                ord[0] = (((t >> 16) - (t & 0xFFFFu)) << 6) | (uint32_t)lane;
            }
            bitonic_wave<1>(ord, lane);
        }
        for (;;) {
            uint32_t k = 0;
            if (lane == 0) k = atomicAdd(&s_qnext, 1u);
            k = (uint32_t)__builtin_amdgcn_readfirstlane((int)k);
            if (k >= cnt) break;
            const uint32_t t = qr[lpt ? (lane_bcast(ord[0], WAVE - 1 - (int)k) & (WAVE - 1)) : k];
            wave_qsort<KPT, LW, K>(sk, t & 0xFFFFu, t >> 16, rule, lane);
        }
    };

    if (tid == 0) s_task[0] = atomicAdd(&ctl->task_next, 1u);
    __syncthreads();
    uint32_t ti = s_task[0];
    for (int par = 1;; par ^= 1) {
        if (ti >= ntask) break;
        uint32_t next = 0;
        if (tid == 0) next = atomicAdd(&ctl->task_next, 1u);  // consumed at the end of the task
        const Task<K> tk = tasks[ti];
        const uint32_t b = tk.b, m = tk.e - tk.b;
        const K *sbuf = tk.src == SRC_BUF0 ? buf0 : buf1;
        const bool sraw = tk.src == SRC_RAW;

        // live list (lane s: packed range s) and queue length, identical in
        // every wave
        uint32_t na = 0, nq = 0, ent = 0;
        // the span's rows, straight from global memory; rows past the task read
        // its last key (kept out of every class by the row masks)
        K x[KPT];
        const uint32_t g0 = b + sb + (uint32_t)lane, glast = b + m - 1;
        if (sraw) {
#pragma unroll
            for (int j = 0; j < KPT; ++j) x[j] = raw_load<F>(raw, min(g0 + (uint32_t)(j * WAVE), glast));
        } else {
#pragma unroll
            for (int j = 0; j < KPT; ++j) x[j] = sbuf[min(g0 + (uint32_t)(j * WAVE), glast)];
        }
        {  // the rows to LDS (every level reads its rows and pivot samples there)
            const int rem = (int)m - (int)(sb + (uint32_t)lane);
#pragma unroll
            for (int j = 0; j < KPT; ++j)
                if (j * WAVE < rem) sk[sb + (uint32_t)(j * WAVE + lane)] = x[j];
        }
        if (m > (uint32_t)KW) {
            na = 1;
            ent = lane == 0 ? m << 16 : 0u;
        } else {
            nq = 1;
            if (tid == 0) qr[0] = m << 16;
        }
        if (tid < 2 * MAXACT) (&s_cnt[0][0])[tid] = 0ull;
        if (tid == 0) s_qnext = 0;
        __syncthreads();

        int lp = 0;            // which of the two live-list / count buffers this level uses
        bool reset_q = false;  // the queue was drained before this level
        // one block level (one copy of its code serves every level: the
        // kernel's hot code stays within the instruction cache)
        auto level = [&]() {
            const bool lv = lane < (int)na;
            const uint32_t eb = ent & 0xFFFFu, ee = ent >> 16;
            const uint64_t mA = ballot(lv && eb <= sb && sb < ee);
            const uint64_t mB = ballot(lv && sb < eb && eb < sb + (uint32_t)KW);
            const uint32_t iA = mA ? (uint32_t)__builtin_ctzll(mA) : NONE;
            const uint32_t iB = mB ? (uint32_t)__builtin_ctzll(mB) : NONE;
            uint32_t bA = 0, eA = 0, bB = 0, eB = 0;
            if (iA != NONE) {
                const uint32_t t = lane_bcast(ent, (int)iA);
                bA = t & 0xFFFFu;
                eA = t >> 16;
            }
            if (iB != NONE) {
                const uint32_t t = lane_bcast(ent, (int)iB);
                bB = t & 0xFFFFu;
                eB = t >> 16;
            }
            // the span's rows
#pragma unroll
            for (int j = 0; j < KPT; ++j) x[j] = sk[sb + (uint32_t)(j * WAVE + lane)];

            // ---- pivots of A and B (keys of the range; every wave holding a
            //      range takes the same samples)
            K pA = 0, pB = 0;
            if (rule == PIVOT_MEDIAN3) {
                if (iA != NONE) pA = med3<K>(sk[bA], sk[bA + (eA - bA - 1) / 2], sk[eA - 1]);
                if (iB != NONE) pB = med3<K>(sk[bB], sk[bB + (eB - bB - 1) / 2], sk[eB - 1]);
            } else {
                // lanes 0-31 sample A, lanes 32-63 sample B; the first five stages of
                // the one-key network sort each half on its own
                const bool hb = lane >= WAVE / 2;
                const bool has = hb ? iB != NONE : iA != NONE;
                const uint32_t rb = hb ? bB : bA, rn = hb ? eB - bB : eA - bA;
                const uint32_t at = has ? rb + ((rn - 1) * (uint32_t)(lane & 31)) / 31u : 0u;
                K v = sk[at];
                bitonic_lanes<5>(v, lane);
                pA = lane_bcast(v, 15);
                pB = lane_bcast(v, 47);
            }

            // row j of the span (positions r0 = sb + 64 j ..): A holds its lanes
            // [0, kA), B its lanes [kB, 64); lanes in between belong to no live
            // range.  Both bounds are uniform, and so is every branch on them.
            auto row_split = [&](int j, uint32_t &kA, uint32_t &kB) {
                const uint32_t r0 = sb + (uint32_t)(j * WAVE);
                kA = iA != NONE ? lanes_to(eA, r0) : 0u;
                kB = iB != NONE ? lanes_to(bB, r0) : (uint32_t)WAVE;
            };
            // the span lies inside A (then B is absent): every row is a full A row
            const bool fullA = iA != NONE && eA >= sb + (uint32_t)KW;

            // ---- pass 1: class counts of A and B in this span
            uint32_t al = 0, aq = 0, bl = 0, bq = 0;
            if (fullA) {
#pragma unroll
                for (int j = 0; j < KPT; ++j) row_count(x[j], pA, ~0ull, al, aq);
            } else {
#pragma unroll
                for (int j = 0; j < KPT; ++j) {
                    uint32_t kA, kB;
                    row_split(j, kA, kB);
                    if (kA) row_count(x[j], pA, lanes_below(kA), al, aq);
                    if (kB < (uint32_t)WAVE) row_count(x[j], pB, ~lanes_below(kB), bl, bq);
                }
            }
            // this wave's shares of A and B: published for the waves after it,
            // and added to the ranges' totals
            if (lane == 0) {
                const unsigned long long cA = iA != NONE ? pack_counts(al, aq, min(eA, sb + (uint32_t)KW) - sb) : 0ull;
                const unsigned long long cB = iB != NONE ? pack_counts(bl, bq, min(eB, sb + (uint32_t)KW) - bB) : 0ull;
                s_wc[w][0] = cA;
                s_wc[w][1] = cB;
                if (iA != NONE) atomicAdd(&s_cnt[lp][iA], cA);
                if (iB != NONE) atomicAdd(&s_cnt[lp][iB], cB);
            }
            __syncthreads();
            if (reset_q && tid == 0) s_qnext = 0;  // every wave is past its drain
            // the shares of A held by the waves before this one (lane l: wave l;
            // A is the B of its first wave unless it starts at that wave's span);
            // B starts in this span, so no earlier wave holds any of it.  Keys
            // thus keep their order within each class: the split is stable.
            unsigned long long preA = 0;
            if (iA != NONE) {
                const uint32_t wa0 = bA / (uint32_t)KW;
                unsigned long long v = 0;
                if ((uint32_t)lane < (uint32_t)w && (uint32_t)lane >= wa0)
                    v = s_wc[lane][(uint32_t)lane == wa0 && bA % (uint32_t)KW != 0u ? 1 : 0];
                v += xor_lanes<1>((uint64_t)v, lane);
                v += xor_lanes<2>((uint64_t)v, lane);
                v += xor_lanes<4>((uint64_t)v, lane);
                if constexpr (NW > 8) v += xor_lanes<8>((uint64_t)v, lane);
                preA = lane_bcast((uint64_t)v, 0);
            }
            const unsigned long long preB = 0;

            // ---- class bases of this wave's share of A and B
            uint32_t aL = 0, aE = 0, aG = 0, gL = 0, gE = 0, gG = 0;
            bool threeA = false, threeB = false;
            auto bases = [&](uint32_t i, uint32_t rb, uint32_t re, unsigned long long pre, bool &three,
                             uint32_t &cl, uint32_t &ce, uint32_t &cg) {
                const unsigned long long t = s_cnt[lp][i];
                const uint32_t nl = (uint32_t)t & 0xFFFFu, ne = ((uint32_t)t >> 16) & 0xFFFFu;
                const uint32_t pl = (uint32_t)pre & 0xFFFFu, pe = ((uint32_t)pre >> 16) & 0xFFFFu,
                               pc = (uint32_t)(pre >> 32);
                three = split_three(nl, ne, re - rb);
                cl = rb + pl;
                ce = rb + nl + pe;
                cg = three ? rb + nl + ne + (pc - pl - pe) : rb + nl + (pc - pl);
            };
            if (iA != NONE) bases(iA, bA, eA, preA, threeA, aL, aE, aG);
            if (iB != NONE) bases(iB, bB, eB, preB, threeB, gL, gE, gG);

            // ---- next level's live list and queued children (wave 0, lane s:
            //      range s), published before the barrier that ends the level
            if (w == 0) {
                uint32_t lb = 0, le = 0, rb = 0, re = 0;
                if (lv) {
                    const unsigned long long t = s_cnt[lp][lane];
                    const uint32_t nl = (uint32_t)t & 0xFFFFu, ne = ((uint32_t)t >> 16) & 0xFFFFu;
                    lb = eb;
                    le = eb + nl;
                    rb = split_three(nl, ne, ee - eb) ? le + ne : le;
                    re = ee;
                }
                const bool aLv = le - lb > (uint32_t)KW, aRv = re - rb > (uint32_t)KW;
                const bool qL = le - lb >= 2u && !aLv, qR = re - rb >= 2u && !aRv;
                const uint32_t na_me = (uint32_t)aLv + (uint32_t)aRv, nq_me = (uint32_t)qL + (uint32_t)qR;
                const uint32_t ai = wave_incl_scan(na_me), qi = wave_incl_scan(nq_me);
                uint32_t ap = ai - na_me, qp = nq + qi - nq_me;
                if (aLv) s_live[lp ^ 1][ap++] = lb | (le << 16);
                if (aRv) s_live[lp ^ 1][ap] = rb | (re << 16);
                if (qL) qr[qp++] = lb | (le << 16);
                if (qR) qr[qp] = rb | (re << 16);
                if (lane < MAXACT) s_cnt[lp ^ 1][lane] = 0ull;
                if (lane == WAVE - 1) {
                    s_na[lp ^ 1] = ai;
                    s_nq = nq + qi;
                }
            }

            // ---- pass 2: every key to its class's next slot, in place
            if (fullA) {
                if (threeA) {
#pragma unroll
                    for (int j = 0; j < KPT; ++j) row_place<true, true>(sk, x[j], pA, ~0ull, aL, aE, aG, lane);
                } else {
#pragma unroll
                    for (int j = 0; j < KPT; ++j) row_place<true, false>(sk, x[j], pA, ~0ull, aL, aE, aG, lane);
                }
            } else {
#pragma unroll
                for (int j = 0; j < KPT; ++j) {
                    uint32_t kA, kB;
                    row_split(j, kA, kB);
                    if (kA) {
                        if (threeA) row_place<false, true>(sk, x[j], pA, lanes_below(kA), aL, aE, aG, lane);
                        else row_place<false, false>(sk, x[j], pA, lanes_below(kA), aL, aE, aG, lane);
                    }
                    if (kB < (uint32_t)WAVE) {
                        if (threeB) row_place<false, true>(sk, x[j], pB, ~lanes_below(kB), gL, gE, gG, lane);
                        else row_place<false, false>(sk, x[j], pB, ~lanes_below(kB), gL, gE, gG, lane);
                    }
                }
            }
            __syncthreads();
            lp ^= 1;
            na = s_na[lp];
            nq = s_nq;
            ent = lane < (int)na ? s_live[lp][lane] : 0u;
        };

        while (na) {
            reset_q = nq + 2u * MAXACT > (uint32_t)MAXQ;
            if (reset_q) {  // make room: sort what is queued
                drain(nq);
                nq = 0;
            }
            level();
        }
        drain(nq);
        __syncthreads();
        {  // LDS -> registers -> global, in the caller's format
            const int rem = (int)m - tid;  // row j holds a key of the task if j * NT < rem
#pragma unroll
            for (int j = 0; j < KPT; ++j) x[j] = sk[j * NT + tid];
#pragma unroll
            for (int j = 0; j < KPT; ++j)
                if (j * NT < rem) raw_store<F>(raw, b + (uint32_t)(j * NT + tid), x[j]);
        }
        if (tid == 0) s_task[par] = next;
        __syncthreads();
        ti = s_task[par];
    }
}

// A whole array of at most LEAF keys: one wave loads it, sorts it with the
// network and stores it back.  Nothing here can fail; lane 0 clears the
// error word a graph plan reads after its replays.  The host sends arrays of
// up to wave_net<K>() keys this way (one wave alone on a SIMD has the
// registers for 16 eight-byte or 8 sixteen-byte keys per lane).
template <typename K> constexpr int wave_net() { return sizeof(K) <= 8 ? 1024 : 512; }
template <int F, int LEAF>
__global__ __launch_bounds__(WAVE) void k_sort_wave(Ctl *ctl, Raw raw, uint32_t n)
{
    using K = typename KeyOf<F>::type;
    const int lane = lane_id();
    if (lane == 0) ctl->err = 0u;
    wave_sort<LEAF, K>(n, lane, [&](uint32_t p) { return raw_load<F>(raw, p); },
                       [&](uint32_t j, K v) { raw_store<F>(raw, j, v); });
}

// A whole array of LEAF+1 .. T keys is one on-chip task: one block clears
// the control block and writes the task, for a one-workgroup k_local.
template <int F>
__global__ __launch_bounds__(256) void k_init_one_task(Ctl *ctl, Task<typename KeyOf<F>::type> *tasks, uint32_t n)
{
    using K = typename KeyOf<F>::type;
    for (uint32_t i = threadIdx.x; i < (uint32_t)(sizeof(Ctl) / 4); i += blockDim.x) ((uint32_t *)ctl)[i] = 0u;
    __syncthreads();
    if (threadIdx.x == 0) {
        Task<K> tk;
        tk.b = 0;
        tk.e = n;
        tk.src = SRC_RAW;
        tk.kind = TASK_LOCAL;
        tk.fill = 0;
        tasks[0] = tk;
        ctl->ntask = 1;
        ctl->local_keys = n;
    }
}

// Small tasks, from the back of the task list: a range of at most LEAF keys
// goes straight from HBM through the bitonic network to the caller's array,
// and a fill task writes its key over its range.  With fewer than four tasks
// per wave, waves take one task each in a grid-stride loop.  With more, they
// take groups of four consecutive tasks: when all four sorts of a group fit
// 16 keys, one wave sorts them together, a quarter of its lanes each (the
// network's first four stages stay inside 16-lane groups); when they fit 32
// keys, two at a time on half-waves; otherwise one after another.
//
// small_first: the small tasks before it are done already (a second launch
// after more partition levels sorts only the tasks they added).  Nothing is
// sorted once a partition level has flagged an error.
template <int F, int LEAF>
__global__ __launch_bounds__(256) void k_small(const Ctl *ctl, const Task<typename KeyOf<F>::type> *tasks,
                                               const typename KeyOf<F>::type *buf0,
                                               const typename KeyOf<F>::type *buf1, Raw raw, uint32_t task_cap,
                                               uint32_t small_first)
{
    using K = typename KeyOf<F>::type;
    const int lane = lane_id();
    const uint32_t nall = ctl->err ? 0u : min(ctl->nsmall, task_cap);
    const uint32_t nsmall = nall > small_first ? nall - small_first : 0u;
    const uint32_t nwaves = gridDim.x * (blockDim.x / WAVE);
    auto task_at = [&](uint32_t i) { return tasks[task_cap - 1 - small_first - i]; };
    auto ld = [&](const Task<K> &tk, uint32_t j) {
        return tk.src == SRC_RAW ? raw_load<F>(raw, tk.b + j) : (tk.src == SRC_BUF0 ? buf0 : buf1)[tk.b + j];
    };
    auto one = [&](const Task<K> &tk) {
        const uint32_t b = tk.b, m = tk.e - tk.b;
        if (tk.kind == TASK_FILL) {
            for (uint32_t j = (uint32_t)lane; j < m; j += WAVE) raw_store<F>(raw, b + j, tk.fill);
        } else if (tk.src == SRC_RAW) {
            wave_sort<LEAF, K>(m, lane, [&](uint32_t p) { return raw_load<F>(raw, b + p); },
                               [&](uint32_t j, K v) { raw_store<F>(raw, b + j, v); });
        } else {
            const K *sbuf = tk.src == SRC_BUF0 ? buf0 : buf1;
            wave_sort<LEAF, K>(m, lane, [&](uint32_t p) { return sbuf[b + p]; },
                               [&](uint32_t j, K v) { raw_store<F>(raw, b + j, v); });
        }
    };
    // lanes [gw*g, gw*(g+1)) sort task i (of m keys) with a network of gw lanes
    auto packed = [&](uint32_t i, bool has, uint32_t r, auto STAGES) {
        Task<K> tk;
        tk.b = tk.e = 0;
        tk.src = SRC_RAW;
        if (has) tk = task_at(i);
        const uint32_t m = tk.e - tk.b;
        K v = key_max<K>();
        if (has && r < m) v = ld(tk, r);
        bitonic_lanes<decltype(STAGES)::value>(v, lane);
        if (has && r < m) raw_store<F>(raw, tk.b + r, v);
    };
    const uint32_t wv = (blockIdx.x * blockDim.x + threadIdx.x) / WAVE;
    if (nsmall < 4u * nwaves) {  // too few tasks to group: one task per wave keeps every wave busy
        for (uint32_t i = wv; i < nsmall; i += nwaves) one(task_at(i));
        return;
    }
    for (uint32_t g = wv; 4ull * g < nsmall; g += nwaves) {
        const uint32_t i0 = 4 * g;
        // sizes of the group's four tasks, one per quarter-wave (past the end: none)
        const uint32_t iq = i0 + (uint32_t)(lane >> 4);
        uint32_t mq = 0;
        bool fill = false;
        if (iq < nsmall) {
            const Task<K> tq = task_at(iq);
            mq = tq.e - tq.b;
            fill = tq.kind == TASK_FILL;
        }
        if (ballot(fill || mq > 16u) == 0) {
            packed(iq, iq < nsmall, (uint32_t)(lane & 15), std::integral_constant<int, 4>{});
        } else if (ballot(fill || mq > 32u) == 0) {
#pragma unroll
            for (uint32_t h = 0; h < 2; ++h) {
                const uint32_t ih = i0 + 2 * h + (uint32_t)(lane >> 5);
                packed(ih, ih < nsmall, (uint32_t)(lane & 31), std::integral_constant<int, 5>{});
            }
        } else {
            for (uint32_t q = 0; q < 4 && i0 + q < nsmall; ++q) one(task_at(i0 + q));
        }
    }
}

}  // namespace hs
