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
// CU (LDS: 160 KB per CU; registers: 16 waves per CU keep the 128-VGPR
// budget that a span of keys per lane needs).  A wave partition level costs
// about 25 lane operations per key, the network's in-register layers 1
// (32-bit words: a min/max pair) or 2.5 (64-bit words) per key and layer, so
// halving a range saves the network fewer operations than the level costs
// down to 512 keys for 64-bit words (measured: 512 beats 256 and 128), and
// 32-bit words go to the network from a span (1024 keys) on.
template <typename K> struct LocalCfg;
template <> struct LocalCfg<uint32_t> { static constexpr int T = 8192, NT = 512, LEAF = 1024, LW = 1024, WPC = 4; };
template <> struct LocalCfg<uint64_t> { static constexpr int T = 8192, NT = 512, LEAF = 512, LW = 512, WPC = 2; };
// 16-byte words: half the keys in the same LDS, eight rows per span.
template <> struct LocalCfg<u128> { static constexpr int T = 4096, NT = 512, LEAF = 256, LW = 256, WPC = 2; };

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

// Three-way partition of one row of keys against pivot p (Sec. III-B, with
// an equal class, as the on-chip levels use it): the slot of a lane's key is
// its class's running base plus the number of lanes of that class below it,
// and the bases advance by the class counts.  row_slot takes a full row;
// row_slot_in a row whose range holds the lanes of mask mk, k0 being the
// lowest of them.  The class masks are the compares' ballots, so the
// bookkeeping is scalar and one ds_write per row places 64 keys.
template <typename K>
__device__ __forceinline__ uint32_t row_slot(K x, K p, uint32_t &cl, uint32_t &ce, uint32_t &cg, int lane)
{
    const uint64_t ml = ballot(x < p), mq = ballot(x == p);
    const uint32_t rl = mask_below(ml), rq = mask_below(mq);
    const uint32_t d = lane_select(ml, cl + rl, lane_select(mq, ce + rq, cg + ((uint32_t)lane - rl - rq)));
    const uint32_t nl = popc(ml), nq = popc(mq);
    cl += nl;
    ce += nq;
    cg += (uint32_t)WAVE - nl - nq;
    return d;
}
template <typename K>
__device__ __forceinline__ uint32_t row_slot_in(K x, K p, uint64_t mk, uint32_t k0, uint32_t &cl, uint32_t &ce,
                                                uint32_t &cg, int lane)
{
    const uint64_t ml = ballot(x < p) & mk, mq = ballot(x == p) & mk;
    const uint32_t rl = mask_below(ml), rq = mask_below(mq);
    const uint32_t d = lane_select(ml, cl + rl, lane_select(mq, ce + rq, cg + ((uint32_t)lane - k0 - rl - rq)));
    const uint32_t nl = popc(ml), nq = popc(mq);
    cl += nl;
    ce += nq;
    cg += popc(mk) - nl - nq;
    return d;
}

// One wave sorts sk[b, e) (at most KR rows of 64 keys; the array has KR*64
// keys of slack past the task, so a row read past e stays in bounds).  A
// range longer than LW is partitioned three ways with its keys held in
// registers (row j: positions b + 64 j + lane): a first pass counts the
// classes in per-lane counters, a second writes each key in place to its
// slot (every key of the range is in registers before the first write).
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
            uint32_t vl = 0, vq = 0;
#pragma unroll
            for (int j = 0; j < KR; ++j) {
                if ((uint32_t)j < nf) {
                    vl += (uint32_t)(x[j] < p);
                    vq += (uint32_t)(x[j] == p);
                } else if ((uint32_t)j == nf) {
                    const bool in = (uint32_t)lane < kp;
                    vl += (uint32_t)(in && x[j] < p);
                    vq += (uint32_t)(in && x[j] == p);
                }
            }
            const uint32_t c = wave_sum(vl | (vq << 16));
            const uint32_t nl = c & 0xFFFFu, ne = c >> 16;
            uint32_t cl = b, ce = b + nl, cg = b + nl + ne;
#pragma unroll
            for (int j = 0; j < KR; ++j) {
                if ((uint32_t)j < nf) {
                    sk[row_slot(x[j], p, cl, ce, cg, lane)] = x[j];
                } else if ((uint32_t)j == nf && kp) {
                    const uint32_t d = row_slot_in(x[j], p, lanes_below(kp), 0u, cl, ce, cg, lane);
                    if ((uint32_t)lane < kp) sk[d] = x[j];
                }
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
// (longer than KW) is partitioned three ways around its pivot, all of them
// at once.  A live range is longer than a span, so a span meets at most two:
// A, holding the span's first position, and B, starting inside the span;
// both are wave-uniform, and so is the split of each row between them.  Two
// compares per row give the class masks as ballots; each wave publishes its
// class counts for A and B, and after one barrier every wave knows where
// its keys of each class go.  The keys, still in registers, are written in
// place to their class's next slot (running base + mbcnt of the class
// mask), and a second barrier ends the level.  The live list is held in
// lanes (lane s: range s, with its pivot), computed identically by every
// wave from per-range totals published by the wave holding the range's
// first position; children of 2..KW keys are queued for the waves.
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
    static_assert(NW * KW == T && 2 * MAXACT <= WAVE && T < 65536, "span layout");

    __shared__ K sk[T + KW];  // one span of slack: wave_qsort reads whole rows past its range
    __shared__ uint32_t qr[MAXQ];
    __shared__ uint32_t wl[NW][MAXACT];
    __shared__ __align__(16) uint32_t wcnt[NW][4];
    __shared__ uint32_t s_qnext, s_task[2];

    // the wave index is uniform: readfirstlane lets the compiler keep the
    // span's row masks and class bases in scalar registers
    const int tid = threadIdx.x, lane = lane_id(), w = __builtin_amdgcn_readfirstlane(tid / WAVE);
    const uint32_t sb = (uint32_t)w * KW;
    const uint32_t ntask = min(ctl->ntask, task_cap);
    auto lds_rd = [&](uint32_t p) { return sk[p]; };

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
        auto g_rd = [&](uint32_t i) { return sraw ? raw_load<F>(raw, b + i) : sbuf[b + i]; };

        // live list (lane s: packed range s and its pivot) and queue length,
        // identical in every wave
        uint32_t na = 0, nq = 0, ent = 0;
        K pv = 0;
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
        if (m > (uint32_t)KW) {
            na = 1;
            ent = m << 16;
            pv = pick_pivot<K>(g_rd, 0, m, rule);
        } else {
            nq = 1;
            const int rem = (int)m - (int)(sb + (uint32_t)lane);
#pragma unroll
            for (int j = 0; j < KPT; ++j)
                if (j * WAVE < rem) sk[sb + (uint32_t)(j * WAVE + lane)] = x[j];
            if (tid == 0) qr[0] = m << 16;
        }
        if (tid == 0) s_qnext = 0;
        __syncthreads();

        bool reset_q = false;  // the queue was drained before this level
        // one block level; FIRST: the rows are in x already
        auto level = [&](auto FIRST) {
            constexpr bool first = decltype(FIRST)::value;
            const bool lv = lane < (int)na;
            const uint32_t eb = ent & 0xFFFFu, ee = ent >> 16;
            const uint64_t mA = ballot(lv && eb <= sb && sb < ee);
            const uint64_t mB = ballot(lv && sb < eb && eb < sb + (uint32_t)KW);
            const uint32_t iA = mA ? (uint32_t)__builtin_ctzll(mA) : NONE;
            const uint32_t iB = mB ? (uint32_t)__builtin_ctzll(mB) : NONE;
            uint32_t bA = 0, eA = 0, bB = 0;
            K pA = 0, pB = 0;
            if (iA != NONE) {
                const uint32_t t = lane_bcast(ent, (int)iA);
                bA = t & 0xFFFFu;
                eA = t >> 16;
                pA = lane_bcast(pv, (int)iA);
            }
            if (iB != NONE) {
                bB = lane_bcast(ent, (int)iB) & 0xFFFFu;
                pB = lane_bcast(pv, (int)iB);
            }
            // rows of the span: [0, jAf) are all A, row jAf holds A in lanes
            // [0, kAp), row jBs holds B in lanes [kBp, 64), rows past jBs are all B
            const uint32_t jAf = iA != NONE ? min((eA - sb) / WAVE, (uint32_t)KPT) : 0u;
            const uint32_t kAp = (iA != NONE && eA - sb < (uint32_t)KW) ? (eA - sb) % WAVE : 0u;
            const uint32_t jBs = iB != NONE ? (bB - sb) / WAVE : (uint32_t)KPT;
            const uint32_t kBp = iB != NONE ? (bB - sb) % WAVE : 0u;
            if constexpr (!first) {
#pragma unroll
                for (int j = 0; j < KPT; ++j) x[j] = sk[sb + (uint32_t)(j * WAVE + lane)];
            }

            // ---- pass 1: class counts of A and B, per lane
            uint32_t al = 0, aq = 0, bl = 0, bq = 0;
#pragma unroll
            for (int j = 0; j < KPT; ++j) {
                if ((uint32_t)j < jAf) {
                    al += (uint32_t)(x[j] < pA);
                    aq += (uint32_t)(x[j] == pA);
                } else if ((uint32_t)j > jBs) {
                    bl += (uint32_t)(x[j] < pB);
                    bq += (uint32_t)(x[j] == pB);
                } else if ((uint32_t)j == jAf || (uint32_t)j == jBs) {
                    const bool inA = (uint32_t)j == jAf && (uint32_t)lane < kAp;
                    const bool inB = (uint32_t)j == jBs && (uint32_t)lane >= kBp;
                    al += (uint32_t)(inA && x[j] < pA);
                    aq += (uint32_t)(inA && x[j] == pA);
                    bl += (uint32_t)(inB && x[j] < pB);
                    bq += (uint32_t)(inB && x[j] == pB);
                }
            }
            const uint32_t cA = wave_sum(al | (aq << 16)), cB = wave_sum(bl | (bq << 16));
            if (lane == 0) *(uint4 *)&wcnt[w][0] = make_uint4(cA, cB, iA, iB);
            __syncthreads();
            if (reset_q && tid == 0) s_qnext = 0;  // every wave is past its drain
            // ---- per-range totals (lane s: range s) and, for A, the counts of the
            //      waves before this one
            uint32_t tot = 0, pre = 0;
#pragma unroll
            for (int l = 0; l < NW; ++l) {
                const uint4 c = *(const uint4 *)&wcnt[l][0];
                const uint32_t v = (c.z == (uint32_t)lane ? c.x : 0u) + (c.w == (uint32_t)lane ? c.y : 0u);
                tot += v;
                pre += l < w ? v : 0u;
            }
            const uint32_t totA = iA != NONE ? lane_bcast(tot, (int)iA) : 0u;
            const uint32_t preA = iA != NONE ? lane_bcast(pre, (int)iA) : 0u;
            const uint32_t totB = iB != NONE ? lane_bcast(tot, (int)iB) : 0u;
            // ---- children: live ones (> KW keys) form the next list, 2..KW keys are
            //      queued (by wave 0, before the barrier that ends the level)
            uint32_t na_n, ent_n;
            {
                uint32_t lb = 0, le = 0, rb = 0, re = 0;
                if (lv) {
                    lb = eb;
                    le = eb + (tot & 0xFFFFu);
                    rb = le + (tot >> 16);
                    re = ee;
                }
                const bool aL = le - lb > (uint32_t)KW, aR = re - rb > (uint32_t)KW;
                const bool qL = le - lb >= 2u && !aL, qR = re - rb >= 2u && !aR;
                const uint32_t na_me = (uint32_t)aL + (uint32_t)aR, nq_me = (uint32_t)qL + (uint32_t)qR;
                const uint32_t ai = wave_incl_scan(na_me), qi = wave_incl_scan(nq_me);
                uint32_t ap = ai - na_me, qp = nq + qi - nq_me;
                if (aL) wl[w][ap++] = lb | (le << 16);
                if (aR) wl[w][ap] = rb | (re << 16);
                if (w == 0) {
                    if (qL) qr[qp++] = lb | (le << 16);
                    if (qR) qr[qp] = rb | (re << 16);
                }
                na_n = lane_bcast(ai, WAVE - 1);
                nq += lane_bcast(qi, WAVE - 1);
                ent_n = lane < (int)na_n ? wl[w][lane] : 0u;  // this wave's own slots: no barrier
            }
            // ---- pass 2: every key to its class's next slot, in place
            {
                const uint32_t nlA = totA & 0xFFFFu, neA = totA >> 16, plA = preA & 0xFFFFu, peA = preA >> 16;
                uint32_t aL = bA + plA, aE = bA + nlA + peA, aG = bA + nlA + neA + (sb - bA) - plA - peA;
                const uint32_t nlB = totB & 0xFFFFu, neB = totB >> 16;
                uint32_t gL = bB, gE = bB + nlB, gG = bB + nlB + neB;
#pragma unroll
                for (int j = 0; j < KPT; ++j) {
                    if ((uint32_t)j < jAf) {
                        sk[row_slot(x[j], pA, aL, aE, aG, lane)] = x[j];
                    } else if ((uint32_t)j > jBs) {
                        sk[row_slot(x[j], pB, gL, gE, gG, lane)] = x[j];
                    } else {
                        if ((uint32_t)j == jAf && kAp) {
                            const uint32_t d = row_slot_in(x[j], pA, lanes_below(kAp), 0u, aL, aE, aG, lane);
                            if ((uint32_t)lane < kAp) sk[d] = x[j];
                        }
                        if ((uint32_t)j == jBs) {
                            const uint32_t d = row_slot_in(x[j], pB, ~lanes_below(kBp), kBp, gL, gE, gG, lane);
                            if ((uint32_t)lane >= kBp) sk[d] = x[j];
                        }
                    }
                }
            }
            __syncthreads();
            na = na_n;
            ent = ent_n;
            pv = 0;
            if (lane < (int)na) pv = pick_pivot<K>(lds_rd, ent & 0xFFFFu, ent >> 16, rule);
        };

        if (na) level(std::true_type{});
        while (na) {
            reset_q = nq + 2u * MAXACT > (uint32_t)MAXQ;
            if (reset_q) {  // make room: sort what is queued
                drain(nq);
                nq = 0;
            }
            level(std::false_type{});
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
template <int F, int LEAF>
__global__ __launch_bounds__(256) void k_small(const Ctl *ctl, const Task<typename KeyOf<F>::type> *tasks,
                                               const typename KeyOf<F>::type *buf0,
                                               const typename KeyOf<F>::type *buf1, Raw raw, uint32_t task_cap)
{
    using K = typename KeyOf<F>::type;
    const int lane = lane_id();
    const uint32_t nsmall = min(ctl->nsmall, task_cap);
    const uint32_t nwaves = gridDim.x * (blockDim.x / WAVE);
    auto task_at = [&](uint32_t i) { return tasks[task_cap - 1 - i]; };
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
