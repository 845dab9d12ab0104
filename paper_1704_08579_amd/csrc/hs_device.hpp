// hs_device.hpp -- device primitives of the gfx950 hybrid sort.
//
//  * order-key codecs: the caller's int32 / uint32 / int64 / float64 /
//    (int32 key, int32 value) / (float64 key, int32 value) formats are
//    mapped to unsigned words whose unsigned order is the key order, so
//    every kernel compares plain unsigned integers;
//  * wavefront (64-lane) scan and lane shuffles;
//  * the same-direction bitonic network of the paper (Sec. II-A, Fig. 2
//    caption; Sec. III-A, Algorithms 1 and 2) held in VGPRs of one wave.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>
#include <utility>

namespace hs {

constexpr int WAVE = 64;

enum Fmt : int { FMT_I32 = 0, FMT_F64 = 1, FMT_KV = 2, FMT_U32 = 3, FMT_I64 = 4, FMT_KV_F64 = 5 };

// 128-bit order word of a (float64 key, int32 value) pair.
using u128 = unsigned __int128;

template <int F> struct KeyOf { using type = uint64_t; };
template <> struct KeyOf<FMT_I32> { using type = uint32_t; };
template <> struct KeyOf<FMT_U32> { using type = uint32_t; };
template <> struct KeyOf<FMT_KV_F64> { using type = u128; };

// Bytes of one key in the caller's key array.
template <int F> constexpr int raw_key_bytes() { return F == FMT_F64 || F == FMT_I64 || F == FMT_KV_F64 ? 8 : 4; }

// Formats with a value array beside the key array.
template <int F> constexpr bool has_vals() { return F == FMT_KV || F == FMT_KV_F64; }

// The caller's arrays, in the caller's format.
struct Raw {
    void *keys;
    int32_t *vals;  // key/value sorts only
};

// ---------------------------------------------------------------- codecs
//
// int32 and int64: flipping the sign bit maps two's-complement order onto
// unsigned order; uint32 keys are their own order words.  float64: IEEE
// 754-2008 totalOrder -- negative values (sign bit set) have every bit
// inverted, non-negative values get the sign bit set.
// key/value: the key's order word in the high half and the value's bits in
// the low half (int32 keys: a 64-bit word; float64 keys: a 128-bit word, the
// value in its low 32 bits), so a pair moves as one word and ties between
// equal keys are broken by value (the method is unstable, so any tie order
// is a valid output; this one is deterministic).

__device__ __forceinline__ uint32_t enc_i32(uint32_t bits) { return bits ^ 0x80000000u; }
__device__ __forceinline__ uint32_t dec_i32(uint32_t k) { return k ^ 0x80000000u; }
__device__ __forceinline__ uint64_t enc_f64(uint64_t b)
{
    return (b >> 63) ? ~b : (b | 0x8000000000000000ull);
}
__device__ __forceinline__ uint64_t dec_f64(uint64_t k)
{
    return (k >> 63) ? (k & 0x7fffffffffffffffull) : ~k;
}
__device__ __forceinline__ uint64_t enc_kv(uint32_t key, uint32_t val)
{
    return ((uint64_t)enc_i32(key) << 32) | val;
}
__device__ __forceinline__ u128 enc_kv_f64(uint64_t key_bits, uint32_t val)
{
    return ((u128)enc_f64(key_bits) << 64) | (u128)val;
}
__device__ __forceinline__ uint64_t enc_i64(uint64_t b) { return b ^ 0x8000000000000000ull; }
__device__ __forceinline__ uint64_t dec_i64(uint64_t k) { return k ^ 0x8000000000000000ull; }

// Order word of one key of a single-array format, from its raw bits.
template <int F> __device__ __forceinline__ typename KeyOf<F>::type enc_word(typename KeyOf<F>::type b)
{
    if constexpr (F == FMT_I32) return enc_i32(b);
    else if constexpr (F == FMT_U32) return b;
    else if constexpr (F == FMT_F64) return enc_f64(b);
    else return enc_i64(b);
}

template <int F>
__device__ __forceinline__ typename KeyOf<F>::type raw_load(const Raw &r, uint32_t i)
{
    if constexpr (F == FMT_KV) {
        return enc_kv(((const uint32_t *)r.keys)[i], (uint32_t)r.vals[i]);
    } else if constexpr (F == FMT_KV_F64) {
        return enc_kv_f64(((const uint64_t *)r.keys)[i], (uint32_t)r.vals[i]);
    } else {
        using K = typename KeyOf<F>::type;
        return enc_word<F>(((const K *)r.keys)[i]);
    }
}

template <int F>
__device__ __forceinline__ void raw_store(const Raw &r, uint32_t i, typename KeyOf<F>::type k)
{
    if constexpr (F == FMT_I32) {
        ((uint32_t *)r.keys)[i] = dec_i32(k);
    } else if constexpr (F == FMT_U32) {
        ((uint32_t *)r.keys)[i] = k;
    } else if constexpr (F == FMT_F64) {
        ((uint64_t *)r.keys)[i] = dec_f64(k);
    } else if constexpr (F == FMT_I64) {
        ((uint64_t *)r.keys)[i] = dec_i64(k);
    } else if constexpr (F == FMT_KV_F64) {
        ((uint64_t *)r.keys)[i] = dec_f64((uint64_t)(k >> 64));
        r.vals[i] = (int32_t)(uint32_t)k;
    } else {
        ((uint32_t *)r.keys)[i] = dec_i32((uint32_t)(k >> 32));
        r.vals[i] = (int32_t)(uint32_t)k;
    }
}

template <typename K> __device__ __forceinline__ constexpr K key_max() { return ~K(0); }

// ---------------------------------------------------------------- lanes

__device__ __forceinline__ int lane_id() { return (int)__lane_id(); }

// Lane exchanges.  xor_lanes<ML>(v) returns v from lane (lane ^ ML).  The
// masks used by the bitonic network map onto cheap gfx950 forms:
//   ML = 1, 2, 3     DPP quad_perm
//   ML = 7, 15       DPP row_half_mirror / row_mirror
//   ML = 4, 8        two DPP moves (lane^7^3, lane^15^7)
//   ML = 16, 31      ds_swizzle in bit-mask mode (xor within 32 lanes)
//   ML = 32          v_permlane32_swap
//   ML = 63          ds_swizzle xor 31, then v_permlane32_swap
// and everything else falls back to ds_bpermute.
template <int CTRL> __device__ __forceinline__ uint32_t dpp_mov(uint32_t v)
{
    return (uint32_t)__builtin_amdgcn_mov_dpp((int)v, CTRL, 0xF, 0xF, false);
}

constexpr int DPP_QP_XOR1 = 0xB1;  // quad_perm [1,0,3,2]
constexpr int DPP_QP_XOR2 = 0x4E;  // quad_perm [2,3,0,1]
constexpr int DPP_QP_XOR3 = 0x1B;  // quad_perm [3,2,1,0]
constexpr int DPP_ROW_MIRROR = 0x140;
constexpr int DPP_ROW_HALF_MIRROR = 0x141;

__device__ __forceinline__ uint32_t swap32_partner(uint32_t v, int lane)
{
    const auto r = __builtin_amdgcn_permlane32_swap(v, v, false, false);
    return lane < 32 ? (uint32_t)r[1] : (uint32_t)r[0];
}

template <int ML> __device__ __forceinline__ uint32_t xor_lanes(uint32_t v, int lane)
{
    if constexpr (ML == 1) return dpp_mov<DPP_QP_XOR1>(v);
    else if constexpr (ML == 2) return dpp_mov<DPP_QP_XOR2>(v);
    else if constexpr (ML == 3) return dpp_mov<DPP_QP_XOR3>(v);
    else if constexpr (ML == 4) return dpp_mov<DPP_QP_XOR3>(dpp_mov<DPP_ROW_HALF_MIRROR>(v));
    else if constexpr (ML == 7) return dpp_mov<DPP_ROW_HALF_MIRROR>(v);
    else if constexpr (ML == 8) return dpp_mov<DPP_ROW_HALF_MIRROR>(dpp_mov<DPP_ROW_MIRROR>(v));
    else if constexpr (ML == 15) return dpp_mov<DPP_ROW_MIRROR>(v);
    else if constexpr (ML == 16) return (uint32_t)__builtin_amdgcn_ds_swizzle((int)v, (16 << 10) | 0x1F);
    else if constexpr (ML == 31) return (uint32_t)__builtin_amdgcn_ds_swizzle((int)v, (31 << 10) | 0x1F);
    else if constexpr (ML == 32) return swap32_partner(v, lane);
    else if constexpr (ML == 63)
        return swap32_partner((uint32_t)__builtin_amdgcn_ds_swizzle((int)v, (31 << 10) | 0x1F), lane);
    else return (uint32_t)__builtin_amdgcn_ds_bpermute((lane ^ ML) << 2, (int)v);
}

template <int ML> __device__ __forceinline__ uint64_t xor_lanes(uint64_t v, int lane)
{
    const uint32_t lo = xor_lanes<ML>((uint32_t)v, lane);
    const uint32_t hi = xor_lanes<ML>((uint32_t)(v >> 32), lane);
    return ((uint64_t)hi << 32) | lo;
}
template <int ML> __device__ __forceinline__ u128 xor_lanes(u128 v, int lane)
{
    const uint64_t lo = xor_lanes<ML>((uint64_t)v, lane);
    const uint64_t hi = xor_lanes<ML>((uint64_t)(v >> 64), lane);
    return ((u128)hi << 64) | lo;
}

// Inclusive prefix sum over the 64 lanes of a wave: four DPP row shifts
// give the scan inside each row of 16 lanes, then two row broadcasts carry
// row totals forward (rows 1 and 3 from lane 15 / 47, rows 2 and 3 from
// lane 31).
__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t v)
{
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x111, 0xF, 0xF, false);  // row_shr:1
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x112, 0xF, 0xF, false);  // row_shr:2
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x114, 0xF, 0xF, false);  // row_shr:4
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x118, 0xF, 0xF, false);  // row_shr:8
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x142, 0xA, 0xF, false);  // row_bcast:15
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x143, 0xC, 0xF, false);  // row_bcast:31
    return v;
}

// Broadcast lane `src` (wave-uniform) to every lane.
__device__ __forceinline__ uint32_t lane_bcast(uint32_t v, int src)
{
    return (uint32_t)__builtin_amdgcn_readlane((int)v, src);
}
__device__ __forceinline__ uint64_t lane_bcast(uint64_t v, int src)
{
    return ((uint64_t)lane_bcast((uint32_t)(v >> 32), src) << 32) | lane_bcast((uint32_t)v, src);
}
__device__ __forceinline__ u128 lane_bcast(u128 v, int src)
{
    return ((u128)lane_bcast((uint64_t)(v >> 64), src) << 64) | lane_bcast((uint64_t)v, src);
}

// Number of set bits of a 64-bit lane mask below the calling lane.
__device__ __forceinline__ uint32_t mask_below(uint64_t m)
{
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}

// base + mask_below(m), the base riding in mbcnt's accumulator.
__device__ __forceinline__ uint32_t mbcnt_add(uint64_t m, uint32_t base)
{
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, base));
}

// The lanes whose predicate holds, as a wave-uniform 64-bit mask.
__device__ __forceinline__ uint64_t ballot(bool p) { return __builtin_amdgcn_ballot_w64(p); }

__device__ __forceinline__ uint32_t popc(uint64_t m) { return (uint32_t)__builtin_popcountll(m); }

// a in the lanes of mask m, b elsewhere: one v_cndmask.  Written out because
// the compiler otherwise turns a select between mbcnt results into branches
// under the exec mask, one per arm.
__device__ __forceinline__ uint32_t lane_select(uint64_t m, uint32_t a, uint32_t b)
{
    // the mask is wave-uniform; readfirstlane keeps it in scalar registers
    // whatever the compiler concluded about it
    const uint64_t ms = ((uint64_t)(uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)(m >> 32)) << 32) |
                        (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)m);
    uint32_t d;
    asm("v_cndmask_b32 %0, %1, %2, %3" : "=v"(d) : "v"(b), "v"(a), "s"(ms));
    return d;
}

// Lanes [0, k) (every lane for k >= 64).
__device__ __forceinline__ uint64_t lanes_below(uint32_t k) { return k >= 64u ? ~0ull : ((1ull << k) - 1ull); }

// Sum of v over the wave, in every lane.
__device__ __forceinline__ uint32_t wave_sum(uint32_t v) { return lane_bcast(wave_incl_scan(v), WAVE - 1); }

// ---------------------------------------------------------------- static loops

template <int B, int E, typename Fn>
__device__ __forceinline__ void static_for(Fn &&fn)
{
    if constexpr (B < E) {
        fn(std::integral_constant<int, B>{});
        static_for<B + 1, E>(fn);
    }
}

constexpr int ilog2(int x) { return x <= 1 ? 0 : 1 + ilog2(x >> 1); }
constexpr int hibit(int x) { return x <= 1 ? x : (hibit(x >> 1) << 1); }

// ---------------------------------------------------------------- bitonic network
//
// A wave holds N = 64*KPL keys, KPL per lane, network index i = lane*KPL + j
// for register j.  One comparator layer with XOR mask M pairs i with i ^ M;
// the lower index keeps the minimum.  When M < KPL both partners sit in the
// same lane and the exchange is a register min/max; otherwise the partner of
// register j is register j ^ (M mod KPL) of lane ^ (M / KPL).  Since every
// key format used here is an injective order word (equal words are equal
// bits), min/max exchanges are exact: a pad with the greatest word and a
// real element equal to it are indistinguishable.

template <int M, int KPL, typename K>
__device__ __forceinline__ void cmpx_layer(K (&x)[KPL], int lane)
{
    if constexpr (M < KPL) {
#pragma unroll
        for (int j = 0; j < KPL; ++j) {
            const int jp = j ^ M;
            if (j < jp) {
                const K a = x[j], b = x[jp];
                const bool lt = a < b;
                x[j] = lt ? a : b;
                x[jp] = lt ? b : a;
            }
        }
    } else {
        constexpr int ML = M / KPL;
        constexpr int MR = M % KPL;
        constexpr int HB = hibit(ML);
        const bool lower = (lane & HB) == 0;
        K y[KPL];
#pragma unroll
        for (int j = 0; j < KPL; ++j) y[j] = xor_lanes<ML>(x[j ^ MR], lane);
#pragma unroll
        for (int j = 0; j < KPL; ++j) {
            const K a = x[j], b = y[j];
            const bool lt = a < b;
            x[j] = (lower == lt) ? a : b;
        }
    }
}

// Stage s merges sorted runs of 2^(s-1) into runs of 2^s: the mirror layer
// (mask 2^s - 1, "extremities to the centre"), then half-cleaners at
// distances 2^(s-2) .. 1 ("linear progression").
// The first STAGES stages of the one-key-per-lane network: none of their
// layers pairs lanes of different groups of 2^STAGES consecutive lanes, so
// every such group ends up sorted on its own and one wave sorts 64 / 2^STAGES
// independent arrays at once.
template <int STAGES, typename K>
__device__ __forceinline__ void bitonic_lanes(K &v, int lane)
{
    K x[1] = {v};
    static_for<1, STAGES + 1>([&](auto S) {
        constexpr int s = decltype(S)::value;
        cmpx_layer<(1 << s) - 1, 1>(x, lane);
        static_for<0, (s >= 2 ? s - 1 : 0)>([&](auto I) {
            constexpr int t = s - 2 - decltype(I)::value;
            cmpx_layer<(1 << t), 1>(x, lane);
        });
    });
    v = x[0];
}

template <int KPL, typename K>
__device__ __forceinline__ void bitonic_wave(K (&x)[KPL], int lane)
{
    constexpr int LOGN = 6 + ilog2(KPL);
    static_for<1, LOGN + 1>([&](auto S) {
        constexpr int s = decltype(S)::value;
        cmpx_layer<(1 << s) - 1, KPL>(x, lane);
        static_for<0, (s >= 2 ? s - 1 : 0)>([&](auto I) {
            constexpr int t = s - 2 - decltype(I)::value;
            cmpx_layer<(1 << t), KPL>(x, lane);
        });
    });
}

}  // namespace hs
