// hs_sort.hip -- host runtime and C ABI of the gfx950 hybrid sort.
//
// Drives the kernels of hs_kernels.hpp level by level (the recursion of
// Sec. III-C, Algorithm 4, one partition level per launch), owns the cached
// per-device workspace and implements every entry point of hsort.h.
#include <hip/hip_runtime.h>

#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "hs_inplace.hpp"
#include "hs_kernels.hpp"
#include "hs_learned.hpp"
#include "hs_local.hpp"
#include "hsort.h"

namespace {

using namespace hs;

constexpr int LMAX = 96;  // cap on global partition levels per call
// k_finalize workgroups (1024 threads) per compute unit: at the deepest
// levels a level has tens of thousands of segments, one wave each, and every
// wave waits on its samples' loads; a workgroup appends its waves' items with
// one atomic per list.
constexpr int FIN_BLOCKS_PER_CU = 2;
constexpr int FIN_NT = 1024;

thread_local std::string g_err;

int fail(int code, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

#define HS_HIP(call)                                                                    \
    do {                                                                                \
        hipError_t e_ = (call);                                                         \
        if (e_ != hipSuccess) return fail(HS_EHIP, "%s: %s", #call, hipGetErrorString(e_)); \
    } while (0)

// Launch a kernel and turn a launch error into HS_EHIP.
#define HS_LAUNCH(kernel, grid, block, stream, ...)                                     \
    do {                                                                                \
        hipLaunchKernelGGL(kernel, dim3(grid), dim3(block), 0, stream, __VA_ARGS__);    \
        HS_LAUNCHED();                                                                  \
    } while (0)

#define HS_LAUNCHED()                                                                   \
    do {                                                                                \
        hipError_t e_ = hipGetLastError();                                              \
        if (e_ != hipSuccess) return fail(HS_EHIP, "kernel launch: %s", hipGetErrorString(e_)); \
    } while (0)

// ---------------------------------------------------------------- per-device state

struct DevState {
    bool probed = false;
    bool supported = false;
    int ncu = 0;
    void *ws = nullptr;
    size_t ws_bytes = 0;
    Ctl *h_ctl = nullptr;        // pinned host mirror of the control block
    hipEvent_t last = nullptr;   // end of the last call that used the cached workspace
    hipEvent_t ev[2 * LMAX + 8] = {};  // timing events (stats only)
    LearnCtl *h_lctl = nullptr;  // pinned host mirror of the learned front end's scalars
    std::mutex mu;               // one call at a time per device
};

constexpr int MAXDEV = 64;
DevState g_dev[MAXDEV];
std::mutex g_probe_mu;

int get_device(DevState **out)
{
    int dev = 0;
    HS_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= MAXDEV) return fail(HS_EUNSUPPORTED, "device index %d out of range", dev);
    DevState &d = g_dev[dev];
    std::lock_guard<std::mutex> lk(g_probe_mu);
    if (!d.probed) {
        hipDeviceProp_t prop;
        HS_HIP(hipGetDeviceProperties(&prop, dev));
        d.supported = std::strncmp(prop.gcnArchName, "gfx950", 6) == 0;
        d.ncu = prop.multiProcessorCount;
        if (d.supported) {
            HS_HIP(hipHostMalloc((void **)&d.h_ctl, sizeof(Ctl), hipHostMallocDefault));
            HS_HIP(hipHostMalloc((void **)&d.h_lctl, sizeof(LearnCtl), hipHostMallocDefault));
            HS_HIP(hipEventCreateWithFlags(&d.last, hipEventDisableTiming));
            for (auto &e : d.ev) HS_HIP(hipEventCreate(&e));
        }
        d.probed = true;
        if (!d.supported) return fail(HS_EUNSUPPORTED, "device %d is %s, this library is built for gfx950", dev,
                                      prop.gcnArchName);
    }
    if (!d.supported) return fail(HS_EUNSUPPORTED, "device %d is not gfx950", dev);
    *out = &d;
    return HS_OK;
}

// ---------------------------------------------------------------- workspace layout

size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

// Parameters of the learned front end of one call.
struct LearnParams {
    bool on = false;
    int mode = JUDGE_AUTO;
    uint32_t m = 0;        // training sample
    uint32_t h = 0;        // held-out sample
    int steps = 0;
    float lr = 0.f;
    uint64_t seed = 0;
};

constexpr int LEARN_STEPS = 100;
constexpr int LEARN_LOG2M = 16;
constexpr float LEARN_LR = 3e-2f;
constexpr uint32_t LEARN_HOLDOUT = 1u << 14;
constexpr uint32_t MW_GMAX = 2048;  // multiway workgroups at most

LearnParams learn_params(const hs_opts *o, int64_t n, int op)
{
    LearnParams P;
    if (!o || o->method != HS_METHOD_LEARNED || op == HS_OP_SORT_SEGMENTED_I32 || op == HS_OP_SORT_SEGMENTED_F64 ||
        op == HS_OP_PARTITION_I32)
        return P;
    P.on = true;
    P.mode = (o->learn_flags & HS_LEARN_FORCE_SAMPLE) ? JUDGE_SAMPLE
             : (o->learn_flags & HS_LEARN_FORCE_MODEL) ? JUDGE_MODEL : JUDGE_AUTO;
    const int lg = o->sample_log2 > 0 ? o->sample_log2 : LEARN_LOG2M;
    P.m = 1u << lg;
    P.h = LEARN_HOLDOUT;
    P.steps = o->train_steps > 0 ? o->train_steps : LEARN_STEPS;
    P.lr = o->learning_rate > 0.f ? o->learning_rate : LEARN_LR;
    P.seed = o->seed;
    (void)n;
    return P;
}

// Guard words (HSORT_GUARD=1 in the environment): 256 bytes after every
// region of the workspace, filled with a pattern before a sort and checked
// after it, so a kernel writing past the end of a buffer, list or counter
// block fails the call instead of going unnoticed.
constexpr int MAX_GUARDS = 40;
constexpr uint32_t GUARD_WORD = 0x5AFE6A2Du;
bool guards_on()
{
    const char *e = std::getenv("HSORT_GUARD");
    return e && e[0] && !(e[0] == '0' && e[1] == 0);
}
struct Guards {
    uint32_t n;
    uint64_t off[MAX_GUARDS];
};

// One workgroup of 64 threads per 256-byte guard: fill it with the pattern,
// and count the words that no longer hold it.
__global__ void k_guard_fill(char *ws, Guards g, uint32_t word)
{
    if (blockIdx.x < g.n) ((uint32_t *)(ws + g.off[blockIdx.x]))[threadIdx.x] = word;
}
__global__ void k_guard_check(const char *ws, Guards g, uint32_t word, unsigned long long *bad)
{
    if (blockIdx.x >= g.n) return;
    const bool diff = ((const uint32_t *)(ws + g.off[blockIdx.x]))[threadIdx.x] != word;
    const uint64_t m = ballot(diff);
    if (lane_id() == 0 && m) atomicAdd(bad, (unsigned long long)popc(m));
}

struct Layout {
    size_t buf0 = 0, buf1 = 0, segA = 0, segB = 0, curA = 0, curB = 0, tasks = 0, ctl = 0, total = 0;
    Guards guards{};
    size_t guard_count = 0;  // one counter word for the check
    // levels partitioned in place: key bits, row prefixes, tile totals and prefixes
    size_t ipmask = 0, iprow = 0, iptot = 0, ipgp = 0;
    uint32_t cand_cap = 0, task_cap = 0;
    // learned front end (LearnParams::on)
    size_t smp_k = 0, smp_v = 0, sub = 0, z = 0, y = 0, par = 0, mom = 0, vel = 0, part = 0, lossb = 0,
           msplit = 0, ssplit = 0, chosen = 0, hold = 0, lctl = 0, hist = 0, btot = 0, bstart = 0, feat = 0;
    size_t sub_bytes = 0;
};

template <typename K>
Layout make_layout(int op, int64_t n, int64_t nseg, uint32_t T, const LearnParams &P = LearnParams(),
                   bool inplace = false)
{
    Layout L;
    size_t off = 0;
    const bool guards = guards_on();
    auto take = [&](size_t bytes) {
        size_t at = off;
        off = align_up(off + bytes, 256);
        if (guards && L.guards.n < (uint32_t)MAX_GUARDS) {
            L.guards.off[L.guards.n++] = off;
            off += 256;
        }
        return at;
    };
    const size_t sk = sizeof(K);
    if (op == HS_OP_PARTITION_I32) {
        L.cand_cap = 1;
        L.task_cap = 1;
        if (!inplace) L.buf1 = take((size_t)n * 4);
    } else {
        L.cand_cap = (uint32_t)(n / ((int64_t)T + 1) + 2);
        const bool seg = op == HS_OP_SORT_SEGMENTED_I32 || op == HS_OP_SORT_SEGMENTED_F64;
        L.task_cap = (uint32_t)((seg ? nseg : 1) + 2ll * LMAX * L.cand_cap + 4);
        // the multiway pass routes up to NB_MAX buckets, fills in chunks
        if (P.on) L.task_cap += (uint32_t)(NB_MAX + n / FILL_CHUNK + 2);
        if (!inplace) {
            L.buf1 = take((size_t)n * sk);
            if (op == HS_OP_SORT_KV_I32 || op == HS_OP_SORT_KV_F64) L.buf0 = take((size_t)n * sk);
        }
    }
    if (inplace) {
        // a level's tiles: the full tiles of its keys plus at most two partial
        // tiles per segment
        const size_t tiles = (size_t)n / PartCfg<K>::TILE + 2ull * L.cand_cap + 2;
        const size_t rows = tiles * (size_t)ip_rows<K>();
        L.ipmask = take(rows * 8);
        L.iprow = take(rows * 4);
        L.iptot = take(tiles * 8);
        L.ipgp = take(tiles * 8);
    }
    L.segA = take((size_t)L.cand_cap * sizeof(Seg<K>));
    L.segB = take((size_t)L.cand_cap * sizeof(Seg<K>));
    L.curA = take((size_t)L.cand_cap * 8 * CUR_STRIDE);
    L.curB = take((size_t)L.cand_cap * 8 * CUR_STRIDE);
    L.tasks = take((size_t)L.task_cap * sizeof(Task<K>));
    L.ctl = take(sizeof(Ctl));
    if (P.on) {
        // The training sample is sorted by a nested plain sort with its own
        // sub-workspace.
        const Layout S = make_layout<K>(op, P.m, 1, T);
        const size_t rk = op == HS_OP_SORT_F64 || op == HS_OP_SORT_I64 || op == HS_OP_SORT_KV_F64 ? 8 : 4;
        L.smp_k = take((size_t)P.m * rk);
        if (op == HS_OP_SORT_KV_I32 || op == HS_OP_SORT_KV_F64) L.smp_v = take((size_t)P.m * 4);
        L.sub = take(S.total);
        L.sub_bytes = S.total;
        L.feat = take((size_t)P.m * 8);
        L.z = take((size_t)ntrain_of(P.m) * 4);
        L.y = take((size_t)ntrain_of(P.m) * 4);
        L.par = take(MLP_NP * 4);
        L.mom = take(MLP_NP * 4);
        L.vel = take(MLP_NP * 4);
        const size_t gblk = (ntrain_of(P.m) + 255) / 256;
        L.part = take(2 * gblk * MLP_PS * 4);  // two halves: the training steps alternate
        L.lossb = take((2 * gblk + 1) * 4);    // per-workgroup losses (two halves), then the mean
        L.msplit = take(NSPLIT * sizeof(K));
        L.ssplit = take(NSPLIT * sizeof(K));
        L.chosen = take(NSPLIT * sizeof(K));
        L.hold = take((size_t)P.h * sizeof(K));
        L.lctl = take(sizeof(LearnCtl));
        L.hist = take((size_t)NB_MAX * MW_GMAX * 4);
        L.btot = take(NB_MAX * 4);
        L.bstart = take((NB_MAX + 1) * 4);
    }
    if (guards) L.guard_count = take(8);
    L.total = off;
    return L;
}

template <typename K> uint32_t local_limit(const hs_opts *o)
{
    const uint32_t Tmax = (uint32_t)LocalCfg<K>::T;
    if (!o || o->local_T <= 0) return Tmax;
    return (uint32_t)o->local_T < Tmax ? (uint32_t)o->local_T : Tmax;
}

int pivot_rule(const hs_opts *o) { return (o && o->pivot_rule > 0) ? o->pivot_rule : PIVOT_SAMPLE; }

// The largest task one wave sorts alone (routing bound of the task lists).
template <typename K> uint32_t leaf_limit(const hs_opts *o)
{
    const uint32_t Lmax = (uint32_t)LocalCfg<K>::LEAF;
    if (!o || o->leaf <= 0) return Lmax;
    return (uint32_t)o->leaf < Lmax ? (uint32_t)o->leaf : Lmax;
}

int check_learn(const hs_opts *o)
{
    if (!o) return HS_OK;
    if (o->driver != HS_DRIVER_AUTO && o->driver != HS_DRIVER_PERSISTENT && o->driver != HS_DRIVER_HOST)
        return fail(HS_EINVAL, "unknown driver %d", o->driver);
    if (o->spin_limit < 0) return fail(HS_EINVAL, "spin_limit is negative");
    if (o->leaf != 0 && (o->leaf < 64 || o->leaf > 1024 || (o->leaf & (o->leaf - 1))))
        return fail(HS_EINVAL, "leaf = %d is not a power of two in 64..1024", o->leaf);
    if (o->local_T < 0) return fail(HS_EINVAL, "local_T = %d is negative", o->local_T);
    if (o->autotune != 0 && o->autotune != 1) return fail(HS_EINVAL, "autotune = %d is not 0 or 1", o->autotune);
    if (o->method != HS_METHOD_PLAIN && o->method != HS_METHOD_LEARNED)
        return fail(HS_EINVAL, "unknown method %d", o->method);
    if (o->method == HS_METHOD_LEARNED) {
        if (o->sample_log2 != 0 && (o->sample_log2 < 10 || o->sample_log2 > 20))
            return fail(HS_EINVAL, "sample_log2 = %d outside 10..20", o->sample_log2);
        if (o->train_steps < 0 || o->train_steps > 100000)
            return fail(HS_EINVAL, "train_steps = %d outside 0..100000", o->train_steps);
        if (!(o->learning_rate >= 0.f) || o->learning_rate > 1.f)
            return fail(HS_EINVAL, "learning_rate outside [0, 1]");
        if ((o->learn_flags & ~(HS_LEARN_FORCE_MODEL | HS_LEARN_FORCE_SAMPLE)) ||
            o->learn_flags == (HS_LEARN_FORCE_MODEL | HS_LEARN_FORCE_SAMPLE))
            return fail(HS_EINVAL, "learn_flags = 0x%x is invalid", o->learn_flags);
    }
    if (o->inplace != 0 && o->inplace != 1) return fail(HS_EINVAL, "inplace = %d is not 0 or 1", o->inplace);
    if (o->inplace) {
        // the in-place levels run with the host-driven loop; the multiway pass
        // and the persistent driver write to a second buffer
        if (o->method == HS_METHOD_LEARNED) return fail(HS_EINVAL, "inplace is not offered with the learned method");
        if (o->driver == HS_DRIVER_PERSISTENT)
            return fail(HS_EINVAL, "inplace levels run with the host-driven loop, not the persistent driver");
        if (o->autotune) return fail(HS_EINVAL, "inplace is not offered with the autotuner");
    }
    return HS_OK;
}

// The sort operation of a key format (whole arrays).
template <int F> constexpr int op_of()
{
    return F == FMT_I32 ? HS_OP_SORT_I32 : F == FMT_F64 ? HS_OP_SORT_F64 : F == FMT_KV ? HS_OP_SORT_KV_I32
         : F == FMT_U32 ? HS_OP_SORT_U32 : F == FMT_I64 ? HS_OP_SORT_I64 : HS_OP_SORT_KV_F64;
}

// Batched (segmented) sorts: int32 and float64 keys.
constexpr bool is_seg(int op) { return op == HS_OP_SORT_SEGMENTED_I32 || op == HS_OP_SORT_SEGMENTED_F64; }
template <int F> constexpr int seg_op_of() { return F == FMT_F64 ? HS_OP_SORT_SEGMENTED_F64 : HS_OP_SORT_SEGMENTED_I32; }

int layout_for(int op, int64_t n, int64_t nseg, const hs_opts *o, Layout *L)
{
    int rc = check_learn(o);
    if (rc) return rc;
    const bool ip = o && o->inplace;
    switch (op) {
    case HS_OP_SORT_I32:
    case HS_OP_SORT_U32:
    case HS_OP_SORT_SEGMENTED_I32:
        *L = make_layout<uint32_t>(op, n, nseg, local_limit<uint32_t>(o), learn_params(o, n, op), ip);
        return HS_OK;
    case HS_OP_PARTITION_I32:
        *L = make_layout<uint32_t>(op, n, nseg, 0, LearnParams(), ip);
        return HS_OK;
    case HS_OP_SORT_F64:
    case HS_OP_SORT_I64:
    case HS_OP_SORT_KV_I32:
    case HS_OP_SORT_SEGMENTED_F64:
        *L = make_layout<uint64_t>(op, n, nseg, local_limit<uint64_t>(o), learn_params(o, n, op), ip);
        return HS_OK;
    case HS_OP_SORT_KV_F64:
        *L = make_layout<u128>(op, n, nseg, local_limit<u128>(o), learn_params(o, n, op), ip);
        return HS_OK;
    default:
        return fail(HS_EINVAL, "unknown op %d", op);
    }
}

// Bind the workspace: the caller's, or the cached one grown to fit.
int bind_workspace(DevState *d, const hs_opts *o, const Layout &L, char **base)
{
    if (o && o->workspace) {
        if (o->workspace_bytes < L.total)
            return fail(HS_EWORKSPACE, "workspace of %zu bytes, %zu needed", o->workspace_bytes, L.total);
        if ((uintptr_t)o->workspace % 256)
            return fail(HS_EINVAL, "workspace must be 256-byte aligned");
        *base = (char *)o->workspace;
        return HS_OK;
    }
    if (d->ws_bytes < L.total) {
        if (d->ws) {
            HS_HIP(hipDeviceSynchronize());
            HS_HIP(hipFree(d->ws));
            d->ws = nullptr;
            d->ws_bytes = 0;
        }
        size_t want = L.total + L.total / 8;
        if (hipMalloc(&d->ws, want) != hipSuccess) {
            (void)hipGetLastError();
            d->ws = nullptr;
            return fail(HS_ENOMEM, "hipMalloc of %zu workspace bytes failed", want);
        }
        d->ws_bytes = want;
    }
    *base = (char *)d->ws;
    return HS_OK;
}

uint32_t zero_grid(size_t bytes)
{
    const size_t blocks = (bytes / 4 + 255) / 256;
    return (uint32_t)(blocks < 1 ? 1 : blocks > 1024 ? 1024 : blocks);
}

// ---------------------------------------------------------------- driver

// Sort n keys whose workspace `ws` (laid out as L) is already bound.  Does
// not lock the device state: the learned front end calls it again for its
// training sample with a sub-workspace.
// Levels that a segment of `size` keys needs with balanced splits down to T,
// plus one.
int levels_for(uint64_t size, uint32_t T)
{
    int l = 1;
    while (size > T) {
        size = (size + 1) / 2;
        ++l;
    }
    return l;
}

// The learned front end up to the judge: the training and held-out samples,
// the nested plain sort of the training sample, features, training, the
// model's splitters and the judge, which leaves the chosen distinct
// splitters in the workspace and its decision in the LearnCtl.  counts_out
// (optional, 2 * NB_MAX words) receives the judge's held-out bucket counts,
// the model's splitters first.
template <int F>
int sort_body(DevState *d, char *ws, const Layout &L, Raw raw, int64_t n, const int64_t *d_off, int64_t nseg,
              const hs_opts *o, const LearnParams &P, hs_stats *st, hipStream_t stream, int graph_levels = 0);

template <int F>
int learn_front(DevState *d, char *ws, const Layout &L, Raw raw, int64_t n, uint32_t T, const hs_opts *o,
                const LearnParams &P, hipStream_t stream, uint32_t *counts_out)
{
    using K = typename KeyOf<F>::type;
    LearnCtl *lctl = (LearnCtl *)(ws + L.lctl);
    Raw smp{ws + L.smp_k, has_vals<F>() ? (int32_t *)(ws + L.smp_v) : nullptr};
    float *z = (float *)(ws + L.z), *y = (float *)(ws + L.y);
    float *par = (float *)(ws + L.par), *mom = (float *)(ws + L.mom), *vel = (float *)(ws + L.vel);
    float *part = (float *)(ws + L.part), *lossb = (float *)(ws + L.lossb);
    K *msplit = (K *)(ws + L.msplit), *ssplit = (K *)(ws + L.ssplit), *chosen = (K *)(ws + L.chosen);
    K *hold = (K *)(ws + L.hold);
    HS_LAUNCH(k_zero_words, 1, 256, stream, (uint32_t *)lctl, (uint32_t)(sizeof(LearnCtl) / 4));
    // sample draws: the training sample from splitmix64(seed), the
    // held-out sample from splitmix64(seed + 1), the weights from
    // splitmix64(seed + 2)
    HS_LAUNCH(k_ls_sample<F>, (P.m + 255) / 256, 256, stream, raw, (uint32_t)n, P.seed, P.m, smp);
    HS_LAUNCH(k_ls_holdout<F>, (P.h + 255) / 256, 256, stream, raw, (uint32_t)n, P.seed + 1, P.h, hold);
    const Layout S = make_layout<K>(op_of<F>(), P.m, 1, T);
    int rc = sort_body<F>(d, ws + L.sub, S, smp, P.m, nullptr, 0, o, LearnParams(), nullptr, stream);
    if (rc) return rc;
    HS_LAUNCH(k_ls_prep<F>, 1, 1024, stream, smp, P.m, z, y, ssplit, lctl, (double *)(ws + L.feat));
    const uint32_t nt = ntrain_of(P.m), gblk = (nt + 255) / 256;
    if (P.mode != JUDGE_SAMPLE) {
        // every step in one launch of gblk resident workgroups (see k_mlp_train)
        HS_LAUNCH(k_mlp_init, (MLP_NP + 255) / 256, 256, stream, par, mom, vel, P.seed + 2, (uint32_t *)nullptr);
        HS_LAUNCH(k_mlp_train, gblk, 256, stream, par, z, y, nt, P.steps, P.lr, part, lossb, &lctl->bar,
                  lossb + 2 * gblk);
        HS_LAUNCH(k_ls_invert<F>, (NSPLIT * WAVE + 255) / 256, 256, stream, par, lctl, smp, P.m, msplit);
    }
    HS_LAUNCH(k_ls_judge<F>, 1, 256, stream, msplit, ssplit, hold, P.h, chosen, lctl, P.mode, counts_out);
    return HS_OK;
}

// graph_levels > 0 (graph plans): record that many per-level launches (a
// level with an empty list costs three empty launches) before the
// persistent driver, which finishes whatever levels remain.
template <int F>
int sort_body(DevState *d, char *ws, const Layout &L, Raw raw, int64_t n, const int64_t *d_off, int64_t nseg,
              const hs_opts *o, const LearnParams &P, hs_stats *st, hipStream_t stream, int graph_levels)
{
    using K = typename KeyOf<F>::type;
    const uint32_t T = local_limit<K>(o);
    const uint32_t LEAF = leaf_limit<K>(o);
    const int rule = pivot_rule(o);
    // on chip, MEDIAN3 takes the 3-value median and every other rule the
    // median of 32 samples
    const int local_rule = (o && o->pivot_rule > 0) ? o->pivot_rule : PIVOT_NINTHER;
    const bool learned = P.on && (uint64_t)n > T;

    // in-place levels keep every key in the caller's arrays: no buffers
    const bool inplace = o && o->inplace;
    K *buf[2];
    buf[0] = inplace ? nullptr : has_vals<F>() ? (K *)(ws + L.buf0) : (K *)raw.keys;
    buf[1] = inplace ? nullptr : (K *)(ws + L.buf1);
    Seg<K> *segs[2] = {(Seg<K> *)(ws + L.segA), (Seg<K> *)(ws + L.segB)};
    unsigned long long *curs[2] = {(unsigned long long *)(ws + L.curA), (unsigned long long *)(ws + L.curB)};
    Task<K> *tasks = (Task<K> *)(ws + L.tasks);
    Ctl *ctl = (Ctl *)(ws + L.ctl);
    Ctl *h = d->h_ctl;
    hipEvent_t *lev = &d->ev[2 * LMAX];  // [0,1] on-chip sort, [2..4] learned front end, [5,6] level driver
    // the on-chip workgroup sort (single: one task, one workgroup); 8-byte
    // words take the half-size shape when the on-chip limit allows it (four
    // workgroups per CU instead of two)
    auto launch_local = [&](bool single) -> int {
        auto go = [&](auto CFG) -> int {
            using LC = decltype(CFG);
            HS_LAUNCH((k_local<F, LC::NT, LC::T, LC::LW, LC::WPC>), single ? 1 : d->ncu * LC::WPC, LC::NT, stream,
                      ctl, tasks, buf[0], buf[1], raw, local_rule, L.task_cap);
            return HS_OK;
        };
        if constexpr (LocalCfgHalf<K>::on) {
            if (T <= (uint32_t)LocalCfgHalf<K>::T) return go(LocalCfgHalf<K>{});
        }
        return go(LocalCfg<K>{});
    };
    hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
    HS_HIP(hipStreamIsCapturing(stream, &cap));
    const bool capturing = cap != hipStreamCaptureStatusNone;
    const int drv = o ? o->driver : HS_DRIVER_AUTO;
    if (capturing && (drv == HS_DRIVER_HOST || inplace))
        return fail(HS_EINVAL, "the host-driven level loop cannot be captured into a graph");
    const bool host_driver = drv == HS_DRIVER_HOST || inplace || (drv == HS_DRIVER_AUTO && !capturing);

    // a whole array that one wave's network holds (1024 keys, unless the
    // caller lowered the on-chip limit or the network bound to force the
    // other tiers): a single launch, no read-back
    constexpr uint32_t NET = (uint32_t)wave_net<K>();
    const uint64_t wave_max = (o && o->leaf > 0) ? LEAF : (uint64_t)(T < NET ? T : NET);
    if (!learned && !d_off && (uint64_t)n <= wave_max) {
        if (st) HS_HIP(hipEventRecord(lev[0], stream));
        HS_LAUNCH((k_sort_wave<F, NET>), 1, WAVE, stream, ctl, raw, (uint32_t)n);
        if (st && !capturing) {
            HS_HIP(hipEventRecord(lev[1], stream));
            HS_HIP(hipEventSynchronize(lev[1]));
            std::memset(st, 0, sizeof *st);
            st->tasks = 1;
            st->bytes_alg = (int64_t)(2 * sizeof(K)) * n;
            float ms = 0.f;
            HS_HIP(hipEventElapsedTime(&ms, lev[0], lev[1]));
            st->local_ms = ms;
        }
        return HS_OK;
    }
    // a whole array that is one on-chip task: set-up and one workgroup, no
    // read-back (neither kernel can report an error for a single task)
    if (!learned && !d_off && (uint64_t)n <= T && (uint64_t)n > LEAF) {
        HS_LAUNCH(k_init_one_task<F>, 1, 256, stream, ctl, tasks, (uint32_t)n);
        if (st) HS_HIP(hipEventRecord(lev[0], stream));
        const int rc = launch_local(true);
        if (rc) return rc;
        if (st && !capturing) {
            HS_HIP(hipEventRecord(lev[1], stream));
            HS_HIP(hipEventSynchronize(lev[1]));
            std::memset(st, 0, sizeof *st);
            st->tasks = 1;
            st->bytes_alg = (int64_t)(2 * sizeof(K)) * n;
            float ms = 0.f;
            HS_HIP(hipEventElapsedTime(&ms, lev[0], lev[1]));
            st->local_ms = ms;
        }
        return HS_OK;
    }

    HS_LAUNCH(k_zero_words, zero_grid(sizeof(Ctl)), 256, stream, (uint32_t *)ctl, (uint32_t)(sizeof(Ctl) / 4));
    int level0 = 0;
    LearnCtl *lctl = nullptr;
    if (learned) {
        // ---- learned splitters and the multiway pass
        lctl = (LearnCtl *)(ws + L.lctl);
        K *chosen = (K *)(ws + L.chosen);
        uint32_t *hist = (uint32_t *)(ws + L.hist), *btot = (uint32_t *)(ws + L.btot);
        uint32_t *bstart = (uint32_t *)(ws + L.bstart);
        if (st) HS_HIP(hipEventRecord(lev[2], stream));
        int rc = learn_front<F>(d, ws, L, raw, n, T, o, P, stream, nullptr);
        if (rc) return rc;
        if (st) HS_HIP(hipEventRecord(lev[3], stream));
        uint32_t chunk = (uint32_t)(((uint64_t)n + MW_GMAX - 1) / MW_GMAX);
        const uint32_t cmin = (uint32_t)(((uint64_t)n + (uint64_t)d->ncu * 8 - 1) / ((uint64_t)d->ncu * 8));
        if (chunk < cmin) chunk = cmin;
        chunk = (chunk + MW_TILE - 1) / MW_TILE * MW_TILE;
        const uint32_t G = (uint32_t)(((uint64_t)n + chunk - 1) / chunk);
        HS_LAUNCH((k_mw_hist<F, true>), G, MW_NT, stream, raw, (const K *)nullptr, (uint32_t)n, chunk, chosen, lctl,
                  hist);
        HS_LAUNCH(k_mw_scan_cols, NB_MAX, 1024, stream, hist, G, lctl, btot);
        HS_LAUNCH(k_mw_scan_starts, 1, 1024, stream, btot, lctl, bstart);
        HS_LAUNCH((k_mw_scatter<F, true, false>), G, MW_NT, stream, raw, (const K *)nullptr, (uint32_t)n, chunk,
                  chosen, lctl, hist, bstart, buf[1], Raw{});
        // the buckets are in buffer 1, where level 1 reads: they form level 1's list
        HS_LAUNCH(k_mw_route<F>, (NB_MAX + 255) / 256, 256, stream, ctl, lctl, bstart, chosen, buf[1], SRC_BUF1,
                  segs[1], curs[1], tasks, T, LEAF, rule, L.cand_cap, L.task_cap);
        if (st) HS_HIP(hipEventRecord(lev[4], stream));
        level0 = 1;
    } else if (d_off) {
        const uint32_t g = (uint32_t)((nseg + 255) / 256);  // one wave per 64 segments
        HS_LAUNCH(k_init_segmented<F>, g, 256, stream, ctl, segs[0], curs[0], tasks, raw, d_off, (uint32_t)nseg,
                  (uint32_t)n, T, LEAF, rule, L.cand_cap, L.task_cap);
    } else {
        HS_LAUNCH(k_init_single<F>, 1, 64, stream, ctl, segs[0], curs[0], tasks, raw, (uint32_t)n, T, LEAF,
                  L.task_cap, rule, 0, K(0));
    }

    int guard = 2;
    for (int64_t x = n; x > 1; x >>= 1) ++guard;  // 2 + log2(n): beyond it, sample-median pivots
    int launches = 0;
    // one level as three fixed-grid launches (every kernel reads the level's
    // size from the control block, so an empty level does nothing)
    int occ_p = 0;
    HS_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ_p, k_partition<F, false, false>, PartCfg<K>::NT, 0));
    if (occ_p < 1) occ_p = 1;
    // two rounds of workgroups: the tiles of a level differ in cost (partial
    // tiles at segment ends, segment changes), and workgroups of a second
    // round start where the first round's finish early (measured: int32 2^28
    // partition passes 6.28 ms, against 6.33 with one round and 6.31 with four)
    const int part_grid = d->ncu * occ_p * 2;
    const int fin_grid = d->ncu * FIN_BLOCKS_PER_CU;
    uint64_t *ipmask = (uint64_t *)(ws + L.ipmask);
    uint32_t *iprow = (uint32_t *)(ws + L.iprow), *iptot = (uint32_t *)(ws + L.iptot), *ipgp = (uint32_t *)(ws + L.ipgp);
    auto launch_level = [&](int level) -> int {
        const int p = level & 1;
        const int lrule = level > guard ? PIVOT_SAMPLE : rule;
        if (st) HS_HIP(hipEventRecord(d->ev[2 * level], stream));
        if (inplace) {
            // classify, rows, scan, swap: the level's keys stay where they are
            HS_LAUNCH((k_ip_classify<F>), part_grid, PartCfg<K>::NT, stream, ctl, p, 1, segs[p], curs[p], raw, ipmask,
                      L.cand_cap);
            HS_LAUNCH((k_ip_rows<F>), d->ncu * 8, IP_NT, stream, ctl, p, segs[p], curs[p], ipmask, iprow, iptot,
                      L.cand_cap);
            HS_LAUNCH((k_ip_scan<F>), 1, 1024, stream, ctl, p, segs[p], iptot, ipgp, L.cand_cap);
            HS_LAUNCH((k_ip_swap<F>), d->ncu * 8, IP_NT, stream, ctl, p, segs[p], curs[p], ipmask, iprow, iptot, ipgp,
                      raw, L.cand_cap);
            if (st) HS_HIP(hipEventRecord(d->ev[2 * level + 1], stream));
            HS_LAUNCH(k_finalize<F>, fin_grid, FIN_NT, stream, ctl, p, segs[p], curs[p], segs[1 - p], curs[1 - p], tasks,
                      (const K *)nullptr, SRC_RAW, raw, T, LEAF, lrule, L.cand_cap, L.task_cap);
            ++launches;
            return HS_OK;
        }
        if (level == 0)
            HS_LAUNCH((k_partition<F, true, false>), part_grid, PartCfg<K>::NT, stream, ctl, p, 1, segs[p], curs[p],
                      (const K *)nullptr, raw, buf[1 - p], Raw{}, L.cand_cap);
        else
            HS_LAUNCH((k_partition<F, false, false>), part_grid, PartCfg<K>::NT, stream, ctl, p, 1, segs[p], curs[p],
                      (const K *)buf[p], raw, buf[1 - p], Raw{}, L.cand_cap);
        if (st) HS_HIP(hipEventRecord(d->ev[2 * level + 1], stream));
        HS_LAUNCH(k_finalize<F>, fin_grid, FIN_NT, stream, ctl, p, segs[p], curs[p], segs[1 - p], curs[1 - p], tasks,
                  buf[1 - p], (uint32_t)(1 - p), raw, T, LEAF, lrule, L.cand_cap, L.task_cap);
        ++launches;
        return HS_OK;
    };
    if (!host_driver) {
        int first = level0;
        if (graph_levels > 0 && !st) {
            for (int l = 0; l < graph_levels && first < LMAX; ++l, ++first) {
                const int rc = launch_level(first);
                if (rc) return rc;
            }
        }
        // one persistent launch runs every (remaining) level; its grid must be resident at once
        int occ = 0;
        HS_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, k_levels<F>, PartCfg<K>::NT, 0));
        if (occ < 1) return fail(HS_EINTERNAL, "the level driver does not fit on a compute unit");
        if (st) HS_HIP(hipEventRecord(lev[5], stream));
        HS_LAUNCH(k_levels<F>, d->ncu * occ, PartCfg<K>::NT, stream, ctl, segs[0], segs[1], curs[0], curs[1], buf[0],
                  buf[1], raw, tasks, T, LEAF, rule, guard, first, LMAX, L.cand_cap, L.task_cap,
                  (o && o->spin_limit > 0) ? (uint32_t)o->spin_limit : BARRIER_SPIN_LIMIT);
        if (st) HS_HIP(hipEventRecord(lev[6], stream));
    }
    // on-chip sorts: fixed grids, the task counts are read on the device
    // (small_first: small tasks already sorted by an earlier launch)
    auto run_onchip = [&](uint32_t small_first) -> int {
        using LC = LocalCfg<K>;
        if (st) HS_HIP(hipEventRecord(lev[0], stream));
        HS_LAUNCH((k_small<F, LC::LEAF>), d->ncu * 8, 256, stream, ctl, tasks, buf[0], buf[1], raw, L.task_cap,
                  small_first);
        const int rc = launch_local(false);
        if (rc) return rc;
        if (st) HS_HIP(hipEventRecord(lev[1], stream));
        return HS_OK;
    };
    // the control block as it is after the on-chip sorts is in h already
    bool have_final = false;
    float local_ms_before = 0.f;  // an earlier on-chip launch's time (stats)
    if (host_driver) {
        // host-driven levels: batches of fixed-grid launches.  For a single
        // array the first batch runs the levels balanced splits would need
        // (levels_for, which counts one more) plus a margin, because sampled
        // pivots spread the segment sizes: two levels up to levels_for = 8,
        // three beyond (measured over uniform, normal, sorted and reversed
        // int32 and float64 arrays of 2^14..2^28 keys: at most levels_for + 1
        // non-empty levels up to 2^20, + 2 at 2^22..2^26, + 3 at 2^28).  An
        // empty level costs its two launches (about 20 us); a missing one a
        // read-back and a second on-chip launch.  The on-chip sorts follow the
        // batch at once, before any read-back: one read-back then usually ends
        // the call.  Should levels remain, further batches run with a
        // read-back each, and the on-chip sorts run again over the tasks the
        // new levels added.
        int level = level0;
        int batch = 0;
        uint32_t ntask_done = 0, nsmall_done = 0;
        bool sorted_some = false;
        if (!learned && !d_off && (uint64_t)n > T) {
            const int lf = levels_for((uint64_t)n, T);
            for (int bi = 0, nb = lf + (lf <= 8 ? 2 : 3); bi < nb && level < LMAX; ++bi, ++level) {
                const int rc = launch_level(level);
                if (rc) return rc;
            }
            const int rc = run_onchip(0);
            if (rc) return rc;
            sorted_some = true;
            HS_HIP(hipMemcpyAsync(h, ctl, sizeof(Ctl), hipMemcpyDeviceToHost, stream));
            HS_HIP(hipStreamSynchronize(stream));
            if (h->err) return fail(HS_EINTERNAL, "partition levels reported error bits 0x%x", h->err);
            const LevelCounts &lc = h->lev[level & 1];
            if ((uint32_t)lc.segs_tiles == 0) {
                have_final = true;
            } else {
                if (level >= LMAX) return fail(HS_EINTERNAL, "more than %d partition levels", LMAX);
                batch = levels_for(lc.max_seg, T);
                ntask_done = h->ntask;
                nsmall_done = h->nsmall;
                if (st) HS_HIP(hipEventElapsedTime(&local_ms_before, lev[0], lev[1]));
            }
        }
        if (!have_final) {
            for (;;) {
                for (int bi = 0; bi < batch && level < LMAX; ++bi, ++level) {
                    const int rc = launch_level(level);
                    if (rc) return rc;
                }
                HS_HIP(hipMemcpyAsync(h, ctl, sizeof(Ctl), hipMemcpyDeviceToHost, stream));
                HS_HIP(hipStreamSynchronize(stream));
                if (h->err) return fail(HS_EINTERNAL, "partition levels reported error bits 0x%x", h->err);
                const LevelCounts &lc = h->lev[level & 1];
                if ((uint32_t)lc.segs_tiles == 0) break;
                if (level >= LMAX) return fail(HS_EINTERNAL, "more than %d partition levels", LMAX);
                batch = levels_for(lc.max_seg, T);
            }
            // the on-chip sort claims tasks from task_next: the earlier launch's
            // tasks end at ntask_done
            if (sorted_some)
                HS_LAUNCH(k_set_word, 1, 64, stream, &ctl->task_next, ntask_done);
            const int rc = run_onchip(nsmall_done);
            if (rc) return rc;
        }
    } else {
        const int rc = run_onchip(0);
        if (rc) return rc;
    }
    if (capturing) return HS_OK;  // the caller checks the error word (plan entry points)
    if (!have_final) HS_HIP(hipMemcpyAsync(h, ctl, sizeof(Ctl), hipMemcpyDeviceToHost, stream));
    float loss = 0.f;
    if (st) {
        if (learned) HS_HIP(hipMemcpyAsync(d->h_lctl, lctl, sizeof(LearnCtl), hipMemcpyDeviceToHost, stream));
        if (learned && P.mode != JUDGE_SAMPLE) {
            const uint32_t gblk = (ntrain_of(P.m) + 255) / 256;
            HS_HIP(hipMemcpyAsync(&loss, (float *)(ws + L.lossb) + 2 * gblk, sizeof(float), hipMemcpyDeviceToHost,
                                  stream));
        }
    }
    HS_HIP(hipStreamSynchronize(stream));
    if (h->err) return fail(HS_EINTERNAL, "the sort reported error bits 0x%x", h->err);
    const uint32_t ntask = h->ntask, nsmall = h->nsmall;
    if ((uint64_t)ntask + nsmall > L.task_cap) return fail(HS_EINTERNAL, "task list overflow");
    if (st) {
        std::memset(st, 0, sizeof *st);
        st->passes = h->levels;
        st->keys_partitioned = (int64_t)h->part_keys;
        st->tasks = ntask + nsmall;
        st->max_depth = h->levels;
        st->bytes_alg = (int64_t)(2 * sizeof(K)) * ((int64_t)h->part_keys + (int64_t)h->local_keys) +
                        (int64_t)sizeof(K) * (int64_t)h->fill_keys;
        if (!host_driver) {
            st->partition_launches = 1;
            float ms = 0.f;
            HS_HIP(hipEventElapsedTime(&ms, lev[5], lev[6]));
            st->partition_ms = ms;
        } else {
            st->partition_launches = launches;
            for (int64_t l = level0; l < level0 + launches; ++l) {
                float ms = 0.f;
                HS_HIP(hipEventElapsedTime(&ms, d->ev[2 * l], d->ev[2 * l + 1]));
                st->partition_ms += ms;
            }
        }
        float ms = 0.f;
        HS_HIP(hipEventElapsedTime(&ms, lev[0], lev[1]));
        st->local_ms = ms + local_ms_before;
        if (learned) {
            const LearnCtl &lc = *d->h_lctl;
            // the multiway pass reads the keys twice and writes them once
            st->bytes_alg += 3 * (int64_t)sizeof(K) * n;
            st->fallback_used = lc.use_model ? 0 : 1;
            st->splitters = (int32_t)lc.k;
            st->model_imbalance = lc.model_imb;
            st->sample_imbalance = lc.sample_imb;
            st->bucket_imbalance = lc.use_model ? lc.model_imb : lc.sample_imb;
            st->final_loss = loss;
            HS_HIP(hipEventElapsedTime(&ms, lev[2], lev[3]));
            st->learn_ms = ms;
            HS_HIP(hipEventElapsedTime(&ms, lev[3], lev[4]));
            st->multiway_ms = ms;
        }
    }
    return HS_OK;
}

template <int F>
int run_sort_tuned(DevState *d, Raw raw, int64_t n, const int64_t *d_off, int64_t nseg, const hs_opts *o,
                   hs_stats *st, hipStream_t stream, int graph_levels = 0)
{
    const int op = d_off ? seg_op_of<F>() : op_of<F>();
    Layout L;
    int rc = layout_for(op, n, nseg, o, &L);
    if (rc) return rc;
    const LearnParams P = learn_params(o, n, op);
    std::lock_guard<std::mutex> lk(d->mu);
    char *ws = nullptr;
    rc = bind_workspace(d, o, L, &ws);
    if (rc) return rc;
    const bool shared_ws = !(o && o->workspace);
    if (shared_ws) HS_HIP(hipStreamWaitEvent(stream, d->last, 0));
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    HS_HIP(hipStreamIsCapturing(stream, &cs));
    const bool guard = L.guards.n > 0 && cs == hipStreamCaptureStatusNone;
    if (guard) HS_LAUNCH(k_guard_fill, L.guards.n, 64, stream, ws, L.guards, GUARD_WORD);
    rc = sort_body<F>(d, ws, L, raw, n, d_off, nseg, o, P, st, stream, graph_levels);
    if (rc == HS_OK && guard) {
        unsigned long long *cnt = (unsigned long long *)(ws + L.guard_count);
        HS_LAUNCH(k_zero_words, 1, 64, stream, (uint32_t *)cnt, 2u);
        HS_LAUNCH(k_guard_check, L.guards.n, 64, stream, ws, L.guards, GUARD_WORD, cnt);
        unsigned long long bad = 0;
        HS_HIP(hipMemcpyAsync(&bad, cnt, 8, hipMemcpyDeviceToHost, stream));
        HS_HIP(hipStreamSynchronize(stream));
        if (bad) rc = fail(HS_EINTERNAL, "%llu workspace guard words were overwritten", bad);
    }
    if (shared_ws) HS_HIP(hipEventRecord(d->last, stream));
    return rc;
}

// ---------------------------------------------------------------- autotuner

int ceil_log2(int64_t x)
{
    int l = 0;
    while (((int64_t)1 << l) < x) ++l;
    return l;
}

using TuneKey = std::tuple<int, int, int, int, int, int>;  // device, op, method, driver, log2 n, log2 (nseg + 1)
std::map<TuneKey, std::tuple<int, int, int>> g_tuned;  // -> local_T, leaf, pivot_rule
std::mutex g_tune_mu;

int tuned_driver(const hs_opts *o) { return (!o || o->driver == HS_DRIVER_AUTO) ? HS_DRIVER_HOST : o->driver; }

TuneKey tune_key(int op, const hs_opts *o, int64_t n, int64_t nseg)
{
    int dev = 0;
    (void)hipGetDevice(&dev);
    return TuneKey{dev, op, o ? o->method : HS_METHOD_PLAIN, tuned_driver(o), ceil_log2(n), ceil_log2(nseg + 1)};
}

struct DevBuf {
    void *p = nullptr;
    ~DevBuf()
    {
        if (p) (void)hipFree(p);
    }
};

struct EventPair {
    hipEvent_t a = nullptr, b = nullptr;
    ~EventPair()
    {
        if (a) (void)hipEventDestroy(a);
        if (b) (void)hipEventDestroy(b);
    }
};

// Measure every candidate on a copy of the input (see hs_autotune).
template <int F>
int autotune_impl(DevState *d, int op, Raw raw, int64_t n, const int64_t *d_off, int64_t nseg, const hs_opts *base,
                  hs_opts *best, hs_tune_report *rep, hipStream_t s)
{
    using K = typename KeyOf<F>::type;
    hs_opts b{};
    if (base) b = *base;
    b.autotune = 0;
    b.driver = tuned_driver(base);
    b.workspace = nullptr;
    b.workspace_bytes = 0;
    hs_tune_report r{};
    const TuneKey key = tune_key(op, &b, n, nseg);
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        auto it = g_tuned.find(key);
        if (it != g_tuned.end()) {
            *best = b;
            std::tie(best->local_T, best->leaf, best->pivot_rule) = it->second;
            r.candidates = 0;
            r.outputs_equal = 1;
            r.local_T = best->local_T;
            r.leaf = best->leaf;
            r.pivot_rule = best->pivot_rule;
            if (rep) *rep = r;
            return HS_OK;
        }
    }
    const size_t kb = (size_t)n * raw_key_bytes<F>(), vb = has_vals<F>() ? (size_t)n * 4 : 0;
    DevBuf src, work, ref, cnt;
    auto alloc = [&](DevBuf &x, size_t bytes) -> int {
        if (hipMalloc(&x.p, bytes ? bytes : 8) != hipSuccess) {
            (void)hipGetLastError();
            x.p = nullptr;
            return fail(HS_ENOMEM, "autotune: hipMalloc of %zu bytes failed", bytes);
        }
        return HS_OK;
    };
    int rc;
    if ((rc = alloc(src, kb + vb)) || (rc = alloc(work, kb + vb)) || (rc = alloc(ref, kb + vb)) || (rc = alloc(cnt, 8)))
        return rc;
    HS_HIP(hipMemcpyAsync(src.p, raw.keys, kb, hipMemcpyDeviceToDevice, s));
    if (vb) HS_HIP(hipMemcpyAsync((char *)src.p + kb, raw.vals, vb, hipMemcpyDeviceToDevice, s));
    EventPair ev;
    HS_HIP(hipEventCreate(&ev.a));
    HS_HIP(hipEventCreate(&ev.b));
    const Raw wr{work.p, vb ? (int32_t *)((char *)work.p + kb) : nullptr};
    const uint32_t Tmax = (uint32_t)LocalCfg<K>::T;
    std::vector<std::tuple<int, int, int>> cands;
    const int Lmax = (int)LocalCfg<K>::LEAF;
    cands.emplace_back((int)Tmax, Lmax, PIVOT_SAMPLE);  // the defaults first: the reference output
    for (int T : {2048, 4096, 8192})
        for (int leaf : {Lmax / 4, Lmax / 2, Lmax})
            for (int piv : {PIVOT_NINTHER, PIVOT_SAMPLE}) {
                if ((uint32_t)T > Tmax) continue;
                auto c = std::make_tuple(T, leaf, piv);
                if (c != cands[0]) cands.push_back(c);
            }
    double best_ms = 1e30;
    std::tuple<int, int, int> best_c = cands[0];
    bool equal = true;
    for (size_t ci = 0; ci < cands.size(); ++ci) {
        hs_opts c = b;
        std::tie(c.local_T, c.leaf, c.pivot_rule) = cands[ci];
        double ms_min = 1e30;
        for (int k = 0; k < 3; ++k) {  // one warm-up, two timed
            HS_HIP(hipMemcpyAsync(work.p, src.p, kb + vb, hipMemcpyDeviceToDevice, s));
            HS_HIP(hipEventRecord(ev.a, s));
            if ((rc = run_sort_tuned<F>(d, wr, n, d_off, nseg, &c, nullptr, s))) return rc;
            HS_HIP(hipEventRecord(ev.b, s));
            HS_HIP(hipEventSynchronize(ev.b));
            float ms = 0.f;
            HS_HIP(hipEventElapsedTime(&ms, ev.a, ev.b));
            if (k > 0 && ms < ms_min) ms_min = ms;
        }
        if (ci == 0) {
            r.default_ms = ms_min;
            HS_HIP(hipMemcpyAsync(ref.p, work.p, kb + vb, hipMemcpyDeviceToDevice, s));
        } else {
            // compare the output with the reference on the device
            HS_LAUNCH(k_zero_words, 1, 64, s, (uint32_t *)cnt.p, 2u);
            const uint64_t words = (kb + vb) / 4;
            const uint64_t g64 = (words + 255) / 256;
            HS_LAUNCH(k_count_diff, (uint32_t)(g64 < 4096 ? (g64 ? g64 : 1) : 4096), 256, s, (const uint32_t *)work.p,
                      (const uint32_t *)ref.p, words, (unsigned long long *)cnt.p);
            unsigned long long diff = 0;
            HS_HIP(hipMemcpyAsync(&diff, cnt.p, 8, hipMemcpyDeviceToHost, s));
            HS_HIP(hipStreamSynchronize(s));
            if (diff) equal = false;
        }
        if (ms_min < best_ms) {
            best_ms = ms_min;
            best_c = cands[ci];
        }
    }
    r.candidates = (int32_t)cands.size();
    r.outputs_equal = equal ? 1 : 0;
    r.best_ms = best_ms;
    std::tie(r.local_T, r.leaf, r.pivot_rule) = best_c;
    *best = b;
    std::tie(best->local_T, best->leaf, best->pivot_rule) = best_c;
    if (rep) *rep = r;
    if (!equal) return fail(HS_EINTERNAL, "autotune: candidate configurations produced different outputs");
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tuned[key] = best_c;
    return HS_OK;
}

template <int F>
int run_sort_logged(DevState *d, Raw raw, int64_t n, const int64_t *d_off, int64_t nseg, const hs_opts *o,
                    hs_stats *st, hipStream_t stream);

// HSORT_LOG=1 in the environment: one line per sort call on stderr (the
// operation, size, method, level mode and result; with statistics asked for,
// the levels, keys partitioned and times).
int log_level()
{
    const char *e = std::getenv("HSORT_LOG");
    return e && e[0] ? std::atoi(e) : 0;
}

template <int F>
int run_sort(DevState *d, Raw raw, int64_t n, const int64_t *d_off, int64_t nseg, const hs_opts *o,
             hs_stats *st, hipStream_t stream)
{
    const int rc = run_sort_logged<F>(d, raw, n, d_off, nseg, o, st, stream);
    if (log_level() > 0) {
        const int op = d_off ? seg_op_of<F>() : op_of<F>();
        std::fprintf(stderr, "[hsort] op=%d n=%lld nseg=%lld method=%d inplace=%d autotune=%d rc=%d", op,
                     (long long)n, (long long)nseg, o ? o->method : 0, o ? o->inplace : 0, o ? o->autotune : 0, rc);
        if (rc) std::fprintf(stderr, " error=\"%s\"", g_err.c_str());
        if (st && rc == HS_OK)
            std::fprintf(stderr, " levels=%d keys_partitioned=%lld tasks=%lld partition_ms=%.3f local_ms=%.3f",
                         (int)st->passes, (long long)st->keys_partitioned, (long long)st->tasks,
                         (double)st->partition_ms, (double)st->local_ms);
        std::fprintf(stderr, "\n");
    }
    return rc;
}

template <int F>
int run_sort_logged(DevState *d, Raw raw, int64_t n, const int64_t *d_off, int64_t nseg, const hs_opts *o,
                    hs_stats *st, hipStream_t stream)
{
    if (o && o->autotune) {
        int rc = check_learn(o);
        if (rc) return rc;
        const int op = d_off ? seg_op_of<F>() : op_of<F>();
        hs_opts tuned;
        if ((rc = autotune_impl<F>(d, op, raw, n, d_off, nseg, o, &tuned, nullptr, stream))) return rc;
        tuned.workspace = o->workspace;
        tuned.workspace_bytes = o->workspace_bytes;
        tuned.driver = o->driver;
        return run_sort_tuned<F>(d, raw, n, d_off, nseg, &tuned, st, stream);
    }
    return run_sort_tuned<F>(d, raw, n, d_off, nseg, o, st, stream);
}

int check_n(int64_t n)
{
    if (n < 0) return fail(HS_EINVAL, "n = %lld is negative", (long long)n);
    if (n >= ((int64_t)1 << 31)) return fail(HS_EINVAL, "n = %lld exceeds 2^31 - 1", (long long)n);
    return HS_OK;
}

bool overlap(const void *a, size_t na, const void *b, size_t nb)
{
    const char *x = (const char *)a, *y = (const char *)b;
    return x < y + nb && y < x + na;
}

// Argument checks shared by the plan and autotune entry points: a sort
// operation over keys (and vals / offsets as the operation needs).
int check_sort_args(int op, const void *keys, const int32_t *vals, int64_t n, const int64_t *d_off, int64_t nseg)
{
    int rc = check_n(n);
    if (rc) return rc;
    switch (op) {
    case HS_OP_SORT_I32:
    case HS_OP_SORT_F64:
    case HS_OP_SORT_U32:
    case HS_OP_SORT_I64:
        break;
    case HS_OP_SORT_KV_I32:
    case HS_OP_SORT_KV_F64: {
        const size_t kb = op == HS_OP_SORT_KV_F64 ? 8 : 4;
        if (n > 0 && !vals) return fail(HS_EINVAL, "vals is NULL");
        if (n > 0 && overlap(keys, (size_t)n * kb, vals, (size_t)n * 4)) return fail(HS_EINVAL, "keys and vals overlap");
        break;
    }
    case HS_OP_SORT_SEGMENTED_I32:
    case HS_OP_SORT_SEGMENTED_F64:
        if (nseg < 0 || nseg >= ((int64_t)1 << 31)) return fail(HS_EINVAL, "nseg = %lld out of range", (long long)nseg);
        if (nseg > 0 && !d_off) return fail(HS_EINVAL, "d_offsets is NULL");
        break;
    default:
        return fail(HS_EINVAL, "op %d is not a sort", op);
    }
    if (n > 0 && !keys) return fail(HS_EINVAL, "keys is NULL");
    return HS_OK;
}

// Call fn with the key format of a sort operation as a template argument.
template <typename Fn> int with_format(int op, Fn &&fn)
{
    switch (op) {
    case HS_OP_SORT_I32:
    case HS_OP_SORT_SEGMENTED_I32:
        return fn(std::integral_constant<int, FMT_I32>());
    case HS_OP_SORT_F64:
    case HS_OP_SORT_SEGMENTED_F64:
        return fn(std::integral_constant<int, FMT_F64>());
    case HS_OP_SORT_KV_I32:
        return fn(std::integral_constant<int, FMT_KV>());
    case HS_OP_SORT_U32:
        return fn(std::integral_constant<int, FMT_U32>());
    case HS_OP_SORT_I64:
        return fn(std::integral_constant<int, FMT_I64>());
    case HS_OP_SORT_KV_F64:
        return fn(std::integral_constant<int, FMT_KV_F64>());
    default:
        return fail(HS_EINVAL, "op %d is not a sort", op);
    }
}

}  // namespace

// ---------------------------------------------------------------- allocation-free sort

// Scratch memory of hs_sort_i32_noalloc: a static device array, one copy per
// GPU, held until the process ends.  It holds the workspace of an int32 sort
// of up to NOALLOC_MAX_N keys (ping-pong buffer, level lists, tasks, control
// block: about 4.3 bytes per key).  Host code must never pass `scratch`
// itself to a kernel or a copy (in host code the name is a host-side
// stand-in, not a device address): it uses the device address that
// hipGetSymbolAddress returned on that device.
namespace {
constexpr int64_t NOALLOC_MAX_N = (int64_t)1 << 22;
constexpr size_t NOALLOC_SCRATCH_BYTES = (size_t)20 << 20;
}  // namespace
static __device__ __align__(256) char scratch[NOALLOC_SCRATCH_BYTES];

namespace {

struct NoAllocDev {
    bool ready = false;
    void *ptr = nullptr;  // device address of `scratch` on this device
    DevState st;          // device facts for the level driver (no pinned memory, no events)
    Ctl h_ctl;            // host copy of the control block (static storage: nothing is allocated)
    std::mutex mu;        // one call at a time per device (host side)
};
NoAllocDev g_noalloc[MAXDEV];
std::mutex g_noalloc_probe_mu;

// Per device, once, with that device current: check the architecture and
// look up the address of the device's copy of `scratch`.
int noalloc_device(NoAllocDev **out)
{
    int dev = 0;
    HS_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= MAXDEV) return fail(HS_EUNSUPPORTED, "device index %d out of range", dev);
    NoAllocDev &nd = g_noalloc[dev];
    std::lock_guard<std::mutex> lk(g_noalloc_probe_mu);
    if (!nd.ready) {
        hipDeviceProp_t prop;
        HS_HIP(hipGetDeviceProperties(&prop, dev));
        if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0)
            return fail(HS_EUNSUPPORTED, "device %d is %s, this library is built for gfx950", dev, prop.gcnArchName);
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return fail(HS_EHIP, "hipGetSymbolAddress(scratch) on device %d: %s", dev, hipGetErrorString(e));
        nd.ptr = p;
        nd.st.probed = true;
        nd.st.supported = true;
        nd.st.ncu = prop.multiProcessorCount;
        nd.st.h_ctl = &nd.h_ctl;
        nd.ready = true;
    }
    *out = &nd;
    return HS_OK;
}

}  // namespace

struct hs_plan {
    int device = 0;
    int op = 0;
    int64_t n = 0, nseg = 0;
    hs_opts opts{};             // the knobs (tuned at the first replay when opts.autotune is set)
    bool tuned = false;
    int graph_levels = -1;      // per-level launches recorded before the persistent driver (-1: not yet known)
    void *ws = nullptr;
    size_t ws_bytes = 0;
    size_t ctl_off = 0;
    const void *bound_keys = nullptr, *bound_vals = nullptr, *bound_off = nullptr;
    hipStream_t cap = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    Ctl *h_ctl = nullptr;
};

namespace {

void plan_release(hs_plan *p)
{
    if (!p) return;
    if (p->exec) (void)hipGraphExecDestroy(p->exec);
    if (p->graph) (void)hipGraphDestroy(p->graph);
    if (p->cap) (void)hipStreamDestroy(p->cap);
    if (p->ws) (void)hipFree(p->ws);
    if (p->h_ctl) (void)hipHostFree(p->h_ctl);
    delete p;
}

}  // namespace

// ---------------------------------------------------------------- C ABI

extern "C" {

int hs_version(void) { return 100; }

const char *hs_last_error(void) { return g_err.c_str(); }

int hs_workspace_size(int op, int64_t n, int64_t nseg, const hs_opts *opts, size_t *bytes)
{
    if (!bytes) return fail(HS_EINVAL, "bytes is NULL");
    int rc = check_n(n);
    if (rc) return rc;
    if (nseg < 0) return fail(HS_EINVAL, "nseg is negative");
    Layout L;
    rc = layout_for(op, n, nseg, opts, &L);
    if (rc) return rc;
    *bytes = L.total;
    return HS_OK;
}

int hs_sort_i32(int32_t *keys, int64_t n, const hs_opts *opts, hs_stats *stats, void *stream)
{
    int rc = check_n(n);
    if (rc) return rc;
    if (n > 0 && !keys) return fail(HS_EINVAL, "keys is NULL");
    if (stats) std::memset(stats, 0, sizeof *stats);
    if (n <= 1) return HS_OK;
    DevState *d;
    if ((rc = get_device(&d))) return rc;
    return run_sort<FMT_I32>(d, Raw{keys, nullptr}, n, nullptr, 0, opts, stats, (hipStream_t)stream);
}

int hs_sort_f64(double *keys, int64_t n, const hs_opts *opts, hs_stats *stats, void *stream)
{
    int rc = check_n(n);
    if (rc) return rc;
    if (n > 0 && !keys) return fail(HS_EINVAL, "keys is NULL");
    if (stats) std::memset(stats, 0, sizeof *stats);
    if (n <= 1) return HS_OK;
    DevState *d;
    if ((rc = get_device(&d))) return rc;
    return run_sort<FMT_F64>(d, Raw{keys, nullptr}, n, nullptr, 0, opts, stats, (hipStream_t)stream);
}

int hs_sort_u32(uint32_t *keys, int64_t n, const hs_opts *opts, hs_stats *stats, void *stream)
{
    int rc = check_n(n);
    if (rc) return rc;
    if (n > 0 && !keys) return fail(HS_EINVAL, "keys is NULL");
    if (stats) std::memset(stats, 0, sizeof *stats);
    if (n <= 1) return HS_OK;
    DevState *d;
    if ((rc = get_device(&d))) return rc;
    return run_sort<FMT_U32>(d, Raw{keys, nullptr}, n, nullptr, 0, opts, stats, (hipStream_t)stream);
}

int hs_sort_i64(int64_t *keys, int64_t n, const hs_opts *opts, hs_stats *stats, void *stream)
{
    int rc = check_n(n);
    if (rc) return rc;
    if (n > 0 && !keys) return fail(HS_EINVAL, "keys is NULL");
    if (stats) std::memset(stats, 0, sizeof *stats);
    if (n <= 1) return HS_OK;
    DevState *d;
    if ((rc = get_device(&d))) return rc;
    return run_sort<FMT_I64>(d, Raw{keys, nullptr}, n, nullptr, 0, opts, stats, (hipStream_t)stream);
}

int hs_argsort_i32(const int32_t *keys, int32_t *keys_out, int32_t *idx_out, int64_t n, const hs_opts *opts,
                   hs_stats *stats, void *stream)
{
    int rc = check_n(n);
    if (rc) return rc;
    if (n > 0 && (!keys || !keys_out || !idx_out)) return fail(HS_EINVAL, "keys, keys_out or idx_out is NULL");
    if (n > 0 && keys != keys_out && overlap(keys, (size_t)n * 4, keys_out, (size_t)n * 4))
        return fail(HS_EINVAL, "keys and keys_out overlap without being the same array");
    if (n > 0 && (overlap(idx_out, (size_t)n * 4, keys_out, (size_t)n * 4) ||
                  overlap(idx_out, (size_t)n * 4, keys, (size_t)n * 4)))
        return fail(HS_EINVAL, "idx_out overlaps the keys");
    if (stats) std::memset(stats, 0, sizeof *stats);
    if (n == 0) return HS_OK;
    DevState *d;
    if ((rc = get_device(&d))) return rc;
    hipStream_t s = (hipStream_t)stream;
    if (keys != keys_out) HS_HIP(hipMemcpyAsync(keys_out, keys, (size_t)n * 4, hipMemcpyDeviceToDevice, s));
    HS_LAUNCH(k_iota, (unsigned)((n + 255) / 256), 256, s, idx_out, (uint32_t)n);
    if (n == 1) return HS_OK;
    // the (key, index) word orders equal keys by index: the sort comes out stable
    return run_sort<FMT_KV>(d, Raw{keys_out, idx_out}, n, nullptr, 0, opts, stats, s);
}

int hs_argsort_f64(const double *keys, double *keys_out, int32_t *idx_out, int64_t n, const hs_opts *opts,
                   hs_stats *stats, void *stream)
{
    int rc = check_n(n);
    if (rc) return rc;
    if (n > 0 && (!keys || !keys_out || !idx_out)) return fail(HS_EINVAL, "keys, keys_out or idx_out is NULL");
    if (n > 0 && keys != keys_out && overlap(keys, (size_t)n * 8, keys_out, (size_t)n * 8))
        return fail(HS_EINVAL, "keys and keys_out overlap without being the same array");
    if (n > 0 && (overlap(idx_out, (size_t)n * 4, keys_out, (size_t)n * 8) ||
                  overlap(idx_out, (size_t)n * 4, keys, (size_t)n * 8)))
        return fail(HS_EINVAL, "idx_out overlaps the keys");
    if (stats) std::memset(stats, 0, sizeof *stats);
    if (n == 0) return HS_OK;
    DevState *d;
    if ((rc = get_device(&d))) return rc;
    hipStream_t s = (hipStream_t)stream;
    if (keys != keys_out) HS_HIP(hipMemcpyAsync(keys_out, keys, (size_t)n * 8, hipMemcpyDeviceToDevice, s));
    HS_LAUNCH(k_iota, (unsigned)((n + 255) / 256), 256, s, idx_out, (uint32_t)n);
    if (n == 1) return HS_OK;
    // the 128-bit (key, index) word orders equal keys by index: the sort comes out stable
    return run_sort<FMT_KV_F64>(d, Raw{keys_out, idx_out}, n, nullptr, 0, opts, stats, s);
}

int hs_sort_kv_i32(int32_t *keys, int32_t *vals, int64_t n, const hs_opts *opts, hs_stats *stats,
                   void *stream)
{
    int rc = check_n(n);
    if (rc) return rc;
    if (n > 0 && (!keys || !vals)) return fail(HS_EINVAL, "keys or vals is NULL");
    if (n > 0 && overlap(keys, (size_t)n * 4, vals, (size_t)n * 4))
        return fail(HS_EINVAL, "keys and vals overlap");
    if (stats) std::memset(stats, 0, sizeof *stats);
    if (n <= 1) return HS_OK;
    DevState *d;
    if ((rc = get_device(&d))) return rc;
    return run_sort<FMT_KV>(d, Raw{keys, vals}, n, nullptr, 0, opts, stats, (hipStream_t)stream);
}

int hs_sort_kv_f64(double *keys, int32_t *vals, int64_t n, const hs_opts *opts, hs_stats *stats, void *stream)
{
    int rc = check_n(n);
    if (rc) return rc;
    if (n > 0 && (!keys || !vals)) return fail(HS_EINVAL, "keys or vals is NULL");
    if (n > 0 && overlap(keys, (size_t)n * 8, vals, (size_t)n * 4))
        return fail(HS_EINVAL, "keys and vals overlap");
    if (stats) std::memset(stats, 0, sizeof *stats);
    if (n <= 1) return HS_OK;
    DevState *d;
    if ((rc = get_device(&d))) return rc;
    return run_sort<FMT_KV_F64>(d, Raw{keys, vals}, n, nullptr, 0, opts, stats, (hipStream_t)stream);
}

int hs_sort_segmented_f64(double *keys, int64_t n_total, const int64_t *d_offsets, int64_t nseg,
                          const hs_opts *opts, hs_stats *stats, void *stream)
{
    int rc = check_n(n_total);
    if (rc) return rc;
    if (nseg < 0 || nseg >= ((int64_t)1 << 31)) return fail(HS_EINVAL, "nseg = %lld out of range", (long long)nseg);
    if (nseg > 0 && !d_offsets) return fail(HS_EINVAL, "d_offsets is NULL");
    if (n_total > 0 && !keys) return fail(HS_EINVAL, "keys is NULL");
    if (stats) std::memset(stats, 0, sizeof *stats);
    if (n_total <= 1 || nseg == 0) return HS_OK;
    DevState *d;
    if ((rc = get_device(&d))) return rc;
    return run_sort<FMT_F64>(d, Raw{keys, nullptr}, n_total, d_offsets, nseg, opts, stats, (hipStream_t)stream);
}

int hs_sort_segmented_i32(int32_t *keys, int64_t n_total, const int64_t *d_offsets, int64_t nseg,
                          const hs_opts *opts, hs_stats *stats, void *stream)
{
    int rc = check_n(n_total);
    if (rc) return rc;
    if (nseg < 0 || nseg >= ((int64_t)1 << 31)) return fail(HS_EINVAL, "nseg = %lld out of range", (long long)nseg);
    if (nseg > 0 && !d_offsets) return fail(HS_EINVAL, "d_offsets is NULL");
    if (n_total > 0 && !keys) return fail(HS_EINVAL, "keys is NULL");
    if (stats) std::memset(stats, 0, sizeof *stats);
    if (n_total <= 1 || nseg == 0) return HS_OK;
    DevState *d;
    if ((rc = get_device(&d))) return rc;
    return run_sort<FMT_I32>(d, Raw{keys, nullptr}, n_total, d_offsets, nseg, opts, stats, (hipStream_t)stream);
}

int hs_partition_i32(int32_t *keys, int64_t n, int32_t pivot, int64_t *d_count_le, const hs_opts *opts,
                     void *stream)
{
    int rc = check_n(n);
    if (rc) return rc;
    if (!d_count_le) return fail(HS_EINVAL, "d_count_le is NULL");
    if (n > 0 && !keys) return fail(HS_EINVAL, "keys is NULL");
    DevState *d;
    if ((rc = get_device(&d))) return rc;
    hipStream_t s = (hipStream_t)stream;
    if (n == 0) {
        HS_LAUNCH(k_zero_words, 1, 64, s, (uint32_t *)d_count_le, 2u);  // a kernel, not a memset node
        return HS_OK;
    }
    Layout L;
    if ((rc = layout_for(HS_OP_PARTITION_I32, n, 1, opts, &L))) return rc;
    std::lock_guard<std::mutex> lk(d->mu);
    char *ws = nullptr;
    if ((rc = bind_workspace(d, opts, L, &ws))) return rc;
    const bool shared_ws = !(opts && opts->workspace);
    if (shared_ws) HS_HIP(hipStreamWaitEvent(s, d->last, 0));
    Seg<uint32_t> *segs = (Seg<uint32_t> *)(ws + L.segA);
    unsigned long long *cur = (unsigned long long *)(ws + L.curA);
    Task<uint32_t> *tasks = (Task<uint32_t> *)(ws + L.tasks);
    Ctl *ctl = (Ctl *)(ws + L.ctl);
    const uint32_t upiv = (uint32_t)pivot ^ 0x80000000u;
    const uint32_t ntiles = seg_tiles<uint32_t>(0, (uint32_t)n);
    const uint32_t maxg = (uint32_t)d->ncu * 8;
    const int g = (int)(ntiles < maxg ? ntiles : maxg);
    HS_LAUNCH(k_zero_words, zero_grid(sizeof(Ctl)), 256, s, (uint32_t *)ctl, (uint32_t)(sizeof(Ctl) / 4));
    if (opts && opts->inplace) {
        // in place: classify, count the misplaced keys, scan, swap
        const Raw raw{keys, nullptr};
        HS_LAUNCH(k_init_single<FMT_I32>, 1, 64, s, ctl, segs, cur, tasks, raw, (uint32_t)n, 0u, 0u, L.task_cap,
                  PIVOT_MEDIAN3, 1, upiv);
        uint64_t *ipmask = (uint64_t *)(ws + L.ipmask);
        uint32_t *iprow = (uint32_t *)(ws + L.iprow), *iptot = (uint32_t *)(ws + L.iptot);
        uint32_t *ipgp = (uint32_t *)(ws + L.ipgp);
        HS_LAUNCH((k_ip_classify<FMT_I32>), g, PartCfg<uint32_t>::NT, s, ctl, 0, 0, segs, cur, raw, ipmask, L.cand_cap);
        HS_LAUNCH((k_ip_rows<FMT_I32>), g, IP_NT, s, ctl, 0, segs, cur, ipmask, iprow, iptot, L.cand_cap);
        HS_LAUNCH((k_ip_scan<FMT_I32>), 1, 1024, s, ctl, 0, segs, iptot, ipgp, L.cand_cap);
        HS_LAUNCH((k_ip_swap<FMT_I32>), g, IP_NT, s, ctl, 0, segs, cur, ipmask, iprow, iptot, ipgp, raw, L.cand_cap);
    } else {
        // out of place: stage the input in the workspace, then partition it
        // back into the caller's array
        int32_t *copy = (int32_t *)(ws + L.buf1);
        HS_HIP(hipMemcpyAsync(copy, keys, (size_t)n * 4, hipMemcpyDeviceToDevice, s));
        HS_LAUNCH(k_init_single<FMT_I32>, 1, 64, s, ctl, segs, cur, tasks, Raw{copy, nullptr}, (uint32_t)n, 0u, 0u,
                  L.task_cap, PIVOT_MEDIAN3, 1, upiv);
        HS_LAUNCH((k_partition<FMT_I32, true, true>), g, PartCfg<uint32_t>::NT, s, ctl, 0, 0, segs, cur,
                  (const uint32_t *)nullptr, Raw{copy, nullptr}, (uint32_t *)nullptr, Raw{keys, nullptr}, L.cand_cap);
    }
    HS_LAUNCH(k_write_count, 1, 64, s, ctl, cur, d_count_le);
    if (shared_ws) HS_HIP(hipEventRecord(d->last, s));
    return HS_OK;
}

int hs_sort_i32_noalloc(int32_t *keys, int64_t n, void *stream)
{
    int rc = check_n(n);
    if (rc) return rc;
    if (n > NOALLOC_MAX_N)
        return fail(HS_EINVAL, "n = %lld exceeds the %lld keys the static scratch of hs_sort_i32_noalloc holds",
                    (long long)n, (long long)NOALLOC_MAX_N);
    if (n > 0 && !keys) return fail(HS_EINVAL, "keys is NULL");
    if (n < 2) return HS_OK;
    NoAllocDev *nd;
    if ((rc = noalloc_device(&nd))) return rc;
    const Layout L = make_layout<uint32_t>(HS_OP_SORT_I32, n, 1, (uint32_t)LocalCfg<uint32_t>::T);
    if (L.total > NOALLOC_SCRATCH_BYTES)
        return fail(HS_EINTERNAL, "a sort of %lld keys needs %zu scratch bytes, %zu are reserved", (long long)n,
                    L.total, NOALLOC_SCRATCH_BYTES);
    std::lock_guard<std::mutex> lk(nd->mu);
    return sort_body<FMT_I32>(&nd->st, (char *)nd->ptr, L, Raw{keys, nullptr}, n, nullptr, 0, nullptr,
                              LearnParams(), nullptr, (hipStream_t)stream);
}

// ---- the learned method's kernels on their own

int hs_mlp_forward_f32(const float *d_params, const float *d_z, int64_t m, float *d_out, void *stream)
{
    if (m < 0 || m > ((int64_t)1 << 30)) return fail(HS_EINVAL, "m = %lld outside 0..2^30", (long long)m);
    if (m > 0 && (!d_params || !d_z || !d_out)) return fail(HS_EINVAL, "NULL pointer");
    if (m == 0) return HS_OK;
    DevState *d;
    int rc;
    if ((rc = get_device(&d))) return rc;
    k_mlp_forward<<<(uint32_t)((m + 255) / 256), 256, 0, (hipStream_t)stream>>>(d_params, d_z, (uint32_t)m, d_out);
    HS_LAUNCHED();
    return HS_OK;
}

namespace {

// Scratch of the MLP entry points: partial gradients of every workgroup,
// per-workgroup losses and the Adam moments.
struct MlpScratch {
    size_t part, lossb, mom, vel, done, total;
};

MlpScratch mlp_scratch(uint32_t m)
{
    MlpScratch S;
    const size_t g = (m + 255) / 256;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        size_t at = off;
        off = align_up(off + bytes, 256);
        return at;
    };
    S.part = take(g * MLP_PS * 4);
    S.lossb = take(g * 4);
    S.mom = take(MLP_NP * 4);
    S.vel = take(MLP_NP * 4);
    S.done = take(4);
    S.total = off;
    return S;
}

int mlp_args(const float *a, const float *b, int64_t m)
{
    if (m < 1 || m > ((int64_t)1 << 20)) return fail(HS_EINVAL, "m = %lld outside 1..2^20", (long long)m);
    if (!a || !b) return fail(HS_EINVAL, "NULL pointer");
    return HS_OK;
}

}  // namespace

int hs_mlp_grad_f32(const float *d_params, const float *d_z, const float *d_y, int64_t m, float *d_grad,
                    void *stream)
{
    int rc = mlp_args(d_z, d_y, m);
    if (rc) return rc;
    if (!d_params || !d_grad) return fail(HS_EINVAL, "NULL pointer");
    DevState *d;
    if ((rc = get_device(&d))) return rc;
    hipStream_t s = (hipStream_t)stream;
    const MlpScratch S = mlp_scratch((uint32_t)m);
    Layout L;
    L.total = S.total;
    std::lock_guard<std::mutex> lk(d->mu);
    char *ws = nullptr;
    if ((rc = bind_workspace(d, nullptr, L, &ws))) return rc;
    HS_HIP(hipStreamWaitEvent(s, d->last, 0));
    const uint32_t G = (uint32_t)((m + 255) / 256);
    float *part = (float *)(ws + S.part);
    k_mlp_grad<<<G, 256, 0, s>>>(d_params, d_z, d_y, (uint32_t)m, part, nullptr);
    HS_LAUNCHED();
    k_mlp_update<<<MLP_UPDATE_GRID, 256, 0, s>>>(nullptr, nullptr, nullptr, part, G, 1, 0.f, d_grad, nullptr, nullptr,
                                                 (uint32_t)m);
    HS_LAUNCHED();
    HS_HIP(hipEventRecord(d->last, s));
    return HS_OK;
}

int hs_mlp_train_f32(const float *d_z, const float *d_y, int64_t m, int32_t steps, float lr, uint64_t seed,
                     float *d_params, float *d_loss, void *stream)
{
    int rc = mlp_args(d_z, d_y, m);
    if (rc) return rc;
    if (!d_params) return fail(HS_EINVAL, "d_params is NULL");
    if (steps < 0 || steps > 100000) return fail(HS_EINVAL, "steps = %d outside 0..100000", steps);
    if (!(lr > 0.f) || lr > 1.f) return fail(HS_EINVAL, "lr outside (0, 1]");
    DevState *d;
    if ((rc = get_device(&d))) return rc;
    hipStream_t s = (hipStream_t)stream;
    const MlpScratch S = mlp_scratch((uint32_t)m);
    Layout L;
    L.total = S.total;
    std::lock_guard<std::mutex> lk(d->mu);
    char *ws = nullptr;
    if ((rc = bind_workspace(d, nullptr, L, &ws))) return rc;
    HS_HIP(hipStreamWaitEvent(s, d->last, 0));
    float *mom = (float *)(ws + S.mom), *vel = (float *)(ws + S.vel);
    float *part = (float *)(ws + S.part), *lossb = (float *)(ws + S.lossb);
    uint32_t *done = (uint32_t *)(ws + S.done);
    const uint32_t G = (uint32_t)((m + 255) / 256);
    k_mlp_init<<<(MLP_NP + 255) / 256, 256, 0, s>>>(d_params, mom, vel, seed, done);
    HS_LAUNCHED();
    for (int t = 1; t <= steps; ++t) {
        float *lt = d_loss ? d_loss + (t - 1) : nullptr;
        if (G <= MLP_STEP_MAX_G) {  // one launch per step (as inside the sort)
            k_mlp_step<<<G, 256, 0, s>>>(d_params, mom, vel, d_z, d_y, (uint32_t)m, part, lossb, done, t, lr, lt);
            HS_LAUNCHED();
        } else {
            k_mlp_grad<<<G, 256, 0, s>>>(d_params, d_z, d_y, (uint32_t)m, part, lossb);
            HS_LAUNCHED();
            k_mlp_update<<<MLP_UPDATE_GRID, 256, 0, s>>>(d_params, mom, vel, part, G, t, lr, nullptr, lossb, lt,
                                                         (uint32_t)m);
            HS_LAUNCHED();
        }
    }
    HS_HIP(hipEventRecord(d->last, s));
    return HS_OK;
}

int hs_multiway_partition_f64(double *keys, int64_t n, const uint64_t *d_splitters, int32_t k, uint32_t *d_start,
                              void *stream)
{
    int rc = check_n(n);
    if (rc) return rc;
    if (k < 0 || k > NSPLIT) return fail(HS_EINVAL, "k = %d outside 0..%d", k, NSPLIT);
    if (!d_start || (n > 0 && !keys) || (k > 0 && !d_splitters)) return fail(HS_EINVAL, "NULL pointer");
    DevState *d;
    if ((rc = get_device(&d))) return rc;
    hipStream_t s = (hipStream_t)stream;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        size_t at = off;
        off = align_up(off + bytes, 256);
        return at;
    };
    const size_t o_copy = take((size_t)n * 8), o_hist = take((size_t)NB_MAX * MW_GMAX * 4),
                 o_tot = take(NB_MAX * 4), o_lctl = take(sizeof(LearnCtl));
    Layout L;
    L.total = off;
    std::lock_guard<std::mutex> lk(d->mu);
    char *ws = nullptr;
    if ((rc = bind_workspace(d, nullptr, L, &ws))) return rc;
    HS_HIP(hipStreamWaitEvent(s, d->last, 0));
    LearnCtl *lc = (LearnCtl *)(ws + o_lctl);
    uint32_t *hist = (uint32_t *)(ws + o_hist), *tot = (uint32_t *)(ws + o_tot);
    k_ls_set_k<<<1, 1, 0, s>>>(lc, (uint32_t)k);
    HS_LAUNCHED();
    if (n > 0) {
        // out of place: stage the input in the workspace, scatter back
        HS_HIP(hipMemcpyAsync(ws + o_copy, keys, (size_t)n * 8, hipMemcpyDeviceToDevice, s));
        uint32_t chunk = (uint32_t)(((uint64_t)n + MW_GMAX - 1) / MW_GMAX);
        const uint32_t cmin = (uint32_t)(((uint64_t)n + (uint64_t)d->ncu * 8 - 1) / ((uint64_t)d->ncu * 8));
        if (chunk < cmin) chunk = cmin;
        chunk = (chunk + MW_TILE - 1) / MW_TILE * MW_TILE;
        const uint32_t G = (uint32_t)(((uint64_t)n + chunk - 1) / chunk);
        const Raw src{ws + o_copy, nullptr};
        const uint64_t *sp = d_splitters;
        k_mw_hist<FMT_F64, true><<<G, MW_NT, 0, s>>>(src, nullptr, (uint32_t)n, chunk, sp, lc, hist);
        HS_LAUNCHED();
        k_mw_scan_cols<<<NB_MAX, 1024, 0, s>>>(hist, G, lc, tot);
        HS_LAUNCHED();
        k_mw_scan_starts<<<1, 1024, 0, s>>>(tot, lc, d_start);
        HS_LAUNCHED();
        k_mw_scatter<FMT_F64, true, true><<<G, MW_NT, 0, s>>>(src, nullptr, (uint32_t)n, chunk, sp, lc, hist,
                                                               d_start, nullptr, Raw{keys, nullptr});
        HS_LAUNCHED();
    } else {
        HS_LAUNCH(k_zero_words, 1, 256, s, d_start, (uint32_t)(2 * k + 2));  // no bucket has keys
    }
    HS_HIP(hipEventRecord(d->last, s));
    return HS_OK;
}

int hs_learn_debug_f64(const double *keys, int64_t n, const hs_opts *opts, float *d_params, uint64_t *d_model_split,
                       uint64_t *d_sample_split, uint64_t *d_chosen, uint64_t *d_holdout, double *d_train_sorted,
                       uint32_t *d_counts, hs_learn_report *report, void *stream)
{
    int rc = check_n(n);
    if (rc) return rc;
    if (n < 1 || !keys) return fail(HS_EINVAL, "the learned front end needs n >= 1 keys");
    if (!d_params || !d_model_split || !d_sample_split || !d_chosen || !d_holdout || !d_train_sorted || !d_counts ||
        !report)
        return fail(HS_EINVAL, "NULL output pointer");
    hs_opts o = opts ? *opts : hs_opts{};
    o.method = HS_METHOD_LEARNED;
    if ((rc = check_learn(&o))) return rc;
    if (o.inplace) return fail(HS_EINVAL, "inplace is not offered with the learned method");
    DevState *d;
    if ((rc = get_device(&d))) return rc;
    const LearnParams P = learn_params(&o, n, HS_OP_SORT_F64);
    const uint32_t T = local_limit<uint64_t>(&o);
    const Layout L = make_layout<uint64_t>(HS_OP_SORT_F64, n, 1, T, P);
    std::lock_guard<std::mutex> lk(d->mu);
    char *ws = nullptr;
    if ((rc = bind_workspace(d, &o, L, &ws))) return rc;
    hipStream_t s = (hipStream_t)stream;
    const bool shared_ws = !o.workspace;
    if (shared_ws) HS_HIP(hipStreamWaitEvent(s, d->last, 0));
    rc = learn_front<FMT_F64>(d, ws, L, Raw{(void *)keys, nullptr}, n, T, &o, P, s, d_counts);
    if (rc) return rc;
    HS_HIP(hipMemcpyAsync(d_params, ws + L.par, MLP_NP * 4, hipMemcpyDeviceToDevice, s));
    HS_HIP(hipMemcpyAsync(d_model_split, ws + L.msplit, NSPLIT * 8, hipMemcpyDeviceToDevice, s));
    HS_HIP(hipMemcpyAsync(d_sample_split, ws + L.ssplit, NSPLIT * 8, hipMemcpyDeviceToDevice, s));
    HS_HIP(hipMemcpyAsync(d_chosen, ws + L.chosen, NSPLIT * 8, hipMemcpyDeviceToDevice, s));
    HS_HIP(hipMemcpyAsync(d_holdout, ws + L.hold, (size_t)P.h * 8, hipMemcpyDeviceToDevice, s));
    HS_HIP(hipMemcpyAsync(d_train_sorted, ws + L.smp_k, (size_t)P.m * 8, hipMemcpyDeviceToDevice, s));
    HS_HIP(hipMemcpyAsync(d->h_lctl, ws + L.lctl, sizeof(LearnCtl), hipMemcpyDeviceToHost, s));
    float loss = 0.f;
    if (P.mode != JUDGE_SAMPLE && P.steps > 0)
        HS_HIP(hipMemcpyAsync(&loss, (float *)(ws + L.lossb) + 2 * ((ntrain_of(P.m) + 255) / 256), 4,
                              hipMemcpyDeviceToHost, s));
    HS_HIP(hipStreamSynchronize(s));
    if (shared_ws) HS_HIP(hipEventRecord(d->last, s));
    const LearnCtl &lc = *d->h_lctl;
    *report = hs_learn_report{};
    report->scale = lc.scale;
    report->mu = lc.mu;
    report->sd = lc.sd;
    report->smin = lc.smin;
    report->smax = lc.smax;
    report->m = (int32_t)P.m;
    report->h = (int32_t)P.h;
    report->k = (int32_t)lc.k;
    report->use_model = (int32_t)lc.use_model;
    report->model_imbalance = lc.model_imb;
    report->sample_imbalance = lc.sample_imb;
    report->final_loss = loss;
    return HS_OK;
}

// ---- plans and the autotuner

int hs_autotune(int op, void *keys, int32_t *vals, int64_t n, const int64_t *d_offsets, int64_t nseg,
                const hs_opts *base, hs_opts *best, hs_tune_report *report, void *stream)
{
    if (!best) return fail(HS_EINVAL, "best is NULL");
    int rc = check_sort_args(op, keys, vals, n, d_offsets, nseg);
    if (rc) return rc;
    if ((rc = check_learn(base))) return rc;
    if (base && base->inplace) return fail(HS_EINVAL, "inplace is not offered with the autotuner");
    if (n < 2 || (is_seg(op) && nseg == 0)) {
        *best = base ? *base : hs_opts{};
        best->autotune = 0;
        if (report) *report = hs_tune_report{};
        return HS_OK;
    }
    DevState *d;
    if ((rc = get_device(&d))) return rc;
    const int64_t *off = is_seg(op) ? d_offsets : nullptr;
    return with_format(op, [&](auto fmt) {
        return autotune_impl<decltype(fmt)::value>(d, op, Raw{keys, vals}, n, off, nseg, base, best, report,
                                                   (hipStream_t)stream);
    });
}

int hs_plan_create(int op, int64_t n, int64_t nseg, const hs_opts *opts, hs_plan **plan)
{
    if (!plan) return fail(HS_EINVAL, "plan is NULL");
    *plan = nullptr;
    // the buffers are bound per replay; check the sizes with placeholders
    static const char probe[1] = {0};
    int rc = check_sort_args(op, probe, (const int32_t *)(probe + 0), 0, (const int64_t *)probe, nseg);
    if (rc) return rc;
    if ((rc = check_n(n))) return rc;
    if ((rc = check_learn(opts))) return rc;
    if (opts && opts->inplace) return fail(HS_EINVAL, "in-place levels cannot be captured into a graph");
    if (opts && opts->driver == HS_DRIVER_HOST)
        return fail(HS_EINVAL, "a plan runs the persistent level driver; HS_DRIVER_HOST cannot be captured");
    if (opts && opts->workspace) return fail(HS_EINVAL, "a plan owns its workspace; pass none");
    DevState *d;
    if ((rc = get_device(&d))) return rc;
    hs_plan *p = new hs_plan();
    HS_HIP(hipGetDevice(&p->device));
    p->op = op;
    p->n = n;
    p->nseg = is_seg(op) ? nseg : 0;
    p->opts = opts ? *opts : hs_opts{};
    p->opts.driver = HS_DRIVER_PERSISTENT;
    if (n < 2 || (is_seg(op) && nseg == 0)) {  // nothing to sort: an empty plan
        *plan = p;
        return HS_OK;
    }
    // The workspace is sized for every on-chip limit the tuner may pick
    // (a smaller limit means more segments per level).
    hs_opts lo = p->opts;
    if (lo.autotune) lo.local_T = 2048;
    Layout L;
    if ((rc = layout_for(op, n, p->nseg, &lo, &L))) {
        plan_release(p);
        return rc;
    }
    if (hipMalloc(&p->ws, L.total) != hipSuccess) {
        (void)hipGetLastError();
        p->ws = nullptr;
        plan_release(p);
        return fail(HS_ENOMEM, "hipMalloc of %zu plan workspace bytes failed", L.total);
    }
    p->ws_bytes = L.total;
    if (hipHostMalloc((void **)&p->h_ctl, sizeof(Ctl), hipHostMallocDefault) != hipSuccess ||
        hipStreamCreateWithFlags(&p->cap, hipStreamNonBlocking) != hipSuccess) {
        plan_release(p);
        return fail(HS_EHIP, "plan set-up failed");
    }
    *plan = p;
    return HS_OK;
}

namespace {

// Record the plan's sort of the given buffers into a graph and make it the
// plan's executable graph: the first time by instantiating it, later by
// updating the executable graph in place (same launches, new arguments).
// The first recording also tunes the knobs (opts.autotune) and counts the
// per-level launches to record from the largest segment; both read the
// buffers, so the caller's stream is synchronized first.
int plan_record(DevState *d, hs_plan *p, void *keys, int32_t *vals, const int64_t *d_off, hipStream_t stream)
{
    const int64_t *off = is_seg(p->op) ? d_off : nullptr;
    if (p->graph_levels < 0) {
        HS_HIP(hipStreamSynchronize(stream));
        if (p->opts.autotune && !p->tuned) {
            hs_opts tuned;
            int rc = with_format(p->op, [&](auto fmt) {
                return autotune_impl<decltype(fmt)::value>(d, p->op, Raw{keys, vals}, p->n, off, p->nseg, &p->opts,
                                                           &tuned, nullptr, nullptr);
            });
            if (rc) return rc;
            tuned.autotune = 0;
            tuned.driver = HS_DRIVER_PERSISTENT;
            tuned.workspace = nullptr;
            tuned.workspace_bytes = 0;
            p->opts = tuned;
            p->tuned = true;
        }
        // Per-level launches recorded before the persistent driver: the
        // levels the largest segment needs with balanced splits, plus two (a
        // level with an empty list costs three empty launches; the
        // persistent driver takes whatever remains).
        const int op = p->op;
        const bool w32 = op == HS_OP_SORT_I32 || op == HS_OP_SORT_U32 || op == HS_OP_SORT_SEGMENTED_I32;
        const uint32_t T = w32 ? local_limit<uint32_t>(&p->opts)
                         : op == HS_OP_SORT_KV_F64 ? local_limit<u128>(&p->opts) : local_limit<uint64_t>(&p->opts);
        uint64_t biggest = (uint64_t)p->n;
        if (is_seg(op)) {
            std::vector<int64_t> h_off((size_t)p->nseg + 1);
            HS_HIP(hipMemcpy(h_off.data(), d_off, h_off.size() * 8, hipMemcpyDeviceToHost));
            biggest = 0;
            for (int64_t i = 0; i < p->nseg; ++i)
                if (h_off[i + 1] - h_off[i] > (int64_t)biggest) biggest = (uint64_t)(h_off[i + 1] - h_off[i]);
        } else if (p->opts.method == HS_METHOD_LEARNED) {
            biggest = (uint64_t)p->n / 64;  // buckets of the multiway pass hold about n/256 keys
        }
        p->graph_levels = biggest > T ? levels_for(biggest, T) + 1 : 0;
    }
    hs_opts o = p->opts;
    o.workspace = p->ws;
    o.workspace_bytes = p->ws_bytes;
    Layout L;
    int rc = layout_for(p->op, p->n, p->nseg, &o, &L);
    if (rc) return rc;
    p->ctl_off = L.ctl;
    if (hipStreamBeginCapture(p->cap, hipStreamCaptureModeThreadLocal) != hipSuccess)
        return fail(HS_EHIP, "hipStreamBeginCapture failed");
    rc = with_format(p->op, [&](auto fmt) {
        return run_sort_tuned<decltype(fmt)::value>(d, Raw{keys, vals}, p->n, off, p->nseg, &o, nullptr, p->cap,
                                                    p->graph_levels);
    });
    hipGraph_t g = nullptr;
    const hipError_t ec = hipStreamEndCapture(p->cap, &g);
    if (rc == HS_OK && ec != hipSuccess) rc = fail(HS_EHIP, "hipStreamEndCapture: %s", hipGetErrorString(ec));
    if (rc) {
        (void)hipGetLastError();
        if (g) (void)hipGraphDestroy(g);
        return rc;
    }
    bool updated = false;
    if (p->exec) {
        hipGraphNode_t err_node = nullptr;
        hipGraphExecUpdateResult res = hipGraphExecUpdateError;
        updated = hipGraphExecUpdate(p->exec, g, &err_node, &res) == hipSuccess && res == hipGraphExecUpdateSuccess;
        if (!updated) {
            (void)hipGetLastError();
            (void)hipGraphExecDestroy(p->exec);
            p->exec = nullptr;
        }
    }
    if (!updated && hipGraphInstantiate(&p->exec, g, nullptr, nullptr, 0) != hipSuccess) {
        (void)hipGetLastError();
        p->exec = nullptr;
        (void)hipGraphDestroy(g);
        return fail(HS_EHIP, "hipGraphInstantiate failed");
    }
    if (p->graph) (void)hipGraphDestroy(p->graph);
    p->graph = g;
    p->bound_keys = keys;
    p->bound_vals = vals;
    p->bound_off = off;
    return HS_OK;
}

}  // namespace

int hs_plan_exec(hs_plan *plan, void *keys, int32_t *vals, const int64_t *d_offsets, void *stream)
{
    if (!plan) return fail(HS_EINVAL, "plan is NULL");
    int rc = check_sort_args(plan->op, keys, vals, plan->n, d_offsets, plan->nseg);
    if (rc) return rc;
    if (plan->n < 2 || (is_seg(plan->op) && plan->nseg == 0)) return HS_OK;
    int dev = 0;
    HS_HIP(hipGetDevice(&dev));
    if (dev != plan->device) return fail(HS_EINVAL, "the plan belongs to device %d, the current device is %d",
                                         plan->device, dev);
    hipStream_t s = (hipStream_t)stream;
    const int64_t *off = is_seg(plan->op) ? d_offsets : nullptr;
    const int32_t *v = (plan->op == HS_OP_SORT_KV_I32 || plan->op == HS_OP_SORT_KV_F64) ? vals : nullptr;
    if (!plan->exec || plan->bound_keys != keys || plan->bound_vals != v || plan->bound_off != off) {
        DevState *d;
        if ((rc = get_device(&d))) return rc;
        if ((rc = plan_record(d, plan, keys, (int32_t *)v, off, s))) return rc;
    }
    HS_HIP(hipGraphLaunch(plan->exec, s));
    return HS_OK;
}

int hs_plan_check(hs_plan *plan, void *stream)
{
    if (!plan) return fail(HS_EINVAL, "plan is NULL");
    if (!plan->exec) return HS_OK;
    hipStream_t s = (hipStream_t)stream;
    HS_HIP(hipMemcpyAsync(plan->h_ctl, (char *)plan->ws + plan->ctl_off, sizeof(Ctl), hipMemcpyDeviceToHost, s));
    HS_HIP(hipStreamSynchronize(s));
    if (plan->h_ctl->err) return fail(HS_EINTERNAL, "the plan's sort reported error bits 0x%x", plan->h_ctl->err);
    return HS_OK;
}

void hs_plan_destroy(hs_plan *plan)
{
    if (plan) (void)hipDeviceSynchronize();
    plan_release(plan);
}

}  // extern "C"
