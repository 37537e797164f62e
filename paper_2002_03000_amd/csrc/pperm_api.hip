// Host side of libpperm.so: the C ABI declared in include/pperm.h.
//
// The library owns no device memory: the caller hands in one workspace (a
// torch tensor in the Python binding) and the library lays its state out in
// it.  Every device operation is enqueued on the caller's stream.
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <mutex>
#include <new>
#include <vector>

#include "pperm.h"
#include "pperm_internal.h"

using namespace pperm;

struct pperm_ctx {
    pperm_config cfg;
    hipStream_t stream;
    unsigned char* ws;
    size_t ws_bytes;
    pperm_layout lay;
    int device;
    uint32_t team_lanes;      // TS: lanes per walk
    uint32_t slots_log2;      // (several walks per wave: slots are a power of two)
    uint32_t slots;
    uint32_t lds_team_bytes;
    uint32_t lds_wg_bytes;
    uint32_t workgroups;
    bool long_walk;           // per-length sums in global memory (see resolve_shape)
    uint64_t merged_tours;    // pooled tours merged so far (per sequence in independent mode)
    uint64_t open_tours;      // tours per sequence run since the last merge
    int sticky_error;
    ProblemDesc desc;         // host copy of the device-resident problem descriptor
    ProblemDesc* desc_dev;
};

namespace {

thread_local char g_last_error[256] = "";

int device_error(hipError_t e, const char* what) {
    snprintf(g_last_error, sizeof(g_last_error), "%s: %s", what, hipGetErrorString(e));
    return PPERM_EDEVICE;
}

#define HIP_TRY(expr)                                   \
    do {                                                \
        hipError_t e_ = (expr);                         \
        if (e_ != hipSuccess) return device_error(e_, #expr); \
    } while (0)

constexpr uint32_t kMaxNmax = 32766;
constexpr uint32_t kMaxSlots = 65536;
constexpr uint32_t kLdsLimit = 163840;   // bytes of LDS one gfx950 workgroup may take
constexpr uint32_t kTeamLdsLimit = 65536;
constexpr uint32_t kDefaultCap = 1u << 31;

uint64_t align_up(uint64_t x, uint64_t a) { return (x + a - 1) / a * a; }

bool is_pow2(uint32_t x) { return x && !(x & (x - 1)); }

uint32_t log2u(uint32_t x) {
    uint32_t r = 0;
    while ((1u << r) < x) ++r;
    return r;
}

// Cubic walks of at most COMPACT3_MAX_N steps run with 32-bit occupancy keys
// in the wave-per-walk kernels (not with observables, which read coordinates
// back from the keys); every other cubic walk with 64-bit keys.
bool compact_key(const pperm_config* c, uint32_t walks_per_wave) {
    return c->dim == 3 && c->n_max <= COMPACT3_MAX_N && walks_per_wave == 1 &&
           !(c->flags & PPERM_FLAG_OBSERVABLES);
}

uint32_t key_bytes(uint32_t dim, bool compact) { return (dim == 2 || compact) ? 4u : 8u; }

// Resolved tuning choices for a configuration (the "auto" values included).
struct Shape {
    uint32_t team_lanes;
    uint32_t slots;
    uint32_t lds_team_bytes;   // occupancy table + slot ids of one walk
    uint32_t lds_wg_bytes;     // LDS of one workgroup
    uint32_t walks_per_wave;
    bool long_walk;            // per-length sums outside LDS
    bool ckey;                 // cubic walks with 32-bit keys
};

// The occupancy table holds at most n_max + 1 sites; at least twice that many
// slots keeps linear-probing runs short.  One walk per wavefront keeps the
// sequence's per-length sums (and, with observables, its sums of W * R^2) in
// LDS beside the table.  Where that does not
// fit (walks of several thousand steps), or where PPERM_FLAG_SUMS_GLOBAL asks
// for more walks per compute unit, the sums stay in global memory and
// the table may fill up to 2/3 (at least 1.5 (n_max + 1) slots) so that table
// and slot ids of walks up to ~10^4 steps fit in LDS.  A walk that has a wave
// of its own may also use 1.5 times a power of two slots (hash_slots).
int resolve_shape(const pperm_config* c, Shape* sh) {
    const uint64_t n1 = c->n_max + 1u;
    const uint32_t row_bytes = (uint32_t)align_up(n1, 16) * 16u;
    const bool obs = (c->flags & PPERM_FLAG_OBSERVABLES) != 0;
    uint32_t wpw = c->walks_per_wave;
    if (wpw == 0) wpw = 1u;   // default shape: one walk per wavefront
    if (!is_pow2(wpw) || wpw > (c->dim == 2 ? 16u : 8u)) return PPERM_EINVAL;
    const bool ck = compact_key(c, wpw);
    auto team_bytes = [&](uint64_t slots) {
        return (uint32_t)align_up(slots * key_bytes(c->dim, ck) + 2ull * n1, 16);
    };
    const bool force_global = (c->flags & PPERM_FLAG_SUMS_GLOBAL) != 0;
    if ((obs || force_global) && wpw != 1) return PPERM_EINVAL;
    uint64_t slots = c->hash_slots;
    if (slots == 0) {
        slots = 64;
        while (slots < 2u * n1) slots <<= 1;
    }
    // a power of two, or (one walk per wave) 3 * 2^k
    const bool three = slots >= 96 && slots % 3u == 0 && is_pow2((uint32_t)(slots / 3u));
    if (!(is_pow2((uint32_t)slots) || (three && wpw == 1)) || slots < 64 || slots > kMaxSlots)
        return PPERM_EINVAL;
    bool lng = false;
    uint64_t bytes;
    if (wpw == 1) {
        bytes = (uint64_t)team_bytes(slots) + row_bytes * (obs ? 2u : 1u);
        if (bytes > kLdsLimit || force_global) {
            lng = true;
            if (c->hash_slots == 0)
                while (team_bytes(slots) > kLdsLimit &&
                       2u * (slots / 2u) >= 3u * n1)
                    slots >>= 1;
            bytes = (uint64_t)team_bytes(slots);
        }
    } else {
        bytes = (uint64_t)team_bytes(slots) * wpw;
    }
    if (lng ? 2u * slots < 3u * n1 : slots < 2u * n1) return PPERM_EINVAL;
    if (bytes > (wpw == 1 ? kLdsLimit : kTeamLdsLimit)) return PPERM_EINVAL;
    sh->slots = (uint32_t)slots;
    sh->lds_team_bytes = team_bytes(slots);
    sh->walks_per_wave = wpw;
    sh->team_lanes = 64u / wpw;
    sh->lds_wg_bytes = (uint32_t)bytes;
    sh->long_walk = lng;
    sh->ckey = ck;
    return PPERM_OK;
}

int validate(const pperm_config* c) {
    if (!c) return PPERM_EINVAL;
    if (c->struct_size != sizeof(pperm_config)) return PPERM_EINVAL;
    if (c->dim != 2 && c->dim != 3) return PPERM_EINVAL;
    if (c->n_max < 1 || c->n_max > kMaxNmax) return PPERM_EINVAL;
    if (c->n_sequences < 1) return PPERM_EINVAL;
    if (c->mode > PPERM_ROSENBLUTH) return PPERM_EINVAL;
    if ((c->flags & ~(PPERM_FLAG_GROUP_STATS | PPERM_FLAG_OBSERVABLES | PPERM_FLAG_SUMS_GLOBAL)) != 0)
        return PPERM_EINVAL;
    if ((c->flags & PPERM_FLAG_OBSERVABLES) && c->mode == PPERM_INDEPENDENT) return PPERM_EINVAL;
    Shape sh;
    return resolve_shape(c, &sh);
}

// Lay the state out in the workspace; every array 256-byte aligned.
void compute_layout(const pperm_config* c, pperm_layout* L) {
    const uint64_t N = c->n_sequences;
    const uint64_t row = align_up(c->n_max + 1u, 16);
    const bool indep = (c->mode == PPERM_INDEPENDENT);
    Shape sh;
    resolve_shape(c, &sh);
    // one copy stack per sequence (a sequence runs on one wavefront at a time)
    const uint64_t stack_slots = align_up(N, sh.walks_per_wave);
    const uint64_t chunks = (N + 63) / 64;
    uint64_t off = 0;
    auto take = [&](uint64_t bytes) {
        uint64_t o = off;
        off = align_up(off + bytes, 256);
        return o;
    };
    memset(L, 0, sizeof(*L));
    L->row = (uint32_t)row;
    L->stack_slots = (uint32_t)stack_slots;
    // state that create() zeroes comes first and is contiguous
    L->G = take((indep ? N : 1) * row * sizeof(SumRec));
    L->HG = take((indep ? N : 1) * row * 8);
    L->MG = take((indep ? N : 1) * 8);
    L->L = take(N * row * sizeof(SumRec));
    L->m = take(N * 4);
    L->t = take(N * 8);
    L->stats = take(N * STATS_WORDS * 8);
    L->groups = take(GROUPS * (sizeof(SumRec) + 8));
    if (c->flags & PPERM_FLAG_OBSERVABLES) {
        L->obs_L = take(N * row * sizeof(SumRec));
        L->obs_G = take(row * sizeof(SumRec));
    }
    L->ctrl = take(CTRL_WORDS * 4 + sizeof(ProblemDesc));
    // private scratch, not zeroed: copy stacks, merge partials (records + counts, x2)
    L->stack = take(stack_slots * c->n_max * sizeof(StackEntry));
    L->scratch = take(2 * chunks * row * (sizeof(SumRec) + 8));
    L->total = off;
}

template <typename T>
T* at(pperm_ctx* x, uint64_t off) {
    return reinterpret_cast<T*>(x->ws + off);
}

int check_device_errors(pperm_ctx* x) {
    uint32_t err = 0;
    HIP_TRY(hipMemcpyAsync(&err, at<uint32_t>(x, x->lay.ctrl) + CTRL_ERR, sizeof(err),
                           hipMemcpyDeviceToHost, x->stream));
    HIP_TRY(hipStreamSynchronize(x->stream));
    if (err & ERR_RANGE) x->sticky_error = PPERM_ERANGE;
    else if (err & ERR_CAP) x->sticky_error = PPERM_EOVERFLOW;
    else if (err & ERR_INCOMPLETE) x->sticky_error = PPERM_EINCOMPLETE;
    return x->sticky_error;
}

// The relative-error estimate of the group sums (all groups nonzero): group
// averages relative to the largest exponent, g_k = ldexp(m_k / C_k, e_k -
// e_max), their mean and sample variance summed in group order, and
// sqrt(var) / (4 mean).  Only correctly rounded operations, in a fixed order,
// so host, device and oracle take the same stop decisions.
double group_rel_err(const SumRec* sum, const uint64_t* tours, int e_top) {
    double g[GROUPS];
    double total = 0.0;
    for (uint32_t k = 0; k < GROUPS; ++k) {
        g[k] = ldexp(sum[k].m / (double)tours[k], sum[k].e - e_top);
        total += g[k];
    }
    const double mean = total / GROUPS;
    double ss = 0.0;
    for (uint32_t k = 0; k < GROUPS; ++k) ss += (g[k] - mean) * (g[k] - mean);
    return sqrt(ss / (GROUPS - 1)) / (4.0 * mean);
}

}  // namespace

bool pperm::config_long_walk(const pperm_config* c) {
    Shape sh;
    return validate(c) == PPERM_OK && resolve_shape(c, &sh) == PPERM_OK && sh.long_walk;
}

extern "C" {

const char* pperm_strerror(int code) {
    switch (code) {
        case PPERM_OK: return "success";
        case PPERM_EINVAL: return "invalid argument or configuration";
        case PPERM_ENOMEM: return "out of host memory";
        case PPERM_EDEVICE: return "HIP device error";
        case PPERM_ESTATE: return "call out of order";
        case PPERM_ERANGE: return "scaled weight out of range";
        case PPERM_EOVERFLOW: return "step cap or counter overflow";
        case PPERM_EINCOMPLETE: return "a chained launch ended before all of its epochs ran";
        default: return "unknown error";
    }
}

const char* pperm_last_device_error(void) { return g_last_error; }

int pperm_workspace_bytes(const pperm_config* cfg, size_t* bytes) {
    if (!bytes) return PPERM_EINVAL;
    int rc = validate(cfg);
    if (rc) return rc;
    pperm_layout L;
    compute_layout(cfg, &L);
    *bytes = (size_t)L.total;
    return PPERM_OK;
}

int pperm_create(const pperm_config* cfg, void* d_workspace, size_t bytes, void* hip_stream,
                 pperm_ctx** out) {
    if (!out || !d_workspace) return PPERM_EINVAL;
    *out = nullptr;
    int rc = validate(cfg);
    if (rc) return rc;
    if (((uintptr_t)d_workspace & 255u) != 0) return PPERM_EINVAL;
    pperm_layout L;
    compute_layout(cfg, &L);
    if (bytes < L.total) return PPERM_EINVAL;
    Shape sh;
    resolve_shape(cfg, &sh);

    pperm_ctx* x = new (std::nothrow) pperm_ctx();
    if (!x) return PPERM_ENOMEM;
    x->cfg = *cfg;
    x->stream = (hipStream_t)hip_stream;
    x->ws = (unsigned char*)d_workspace;
    x->ws_bytes = bytes;
    x->lay = L;
    x->team_lanes = sh.team_lanes;
    x->slots_log2 = log2u(sh.slots);
    x->slots = sh.slots;
    x->lds_team_bytes = sh.lds_team_bytes;
    x->lds_wg_bytes = sh.lds_wg_bytes;
    x->long_walk = sh.long_walk;

    hipError_t e = hipGetDevice(&x->device);
    if (e != hipSuccess) { delete x; return device_error(e, "hipGetDevice"); }
    int cus = 0;
    e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, x->device);
    if (e != hipSuccess) { delete x; return device_error(e, "hipDeviceGetAttribute"); }
    int per_cu = 0;
    e = run_kernel_lds_ok(cfg->dim, sh.team_lanes, sh.lds_wg_bytes, &per_cu);
    if (e != hipSuccess) { delete x; return device_error(e, "occupancy"); }
    if (per_cu < 1) { delete x; return PPERM_EINVAL; }
    uint64_t wgs = ((uint64_t)cfg->n_sequences + sh.walks_per_wave - 1) / sh.walks_per_wave;
    const uint64_t resident = (uint64_t)per_cu * (uint64_t)cus;
    if (wgs > resident) wgs = resident;
    const uint64_t by_stack = L.stack_slots / sh.walks_per_wave;
    if (wgs > by_stack) wgs = by_stack;
    x->workgroups = (uint32_t)wgs;

    int max_lds = 0;
    e = hipDeviceGetAttribute(&max_lds, hipDeviceAttributeMaxSharedMemoryPerBlock, x->device);
    if (e != hipSuccess) { delete x; return device_error(e, "hipDeviceGetAttribute"); }
    if (sh.lds_wg_bytes > (uint32_t)max_lds) { delete x; return PPERM_EINVAL; }

    // the device-resident description of this problem (read by the growth kernel)
    ProblemDesc& d = x->desc;
    memset(&d, 0, sizeof(d));
    d.L = at<SumRec>(x, L.L);
    d.G = at<SumRec>(x, L.G);
    d.MG = at<uint64_t>(x, L.MG);
    d.HG = at<uint64_t>(x, L.HG);
    d.m = at<uint32_t>(x, L.m);
    d.t = at<uint64_t>(x, L.t);
    d.stats = at<uint64_t>(x, L.stats);
    d.stack = at<StackEntry>(x, L.stack);
    d.ctrl = at<uint32_t>(x, L.ctrl);
    d.dim = cfg->dim;
    d.N = cfg->n_sequences;
    d.n_max = cfg->n_max;
    d.row = L.row;
    d.mode = cfg->mode;
    d.slots_log2 = x->slots_log2;
    d.slots = x->slots;
    d.lds_team_bytes = sh.lds_team_bytes;
    d.key0 = (uint32_t)cfg->seed;
    d.key1 = (uint32_t)(cfg->seed >> 32) ^ cfg->stream_id;
    d.step_cap = cfg->step_cap;
    d.ckey = sh.ckey ? 1u : 0u;
    d.LR = (cfg->flags & PPERM_FLAG_OBSERVABLES) ? at<SumRec>(x, L.obs_L) : nullptr;
    x->desc_dev = reinterpret_cast<ProblemDesc*>(at<uint32_t>(x, L.ctrl) + CTRL_WORDS);

    // zero the state (G .. ctrl are contiguous) and seed the digests
    const uint64_t zero_bytes = L.ctrl + CTRL_WORDS * 4 - L.G;
    e = launch_init_state(at<uint64_t>(x, L.stats), cfg->n_sequences, x->ws + L.G, zero_bytes,
                          x->stream);
    if (e != hipSuccess) { delete x; return device_error(e, "init_state"); }
    e = hipMemcpyAsync(x->desc_dev, &x->desc, sizeof(ProblemDesc), hipMemcpyHostToDevice, x->stream);
    if (e != hipSuccess) { delete x; return device_error(e, "descriptor copy"); }
    *out = x;
    return PPERM_OK;
}

int pperm_run_tours(pperm_ctx* x, uint32_t tours) {
    if (!x || tours == 0) return PPERM_EINVAL;
    const uint64_t N = x->cfg.n_sequences;
    const uint64_t per_seq_total = x->open_tours + tours;
    // r <= M + m bounds every copy count; keep M + m and every tour index in 32 bits
    const uint64_t pooled = (x->cfg.mode == PPERM_SHARED) ? x->merged_tours + N * per_seq_total
                                                          : x->merged_tours + per_seq_total;
    if (pooled > 0xFFFFFFFFull || per_seq_total > 0xFFFFFFFFull) return PPERM_EOVERFLOW;

    RunArgs a;
    a.G = at<SumRec>(x, x->lay.G);
    a.MG = at<uint64_t>(x, x->lay.MG);
    a.L = at<SumRec>(x, x->lay.L);
    a.m = at<uint32_t>(x, x->lay.m);
    a.t = at<uint64_t>(x, x->lay.t);
    a.stats = at<uint64_t>(x, x->lay.stats);
    a.stack = at<StackEntry>(x, x->lay.stack);
    a.ctrl = at<uint32_t>(x, x->lay.ctrl);
    a.N = x->cfg.n_sequences;
    a.n_max = x->cfg.n_max;
    a.row = x->lay.row;
    a.tours = tours;
    a.mode = x->cfg.mode;
    a.slots_log2 = x->slots_log2;
    a.lds_team_bytes = x->lds_team_bytes;
    a.key0 = (uint32_t)x->cfg.seed;
    a.key1 = (uint32_t)(x->cfg.seed >> 32) ^ x->cfg.stream_id;
    // watchdog: a sequence may take at most step_cap growth steps per call; by
    // default 4096 times the flat-histogram expectation of one sample per length
    // per tour, so that a runaway enrichment tree ends with PPERM_EOVERFLOW
    uint64_t cap = x->cfg.step_cap;
    if (cap == 0) {
        cap = 4096ull * tours * (x->cfg.n_max + 1ull);
        if (cap > kDefaultCap) cap = kDefaultCap;
    }
    a.step_cap = (uint32_t)cap;

    HIP_TRY(launch_reset_ctrl(a.ctrl, x->stream));
    if (x->team_lanes == 64) {
        // one walk per wavefront: the problem alone is a batch of one
        BatchArgs b;
        memset(&b, 0, sizeof(b));
        b.entries = nullptr;
        b.single.desc = x->desc_dev;
        b.single.tours = tours;
        b.single.step_cap = a.step_cap;
        b.single.first_item = 0;
        b.count = 1;
        b.total_items = N;
        b.queue = a.ctrl + CTRL_QUEUE;
        HIP_TRY(launch_batch(b, x->workgroups, x->lds_wg_bytes, x->stream,
                             (x->cfg.flags & PPERM_FLAG_OBSERVABLES) != 0, x->long_walk));
    } else {
        HIP_TRY(launch_run(a, x->cfg.dim, x->team_lanes, x->workgroups, x->lds_wg_bytes, x->stream));
    }
    x->open_tours = per_seq_total;
    return PPERM_OK;
}

int pperm_merge_epoch(pperm_ctx* x) {
    if (!x) return PPERM_EINVAL;
    const uint32_t N = x->cfg.n_sequences;
    const uint32_t row = x->lay.row;
    SumRec* L = at<SumRec>(x, x->lay.L);
    uint32_t* m = at<uint32_t>(x, x->lay.m);
    SumRec* G = at<SumRec>(x, x->lay.G);
    uint64_t* HG = at<uint64_t>(x, x->lay.HG);
    uint64_t* MG = at<uint64_t>(x, x->lay.MG);
    if (x->cfg.flags & PPERM_FLAG_GROUP_STATS) {
        SumRec* gsum = at<SumRec>(x, x->lay.groups);
        HIP_TRY(launch_group_sums(L, m, N, row, x->cfg.n_max, gsum,
                                  reinterpret_cast<uint64_t*>(gsum + GROUPS), x->stream));
    }
    if (x->cfg.mode == PPERM_INDEPENDENT) {
        HIP_TRY(launch_merge_independent(L, m, G, HG, MG, N, row, x->stream));
        x->merged_tours += x->open_tours;
        x->open_tours = 0;
        return PPERM_OK;
    }
    HIP_TRY(launch_merge_counts(m, N, MG, m, x->stream));
    // aligned pairwise tree over sequences, 64 rows per pass
    const uint64_t chunks = (N + 63) / 64;
    SumRec* bufd[2] = {at<SumRec>(x, x->lay.scratch), at<SumRec>(x, x->lay.scratch) + chunks * row};
    uint64_t* bufh[2] = {reinterpret_cast<uint64_t*>(bufd[1] + chunks * row),
                         reinterpret_cast<uint64_t*>(bufd[1] + chunks * row) + chunks * row};
    MergeArgs a;
    a.in = L;
    a.hin = nullptr;
    a.zero = L;
    a.rows = N;
    a.row = row;
    a.ncols = x->cfg.n_max + 1;
    int cur = 0;
    for (;;) {
        const bool final_pass = (a.rows <= 64);
        a.out = final_pass ? G : bufd[cur];
        a.hout = final_pass ? HG : bufh[cur];
        a.accumulate = final_pass ? 1u : 0u;
        HIP_TRY(launch_merge_pass(a, x->stream));
        if (final_pass) break;
        a.in = bufd[cur];
        a.hin = bufh[cur];
        a.zero = nullptr;
        a.rows = (uint32_t)((a.rows + 63) / 64);
        cur ^= 1;
    }
    if (x->cfg.flags & PPERM_FLAG_OBSERVABLES) {
        // the sums of W * R^2 through the same tree (no counts)
        SumRec* LR = at<SumRec>(x, x->lay.obs_L);
        a.in = LR;
        a.hin = nullptr;
        a.zero = LR;
        a.rows = N;
        for (;;) {
            const bool final_pass = (a.rows <= 64);
            a.out = final_pass ? at<SumRec>(x, x->lay.obs_G) : bufd[cur];
            a.hout = nullptr;
            a.accumulate = final_pass ? 1u : 0u;
            HIP_TRY(launch_merge_pass(a, x->stream));
            if (final_pass) break;
            a.in = bufd[cur];
            a.zero = nullptr;
            a.rows = (uint32_t)((a.rows + 63) / 64);
            cur ^= 1;
        }
    }
    x->merged_tours += (uint64_t)N * x->open_tours;
    x->open_tours = 0;
    return PPERM_OK;
}

// ---- batched launches --------------------------------------------------------
namespace {

constexpr int kBatchStreams = 4;

struct DeviceStreams {
    bool ready = false;
    hipStream_t s[kBatchStreams];
    hipEvent_t fork;
    hipEvent_t join[kBatchStreams];
};

std::mutex g_batch_mutex;
DeviceStreams g_streams[64];

int batch_streams(int device, DeviceStreams** out) {
    if (device < 0 || device >= 64) return PPERM_EINVAL;
    DeviceStreams& d = g_streams[device];
    if (!d.ready) {
        for (int i = 0; i < kBatchStreams; ++i) {
            HIP_TRY(hipStreamCreateWithFlags(&d.s[i], hipStreamNonBlocking));
            HIP_TRY(hipEventCreateWithFlags(&d.join[i], hipEventDisableTiming));
        }
        HIP_TRY(hipEventCreateWithFlags(&d.fork, hipEventDisableTiming));
        d.ready = true;
    }
    *out = &d;
    return PPERM_OK;
}

struct BatchItem {
    pperm_ctx* ctx;
    uint32_t tours;
    uint32_t lds;
    double work;
    bool lng;        // per-length sums in global memory (the long-walk kernel)
};

}  // namespace

int pperm_batch_workspace_bytes(size_t count, size_t* bytes) {
    if (!bytes || count == 0) return PPERM_EINVAL;
    *bytes = (size_t)align_up(count * sizeof(LaunchEntry), 256) + 256;
    return PPERM_OK;
}

namespace {

// A batched epoch step, planned on the host: the validated items, their LDS
// classes (one persistent launch each) and the launch entries in class order.
struct BatchClass { size_t begin, end; uint32_t lds; uint32_t total; bool lng; };
struct BatchPlan {
    std::vector<BatchItem> items;
    std::vector<BatchClass> classes;
    std::vector<LaunchEntry> entries;
};

int plan_batch(pperm_ctx* const* ctxs, size_t count, const uint32_t* tours_each, int device,
               BatchPlan* plan) {
    // validate and size every problem's share
    std::vector<BatchItem>& items = plan->items;
    items.clear();
    items.reserve(count);
    for (size_t i = 0; i < count; ++i) {
        pperm_ctx* x = ctxs[i];
        if (!x || x->device != device) return PPERM_EINVAL;
        if (x->cfg.flags & PPERM_FLAG_OBSERVABLES) return PPERM_EINVAL;
        for (size_t j = 0; j < i; ++j)
            if (ctxs[j] == x) return PPERM_EINVAL;          // a problem at most once per batch
        if (tours_each[i] == 0) continue;
        const uint64_t N = x->cfg.n_sequences;
        const uint64_t per_seq_total = x->open_tours + tours_each[i];
        const uint64_t pooled = (x->cfg.mode == PPERM_SHARED) ? x->merged_tours + N * per_seq_total
                                                              : x->merged_tours + per_seq_total;
        if (pooled > 0xFFFFFFFFull || per_seq_total > 0xFFFFFFFFull) return PPERM_EOVERFLOW;
        // LDS of one walk: occupancy table and slot ids, and the sequence's
        // sums unless they stay in global memory
        const uint32_t lds = x->desc.lds_team_bytes + (x->long_walk ? 0u : x->desc.row * (uint32_t)sizeof(SumRec));
        items.push_back({x, tours_each[i], lds,
                         (double)N * tours_each[i] * (double)(x->cfg.n_max + 1), x->long_walk});
    }
    plan->classes.clear();
    plan->entries.clear();
    if (items.empty()) return PPERM_OK;

    // classes by kernel (sums in LDS, or in global memory for long walks) and
    // LDS size (a launch gives every wave the largest share of its class);
    // inside a class the largest expected work goes first
    std::sort(items.begin(), items.end(), [](const BatchItem& a, const BatchItem& b) {
        if (a.lng != b.lng) return !a.lng;
        if (a.lds != b.lds) return a.lds < b.lds;
        return a.work > b.work;
    });
    std::vector<BatchClass>& classes = plan->classes;
    for (size_t i = 0; i < items.size();) {
        uint32_t cls = 8192;
        while (cls < items[i].lds) cls <<= 1;
        size_t j = i;
        while (j < items.size() && items[j].lng == items[i].lng && items[j].lds <= cls) ++j;
        classes.push_back({i, j, 0, 0, items[i].lng});
        i = j;
    }
    // fold the smallest classes of one kernel together (their waves then take
    // the larger share) until at most kBatchStreams remain
    while (classes.size() > (size_t)kBatchStreams) {
        size_t k = 0;
        while (k + 1 < classes.size() && classes[k].lng != classes[k + 1].lng) ++k;
        if (k + 1 == classes.size()) return PPERM_EINVAL;   // (two kernels leave at most two classes)
        classes[k + 1].begin = classes[k].begin;
        classes.erase(classes.begin() + (long)k);
    }
    std::vector<LaunchEntry>& host = plan->entries;
    host.resize(items.size());
    for (BatchClass& c : classes) {
        uint32_t first = 0, lds = 0;
        // the class's entries in LPT order (largest expected work first)
        std::sort(items.begin() + c.begin, items.begin() + c.end,
                  [](const BatchItem& a, const BatchItem& b) { return a.work > b.work; });
        for (size_t i = c.begin; i < c.end; ++i) {
            host[i].desc = items[i].ctx->desc_dev;
            host[i].tours = items[i].tours;
            uint64_t cap = items[i].ctx->cfg.step_cap;
            if (cap == 0) {
                cap = 4096ull * items[i].tours * (items[i].ctx->cfg.n_max + 1ull);
                if (cap > kDefaultCap) cap = kDefaultCap;
            }
            host[i].step_cap = (uint32_t)cap;
            host[i].first_item = first;
            host[i].pad = 0;
            first += items[i].ctx->cfg.n_sequences;
            lds = std::max(lds, items[i].lds);
        }
        c.lds = lds;
        c.total = first;
    }
    return PPERM_OK;
}

// Enqueue a planned batch: copy its entries to dev_entries, clear the queue
// words (four per class, by a kernel) and launch one persistent grid per class.
// With ds the classes run concurrently on the library's streams (forked from
// and joined into `stream`); without, one after another on `stream` itself.
int launch_plan(const BatchPlan& plan, int device, LaunchEntry* dev_entries, uint32_t* queues,
                hipStream_t stream, DeviceStreams* ds) {
    const std::vector<BatchClass>& classes = plan.classes;
    HIP_TRY(hipMemcpyAsync(dev_entries, plan.entries.data(), plan.entries.size() * sizeof(LaunchEntry),
                           hipMemcpyHostToDevice, stream));
    for (size_t c = 0; c < classes.size(); ++c) HIP_TRY(launch_reset_ctrl(queues + 4 * c, stream));
    if (ds) HIP_TRY(hipEventRecord(ds->fork, stream));
    int cus = 0;
    HIP_TRY(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device));
    for (size_t c = 0; c < classes.size(); ++c) {
        const BatchClass& C = classes[c];
        int per_cu = 0;
        HIP_TRY(batch_occupancy(C.lds, &per_cu, C.lng));
        if (per_cu < 1) return PPERM_EINVAL;
        uint64_t wgs = (uint64_t)per_cu * cus;
        if (wgs > C.total) wgs = C.total;
        BatchArgs b;
        memset(&b, 0, sizeof(b));
        b.entries = dev_entries + C.begin;
        b.single = plan.entries[C.begin];
        b.count = (uint32_t)(C.end - C.begin);
        b.total_items = C.total;
        b.queue = queues + 4 * c;
        hipStream_t s = stream;
        if (ds) {
            HIP_TRY(hipStreamWaitEvent(ds->s[c], ds->fork, 0));
            s = ds->s[c];
        }
        HIP_TRY(launch_batch(b, (uint32_t)wgs, C.lds, s, false, C.lng));
        if (ds) HIP_TRY(hipEventRecord(ds->join[c], ds->s[c]));
    }
    if (ds)
        for (size_t c = 0; c < classes.size(); ++c) HIP_TRY(hipStreamWaitEvent(stream, ds->join[c], 0));
    for (const BatchItem& it : plan.items) it.ctx->open_tours += it.tours;
    return PPERM_OK;
}

}  // namespace

int pperm_run_batch(pperm_ctx* const* ctxs, size_t count, const uint32_t* tours_each,
                    void* d_workspace, size_t bytes, void* hip_stream) {
    if (!ctxs || !tours_each || !d_workspace || count == 0) return PPERM_EINVAL;
    size_t need = 0;
    pperm_batch_workspace_bytes(count, &need);
    if (bytes < need || ((uintptr_t)d_workspace & 255u)) return PPERM_EINVAL;
    int device = -1;
    HIP_TRY(hipGetDevice(&device));
    BatchPlan plan;
    int rc = plan_batch(ctxs, count, tours_each, device, &plan);
    if (rc || plan.items.empty()) return rc;
    std::lock_guard<std::mutex> lock(g_batch_mutex);
    DeviceStreams* ds = nullptr;
    rc = batch_streams(device, &ds);
    if (rc) return rc;
    unsigned char* ws = (unsigned char*)d_workspace;
    return launch_plan(plan, device, reinterpret_cast<LaunchEntry*>(ws),
                       reinterpret_cast<uint32_t*>(ws + align_up(count * sizeof(LaunchEntry), 256)),
                       (hipStream_t)hip_stream, ds);
}

int pperm_run_batch_noalloc(pperm_ctx* const* ctxs, size_t count, const uint32_t* tours_each,
                            void* hip_stream) {
    if (!ctxs || !tours_each || count == 0) return PPERM_EINVAL;
    if (count > NOALLOC_MAX_PROBLEMS) return PPERM_EINVAL;
    int device = -1;
    HIP_TRY(hipGetDevice(&device));
    // the library's scratch on this device (its address, never its host name)
    void* base = nullptr;
    size_t cap = 0;
    HIP_TRY(noalloc_scratch(&base, &cap));
    if (NOALLOC_QUEUE_BYTES + count * sizeof(LaunchEntry) > cap) return PPERM_EINVAL;
    BatchPlan plan;
    int rc = plan_batch(ctxs, count, tours_each, device, &plan);
    if (rc || plan.items.empty()) return rc;
    unsigned char* ws = static_cast<unsigned char*>(base);
    return launch_plan(plan, device, reinterpret_cast<LaunchEntry*>(ws + NOALLOC_QUEUE_BYTES),
                       reinterpret_cast<uint32_t*>(ws), (hipStream_t)hip_stream, nullptr);
}

// ---- one epoch as a captured HIP graph -------------------------------------------
struct pperm_graph {
    pperm_ctx* ctx;
    uint32_t tours;
    hipGraph_t graph;
    hipGraphExec_t exec;
};

extern "C" int pperm_epoch_graph_create(pperm_ctx* x, uint32_t tours, pperm_graph** out) {
    if (!x || !out || tours == 0) return PPERM_EINVAL;
    *out = nullptr;
    if (x->open_tours != 0) return PPERM_ESTATE;
    hipStream_t cap = nullptr;
    HIP_TRY(hipStreamCreateWithFlags(&cap, hipStreamNonBlocking));
    // capture on a private stream (the legacy default stream cannot be
    // captured); the context's counters are restored afterwards
    const hipStream_t keep = x->stream;
    const uint64_t merged = x->merged_tours, open = x->open_tours;
    hipGraph_t g = nullptr;
    int rc = PPERM_OK;
    hipError_t e = hipStreamBeginCapture(cap, hipStreamCaptureModeRelaxed);
    if (e == hipSuccess) {
        x->stream = cap;
        rc = pperm_run_tours(x, tours);
        if (rc == PPERM_OK) rc = pperm_merge_epoch(x);
        x->stream = keep;
        e = hipStreamEndCapture(cap, &g);
    }
    x->merged_tours = merged;
    x->open_tours = open;
    (void)hipStreamDestroy(cap);
    if (e != hipSuccess) {
        if (g) (void)hipGraphDestroy(g);
        return device_error(e, "graph capture");
    }
    if (rc) {
        (void)hipGraphDestroy(g);
        return rc;
    }
    hipGraphExec_t exec = nullptr;
    e = hipGraphInstantiate(&exec, g, nullptr, nullptr, 0);
    if (e != hipSuccess) {
        (void)hipGraphDestroy(g);
        return device_error(e, "graph instantiate");
    }
    pperm_graph* G = new (std::nothrow) pperm_graph{x, tours, g, exec};
    if (!G) {
        (void)hipGraphExecDestroy(exec);
        (void)hipGraphDestroy(g);
        return PPERM_ENOMEM;
    }
    *out = G;
    return PPERM_OK;
}

extern "C" int pperm_epoch_graph_launch(pperm_graph* G) {
    if (!G) return PPERM_EINVAL;
    pperm_ctx* x = G->ctx;
    if (x->open_tours != 0) return PPERM_ESTATE;
    const uint64_t N = x->cfg.n_sequences;
    const uint64_t add = (x->cfg.mode == PPERM_SHARED) ? N * G->tours : G->tours;
    if (x->merged_tours + add > 0xFFFFFFFFull) return PPERM_EOVERFLOW;
    HIP_TRY(hipGraphLaunch(G->exec, x->stream));
    x->merged_tours += add;
    return PPERM_OK;
}

extern "C" int pperm_epoch_graph_destroy(pperm_graph* G) {
    if (!G) return PPERM_EINVAL;
    (void)hipGraphExecDestroy(G->exec);
    (void)hipGraphDestroy(G->graph);
    delete G;
    return PPERM_OK;
}

// ---- device-side epoch chaining ----------------------------------------------
namespace {

uint32_t lds_of(const pperm_ctx* x) {
    return x->desc.lds_team_bytes + (x->long_walk ? 0u : x->desc.row * (uint32_t)sizeof(SumRec));
}

uint32_t pow2_at_least(uint32_t n) {
    uint32_t p = 1;
    while (p < n) p <<= 1;
    return p;
}

// Workspace of a job: the common part, then per problem its schedule, the
// per-epoch copies of its pooled sums and its merge-tree flags.
struct JobLayout {
    uint64_t probs, state, order, counters, results, total;
    std::vector<uint64_t> sched, gver, flags, stage, stage_m;
};

void job_layout(pperm_ctx* const* ctxs, const uint32_t* epochs, size_t count, JobLayout* L) {
    uint64_t off = 0;
    auto take = [&](uint64_t bytes) {
        const uint64_t o = off;
        off = align_up(off + (bytes ? bytes : 1), 256);
        return o;
    };
    L->counters = take(JOB_COUNTER_WORDS * 4);        // first: pperm_job_report reads it
    L->probs = take(count * sizeof(JobProblem));
    L->state = take(count * sizeof(JobState));
    L->order = take(count * 4);
    L->results = take(count * 4 * 4);
    L->sched.assign(count, 0);
    L->gver.assign(count, 0);
    L->flags.assign(count, 0);
    L->stage.assign(count, 0);
    L->stage_m.assign(count, 0);
    for (size_t i = 0; i < count; ++i) {
        const pperm_ctx* x = ctxs[i];
        L->sched[i] = take((uint64_t)epochs[i] * 4);
        L->gver[i] = take((uint64_t)epochs[i] * (x->lay.row + JOB_GAP) * sizeof(SumRec));
        L->flags[i] = take((uint64_t)pow2_at_least(x->cfg.n_sequences) * 4);
        L->stage[i] = take((uint64_t)x->cfg.n_sequences * sizeof(SumRec));
        L->stage_m[i] = take((uint64_t)x->cfg.n_sequences * 4);
    }
    L->total = off;
}

int job_validate(pperm_ctx* const* ctxs, const uint32_t* const* schedules, const uint32_t* epochs,
                 size_t count, int* device_out) {
    if (!ctxs || !epochs || count == 0) return PPERM_EINVAL;
    int device = -1;
    HIP_TRY(hipGetDevice(&device));
    for (size_t i = 0; i < count; ++i) {
        pperm_ctx* x = ctxs[i];
        if (!x || x->device != device || x->team_lanes != 64) return PPERM_EINVAL;
        if (x->cfg.mode == PPERM_INDEPENDENT) return PPERM_EINVAL;
        if (x->cfg.flags & PPERM_FLAG_OBSERVABLES) return PPERM_EINVAL;
        for (size_t j = 0; j < i; ++j)
            if (ctxs[j] == x) return PPERM_EINVAL;
        if (x->open_tours != 0) return PPERM_ESTATE;
        if (schedules) {
            if (epochs[i] && !schedules[i]) return PPERM_EINVAL;
            uint64_t total = 0;
            for (uint32_t e = 0; e < epochs[i]; ++e) {
                if (schedules[i][e] == 0) return PPERM_EINVAL;
                total += schedules[i][e];
            }
            if (x->merged_tours + (uint64_t)x->cfg.n_sequences * total > 0xFFFFFFFFull) return PPERM_EOVERFLOW;
        }
    }
    if (device_out) *device_out = device;
    return PPERM_OK;
}

}  // namespace

int pperm_job_workspace_bytes(pperm_ctx* const* ctxs, const uint32_t* epochs, size_t count, size_t* bytes) {
    if (!bytes) return PPERM_EINVAL;
    int rc = job_validate(ctxs, nullptr, epochs, count, nullptr);
    if (rc) return rc;
    JobLayout L;
    job_layout(ctxs, epochs, count, &L);
    *bytes = (size_t)L.total;
    return PPERM_OK;
}

namespace {

// The chained launch; limits (per problem, may be NULL) switch the on-device
// stop rule on, slice_us (0: none) closes the starting of epochs after that
// long.  Host counters of the contexts are left to the callers.
int run_job_impl(pperm_ctx* const* ctxs, const uint32_t* const* schedules, const uint32_t* epochs,
                 size_t count, void* d_workspace, size_t bytes, void* hip_stream,
                 const pperm_job_limits* limits, uint32_t slice_us, JobLayout* Lout) {
    if (!schedules || !d_workspace) return PPERM_EINVAL;
    int device = -1;
    int rc = job_validate(ctxs, schedules, epochs, count, &device);
    if (rc) return rc;
    if (limits)
        for (size_t i = 0; i < count; ++i)
            if (limits[i].target_rel_err > 0.0 && !(ctxs[i]->cfg.flags & PPERM_FLAG_GROUP_STATS))
                return PPERM_EINVAL;
    JobLayout L;
    job_layout(ctxs, epochs, count, &L);
    if (bytes < L.total || ((uintptr_t)d_workspace & 255u)) return PPERM_EINVAL;
    hipStream_t stream = (hipStream_t)hip_stream;
    unsigned char* ws = (unsigned char*)d_workspace;

    // LDS classes (bounds at powers of two from 8 KB, at most four: the
    // smallest fold upwards; each class launched with the largest LDS one of
    // its problems needs), then the order in which waves look for work:
    // classes from the largest, inside a class the longest chain of steps first
    std::vector<uint32_t> cls_lds;
    std::vector<uint32_t> pcls(count, 0);
    {
        std::vector<uint32_t> sizes;
        for (size_t i = 0; i < count; ++i) {
            if (!epochs[i]) continue;
            uint32_t c = 8192;
            while (c < lds_of(ctxs[i])) c <<= 1;
            sizes.push_back(c);
        }
        std::sort(sizes.begin(), sizes.end());
        sizes.erase(std::unique(sizes.begin(), sizes.end()), sizes.end());
        while (sizes.size() > (size_t)kBatchStreams) sizes.erase(sizes.begin());
        cls_lds.assign(sizes.size(), 0u);
        for (size_t i = 0; i < count; ++i) {
            if (!epochs[i]) continue;
            const uint32_t need = lds_of(ctxs[i]);
            uint32_t c = 0;
            while (sizes[c] < need) ++c;
            pcls[i] = c;
            cls_lds[c] = std::max(cls_lds[c], need);
        }
    }
    if (cls_lds.empty()) return PPERM_OK;               // no epochs at all
    const uint32_t K = (uint32_t)cls_lds.size();
    std::vector<double> chain(count, 0.0), work(K, 0.0);
    std::vector<uint32_t> in_cls(K, 0), seqs_upto(K, 0);
    std::vector<uint32_t> order;
    for (size_t i = 0; i < count; ++i) {
        if (!epochs[i]) continue;
        double t = 0;
        for (uint32_t e = 0; e < epochs[i]; ++e) t += schedules[i][e];
        chain[i] = t * (ctxs[i]->cfg.n_max + 1.0);
        work[pcls[i]] += chain[i] * ctxs[i]->cfg.n_sequences;
        in_cls[pcls[i]] += 1;
        order.push_back((uint32_t)i);
    }
    std::sort(order.begin(), order.end(), [&](uint32_t a, uint32_t b) {
        if (pcls[a] != pcls[b]) return pcls[a] > pcls[b];
        if (chain[a] != chain[b]) return chain[a] > chain[b];
        return a < b;
    });
    std::vector<uint32_t> start(K, 0), need(K, 0);
    for (uint32_t c = 0; c < K; ++c) {
        uint32_t before = 0;
        for (uint32_t d = c + 1; d < K; ++d) before += in_cls[d];
        start[c] = before;
        for (uint32_t d = 0; d <= c; ++d) need[c] += in_cls[d];
    }
    for (size_t i = 0; i < count; ++i)
        if (epochs[i]) seqs_upto[pcls[i]] += ctxs[i]->cfg.n_sequences;
    for (uint32_t c = 1; c < K; ++c) seqs_upto[c] += seqs_upto[c - 1];

    // the problems' device records
    std::vector<JobProblem> host(count);
    for (size_t i = 0; i < count; ++i) {
        pperm_ctx* x = ctxs[i];
        JobProblem& J = host[i];
        memset(&J, 0, sizeof(J));
        J.desc = x->desc_dev;
        J.sched = reinterpret_cast<const uint32_t*>(ws + L.sched[i]);
        J.gver = reinterpret_cast<SumRec*>(ws + L.gver[i]);
        J.flags = reinterpret_cast<uint32_t*>(ws + L.flags[i]);
        J.epochs = epochs[i];
        J.N = x->cfg.n_sequences;
        J.p2 = pow2_at_least(J.N);
        J.levels = log2u(J.p2);
        J.cls = pcls[i];
        J.lds = lds_of(x);
        J.lng = x->long_walk ? 1u : 0u;
        J.result = reinterpret_cast<uint32_t*>(ws + L.results) + 4 * i;
        if (limits) {
            J.stage = reinterpret_cast<SumRec*>(ws + L.stage[i]);
            J.stage_m = reinterpret_cast<uint32_t*>(ws + L.stage_m[i]);
            J.gsum = at<SumRec>(x, x->lay.groups);
            J.target = limits[i].target_rel_err;
            J.cap = limits[i].tour_cap;
        }
        // chains within a factor 2, 4, 8 of the longest get priorities 3, 2, 1
        const double top = *std::max_element(chain.begin(), chain.end());
        J.prio = (top > 0 && chain[i] * 2 >= top) ? 3u : (chain[i] * 4 >= top) ? 2u : (chain[i] * 8 >= top) ? 1u : 0u;
    }
    HIP_TRY(launch_fill_zero(ws, L.total, stream));     // state, counters, flags
    HIP_TRY(hipMemcpyAsync(ws + L.probs, host.data(), count * sizeof(JobProblem), hipMemcpyHostToDevice,
                           stream));
    HIP_TRY(hipMemcpyAsync(ws + L.order, order.data(), order.size() * 4, hipMemcpyHostToDevice, stream));
    for (size_t i = 0; i < count; ++i)
        if (epochs[i])
            HIP_TRY(hipMemcpyAsync(ws + L.sched[i], schedules[i], (size_t)epochs[i] * 4,
                                   hipMemcpyHostToDevice, stream));

    // one persistent launch per class, each on its own library stream with a
    // share of the chip's LDS in proportion to its work times its LDS need
    std::lock_guard<std::mutex> lock(g_batch_mutex);
    DeviceStreams* ds = nullptr;
    rc = batch_streams(device, &ds);
    if (rc) return rc;
    int cus = 0;
    HIP_TRY(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device));
    double demand = 0;
    for (uint32_t c = 0; c < K; ++c) demand += work[c] * cls_lds[c];
    HIP_TRY(hipEventRecord(ds->fork, stream));
    for (uint32_t c = 0; c < K; ++c) {
        int per_cu = 0;
        HIP_TRY(job_occupancy(cls_lds[c], &per_cu));
        if (per_cu < 1) return PPERM_EINVAL;
        const uint64_t most = std::min<uint64_t>((uint64_t)per_cu * cus, seqs_upto[c]);
        const double share = demand > 0 ? work[c] * cls_lds[c] / demand : 1.0;
        uint64_t wgs = (uint64_t)(share * cus * (double)kLdsLimit / cls_lds[c]);
        wgs = std::max<uint64_t>(wgs, std::min<uint64_t>(most, (uint64_t)cus));
        wgs = std::min<uint64_t>(wgs, most);
        JobArgs a;
        memset(&a, 0, sizeof(a));
        a.probs = reinterpret_cast<const JobProblem*>(ws + L.probs);
        a.state = reinterpret_cast<JobState*>(ws + L.state);
        a.order = reinterpret_cast<const uint32_t*>(ws + L.order);
        a.counters = reinterpret_cast<uint32_t*>(ws + L.counters);
        a.count = (uint32_t)order.size();
        a.start = start[c];
        a.cls = c;
        a.need = need[c];
        a.slice_ticks = (uint64_t)slice_us * 100u;   // the 100 MHz real-time clock
        HIP_TRY(hipStreamWaitEvent(ds->s[c], ds->fork, 0));
        HIP_TRY(launch_job(a, (uint32_t)wgs, cls_lds[c], ds->s[c]));
        HIP_TRY(hipEventRecord(ds->join[c], ds->s[c]));
    }
    for (uint32_t c = 0; c < K; ++c) HIP_TRY(hipStreamWaitEvent(stream, ds->join[c], 0));
    if (slice_us == 0u && !limits) {
        // every epoch given must have run: flag any context whose did not
        JobArgs a;
        memset(&a, 0, sizeof(a));
        a.probs = reinterpret_cast<const JobProblem*>(ws + L.probs);
        a.order = reinterpret_cast<const uint32_t*>(ws + L.order);
        a.counters = reinterpret_cast<uint32_t*>(ws + L.counters);
        a.count = (uint32_t)order.size();
        HIP_TRY(launch_job_check(a, stream));
    }
    // the state a merge leaves: sums of the open epoch zero
    for (size_t i = 0; i < count; ++i) {
        pperm_ctx* x = ctxs[i];
        if (!epochs[i]) continue;
        HIP_TRY(launch_fill_zero(x->ws + x->lay.L, (size_t)x->cfg.n_sequences * x->lay.row * sizeof(SumRec),
                                 stream));
    }
    if (Lout) *Lout = L;
    return PPERM_OK;
}

}  // namespace

int pperm_run_job(pperm_ctx* const* ctxs, const uint32_t* const* schedules, const uint32_t* epochs,
                  size_t count, void* d_workspace, size_t bytes, void* hip_stream) {
    int rc = run_job_impl(ctxs, schedules, epochs, count, d_workspace, bytes, hip_stream, nullptr, 0, nullptr);
    if (rc) return rc;
    for (size_t i = 0; i < count; ++i) {
        uint64_t total = 0;
        for (uint32_t e = 0; e < epochs[i]; ++e) total += schedules[i][e];
        ctxs[i]->merged_tours += (uint64_t)ctxs[i]->cfg.n_sequences * total;
    }
    return PPERM_OK;
}

int pperm_run_job_sliced(pperm_ctx* const* ctxs, const uint32_t* const* schedules, const uint32_t* epochs,
                         size_t count, void* d_workspace, size_t bytes, void* hip_stream,
                         const pperm_job_limits* limits, uint32_t slice_us, uint32_t* epochs_done,
                         uint32_t* stop, double* rel_err) {
    if (!epochs_done) return PPERM_EINVAL;
    JobLayout L;
    int rc = run_job_impl(ctxs, schedules, epochs, count, d_workspace, bytes, hip_stream, limits, slice_us, &L);
    if (rc) return rc;
    std::vector<uint32_t> res(count * 4, 0);
    HIP_TRY(hipMemcpyAsync(res.data(), (unsigned char*)d_workspace + L.results, res.size() * 4,
                           hipMemcpyDeviceToHost, (hipStream_t)hip_stream));
    HIP_TRY(hipStreamSynchronize((hipStream_t)hip_stream));
    for (size_t i = 0; i < count; ++i) {
        const uint32_t done = res[4 * i];
        uint64_t total = 0;
        for (uint32_t e = 0; e < done && e < epochs[i]; ++e) total += schedules[i][e];
        ctxs[i]->merged_tours += (uint64_t)ctxs[i]->cfg.n_sequences * total;
        epochs_done[i] = done;
        if (stop) stop[i] = res[4 * i + 1];
        if (rel_err) {
            const uint64_t bits = (uint64_t)res[4 * i + 2] | ((uint64_t)res[4 * i + 3] << 32);
            double r;
            memcpy(&r, &bits, 8);
            rel_err[i] = done ? r : INFINITY;
        }
    }
    return PPERM_OK;
}

int pperm_job_report(const void* d_workspace, size_t bytes, void* hip_stream, pperm_job_report_t* out) {
    if (!d_workspace || !out || bytes < JOB_COUNTER_WORDS * 4) return PPERM_EINVAL;
    uint32_t c[JOB_COUNTER_WORDS];
    HIP_TRY(hipMemcpyAsync(c, d_workspace, sizeof(c), hipMemcpyDeviceToHost, (hipStream_t)hip_stream));
    HIP_TRY(hipStreamSynchronize((hipStream_t)hip_stream));
    out->problems_finished = c[JOB_FINISHED0] + c[JOB_FINISHED0 + 1] + c[JOB_FINISHED0 + 2] + c[JOB_FINISHED0 + 3];
    out->items_run = c[JOB_PROGRESS];
    out->problems_failed = c[JOB_FAILED];
    out->waves_left_idle = c[JOB_BACKSTOP];
    out->problems_incomplete = c[JOB_INCOMPLETE];
    return PPERM_OK;
}

int pperm_estimates(pperm_ctx* x, double* log_cn, uint64_t* hist, uint64_t* tours, size_t len) {
    if (!x || !log_cn) return PPERM_EINVAL;
    const uint32_t n1 = x->cfg.n_max + 1;
    if (len < n1) return PPERM_EINVAL;
    int rc = check_device_errors(x);
    if (rc) return rc;
    const uint32_t row = x->lay.row;
    const double ln2 = 0.69314718055994530942;
    if (x->cfg.mode == PPERM_INDEPENDENT) {
        const uint32_t N = x->cfg.n_sequences;
        std::vector<SumRec> G((size_t)N * row);
        std::vector<uint64_t> HG((size_t)N * row), MG(N);
        HIP_TRY(hipMemcpy(G.data(), at<SumRec>(x, x->lay.G), G.size() * sizeof(SumRec),
                          hipMemcpyDeviceToHost));
        HIP_TRY(hipMemcpy(HG.data(), at<uint64_t>(x, x->lay.HG), HG.size() * 8,
                          hipMemcpyDeviceToHost));
        HIP_TRY(hipMemcpy(MG.data(), at<uint64_t>(x, x->lay.MG), MG.size() * 8,
                          hipMemcpyDeviceToHost));
        uint64_t total = 0;
        for (uint32_t s = 0; s < N; ++s) {
            if (MG[s] == 0) return PPERM_ESTATE;
            total += MG[s];
        }
        std::vector<double> lg(N);
        for (uint32_t n = 0; n < n1; ++n) {
            // eqn (7): the mean over sequences of each sequence's own average,
            // summed in the log domain (the averages span any range)
            double top = -INFINITY;
            uint64_t h = 0;
            for (uint32_t s = 0; s < N; ++s) {
                const SumRec& g = G[(size_t)s * row + n];
                lg[s] = log(g.m) + g.e * ln2 - log((double)MG[s]);
                if (lg[s] > top) top = lg[s];
                h += HG[(size_t)s * row + n];
            }
            double acc = 0.0;
            if (top > -INFINITY)
                for (uint32_t s = 0; s < N; ++s) acc += exp(lg[s] - top);
            log_cn[n] = (top > -INFINITY) ? top + log(acc) - log((double)N) : -INFINITY;
            if (hist) hist[n] = h;
        }
        if (tours) *tours = total;
        return PPERM_OK;
    }
    std::vector<SumRec> G(n1);
    std::vector<uint64_t> HG(n1);
    uint64_t MG = 0;
    HIP_TRY(hipMemcpy(G.data(), at<SumRec>(x, x->lay.G), n1 * sizeof(SumRec), hipMemcpyDeviceToHost));
    HIP_TRY(hipMemcpy(HG.data(), at<uint64_t>(x, x->lay.HG), n1 * 8, hipMemcpyDeviceToHost));
    HIP_TRY(hipMemcpy(&MG, at<uint64_t>(x, x->lay.MG), 8, hipMemcpyDeviceToHost));
    if (MG == 0) return PPERM_ESTATE;
    for (uint32_t n = 0; n < n1; ++n) {
        log_cn[n] = log(G[n].m) + G[n].e * ln2 - log((double)MG);
        if (hist) hist[n] = HG[n];
    }
    if (tours) *tours = MG;
    return PPERM_OK;
}

int pperm_sequence_estimates(pperm_ctx* x, double* log_cn, size_t len) {
    if (!x || !log_cn) return PPERM_EINVAL;
    if (x->cfg.mode != PPERM_INDEPENDENT) return PPERM_EINVAL;
    const uint32_t N = x->cfg.n_sequences, n1 = x->cfg.n_max + 1, row = x->lay.row;
    if (len < (size_t)N * n1) return PPERM_EINVAL;
    int rc = check_device_errors(x);
    if (rc) return rc;
    std::vector<SumRec> G((size_t)N * row);
    std::vector<uint64_t> MG(N);
    HIP_TRY(hipMemcpy(G.data(), at<SumRec>(x, x->lay.G), G.size() * sizeof(SumRec), hipMemcpyDeviceToHost));
    HIP_TRY(hipMemcpy(MG.data(), at<uint64_t>(x, x->lay.MG), MG.size() * 8, hipMemcpyDeviceToHost));
    const double ln2 = 0.69314718055994530942;
    for (uint32_t s = 0; s < N; ++s) {
        if (MG[s] == 0) return PPERM_ESTATE;
        const double lm = log((double)MG[s]);
        // eqn (4) for sequence s alone: its weight sum over its own tours
        for (uint32_t n = 0; n < n1; ++n) {
            const SumRec& g = G[(size_t)s * row + n];
            log_cn[(size_t)s * n1 + n] = (g.m == 0.0) ? -INFINITY : log(g.m) + g.e * ln2 - lm;
        }
    }
    return PPERM_OK;
}

int pperm_error_estimate(pperm_ctx* x, double* rel_err, double* log_groups) {
    if (!x || !rel_err) return PPERM_EINVAL;
    if (!(x->cfg.flags & PPERM_FLAG_GROUP_STATS)) return PPERM_EINVAL;
    struct {
        SumRec sum[GROUPS];
        uint64_t tours[GROUPS];
    } g;
    static_assert(sizeof(g) == GROUPS * (sizeof(SumRec) + 8), "group record layout");
    HIP_TRY(hipMemcpyAsync(&g, at<unsigned char>(x, x->lay.groups), sizeof(g),
                           hipMemcpyDeviceToHost, x->stream));
    HIP_TRY(hipStreamSynchronize(x->stream));
    const double ln2 = 0.69314718055994530942;
    bool defined = true;
    int e_top = INT32_MIN;
    for (uint32_t k = 0; k < GROUPS; ++k) {
        if (g.tours[k] == 0 || g.sum[k].m == 0.0) defined = false;
        else if (g.sum[k].e > e_top) e_top = g.sum[k].e;
        if (log_groups)
            log_groups[k] = (g.tours[k] == 0 || g.sum[k].m == 0.0)
                                ? -INFINITY
                                : log(g.sum[k].m) + g.sum[k].e * ln2 - log((double)g.tours[k]);
    }
    *rel_err = defined ? group_rel_err(g.sum, g.tours, e_top) : INFINITY;
    return PPERM_OK;
}

int pperm_observable_r2(pperm_ctx* x, double* out, size_t len) {
    if (!x || !out) return PPERM_EINVAL;
    if (!(x->cfg.flags & PPERM_FLAG_OBSERVABLES)) return PPERM_EINVAL;
    const uint32_t n1 = x->cfg.n_max + 1;
    if (len < n1) return PPERM_EINVAL;
    int rc = check_device_errors(x);
    if (rc) return rc;
    if (x->merged_tours == 0) return PPERM_ESTATE;
    std::vector<SumRec> G(n1), GR(n1);
    HIP_TRY(hipMemcpy(G.data(), at<SumRec>(x, x->lay.G), n1 * sizeof(SumRec), hipMemcpyDeviceToHost));
    HIP_TRY(hipMemcpy(GR.data(), at<SumRec>(x, x->lay.obs_G), n1 * sizeof(SumRec),
                      hipMemcpyDeviceToHost));
    // eqn (5): the pooled sum of W * R^2 over the pooled sum of W (the
    // tour counts of numerator and denominator cancel)
    for (uint32_t n = 0; n < n1; ++n)
        out[n] = (G[n].m == 0.0) ? NAN : ldexp(GR[n].m / G[n].m, GR[n].e - G[n].e);
    return PPERM_OK;
}

int pperm_sequence_stats(pperm_ctx* x, pperm_seq_stats* out, size_t count) {
    if (!x || !out || count < x->cfg.n_sequences) return PPERM_EINVAL;
    HIP_TRY(hipStreamSynchronize(x->stream));
    HIP_TRY(hipMemcpy(out, at<uint64_t>(x, x->lay.stats),
                      (size_t)x->cfg.n_sequences * sizeof(pperm_seq_stats), hipMemcpyDeviceToHost));
    return PPERM_OK;
}

int pperm_stats(pperm_ctx* x, pperm_seq_stats* total) {
    if (!x || !total) return PPERM_EINVAL;
    std::vector<pperm_seq_stats> all(x->cfg.n_sequences);
    int rc = pperm_sequence_stats(x, all.data(), all.size());
    if (rc) return rc;
    memset(total, 0, sizeof(*total));
    for (const auto& s : all) {
        total->steps += s.steps;
        total->events += s.events;
        total->enrich += s.enrich;
        total->copies += s.copies;
        total->prunes += s.prunes;
        total->traps += s.traps;
        total->tours += s.tours;
        if (s.max_depth > total->max_depth) total->max_depth = s.max_depth;
        total->digest ^= s.digest;
        total->capped += s.capped;
    }
    return PPERM_OK;
}

int pperm_sync(pperm_ctx* x) {
    if (!x) return PPERM_EINVAL;
    return check_device_errors(x);
}

// ---- checkpoint / resume -----------------------------------------------------
namespace {

constexpr uint64_t kCkptMagic = 0x314B43504D524550ull;   // "PERMPCK1", little endian
constexpr uint32_t kCkptVersion = 1;

struct CkptHeader {
    uint64_t magic;
    uint32_t version;
    uint32_t sections;
    pperm_config cfg;
    uint64_t merged_tours;
    uint64_t payload_bytes;
};

// The merged state of a context as (workspace offset, bytes) sections, in
// checkpoint order.  Per-sequence epoch sums and tour counts are not part of
// it: they are zero between a merge and the next run.
int ckpt_sections(const pperm_ctx* x, uint64_t off[8], uint64_t len[8]) {
    const uint64_t N = x->cfg.n_sequences;
    const uint64_t row = x->lay.row;
    const uint64_t g = (x->cfg.mode == PPERM_INDEPENDENT) ? N : 1;
    int k = 0;
    off[k] = x->lay.G;      len[k++] = g * row * sizeof(SumRec);
    off[k] = x->lay.HG;     len[k++] = g * row * 8;
    off[k] = x->lay.MG;     len[k++] = g * 8;
    off[k] = x->lay.t;      len[k++] = N * 8;
    off[k] = x->lay.stats;  len[k++] = N * STATS_WORDS * 8;
    off[k] = x->lay.groups; len[k++] = GROUPS * (sizeof(SumRec) + 8);
    if (x->cfg.flags & PPERM_FLAG_OBSERVABLES) {
        off[k] = x->lay.obs_G;
        len[k++] = row * sizeof(SumRec);
    }
    return k;
}

bool same_problem(const pperm_config& a, const pperm_config& b) {
    const uint32_t result_flags = PPERM_FLAG_GROUP_STATS | PPERM_FLAG_OBSERVABLES;
    return a.dim == b.dim && a.n_max == b.n_max && a.n_sequences == b.n_sequences && a.seed == b.seed &&
           a.mode == b.mode && a.stream_id == b.stream_id &&
           (a.flags & result_flags) == (b.flags & result_flags);
}

}  // namespace

int pperm_checkpoint_bytes(const pperm_ctx* x, size_t* bytes) {
    if (!x || !bytes) return PPERM_EINVAL;
    uint64_t off[8], len[8];
    const int k = ckpt_sections(x, off, len);
    uint64_t total = sizeof(CkptHeader);
    for (int i = 0; i < k; ++i) total += len[i];
    *bytes = (size_t)total;
    return PPERM_OK;
}

int pperm_checkpoint_save(pperm_ctx* x, void* host_buf, size_t bytes) {
    if (!x || !host_buf) return PPERM_EINVAL;
    size_t need = 0;
    pperm_checkpoint_bytes(x, &need);
    if (bytes < need) return PPERM_EINVAL;
    if (x->open_tours != 0) return PPERM_ESTATE;
    int rc = check_device_errors(x);
    if (rc) return rc;
    uint64_t off[8], len[8];
    const int k = ckpt_sections(x, off, len);
    CkptHeader h;
    memset(&h, 0, sizeof(h));
    h.magic = kCkptMagic;
    h.version = kCkptVersion;
    h.sections = (uint32_t)k;
    h.cfg = x->cfg;
    h.merged_tours = x->merged_tours;
    h.payload_bytes = need - sizeof(CkptHeader);
    unsigned char* dst = static_cast<unsigned char*>(host_buf);
    memcpy(dst, &h, sizeof(h));
    dst += sizeof(h);
    for (int i = 0; i < k; ++i) {
        HIP_TRY(hipMemcpyAsync(dst, x->ws + off[i], len[i], hipMemcpyDeviceToHost, x->stream));
        dst += len[i];
    }
    HIP_TRY(hipStreamSynchronize(x->stream));
    return PPERM_OK;
}

int pperm_checkpoint_load(pperm_ctx* x, const void* host_buf, size_t bytes) {
    if (!x || !host_buf || bytes < sizeof(CkptHeader)) return PPERM_EINVAL;
    CkptHeader h;
    memcpy(&h, host_buf, sizeof(h));
    if (h.magic != kCkptMagic || h.version != kCkptVersion) return PPERM_EINVAL;
    if (!same_problem(h.cfg, x->cfg)) return PPERM_EINVAL;
    size_t need = 0;
    pperm_checkpoint_bytes(x, &need);
    uint64_t off[8], len[8];
    const int k = ckpt_sections(x, off, len);
    if (bytes < need || h.payload_bytes != need - sizeof(CkptHeader) || h.sections != (uint32_t)k)
        return PPERM_EINVAL;
    if (x->open_tours != 0) return PPERM_ESTATE;
    int rc = check_device_errors(x);
    if (rc) return rc;
    const unsigned char* src = static_cast<const unsigned char*>(host_buf) + sizeof(h);
    for (int i = 0; i < k; ++i) {
        HIP_TRY(hipMemcpyAsync(x->ws + off[i], src, len[i], hipMemcpyHostToDevice, x->stream));
        src += len[i];
    }
    HIP_TRY(hipStreamSynchronize(x->stream));
    x->merged_tours = h.merged_tours;
    return PPERM_OK;
}

int pperm_layout_of(const pperm_ctx* x, pperm_layout* out) {
    if (!x || !out) return PPERM_EINVAL;
    *out = x->lay;
    return PPERM_OK;
}

int pperm_launch_shape(const pperm_ctx* x, uint32_t* walks_per_wave, uint32_t* hash_slots,
                       uint32_t* workgroups) {
    if (!x) return PPERM_EINVAL;
    if (walks_per_wave) *walks_per_wave = 64u / x->team_lanes;
    if (hash_slots) *hash_slots = x->slots;
    if (workgroups) *workgroups = x->workgroups;
    return PPERM_OK;
}

int pperm_destroy(pperm_ctx* x) {
    if (!x) return PPERM_EINVAL;
    delete x;
    return PPERM_OK;
}

}  // extern "C"
