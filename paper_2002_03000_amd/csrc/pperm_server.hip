// Serving on top of the chained launch: continuous batching of sampling jobs.
//
// Host code only.  The server carves job workspaces out of one caller-owned
// device pool (first-fit over 256-byte blocks, neighbours coalesced on free),
// admits queued jobs in arrival order while their workspace and their
// sequences fit, and advances every active job by one time slice per step: one
// pperm_run_job_sliced call in which each job runs its next epochs at its own
// pace, with its stop rule evaluated on the device after every merge.  Between
// steps a job's resident state is its context (pooled sums, group sums,
// counters); a job that has met its stop rule is retired, its estimates are
// copied to the host and its pool block is returned.
#include <math.h>
#include <string.h>

#include <algorithm>
#include <deque>
#include <iterator>
#include <map>
#include <new>
#include <unordered_map>
#include <vector>

#include "pperm.h"
#include "pperm_internal.h"

namespace {

constexpr uint64_t kBlock = 256;
constexpr uint32_t kSliceEpochs = 64;   // most epochs of one job per step

uint64_t round_block(uint64_t x) { return (x + kBlock - 1) / kBlock * kBlock; }

// First-fit allocator over byte offsets [0, capacity).
class Pool {
public:
    explicit Pool(uint64_t capacity) : capacity_(capacity / kBlock * kBlock) {
        if (capacity_) free_[0] = capacity_;
    }
    // offset of a new block of at least `bytes`, or -1
    int64_t alloc(uint64_t bytes) {
        const uint64_t need = round_block(bytes ? bytes : 1);
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second < need) continue;
            const uint64_t off = it->first, size = it->second;
            free_.erase(it);
            if (size > need) free_[off + need] = size - need;
            used_[off] = need;
            in_use_ += need;
            return (int64_t)off;
        }
        return -1;
    }
    bool release(uint64_t off) {
        auto u = used_.find(off);
        if (u == used_.end()) return false;
        uint64_t start = off, size = u->second;
        in_use_ -= size;
        used_.erase(u);
        auto next = free_.lower_bound(start);
        if (next != free_.end() && start + size == next->first) {
            size += next->second;
            next = free_.erase(next);
        }
        if (next != free_.begin()) {
            auto prev = std::prev(next);
            if (prev->first + prev->second == start) {
                start = prev->first;
                size += prev->second;
                free_.erase(prev);
            }
        }
        free_[start] = size;
        return true;
    }
    uint64_t in_use() const { return in_use_; }
    uint64_t capacity() const { return capacity_; }

private:
    uint64_t capacity_;
    uint64_t in_use_ = 0;
    std::map<uint64_t, uint64_t> free_;   // offset -> size
    std::map<uint64_t, uint64_t> used_;
};

// Tours per sequence of epoch e of a job: with warm-up the first T tours are
// split into epochs of 1, 1, 2, 4, ... (doubling while the running total stays
// within T) and one epoch of the remainder; every later epoch has T tours.
uint32_t epoch_tours(const pperm_job& j, uint32_t e) {
    const uint64_t T = j.tours_per_epoch;
    if (!j.warmup || T == 1) return (uint32_t)T;
    if (e == 0) return 1;
    uint64_t sum = 1;
    uint32_t i = 1;
    while (2 * sum <= T) {
        if (e == i) return (uint32_t)sum;
        sum += sum;
        ++i;
    }
    if (sum < T) {
        if (e == i) return (uint32_t)(T - sum);
        ++i;
    }
    return (uint32_t)T;
}

struct Job {
    uint64_t id = 0;
    pperm_job spec;
    pperm_config cfg;
    uint64_t bytes = 0;
    int64_t off = -1;
    pperm_ctx* ctx = nullptr;
    pperm_job_info info;
    uint32_t running = 0;          // tours per sequence of the epoch in flight
    std::vector<double> log_cn;
    std::vector<uint64_t> hist;
};

}  // namespace

struct pperm_server {
    unsigned char* pool_base = nullptr;
    Pool pool{0};
    uint32_t max_seq = 0;
    hipStream_t stream = nullptr;
    unsigned char* scratch = nullptr;   // workspace of the chained launches
    size_t scratch_bytes = 0;
    uint32_t slice_us = 100000;
    uint64_t next_id = 1;
    uint64_t active_seq = 0;
    std::deque<Job*> queue;
    std::vector<Job*> active;
    std::unordered_map<uint64_t, Job*> jobs;
};

namespace {

void retire(pperm_server* S, Job* j, uint32_t state, int error) {
    j->info.state = state;
    j->info.error = error;
    if (j->ctx) {
        pperm_destroy(j->ctx);
        j->ctx = nullptr;
    }
    if (j->off >= 0) {
        S->pool.release((uint64_t)j->off);
        j->off = -1;
    }
}

// Copy a finished job's estimates and counters to the host.
int collect(Job* j) {
    const size_t n1 = j->cfg.n_max + 1u;
    j->log_cn.assign(n1, 0.0);
    j->hist.assign(n1, 0);
    uint64_t tours = 0;
    int rc = pperm_estimates(j->ctx, j->log_cn.data(), j->hist.data(), &tours, n1);
    if (rc) return rc;
    pperm_seq_stats tot;
    rc = pperm_stats(j->ctx, &tot);
    if (rc) return rc;
    j->info.steps = tot.steps;
    return PPERM_OK;
}

}  // namespace

extern "C" {

int64_t pperm_pool_script(uint64_t pool_bytes, const int64_t* ops, size_t count, int64_t* offsets) {
    if (!ops || !offsets) return -1;
    Pool p(pool_bytes);
    for (size_t i = 0; i < count; ++i) {
        if (ops[i] > 0) {
            offsets[i] = p.alloc((uint64_t)ops[i]);
        } else {
            const int64_t k = -ops[i] - 1;
            offsets[i] = 0;
            if (k >= 0 && (size_t)k < i && offsets[k] >= 0 && ops[k] > 0) p.release((uint64_t)offsets[k]);
        }
    }
    return (int64_t)p.in_use();
}

int pperm_server_create(void* d_pool, size_t pool_bytes, uint32_t max_active_sequences,
                        void* hip_stream, pperm_server** out) {
    if (!out || !d_pool || max_active_sequences == 0) return PPERM_EINVAL;
    *out = nullptr;
    if (((uintptr_t)d_pool & (kBlock - 1)) != 0) return PPERM_EINVAL;
    pperm_server* S = new (std::nothrow) pperm_server();
    if (!S) return PPERM_ENOMEM;
    S->pool_base = (unsigned char*)d_pool;
    S->pool = Pool(pool_bytes);
    S->max_seq = max_active_sequences;
    S->stream = (hipStream_t)hip_stream;
    // an eighth of the pool (at least 64 KiB) for the chained launches
    S->scratch_bytes = std::max<size_t>(pool_bytes / 8 / kBlock * kBlock, 65536);
    const int64_t off = S->pool.alloc(S->scratch_bytes);
    if (off < 0) {
        delete S;
        return PPERM_EINVAL;
    }
    S->scratch = S->pool_base + off;
    *out = S;
    return PPERM_OK;
}

int pperm_server_submit(pperm_server* S, const pperm_job* job, uint64_t* id) {
    if (!S || !job || !id) return PPERM_EINVAL;
    if (job->struct_size != sizeof(pperm_job)) return PPERM_EINVAL;
    if (job->tours_per_epoch == 0 || job->tour_cap == 0 || job->n_sequences > S->max_seq)
        return PPERM_EINVAL;
    if (job->mode == PPERM_INDEPENDENT) return PPERM_EINVAL;   // chained launches pool the sums
    if (!(job->target_rel_err >= 0.0)) return PPERM_EINVAL;
    // the pooled tour count stays below 2^32: the job stops at the first merge
    // with M >= tour_cap, so M < tour_cap + N * T
    if (job->tour_cap + (uint64_t)job->n_sequences * job->tours_per_epoch > 0xFFFFFFFFull)
        return PPERM_EOVERFLOW;
    Job* j = new (std::nothrow) Job();
    if (!j) return PPERM_ENOMEM;
    j->spec = *job;
    memset(&j->cfg, 0, sizeof(j->cfg));
    j->cfg.struct_size = sizeof(pperm_config);
    j->cfg.dim = job->dim;
    j->cfg.n_max = job->n_max;
    j->cfg.n_sequences = job->n_sequences;
    j->cfg.seed = job->seed;
    j->cfg.mode = job->mode;
    j->cfg.stream_id = job->stream_id;
    j->cfg.walks_per_wave = 1;
    j->cfg.flags = PPERM_FLAG_GROUP_STATS;
    size_t bytes = 0;
    int rc = pperm_workspace_bytes(&j->cfg, &bytes);
    if (rc == PPERM_OK && round_block(bytes) + S->scratch_bytes > S->pool.capacity())
        rc = PPERM_EINVAL;
    if (rc == PPERM_OK && pperm::config_long_walk(&j->cfg)) rc = PPERM_EINVAL;   // chained launches keep sums in LDS
    if (rc) {
        delete j;
        return rc;
    }
    j->bytes = bytes;
    memset(&j->info, 0, sizeof(j->info));
    j->info.state = PPERM_JOB_QUEUED;
    j->info.rel_err = INFINITY;
    j->info.workspace_bytes = round_block(bytes);
    j->id = S->next_id++;
    S->jobs[j->id] = j;
    S->queue.push_back(j);
    *id = j->id;
    return PPERM_OK;
}

int pperm_server_step(pperm_server* S, uint64_t* finished, size_t cap, size_t* n_finished) {
    if (!S || !n_finished || (cap && !finished)) return PPERM_EINVAL;
    size_t nf = 0;
    auto report = [&](Job* j) {
        if (nf < cap) finished[nf] = j->id;
        ++nf;
    };

    // admission, in arrival order
    while (!S->queue.empty()) {
        Job* j = S->queue.front();
        if (S->active_seq + j->cfg.n_sequences > S->max_seq) break;
        const int64_t off = S->pool.alloc(j->bytes);
        if (off < 0) break;
        S->queue.pop_front();
        j->off = off;
        const int rc = pperm_create(&j->cfg, S->pool_base + off, j->bytes, S->stream, &j->ctx);
        if (rc) {
            retire(S, j, PPERM_JOB_FAILED, rc);
            report(j);
            continue;
        }
        j->info.state = PPERM_JOB_ACTIVE;
        S->active.push_back(j);
        S->active_seq += j->cfg.n_sequences;
    }
    if (S->active.empty()) {
        *n_finished = nf;
        return PPERM_OK;
    }

    // the next epochs of every active job (up to its tour cap, at most
    // kSliceEpochs; fewer while the launch's workspace does not fit)
    const size_t na = S->active.size();
    std::vector<pperm_ctx*> ctxs(na);
    std::vector<std::vector<uint32_t>> sched(na);
    std::vector<const uint32_t*> sp(na);
    std::vector<uint32_t> ep(na), done(na), stop(na);
    std::vector<double> rel(na);
    std::vector<pperm_job_limits> lim(na);
    size_t need = 0;
    for (uint32_t limit = kSliceEpochs;; limit = std::max<uint32_t>(1u, limit / 2)) {
        for (size_t i = 0; i < na; ++i) {
            Job* j = S->active[i];
            ctxs[i] = j->ctx;
            sched[i].clear();
            uint64_t M = j->info.tours;
            while (sched[i].size() < limit && M < j->spec.tour_cap) {
                const uint32_t T = epoch_tours(j->spec, j->info.epochs + (uint32_t)sched[i].size());
                sched[i].push_back(T);
                M += (uint64_t)j->cfg.n_sequences * T;
            }
            ep[i] = (uint32_t)sched[i].size();
            sp[i] = sched[i].data();
            lim[i].target_rel_err = j->spec.target_rel_err;
            lim[i].tour_cap = j->spec.tour_cap;
        }
        int rc = pperm_job_workspace_bytes(ctxs.data(), ep.data(), na, &need);
        if (rc) return rc;
        if (need <= S->scratch_bytes) break;
        if (limit == 1u) return PPERM_ENOMEM;
    }
    int rc = pperm_run_job_sliced(ctxs.data(), sp.data(), ep.data(), na, S->scratch, S->scratch_bytes, S->stream,
                                  lim.data(), S->slice_us, done.data(), stop.data(), rel.data());
    if (rc) return rc;

    // progress, stop rules, retirement
    std::vector<Job*> still;
    still.reserve(na);
    for (size_t i = 0; i < na; ++i) {
        Job* j = S->active[i];
        for (uint32_t e = 0; e < done[i]; ++e) j->info.tours += (uint64_t)j->cfg.n_sequences * sched[i][e];
        j->info.epochs += done[i];
        if (done[i] && j->spec.target_rel_err > 0.0) j->info.rel_err = rel[i];
        rc = pperm_sync(j->ctx);
        if (rc == PPERM_EDEVICE) return rc;
        if (rc == PPERM_OK && stop[i] == 0u) {
            still.push_back(j);
            continue;
        }
        if (rc == PPERM_OK) rc = collect(j);
        if (rc == PPERM_EDEVICE) return rc;
        j->info.stop = stop[i];
        S->active_seq -= j->cfg.n_sequences;
        retire(S, j, rc == PPERM_OK ? PPERM_JOB_DONE : PPERM_JOB_FAILED, rc);
        report(j);
    }
    S->active.swap(still);
    *n_finished = nf;
    return PPERM_OK;
}

int pperm_server_set_slice(pperm_server* S, uint32_t slice_us) {
    if (!S || slice_us == 0) return PPERM_EINVAL;
    S->slice_us = slice_us;
    return PPERM_OK;
}

int pperm_server_info(pperm_server* S, uint64_t id, pperm_job_info* info) {
    if (!S || !info) return PPERM_EINVAL;
    auto it = S->jobs.find(id);
    if (it == S->jobs.end()) return PPERM_EINVAL;
    *info = it->second->info;
    return PPERM_OK;
}

int pperm_server_result(pperm_server* S, uint64_t id, double* log_cn, uint64_t* hist, size_t len) {
    if (!S || !log_cn) return PPERM_EINVAL;
    auto it = S->jobs.find(id);
    if (it == S->jobs.end()) return PPERM_EINVAL;
    const Job* j = it->second;
    if (j->info.state != PPERM_JOB_DONE) return PPERM_ESTATE;
    if (len < j->log_cn.size()) return PPERM_EINVAL;
    memcpy(log_cn, j->log_cn.data(), j->log_cn.size() * sizeof(double));
    if (hist) memcpy(hist, j->hist.data(), j->hist.size() * sizeof(uint64_t));
    return PPERM_OK;
}

int pperm_server_release(pperm_server* S, uint64_t id) {
    if (!S) return PPERM_EINVAL;
    auto it = S->jobs.find(id);
    if (it == S->jobs.end()) return PPERM_EINVAL;
    Job* j = it->second;
    if (j->info.state != PPERM_JOB_DONE && j->info.state != PPERM_JOB_FAILED) return PPERM_ESTATE;
    S->jobs.erase(it);
    delete j;
    return PPERM_OK;
}

int pperm_server_counts(pperm_server* S, uint32_t* queued, uint32_t* active, uint64_t* pool_used) {
    if (!S) return PPERM_EINVAL;
    if (queued) *queued = (uint32_t)S->queue.size();
    if (active) *active = (uint32_t)S->active.size();
    if (pool_used) *pool_used = S->pool.in_use();
    return PPERM_OK;
}

int pperm_server_destroy(pperm_server* S) {
    if (!S) return PPERM_EINVAL;
    const hipError_t e = hipStreamSynchronize(S->stream);
    for (auto& kv : S->jobs) {
        if (kv.second->ctx) pperm_destroy(kv.second->ctx);
        delete kv.second;
    }
    delete S;
    return e == hipSuccess ? PPERM_OK : PPERM_EDEVICE;
}

}  // extern "C"
