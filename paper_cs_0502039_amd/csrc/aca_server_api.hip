// aca_server_api.hip -- C-ABI of the job server (declared in include/aca.h).
//
// Continuous batching of simulation jobs on one GPU: a FIFO admission queue,
// a first-fit allocator over the caller's device arena (the HBM budget), and
// one batch whose steps the server drives.  Admission happens between steps:
// a job is given arena memory for its state buffers and scratch, its initial
// state is drawn on the device, and it joins the batch; jobs that reach their
// horizon leave the batch with their state in their arena buffers, where the
// client reads it before releasing the job.
#include <hip/hip_runtime.h>

#include <stdint.h>
#include <string.h>

#include <algorithm>
#include <chrono>
#include <deque>
#include <iterator>
#include <map>
#include <unordered_map>
#include <vector>

#include "../../include/aca.h"
#include "aca_host.h"

using namespace aca_host;

namespace {

// First-fit allocator over [0, size) with coalescing of free neighbours.
class Arena {
public:
    void reset(uint64_t size)
    {
        free_.clear();
        if (size) free_[0] = size;
        size_ = size;
        used_ = 0;
        peak_ = 0;
    }

    bool alloc(uint64_t bytes, uint64_t *off)
    {
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second < bytes) continue;
            *off = it->first;
            const uint64_t rest = it->second - bytes;
            const uint64_t at = it->first + bytes;
            free_.erase(it);
            if (rest) free_[at] = rest;
            used_ += bytes;
            peak_ = std::max(peak_, used_);
            return true;
        }
        return false;
    }

    void release(uint64_t off, uint64_t bytes)
    {
        auto next = free_.lower_bound(off);
        uint64_t start = off, len = bytes;
        if (next != free_.begin()) {
            auto prev = std::prev(next);
            if (prev->first + prev->second == off) {
                start = prev->first;
                len += prev->second;
                free_.erase(prev);
            }
        }
        if (next != free_.end() && off + bytes == next->first) {
            len += next->second;
            free_.erase(next);
        }
        free_[start] = len;
        used_ -= bytes;
    }

    uint64_t size() const { return size_; }
    uint64_t peak() const { return peak_; }

private:
    std::map<uint64_t, uint64_t> free_;   // offset -> length
    uint64_t size_ = 0, used_ = 0, peak_ = 0;
};

struct JobLayout {
    uint64_t spin, time, count, scratch, scratch_bytes, total;
};

aca_status job_layout(const aca_params *p, JobLayout *l)
{
    uint64_t n = 0, sb = 0;
    aca_status st = aca_query(p, &n, &sb);
    if (st != ACA_OK) return st;
    uint64_t off = 0;
    l->spin = off;
    off = align_up(off + n);
    l->time = off;
    off = align_up(off + 8 * n);
    l->count = off;
    off = align_up(off + 4 * n);
    l->scratch = off;
    l->scratch_bytes = sb;
    off = align_up(off + sb);
    l->total = off;
    return ACA_OK;
}

struct Job {
    aca_params p;
    double T = 0.0;
    int32_t state = ACA_JOB_QUEUED;
    aca_lattice *lat = nullptr;
    uint64_t off = 0, bytes = 0;
    bool has_memory = false;
    aca_stats stats;
};

}  // namespace

struct aca_server {
    char *arena = nullptr;
    Arena alloc;
    aca_batch *batch = nullptr;
    int32_t max_jobs = 0;
    int32_t running = 0;
    uint64_t next_id = 0;
    std::deque<uint64_t> queue;
    std::unordered_map<uint64_t, Job> jobs;
    std::unordered_map<const aca_lattice *, uint64_t> by_lattice;
    aca_server_stats stats;
};

namespace {

void drop_memory(aca_server *srv, Job &job)
{
    if (job.lat) {
        srv->by_lattice.erase(job.lat);
        aca_destroy(job.lat);
        job.lat = nullptr;
    }
    if (job.has_memory) {
        srv->alloc.release(job.off, job.bytes);
        job.has_memory = false;
    }
}

// Give the job memory, draw its initial state and attach it; false (and the
// job untouched) when the arena has no room for it now.
aca_status admit(aca_server *srv, uint64_t id, Job &job, hipStream_t s, bool *admitted)
{
    *admitted = false;
    JobLayout l;
    aca_status st = job_layout(&job.p, &l);
    if (st != ACA_OK) return st;
    uint64_t off = 0;
    if (!srv->alloc.alloc(l.total, &off)) return ACA_OK;
    job.off = off;
    job.bytes = l.total;
    job.has_memory = true;
    char *base = srv->arena + off;
    st = aca_create(&job.p, reinterpret_cast<int8_t *>(base + l.spin),
                    reinterpret_cast<double *>(base + l.time),
                    reinterpret_cast<uint32_t *>(base + l.count), base + l.scratch,
                    l.scratch_bytes, &job.lat);
    if (st == ACA_OK) st = aca_init(job.lat, s);
    if (st == ACA_OK) st = aca_batch_attach(srv->batch, job.lat, job.T);
    if (st != ACA_OK) {
        drop_memory(srv, job);
        job.state = ACA_JOB_FAILED;
        srv->stats.failed += 1;
        return st;
    }
    srv->by_lattice[job.lat] = id;
    job.state = ACA_JOB_RUNNING;
    srv->running += 1;
    srv->stats.admitted += 1;
    *admitted = true;
    return ACA_OK;
}

}  // namespace

ACA_EXPORT aca_status aca_server_query(int32_t max_jobs, uint64_t *work_bytes)
{
    return aca_batch_query(max_jobs, work_bytes);
}

ACA_EXPORT aca_status aca_server_job_bytes(const aca_params *p, uint64_t *bytes)
{
    if (!bytes) return fail(ACA_EINVAL, "bytes is NULL");
    JobLayout l;
    aca_status st = job_layout(p, &l);
    if (st != ACA_OK) return st;
    *bytes = l.total;
    return ACA_OK;
}

ACA_EXPORT aca_status aca_server_create(void *d_arena, uint64_t arena_bytes, void *d_work,
                                        uint64_t work_bytes, int32_t max_jobs,
                                        aca_server **out)
{
    if (!d_arena || !out) return fail(ACA_EINVAL, "NULL argument");
    if (((uintptr_t)d_arena) % kAlign != 0)
        return fail(ACA_EINVAL, "arena must be %zu-byte aligned", kAlign);
    if (arena_bytes < kAlign) return fail(ACA_EINVAL, "arena of %llu bytes is too small",
                                          (unsigned long long)arena_bytes);
    aca_batch *batch = nullptr;
    aca_status st = aca_batch_create(max_jobs, d_work, work_bytes, &batch);
    if (st != ACA_OK) return st;
    aca_server *srv = new (std::nothrow) aca_server();
    if (!srv) {
        aca_batch_destroy(batch);
        return fail(ACA_ENOMEM, "host allocation failed");
    }
    srv->arena = static_cast<char *>(d_arena);
    srv->alloc.reset(arena_bytes & ~(uint64_t)(kAlign - 1));
    srv->batch = batch;
    srv->max_jobs = max_jobs;
    // serve jobs in arrival order: a job's wait is bounded by the ones before it
    aca_batch_set_order(batch, ACA_ORDER_ARRIVAL);
    memset(&srv->stats, 0, sizeof srv->stats);
    srv->stats.struct_size = sizeof(aca_server_stats);
    srv->stats.arena_bytes = srv->alloc.size();
    *out = srv;
    return ACA_OK;
}

ACA_EXPORT aca_status aca_server_set_tuning(aca_server *srv, int32_t dim, const aca_tuning *t)
{
    if (!srv) return fail(ACA_EINVAL, "server is NULL");
    return aca_batch_set_tuning(srv->batch, dim, t);
}

ACA_EXPORT aca_status aca_server_set_order(aca_server *srv, int32_t order)
{
    if (!srv) return fail(ACA_EINVAL, "server is NULL");
    return aca_batch_set_order(srv->batch, order);
}

ACA_EXPORT aca_status aca_server_submit(aca_server *srv, const aca_params *p, double T,
                                        uint64_t *job)
{
    if (!srv || !p) return fail(ACA_EINVAL, "NULL argument");
    aca_params full;
    aca_status st = check_params(p, nullptr, &full);
    if (st != ACA_OK) return st;
    if (full.range > 1)
        return fail(ACA_EINVAL, "q-th degree neighbourhoods run on the single-lattice path");
    p = &full;
    JobLayout l;
    st = job_layout(p, &l);
    if (st != ACA_OK) return st;
    if (!is_finite(T) || T <= 0.0) return fail(ACA_EINVAL, "horizon must be finite and > 0");
    if (!aca_host::horizon_fits_counts(p->rate, T))
        return fail(ACA_EINVAL, "rate * horizon = %.17g exceeds 2^30 (arrival counts are 31-bit)",
                    p->rate * T);
    if (l.total > srv->alloc.size())
        return fail(ACA_ENOMEM, "job needs %llu arena bytes, the arena has %llu",
                    (unsigned long long)l.total, (unsigned long long)srv->alloc.size());
    const uint64_t id = srv->next_id++;
    Job j;
    j.p = *p;
    j.T = T;
    memset(&j.stats, 0, sizeof j.stats);
    j.stats.struct_size = sizeof(aca_stats);
    srv->jobs.emplace(id, j);
    srv->queue.push_back(id);
    srv->stats.submitted += 1;
    srv->stats.queued_peak = std::max<uint64_t>(srv->stats.queued_peak, srv->queue.size());
    if (job) *job = id;
    return ACA_OK;
}

ACA_EXPORT aca_status aca_server_step(aca_server *srv, double budget_ms, void *stream,
                                      uint64_t *done, int32_t cap, int32_t *n_done)
{
    if (!srv || !n_done || (cap > 0 && !done)) return fail(ACA_EINVAL, "NULL argument");
    const auto t0 = std::chrono::steady_clock::now();
    hipStream_t s = static_cast<hipStream_t>(stream);
    *n_done = 0;
    aca_status result = ACA_OK;
    // admission: arrival order, while a slot and arena room are free
    while (!srv->queue.empty() && srv->running < srv->max_jobs) {
        const uint64_t id = srv->queue.front();
        Job &job = srv->jobs.at(id);
        bool admitted = false;
        aca_status st = admit(srv, id, job, s, &admitted);
        if (st != ACA_OK) {
            srv->queue.pop_front();       // failed: released, reported
            if (result == ACA_OK) result = st;
            continue;
        }
        if (!admitted) break;             // wait for memory to free up
        srv->queue.pop_front();
    }
    if (srv->running == 0) return result;
    aca_batch_stats before;
    aca_batch_get_stats(srv->batch, &before);
    int32_t left = 0;
    aca_status st = aca_batch_step(srv->batch, budget_ms, 0, stream, &left);
    if (st != ACA_OK && result == ACA_OK) result = st;
    aca_batch_stats after;
    aca_batch_get_stats(srv->batch, &after);
    srv->stats.steps += 1;
    srv->stats.kernel_ms += after.kernel_ms - before.kernel_ms;
    // finished jobs
    std::vector<aca_lattice *> fin(srv->max_jobs);
    int32_t nf = 0;
    aca_batch_poll(srv->batch, fin.data(), (int32_t)fin.size(), &nf);
    int32_t nd = 0;
    for (int32_t i = 0; i < nf; ++i) {
        const uint64_t id = srv->by_lattice.at(fin[i]);
        Job &job = srv->jobs.at(id);
        job.state = ACA_JOB_DONE;
        aca_get_stats(job.lat, &job.stats);
        srv->running -= 1;
        srv->stats.finished += 1;
        srv->stats.events += job.stats.events;
        if (nd < cap) done[nd] = id;
        ++nd;
    }
    // members the batch dropped with an error
    if (st != ACA_OK && srv->running > 0) {
        std::vector<aca_lattice *> mem(srv->max_jobs);
        int32_t nm = 0;
        aca_batch_members(srv->batch, mem.data(), (int32_t)mem.size(), &nm);
        std::vector<uint64_t> lost;
        for (auto &kv : srv->by_lattice) {
            if (srv->jobs.at(kv.second).state != ACA_JOB_RUNNING) continue;
            if (std::find(mem.begin(), mem.begin() + nm, kv.first) == mem.begin() + nm)
                lost.push_back(kv.second);
        }
        for (uint64_t id : lost) {
            Job &job = srv->jobs.at(id);
            drop_memory(srv, job);
            job.state = ACA_JOB_FAILED;
            srv->running -= 1;
            srv->stats.failed += 1;
        }
    }
    *n_done = nd;
    srv->stats.arena_peak = srv->alloc.peak();
    srv->stats.device_ms +=
        std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0)
            .count();
    return result;
}

ACA_EXPORT aca_status aca_server_job(const aca_server *srv, uint64_t job, int32_t *state,
                                     aca_stats *stats)
{
    if (!srv) return fail(ACA_EINVAL, "server is NULL");
    auto it = srv->jobs.find(job);
    if (it == srv->jobs.end()) return fail(ACA_EINVAL, "unknown job %llu", (unsigned long long)job);
    if (state) *state = it->second.state;
    if (stats) *stats = it->second.stats;
    return ACA_OK;
}

ACA_EXPORT aca_status aca_server_read(aca_server *srv, uint64_t job, int8_t *h_spin,
                                      double *h_time, uint32_t *h_count, void *stream)
{
    if (!srv) return fail(ACA_EINVAL, "server is NULL");
    auto it = srv->jobs.find(job);
    if (it == srv->jobs.end()) return fail(ACA_EINVAL, "unknown job %llu", (unsigned long long)job);
    if (it->second.state != ACA_JOB_DONE)
        return fail(ACA_ESTATE, "job %llu is not done", (unsigned long long)job);
    return aca_read(it->second.lat, h_spin, h_time, h_count, stream);
}

ACA_EXPORT aca_status aca_server_release(aca_server *srv, uint64_t job)
{
    if (!srv) return fail(ACA_EINVAL, "server is NULL");
    auto it = srv->jobs.find(job);
    if (it == srv->jobs.end()) return fail(ACA_EINVAL, "unknown job %llu", (unsigned long long)job);
    if (it->second.state != ACA_JOB_DONE && it->second.state != ACA_JOB_FAILED)
        return fail(ACA_ESTATE, "job %llu is still queued or running", (unsigned long long)job);
    drop_memory(srv, it->second);
    srv->jobs.erase(it);
    return ACA_OK;
}

ACA_EXPORT aca_status aca_server_load(const aca_server *srv, int32_t *queued, int32_t *running)
{
    if (!srv) return fail(ACA_EINVAL, "server is NULL");
    if (queued) *queued = (int32_t)srv->queue.size();
    if (running) *running = srv->running;
    return ACA_OK;
}

ACA_EXPORT aca_status aca_server_get_stats(const aca_server *srv, aca_server_stats *out)
{
    if (!srv || !out) return fail(ACA_EINVAL, "NULL argument");
    *out = srv->stats;
    return ACA_OK;
}

ACA_EXPORT aca_status aca_server_destroy(aca_server *srv)
{
    if (!srv) return ACA_OK;
    if (!srv->queue.empty() || srv->running > 0)
        return fail(ACA_ESTATE, "server still has queued or running jobs");
    for (auto &kv : srv->jobs) drop_memory(srv, kv.second);
    aca_batch_destroy(srv->batch);
    delete srv;
    return ACA_OK;
}
