// Serving loop: memory-admitted, continuously batched sort and region jobs.
//
// Jobs arrive at any time (meld_server_submit, non-blocking) and wait in a
// FIFO. A dispatcher thread admits the head of the queue as soon as a slot
// (a HIP stream with its own library context, so that concurrent jobs never
// share scratch) and enough of the device-memory budget are free; small sort
// jobs (<= 65536 keys) standing next to each other at the head of the queue
// are packed into one segmented-sort launch (continuous batching: whatever
// has arrived while earlier work was on the GPU is admitted together). Large
// sorts and region jobs run one per slot; slots overlap on the device. A job's
// result stays resident in the budget until the caller releases it.
//
// The scheduling core is independent of HIP: an Executor runs units of work.
// The HIP executor enqueues the library's kernels; the simulated executor
// (for host-only tests) completes a unit after a modelled duration and can
// fail chosen jobs.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <unordered_set>
#include <vector>

#include "../../include/meld.h"
#include "kernels.h"

namespace {

thread_local std::string s_err;

meld_status serve_fail(meld_status st, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    s_err = buf;
    return st;
}

constexpr size_t kSmallSortMax = 65536;  // longest sort job packed into a batch
constexpr size_t kMaxBatchJobs = 4096;
constexpr size_t kAlign = 256;

size_t round_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

size_t job_bytes(const meld_job &j) {
    return j.kind == MELD_JOB_SORT ? round_up(j.n * sizeof(uint32_t))
                                   : round_up(j.n * sizeof(float)) * 2;  // x and y
}

struct JobRec {
    meld_job job;
    uint64_t id = 0;
    double arrival_s = 0, submit_s = 0, start_s = 0, done_s = 0;
    meld_status status = MELD_OK;
    size_t offset = 0;     // within the unit's arena block
    int unit = -1;         // index into Server::units_
    int batched = 1;
    bool done = false;
};

// A unit of work on one slot: one job, or a batch of small sorts.
struct Unit {
    std::vector<uint64_t> jobs;
    size_t arena_off = 0, arena_bytes = 0;
    int slot = -1;
    bool batch = false;
    int live = 0;          // jobs not yet released
    bool finished = false;
};

// First-fit allocator over [0, size) (host bookkeeping of the device arena).
class Arena {
  public:
    explicit Arena(size_t size) : size_(size) { free_[0] = size; }
    bool alloc(size_t bytes, size_t *off) {
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second >= bytes) {
                *off = it->first;
                const size_t rest = it->second - bytes;
                const size_t at = it->first + bytes;
                free_.erase(it);
                if (rest) free_[at] = rest;
                used_ += bytes;
                return true;
            }
        }
        return false;
    }
    void release(size_t off, size_t bytes) {
        used_ -= bytes;
        auto it = free_.emplace(off, bytes).first;
        auto next = std::next(it);
        if (next != free_.end() && it->first + it->second == next->first) {
            it->second += next->second;
            free_.erase(next);
        }
        if (it != free_.begin()) {
            auto prev = std::prev(it);
            if (prev->first + prev->second == it->first) {
                prev->second += it->second;
                free_.erase(it);
            }
        }
    }
    size_t used() const { return used_; }
    size_t size() const { return size_; }

  private:
    size_t size_;
    size_t used_ = 0;
    std::map<size_t, size_t> free_;
};

class Executor {
  public:
    virtual ~Executor() = default;
    virtual int slots() const = 0;
    // Enqueues the unit on its slot; must not wait for the device.
    virtual meld_status launch(Unit &u, std::vector<JobRec *> &jobs) = 0;
    // 1: finished (statuses set on the jobs), 0: running.
    virtual int poll(Unit &u, std::vector<JobRec *> &jobs) = 0;
    virtual const void *result(const Unit &u, const JobRec &j) const = 0;
    virtual void thread_init() {}
};

class SimExecutor : public Executor {
  public:
    SimExecutor(int slots, double ns_per_unit, const uint64_t *fail, size_t n_fail)
        : slots_(slots), ns_(ns_per_unit), fail_(fail, fail + n_fail) {}
    int slots() const override { return slots_; }
    meld_status launch(Unit &u, std::vector<JobRec *> &jobs) override {
        double work = 0;
        for (auto *j : jobs) work += (double)j->job.n;
        done_at_[u.slot] = now() + work * ns_ * 1e-9;
        return MELD_OK;
    }
    int poll(Unit &u, std::vector<JobRec *> &jobs) override {
        if (now() < done_at_[u.slot]) return 0;
        for (auto *j : jobs) j->status = fail_.count(j->id) ? MELD_EHIP : MELD_OK;
        return 1;
    }
    const void *result(const Unit &, const JobRec &) const override { return nullptr; }

  private:
    static double now() {
        return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch())
            .count();
    }
    int slots_;
    double ns_;
    std::unordered_set<uint64_t> fail_;
    std::map<int, double> done_at_;
};

class HipExecutor : public Executor {
  public:
    HipExecutor(int device, int slots, meld_variant v)
        : device_(device), slots_(slots), variant_(v) {}
    ~HipExecutor() override {
        (void)hipSetDevice(device_);
        for (auto &s : slot_) {
            if (s.stream) (void)hipStreamSynchronize(s.stream);
            if (s.done) (void)hipEventDestroy(s.done);
            if (s.stream) (void)hipStreamDestroy(s.stream);
            if (s.off_host) (void)hipHostFree(s.off_host);
            if (s.seed_host) (void)hipHostFree(s.seed_host);
            if (s.off_dev) (void)hipFree(s.off_dev);
            if (s.seed_dev) (void)hipFree(s.seed_dev);
            if (s.lib) meld_destroy(s.lib);
        }
        if (arena_) (void)hipFree(arena_);
        if (table_) (void)hipFree(table_);
    }
    meld_status init(size_t arena_bytes, uint64_t table_seed, uint32_t table_log2) {
        if (hipSetDevice(device_) != hipSuccess) return serve_fail(MELD_EHIP, "hipSetDevice");
        if (hipMalloc(&arena_, arena_bytes) != hipSuccess)
            return serve_fail(MELD_ENOMEM, "cannot allocate the %zu-byte job arena", arena_bytes);
        table_len_ = (size_t)1 << table_log2;
        if (hipMalloc(&table_, table_len_ * sizeof(float)) != hipSuccess)
            return serve_fail(MELD_ENOMEM, "cannot allocate the region table");
        if (meld::launch_gen_tab(table_, (uint32_t)table_len_, table_seed, nullptr) != hipSuccess ||
            hipDeviceSynchronize() != hipSuccess)
            return serve_fail(MELD_EHIP, "generating the region table");
        slot_.resize(slots_);
        for (auto &s : slot_) {
            if (meld_create(device_, &s.lib) != MELD_OK)
                return serve_fail(MELD_EHIP, "%s", meld_last_error());
            (void)meld_set_option(s.lib, MELD_OPT_USE_GRAPHS, 0);  // shapes change per batch
            if (hipStreamCreateWithFlags(&s.stream, hipStreamNonBlocking) != hipSuccess ||
                hipEventCreateWithFlags(&s.done, hipEventDisableTiming) != hipSuccess)
                return serve_fail(MELD_EHIP, "creating a slot stream");
            if (hipHostMalloc(reinterpret_cast<void **>(&s.off_host),
                              (kMaxBatchJobs + 1) * sizeof(uint32_t)) != hipSuccess ||
                hipHostMalloc(reinterpret_cast<void **>(&s.seed_host),
                              kMaxBatchJobs * sizeof(uint64_t)) != hipSuccess ||
                hipMalloc(reinterpret_cast<void **>(&s.off_dev),
                          (kMaxBatchJobs + 1) * sizeof(uint32_t)) != hipSuccess ||
                hipMalloc(reinterpret_cast<void **>(&s.seed_dev),
                          kMaxBatchJobs * sizeof(uint64_t)) != hipSuccess)
                return serve_fail(MELD_ENOMEM, "allocating slot staging");
        }
        return MELD_OK;
    }
    int slots() const override { return slots_; }
    void thread_init() override { (void)hipSetDevice(device_); }

    meld_status launch(Unit &u, std::vector<JobRec *> &jobs) override {
        Slot &s = slot_[u.slot];
        char *base = static_cast<char *>(arena_) + u.arena_off;
        meld_status st = MELD_OK;
        if (u.batch) {
            const uint32_t nseg = (uint32_t)jobs.size();
            uint32_t acc = 0, max_len = 0;
            for (uint32_t i = 0; i < nseg; ++i) {
                s.off_host[i] = acc;
                s.seed_host[i] = jobs[i]->job.seed;
                acc += (uint32_t)jobs[i]->job.n;
                max_len = std::max<uint32_t>(max_len, (uint32_t)jobs[i]->job.n);
            }
            s.off_host[nseg] = acc;
            uint32_t *keys = reinterpret_cast<uint32_t *>(base);
            hipError_t e = hipMemcpyAsync(s.off_dev, s.off_host, (nseg + 1) * sizeof(uint32_t),
                                          hipMemcpyHostToDevice, s.stream);
            if (e == hipSuccess)
                e = hipMemcpyAsync(s.seed_dev, s.seed_host, nseg * sizeof(uint64_t),
                                   hipMemcpyHostToDevice, s.stream);
            if (e == hipSuccess)
                e = meld::launch_gen_keys_segments(keys, s.off_dev, s.seed_dev, nseg, max_len,
                                                   s.stream);
            if (e != hipSuccess) return serve_fail(MELD_EHIP, "batch inputs: %s", hipGetErrorString(e));
            st = meld_segmented_sort_u32(s.lib, keys, acc, s.off_dev, nseg, variant_, s.stream);
        } else {
            JobRec *j = jobs[0];
            if (j->job.kind == MELD_JOB_SORT) {
                uint32_t *keys = reinterpret_cast<uint32_t *>(base);
                hipError_t e = meld::launch_gen_keys(keys, (uint32_t)j->job.n, j->job.seed, s.stream);
                if (e != hipSuccess) return serve_fail(MELD_EHIP, "sort input: %s", hipGetErrorString(e));
                st = meld_sort_u32(s.lib, keys, nullptr, j->job.n, variant_, s.stream);
            } else {
                float *x = reinterpret_cast<float *>(base);
                float *y = reinterpret_cast<float *>(base + round_up(j->job.n * sizeof(float)));
                hipError_t e = meld::launch_gen_x(x, (uint32_t)j->job.n, j->job.seed, s.stream);
                if (e != hipSuccess) return serve_fail(MELD_EHIP, "region input: %s", hipGetErrorString(e));
                st = meld_divergent_region_f32(s.lib, x, y, j->job.n, table_, table_len_,
                                               j->job.seed, j->job.thr, j->job.side_true,
                                               j->job.side_false, variant_, s.stream);
            }
        }
        if (st != MELD_OK) return serve_fail(st, "%s", meld_last_error());
        if (hipEventRecord(s.done, s.stream) != hipSuccess)
            return serve_fail(MELD_EHIP, "hipEventRecord");
        return MELD_OK;
    }

    int poll(Unit &u, std::vector<JobRec *> &jobs) override {
        const hipError_t e = hipEventQuery(slot_[u.slot].done);
        if (e == hipErrorNotReady) return 0;
        const meld_status st = e == hipSuccess ? MELD_OK : MELD_EHIP;
        for (auto *j : jobs) j->status = st;
        return 1;
    }

    const void *result(const Unit &u, const JobRec &j) const override {
        const char *base = static_cast<const char *>(arena_) + u.arena_off;
        if (u.batch) return base + j.offset;
        if (j.job.kind == MELD_JOB_SORT) return base;
        return base + round_up(j.job.n * sizeof(float));
    }

  private:
    struct Slot {
        meld_ctx *lib = nullptr;
        hipStream_t stream = nullptr;
        hipEvent_t done = nullptr;
        uint32_t *off_host = nullptr, *off_dev = nullptr;
        uint64_t *seed_host = nullptr, *seed_dev = nullptr;
    };
    int device_;
    int slots_;
    meld_variant variant_;
    void *arena_ = nullptr;
    float *table_ = nullptr;
    size_t table_len_ = 0;
    std::vector<Slot> slot_;
};

}  // namespace

struct meld_server {
    std::unique_ptr<Executor> exec;
    Arena arena;
    std::mutex mu;
    std::condition_variable cv;
    std::thread worker;
    bool stop = false;
    std::chrono::steady_clock::time_point t0 = std::chrono::steady_clock::now();
    uint64_t next_id = 1;
    std::deque<uint64_t> pending;
    // Jobs submitted ahead of their arrival, by (arrival, submission order):
    // they join the queue when the server's clock reaches their arrival.
    std::multimap<double, uint64_t> future;
    std::map<uint64_t, JobRec> jobs;
    std::deque<uint64_t> completed;
    std::vector<Unit> units;           // indexed by unit id
    std::vector<int> slot_unit;        // running unit per slot, -1 if free
    std::vector<int> free_units;
    meld_server_stats stats;
    size_t max_job_bytes;

    explicit meld_server(size_t budget) : arena(budget) {
        std::memset(&stats, 0, sizeof stats);
        stats.budget_bytes = budget;
        max_job_bytes = budget;
    }
    double now() const {
        return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    }

    int new_unit() {
        if (!free_units.empty()) {
            const int u = free_units.back();
            free_units.pop_back();
            units[u] = Unit();
            return u;
        }
        units.emplace_back();
        return (int)units.size() - 1;
    }

    // Admits from the head of the queue while a slot and memory are free.
    void admit() {
        for (;;) {
            if (pending.empty()) return;
            int slot = -1;
            for (int s = 0; s < (int)slot_unit.size(); ++s)
                if (slot_unit[s] < 0) {
                    slot = s;
                    break;
                }
            if (slot < 0) return;
            JobRec &head = jobs[pending.front()];
            const bool small =
                head.job.kind == MELD_JOB_SORT && head.job.n <= kSmallSortMax;
            std::vector<uint64_t> take{head.id};
            size_t keys = head.job.n;
            if (small) {
                // Pack the small sorts that follow the head (continuous batching).
                for (size_t q = 1; q < pending.size() && take.size() < kMaxBatchJobs; ++q) {
                    const JobRec &j = jobs[pending[q]];
                    if (j.job.kind != MELD_JOB_SORT || j.job.n > kSmallSortMax) break;
                    keys += j.job.n;
                    take.push_back(j.id);
                }
            }
            // The largest prefix of the pack that fits; strict FIFO: if even
            // the head does not fit, wait for memory.
            size_t off = 0, bytes = 0;
            for (;;) {
                bytes = small ? round_up(keys * sizeof(uint32_t)) : job_bytes(head.job);
                if (arena.alloc(bytes, &off)) break;
                if (take.size() == 1) return;
                keys -= jobs[take.back()].job.n;
                take.pop_back();
            }
            const int u = new_unit();
            Unit &unit = units[u];
            unit.jobs = take;
            unit.arena_off = off;
            unit.arena_bytes = bytes;
            unit.slot = slot;
            unit.batch = small;
            unit.live = (int)take.size();
            std::vector<JobRec *> recs;
            size_t pos = 0;
            const double t = now();
            for (uint64_t id : take) {
                JobRec &j = jobs[id];
                j.unit = u;
                j.start_s = t;
                j.offset = pos;
                j.batched = (int)take.size();
                pos += j.job.n * sizeof(uint32_t);
                recs.push_back(&j);
                pending.pop_front();
            }
            slot_unit[slot] = u;
            stats.launches++;
            if (take.size() > 1) stats.batched_jobs += take.size();
            stats.inflight_bytes = arena.used();
            stats.max_inflight_bytes = std::max(stats.max_inflight_bytes, stats.inflight_bytes);
            int running = 0;
            for (int su : slot_unit) running += su >= 0;
            stats.max_concurrent = std::max(stats.max_concurrent, running);
            const meld_status st = exec->launch(unit, recs);
            if (st != MELD_OK) {
                // A unit that failed to launch completes at once with the error.
                for (auto *j : recs) j->status = st;
                finish(u, recs);
            }
        }
    }

    void finish(int u, std::vector<JobRec *> &recs) {
        Unit &unit = units[u];
        const double t = now();
        for (auto *j : recs) {
            j->done_s = t;
            j->done = true;
            completed.push_back(j->id);
            stats.completed++;
            if (j->status != MELD_OK) stats.failed++;
        }
        unit.finished = true;
        slot_unit[unit.slot] = -1;
    }

    void poll_units() {
        for (int s = 0; s < (int)slot_unit.size(); ++s) {
            const int u = slot_unit[s];
            if (u < 0) continue;
            std::vector<JobRec *> recs;
            for (uint64_t id : units[u].jobs) recs.push_back(&jobs[id]);
            if (exec->poll(units[u], recs)) finish(u, recs);
        }
    }

    void release_job(uint64_t id) {
        JobRec &j = jobs[id];
        Unit &unit = units[j.unit];
        if (--unit.live == 0) {
            arena.release(unit.arena_off, unit.arena_bytes);
            stats.inflight_bytes = arena.used();
            free_units.push_back(j.unit);
        }
        jobs.erase(id);
    }

    // Moves the jobs whose arrival has come from `future` to the queue.
    void arrive() {
        const double t = now();
        while (!future.empty() && future.begin()->first <= t) {
            pending.push_back(future.begin()->second);
            future.erase(future.begin());
        }
    }

    void run() {
        exec->thread_init();
        std::unique_lock<std::mutex> lk(mu);
        while (!stop) {
            arrive();
            poll_units();
            admit();
            bool busy = false;
            for (int su : slot_unit) busy |= su >= 0;
            double wait_s = busy ? 20e-6 : 2e-3;
            if (!future.empty()) wait_s = std::min(wait_s, std::max(0.0, future.begin()->first - now()));
            cv.wait_for(lk, std::chrono::duration<double>(wait_s));
        }
    }
};

namespace {

meld_status start_server(meld_server *srv, int slots) {
    srv->slot_unit.assign(slots, -1);
    srv->stats.slots = slots;
    try {
        srv->worker = std::thread([srv]() { srv->run(); });
    } catch (...) {
        return serve_fail(MELD_EHIP, "cannot start the dispatcher thread");
    }
    return MELD_OK;
}

}  // namespace

extern "C" {

const char *meld_server_last_error(void) { return s_err.c_str(); }

meld_status meld_server_create(int hip_device, size_t mem_budget_bytes, int slots,
                               meld_variant variant, uint64_t table_seed, uint32_t table_log2,
                               meld_server **out) {
    if (out == nullptr) return serve_fail(MELD_EINVAL, "meld_server_create: out is NULL");
    *out = nullptr;
    if (slots < 1 || slots > 64) return serve_fail(MELD_EINVAL, "meld_server_create: slots not in 1..64");
    if (mem_budget_bytes < kAlign)
        return serve_fail(MELD_EINVAL, "meld_server_create: budget below %zu bytes", kAlign);
    if (table_log2 < 2 || table_log2 > 30)
        return serve_fail(MELD_EINVAL, "meld_server_create: table_log2 not in 2..30");
    if ((unsigned)variant > MELD_MELDED_INPLACE)
        return serve_fail(MELD_EINVAL, "meld_server_create: bad variant");
    std::unique_ptr<meld_server> srv(new (std::nothrow) meld_server(mem_budget_bytes));
    if (!srv) return serve_fail(MELD_ENOMEM, "meld_server_create: out of host memory");
    auto exec = std::make_unique<HipExecutor>(hip_device, slots, variant);
    meld_status st = exec->init(mem_budget_bytes, table_seed, table_log2);
    if (st != MELD_OK) return st;
    srv->exec = std::move(exec);
    st = start_server(srv.get(), slots);
    if (st != MELD_OK) return st;
    *out = srv.release();
    return MELD_OK;
}

meld_status meld_server_create_simulated(size_t mem_budget_bytes, int slots, double ns_per_item,
                                         const uint64_t *fail_ids, size_t n_fail,
                                         meld_server **out) {
    if (out == nullptr) return serve_fail(MELD_EINVAL, "meld_server_create_simulated: out is NULL");
    *out = nullptr;
    if (slots < 1 || slots > 64 || mem_budget_bytes < kAlign || ns_per_item < 0)
        return serve_fail(MELD_EINVAL, "meld_server_create_simulated: bad arguments");
    std::unique_ptr<meld_server> srv(new (std::nothrow) meld_server(mem_budget_bytes));
    if (!srv) return serve_fail(MELD_ENOMEM, "out of host memory");
    srv->exec = std::make_unique<SimExecutor>(slots, ns_per_item, fail_ids, n_fail);
    meld_status st = start_server(srv.get(), slots);
    if (st != MELD_OK) return st;
    *out = srv.release();
    return MELD_OK;
}

meld_status meld_server_submit(meld_server *srv, const meld_job *job, uint64_t *job_id) {
    if (srv == nullptr || job == nullptr)
        return serve_fail(MELD_EINVAL, "meld_server_submit: NULL argument");
    if ((job->kind != MELD_JOB_SORT && job->kind != MELD_JOB_REGION) || job->n == 0 ||
        job->n >= (1ull << 31))
        return serve_fail(MELD_EINVAL, "meld_server_submit: bad kind or size");
    if (job->kind == MELD_JOB_REGION &&
        (job->thr > (1ull << 32) || job->side_true.trips > 65536 || job->side_false.trips > 65536))
        return serve_fail(MELD_EINVAL, "meld_server_submit: bad region parameters");
    if (!std::isfinite(job->arrival_s))
        return serve_fail(MELD_EINVAL, "meld_server_submit: arrival_s is not finite");
    const size_t bytes = job_bytes(*job);
    std::lock_guard<std::mutex> lk(srv->mu);
    srv->stats.submitted++;
    if (bytes > srv->arena.size()) {
        srv->stats.rejected++;
        return serve_fail(MELD_ENOMEM, "meld_server_submit: job needs %zu bytes, budget is %zu",
                          bytes, srv->arena.size());
    }
    JobRec rec;
    rec.job = *job;
    rec.id = srv->next_id++;
    rec.submit_s = srv->now();
    // A job scheduled ahead waits for its arrival; one submitted at or after
    // its arrival (or with none, arrival_s <= 0) joins the queue now.
    rec.arrival_s = job->arrival_s > 0 ? job->arrival_s : rec.submit_s;
    srv->jobs[rec.id] = rec;
    if (rec.arrival_s > rec.submit_s)
        srv->future.emplace(rec.arrival_s, rec.id);
    else
        srv->pending.push_back(rec.id);
    if (job_id) *job_id = rec.id;
    srv->cv.notify_one();
    return MELD_OK;
}

meld_status meld_server_poll(meld_server *srv, meld_completion *out, size_t cap, size_t *n_out) {
    if (srv == nullptr || n_out == nullptr || (cap > 0 && out == nullptr))
        return serve_fail(MELD_EINVAL, "meld_server_poll: NULL argument");
    std::lock_guard<std::mutex> lk(srv->mu);
    size_t n = 0;
    while (n < cap && !srv->completed.empty()) {
        const uint64_t id = srv->completed.front();
        srv->completed.pop_front();
        const JobRec &j = srv->jobs[id];
        meld_completion &c = out[n++];
        c.job_id = id;
        c.status = j.status;
        c.kind = j.job.kind;
        c.n = j.job.n;
        c.arrival_s = j.arrival_s;
        c.submit_s = j.submit_s;
        c.start_s = j.start_s;
        c.done_s = j.done_s;
        c.batched = j.batched;
        c.result_dev = j.status == MELD_OK ? srv->exec->result(srv->units[j.unit], j) : nullptr;
    }
    *n_out = n;
    return MELD_OK;
}

meld_status meld_server_release(meld_server *srv, uint64_t job_id) {
    if (srv == nullptr) return serve_fail(MELD_EINVAL, "meld_server_release: NULL server");
    std::lock_guard<std::mutex> lk(srv->mu);
    auto it = srv->jobs.find(job_id);
    if (it == srv->jobs.end() || !it->second.done)
        return serve_fail(MELD_EINVAL, "meld_server_release: job %llu is not completed",
                          (unsigned long long)job_id);
    srv->release_job(job_id);
    srv->cv.notify_one();
    return MELD_OK;
}

meld_status meld_server_drain(meld_server *srv, double timeout_s) {
    if (srv == nullptr) return serve_fail(MELD_EINVAL, "meld_server_drain: NULL server");
    const auto deadline = std::chrono::steady_clock::now() +
                          std::chrono::duration_cast<std::chrono::steady_clock::duration>(
                              std::chrono::duration<double>(timeout_s));
    for (;;) {
        {
            std::lock_guard<std::mutex> lk(srv->mu);
            bool busy = !srv->pending.empty() || !srv->future.empty();
            for (int su : srv->slot_unit) busy |= su >= 0;
            if (!busy) return MELD_OK;
        }
        if (std::chrono::steady_clock::now() > deadline)
            return serve_fail(MELD_EHIP, "meld_server_drain: timed out");
        std::this_thread::sleep_for(std::chrono::microseconds(200));
    }
}

meld_status meld_server_read(meld_server *srv, uint64_t job_id, void *host_dst, size_t bytes) {
    if (srv == nullptr || host_dst == nullptr)
        return serve_fail(MELD_EINVAL, "meld_server_read: NULL argument");
    const void *src = nullptr;
    size_t have = 0;
    {
        std::lock_guard<std::mutex> lk(srv->mu);
        auto it = srv->jobs.find(job_id);
        if (it == srv->jobs.end() || !it->second.done || it->second.status != MELD_OK)
            return serve_fail(MELD_EINVAL, "meld_server_read: job %llu has no result",
                              (unsigned long long)job_id);
        src = srv->exec->result(srv->units[it->second.unit], it->second);
        have = it->second.job.n * 4;
    }
    if (src == nullptr) return serve_fail(MELD_EUNSUPPORTED, "meld_server_read: simulated server");
    if (bytes > have) return serve_fail(MELD_EINVAL, "meld_server_read: result has %zu bytes", have);
    if (hipMemcpy(host_dst, src, bytes, hipMemcpyDeviceToHost) != hipSuccess)
        return serve_fail(MELD_EHIP, "meld_server_read: hipMemcpy failed");
    return MELD_OK;
}

meld_status meld_server_stats_get(meld_server *srv, meld_server_stats *out) {
    if (srv == nullptr || out == nullptr) return serve_fail(MELD_EINVAL, "meld_server_stats_get: NULL");
    std::lock_guard<std::mutex> lk(srv->mu);
    *out = srv->stats;
    out->pending = srv->pending.size() + srv->future.size();
    return MELD_OK;
}

double meld_server_now(meld_server *srv) { return srv == nullptr ? 0.0 : srv->now(); }

void meld_server_destroy(meld_server *srv) {
    if (srv == nullptr) return;
    {
        std::lock_guard<std::mutex> lk(srv->mu);
        srv->stop = true;
    }
    srv->cv.notify_all();
    if (srv->worker.joinable()) srv->worker.join();
    delete srv;
}

}  // extern "C"
