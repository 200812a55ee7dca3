// Continuous-batching server for complex128 permanents (include/perm.h).
//
// Requests are admitted by the footprint of their table of stored
// sub-permanents (16 * 2^n bytes, section 4's "storage" of every minor)
// against a budget, and run on the device as soon as a slot and memory are
// free:
//   * small orders (n <= small_n_max) wait in one FIFO and are launched
//     together through the batched on-chip kernel; up to two batches are in
//     flight on their own streams, so requests that arrive while one batch
//     runs join the next one;
//   * large orders wait in another FIFO and each runs the layer sweep on one
//     of max_large_slots streams, the head of the queue first (no request is
//     passed over, so a large request cannot starve).
// Device memory for every running request is carved from the caller's pool
// (first fit, 256-byte aligned) and returned when it completes.  One
// scheduler thread issues all device work and watches completion events;
// submit and poll only touch the queues under a mutex.
#include <algorithm>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

#include "perm_host.h"

using namespace permgpu;

namespace {

struct Request {
    uint64_t ticket = 0;
    int n = 0;
    std::vector<perm_c128_t> a;  // packed n x n
    perm_c128_t result{0.0, 0.0};
    int status = PERM_PENDING;
    size_t charge = 0;
    double t_submit = 0, t_admit = 0, t_start = 0, t_done = 0;
};

// First-fit allocator over [0, size) of the pool.
class Arena {
  public:
    void init(size_t size) {
        free_.clear();
        if (size) free_[0] = size;
    }
    bool alloc(size_t bytes, size_t *off) {
        bytes = (bytes + 255) & ~(size_t)255;
        if (bytes == 0) bytes = 256;
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second >= bytes) {
                *off = it->first;
                const size_t rest = it->second - bytes, start = it->first + bytes;
                free_.erase(it);
                if (rest) free_[start] = rest;
                return true;
            }
        }
        return false;
    }
    void release(size_t off, size_t bytes) {
        bytes = (bytes + 255) & ~(size_t)255;
        if (bytes == 0) bytes = 256;
        auto it = free_.emplace(off, bytes).first;
        auto nx = std::next(it);
        if (nx != free_.end() && it->first + it->second == nx->first) {
            it->second += nx->second;
            free_.erase(nx);
        }
        if (it != free_.begin()) {
            auto pv = std::prev(it);
            if (pv->first + pv->second == it->first) {
                pv->second += it->second;
                free_.erase(it);
            }
        }
    }

  private:
    std::map<size_t, size_t> free_;
};

struct Running {
    std::vector<Request *> reqs;
    hipEvent_t done = nullptr;
    size_t off = 0, bytes = 0;
    perm_c128_t *host_out = nullptr;  // pinned results
    bool busy = false;
};

constexpr int kSmallSlots = 2;

}  // namespace

struct perm_server {
    perm_server_config_t cfg{};
    int device = 0;
    std::mutex mu;
    std::condition_variable cv;
    std::deque<Request *> small_q, large_q;
    std::unordered_map<uint64_t, std::unique_ptr<Request>> all;
    size_t queued = 0, in_use = 0, budget = 0;
    uint64_t next_ticket = 1;
    bool stop = false;
    Arena arena;
    std::thread thr;
    hipStream_t small_stream[kSmallSlots] = {};
    std::vector<hipStream_t> large_stream;
    Running small_run[kSmallSlots];
    std::vector<Running> large_run;
    perm_c128_t *pin_small_in[kSmallSlots] = {};
    perm_c128_t *pin_small_out[kSmallSlots] = {};
    std::vector<perm_c128_t *> pin_large_in, pin_large_out;
    int thread_error = PERM_OK;
};

namespace {

size_t footprint(int n) { return (size_t)16 << (n < 1 ? 0 : n); }

void finish(perm_server_t *s, Running &r, int status) {
    const double t = now_seconds();
    for (size_t i = 0; i < r.reqs.size(); i++) {
        Request *q = r.reqs[i];
        q->status = status;
        if (status == PERM_OK) q->result = r.host_out[i];
        q->t_done = t;
        s->in_use -= q->charge;
    }
    s->arena.release(r.off, r.bytes);
    r.reqs.clear();
    r.busy = false;
}

// Device work of a small batch on slot i (no lock held: only the scheduler
// thread touches slots, the arena and running requests).  The carve-out at
// `off` was reserved under the lock.
int issue_small(perm_server_t *s, int i, const std::vector<Request *> &reqs, size_t off, size_t ws, size_t mats_b,
                size_t res_b) {
    const int count = (int)reqs.size();
    std::vector<int32_t> ns(count);
    std::vector<int64_t> offs(count);
    int64_t elems = 0;
    for (int j = 0; j < count; j++) {
        ns[j] = reqs[j]->n;
        offs[j] = elems;
        elems += (int64_t)reqs[j]->n * reqs[j]->n;
    }
    char *base = (char *)s->cfg.pool + off;
    perm_c128_t *pin_in = s->pin_small_in[i];
    for (int j = 0; j < count; j++)
        std::memcpy(pin_in + offs[j], reqs[j]->a.data(), (size_t)reqs[j]->n * reqs[j]->n * 16);
    hipStream_t st = s->small_stream[i];
    const double t = now_seconds();
    for (auto *q : reqs) q->t_admit = q->t_start = t;
    int rc = PERM_OK;
    if (elems && hipMemcpyAsync(base, pin_in, (size_t)elems * 16, hipMemcpyHostToDevice, st) != hipSuccess)
        rc = PERM_EDEVICE;
    if (rc == PERM_OK)
        rc = perm_solve_batch(PERM_COMPLEX128, count, ns.data(), offs.data(), base, base + mats_b, base + mats_b + res_b,
                              ws, st, 0);
    if (rc == PERM_OK &&
        hipMemcpyAsync(s->pin_small_out[i], base + mats_b, (size_t)count * 16, hipMemcpyDeviceToHost, st) != hipSuccess)
        rc = PERM_EDEVICE;
    if (rc == PERM_OK && hipEventRecord(s->small_run[i].done, st) != hipSuccess) rc = PERM_EDEVICE;
    if (rc != PERM_OK) (void)hipStreamSynchronize(st);
    return rc;
}

// Bytes a small batch needs from the pool: workspace, matrices, results.
void small_bytes(const std::vector<Request *> &reqs, size_t *ws, size_t *mats_b, size_t *res_b) {
    std::vector<int32_t> ns;
    int64_t elems = 0;
    for (auto *q : reqs) {
        ns.push_back(q->n);
        elems += (int64_t)q->n * q->n;
    }
    *ws = perm_batch_workspace_bytes(PERM_COMPLEX128, (int)ns.size(), ns.data());
    *mats_b = ((size_t)std::max<int64_t>(elems, 1) * 16 + 255) & ~(size_t)255;
    *res_b = ((size_t)reqs.size() * 16 + 255) & ~(size_t)255;
}

// Device work of one large request on slot i (no lock held).
int issue_large(perm_server_t *s, int i, Request *q, size_t off) {
    const int n = q->n;
    const size_t ws = c128_workspace_bytes(n);
    const size_t mat_b = ((size_t)n * n * 16 + 255) & ~(size_t)255;
    char *base = (char *)s->cfg.pool + off;
    char *d_a = base + ws, *d_res = base + ws + mat_b;
    hipStream_t st = s->large_stream[i];
    std::memcpy(s->pin_large_in[i], q->a.data(), (size_t)n * n * 16);
    q->t_admit = q->t_start = now_seconds();
    int rc = PERM_OK;
    if (n > 0 && hipMemcpyAsync(d_a, s->pin_large_in[i], (size_t)n * n * 16, hipMemcpyHostToDevice, st) != hipSuccess)
        rc = PERM_EDEVICE;
    if (rc == PERM_OK) rc = solve_c128_device(n, d_a, n > 0 ? n : 1, d_res, base, ws, st);
    if (rc == PERM_OK && hipMemcpyAsync(s->pin_large_out[i], d_res, 16, hipMemcpyDeviceToHost, st) != hipSuccess)
        rc = PERM_EDEVICE;
    if (rc == PERM_OK && hipEventRecord(s->large_run[i].done, st) != hipSuccess) rc = PERM_EDEVICE;
    if (rc != PERM_OK) (void)hipStreamSynchronize(st);
    return rc;
}

size_t large_bytes(int n) { return c128_workspace_bytes(n) + (((size_t)n * n * 16 + 255) & ~(size_t)255) + 256; }

// One launch decided under the lock and issued after it is released.
struct Planned {
    bool small;
    int slot;
    std::vector<Request *> reqs;
    size_t off, ws, mats_b, res_b;
};

// The scheduler holds the mutex only to look at completions, admit
// requests (budget, carve-out, slot) and record outcomes; copies into
// pinned memory and every launch happen with the mutex released, so
// submit and poll never wait behind host-side launch work.
void scheduler(perm_server_t *s) {
    (void)hipSetDevice(s->device);
    std::unique_lock<std::mutex> lk(s->mu);
    std::vector<Planned> plan;
    for (;;) {
        bool progress = false;
        // completions
        auto poll = [&](Running &r) {
            if (!r.busy) return;
            const hipError_t e = hipEventQuery(r.done);
            if (e == hipSuccess) {
                finish(s, r, PERM_OK);
                progress = true;
            } else if (e != hipErrorNotReady) {
                finish(s, r, PERM_EDEVICE);
                progress = true;
            }
        };
        for (auto &r : s->small_run) poll(r);
        for (auto &r : s->large_run) poll(r);
        if (s->stop) {
            bool busy = false;
            for (auto &r : s->small_run) busy |= r.busy;
            for (auto &r : s->large_run) busy |= r.busy;
            if (!busy) break;
        } else {
            plan.clear();
            // large requests: strict FIFO, one per free slot while memory allows
            for (size_t i = 0; i < s->large_run.size() && !s->large_q.empty(); i++) {
                if (s->large_run[i].busy) continue;
                Request *q = s->large_q.front();
                if (s->in_use + q->charge > s->budget) break;
                size_t off;
                const size_t bytes = large_bytes(q->n);
                if (!s->arena.alloc(bytes, &off)) break;  // pool fragmented: wait
                Running &run = s->large_run[i];
                run.reqs.assign(1, q);
                run.off = off;
                run.bytes = bytes;
                run.host_out = s->pin_large_out[i];
                run.busy = true;
                s->in_use += q->charge;
                s->large_q.pop_front();
                s->queued--;
                plan.push_back({false, (int)i, {q}, off, 0, 0, 0});
                progress = true;
            }
            // small requests: everything waiting (up to the batch limit) that fits
            for (int i = 0; i < kSmallSlots && !s->small_q.empty(); i++) {
                if (s->small_run[i].busy) continue;
                std::vector<Request *> take;
                size_t charge = 0;
                while (!s->small_q.empty() && (int)take.size() < s->cfg.max_small_batch) {
                    Request *q = s->small_q.front();
                    if (s->in_use + charge + q->charge > s->budget) break;
                    charge += q->charge;
                    take.push_back(q);
                    s->small_q.pop_front();
                }
                if (take.empty()) break;
                size_t ws, mats_b, res_b, off;
                small_bytes(take, &ws, &mats_b, &res_b);
                if (!s->arena.alloc(ws + mats_b + res_b, &off)) {
                    for (auto it = take.rbegin(); it != take.rend(); ++it) s->small_q.push_front(*it);
                    break;
                }
                Running &run = s->small_run[i];
                run.reqs = take;
                run.off = off;
                run.bytes = ws + mats_b + res_b;
                run.host_out = s->pin_small_out[i];
                run.busy = true;
                s->in_use += charge;
                s->queued -= take.size();
                plan.push_back({true, i, take, off, ws, mats_b, res_b});
                progress = true;
            }
            if (!plan.empty()) {
                lk.unlock();
                std::vector<int> rcs;
                for (auto &pl : plan)
                    rcs.push_back(pl.small ? issue_small(s, pl.slot, pl.reqs, pl.off, pl.ws, pl.mats_b, pl.res_b)
                                           : issue_large(s, pl.slot, pl.reqs[0], pl.off));
                lk.lock();
                for (size_t k = 0; k < plan.size(); k++) {
                    if (rcs[k] == PERM_OK) continue;
                    Running &run = plan[k].small ? s->small_run[plan[k].slot] : s->large_run[plan[k].slot];
                    finish(s, run, rcs[k] < 0 ? rcs[k] : PERM_EDEVICE);
                }
            }
        }
        if (!progress) s->cv.wait_for(lk, std::chrono::microseconds(20));
    }
}

}  // namespace

extern "C" {

int perm_server_create(const perm_server_config_t *cfg, perm_server_t **out) {
    try {
        if (!cfg || !out) return set_error(PERM_EINVAL, "null pointer");
        if (!cfg->pool || cfg->pool_bytes == 0) return set_error(PERM_EINVAL, "empty pool");
        if (cfg->max_large_slots < 1 || cfg->max_large_slots > 16)
            return set_error(PERM_EINVAL, "max_large_slots = %d (1..16)", cfg->max_large_slots);
        if (cfg->queue_capacity < 1) return set_error(PERM_EINVAL, "queue_capacity < 1");
        if (cfg->small_n_max < 0 || cfg->small_n_max > PERM_BATCH_N_MAX)
            return set_error(PERM_EINVAL, "small_n_max = %d (0..%d)", cfg->small_n_max, PERM_BATCH_N_MAX);
        if (cfg->max_small_batch < 1 || cfg->max_small_batch > (1 << 20))
            return set_error(PERM_EINVAL, "max_small_batch = %d", cfg->max_small_batch);
        if (cfg->budget_bytes > cfg->pool_bytes) return set_error(PERM_EINVAL, "budget above the pool size");
        auto s = std::make_unique<perm_server>();
        s->cfg = *cfg;
        s->budget = cfg->budget_bytes ? cfg->budget_bytes : cfg->pool_bytes;
        s->arena.init(cfg->pool_bytes);
        if (hipGetDevice(&s->device) != hipSuccess) return set_error(PERM_EDEVICE, "no device");
        int rc = prepare_device(nullptr, nullptr);
        if (rc) return rc;
        const size_t small_elems = (size_t)cfg->max_small_batch * (PERM_BATCH_N_MAX * PERM_BATCH_N_MAX);
        for (int i = 0; i < kSmallSlots; i++) {
            if (hipStreamCreateWithFlags(&s->small_stream[i], hipStreamNonBlocking) != hipSuccess ||
                hipEventCreateWithFlags(&s->small_run[i].done, hipEventDisableTiming) != hipSuccess ||
                hipHostMalloc((void **)&s->pin_small_in[i], std::max<size_t>(small_elems, 1) * 16, 0) != hipSuccess ||
                hipHostMalloc((void **)&s->pin_small_out[i], (size_t)cfg->max_small_batch * 16, 0) != hipSuccess) {
                perm_server_destroy(s.release());
                return set_error(PERM_EDEVICE, "server stream/event/pinned buffer creation failed");
            }
        }
        s->large_stream.resize(cfg->max_large_slots, nullptr);
        s->large_run.resize(cfg->max_large_slots);
        s->pin_large_in.resize(cfg->max_large_slots, nullptr);
        s->pin_large_out.resize(cfg->max_large_slots, nullptr);
        for (int i = 0; i < cfg->max_large_slots; i++) {
            if (hipStreamCreateWithFlags(&s->large_stream[i], hipStreamNonBlocking) != hipSuccess ||
                hipEventCreateWithFlags(&s->large_run[i].done, hipEventDisableTiming) != hipSuccess ||
                hipHostMalloc((void **)&s->pin_large_in[i], PERM_N_MAX * PERM_N_MAX * 16, 0) != hipSuccess ||
                hipHostMalloc((void **)&s->pin_large_out[i], 16, 0) != hipSuccess) {
                perm_server_destroy(s.release());
                return set_error(PERM_EDEVICE, "server stream/event/pinned buffer creation failed");
            }
        }
        s->thr = std::thread(scheduler, s.get());
        *out = s.release();
        return PERM_OK;
    } catch (const std::exception &e) {
        return set_error(PERM_EDEVICE, "internal error: %s", e.what());
    }
}

int perm_server_submit(perm_server_t *s, perm_dtype_t dt, int n, const void *a, int64_t lda, uint64_t *ticket) {
    try {
        if (!s || !ticket || (n > 0 && !a)) return set_error(PERM_EINVAL, "null pointer");
        if (dt != PERM_COMPLEX128) return set_error(PERM_EINVAL, "the server takes complex128 requests");
        if (n < 0) return set_error(PERM_EINVAL, "n = %d < 0", n);
        if (n > PERM_N_MAX) return set_error(PERM_ERANGE, "n = %d > %d", n, PERM_N_MAX);
        if (n > 0 && lda < n) return set_error(PERM_EINVAL, "lda < n");
        auto q = std::make_unique<Request>();
        q->n = n;
        q->charge = footprint(n);
        q->a.resize((size_t)n * n);
        const perm_c128_t *src = (const perm_c128_t *)a;
        for (int i = 0; i < n; i++)
            std::memcpy(&q->a[(size_t)i * n], src + (int64_t)i * lda, (size_t)n * 16);
        std::lock_guard<std::mutex> lk(s->mu);
        if (s->stop) return set_error(PERM_ECANCELLED, "server is shutting down");
        if (q->charge > s->budget)
            return set_error(PERM_ENOMEM, "footprint %zu bytes above the budget %zu", q->charge, s->budget);
        if (s->queued >= (size_t)s->cfg.queue_capacity) return set_error(PERM_EAGAIN, "queue full");
        q->ticket = s->next_ticket++;
        q->t_submit = now_seconds();
        *ticket = q->ticket;
        Request *raw = q.get();
        s->all.emplace(q->ticket, std::move(q));
        if (n <= s->cfg.small_n_max) s->small_q.push_back(raw);
        else s->large_q.push_back(raw);
        s->queued++;
        s->cv.notify_one();
        return PERM_OK;
    } catch (const std::exception &e) {
        return set_error(PERM_EDEVICE, "internal error: %s", e.what());
    }
}

int perm_server_poll(perm_server_t *s, uint64_t ticket, void *result, perm_req_stats_t *stats) {
    if (!s || !result) return set_error(PERM_EINVAL, "null pointer");
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->all.find(ticket);
    if (it == s->all.end()) return set_error(PERM_ENOTFOUND, "unknown ticket %llu", (unsigned long long)ticket);
    Request *q = it->second.get();
    if (q->status == PERM_PENDING) return PERM_PENDING;
    *(perm_c128_t *)result = q->result;
    if (stats) {
        stats->t_submit = q->t_submit;
        stats->t_admit = q->t_admit;
        stats->t_start = q->t_start;
        stats->t_done = q->t_done;
        stats->n = q->n;
        stats->status = q->status;
    }
    const int st = q->status;
    s->all.erase(it);
    if (st != PERM_OK) return set_error(st, "request %llu failed", (unsigned long long)ticket);
    return PERM_OK;
}

int perm_server_destroy(perm_server_t *s) {
    if (!s) return set_error(PERM_EINVAL, "null pointer");
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stop = true;
        for (auto *q : s->small_q) q->status = PERM_ECANCELLED;
        for (auto *q : s->large_q) q->status = PERM_ECANCELLED;
        s->small_q.clear();
        s->large_q.clear();
        s->cv.notify_one();
    }
    if (s->thr.joinable()) s->thr.join();
    for (int i = 0; i < kSmallSlots; i++) {
        if (s->small_stream[i]) (void)hipStreamDestroy(s->small_stream[i]);
        if (s->small_run[i].done) (void)hipEventDestroy(s->small_run[i].done);
        if (s->pin_small_in[i]) (void)hipHostFree(s->pin_small_in[i]);
        if (s->pin_small_out[i]) (void)hipHostFree(s->pin_small_out[i]);
    }
    for (size_t i = 0; i < s->large_stream.size(); i++) {
        if (s->large_stream[i]) (void)hipStreamDestroy(s->large_stream[i]);
        if (s->large_run[i].done) (void)hipEventDestroy(s->large_run[i].done);
        if (s->pin_large_in[i]) (void)hipHostFree(s->pin_large_in[i]);
        if (s->pin_large_out[i]) (void)hipHostFree(s->pin_large_out[i]);
    }
    delete s;
    return PERM_OK;
}

}  // extern "C"
