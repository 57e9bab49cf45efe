// Serving loop of librsaw (declared in include/rsaw.h): requests (one
// ensemble each) are queued by rsaw_server_submit, a scheduler thread forms
// batches from the queue head and launches each with rsaw_gen_batch on one
// of S streams, and a completion thread per stream waits for the batch's
// event, copies the summaries out and retires the tickets.
//
// Admission by device memory: each stream owns a device workspace of
// bytes_per_stream (capped at creation so that all of them fit in 90 % of
// the device's free memory), bound with rsaw_set_workspace, and a pinned
// staging buffer sized for max_batch requests, both allocated once at
// creation: serving allocates and frees nothing.  A batch takes requests
// while the workspace bytes they need (the layout of rsaw_workspace_size
// plus their descriptor-table entries) fit in the stream's workspace and
// the batch holds at most max_batch requests.  A new batch starts on any
// free stream while others run, so short requests arriving during a long
// batch do not wait for it.
//
// Size classes: a request whose estimated service time alone exceeds
// large_ms is "large".  At most one large request is in flight at a time
// (and a batch holds at most one): large requests run one after another in
// arrival order, each sharing the GPU only with batches of small requests,
// which skip past queued large ones.  Two large requests run side by side
// would each take about twice as long, so the tail latency is set by
// serving them in series, while the small ones keep the concurrency.
// Every result is that of a stand-alone rsaw_gen_chains call (batched
// growth and reduction are bit-identical to single calls).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <mutex>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "rsaw.h"
#include "rsaw_reduce.hpp"

namespace rsaw {
rsaw_status check_config(const rsaw_config *cfg); // the checks of rsaw_gen_chains
} // namespace rsaw

namespace {

using Clock = std::chrono::steady_clock;

struct Ticket {
    rsaw_config cfg;
    Clock::time_point submitted, started, done_at;
    bool done = false;
    rsaw_status status = RSAW_OK;
    rsaw_summary summary;
};

struct Slot {
    bool large = false;             // the batch holds a large request
    hipStream_t stream = nullptr;
    void *ws = nullptr;             // the stream's device workspace (budget bytes)
    hipEvent_t done = nullptr;
    rsaw_summary *d_summ = nullptr; // max_batch summaries (device)
    rsaw_summary *h_summ = nullptr; // pinned copy
    std::vector<uint64_t> tickets;  // the batch assigned to the slot (empty: free)
    bool launched = false;          // its launch and completion event are enqueued
    std::thread waiter;
    std::condition_variable cv;     // a batch was launched on this slot
};

// Device workspace bytes a request holds while its batch runs.
size_t request_bytes(const rsaw_config &c) { return rsaw::batch_entry_bytes(&c); }

// Estimated growth time of a request alone on the device, in ms, for the
// size classes only (it never affects a result).  A chain's scan work grows
// as N^2; the constants are per-chain times at N = 64 on one MI355X: 0.2 ns
// (lattice, registers), 0.65 ns (26-neighbour lattice), 1 ns per trial
// (hard spheres), and 3x on the lattices beyond N = 64 (group kernels).
double estimate_ms(const rsaw_config &c)
{
    const double n = c.n_monomers / 64.0;
    double ns = c.geometry == RSAW_REAL_HS ? 1.0 * c.k_trials : (c.geometry == RSAW_LATTICE_26 ? 0.65 : 0.2);
    if (c.geometry != RSAW_REAL_HS && c.n_monomers > 64) ns *= 3.0;
    return (double)c.n_chains * ns * n * n * 1e-6;
}

} // namespace

struct rsaw_server {
    rsaw_server_params p;
    int device = 0;
    std::mutex mu;
    std::condition_variable cv_sched; // new request or a slot became free
    std::condition_variable cv_done;  // a ticket completed
    std::deque<uint64_t> queue;
    std::unordered_map<uint64_t, Ticket> tickets;
    uint64_t next_ticket = 1;
    bool stopping = false;
    std::vector<Slot> slots;
    std::thread scheduler;
    std::string error;
    size_t budget = 0; // workspace bytes of each stream

    bool is_large(const rsaw_config &c) const { return p.large_ms >= 0.0 && estimate_ms(c) > large_ms(); }
    double large_ms() const { return p.large_ms > 0.0 ? p.large_ms : 2.0; }

    void fail_batch(Slot &sl, rsaw_status st)
    {
        for (uint64_t t : sl.tickets) {
            Ticket &tk = tickets[t];
            tk.status = st;
            tk.done = true;
            tk.done_at = Clock::now();
        }
        sl.tickets.clear();
    }

    void schedule_loop()
    {
        hipSetDevice(device);
        std::unique_lock<std::mutex> lk(mu);
        while (true) {
            cv_sched.wait(lk, [&] {
                if (stopping) return true;
                if (queue.empty()) return false;
                bool free = false, large_busy = false;
                for (Slot &sl : slots) {
                    free = free || sl.tickets.empty();
                    large_busy = large_busy || (!sl.tickets.empty() && sl.large);
                }
                if (!free) return false;
                if (!large_busy) return true;
                for (uint64_t t : queue)
                    if (!is_large(tickets[t].cfg)) return true; // a small request can start
                return false;
            });
            if (stopping && queue.empty()) break;
            if (stopping) {
                // drain: fail what never started
                for (uint64_t t : queue) {
                    Ticket &tk = tickets[t];
                    tk.status = RSAW_E_DEVICE;
                    tk.done = true;
                    tk.done_at = Clock::now();
                }
                queue.clear();
                cv_done.notify_all();
                break;
            }
            Slot *free_slot = nullptr;
            for (Slot &sl : slots)
                if (sl.tickets.empty()) {
                    free_slot = &sl;
                    break;
                }
            if (!free_slot) continue;
            // admission in arrival order; a large request only while no
            // other large one is in flight or in this batch (it stays queued
            // in order otherwise)
            bool large_busy = false;
            for (Slot &sl : slots) large_busy = large_busy || (!sl.tickets.empty() && sl.large);
            std::vector<uint64_t> batch;
            size_t bytes = 0;
            bool batch_large = false;
            for (auto it = queue.begin(); it != queue.end() && (int)batch.size() < p.max_batch;) {
                const Ticket &tk = tickets[*it];
                const bool large = is_large(tk.cfg);
                if (large && (large_busy || batch_large)) {
                    ++it;
                    continue;
                }
                const size_t need = request_bytes(tk.cfg);
                if (bytes + need + rsaw::kBatchFixedBytes > budget) break;
                bytes += need;
                batch_large = batch_large || large;
                batch.push_back(*it);
                it = queue.erase(it);
            }
            if (batch.empty()) continue;
            free_slot->large = batch_large;
            std::vector<rsaw_config> cfgs;
            const Clock::time_point now = Clock::now();
            for (uint64_t t : batch) {
                Ticket &tk = tickets[t];
                tk.started = now;
                cfgs.push_back(tk.cfg);
            }
            free_slot->tickets = batch;
            lk.unlock();
            // the launch itself runs outside the lock; only this thread launches
            rsaw_status st = rsaw_gen_batch(cfgs.data(), nullptr, (int32_t)cfgs.size(), free_slot->d_summ,
                                            nullptr, nullptr, free_slot->stream);
            hipError_t e = hipSuccess;
            if (st == RSAW_OK)
                e = hipMemcpyAsync(free_slot->h_summ, free_slot->d_summ, cfgs.size() * sizeof(rsaw_summary),
                                   hipMemcpyDeviceToHost, free_slot->stream);
            if (st == RSAW_OK && e == hipSuccess) e = hipEventRecord(free_slot->done, free_slot->stream);
            lk.lock();
            if (st != RSAW_OK || e != hipSuccess) {
                error = st != RSAW_OK ? rsaw_last_error() : hipGetErrorString(e);
                fail_batch(*free_slot, st != RSAW_OK ? st : RSAW_E_DEVICE);
                cv_done.notify_all();
                continue;
            }
            free_slot->launched = true;
            free_slot->cv.notify_one();
        }
    }

    void wait_loop(Slot *sl)
    {
        hipSetDevice(device);
        std::unique_lock<std::mutex> lk(mu);
        while (true) {
            sl->cv.wait(lk, [&] { return sl->launched || (stopping && sl->tickets.empty()); });
            if (!sl->launched) break;
            lk.unlock();
            hipError_t e = hipEventSynchronize(sl->done);
            const Clock::time_point now = Clock::now();
            lk.lock();
            for (size_t i = 0; i < sl->tickets.size(); ++i) {
                Ticket &tk = tickets[sl->tickets[i]];
                tk.done_at = now;
                tk.done = true;
                if (e != hipSuccess) {
                    tk.status = RSAW_E_DEVICE;
                } else {
                    tk.summary = sl->h_summ[i];
                    tk.status = (rsaw_status)tk.summary.status;
                }
            }
            sl->tickets.clear();
            sl->launched = false;
            cv_done.notify_all();
            cv_sched.notify_one();
        }
    }
};

extern "C" {

rsaw_status rsaw_server_create(const rsaw_server_params *params, int32_t device, rsaw_server **out)
{
    if (!out) return RSAW_E_INVALID;
    *out = nullptr;
    rsaw_server_params p{};
    p.bytes_per_stream = (size_t)2 << 30;
    p.max_batch = 256;
    p.streams = 2;
    p.large_ms = 0.0;
    if (params) p = *params;
    if (p.streams < 1 || p.streams > 16 || p.max_batch < 1 || p.max_batch > 4096 || p.bytes_per_stream == 0)
        return RSAW_E_INVALID;
    int count = 0;
    if (hipGetDeviceCount(&count) != hipSuccess || device < 0 || device >= count) return RSAW_E_DEVICE;
    int prev = 0;
    (void)hipGetDevice(&prev);
    if (hipSetDevice(device) != hipSuccess) return RSAW_E_DEVICE;
    rsaw_server *s = new rsaw_server();
    s->p = p;
    s->device = device;
    s->slots = std::vector<Slot>(p.streams);
    // each stream's workspace: bytes_per_stream, within 90 % of free memory
    size_t free_b = 0, total_b = 0;
    bool ok = hipMemGetInfo(&free_b, &total_b) == hipSuccess;
    s->budget = (size_t)p.bytes_per_stream;
    if (ok) s->budget = std::min(s->budget, (size_t)((double)free_b * 0.9 / p.streams));
    s->budget &= ~(size_t)255;
    for (Slot &sl : s->slots) {
        ok = ok && hipStreamCreateWithFlags(&sl.stream, hipStreamNonBlocking) == hipSuccess;
        ok = ok && hipEventCreateWithFlags(&sl.done, hipEventDisableTiming) == hipSuccess;
        ok = ok && hipMalloc(&sl.d_summ, (size_t)p.max_batch * sizeof(rsaw_summary)) == hipSuccess;
        ok = ok && hipHostMalloc(&sl.h_summ, (size_t)p.max_batch * sizeof(rsaw_summary), hipHostMallocDefault) ==
                       hipSuccess;
        ok = ok && hipMalloc(&sl.ws, s->budget) == hipSuccess;
        ok = ok && rsaw_set_workspace(sl.ws, s->budget, sl.stream) == RSAW_OK;
        ok = ok && rsaw::reserve_staging(sl.stream, rsaw::batch_stage_bytes(p.max_batch)) == RSAW_OK;
        if (!ok) break;
    }
    if (!ok) {
        (void)hipGetLastError(); // the failed call must not fail the thread's next launch check
        for (Slot &sl : s->slots) {
            if (sl.stream) {
                (void)rsaw_set_workspace(nullptr, 0, sl.stream);
                (void)rsaw::release_stream(sl.stream);
            }
            if (sl.ws) (void)hipFree(sl.ws);
            if (sl.d_summ) (void)hipFree(sl.d_summ);
            if (sl.h_summ) (void)hipHostFree(sl.h_summ);
            if (sl.done) (void)hipEventDestroy(sl.done);
            if (sl.stream) (void)hipStreamDestroy(sl.stream);
        }
        (void)hipSetDevice(prev);
        delete s;
        return RSAW_E_NOMEM;
    }
    (void)hipSetDevice(prev);
    for (Slot &sl : s->slots) sl.waiter = std::thread(&rsaw_server::wait_loop, s, &sl);
    s->scheduler = std::thread(&rsaw_server::schedule_loop, s);
    *out = s;
    return RSAW_OK;
}

rsaw_status rsaw_server_submit(rsaw_server *s, const rsaw_config *cfg, uint64_t *ticket)
{
    if (!s || !cfg || !ticket) return RSAW_E_INVALID;
    rsaw_status st = rsaw::check_config(cfg);
    if (st != RSAW_OK) return st;
    if (request_bytes(*cfg) + rsaw::kBatchFixedBytes > s->budget) return RSAW_E_NOMEM;
    std::lock_guard<std::mutex> lk(s->mu);
    if (s->stopping) return RSAW_E_INVALID;
    const uint64_t t = s->next_ticket++;
    Ticket &tk = s->tickets[t];
    tk.cfg = *cfg;
    tk.submitted = Clock::now();
    std::memset(&tk.summary, 0, sizeof(tk.summary));
    s->queue.push_back(t);
    *ticket = t;
    s->cv_sched.notify_one();
    return RSAW_OK;
}

static rsaw_status take(rsaw_server *s, uint64_t ticket, rsaw_summary *h_summary, double *times_us)
{
    Ticket &tk = s->tickets[ticket];
    if (h_summary) *h_summary = tk.summary;
    if (times_us) {
        times_us[0] = std::chrono::duration<double, std::micro>(tk.started - tk.submitted).count();
        times_us[1] = std::chrono::duration<double, std::micro>(tk.done_at - tk.submitted).count();
    }
    const rsaw_status st = tk.status;
    s->tickets.erase(ticket);
    return st;
}

rsaw_status rsaw_server_poll(rsaw_server *s, uint64_t ticket, int32_t *done, rsaw_summary *h_summary,
                             double *times_us)
{
    if (!s || !done) return RSAW_E_INVALID;
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->tickets.find(ticket);
    if (it == s->tickets.end()) return RSAW_E_INVALID;
    *done = it->second.done ? 1 : 0;
    if (!it->second.done) return RSAW_OK;
    return take(s, ticket, h_summary, times_us);
}

rsaw_status rsaw_server_wait(rsaw_server *s, uint64_t ticket, rsaw_summary *h_summary, double *times_us)
{
    if (!s) return RSAW_E_INVALID;
    std::unique_lock<std::mutex> lk(s->mu);
    auto it = s->tickets.find(ticket);
    if (it == s->tickets.end()) return RSAW_E_INVALID;
    s->cv_done.wait(lk, [&] { return s->tickets[ticket].done; });
    return take(s, ticket, h_summary, times_us);
}

void rsaw_server_destroy(rsaw_server *s)
{
    if (!s) return;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stopping = true;
    }
    s->cv_sched.notify_all();
    if (s->scheduler.joinable()) s->scheduler.join();
    for (Slot &sl : s->slots) {
        {
            std::lock_guard<std::mutex> lk(s->mu);
        }
        sl.cv.notify_all();
        if (sl.waiter.joinable()) sl.waiter.join();
    }
    int prev = 0;
    (void)hipGetDevice(&prev);
    (void)hipSetDevice(s->device);
    for (Slot &sl : s->slots) {
        (void)hipStreamSynchronize(sl.stream);
        (void)rsaw_set_workspace(nullptr, 0, sl.stream);
        (void)rsaw::release_stream(sl.stream);
        (void)hipFree(sl.ws);
        (void)hipFree(sl.d_summ);
        (void)hipHostFree(sl.h_summ);
        (void)hipEventDestroy(sl.done);
        (void)hipStreamDestroy(sl.stream);
    }
    (void)hipSetDevice(prev);
    delete s;
}

} // extern "C"
