// Serving: a request loop that admits copy requests within an HBM budget and
// runs them with continuous batching.
//
// Submitted requests are validated and queued.  An engine thread repeats:
//  1. finished launches (an event per launch) complete their requests and
//     return their bytes to the budget;
//  2. while a stream slot is free, queued requests are admitted in arrival
//     order as long as the bytes in flight (source plus destination blobs)
//     stay within the budget and no admitted range conflicts with a range in
//     flight; the admitted requests form one work table, uploaded from pinned
//     memory and run by the persistent batch kernel on that slot's stream.
// Requests that arrive while launches run join the next launch as soon as a
// slot and budget free up, and launches on different streams overlap.
#include <hip/hip_runtime_api.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <mutex>
#include <thread>

#include "batch.hpp"
#include "serve.hpp"

namespace llama {

namespace {

using Clock = std::chrono::steady_clock;

void check_hip(hipError_t e, const char* what)
{
    if (e != hipSuccess)
        fail(LLAMA_E_HIP, std::string(what) + ": " + hipGetErrorString(e));
}

struct Range {
    uint64_t lo, hi;
    bool write;
};

bool conflicts(const std::vector<Range>& a, const std::vector<Range>& b)
{
    for (const Range& x : a)
        for (const Range& y : b)
            if ((x.write || y.write) && x.lo < y.hi && y.lo < x.hi)
                return true;
    return false;
}

struct Pending {
    uint64_t ticket;
    Request rq;
    uint64_t bytes;
    std::vector<Range> ranges;
    Clock::time_point arrival;
};

// One launch in flight: its event, and (batched policy) its work table.
struct Slot {
    hipStream_t stream = nullptr; // one of the server's streams
    hipEvent_t done = nullptr;
    void* dev = nullptr;
    size_t dev_cap = 0;
    void* host = nullptr; // pinned
    size_t host_cap = 0;
    bool busy = false;
    std::vector<uint64_t> tickets;
    std::vector<Clock::time_point> arrivals;
    std::vector<Range> ranges;
    uint64_t bytes = 0;
};

struct Outcome {
    bool done = false;
    int status = LLAMA_OK;
    double latency = 0;
};

} // namespace

struct Server {
    llama_server_config cfg{};
    int device = 0;
    std::vector<hipStream_t> streams;
    std::vector<Slot> slots;
    std::mutex mu;
    std::condition_variable work_cv;  // engine waits for submissions
    std::condition_variable done_cv;  // waiters wait for completions
    std::deque<Pending> queue;
    std::map<uint64_t, Outcome> outcomes;
    uint64_t next_ticket = 1;
    uint64_t inflight_bytes = 0;
    bool stop = false;
    std::thread engine;
    std::string engine_error;
    // statistics
    uint64_t submitted = 0, completed = 0, failed = 0, launches = 0, bytes_done = 0, max_inflight_bytes = 0;
    uint64_t admitted_total = 0;
    std::vector<double> latencies;
    Clock::time_point first_arrival{}, last_completion{};
    bool any_arrival = false;

    void run();
    bool complete_finished(std::unique_lock<std::mutex>& lock);
    bool admit(std::unique_lock<std::mutex>& lock);
    void launch_slot(Slot& s, std::vector<Pending>& group);
};

namespace {

void ensure_capacity(Slot& s, size_t bytes)
{
    if (bytes > s.dev_cap) {
        if (s.dev)
            check_hip(hipFree(s.dev), "hipFree");
        s.dev = nullptr;
        size_t cap = std::max<size_t>(bytes, 1 << 16);
        check_hip(hipMalloc(&s.dev, cap), "hipMalloc(server table)");
        s.dev_cap = cap;
    }
    if (bytes > s.host_cap) {
        if (s.host)
            check_hip(hipHostFree(s.host), "hipHostFree");
        s.host = nullptr;
        size_t cap = std::max<size_t>(bytes, 1 << 16);
        check_hip(hipHostMalloc(&s.host, cap, hipHostMallocDefault), "hipHostMalloc(server table)");
        s.host_cap = cap;
    }
}

} // namespace

// Launches `group` on slot `s` according to the policy.
void Server::launch_slot(Slot& s, std::vector<Pending>& group)
{
    if (cfg.policy == LLAMA_SERVE_BATCHED) {
        BatchTable t;
        for (Pending& p : group)
            t.add(p.rq, cfg.threads, 0);
        if (t.units > 0) {
            const size_t bytes = t.bytes();
            ensure_capacity(s, bytes);
            BatchArgs args{};
            t.serialise((uint8_t*)s.host, uint64_t(uintptr_t(s.dev)), args);
            check_hip(hipMemcpyAsync(s.dev, s.host, bytes, hipMemcpyHostToDevice, s.stream), "hipMemcpyAsync(table)");
            const uint32_t wg = batch_wg_per_cu(t.lds_bytes, cfg.threads);
            const uint32_t grid =
                uint32_t(std::min<uint64_t>(std::max<uint64_t>(t.units, 1), uint64_t(device_cu_count()) * wg));
            launch_batch_args(args, grid, cfg.threads, t.lds_bytes, s.stream);
        }
    } else {
        llama_copy_options o{cfg.policy == LLAMA_SERVE_NAIVE ? uint32_t(LLAMA_PATH_NAIVE) : uint32_t(LLAMA_PATH_AUTO),
                             0, 0, 0, 0};
        for (Pending& p : group)
            launch(make_plan(p.rq, &o), s.stream);
    }
    check_hip(hipEventRecord(s.done, s.stream), "hipEventRecord");
}

bool Server::complete_finished(std::unique_lock<std::mutex>& lock)
{
    (void)lock;
    bool any = false;
    for (Slot& s : slots) {
        if (!s.busy)
            continue;
        hipError_t q = hipEventQuery(s.done);
        if (q == hipErrorNotReady)
            continue;
        const Clock::time_point now = Clock::now();
        const int status = q == hipSuccess ? LLAMA_OK : LLAMA_E_HIP;
        for (size_t k = 0; k < s.tickets.size(); k++) {
            Outcome& o = outcomes[s.tickets[k]];
            o.done = true;
            o.status = status;
            o.latency = std::chrono::duration<double>(now - s.arrivals[k]).count();
            if (status == LLAMA_OK) {
                completed++;
                latencies.push_back(o.latency);
            } else {
                failed++;
            }
        }
        if (status == LLAMA_OK)
            bytes_done += s.bytes;
        last_completion = now;
        inflight_bytes -= s.bytes;
        s.tickets.clear();
        s.arrivals.clear();
        s.ranges.clear();
        s.bytes = 0;
        s.busy = false;
        any = true;
    }
    if (any)
        done_cv.notify_all();
    return any;
}

bool Server::admit(std::unique_lock<std::mutex>& lock)
{
    bool any = false;
    for (Slot& s : slots) {
        if (s.busy || queue.empty())
            continue;
        std::vector<Pending> group;
        std::vector<Range> ranges;
        uint64_t bytes = 0;
        const uint32_t max_group = cfg.policy == LLAMA_SERVE_BATCHED ? cfg.max_batch : 1;
        while (!queue.empty() && group.size() < max_group) {
            Pending& p = queue.front();
            if (inflight_bytes + bytes + p.bytes > cfg.budget_bytes)
                break; // the budget is full: later requests wait (arrival order is kept)
            bool clash = conflicts(p.ranges, ranges);
            for (const Slot& o : slots)
                clash = clash || (o.busy && conflicts(p.ranges, o.ranges));
            if (clash)
                break;
            bytes += p.bytes;
            ranges.insert(ranges.end(), p.ranges.begin(), p.ranges.end());
            group.push_back(std::move(p));
            queue.pop_front();
        }
        if (group.empty())
            break;
        s.busy = true;
        s.bytes = bytes;
        s.ranges = std::move(ranges);
        for (const Pending& p : group) {
            s.tickets.push_back(p.ticket);
            s.arrivals.push_back(p.arrival);
        }
        inflight_bytes += bytes;
        max_inflight_bytes = std::max(max_inflight_bytes, inflight_bytes);
        launches++;
        admitted_total += group.size();
        // the launch itself runs without the lock (planning, upload)
        lock.unlock();
        int status = LLAMA_OK;
        try {
            launch_slot(s, group);
        } catch (const Error& e) {
            status = e.status;
        }
        lock.lock();
        if (status != LLAMA_OK) {
            // nothing of this group is on the GPU: fail its requests now
            for (uint64_t t : s.tickets) {
                outcomes[t] = Outcome{true, status, 0};
                failed++;
            }
            inflight_bytes -= s.bytes;
            s.tickets.clear();
            s.arrivals.clear();
            s.ranges.clear();
            s.bytes = 0;
            s.busy = false;
            done_cv.notify_all();
        }
        any = true;
    }
    return any;
}

void Server::run()
{
    (void)hipSetDevice(device);
    std::unique_lock<std::mutex> lock(mu);
    for (;;) {
        bool progress = complete_finished(lock);
        progress = admit(lock) || progress;
        bool busy = false;
        for (const Slot& s : slots)
            busy = busy || s.busy;
        if (stop && queue.empty() && !busy)
            break;
        if (!progress) {
            // launches in flight: poll their events soon; idle: sleep until a
            // request arrives
            if (busy)
                work_cv.wait_for(lock, std::chrono::microseconds(20));
            else
                work_cv.wait_for(lock, std::chrono::milliseconds(50));
        }
    }
}

Server* create_server(const llama_server_config* cfg)
{
    std::unique_ptr<Server> s(new Server());
    llama_server_config c{};
    if (cfg)
        c = *cfg;
    if (c.budget_bytes == 0)
        fail(LLAMA_E_INVALID_ARG, "budget_bytes must be positive");
    if (c.policy > LLAMA_SERVE_PER_REQUEST)
        fail(LLAMA_E_INVALID_ARG, "unknown serving policy");
    if (c.streams == 0)
        c.streams = c.policy == LLAMA_SERVE_NAIVE ? 1 : 2;
    if (c.streams > 16)
        fail(LLAMA_E_INVALID_ARG, "at most 16 streams");
    if (c.max_batch == 0)
        c.max_batch = 1024;
    if (c.queue_capacity == 0)
        c.queue_capacity = 1u << 20;
    if (c.threads == 0)
        c.threads = kDefaultThreads;
    if (c.threads % 64 != 0 || c.threads > 1024)
        fail(LLAMA_E_INVALID_ARG, "threads must be a multiple of 64 in 64..1024");
    s->cfg = c;
    check_hip(hipGetDevice(&s->device), "hipGetDevice");
    // batched: one launch per stream in flight, so that requests arriving
    // meanwhile gather into the next launch; one request per launch
    // otherwise, up to 256 launches queued back to back
    s->streams.assign(c.streams, nullptr);
    s->slots.resize(c.policy == LLAMA_SERVE_BATCHED ? c.streams : 256);
    try {
        for (hipStream_t& st : s->streams)
            check_hip(hipStreamCreateWithFlags(&st, hipStreamNonBlocking), "hipStreamCreate");
        for (size_t k = 0; k < s->slots.size(); k++) {
            s->slots[k].stream = s->streams[k % s->streams.size()];
            check_hip(hipEventCreateWithFlags(&s->slots[k].done, hipEventDisableTiming), "hipEventCreate");
        }
    } catch (...) {
        for (Slot& sl : s->slots)
            if (sl.done)
                hipEventDestroy(sl.done);
        for (hipStream_t st : s->streams)
            if (st)
                hipStreamDestroy(st);
        throw;
    }
    s->engine = std::thread([srv = s.get()] { srv->run(); });
    return s.release();
}

uint64_t server_submit(Server* s, const llama_copy_item* item)
{
    if (!item)
        fail(LLAMA_E_INVALID_ARG, "item is NULL");
    Pending p;
    p.rq = make_request(item->src, item->src_blobs, item->dst, item->dst_blobs, true);
    int dev = 0;
    check_hip(hipGetDevice(&dev), "hipGetDevice");
    if (dev != s->device)
        fail(LLAMA_E_INVALID_ARG, "request submitted from device " + std::to_string(dev) + " to a server on device " +
                                      std::to_string(s->device));
    if (s->cfg.policy != LLAMA_SERVE_NAIVE) {
        llama_copy_options o{LLAMA_PATH_AUTO, 0, s->cfg.threads, 0, 0};
        if (s->cfg.policy == LLAMA_SERVE_BATCHED && make_plan(p.rq, &o).path == LLAMA_PATH_NAIVE)
            fail(LLAMA_E_UNSUPPORTED, "the record does not fit the tiled kernel; copy it with llama_copy");
    }
    p.bytes = 0;
    for (size_t b = 0; b < p.rq.src_ptr.size(); b++) {
        p.bytes += p.rq.src.blob_size[b];
        p.ranges.push_back({p.rq.src_ptr[b], p.rq.src_ptr[b] + p.rq.src.blob_size[b], false});
    }
    for (size_t b = 0; b < p.rq.dst_ptr.size(); b++) {
        p.bytes += p.rq.dst.blob_size[b];
        p.ranges.push_back({p.rq.dst_ptr[b], p.rq.dst_ptr[b] + p.rq.dst.blob_size[b], true});
    }
    std::lock_guard<std::mutex> lock(s->mu);
    if (p.bytes > s->cfg.budget_bytes)
        fail(LLAMA_E_NO_BUDGET, "the request needs " + std::to_string(p.bytes) + " bytes, the budget is " +
                                    std::to_string(s->cfg.budget_bytes));
    if (s->stop)
        fail(LLAMA_E_INVALID_ARG, "the server is shutting down");
    if (s->queue.size() >= s->cfg.queue_capacity)
        fail(LLAMA_E_BUSY, "the request queue is full");
    p.ticket = s->next_ticket++;
    s->submitted++;
    p.arrival = Clock::now();
    if (!s->any_arrival) {
        s->first_arrival = p.arrival;
        s->any_arrival = true;
    }
    s->outcomes[p.ticket] = Outcome{};
    const uint64_t t = p.ticket;
    s->queue.push_back(std::move(p));
    s->work_cv.notify_one();
    return t;
}

bool server_poll(Server* s, uint64_t ticket, bool wait, int& status, double& latency)
{
    std::unique_lock<std::mutex> lock(s->mu);
    auto it = s->outcomes.find(ticket);
    if (it == s->outcomes.end())
        fail(LLAMA_E_INVALID_ARG, "unknown ticket " + std::to_string(ticket));
    if (wait)
        s->done_cv.wait(lock, [&] { return s->outcomes[ticket].done; });
    const Outcome& o = s->outcomes[ticket];
    if (!o.done)
        return false;
    status = o.status;
    latency = o.latency;
    return true;
}

void server_stats(Server* s, llama_server_stats& st)
{
    std::lock_guard<std::mutex> lock(s->mu);
    st.submitted = s->submitted;
    st.completed = s->completed;
    st.failed = s->failed;
    st.queued = s->queue.size();
    st.launches = s->launches;
    st.bytes_done = s->bytes_done;
    st.max_inflight_bytes = s->max_inflight_bytes;
    st.mean_batch = s->launches ? double(s->admitted_total) / double(s->launches) : 0;
    std::vector<double> l = s->latencies;
    std::sort(l.begin(), l.end());
    auto pct = [&](double q) {
        if (l.empty())
            return 0.0;
        size_t k = size_t(q * double(l.size() - 1) + 0.5);
        return l[std::min(k, l.size() - 1)];
    };
    st.p50_latency = pct(0.50);
    st.p99_latency = pct(0.99);
    st.max_latency = l.empty() ? 0 : l.back();
    st.window = s->any_arrival && s->completed
                    ? std::chrono::duration<double>(s->last_completion - s->first_arrival).count()
                    : 0;
}

void server_reset_stats(Server* s)
{
    std::lock_guard<std::mutex> lock(s->mu);
    s->submitted = s->completed = s->failed = s->launches = s->bytes_done = s->max_inflight_bytes = 0;
    s->admitted_total = 0;
    s->latencies.clear();
    s->any_arrival = false;
}

void destroy_server(Server* s)
{
    if (!s)
        return;
    {
        std::lock_guard<std::mutex> lock(s->mu);
        s->stop = true;
    }
    s->work_cv.notify_all();
    if (s->engine.joinable())
        s->engine.join();
    (void)hipSetDevice(s->device);
    for (hipStream_t st : s->streams)
        (void)hipStreamSynchronize(st);
    for (Slot& sl : s->slots) {
        if (sl.dev)
            (void)hipFree(sl.dev);
        if (sl.host)
            (void)hipHostFree(sl.host);
        (void)hipEventDestroy(sl.done);
    }
    for (hipStream_t st : s->streams)
        (void)hipStreamDestroy(st);
    (void)hipGetLastError();
    delete s;
}

} // namespace llama
