// Serving: a request loop that admits copy requests within an HBM budget and
// runs them with continuous batching.
//
// Submitted requests are validated and queued.  An engine thread repeats:
//  1. finished launches (an event per launch) complete their requests and
//     return their bytes to the budget;
//  2. while a launch slot is free, queued requests are admitted in arrival
//     order as long as the bytes in flight (source plus destination blobs)
//     stay within the budget and no admitted range conflicts with a range in
//     flight; a group closes once its bytes reach group_bytes; the admitted
//     requests form one work table, uploaded from pinned memory and run by
//     the batch kernels on that slot's stream, one launch per tile mode (a
//     group of one request is launched as that request's own copy).
// Each stream holds up to `depth` launches, so the next launches wait on the
// device while one runs, and launches on different streams overlap.  Batched:
// requests never wait to be batched.  A request of group_bytes or more runs
// alone (as its own copy, with its tuned plan); smaller requests queued at
// the same time share one launch of the batch kernel, up to group_bytes, so
// that many small requests do not pay one launch each.  With stream_bytes
// set, no launch joins a stream holding that many bytes, and arrivals gather
// in the queue meanwhile (fewer, larger launches at the cost of latency).
#include <hip/hip_runtime_api.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <memory>
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

// A request's descriptors and blob arrays copied at submit, for an executor
// (the caller's own are borrowed only for the duration of the call).
struct OwnedItem {
    std::vector<llama_field> src_nodes, dst_nodes;
    llama_record_desc src_record{}, dst_record{};
    llama_mapping_desc src{}, dst{};
    std::vector<llama_blob> src_blobs, dst_blobs;
    llama_copy_item item{};
};

std::unique_ptr<OwnedItem> own_item(const llama_copy_item* it, const Request& rq)
{
    std::unique_ptr<OwnedItem> o(new OwnedItem());
    o->src_nodes.assign(it->src->record->nodes, it->src->record->nodes + it->src->record->num_nodes);
    o->dst_nodes.assign(it->dst->record->nodes, it->dst->record->nodes + it->dst->record->num_nodes);
    o->src_record = llama_record_desc{uint32_t(o->src_nodes.size()), o->src_nodes.data()};
    o->dst_record = llama_record_desc{uint32_t(o->dst_nodes.size()), o->dst_nodes.data()};
    o->src = *it->src;
    o->dst = *it->dst;
    o->src.record = &o->src_record;
    o->dst.record = &o->dst_record;
    o->src_blobs.assign(it->src_blobs, it->src_blobs + rq.src_ptr.size());
    o->dst_blobs.assign(it->dst_blobs, it->dst_blobs + rq.dst_ptr.size());
    o->item = llama_copy_item{&o->src, o->src_blobs.data(), &o->dst, o->dst_blobs.data()};
    return o;
}

struct Pending {
    uint64_t ticket;
    Request rq;
    std::vector<SubCopy> parts; // a request with a Split side: its part copies, else empty
    uint64_t bytes;
    std::vector<Range> ranges;
    Clock::time_point arrival;
    std::unique_ptr<OwnedItem> owned; // with an executor only
};

// One launch in flight: its event, and (batched policy) its work table.
struct Slot {
    hipStream_t stream = nullptr; // one of the server's streams
    uint32_t stream_index = 0;
    hipEvent_t done = nullptr;
    hipEvent_t uploaded = nullptr; // BATCHED: the work table's upload has finished
    void* dev = nullptr;
    size_t dev_cap = 0;
    void* host = nullptr; // pinned
    size_t host_cap = 0;
    bool own_dev = false, own_host = false; // false: a piece of the server's preallocated tables
    bool busy = false;
    uint64_t launch_id = 0;                      // with an executor
    std::vector<std::unique_ptr<OwnedItem>> owned; // with an executor: the launch's items
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
    bool has_exec = false; // runs on `exec` instead of HIP
    llama_executor exec{};
    uint64_t launch_counter = 0;
    std::vector<hipStream_t> streams;
    hipStream_t upload = nullptr; // BATCHED: work-table uploads, off the launch streams
    std::vector<Slot> slots;
    // per stream: busy slots in launch order (they finish in that order),
    // free slots, and the bytes of the launches in flight
    void* table_dev = nullptr;  // BATCHED: kSlotTableBytes of device memory per slot
    void* table_host = nullptr; // and as much pinned host memory
    std::vector<std::deque<uint32_t>> order;
    std::vector<std::vector<uint32_t>> free_slots;
    std::vector<uint64_t> stream_bytes;
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

// Work-table memory preallocated per slot of a batched server, so that
// launches allocate nothing (a table of about 400 items fits); a larger
// table gets memory of its own, kept by the slot.
constexpr size_t kSlotTableBytes = size_t(256) << 10;

void ensure_capacity(Slot& s, size_t bytes)
{
    if (bytes > s.dev_cap) {
        if (s.dev && s.own_dev)
            check_hip(hipFree(s.dev), "hipFree");
        s.dev = nullptr;
        s.dev_cap = 0;
        s.own_dev = true;
        check_hip(hipMalloc(&s.dev, bytes), "hipMalloc(server table)");
        s.dev_cap = bytes;
    }
    if (bytes > s.host_cap) {
        if (s.host && s.own_host)
            check_hip(hipHostFree(s.host), "hipHostFree");
        s.host = nullptr;
        s.host_cap = 0;
        s.own_host = true;
        check_hip(hipHostMalloc(&s.host, bytes, hipHostMallocDefault), "hipHostMalloc(server table)");
        s.host_cap = bytes;
    }
}

} // namespace

// Launches `group` on slot `s` according to the policy.
void Server::launch_slot(Slot& s, std::vector<Pending>& group)
{
    if (has_exec) {
        std::vector<llama_copy_item> items;
        for (const Pending& p : group)
            items.push_back(p.owned->item);
        s.launch_id = ++launch_counter;
        const int st = exec.start(exec.context, s.launch_id, items.size(), items.data());
        if (st != LLAMA_OK)
            fail(st < 0 ? st : LLAMA_E_INVALID_ARG, "the executor did not start launch " + std::to_string(s.launch_id));
        for (Pending& p : group)
            s.owned.push_back(std::move(p.owned));
        return;
    }
    if (cfg.policy == LLAMA_SERVE_BATCHED && group.size() == 1) {
        // a group of one is the request's own launch (its tuned plan, no
        // work table to upload); a Split request's part copies in order
        if (group[0].parts.empty())
            launch(make_plan(group[0].rq, nullptr), s.stream);
        for (const SubCopy& c : group[0].parts)
            launch(make_plan(c.rq, nullptr), s.stream);
    } else if (cfg.policy == LLAMA_SERVE_BATCHED) {
        BatchTable t;
        for (Pending& p : group) {
            if (p.parts.empty())
                t.add(p.rq, cfg.threads, 0);
            for (const SubCopy& c : p.parts) // disjoint bytes: side by side
                t.add(c.rq, cfg.threads, 0);
        }
        if (t.units > 0) {
            // one launch per tile mode, each mode's own compiled body, like a
            // batch (the default of llama_batch_create)
            const std::vector<BatchRange> ranges = kBatchByModeDefault ? t.sort_by_mode() : std::vector<BatchRange>{};
            const size_t bytes = t.bytes();
            ensure_capacity(s, bytes);
            BatchArgs args{};
            t.serialise((uint8_t*)s.host, uint64_t(uintptr_t(s.dev)), args);
            // the upload runs on its own stream, so that it overlaps the
            // launches already queued on the slot's stream; the launch waits
            // for it (the slot's table is reused only after its launch ends)
            check_hip(hipMemcpyAsync(s.dev, s.host, bytes, hipMemcpyHostToDevice, upload), "hipMemcpyAsync(table)");
            check_hip(hipEventRecord(s.uploaded, upload), "hipEventRecord(upload)");
            check_hip(hipStreamWaitEvent(s.stream, s.uploaded, 0), "hipStreamWaitEvent(upload)");
            if (!ranges.empty()) {
                launch_batch_ranges(args, ranges, cfg.threads, s.stream);
            } else {
                const uint32_t w = batch_per_unit(t) ? 0 : batch_wg_per_cu(t.lds_bytes, cfg.threads);
                launch_batch_args(args, batch_grid(t.units, w), cfg.threads, t.lds_bytes, w != 0, s.stream);
            }
        }
    } else {
        llama_copy_options o{cfg.policy == LLAMA_SERVE_NAIVE ? uint32_t(LLAMA_PATH_NAIVE) : uint32_t(LLAMA_PATH_AUTO),
                             0, 0, 0, 0};
        llama_copy_options naive{uint32_t(LLAMA_PATH_NAIVE), 0, 0, 0, 0};
        for (Pending& p : group) {
            if (p.parts.empty())
                launch(make_plan(p.rq, &o), s.stream);
            for (const SubCopy& c : p.parts)
                launch(make_plan(c.rq, c.naive ? &naive : &o), s.stream);
        }
    }
    check_hip(hipEventRecord(s.done, s.stream), "hipEventRecord");
}

bool Server::complete_finished(std::unique_lock<std::mutex>& lock)
{
    (void)lock;
    bool any = false;
    for (size_t st = 0; st < streams.size(); st++) {
        for (size_t pos = 0; pos < order[st].size();) {
            const uint32_t idx = order[st][pos];
            Slot& s = slots[idx];
            int status = LLAMA_OK;
            if (has_exec) {
                // an executor may finish launches in any order
                const int q = exec.poll(exec.context, s.launch_id);
                if (q == 0) {
                    pos++;
                    continue;
                }
                status = q > 0 ? LLAMA_OK : q;
            } else {
                const hipError_t q = hipEventQuery(s.done);
                if (q == hipErrorNotReady)
                    break; // later launches of this stream are not done either
                status = q == hipSuccess ? LLAMA_OK : LLAMA_E_HIP;
            }
            const Clock::time_point now = Clock::now();
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
            stream_bytes[st] -= s.bytes;
            s.tickets.clear();
            s.arrivals.clear();
            s.ranges.clear();
            s.owned.clear();
            s.bytes = 0;
            s.busy = false;
            order[st].erase(order[st].begin() + pos);
            free_slots[st].push_back(idx);
            any = true;
        }
    }
    if (any)
        done_cv.notify_all();
    return any;
}

bool Server::admit(std::unique_lock<std::mutex>& lock)
{
    bool any = false;
    while (!queue.empty()) {
        // the stream with the fewest bytes in flight among those with a free slot
        size_t st = streams.size();
        for (size_t k = 0; k < streams.size(); k++)
            if (!free_slots[k].empty() && (st == streams.size() || stream_bytes[k] < stream_bytes[st]))
                st = k;
        if (st == streams.size())
            break;
        // batched: while every stream holds enough work, requests gather in
        // the queue and leave later as one launch
        if (cfg.policy == LLAMA_SERVE_BATCHED && stream_bytes[st] >= cfg.stream_bytes)
            break;
        std::vector<Pending> group;
        std::vector<Range> ranges;
        uint64_t bytes = 0;
        const uint32_t max_group = cfg.policy == LLAMA_SERVE_BATCHED ? cfg.max_batch : 1;
        while (!queue.empty() && group.size() < max_group && bytes < cfg.group_bytes) {
            Pending& p = queue.front();
            if (!group.empty() && p.bytes >= cfg.group_bytes)
                break; // a large request runs alone, in the next launch
            if (inflight_bytes + bytes + p.bytes > cfg.budget_bytes)
                break; // the budget is full: later requests wait (arrival order is kept)
            bool clash = conflicts(p.ranges, ranges);
            for (size_t k = 0; k < streams.size() && !clash; k++)
                for (uint32_t b : order[k])
                    if (conflicts(p.ranges, slots[b].ranges)) {
                        clash = true;
                        break;
                    }
            if (clash)
                break;
            bytes += p.bytes;
            ranges.insert(ranges.end(), p.ranges.begin(), p.ranges.end());
            group.push_back(std::move(p));
            queue.pop_front();
        }
        if (group.empty())
            break;
        const uint32_t idx = free_slots[st].back();
        free_slots[st].pop_back();
        Slot& s = slots[idx];
        s.busy = true;
        s.bytes = bytes;
        s.ranges = std::move(ranges);
        for (const Pending& p : group) {
            s.tickets.push_back(p.ticket);
            s.arrivals.push_back(p.arrival);
        }
        order[st].push_back(idx);
        stream_bytes[st] += bytes;
        inflight_bytes += bytes;
        max_inflight_bytes = std::max(max_inflight_bytes, inflight_bytes);
        launches++;
        admitted_total += group.size();
        // the launch itself runs without the lock (planning, upload); only
        // this thread changes the slots, so `idx` is still last in order[st]
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
            stream_bytes[st] -= s.bytes;
            s.tickets.clear();
            s.arrivals.clear();
            s.ranges.clear();
            s.owned.clear();
            s.bytes = 0;
            s.busy = false;
            order[st].pop_back();
            free_slots[st].push_back(idx);
            done_cv.notify_all();
        }
        any = true;
    }
    return any;
}

void Server::run()
{
    if (!has_exec)
        (void)hipSetDevice(device);
    std::unique_lock<std::mutex> lock(mu);
    for (;;) {
        bool progress = complete_finished(lock);
        progress = admit(lock) || progress;
        bool busy = false;
        for (const auto& o : order)
            busy = busy || !o.empty();
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

Server* create_server(const llama_server_config* cfg, const llama_executor* exec)
{
    std::unique_ptr<Server> s(new Server());
    if (exec) {
        if (!exec->start || !exec->poll)
            fail(LLAMA_E_INVALID_ARG, "the executor needs both start and poll");
        s->has_exec = true;
        s->exec = *exec;
    }
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
    if (c.depth == 0)
        c.depth = c.policy == LLAMA_SERVE_BATCHED ? 64 : c.policy == LLAMA_SERVE_PER_REQUEST ? 128 : 256;
    if (c.depth > 1024)
        fail(LLAMA_E_INVALID_ARG, "at most 1024 launches in flight per stream");
    if (c.group_bytes == 0)
        c.group_bytes = uint64_t(8) << 20;
    if (c.stream_bytes == 0)
        c.stream_bytes = ~uint64_t(0);
    if (c.max_batch == 0)
        c.max_batch = 1024;
    if (c.queue_capacity == 0)
        c.queue_capacity = 1u << 20;
    if (c.threads == 0)
        c.threads = kDefaultThreads;
    if (c.threads % 64 != 0 || c.threads > 1024)
        fail(LLAMA_E_INVALID_ARG, "threads must be a multiple of 64 in 64..1024");
    s->cfg = c;
    // `depth` launches in flight per stream, slots taking the streams in turn
    s->streams.assign(c.streams, nullptr);
    s->slots.resize(size_t(c.streams) * c.depth);
    s->order.resize(c.streams);
    s->free_slots.resize(c.streams);
    s->stream_bytes.assign(c.streams, 0);
    for (size_t k = 0; k < s->slots.size(); k++)
        s->slots[k].stream_index = uint32_t(k % s->streams.size());
    for (size_t k = s->slots.size(); k-- > 0;)
        s->free_slots[s->slots[k].stream_index].push_back(uint32_t(k));
    if (s->has_exec) {
        s->device = -1; // no GPU: the executor runs the launches
        s->engine = std::thread([srv = s.get()] { srv->run(); });
        return s.release();
    }
    check_hip(hipGetDevice(&s->device), "hipGetDevice");
    try {
        for (hipStream_t& st : s->streams)
            check_hip(hipStreamCreateWithFlags(&st, hipStreamNonBlocking), "hipStreamCreate");
        for (Slot& sl : s->slots) {
            sl.stream = s->streams[sl.stream_index];
            check_hip(hipEventCreateWithFlags(&sl.done, hipEventDisableTiming), "hipEventCreate");
        }
        if (c.policy == LLAMA_SERVE_BATCHED) {
            check_hip(hipStreamCreateWithFlags(&s->upload, hipStreamNonBlocking), "hipStreamCreate(upload)");
            for (Slot& sl : s->slots)
                check_hip(hipEventCreateWithFlags(&sl.uploaded, hipEventDisableTiming), "hipEventCreate");
            const size_t n = s->slots.size();
            check_hip(hipMalloc(&s->table_dev, n * kSlotTableBytes), "hipMalloc(server tables)");
            check_hip(hipHostMalloc(&s->table_host, n * kSlotTableBytes, hipHostMallocDefault),
                      "hipHostMalloc(server tables)");
            for (size_t k = 0; k < n; k++) {
                s->slots[k].dev = (uint8_t*)s->table_dev + k * kSlotTableBytes;
                s->slots[k].host = (uint8_t*)s->table_host + k * kSlotTableBytes;
                s->slots[k].dev_cap = s->slots[k].host_cap = kSlotTableBytes;
            }
        }
    } catch (...) {
        for (Slot& sl : s->slots) {
            if (sl.done)
                hipEventDestroy(sl.done);
            if (sl.uploaded)
                hipEventDestroy(sl.uploaded);
        }
        if (s->upload)
            hipStreamDestroy(s->upload);
        if (s->table_dev)
            hipFree(s->table_dev);
        if (s->table_host)
            hipHostFree(s->table_host);
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
    p.rq = make_request(item->src, item->src_blobs, item->dst, item->dst_blobs, true, true);
    const bool split = item->src->kind == LLAMA_SPLIT || item->dst->kind == LLAMA_SPLIT;
    if (split) {
        if (s->has_exec)
            fail(LLAMA_E_UNSUPPORTED, "a server with an executor takes plain mappings only");
        p.parts = split_copies(item->src, item->dst, p.rq);
    }
    if (s->has_exec) {
        p.owned = own_item(item, p.rq);
    } else {
        int dev = 0;
        check_hip(hipGetDevice(&dev), "hipGetDevice");
        if (dev != s->device)
            fail(LLAMA_E_INVALID_ARG, "request submitted from device " + std::to_string(dev) +
                                          " to a server on device " + std::to_string(s->device));
    }
    if (!s->has_exec && s->cfg.policy != LLAMA_SERVE_NAIVE) {
        llama_copy_options o{LLAMA_PATH_AUTO, 0, s->cfg.threads, 0, 0};
        if (s->cfg.policy == LLAMA_SERVE_BATCHED && !split && make_plan(p.rq, &o).path == LLAMA_PATH_NAIVE)
            fail(LLAMA_E_UNSUPPORTED, "the record does not fit the tiled kernel; copy it with llama_copy");
        for (const SubCopy& c : p.parts)
            if (s->cfg.policy == LLAMA_SERVE_BATCHED && (c.naive || make_plan(c.rq, &o).path == LLAMA_PATH_NAIVE))
                fail(LLAMA_E_UNSUPPORTED, "a part copy of this Split request runs element-wise; copy it with llama_copy");
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
    if (s->has_exec) { // the engine has drained every launch
        delete s;
        return;
    }
    (void)hipSetDevice(s->device);
    for (hipStream_t st : s->streams)
        (void)hipStreamSynchronize(st);
    for (Slot& sl : s->slots) {
        if (sl.dev && sl.own_dev)
            (void)hipFree(sl.dev);
        if (sl.host && sl.own_host)
            (void)hipHostFree(sl.host);
        (void)hipEventDestroy(sl.done);
        if (sl.uploaded)
            (void)hipEventDestroy(sl.uploaded);
    }
    if (s->upload) {
        (void)hipStreamSynchronize(s->upload);
        (void)hipStreamDestroy(s->upload);
    }
    if (s->table_dev)
        (void)hipFree(s->table_dev);
    if (s->table_host)
        (void)hipHostFree(s->table_host);
    for (hipStream_t st : s->streams)
        (void)hipStreamDestroy(st);
    (void)hipGetLastError();
    delete s;
}

} // namespace llama
