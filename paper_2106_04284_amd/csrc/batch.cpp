// Batches: many independent copies in one persistent launch, replayed from a
// hipGraph.
#include <hip/hip_runtime_api.h>

#include <algorithm>
#include <cstring>
#include <map>
#include <mutex>
#include <tuple>
#include <vector>

#include "batch.hpp"

namespace llama {

namespace {

void check_hip(hipError_t e, const char* what)
{
    if (e != hipSuccess)
        fail(LLAMA_E_HIP, std::string(what) + ": " + hipGetErrorString(e));
}

struct Range {
    uint64_t lo, hi; // [lo, hi)
    size_t item;
};

// Destination ranges must be disjoint from every other destination range and
// from every source range of any item (a batch runs its items in no fixed
// order, so a read of one item could meet a write of another).
void check_batch_overlap(const std::vector<Request>& rqs)
{
    std::vector<Range> dst, src;
    for (size_t k = 0; k < rqs.size(); k++) {
        for (size_t b = 0; b < rqs[k].dst_ptr.size(); b++)
            if (rqs[k].dst.blob_size[b])
                dst.push_back({rqs[k].dst_ptr[b], rqs[k].dst_ptr[b] + rqs[k].dst.blob_size[b], k});
        for (size_t b = 0; b < rqs[k].src_ptr.size(); b++)
            if (rqs[k].src.blob_size[b])
                src.push_back({rqs[k].src_ptr[b], rqs[k].src_ptr[b] + rqs[k].src.blob_size[b], k});
    }
    std::sort(dst.begin(), dst.end(), [](const Range& a, const Range& b) { return a.lo < b.lo; });
    for (size_t k = 1; k < dst.size(); k++)
        if (dst[k].lo < dst[k - 1].hi)
            fail(LLAMA_E_OVERLAP, "batch items " + std::to_string(dst[k - 1].item) + " and " +
                                      std::to_string(dst[k].item) + " write overlapping ranges");
    for (const Range& s : src) {
        // the last destination range starting before s.hi
        auto it = std::upper_bound(dst.begin(), dst.end(), s.hi - 1, [](uint64_t v, const Range& r) { return v < r.lo; });
        if (it != dst.begin()) {
            --it;
            if (it->hi > s.lo)
                fail(LLAMA_E_OVERLAP, "batch item " + std::to_string(it->item) + " writes a range that item " +
                                          std::to_string(s.item) + " reads");
        }
    }
}

std::mutex g_retired_mutex;
std::vector<std::pair<Batch*, hipEvent_t>> g_retired; // one-shot batches waiting for their launch to end

void reap_retired()
{
    std::lock_guard<std::mutex> lock(g_retired_mutex);
    for (size_t k = 0; k < g_retired.size();) {
        if (hipEventQuery(g_retired[k].second) == hipSuccess) {
            (void)hipEventDestroy(g_retired[k].second);
            destroy_batch(g_retired[k].first);
            g_retired[k] = g_retired.back();
            g_retired.pop_back();
        } else {
            k++;
        }
    }
    (void)hipGetLastError();
}

// the largest tile that fitted kBatchLdsBytes, per class of copies (leaf
// hash, source kind and lanes, destination kind and lanes, threads, flags)
std::mutex g_tile_memo_mutex;
std::map<std::tuple<uint64_t, uint32_t, uint64_t, uint32_t, uint64_t, uint32_t, uint32_t>, uint32_t> g_tile_memo;

} // namespace

Plan batch_plan(const Request& rq, uint32_t threads, uint32_t tile_records, uint32_t flags, uint32_t lds_budget)
{
    const uint32_t budget = lds_budget ? lds_budget : kBatchLdsBytes;
    if (rq.src.kind == LLAMA_ONE)
        fail(LLAMA_E_UNSUPPORTED, "a One source is copied element-wise; copy it with llama_copy");
    llama_copy_options o{LLAMA_PATH_AUTO, tile_records, threads, 0, flags};
    Plan p;
    if (tile_records) {
        p = make_plan(rq, &o);
    } else {
        // Every workgroup of the launch reserves the same LDS and about five
        // fit a compute unit, so the bytes in flight per compute unit grow
        // with the bytes per tile: take the largest tile whose plan fits
        // kBatchLdsBytes (a standalone launch's tuned tile may be small
        // because many of its workgroups fit a compute unit at once).
        // the tile found for a class of copies is remembered, so that a
        // repeated class costs one plan instead of a search
        TuneKey k = tune_key(rq);
        k.bucket = 0;
        const auto key =
            std::make_tuple(k.leaves, k.src_kind, k.src_lanes, k.dst_kind, k.dst_lanes, threads, flags | (budget << 8));
        uint32_t start = 4096;
        {
            std::lock_guard<std::mutex> lock(g_tile_memo_mutex);
            auto it = g_tile_memo.find(key);
            if (it != g_tile_memo.end())
                start = it->second;
        }
        bool found = false;
        uint32_t T = start;
        for (; T >= 16 && !found; T /= 2) {
            o.tile_records = T;
            p = make_plan(rq, &o);
            // a gathering tile (no destination region) is sized like its
            // staged twin, as if it held both regions: the largest gathering
            // tile that fits measured 6% slower over the 1,000-array batch,
            // the twin's size 4% faster than staging; halving every tile
            // lost 15%
            const uint32_t lds = p.tile.h.lds_bytes * ((p.tile.h.flags & kTileGatherStore) ? 2u : 1u);
            found = p.path == LLAMA_PATH_STREAM || p.path == LLAMA_PATH_EMPTY ||
                    (p.path == LLAMA_PATH_TILE &&
                     (lds <= budget || (T == 16 && p.tile.h.lds_bytes <= budget)));
        }
        if (!found)
            fail(LLAMA_E_UNSUPPORTED, "its record does not fit the tiled kernel; copy it with llama_copy");
        if (T * 2 != start) {
            std::lock_guard<std::mutex> lock(g_tile_memo_mutex);
            g_tile_memo[key] = T * 2;
        }
    }
    if (p.path != LLAMA_PATH_EMPTY && p.path != LLAMA_PATH_TILE && p.path != LLAMA_PATH_STREAM)
        fail(LLAMA_E_UNSUPPORTED, "its record does not fit the tiled kernel; copy it with llama_copy");
    return p;
}

void BatchTable::add(const Request& rq, uint32_t threads, uint32_t tile_records, uint32_t flags, uint32_t lds_budget)
{
    add_plan(batch_plan(rq, threads, tile_records, flags, lds_budget));
}

void BatchTable::add_plan(const Plan& p)
{
    if (p.then) // the zero fill of an aligned SoA destination's padding: an item of its own
        add_plan(*p.then);
    read_bytes += p.read_bytes;
    write_bytes += p.write_bytes;
    if (p.path == LLAMA_PATH_EMPTY)
        return;
    uint32_t cls = 0;
    if (p.path == LLAMA_PATH_TILE)
        for (cls = 1; (uint64_t(1024) << (cls - 1)) < p.tile.h.lds_bytes && cls < 31; cls++) {
        }
    classes |= 1u << cls;
    BatchItem it{};
    if (p.path == LLAMA_PATH_TILE && (p.tile.h.flags & kTileVirtualSrc))
        fail(LLAMA_E_UNSUPPORTED, "a source gathered from several parts runs as its own copy");
    if (p.path == LLAMA_PATH_TILE) {
        it.kind = kItemTile;
        it.count = p.tile.h.num_entries;
        if (p.tile.h.flags & kTileGatherStore) { // the word table follows the entries
            it.gather = p.tile.gather;
            it.count += uint32_t((uint64_t(p.tile.gather.table) * 4 + sizeof(TileEntry) - 1) / sizeof(TileEntry));
        }
        it.first = entries.size();
        it.h = p.tile.h;
        entries.insert(entries.end(), p.tile.e, p.tile.e + it.count);
        lds_bytes = std::max(lds_bytes, p.tile.h.lds_bytes);
        tile_items++;
    } else if (p.path == LLAMA_PATH_STREAM) {
        // a batch moves a run in 16 KiB units (four 16-byte loads per thread
        // in flight): 4 KiB units starved the persistent grid's workgroups
        it.kind = kItemStream;
        it.count = p.stream.num_runs;
        it.first = runs.size();
        uint64_t chunks = 0;
        for (uint32_t r = 0; r < p.stream.num_runs; r++) {
            StreamRun run = p.stream.r[r];
            run.first_chunk = chunks;
            chunks += (run.bytes + (uint64_t(1) << kBatchStreamChunkLog2) - 1) >> kBatchStreamChunkLog2;
            runs.push_back(run);
        }
        it.h.num_tiles = chunks;
        stream_items++;
    } else {
        fail(LLAMA_E_UNSUPPORTED, "its record does not fit the tiled kernel; copy it with llama_copy");
    }
    unit_begin.push_back(units);
    units += it.h.num_tiles;
    items.push_back(it);
}

namespace {
size_t align256(size_t x) { return (x + 255) & ~size_t(255); }
struct TableLayout {
    size_t counters, begin, hint, items, entries, runs, total;
};
size_t hint_count(uint64_t units) { return size_t((units >> kBatchHintLog2) + 2); }
TableLayout table_layout(const BatchTable& t)
{
    TableLayout l;
    l.counters = 0;
    l.begin = align256(2 * sizeof(unsigned long long));
    l.hint = align256(l.begin + (t.unit_begin.size() + 1) * sizeof(uint64_t));
    l.items = align256(l.hint + hint_count(t.units) * sizeof(uint32_t));
    l.entries = align256(l.items + std::max<size_t>(t.items.size(), 1) * sizeof(BatchItem));
    l.runs = align256(l.entries + std::max<size_t>(t.entries.size(), 1) * sizeof(TileEntry));
    l.total = align256(l.runs + std::max<size_t>(t.runs.size(), 1) * sizeof(StreamRun));
    return l;
}
} // namespace

std::vector<BatchRange> BatchTable::sort_by_mode()
{
    std::vector<size_t> order(items.size());
    for (size_t k = 0; k < order.size(); k++)
        order[k] = k;
    std::vector<uint32_t> key(items.size());
    for (size_t k = 0; k < items.size(); k++)
        key[k] = batch_mode_key(items[k]);
    std::stable_sort(order.begin(), order.end(), [&](size_t a, size_t b) { return key[a] < key[b]; });
    std::vector<BatchItem> sorted;
    sorted.reserve(items.size());
    std::vector<BatchRange> ranges;
    unit_begin.clear();
    units = 0;
    for (size_t k : order) {
        const BatchItem& it = items[k];
        if (ranges.empty() || ranges.back().key != key[k])
            ranges.push_back(BatchRange{key[k], units, 0, 0});
        BatchRange& r = ranges.back();
        r.units += it.h.num_tiles;
        if (it.kind == kItemTile)
            r.lds_bytes = std::max(r.lds_bytes, it.h.lds_bytes);
        unit_begin.push_back(units);
        units += it.h.num_tiles;
        sorted.push_back(it);
    }
    items = std::move(sorted);
    std::vector<BatchRange> nonempty;
    for (const BatchRange& r : ranges)
        if (r.units)
            nonempty.push_back(r);
    return nonempty;
}

size_t BatchTable::bytes() const
{
    return table_layout(*this).total;
}

void BatchTable::serialise(uint8_t* host, uint64_t device, BatchArgs& args) const
{
    const TableLayout l = table_layout(*this);
    std::memset(host, 0, l.total);
    std::memcpy(host + l.begin, unit_begin.data(), unit_begin.size() * sizeof(uint64_t));
    std::memcpy(host + l.begin + unit_begin.size() * sizeof(uint64_t), &units, sizeof(uint64_t));
    // the item of every 2^kBatchHintLog2-th unit (the last item past the end)
    uint32_t* hint = (uint32_t*)(host + l.hint);
    size_t j = 0;
    for (size_t c = 0; c < hint_count(units); c++) {
        const uint64_t g = uint64_t(c) << kBatchHintLog2;
        while (j + 1 < unit_begin.size() && unit_begin[j + 1] <= g)
            j++;
        hint[c] = uint32_t(j);
    }
    if (!items.empty())
        std::memcpy(host + l.items, items.data(), items.size() * sizeof(BatchItem));
    if (!entries.empty())
        std::memcpy(host + l.entries, entries.data(), entries.size() * sizeof(TileEntry));
    if (!runs.empty())
        std::memcpy(host + l.runs, runs.data(), runs.size() * sizeof(StreamRun));
    args.counters = (unsigned long long*)(device + l.counters);
    args.unit_begin = (const uint64_t*)(device + l.begin);
    args.hint = (const uint32_t*)(device + l.hint);
    args.items = (const BatchItem*)(device + l.items);
    args.entries = (const TileEntry*)(device + l.entries);
    args.runs = (const StreamRun*)(device + l.runs);
    args.total_units = units;
    args.num_items = uint32_t(items.size());
    args.flags = read_bytes >= kStreamLoadBytes ? kBatchLoadsOnce : 0u;
}

// A batch whose items share one LDS class runs one workgroup per work unit:
// the dispatcher keeps every workgroup's footprint small and starts them as
// residency allows (4,096 particle frames of one class: 2.7x faster than a
// persistent grid).  A batch spanning several classes runs a persistent grid
// over one table instead: every workgroup of a launch reserves the largest
// class's LDS, and the persistent workgroups overlap items of different
// kinds (the 1,000-array batch: +5% over one workgroup per unit, with or
// without one launch per class).
bool batch_per_unit(const BatchTable& t)
{
    return (t.classes & (t.classes - 1)) == 0;
}

uint32_t batch_wg_per_cu(uint32_t lds_bytes, uint32_t threads)
{
    const uint32_t waves = threads / 64;
    // 64 bytes of static LDS (the block counters) per workgroup besides the tile
    const uint32_t fit = std::min<uint32_t>(lds_bytes ? kHardLdsBytes / (lds_bytes + 64) : 16, kMaxWavesPerCu / waves);
    return std::max<uint32_t>(1, std::min<uint32_t>(fit, 8));
}

uint32_t batch_grid(uint64_t units, uint32_t wg_per_cu)
{
    const uint64_t u = std::max<uint64_t>(units, 1);
    if (wg_per_cu == 0)
        return uint32_t(std::min<uint64_t>(u, kBatchMaxGrid));
    return uint32_t(std::min<uint64_t>(u, uint64_t(device_cu_count()) * wg_per_cu));
}

BatchTable build_batch_table(size_t n, const llama_copy_item* items, const llama_copy_options* opt,
                             uint32_t& threads, std::vector<Request>* work)
{
    reap_retired();
    if (n > 0 && !items)
        fail(LLAMA_E_INVALID_ARG, "batch item array is NULL");
    if (opt && (opt->path != LLAMA_PATH_AUTO || (opt->flags & ~kCopyFlags) != 0))
        fail(LLAMA_E_INVALID_ARG, "batch options take tile_records, threads, wg_per_cu and LLAMA_COPY_* flags");
    threads = (opt && opt->threads) ? opt->threads : kDefaultThreads;
    if (threads % 64 != 0 || threads == 0 || threads > 1024)
        fail(LLAMA_E_INVALID_ARG, "threads must be a multiple of 64 in 64..1024");
    if (opt && opt->wg_per_cu > 16)
        fail(LLAMA_E_INVALID_ARG, "wg_per_cu must be 0..16");
    const uint32_t T = opt ? opt->tile_records : 0;
    if (T && (T < 16 || T > 4096 || (T & (T - 1))))
        fail(LLAMA_E_INVALID_ARG, "tile_records must be a power of two in 16..4096");

    std::vector<Request> rqs;
    rqs.reserve(n);
    for (size_t k = 0; k < n; k++) {
        try {
            rqs.push_back(make_request(items[k].src, items[k].src_blobs, items[k].dst, items[k].dst_blobs, true, true));
        } catch (const Error& e) {
            fail(e.status, "batch item " + std::to_string(k) + ": " + e.message);
        }
    }
    check_batch_overlap(rqs);

    // An item with a Split side becomes its part copies, which write disjoint
    // bytes and so may run side by side; one that would write part of the
    // records of a record-major destination part needs its part copies in
    // order and is refused.
    BatchTable t;
    for (size_t k = 0; k < n; k++) {
        try {
            if (items[k].src->kind != LLAMA_SPLIT && items[k].dst->kind != LLAMA_SPLIT) {
                t.add(rqs[k], threads, T, opt ? opt->flags : 0u);
                if (work)
                    work->push_back(rqs[k]);
                continue;
            }
            std::vector<SubCopy> parts = split_copies(items[k].src, items[k].dst, rqs[k]);
            for (const SubCopy& c : parts)
                if (c.naive) // then the copies into that part depend on their order
                    fail(LLAMA_E_UNSUPPORTED, "its part copies write parts of the records of a record-major "
                                              "destination part in turn; copy it with llama_copy");
            for (const SubCopy& c : parts) {
                t.add(c.rq, threads, T, opt ? opt->flags : 0u);
                if (work)
                    work->push_back(c.rq);
            }
        } catch (const Error& e) {
            fail(e.status, "batch item " + std::to_string(k) + ": " + e.message);
        }
    }
    return t;
}

namespace {

// Fills `b` (counts, grid) from table `t` and uploads the table into a new
// device allocation, freeing the previous one.  by_mode: the table sorted by
// tile mode, one launch per mode (wg_per_cu is then ignored).
void install_table(Batch* b, BatchTable t, uint32_t wg_per_cu, bool by_mode)
{
    b->ranges.clear();
    if (by_mode)
        b->ranges = t.sort_by_mode();
    b->total_units = t.units;
    b->lds_bytes = t.lds_bytes;
    b->items = t.items.size();
    b->tile_items = t.tile_items;
    b->stream_items = t.stream_items;
    b->read_bytes = t.read_bytes;
    b->write_bytes = t.write_bytes;
    b->wg_per_cu = by_mode ? 0 : wg_per_cu ? wg_per_cu : batch_per_unit(t) ? 0 : batch_wg_per_cu(t.lds_bytes, b->threads);
    b->grid = batch_grid(t.units, b->wg_per_cu);
    const size_t total = t.bytes();
    std::vector<uint8_t> host(total);
    void* table = nullptr;
    check_hip(hipMalloc(&table, total), "hipMalloc(batch table)");
    BatchArgs args{};
    t.serialise(host.data(), uint64_t(uintptr_t(table)), args);
    hipError_t e = hipMemcpy(table, host.data(), total, hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        (void)hipFree(table);
        check_hip(e, "hipMemcpy(batch table)");
    }
    if (b->table)
        (void)hipFree(b->table);
    if (b->graph_exec)
        (void)hipGraphExecDestroy((hipGraphExec_t)b->graph_exec);
    b->graph_exec = nullptr;
    b->table = table;
    b->table_bytes = total;
    b->args = args;
}

} // namespace

Batch* create_batch(size_t n, const llama_copy_item* items, const llama_copy_options* opt)
{
    uint32_t threads = 0;
    std::unique_ptr<Batch> b(new Batch());
    const BatchTable t = build_batch_table(n, items, opt, threads, &b->work);
    b->flags = opt ? opt->flags : 0u;
    b->tile_records = opt ? opt->tile_records : 0u;
    b->threads = threads;
    check_hip(hipGetDevice(&b->device), "hipGetDevice");
    install_table(b.get(), t, opt ? opt->wg_per_cu : 0, kBatchByModeDefault && !(opt && opt->wg_per_cu));
    return b.release();
}

void autotune_batch(Batch* b, void* stream_ptr, int reps, double* best_gbs)
{
    hipStream_t stream = (hipStream_t)stream_ptr;
    int dev = 0;
    check_hip(hipGetDevice(&dev), "hipGetDevice");
    if (dev != b->device)
        fail(LLAMA_E_INVALID_ARG, "batch was created on another device");
    if (b->total_units == 0)
        return;
    if (reps <= 0)
        reps = 3;
    // the destinations of the current plan, hashed: every candidate must match
    std::vector<std::pair<uint64_t, uint64_t>> dsts;
    for (const Request& rq : b->work)
        for (size_t k = 0; k < rq.dst_ptr.size(); k++)
            if (rq.dst.blob_size[k])
                dsts.push_back({rq.dst_ptr[k], rq.dst.blob_size[k]});
    std::sort(dsts.begin(), dsts.end());
    dsts.erase(std::unique(dsts.begin(), dsts.end()), dsts.end());
    void* acc_p = nullptr;
    check_hip(hipMalloc(&acc_p, sizeof(unsigned long long)), "hipMalloc(hash)");
    unsigned long long* acc = (unsigned long long*)acc_p;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    auto cleanup = [&] {
        if (e0)
            (void)hipEventDestroy(e0);
        if (e1)
            (void)hipEventDestroy(e1);
        (void)hipFree(acc_p);
    };
    try {
        check_hip(hipEventCreate(&e0), "hipEventCreate");
        check_hip(hipEventCreate(&e1), "hipEventCreate");
        auto hash = [&](int fill) {
            for (const auto& d : dsts)
                check_hip(hipMemsetAsync((void*)d.first, fill, d.second, stream), "hipMemsetAsync");
            launch_batch_kernel(*b, stream);
            check_hip(hipMemsetAsync(acc, 0, sizeof(*acc), stream), "hipMemsetAsync");
            for (const auto& d : dsts)
                launch_hash((const void*)d.first, d.second, acc, stream);
            unsigned long long h = 0;
            check_hip(hipMemcpyAsync(&h, acc, sizeof(h), hipMemcpyDeviceToHost, stream), "hipMemcpyAsync");
            check_hip(hipStreamSynchronize(stream), "hipStreamSynchronize");
            return uint64_t(h);
        };
        auto time_it = [&] {
            launch_batch_kernel(*b, stream);
            double best = 1e30;
            for (int r = 0; r < reps; r++) {
                check_hip(hipEventRecord(e0, stream), "hipEventRecord");
                launch_batch_kernel(*b, stream);
                check_hip(hipEventRecord(e1, stream), "hipEventRecord");
                check_hip(hipEventSynchronize(e1), "hipEventSynchronize");
                float ms = 0;
                check_hip(hipEventElapsedTime(&ms, e0, e1), "hipEventElapsedTime");
                best = std::min(best, double(ms));
            }
            return best;
        };
        const uint64_t want = hash(0x5A);
        struct Cand {
            uint32_t budget, threads, wg;
            bool by_mode;
        };
        Cand best{b->lds_budget, b->threads, b->wg_per_cu, !b->ranges.empty()};
        double best_ms = time_it();
        // LDS per tiled item (the tile each item takes), threads, and the grid
        // (0: the default rule, else a persistent grid of that many
        // workgroups per compute unit)
        // (grid 17: one launch per tile mode over a table sorted by mode)
        const uint32_t budgets[] = {8 * 1024, 16 * 1024, kBatchLdsBytes, 48 * 1024};
        const uint32_t threads[] = {128, 256, 512};
        const uint32_t grids[] = {0, 2, 4, 8, 17};
        for (uint32_t bud : budgets)
            for (uint32_t th : threads)
                for (uint32_t wg : grids) {
                    BatchTable t;
                    try {
                        for (const Request& rq : b->work)
                            t.add(rq, th, b->tile_records, b->flags, bud);
                    } catch (const Error&) {
                        continue; // an item does not fit this budget
                    }
                    b->threads = th;
                    b->lds_budget = bud;
                    install_table(b, t, wg == 17 ? 0 : wg, wg == 17);
                    if (hash(0xA5) != want)
                        fail(LLAMA_E_HIP, "a batch tuning candidate wrote different bytes");
                    const double ms = time_it();
                    if (ms < best_ms) {
                        best_ms = ms;
                        best = {bud, th, wg == 17 ? 0 : wg, wg == 17};
                    }
                }
        // re-plan with the fastest
        BatchTable t;
        for (const Request& rq : b->work)
            t.add(rq, best.threads, b->tile_records, b->flags, best.budget);
        b->threads = best.threads;
        b->lds_budget = best.budget;
        install_table(b, t, best.wg, best.by_mode);
        if (best_gbs)
            *best_gbs = double(b->read_bytes + b->write_bytes) / (best_ms * 1e-3) / 1e9;
    } catch (...) {
        cleanup();
        throw;
    }
    cleanup();
}

void copy_batch_noalloc(size_t n, const llama_copy_item* items, void* stream)
{
    uint32_t threads = 0;
    BatchTable t = build_batch_table(n, items, nullptr, threads);
    std::vector<BatchRange> ranges;
    if (kBatchByModeDefault)
        ranges = t.sort_by_mode();
    if (t.units == 0)
        return;
    const size_t total = t.bytes();
    if (total > kScratchBytes)
        fail(LLAMA_E_NO_BUDGET, "the batch's work table needs " + std::to_string(total) +
                                    " bytes, more than the " + std::to_string(kScratchBytes) +
                                    " bytes of the library's static work-table buffer; use llama_copy_batch");
    const uint64_t dev_table = scratch_address(); // this device's copy of the static buffer
    // the host image is kept per thread and reused; hipMemcpyAsync has read a
    // pageable source by the time it returns
    static thread_local std::vector<uint8_t> host;
    if (host.size() < total)
        host.resize(total);
    BatchArgs args{};
    t.serialise(host.data(), dev_table, args); // the counters go up as zeros with the table
    check_hip(hipMemcpyAsync((void*)uintptr_t(dev_table), host.data(), total, hipMemcpyHostToDevice,
                             (hipStream_t)stream),
              "hipMemcpyAsync(batch table into the static buffer)");
    if (!ranges.empty()) {
        launch_batch_ranges(args, ranges, threads, stream);
        return;
    }
    const uint32_t wg = batch_per_unit(t) ? 0 : batch_wg_per_cu(t.lds_bytes, threads);
    launch_batch_args(args, batch_grid(t.units, wg), threads, t.lds_bytes, wg != 0, stream);
}

void launch_batch(Batch* b, void* stream_ptr)
{
    hipStream_t stream = (hipStream_t)stream_ptr;
    int dev = 0;
    check_hip(hipGetDevice(&dev), "hipGetDevice");
    if (dev != b->device)
        fail(LLAMA_E_INVALID_ARG, "batch was created on device " + std::to_string(b->device) +
                                      " and launched on device " + std::to_string(dev));
    if (b->total_units == 0)
        return;
    if (!stream) { // the null stream cannot be captured: launch directly
        launch_batch_kernel(*b, stream);
        return;
    }
    if (!b->graph_exec) {
        hipGraph_t graph = nullptr;
        check_hip(hipStreamBeginCapture(stream, hipStreamCaptureModeThreadLocal), "hipStreamBeginCapture");
        try {
            launch_batch_kernel(*b, stream);
        } catch (...) {
            hipStreamEndCapture(stream, &graph);
            if (graph)
                hipGraphDestroy(graph);
            throw;
        }
        check_hip(hipStreamEndCapture(stream, &graph), "hipStreamEndCapture");
        hipGraphExec_t exec = nullptr;
        hipError_t e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
        hipGraphDestroy(graph);
        check_hip(e, "hipGraphInstantiate");
        b->graph_exec = exec;
    }
    check_hip(hipGraphLaunch((hipGraphExec_t)b->graph_exec, stream), "hipGraphLaunch");
}

void destroy_batch(Batch* b)
{
    if (!b)
        return;
    int prev = 0;
    (void)hipGetDevice(&prev);
    (void)hipSetDevice(b->device);
    (void)hipDeviceSynchronize();
    if (b->graph_exec)
        (void)hipGraphExecDestroy((hipGraphExec_t)b->graph_exec);
    if (b->table)
        (void)hipFree(b->table);
    (void)hipSetDevice(prev);
    (void)hipGetLastError();
    delete b;
}

void retire_batch(Batch* b, void* stream_ptr)
{
    hipEvent_t ev;
    check_hip(hipEventCreateWithFlags(&ev, hipEventDisableTiming), "hipEventCreate");
    hipError_t e = hipEventRecord(ev, (hipStream_t)stream_ptr);
    if (e != hipSuccess) {
        (void)hipEventDestroy(ev);
        check_hip(e, "hipEventRecord");
    }
    std::lock_guard<std::mutex> lock(g_retired_mutex);
    g_retired.push_back({b, ev});
}

} // namespace llama
