// extern "C" entry points declared in include/llama_mi355x.h.
#include <algorithm>
#include <cstring>
#include <memory>
#include <mutex>
#include <exception>
#include <string>

#include "batch.hpp"
#include "core.hpp"
#include "serve.hpp"

using namespace llama;

namespace {

thread_local std::string g_last_error;

int set_error(int status, const std::string& message)
{
    g_last_error = message;
    return status;
}

template <typename F>
int guarded(F&& body)
{
    try {
        body();
        return LLAMA_OK;
    } catch (const Error& e) {
        return set_error(e.status, e.message);
    } catch (const std::bad_alloc&) {
        return set_error(LLAMA_E_INVALID_ARG, "host memory exhausted");
    } catch (const std::exception& e) {
        return set_error(LLAMA_E_INVALID_ARG, e.what());
    } catch (...) {
        return set_error(LLAMA_E_INVALID_ARG, "unknown error");
    }
}

void need(const void* p, const char* what)
{
    if (!p)
        fail(LLAMA_E_INVALID_ARG, std::string(what) + " is NULL");
}

} // namespace

extern "C" {

const char* llama_last_error(void)
{
    return g_last_error.c_str();
}

const char* llama_status_string(int status)
{
    switch (status) {
    case LLAMA_OK: return "LLAMA_OK";
    case LLAMA_E_INVALID_ARG: return "LLAMA_E_INVALID_ARG";
    case LLAMA_E_RECORD_MISMATCH: return "LLAMA_E_RECORD_MISMATCH";
    case LLAMA_E_EXTENT_MISMATCH: return "LLAMA_E_EXTENT_MISMATCH";
    case LLAMA_E_BLOB_TOO_SMALL: return "LLAMA_E_BLOB_TOO_SMALL";
    case LLAMA_E_OVERLAP: return "LLAMA_E_OVERLAP";
    case LLAMA_E_OVERFLOW: return "LLAMA_E_OVERFLOW";
    case LLAMA_E_UNSUPPORTED: return "LLAMA_E_UNSUPPORTED";
    case LLAMA_E_HIP: return "LLAMA_E_HIP";
    case LLAMA_E_NO_BUDGET: return "LLAMA_E_NO_BUDGET";
    case LLAMA_E_BUSY: return "LLAMA_E_BUSY";
    default: return "LLAMA_E_UNKNOWN";
    }
}

int llama_record_info(const llama_record_desc* record, uint32_t* leaf_count, uint64_t* packed_size,
                      uint64_t* aligned_size)
{
    return guarded([&] {
        Record r = flatten(record);
        if (leaf_count)
            *leaf_count = uint32_t(r.leaves.size());
        if (packed_size)
            *packed_size = r.packed_size;
        if (aligned_size)
            *aligned_size = r.aligned_size;
    });
}

int llama_record_leaf(const llama_record_desc* record, uint32_t leaf, uint32_t* size, uint32_t* align,
                      uint64_t* packed_offset, uint64_t* aligned_offset)
{
    return guarded([&] {
        Record r = flatten(record);
        if (leaf >= r.leaves.size())
            fail(LLAMA_E_INVALID_ARG, "leaf " + std::to_string(leaf) + " out of range");
        const Leaf& l = r.leaves[leaf];
        if (size)
            *size = l.size;
        if (align)
            *align = l.align;
        if (packed_offset)
            *packed_offset = l.packed_offset;
        if (aligned_offset)
            *aligned_offset = l.aligned_offset;
    });
}

int llama_mapping_blob_count(const llama_mapping_desc* mapping, uint32_t* count)
{
    return guarded([&] {
        need(mapping, "mapping");
        need(count, "count");
        Record r = flatten(mapping->record);
        Side s = make_side(mapping, r);
        *count = uint32_t(s.blob_size.size());
    });
}

int llama_mapping_blob_size(const llama_mapping_desc* mapping, uint32_t blob, uint64_t* size)
{
    return guarded([&] {
        need(mapping, "mapping");
        need(size, "size");
        Record r = flatten(mapping->record);
        Side s = make_side(mapping, r);
        if (blob >= s.blob_size.size())
            fail(LLAMA_E_INVALID_ARG, "blob " + std::to_string(blob) + " out of range");
        *size = s.blob_size[blob];
    });
}

int llama_mapping_offset(const llama_mapping_desc* mapping, const uint64_t* coord, uint32_t leaf, uint32_t* blob,
                         uint64_t* offset)
{
    return guarded([&] {
        need(mapping, "mapping");
        need(coord, "coord");
        need(blob, "blob");
        need(offset, "offset");
        Record r = flatten(mapping->record);
        Side s = make_side(mapping, r);
        if (leaf >= r.leaves.size())
            fail(LLAMA_E_INVALID_ARG, "leaf " + std::to_string(leaf) + " out of range");
        for (uint32_t d = 0; d < s.rank; d++)
            if (coord[d] >= s.extents[d])
                fail(LLAMA_E_INVALID_ARG, "coordinate out of range in dimension " + std::to_string(d));
        const uint64_t i = linearize(s, coord);
        *blob = s.blob[leaf];
        *offset = s.offset(i, leaf, r);
    });
}

namespace {

void fill_info(const Plan& p, llama_plan_info* info)
{
    std::memset(info, 0, sizeof(*info));
    info->path = p.path;
    info->threads = p.threads;
    info->tile_records = p.path == LLAMA_PATH_TILE  ? (1u << p.tile.h.log2_tile)
                         : p.path == LLAMA_PATH_BOX ? (1u << p.box.h.qlog_sum)
                                                    : 0;
    info->lds_bytes = p.lds_bytes;
    info->workgroups = p.workgroups;
    info->runs = p.path == LLAMA_PATH_STREAM ? p.stream.num_runs : 0;
    info->wg_per_cu = p.wg_per_cu;
    info->tiles = p.tiles;
    info->read_bytes = p.read_bytes;
    info->write_bytes = p.write_bytes;
    info->tile_mode = 0;
    info->cache_hints = 0;
    info->plan_flags = 0;
    if (p.path == LLAMA_PATH_TILE) {
        const uint32_t f = p.tile.h.flags;
        info->tile_mode = (f & kTileDirectStore)   ? LLAMA_TILE_DIRECT_STORE
                          : (f & kTileDirectLoad)  ? LLAMA_TILE_DIRECT_LOAD
                          : (f & kTileGatherStore) ? LLAMA_TILE_GATHER_STORE
                                                   : LLAMA_TILE_STAGED;
        info->cache_hints = ((f & kTileStreamLoads) ? LLAMA_HINT_STREAM_LOADS : 0u) |
                            ((f & kTileStreamStores) ? LLAMA_HINT_STREAM_STORES : 0u);
        info->plan_flags = ((f & kTileVirtualSrc) ? LLAMA_PLAN_GATHERED_SOURCE : 0u) |
                           ((f & kTilePreserve) ? LLAMA_PLAN_KEEPS_DESTINATION : 0u) |
                           ((f & kTileVirtualDst) ? LLAMA_PLAN_SCATTERED_DESTINATION : 0u);
        info->source_chunks = (f & kTileVirtualSrc) ? p.tile.h.slots : 0u;
    } else if (p.path == LLAMA_PATH_STREAM) {
        info->cache_hints = (p.stream.flags & kStreamLoadsOnce) ? LLAMA_HINT_STREAM_LOADS : 0u;
    }
}

} // namespace

int llama_plan(const llama_mapping_desc* src, const llama_mapping_desc* dst, const llama_copy_options* options,
               llama_plan_info* info)
{
    return guarded([&] {
        need(info, "info");
        Request rq = make_request(src, nullptr, dst, nullptr, false);
        Plan p;
        if (needs_box(rq)) {
            const uint64_t zero[LLAMA_MAX_RANK] = {};
            std::vector<Plan> ps = make_box_plans(rq, zero, zero, rq.dst.extents, true, options);
            if (!ps.empty())
                p = ps[0];
        } else {
            p = make_plan(rq, options);
        }
        if (trace_enabled())
            trace_plan(p);
        fill_info(p, info);
    });
}

namespace {

// The launches of llama_copy_ex, in order (without `need_blobs`: plans only,
// for distinct blobs aligned to 256 bytes).
std::vector<Plan> copy_plans(const llama_mapping_desc* src, const llama_blob* src_blobs, const llama_mapping_desc* dst,
                             const llama_blob* dst_blobs, const llama_copy_options* options, bool need_blobs)
{
    Request rq = make_request(src, src_blobs, dst, dst_blobs, need_blobs, true);
    if (needs_box(rq)) {
        // records at different linear indices: the whole extents as one box
        if (src->kind == LLAMA_SPLIT || dst->kind == LLAMA_SPLIT)
            fail(LLAMA_E_UNSUPPORTED, "Split copies take views with equal linear indices");
        const uint64_t zero[LLAMA_MAX_RANK] = {};
        std::vector<Plan> ps = make_box_plans(rq, zero, zero, rq.dst.extents, true, options);
        if (!rq.dst.blob_gaps.empty() && !(options && (options->flags & LLAMA_COPY_PRESERVE_PADDING)))
            ps.push_back(zero_fill_plan(rq)); // the padding between aligned SoA sub-arrays
        return ps;
    }
    if (src->kind != LLAMA_SPLIT && dst->kind != LLAMA_SPLIT)
        return {make_plan(rq, options)};
    // a Split side: one copy per destination part and source part sharing
    // leaves (or one from every source part feeding a destination part), in
    // order on the stream; every plan is made before the first launch
    std::vector<Plan> plans;
    for (const SubCopy& c : split_copies(src, dst, rq, true, options)) {
        if (c.gathered) {
            // one tile copy from every source part feeding this destination part
            plans.push_back(*c.plan);
            continue;
        }
        if (c.naive && c.rq.dst.lanes == 1 && c.rq.dst.gaps.empty() && c.rq.dst.npad == c.rq.dst.n) {
            // into AoS records another part copy has already written
            // whole: a staged tile that keeps every byte outside these
            // leaves (taken as gaps) by storing each loaded region back
            Request kept = c.rq;
            std::vector<std::pair<uint64_t, uint64_t>> cover;
            for (size_t k = 0; k < kept.record.leaves.size(); k++)
                cover.push_back({kept.dst.base[k], kept.record.leaves[k].size});
            std::sort(cover.begin(), cover.end());
            uint64_t cur = 0;
            for (const auto& cv : cover) {
                if (cv.first > cur)
                    kept.dst.gaps.push_back({cur, cv.first - cur});
                cur = std::max(cur, cv.first + cv.second);
            }
            if (kept.dst.block > cur)
                kept.dst.gaps.push_back({cur, kept.dst.block - cur});
            kept.dst.partial = false;
            llama_copy_options o = options ? *options : llama_copy_options{0, 0, 0, 0, 0};
            o.flags |= LLAMA_COPY_PRESERVE_PADDING;
            bool planned = false;
            try {
                plans.push_back(make_plan(kept, &o));
                planned = true;
            } catch (const Error&) {
                // too many gap entries: element-wise below
            }
            if (planned)
                continue;
        }
        if (c.naive) {
            // a tile plan that stores 16-byte granules of its own leaves
            // straight from the staged source (direct store, no padding
            // gaps) writes no other byte of the part's blocks either
            try {
                Plan t = make_plan(c.rq, options);
                if (t.path == LLAMA_PATH_TILE && (t.tile.h.flags & kTileDirectStore) && c.rq.dst.gaps.empty()) {
                    plans.push_back(t);
                    continue;
                }
            } catch (const Error&) {
                // the caller's path or tile size does not fit this part copy
            }
            llama_copy_options o = options ? *options : llama_copy_options{0, 0, 0, 0, 0};
            o.path = LLAMA_PATH_NAIVE;
            o.tile_records = 0;
            plans.push_back(make_plan(c.rq, &o));
        } else {
            plans.push_back(make_plan(c.rq, options));
        }
    }
    return plans;
}

// llama_copy_ex's body (also run under the Heatmap's counting)
void copy_ex(const llama_mapping_desc* src, const llama_blob* src_blobs, const llama_mapping_desc* dst,
             const llama_blob* dst_blobs, const llama_copy_options* options, void* stream)
{
    for (const Plan& p : copy_plans(src, src_blobs, dst, dst_blobs, options, true))
        launch(p, stream);
}

// the blob sizes a mapping needs
std::vector<uint64_t> blob_sizes(const llama_mapping_desc* m)
{
    need(m, "mapping");
    need(m->record, "record");
    return make_side(m, flatten(m->record)).blob_size;
}

// adds the blobs with counters to a count list
void add_counted(CountBlob* list, uint32_t& n, const llama_mapping_desc* m, const llama_blob* blobs,
                 uint32_t* const* counters)
{
    if (!counters)
        return;
    const std::vector<uint64_t> sizes = blob_sizes(m);
    for (size_t b = 0; b < sizes.size(); b++) {
        if (!counters[b] || sizes[b] == 0)
            continue;
        if (n >= uint32_t(kCountMaxBlobs))
            fail(LLAMA_E_UNSUPPORTED, "a Heatmap counts at most " + std::to_string(kCountMaxBlobs) +
                                          " blobs per list");
        const uint64_t lo = uint64_t(uintptr_t(blobs[b].ptr));
        list[n++] = {lo, lo + sizes[b], uint64_t(uintptr_t(counters[b]))};
    }
}

} // namespace

int llama_plan_copy(const llama_mapping_desc* src, const llama_mapping_desc* dst, const uint32_t* src_leaf,
                    const llama_copy_options* options, llama_plan_info* infos, uint32_t capacity, uint32_t* count)
{
    return guarded([&] {
        need(count, "count");
        *count = 0;
        const std::vector<Plan> plans = src_leaf ? leaves_plans(src, nullptr, dst, nullptr, src_leaf, options, false)
                                                 : copy_plans(src, nullptr, dst, nullptr, options, false);
        std::vector<const Plan*> all; // with the launches chained after each plan
        for (const Plan& p : plans)
            for (const Plan* q = &p; q; q = q->then.get())
                all.push_back(q);
        if (all.size() > capacity)
            fail(LLAMA_E_INVALID_ARG, "the copy makes " + std::to_string(all.size()) + " launches, capacity is " +
                                          std::to_string(capacity));
        if (!all.empty())
            need(infos, "infos");
        for (size_t k = 0; k < all.size(); k++)
            fill_info(*all[k], &infos[k]);
        *count = uint32_t(all.size());
    });
}

int llama_copy_ex(const llama_mapping_desc* src, const llama_blob* src_blobs, const llama_mapping_desc* dst,
                  const llama_blob* dst_blobs, const llama_copy_options* options, void* stream)
{
    return guarded([&] { copy_ex(src, src_blobs, dst, dst_blobs, options, stream); });
}

int llama_copy_heatmap(const llama_mapping_desc* src, const llama_blob* src_blobs, const llama_mapping_desc* dst,
                       const llama_blob* dst_blobs, const uint32_t* src_leaf, const llama_copy_options* options,
                       const llama_heatmap* heat, void* stream)
{
    return guarded([&] {
        need(heat, "heatmap");
        need(src_blobs, "source blobs");
        need(dst_blobs, "destination blobs");
        // validates like the copy itself before anything is enqueued (the
        // records of a copy between differing records are checked side by side)
        if (src_leaf) {
            need(src, "source mapping");
            need(dst, "destination mapping");
            need(src->record, "source record");
            need(dst->record, "destination record");
            std::vector<uint64_t> ptrs;
            check_blobs("source", make_side(src, flatten(src->record)), src_blobs, ptrs);
            check_blobs("destination", make_side(dst, flatten(dst->record)), dst_blobs, ptrs);
        } else {
            (void)make_request(src, src_blobs, dst, dst_blobs, true, true);
        }
        static CountTable table; // large; filled and uploaded under the lock
        static std::mutex lock;
        std::lock_guard<std::mutex> g(lock);
        std::memset(&table, 0, sizeof(table));
        add_counted(table.r, table.nr, src, src_blobs, heat->src_reads);
        add_counted(table.r, table.nr, dst, dst_blobs, heat->dst_reads);
        add_counted(table.w, table.nw, dst, dst_blobs, heat->dst_writes);
        set_counting(&table, stream);
        try {
            if (src_leaf)
                copy_leaves(src, src_blobs, dst, dst_blobs, src_leaf, options, stream);
            else
                copy_ex(src, src_blobs, dst, dst_blobs, options, stream);
        } catch (...) {
            set_counting(nullptr, stream);
            throw;
        }
        set_counting(nullptr, stream);
    });
}

int llama_heatmap_begin(size_t nreads, const llama_count_range* reads, size_t nwrites,
                        const llama_count_range* writes, void* stream)
{
    return guarded([&] {
        if ((nreads && !reads) || (nwrites && !writes))
            fail(LLAMA_E_INVALID_ARG, "count range array is NULL");
        if (nreads > size_t(kCountMaxBlobs) || nwrites > size_t(kCountMaxBlobs))
            fail(LLAMA_E_UNSUPPORTED, "a Heatmap counts at most " + std::to_string(kCountMaxBlobs) +
                                          " ranges per list");
        static CountTable table;
        std::memset(&table, 0, sizeof(table));
        auto fill = [](CountBlob* out, uint32_t& n, size_t count, const llama_count_range* in) {
            for (size_t k = 0; k < count; k++) {
                if (in[k].size && (!in[k].ptr || !in[k].counters))
                    fail(LLAMA_E_INVALID_ARG, "count range " + std::to_string(k) + " has a NULL pointer");
                const uint64_t lo = uint64_t(uintptr_t(in[k].ptr));
                out[n++] = {lo, lo + in[k].size, uint64_t(uintptr_t(in[k].counters))};
            }
        };
        fill(table.r, table.nr, nreads, reads);
        fill(table.w, table.nw, nwrites, writes);
        set_counting(&table, stream);
    });
}

int llama_heatmap_end(void)
{
    return guarded([&] { set_counting(nullptr, nullptr); });
}

int llama_trace_leaves(const llama_mapping_desc* mapping, uint32_t* const* counters, uint64_t* sums, void* stream)
{
    return guarded([&] {
        need(mapping, "mapping");
        need(mapping->record, "record");
        need(counters, "counters");
        need(sums, "sums");
        trace_leaves(mapping, counters, sums, stream);
    });
}

int llama_copy_transfer(const llama_mapping_desc* src, const llama_blob* src_blobs, uint32_t src_memory,
                        const llama_mapping_desc* dst, const llama_blob* dst_blobs, uint32_t dst_memory,
                        uint64_t chunk_bytes, void* stream)
{
    return guarded(
        [&] { copy_transfer(src, src_blobs, src_memory, dst, dst_blobs, dst_memory, chunk_bytes, stream); });
}

int llama_copy_box(const llama_mapping_desc* src, const llama_blob* src_blobs, const uint64_t* src_offset,
                   const llama_mapping_desc* dst, const llama_blob* dst_blobs, const uint64_t* dst_offset,
                   const uint64_t* box, const llama_copy_options* options, void* stream)
{
    return guarded([&] { copy_box(src, src_blobs, src_offset, dst, dst_blobs, dst_offset, box, options, stream); });
}

int llama_copy_leaves(const llama_mapping_desc* src, const llama_blob* src_blobs, const llama_mapping_desc* dst,
                      const llama_blob* dst_blobs, const uint32_t* src_leaf, const llama_copy_options* options,
                      void* stream)
{
    return guarded([&] { copy_leaves(src, src_blobs, dst, dst_blobs, src_leaf, options, stream); });
}

int llama_copy(const llama_mapping_desc* src, const llama_blob* src_blobs, const llama_mapping_desc* dst,
               const llama_blob* dst_blobs, void* stream)
{
    return llama_copy_ex(src, src_blobs, dst, dst_blobs, nullptr, stream);
}

int llama_copy_naive(const llama_mapping_desc* src, const llama_blob* src_blobs, const llama_mapping_desc* dst,
                     const llama_blob* dst_blobs, void* stream)
{
    llama_copy_options o{LLAMA_PATH_NAIVE, 0, 0, 0, 0};
    return llama_copy_ex(src, src_blobs, dst, dst_blobs, &o, stream);
}

int llama_autotune(const llama_mapping_desc* src, const llama_blob* src_blobs, const llama_mapping_desc* dst,
                   const llama_blob* dst_blobs, void* stream, uint32_t reps, llama_copy_options* best,
                   double* best_gbs)
{
    return guarded([&] {
        if (reps > 1000)
            fail(LLAMA_E_INVALID_ARG, "reps must be at most 1000");
        Request rq = make_request(src, src_blobs, dst, dst_blobs, true);
        llama_copy_options o;
        double gbs = 0;
        autotune(rq, stream, reps ? int(reps) : 3, o, gbs);
        if (best)
            *best = o;
        if (best_gbs)
            *best_gbs = gbs;
    });
}

int llama_tune_lookup(const llama_mapping_desc* src, const llama_mapping_desc* dst, llama_copy_options* options,
                      int* found)
{
    return guarded([&] {
        need(options, "options");
        need(found, "found");
        Request rq = make_request(src, nullptr, dst, nullptr, false);
        llama_copy_options o{0, 0, 0, 0, 0};
        *found = tune_lookup(tune_key(rq), o) ? 1 : 0;
        *options = o;
    });
}

int llama_tune_clear(void)
{
    return guarded([&] { tune_clear(); });
}

int llama_tune_save(const char* path)
{
    return guarded([&] {
        need(path, "path");
        tune_save(path);
    });
}

int llama_tune_load(const char* path, uint32_t* entries)
{
    return guarded([&] {
        need(path, "path");
        uint32_t n = tune_load(path);
        if (entries)
            *entries = n;
    });
}

struct llama_batch {
    llama::Batch* b;
};

int llama_batch_create(size_t n, const llama_copy_item* items, const llama_copy_options* options,
                       llama_batch** batch)
{
    return guarded([&] {
        need(batch, "batch");
        *batch = nullptr;
        std::unique_ptr<llama_batch> h(new llama_batch{create_batch(n, items, options)});
        *batch = h.release();
    });
}

int llama_batch_launch(llama_batch* batch, void* stream)
{
    return guarded([&] {
        need(batch, "batch");
        launch_batch(batch->b, stream);
    });
}

int llama_batch_autotune(llama_batch* batch, void* stream, uint32_t reps, double* best_gbs)
{
    return guarded([&] {
        need(batch, "batch");
        autotune_batch(batch->b, stream, int(reps), best_gbs);
    });
}

int llama_batch_get_info(const llama_batch* batch, llama_batch_info* info)
{
    return guarded([&] {
        need(batch, "batch");
        need(info, "info");
        const Batch& b = *batch->b;
        info->items = b.items;
        info->tile_items = b.tile_items;
        info->stream_items = b.stream_items;
        info->work_units = b.total_units;
        info->read_bytes = b.read_bytes;
        info->write_bytes = b.write_bytes;
        info->threads = b.threads;
        info->wg_per_cu = b.wg_per_cu;
        info->workgroups = b.grid;
        info->lds_bytes = b.lds_bytes;
        info->launches = b.ranges.empty() ? 1u : uint32_t(b.ranges.size());
        info->reserved = 0;
    });
}

int llama_batch_destroy(llama_batch* batch)
{
    return guarded([&] {
        if (!batch)
            return;
        destroy_batch(batch->b);
        delete batch;
    });
}

int llama_copy_batch(size_t n, const llama_copy_item* items, void* stream)
{
    return guarded([&] {
        Batch* b = create_batch(n, items, nullptr);
        try {
            if (b->total_units)
                launch_batch_kernel(*b, stream);
            retire_batch(b, stream);
        } catch (...) {
            destroy_batch(b);
            throw;
        }
    });
}

int llama_copy_batch_noalloc(size_t n, const llama_copy_item* items, void* stream)
{
    return guarded([&] { copy_batch_noalloc(n, items, stream); });
}

struct llama_server {
    llama::Server* s;
};

int llama_server_create(const llama_server_config* config, llama_server** server)
{
    return guarded([&] {
        need(server, "server");
        *server = nullptr;
        *server = new llama_server{create_server(config)};
    });
}

int llama_server_create_ex(const llama_server_config* config, const llama_executor* executor, llama_server** server)
{
    return guarded([&] {
        need(server, "server");
        *server = nullptr;
        *server = new llama_server{create_server(config, executor)};
    });
}

int llama_server_submit(llama_server* server, const llama_copy_item* item, uint64_t* ticket)
{
    return guarded([&] {
        need(server, "server");
        need(ticket, "ticket");
        *ticket = server_submit(server->s, item);
    });
}

int llama_server_poll(llama_server* server, uint64_t ticket, int* done, int* status, double* latency_s)
{
    return guarded([&] {
        need(server, "server");
        need(done, "done");
        int st = 0;
        double lat = 0;
        *done = server_poll(server->s, ticket, false, st, lat) ? 1 : 0;
        if (*done && status)
            *status = st;
        if (*done && latency_s)
            *latency_s = lat;
    });
}

int llama_server_wait(llama_server* server, uint64_t ticket, int* status, double* latency_s)
{
    return guarded([&] {
        need(server, "server");
        int st = 0;
        double lat = 0;
        server_poll(server->s, ticket, true, st, lat);
        if (status)
            *status = st;
        if (latency_s)
            *latency_s = lat;
    });
}

int llama_server_get_stats(llama_server* server, llama_server_stats* stats)
{
    return guarded([&] {
        need(server, "server");
        need(stats, "stats");
        server_stats(server->s, *stats);
    });
}

int llama_server_reset_stats(llama_server* server)
{
    return guarded([&] {
        need(server, "server");
        server_reset_stats(server->s);
    });
}

int llama_server_destroy(llama_server* server)
{
    return guarded([&] {
        if (!server)
            return;
        destroy_server(server->s);
        delete server;
    });
}

} // extern "C"
