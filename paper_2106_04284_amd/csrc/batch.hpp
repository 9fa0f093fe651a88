// Batches of copies run by one persistent kernel.
#pragma once

#include <memory>
#include <vector>

#include "core.hpp"

namespace llama {

struct Batch {
    int device = 0;
    uint32_t threads = 0;
    uint32_t wg_per_cu = 0;
    uint32_t grid = 0;
    uint32_t lds_bytes = 0; // largest TILE item
    uint64_t total_units = 0;
    uint64_t items = 0, tile_items = 0, stream_items = 0;
    uint64_t read_bytes = 0, write_bytes = 0;
    void* table = nullptr; // device work table (counters, prefix, items, entries, runs)
    size_t table_bytes = 0;
    void* graph_exec = nullptr; // hipGraphExec_t of the captured launch
    BatchArgs args{};
};

// Host image of a work table, built item by item.
struct BatchTable {
    std::vector<BatchItem> items;
    std::vector<TileEntry> entries;
    std::vector<StreamRun> runs;
    std::vector<uint64_t> unit_begin; // prefix sums; the total is units
    uint64_t units = 0;
    uint32_t lds_bytes = 0;
    uint64_t tile_items = 0, stream_items = 0;
    uint64_t read_bytes = 0, write_bytes = 0;

    // plans `rq` with `threads` per workgroup and adds it; fails with
    // LLAMA_E_UNSUPPORTED for a record the tiled kernel cannot hold
    void add(const Request& rq, uint32_t threads, uint32_t tile_records, uint32_t flags = 0);
    // bytes of the serialised table
    size_t bytes() const;
    // writes the table to `host` (bytes() long) as it must lie at device
    // address `device`, and points `args` at it (counters start at zero)
    void serialise(uint8_t* host, uint64_t device, BatchArgs& args) const;
};

// LDS per workgroup that a batch item may use unless the caller fixes the
// tile size: five workgroups fit one compute unit
constexpr uint32_t kBatchLdsBytes = kHardLdsBytes / 5 - 64;

// resident workgroups per compute unit for a table run with `threads`: as
// many as LDS and wave slots allow, at most 8
uint32_t batch_wg_per_cu(uint32_t lds_bytes, uint32_t threads);
// the persistent grid: wg_per_cu (0: batch_wg_per_cu) workgroups per compute
// unit, and no more than there are units
uint32_t batch_grid(uint64_t units, uint32_t lds_bytes, uint32_t threads, uint32_t wg_per_cu);

Batch* create_batch(size_t n, const llama_copy_item* items, const llama_copy_options* opt);
void launch_batch(Batch* b, void* stream);
void destroy_batch(Batch* b);
// frees `b` once the work enqueued so far on `stream` has finished
void retire_batch(Batch* b, void* stream);

// kernels.hip
void launch_batch_kernel(const Batch& b, void* stream);

} // namespace llama
