// Batches of copies run by one persistent kernel.
#pragma once

#include <memory>
#include <vector>

#include "core.hpp"

namespace llama {

// The units of a table sorted by tile mode that share one mode key: one
// launch of the batch kernel compiled for that mode.
struct BatchRange {
    uint32_t key = 0;       // a tile mode (with kModeSplitSrc / kModeSplitDst), or long runs
    uint64_t first_unit = 0, units = 0;
    uint32_t lds_bytes = 0; // the range's largest item
};

struct Batch {
    int device = 0;
    // non-empty: one launch per mode range (a table sorted by mode), else one
    // launch of the run-time dispatching kernel
    std::vector<BatchRange> ranges;
    std::vector<Request> work; // the copies the table holds (a Split item as its part copies)
    uint32_t flags = 0;        // LLAMA_COPY_* bits of the batch
    uint32_t tile_records = 0; // fixed tile size (0: each item's own)
    uint32_t lds_budget = 0;   // LDS a tiled item's plan may take (without a fixed tile size)
    uint32_t threads = 0;
    uint32_t wg_per_cu = 0; // persistent: workgroups per compute unit; 0: one workgroup per work unit
    uint32_t grid = 0;
    uint32_t lds_bytes = 0; // largest TILE item
    uint64_t total_units = 0;
    uint64_t items = 0, tile_items = 0, stream_items = 0;
    uint64_t read_bytes = 0, write_bytes = 0;
    void* table = nullptr; // device work table (counters, prefix, hints, items, entries, runs)
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
    // LDS classes of the items: bit 0 long runs, bit c >= 1 tiles of at
    // most 2^(c + 9) bytes of LDS
    uint32_t classes = 0;

    // plans `rq` with `threads` per workgroup and adds it; fails with
    // LLAMA_E_UNSUPPORTED for a record the tiled kernel cannot hold
    void add(const Request& rq, uint32_t threads, uint32_t tile_records, uint32_t flags = 0,
             uint32_t lds_budget = 0);
    // adds an item planned by batch_plan
    void add_plan(const Plan& p);
    // reorders the items by tile mode (stable) and returns the mode ranges
    std::vector<BatchRange> sort_by_mode();
    // bytes of the serialised table
    size_t bytes() const;
    // writes the table to `host` (bytes() long) as it must lie at device
    // address `device`, and points `args` at it (counters start at zero)
    void serialise(uint8_t* host, uint64_t device, BatchArgs& args) const;
};

// The default launch of a batch (and of the allocation-free batch): one
// launch per tile mode over a table sorted by mode, each mode in its own
// compiled kernel (the 1,000-array batch: 4.26 -> 5.0 TB/s over one launch of
// the run-time dispatching kernel); a persistent grid (wg_per_cu) keeps the
// one dispatching launch
constexpr bool kBatchByModeDefault = true;

// LDS per workgroup that a batch item may use unless the caller fixes the
// tile size: five workgroups fit one compute unit
constexpr uint32_t kBatchLdsBytes = kHardLdsBytes / 5 - 64;

// How a table runs: one workgroup per work unit when its items share one LDS
// class, else a persistent grid (see create_batch).
bool batch_per_unit(const BatchTable& t);
// resident workgroups per compute unit of a persistent grid: as many as LDS
// and wave slots allow, at most 8
uint32_t batch_wg_per_cu(uint32_t lds_bytes, uint32_t threads);
// The grid of a batch launch: wg_per_cu 0 launches one workgroup per work
// unit (at most kBatchMaxGrid workgroups, which then loop over the units);
// 1 .. 16 a persistent grid of that many workgroups per compute unit, no
// more than there are units.
constexpr uint64_t kBatchMaxGrid = uint64_t(1) << 24;
uint32_t batch_grid(uint64_t units, uint32_t wg_per_cu);

// the plan of a batch item (see BatchTable::add)
// (lds_budget 0: kBatchLdsBytes)
Plan batch_plan(const Request& rq, uint32_t threads, uint32_t tile_records, uint32_t flags, uint32_t lds_budget = 0);

// validates the items and plans them into one work table (nothing on the device)
BatchTable build_batch_table(size_t n, const llama_copy_item* items, const llama_copy_options* opt,
                             uint32_t& threads, std::vector<Request>* work = nullptr);
// llama_batch_autotune: times candidate LDS budgets, thread counts and grids
// on the batch's own blobs, keeps those whose output hashes like the current
// plan's, and re-plans the batch with the fastest
void autotune_batch(Batch* b, void* stream, int reps, double* best_gbs);
Batch* create_batch(size_t n, const llama_copy_item* items, const llama_copy_options* opt);
// llama_copy_batch_noalloc: the work table goes into the library's static
// device buffer (kScratchBytes) instead of an allocation
void copy_batch_noalloc(size_t n, const llama_copy_item* items, void* stream);
void launch_batch(Batch* b, void* stream);
void destroy_batch(Batch* b);
// frees `b` once the work enqueued so far on `stream` has finished
void retire_batch(Batch* b, void* stream);

// Size of the library's static device buffer for the work table of
// llama_copy_batch_noalloc (one per device, held until the process ends).
constexpr size_t kScratchBytes = size_t(8) << 20;

// kernels.hip
void launch_batch_kernel(const Batch& b, void* stream);
// one launch per mode range of a table sorted by mode
void launch_batch_ranges(const BatchArgs& args, const std::vector<BatchRange>& ranges, uint32_t threads,
                         void* stream);
// the mode key of an item (batch_mode_kernel's Mode)
uint32_t batch_mode_key(const BatchItem& it);
void launch_batch_args(const BatchArgs& args, uint32_t grid, uint32_t threads, uint32_t lds_bytes, bool persistent,
                       void* stream);
// device address of the current device's static work-table buffer
// (resolved with hipGetSymbolAddress on the first call on each device)
uint64_t scratch_address();

} // namespace llama
