// Kernel argument blocks shared by the host planner and the HIP kernels.
// Everything here is plain data passed by value as kernel arguments (each
// block stays below the 4 KiB kernel-argument limit).
#pragma once

#include <cstdint>

namespace llama {

// ---------------------------------------------------------------------------
// TILE: records [i0, i0 + T) of one tile are staged through LDS.
//
// A side is "record-major" when its lanes L satisfy 1 <= L <= T: the tile is
// then one contiguous span of (T / L) blocks.  Otherwise (unblocked SoA, or
// L > T) it is "field-major": the tile is one span of T values per leaf.
// ---------------------------------------------------------------------------

constexpr int kTileMaxEntries = 150;

enum : uint32_t { kRecordMajor = 0, kFieldMajor = 1 };

struct TileSide {
    uint64_t span_base; // record-major: device address of the blob
    uint64_t lanes;     // L (0: unblocked)
    uint64_t block;     // K: bytes per block
    uint32_t mode;      // kRecordMajor / kFieldMajor
    uint32_t log2_lanes;
    uint32_t lds_base;  // byte offset of this side's LDS region
    uint32_t lds_bytes; // bytes of this side's LDS region
};

// One entry of the remap: a leaf (source and destination), or a zero-filled
// destination gap inside every record (aligned AoS padding, src_addr == 0).
struct TileEntry {
    uint64_t src_addr; // leaf: device address of blob + base offset; gap: 0
    uint64_t dst_addr; // device address of blob + base offset
    uint32_t size;     // bytes per record
    uint16_t src_lds16; // field-major source: LDS offset of this leaf's span / 16
    uint16_t dst_lds16; // field-major destination: LDS offset of this leaf's span / 16
};

struct TileArgs {
    uint64_t n;         // records with values
    uint64_t npad;      // records the destination spans (>= n)
    uint64_t num_tiles; // ceil(npad / T)
    uint32_t log2_tile; // T = 1 << log2_tile
    uint32_t num_leaves;
    uint32_t num_entries; // leaves, then gaps
    uint32_t lds_bytes;
    TileSide src, dst;
    TileEntry e[kTileMaxEntries];
};

// ---------------------------------------------------------------------------
// STREAM: contiguous byte runs copied with 16-byte accesses; a run with
// src == 0 is filled with zeros.  Every run has src and dst congruent
// modulo 4.
// ---------------------------------------------------------------------------

constexpr int kStreamMaxRuns = 120;
constexpr uint32_t kStreamChunkLog2 = 16; // 64 KiB per workgroup

struct StreamRun {
    uint64_t src;
    uint64_t dst;
    uint64_t bytes;
    uint64_t first_chunk; // exclusive prefix sum of chunk counts
};

struct StreamArgs {
    uint32_t num_runs;
    uint32_t pad;
    uint64_t num_chunks;
    StreamRun r[kStreamMaxRuns];
};

// ---------------------------------------------------------------------------
// NAIVE: one thread per record, mapping arithmetic with run-time '/' and '%'.
// ---------------------------------------------------------------------------

constexpr int kNaiveMaxEntries = 120;

struct NaiveSide {
    uint64_t lanes; // 0: unblocked
    uint64_t block;
};

struct NaiveEntry {
    uint64_t src_addr; // blob + base (0 for a gap)
    uint64_t dst_addr;
    uint32_t size;
    uint32_t width; // bytes per load/store: largest power of two dividing every address
};

struct NaiveArgs {
    uint64_t n;
    uint64_t npad;
    uint32_t num_leaves;
    uint32_t num_entries;
    NaiveSide src, dst;
    NaiveEntry e[kNaiveMaxEntries];
};

} // namespace llama
