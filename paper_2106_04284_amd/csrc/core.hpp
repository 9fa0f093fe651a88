// Host-side core of the layout-aware copy: record flattening, the affine form
// of each mapping, validation and the copy planner.
#pragma once

#include <cstdint>
#include <string>
#include <memory>
#include <vector>

#include "llama_mi355x.h"
#include "kernel_args.hpp"

namespace llama {

// A status with its message; thrown inside the library, converted to a return
// code and a thread-local message at the C boundary.
struct Error {
    int status;
    std::string message;
};
[[noreturn]] void fail(int status, const std::string& message);

// One leaf of a flattened record (sec. 3.3: leaves in depth-first declaration
// order; sec. 3.7: sizes and offsets in the record dimension).
struct Leaf {
    uint32_t size;
    uint32_t align;
    uint64_t packed_offset;  // sum of the sizes of the leaves before it
    uint64_t aligned_offset; // next multiple of align after the previous leaf's end
};

struct Record {
    std::vector<Leaf> leaves;
    uint64_t packed_size = 0;  // S
    uint64_t aligned_size = 0; // R
    uint32_t max_align = 1;
};

Record flatten(const llama_record_desc* desc);
bool same_leaves(const Record& a, const Record& b);
// the record of leaves `pick` of `r` (in that order), offsets recomputed
Record sub_record(const Record& r, const std::vector<uint32_t>& pick);

// The affine form of a mapping (sec. 3.7 blobNrAndOffset): leaf f of the
// record with row-major linear index i lives in blob `blob[f]` at
//     base[f] + (i / L) * K + (i % L) * size[f]     (blocked, L >= 1)
//     base[f] + i * size[f]                          (unblocked, L == 0)
// AoS packed is blocked with L = 1, K = S; AoS aligned L = 1, K = R; AoSoA
// L = lanes, K = lanes * S; both SoA kinds are unblocked.
struct Side {
    uint32_t kind = 0;
    uint32_t rank = 0;
    uint64_t extents[LLAMA_MAX_RANK] = {};
    // the linearizer (llama_linearizer; rank 1: always row-major) and, for
    // Morton order, the bits per dimension of the index
    uint32_t lin = LLAMA_ROW_MAJOR;
    uint32_t morton_bits = 0;
    uint64_t records = 0; // coordinates: the product of the extents
    uint64_t n = 0;     // linear indices laid out: the records, or with Morton order the last
                        // coordinate's index + 1 (indices no coordinate reaches are padding)
    uint64_t lanes = 0; // L (0: unblocked)
    uint64_t block = 0; // K
    uint64_t npad = 0;  // records the blob spans, trailing AoSoA lanes included
    std::vector<uint32_t> blob;
    std::vector<uint64_t> base;
    std::vector<uint64_t> blob_size;
    // byte ranges inside one record that no leaf covers (aligned AoS only):
    // (offset, length) pairs
    std::vector<std::pair<uint64_t, uint64_t>> gaps;
    // LLAMA_SPLIT (sec. 3.7): each leaf keeps its part's L and K; a Split side
    // describes offsets only and is copied part by part (split_copies)
    std::vector<uint64_t> leaf_lanes, leaf_block;
    // a side of one part-to-part copy whose leaves leave other bytes of its
    // records to other copies: never treated as one whole-blob copy
    bool partial = false;
    // LLAMA_SOA_ALIGNED: the byte ranges between sub-arrays (blob, offset,
    // length), padding that belongs to no record
    struct BlobGap {
        uint32_t blob;
        uint64_t offset, length;
        bool operator==(const BlobGap& o) const { return blob == o.blob && offset == o.offset && length == o.length; }
    };
    std::vector<BlobGap> blob_gaps;
    bool has_padding() const { return !gaps.empty() || npad != n || !blob_gaps.empty(); }
    uint64_t offset(uint64_t i, uint32_t f, const Record& r) const
    {
        const uint64_t L = leaf_lanes.empty() ? lanes : leaf_lanes[f];
        const uint64_t K = leaf_block.empty() ? block : leaf_block[f];
        if (L == 0)
            return base[f] + i * r.leaves[f].size;
        return base[f] + (i / L) * K + (i % L) * r.leaves[f].size;
    }
};

Side make_side(const llama_mapping_desc* m, const Record& r);

// the linear index of coordinate c on side s (its linearizer)
uint64_t linearize(const Side& s, const uint64_t* c);

// One chunk of a virtual source block (a source gathered from several parts,
// kTileVirtualSrc): a whole block of a record-major part, or the L values of
// one leaf of a field-major part.
struct SrcChunk {
    uint64_t addr;         // device address of the chunk in virtual block 0
    uint64_t block_stride; // device bytes from one virtual block to the next
    uint32_t offset;       // byte offset in a virtual block
    uint32_t bytes;
    uint32_t per_record;   // 0: a whole part block; else the leaf's bytes per record
};

// A validated copy request: both sides plus device addresses.
struct Request {
    Record record;
    Side src, dst;
    std::vector<uint64_t> src_ptr, dst_ptr; // device addresses of the blobs
    // non-empty: the source is gathered from several parts, and src is a
    // record-major side of virtual blocks whose leaves sit at their chunk's
    // place (planned as TILE only)
    std::vector<SrcChunk> chunks;
    // non-empty: the destination is scattered over several parts, and dst is
    // a record-major side of L lanes whose leaf j's runs of L values lie
    // dst_stride[j] bytes apart in its own part (planned as a direct-store
    // tile only); dst_values_only[j]: an SoA leaf, written for records with
    // values only
    std::vector<uint32_t> dst_stride;
    std::vector<uint8_t> dst_values_only;
};

// Checks a side's blob array (sizes, NULL pointers, address overflow) and
// collects the device addresses.
void check_blobs(const char* which, const Side& s, const llama_blob* blobs, std::vector<uint64_t>& ptrs);

// Validates descriptors (and blobs when given) and builds the request.  A
// Split side fails with LLAMA_E_UNSUPPORTED unless `allow_split`.
Request make_request(const llama_mapping_desc* src, const llama_blob* src_blobs, const llama_mapping_desc* dst,
                     const llama_blob* dst_blobs, bool need_blobs, bool allow_split = false);

// One part-to-part copy of a copy with a Split side: the leaves both parts
// hold, from the source part to the destination part.  `naive`: it writes part
// of the records of a record-major destination part, so only the element-wise
// path writes nothing but its own leaves.
struct Plan;
struct SubCopy {
    Request rq;
    bool naive = false;
    // a copy from several source parts at once, or into several destination
    // parts at once, already planned (`plan`)
    bool gathered = false;
    std::shared_ptr<Plan> plan;
};
// The part-to-part copies of `whole` (made with allow_split), destination part
// by destination part; a plain side is one part holding every leaf.  The
// padding of a destination part is written by the first copy into it.  With
// `gather`, a destination part fed by several source parts is copied by one
// tile copy whose source gathers those parts (when their layouts allow it and
// a plan with `options` exists), instead of one copy per source part.
std::vector<SubCopy> split_copies(const llama_mapping_desc* src, const llama_mapping_desc* dst, const Request& whole,
                                  bool gather = false, const llama_copy_options* options = nullptr);

// llama_copy_leaves (leaves.cpp): validates and plans the copy between
// differing records (without `need_blobs`: plans only, for distinct blobs
// aligned to 256 bytes).
struct Plan;
std::vector<Plan> leaves_plans(const llama_mapping_desc* src, const llama_blob* src_blobs,
                               const llama_mapping_desc* dst, const llama_blob* dst_blobs, const uint32_t* src_leaf,
                               const llama_copy_options* options, bool need_blobs);
// ... and enqueues its launches.
void copy_leaves(const llama_mapping_desc* src, const llama_blob* src_blobs, const llama_mapping_desc* dst,
                 const llama_blob* dst_blobs, const uint32_t* src_leaf, const llama_copy_options* options,
                 void* stream);

// A complete launch plan for one copy.
struct Plan {
    uint32_t path = LLAMA_PATH_EMPTY;
    uint32_t threads = 256;
    uint64_t workgroups = 0;
    uint32_t lds_bytes = 0;
    uint32_t wg_per_cu = 0;
    uint64_t tiles = 0;
    uint32_t flags_in = 0; // llama_copy_options.flags of the request
    uint64_t read_bytes = 0, write_bytes = 0;
    TileArgs tile{};     // path == TILE
    StreamArgs stream{}; // path == STREAM
    NaiveArgs naive{};   // path == NAIVE
    BoxArgs box{};       // path == BOX (box_naive: its element-wise baseline)
    bool box_naive = false;
    // a launch that follows this one: the zero fill of the padding between a
    // destination's aligned SoA sub-arrays (a STREAM plan of zero runs)
    std::shared_ptr<Plan> then;
};

Plan make_plan(const Request& rq, const llama_copy_options* opt);
// the zero fill of the padding between a destination's aligned SoA
// sub-arrays (rq.dst.blob_gaps), as STREAM plans chained through `then`
Plan zero_fill_plan(const Request& rq);

// A copy whose records sit at different linear indices on the two sides
// (differing linearizers, or Morton indices that no coordinate reaches): it
// runs through the box kernel (box.cpp), not the linear-index planner.
bool needs_box(const Request& rq);

// Plans of the box kernel for a box copy (sec. 3.2 VirtualView, sec. 3.9) or,
// with `full`, for a whole copy between views whose linearizers differ: the
// box launch, then (full copies into AoSoA) a zero fill of the lanes past the
// last index.  rq's sides may have different extents; so / dof / box give
// the box in each view's coordinates.
std::vector<Plan> make_box_plans(const Request& rq, const uint64_t* so, const uint64_t* dof, const uint64_t* box,
                                 bool full, const llama_copy_options* opt);

// llama_copy_transfer (transfer.cpp): validates, plans and enqueues.
void copy_transfer(const llama_mapping_desc* src, const llama_blob* src_blobs, uint32_t src_memory,
                   const llama_mapping_desc* dst, const llama_blob* dst_blobs, uint32_t dst_memory,
                   uint64_t chunk_bytes, void* stream);

// llama_copy_box (box.cpp): validates, plans and enqueues.
void copy_box(const llama_mapping_desc* src, const llama_blob* src_blobs, const uint64_t* src_offset,
              const llama_mapping_desc* dst, const llama_blob* dst_blobs, const uint64_t* dst_offset,
              const uint64_t* box, const llama_copy_options* options, void* stream);

constexpr uint32_t kPlanNoDirect = LLAMA_COPY_NO_DIRECT;
constexpr uint32_t kPlanNoSplit = LLAMA_COPY_NO_SPLIT;
constexpr uint32_t kPlanPreserve = LLAMA_COPY_PRESERVE_PADDING;
constexpr uint32_t kPlanNoGather = LLAMA_COPY_NO_GATHER;
constexpr uint32_t kCopyFlags =
    LLAMA_COPY_NO_DIRECT | LLAMA_COPY_NO_SPLIT | LLAMA_COPY_PRESERVE_PADDING | LLAMA_COPY_NO_GATHER; // every bit
// the flags that change only speed, which the tuner may choose and cache
constexpr uint32_t kTuneFlags = LLAMA_COPY_NO_DIRECT | LLAMA_COPY_NO_SPLIT | LLAMA_COPY_NO_GATHER;

// LLAMA_TRACE set in the environment (to anything but "0"): every launch
// writes one line describing its plan to stderr
bool trace_enabled();
void trace_plan(const Plan& p);

// kernels.hip
void launch(const Plan& p, void* stream);
// table != NULL: uploads the Heatmap's count table on `stream` and makes
// this thread's launches take the counted kernel variants; NULL: plain again
void set_counting(const CountTable* table, void* stream);
// llama_trace_leaves: per-leaf sums of a view's per-byte counters
// (sums[0 .. F-1]) and the sum over the bytes no leaf owns (sums[F])
void trace_leaves(const llama_mapping_desc* m, uint32_t* const* counters, uint64_t* sums, void* stream);
uint32_t device_cu_count(); // compute units of the current device (256 when none is visible)
// adds a 64-bit hash of bytes [p, p + len) to *acc (device memory), on `stream`
void launch_hash(const void* p, uint64_t len, unsigned long long* acc, void* stream);

// The tuning cache (tune.cpp): kernel parameters measured fastest for a class
// of copies (same leaves, same source and destination kind and lanes, same
// power-of-two size bucket).
struct TuneKey {
    uint64_t leaves;   // hash of the flattened leaf sizes and alignments
    uint32_t src_kind, dst_kind;
    uint64_t src_lanes, dst_lanes;
    uint32_t bucket;   // floor(log2(records))
    bool operator<(const TuneKey& o) const;
};
TuneKey tune_key(const Request& rq);
bool tune_lookup(const TuneKey& k, llama_copy_options& out);
void autotune(const Request& rq, void* stream, int reps, llama_copy_options& best, double& best_gbs);
void tune_clear();
void tune_save(const char* path);
uint32_t tune_load(const char* path);
uint32_t tune_size();

// default kernel parameters
constexpr uint32_t kDefaultThreads = 256;      // threads per workgroup
constexpr uint32_t kDefaultTileBytes = 16384;  // TILE: target source bytes per tile
constexpr uint32_t kMaxLdsBytes = 65536;       // TILE: LDS budget per workgroup for the default plan
constexpr uint32_t kHardLdsBytes = 160 * 1024; // LDS of one gfx950 compute unit
constexpr uint32_t kMaxWavesPerCu = 32;
// TILE: destinations of at least this many bytes get nontemporal stores
// (4x the 256 MB Infinity Cache, which then holds at most a quarter of them)
constexpr uint64_t kStreamStoreBytes = uint64_t(1) << 30;
// sources of at least this many bytes (the Infinity Cache) get nontemporal
// loads: smaller ones may still sit in that cache
constexpr uint64_t kStreamLoadBytes = uint64_t(256) << 20;

} // namespace llama
