// Kernel argument blocks shared by the host planner and the HIP kernels.
// Everything here is plain data passed by value as kernel arguments (each
// block stays below the 4 KiB kernel-argument limit).
#pragma once

#include <cstdint>

#include "llama_mi355x.h"

namespace llama {

// ---------------------------------------------------------------------------
// TILE: records [i0, i0 + T) of one tile are staged through LDS.
//
// A side is "record-major" when its lanes L satisfy 1 <= L <= T: the tile is
// then one contiguous span of (T / L) blocks.  Otherwise (unblocked SoA, or
// L > T) it is "field-major": the tile is one span of T values per leaf.
// ---------------------------------------------------------------------------

constexpr int kTileMaxEntries = 118;

enum : uint32_t { kRecordMajor = 0, kFieldMajor = 1 };

// T is a power of two >= 16, so every tile starts at the same offset modulo
// 16 inside each span; LDS positions are therefore the same for every tile
// and are computed once on the host.
struct TileSide {
    uint64_t span_base;  // record-major: device address of the blob
    uint64_t tile_bytes; // record-major: bytes of one full tile, (T / L) * K
    uint64_t block;      // K: bytes per block
    uint64_t lanes;      // L (0: unblocked)
    uint32_t mode;       // kRecordMajor / kFieldMajor
    uint32_t log2_lanes;
    uint32_t lds_base;   // byte offset of this side's LDS region
    uint32_t lds_bytes;  // bytes of this side's LDS region
    // LDS position of record r of an entry: pos + (r >> pos_lg) * pos_k + (r & pos_m) * size
    uint32_t pos_lg, pos_k, pos_m, pad;
};

// One entry of the remap: a leaf, or a destination gap inside every record
// (aligned AoS padding) that is filled with zeros.
struct TileEntry {
    uint64_t src_addr; // field-major source: device address of the leaf's values (blob + base); 0 for a gap
    uint64_t dst_addr; // field-major destination: device address of the leaf's values
    uint32_t src_pos;  // LDS byte of record 0 in the source region (region offset and 16-byte phase
                       // included); with kTileDirectLoad, the leaf's first granule slot
    uint32_t dst_pos;  // LDS byte of record 0 in the destination region
    uint32_t size;     // bytes per record
    uint32_t move;     // bits 0-2: log2 of the move width (1 .. 16 bytes); bit 3: split move
                       // (kMoveSplit); bits 4-7: first loading wave of this leaf's source span;
                       // bits 8-19: first storing thread of this leaf's destination span;
                       // bits 20-22: log2 of the read alignment; bits 24-26: log2 of the write
                       // alignment (split moves); with kTileDirectStore, bits 20-23: the
                       // destination span's phase in values, (dst_addr mod 16) / size;
                       // bit 31: gap (write zeros)
};

// A leaf of 2, 4 or 8 bytes whose source or destination positions are aligned
// to less than 4 bytes (a packed record of odd size): each value is read
// whole (from the 4-byte words that hold it, when the source is misaligned)
// and written in pieces of the destination's alignment, instead of moving
// every byte on its own.
constexpr uint32_t kMoveSplit = 1u << 3;

// kTileGatherStore: where the words of the destination find their sources.
// The word table covers a super-block: 1, 2 or 4 destination blocks (2^lg
// records), enough that its bytes, and the source bytes that its records
// advance by, are whole 4-byte words.  A word's bytes come in pieces: bytes
// that are one 4-byte window of the source region in every super-block.  A
// piece entry holds the LDS byte p0 that the word's byte 0 lines up with in
// super-block 0 (bits 0-17; the window is read from the two aligned words
// that hold it), log2 of the bytes of 2^lg values of its leaf (run, bits
// 18-22; 0 when q = 0) and the word bytes it gives (bits 23-26).  Entry w of
// the table describes word w of super-block 0:
//   bits 31-30 = 00:  the word is one piece, this entry (no byte: padding);
//   bits 31-30 = 01:  two pieces, the entries at table index bits 0-15;
//   bits 31-30 = 10:  three or four pieces: four entries at index bits 0-15
//                     (16-byte aligned) give its bytes one by one, entry k the
//                     LDS byte p0 of byte k in super-block 0 and its run in
//                     the same bits (bit 31: a zero byte).
// The word entries are padded to a multiple of 4; the groups of four follow,
// then the pairs.  Records without values (tail lanes of the last AoSoA
// block) are cleared in the source region before the tile's words are read.
// The table follows the entries: in the argument block at entry num_entries
// (reinterpreted as 32-bit words), in a batch after the item's entries; in
// LDS it sits at dst.lds_base, 16-byte aligned.  A piece of super-block b lies
// at LDS byte
//   p0 + (b >> q) * kq + ((b & (2^q - 1)) << run)
// (a source with at most 2^lg lanes per block: q = 0 and kq the source bytes
// of 2^lg records; a source with more: q = log2 of its lanes over 2^lg (31
// for a field-major source) and kq the source block).  Six words, so that the
// argument block keeps its size (the hidden arguments behind it moving by 8
// bytes measured 4-13% slower on some direct-store pairs).
struct TileGather {
    uint32_t words; // 4-byte words per destination super-block
    uint32_t magic; // ceil(2^32 / words): u / words == mulhi(u, magic) for u * words < 2^32
    uint32_t q, lg; // lg: log2 of the records of a super-block
    uint32_t kq;
    uint32_t table; // 32-bit words of the table: word entries, groups of four, pairs
};

struct TileHeader {
    uint64_t n;         // records with values
    uint64_t npad;      // records the destination spans (>= n)
    uint64_t num_tiles; // ceil(npad / T)
    uint32_t log2_tile; // T = 1 << log2_tile
    uint32_t num_leaves;
    uint32_t num_entries; // leaves, then gaps
    uint32_t lds_bytes;
    uint32_t flags;       // kTileDirectStore, kTileDirectLoad, kTilePreserve, kTileGatherStore,
                          // kTileStreamStores, kTileStreamLoads, kTileGatherOdd, kTileVirtualSrc,
                          // kTileVirtualDst, kTileSplitSrc, kTileSplitDst
    uint32_t slots;       // kTileDirectLoad: granule slots of a tile (a multiple of 64);
                          // kTileVirtualSrc: the chunks after the entries
    TileSide src, dst;
};

// Destination field-major with 16-byte aligned leaf spans and leaf sizes of 1,
// 2, 4, 8 or 16 bytes: every 16-byte granule of a destination span holds whole
// values of one leaf, gathered straight from the source region into registers
// and stored; the tile needs no destination region in LDS.
constexpr uint32_t kTileDirectStore = 1;

// Source field-major with 16-byte aligned leaf spans and leaf sizes of 4, 8
// or 16 bytes: every thread loads its granules of the source spans into
// registers (all loads of the tile in flight at once) and writes the values to
// their destination positions in LDS; the tile needs no source region.  Leaf f
// owns slots [src_pos, src_pos + 64 * ceil(G_f / 64)) of the tile's granule
// slots (G_f granules of 16 bytes), so each wave's slot lies in one leaf;
// thread t takes slots t + j * threads, j < kDirectLoadSlots.
constexpr uint32_t kTileDirectLoad = 2;
constexpr uint32_t kDirectLoadSlots = 8;

// Destination padding keeps its bytes: no zeros are written; a record-major
// destination region is loaded from the destination before the values move
// in (never combined with kTileDirectLoad), and field-major spans are stored
// only for records with values.
constexpr uint32_t kTilePreserve = 4;

// Destination record-major (AoS, or AoSoA with L_d <= 128 lanes) with blocks
// of whole 4-byte words and 16-byte aligned tile spans: the source is staged
// in LDS as usual, then every thread assembles whole 16-byte granules of the
// destination span word by word from the source region (the word table maps
// each word to its source, or to the sources of its 4 bytes) and stores
// them; the tile needs no destination region and no second barrier.  A
// source with more lanes per block than the destination (field-major
// included) needs leaf sizes that are powers of two.
constexpr uint32_t kTileGatherStore = 8;
constexpr uint32_t kGatherMaxWords = 4096; // words per super-block (16 KiB of word entries in LDS)
constexpr uint32_t kGatherMaxLanes = 128;
// the gather store takes a tile while its words average at most
// kGatherMaxReadsPct / 100 piece reads (a word of two pieces reads 2, of three
// or four 4).  Measured against the mode taken without it (staged or direct
// load): 1.00 to 1.38 reads gain up to 140% (particle, lattice-Boltzmann,
// mixed and listing 1 records; one pair -1%), 1.48 gains 22% (listing 1
// aligned into packed AoS), 1.52 gives -17 to +9% (listing 1's u16 and bool
// lanes into AoSoA), 1.65 and more lose 24-27% to the direct load (the
// 49-byte packed mixed record and listing 1's from SoA or AoSoA)
constexpr uint32_t kGatherMaxReadsPct = 150;

// The tile's 16-byte destination stores carry the nontemporal hint: set for
// destinations several times larger than the 256 MB Infinity Cache.
constexpr uint32_t kTileStreamStores = 16;
// The tile's source loads carry the nontemporal hint: set for sources at
// least as large as the Infinity Cache.
constexpr uint32_t kTileStreamLoads = 32;
// A gathering tile whose destination blocks are not whole words (a packed
// record of odd size: a span can end inside a word, whose bytes are written
// one by one): the gather runs in its own kernel variant, so that the common
// case keeps its registers.
constexpr uint32_t kTileGatherOdd = 64;

// A source gathered from several parts (a Split source, sec. 3.7): the tile's
// source region is a run of virtual blocks of L records and K bytes (h.src
// describes them as a record-major side with lanes L and block K), and every
// virtual block is assembled from chunks that each come from one contiguous
// global range: a whole block of an AoSoA (or AoS) part with L lanes, or the
// L values of one leaf of an SoA part.  The chunks (h.slots of them, in the
// order of their place in a virtual block) follow the entries and gaps as
// TileEntry-sized records read with these meanings:
//   src_addr: global address of the chunk in virtual block 0 of tile 0;
//   dst_addr: global bytes from one virtual block to the next;
//   src_pos:  byte offset of the chunk in a virtual block (a multiple of 16);
//   dst_pos:  unused;
//   size:     bytes of the chunk (a multiple of 16);
//   move:     0 for a whole part block, else the bytes per record of a leaf
//             chunk, which is read only for records with values.
// Tile t starts T / L virtual blocks after tile t - 1.  h.src.pad holds
// ceil(2^32 / (K / 16)) for the division of a granule index by the granules
// per virtual block.  Direct load is never combined with it.
constexpr uint32_t kTileVirtualSrc = 128;
constexpr uint32_t kTileMaxChunks = 32;

// A destination scattered over several parts (a Split destination, sec.
// 3.7), stored in direct-store mode only: every leaf's values of a tile are
// runs of L values (L * size a multiple of 16 bytes) in its own part, one run
// per L records, `dst_pos` bytes apart (an AoSoA part's block, or L values of
// an SoA leaf); dst_addr is the leaf's first value.  A leaf of an SoA part
// (kMoveValuesOnly in `move`) ends at the last record with values; an AoSoA
// part's tail lanes are zero.
constexpr uint32_t kTileVirtualDst = 256;
constexpr uint32_t kMoveValuesOnly = 1u << 30;

// Direct store from a source whose values sit below their size's alignment (a
// packed record of odd size): leaves of 2, 4 or 8 bytes whose source position
// is aligned to 2^a < size only carry a in bits 24-26 of `move` and are read
// from the aligned 4-byte words that hold them.
constexpr uint32_t kTileSplitSrc = 512;
// Direct load into a destination region whose values sit below their size's
// alignment, or with leaves of 1 or 2 bytes: every value is written into the
// region in pieces of its alignment (bits 24-26 of `move`: log2 of it).
constexpr uint32_t kTileSplitDst = 1024;

// The gather geometry follows the entries, so that the header and entries
// keep their offsets in the argument block (entries 16-byte aligned; a
// header grown by 24 bytes measured 3-5% slower for the other modes).  The
// word table follows the entries, gaps and chunks.
struct TileArgs {
    TileHeader h;
    TileEntry e[kTileMaxEntries];
    TileGather gather; // kTileGatherStore
};
static_assert(sizeof(TileArgs) <= 4096, "kernel arguments are limited to 4 KiB");

// ---------------------------------------------------------------------------
// STREAM: contiguous byte runs copied with 16-byte accesses; a run with
// src == 0 is filled with zeros.  Every run has src and dst congruent
// modulo 4.
// ---------------------------------------------------------------------------

constexpr int kStreamMaxRuns = 120;
constexpr uint32_t kStreamChunkLog2 = 12;      // 4 KiB per workgroup (a single copy)
constexpr uint32_t kBatchStreamChunkLog2 = 14; // 16 KiB per work unit of a batch

struct StreamRun {
    uint64_t src;
    uint64_t dst;
    uint64_t bytes;
    uint64_t first_chunk; // exclusive prefix sum of chunk counts
};

// StreamArgs.flags: the source loads carry the nontemporal hint
constexpr uint32_t kStreamLoadsOnce = 1;

struct StreamArgs {
    uint32_t num_runs;
    uint32_t flags; // kStreamLoadsOnce
    uint64_t num_chunks;
    StreamRun r[kStreamMaxRuns];
};
static_assert(sizeof(StreamArgs) <= 4096, "kernel arguments are limited to 4 KiB");

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
    uint32_t preserve; // 1: padding keeps its bytes (gap entries and records >= n are skipped)
    uint32_t pad;
    NaiveSide src, dst;
    NaiveEntry e[kNaiveMaxEntries];
};
static_assert(sizeof(NaiveArgs) <= 4096, "kernel arguments are limited to 4 KiB");

// ---------------------------------------------------------------------------
// BATCH: many copies in one persistent launch whose workgroups take blocks of
// work units from counters[0] until none is left.  The work table lives in
// device memory;
// work unit g (a tile of a TILE item, a 4 KiB chunk of a STREAM item) belongs
// to the item j with unit_begin[j] <= g < unit_begin[j + 1].
// ---------------------------------------------------------------------------

enum : uint32_t { kItemTile = 0, kItemStream = 1 };

struct BatchItem {
    uint32_t kind;  // kItemTile / kItemStream
    uint32_t count; // entries (TILE; the gather word table after them included) or runs (STREAM)
    uint64_t first; // index of the item's first entry or run
    TileHeader h;   // TILE: the tile geometry; STREAM: h.num_tiles = chunks
    TileGather gather; // TILE with kTileGatherStore
    uint32_t pad[2];
};

// hint[c] = the item of work unit c << kBatchHintLog2 (the one-workgroup-
// per-unit launch searches only the items between two hints: at most 5
// dependent table loads where items hold one unit each, as the frames of a
// particle-in-cell batch do, instead of 10 with a hint every 1,024 units)
constexpr uint32_t kBatchHintLog2 = 5;

struct BatchArgs {
    const uint64_t* unit_begin; // num_items + 1 prefix sums of work units
    const uint32_t* hint;       // ceil(total_units / 2^kBatchHintLog2) + 1 item indices
    const BatchItem* items;
    const TileEntry* entries;
    const StreamRun* runs;
    unsigned long long* counters; // [0]: next work unit, [1]: workgroups finished
    uint64_t total_units;
    uint32_t num_items;
    uint32_t flags; // kBatchLoadsOnce
};

// BatchArgs.flags: the source loads carry the nontemporal hint
constexpr uint32_t kBatchLoadsOnce = 1;

// ---------------------------------------------------------------------------
// BOX: copies whose records sit at different linear indices on the two sides:
// a box of the array dimensions between views of different extents (sec. 3.2
// VirtualView, sec. 3.9), or views whose linearizers differ (sec. 3.7).
//
// A work unit is a tile: a box of 2^qlog[d] coordinates per dimension,
// clipped to the copy's box.  Each side walks the tile's records as runs of
// consecutive linear indices of its own order:
//   kOrderRow     runs along the last dimension (row-major side);
//   kOrderCol     runs along the first dimension (column-major side);
//   kOrderMorton  one run over the whole tile (a Morton side whose tiles are
//                 aligned cubes: such a cube is one range of Morton indices);
//   kOrderPoint   one run per record (a Morton side whose tiles are not
//                 aligned);
//   kOrderOne     a One source: a single run of its single record.
// The source runs are loaded into LDS (a record-major side as the 16-byte
// granules of the blocks a run touches, a field-major side per leaf); the
// destination is written value by value from there (field-major and AoSoA
// destinations), or through a destination region of whole records stored as
// exact byte spans (AoS destinations).
// ---------------------------------------------------------------------------

enum : uint32_t { kOrderRow = 0, kOrderCol = 1, kOrderMorton = 2, kOrderPoint = 3, kOrderOne = 4 };
enum : uint32_t { kLinRow = 0, kLinCol = 1, kLinMorton = 2 };

constexpr int kBoxMaxEntries = 80;

struct BoxSide {
    uint64_t offset[LLAMA_MAX_RANK]; // the box's origin in this view's coordinates
    uint64_t extent[LLAMA_MAX_RANK]; // this view's extents
    uint64_t blob;     // record-major: device address of the blob
    uint64_t npad;     // linear indices the blob spans (loads and stores stay below)
    uint64_t block;    // K (record-major)
    uint32_t log2_lanes; // record-major: log2 L (AoS: 0)
    uint32_t mode;     // kRecordMajor / kFieldMajor (SoA)
    uint32_t lin;      // kLin*: the view's linearizer
    uint32_t order;    // kOrder*: how a tile's records form runs
    uint32_t morton_bits; // bits per dimension of the Morton index
    uint32_t run_log2; // log2 of a run's records (unclipped)
    uint32_t gran;     // record-major source, staged destination: 16-byte granules of a run's LDS slot
    uint32_t magic;    // ceil(2^32 / gran): g / gran == mulhi(g, magic) for the granule counts of a tile
    uint32_t lds_base; // LDS byte of run 0
    uint32_t table;    // LDS byte of the run table (one 64-bit start index per run)
};

struct BoxEntry {
    uint64_t src_addr; // field-major source: blob + leaf base; else 0
    uint64_t dst_addr; // destination: blob + leaf base (direct stores); 0 for a gap
    uint32_t size;     // bytes per value (a gap: bytes of the gap)
    uint32_t src_off;  // record-major source: the leaf's byte in a block; field-major: the LDS byte of its
                       // runs' slots (leaf by leaf)
    uint32_t dst_off;  // AoS destination: the leaf's (or gap's) byte in a record
    uint32_t gap;      // 1: a destination gap (zeros)
    uint32_t gran;     // field-major source: 16-byte granules of one run's slot of this leaf
    uint32_t magic;    // ceil(2^32 / gran)
};

struct BoxHeader {
    uint32_t rank;
    uint32_t num_leaves;
    uint32_t num_entries; // leaves, then the gaps of an AoS destination
    uint32_t flags;       // kBoxFull, kBoxPreserve, kBoxStaged, kBoxUnitMorton
    uint32_t qlog[LLAMA_MAX_RANK]; // tile extents, log2
    uint32_t qlog_sum;             // log2 of the records of a tile
    uint32_t lds_bytes;
    uint32_t map;                  // LDS byte of the record map (16 bytes per record of a tile)
    uint32_t words;                // kBoxGather: 4-byte words of a destination record
    uint32_t wtab;                 // kBoxGather: LDS byte of the word table, then the leaves' source fields
    uint32_t kmagic;               // kBoxGather: ceil(2^32 / K) for the destination record stride K
    uint32_t pad;
    uint64_t box[LLAMA_MAX_RANK];   // the copy's box (full copies: the extents)
    uint64_t grid[LLAMA_MAX_RANK];  // tiles per dimension
    uint64_t shift[LLAMA_MAX_RANK]; // tile t covers box coordinates [t q - shift, (t + 1) q - shift)
    uint64_t num_units;
};

// a full copy: records outside the extents within a destination run (Morton
// holes, AoSoA lanes past the last index) are written with zeros
constexpr uint32_t kBoxFull = 1;
// padding keeps its bytes (no zeros; a staged destination is loaded first)
constexpr uint32_t kBoxPreserve = 2;
// an AoS destination: staged in LDS and stored as exact byte spans
constexpr uint32_t kBoxStaged = 4;
// units enumerate aligned cubes in Morton order (a full copy into a Morton
// destination, whose holes and tail must be written)
constexpr uint32_t kBoxUnitMorton = 8;
// an AoS destination whose records are whole 4-byte words of whole 4-byte
// values: every 16-byte granule of a destination run is assembled word by
// word from the source region (word table `words`) and stored, without a
// destination region in LDS
constexpr uint32_t kBoxGather = 16;
constexpr int kBoxMaxWords = 52;
// a word-table entry: the leaf (bits 0-7; kBoxWordZero: a gap) and the byte
// of the leaf's value (bits 8-19)
constexpr uint32_t kBoxWordZero = 0xFFu;

struct BoxArgs {
    BoxHeader h;
    BoxSide src, dst;
    BoxEntry e[kBoxMaxEntries];
    uint32_t words[kBoxMaxWords]; // kBoxGather: the destination record's words
};
static_assert(sizeof(BoxArgs) <= 4096, "kernel arguments are limited to 4 KiB");

// ---------------------------------------------------------------------------
// HEATMAP (sec. 3.7): the counted kernel variants add one to a 32-bit counter
// per byte for every byte a global load reads (blobs in r) and every byte a
// global store writes (blobs in w).  counters: device address of the blob's
// hi - lo counters.  The table lives in a device global, written before the
// counted launches.
// ---------------------------------------------------------------------------

constexpr int kCountMaxBlobs = 128;

struct CountBlob {
    uint64_t lo, hi;   // device byte range [lo, hi) of the blob
    uint64_t counters; // device address of hi - lo 32-bit counters
};

struct CountTable {
    uint32_t nr, nw;
    CountBlob r[kCountMaxBlobs];
    CountBlob w[kCountMaxBlobs];
};

} // namespace llama
