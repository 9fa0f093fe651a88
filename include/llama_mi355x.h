/*
 * llama_mi355x.h -- C ABI of the MI355X layout-aware copy.
 *
 * The library implements the layout-aware copy of LLAMA (Gruber et al.,
 * "LLAMA: The Low-Level Abstraction for Memory Access", arXiv 2106.04284): a
 * multi-dimensional array of nested, structured records (the paper's "data
 * space", sec. 3.1) is held by a view, that is a mapping plus an array of
 * blobs (sec. 3.2, sec. 3.8), and is copied into a second view of the same
 * data space whose mapping differs (sec. 3.9).  The copy runs in HIP kernels
 * on an AMD Instinct MI355X (gfx950).
 *
 * Conventions shared by every entry point:
 *  - Return value: LLAMA_OK (0) or a negative llama_status.  After a non-OK
 *    status llama_last_error() describes it (thread-local string).  No C++
 *    exception crosses this interface.
 *  - Ownership: the caller owns every descriptor and every blob.  Descriptors
 *    are read during the call only.  The library never allocates or frees a
 *    blob (blobs are supplied by the user, sec. 3.8); it owns only its small
 *    internal state (batch tables, server queues, the tuning cache).
 *  - Asynchrony: llama_copy, llama_copy_naive, llama_copy_ex and
 *    llama_batch_launch validate synchronously, enqueue on `stream` and return;
 *    they behave like hipMemcpyAsync.  Blobs must stay valid until the stream
 *    work has finished.  `stream` is a hipStream_t (NULL: the null stream).
 *  - Errors in the arguments are reported before anything is enqueued.
 *  - Bytes are moved verbatim: NaN payloads, -0, subnormals and non-canonical
 *    booleans survive unchanged.
 */
#ifndef LLAMA_MI355X_H
#define LLAMA_MI355X_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ------------------------------------------------------------------------ */
/* Status codes                                                             */
/* ------------------------------------------------------------------------ */

typedef enum {
    LLAMA_OK = 0,
    LLAMA_E_INVALID_ARG = -1,      /* NULL pointer, bad kind, bad size/alignment/count, bad lanes */
    LLAMA_E_RECORD_MISMATCH = -2,  /* source and destination flatten to different leaves */
    LLAMA_E_EXTENT_MISMATCH = -3,  /* source and destination array dimensions differ */
    LLAMA_E_BLOB_TOO_SMALL = -4,   /* a blob is smaller than the mapping needs */
    LLAMA_E_OVERLAP = -6,          /* a source blob range overlaps a destination blob range */
    LLAMA_E_OVERFLOW = -7,         /* a size or offset does not fit 64 bits */
    LLAMA_E_UNSUPPORTED = -8,      /* a valid request this build cannot run */
    LLAMA_E_HIP = -9,              /* the HIP runtime reported an error */
    LLAMA_E_NO_BUDGET = -10,       /* a request is larger than a server's memory budget */
    LLAMA_E_BUSY = -11             /* a server queue is full */
} llama_status;

/* Thread-local text for the last non-OK status returned on this thread. */
const char* llama_last_error(void);

/* Constant name of a status code. */
const char* llama_status_string(int status);

/* ------------------------------------------------------------------------ */
/* Record dimension (sec. 3.3, Listings 1 and 2)                            */
/* ------------------------------------------------------------------------ */

/* One node of a record tree, listed in pre-order (a node, then its children).
 *  - Leaf (an elemental type): size > 0 (at most 4096), children == 0.
 *    `align` is its alignment, a power of two (at most 4096); 0 means the
 *    largest power of two dividing `size`, capped at 16.
 *  - Nested record: size == 0, children > 0 = number of direct child nodes,
 *    each followed by its own subtree.
 *  - count >= 1: the node is a static array of `count` elements (sec. 3.3:
 *    an array field T[n] is a record of n fields of T); count applies to
 *    leaves and to nested records alike.
 * Leaves are numbered depth first in declaration order (forEachLeaf, sec. 3.6);
 * that leaf number is the record coordinate used by this interface. */
typedef struct {
    uint32_t size;
    uint32_t align;
    uint32_t count;
    uint32_t children;
} llama_field;

/* A record: the top-level members, each member's subtree in pre-order. */
typedef struct {
    uint32_t num_nodes;
    const llama_field* nodes;
} llama_record_desc;

/* Leaf count, packed record size S (sum of leaf sizes) and aligned record
 * stride R (each leaf at the next multiple of its alignment, the stride
 * rounded up to the largest alignment: the C struct rule applied to the
 * flattened leaves).  Any output pointer may be NULL. */
int llama_record_info(const llama_record_desc* record, uint32_t* leaf_count, uint64_t* packed_size,
                      uint64_t* aligned_size);

/* Size, alignment, packed offset and aligned offset of leaf `leaf`.  Any
 * output pointer may be NULL. */
int llama_record_leaf(const llama_record_desc* record, uint32_t leaf, uint32_t* size, uint32_t* align,
                      uint64_t* packed_offset, uint64_t* aligned_offset);

/* ------------------------------------------------------------------------ */
/* Mappings (sec. 3.7)                                                      */
/* ------------------------------------------------------------------------ */

typedef enum {
    LLAMA_AOS_PACKED = 0,  /* records one after another, leaves tightly packed: 1 blob of N*S */
    LLAMA_AOS_ALIGNED = 1, /* records one after another, leaves aligned: 1 blob of N*R */
    LLAMA_SOA_SINGLE = 2,  /* per leaf f, N values contiguous at N*(packed offset of f): 1 blob of N*S */
    LLAMA_SOA_MULTI = 3,   /* per leaf f, N values contiguous in blob f: F blobs of N*s_f */
    LLAMA_AOSOA = 4,       /* blocks of `lanes` records; inside a block leaf f's values are
                              contiguous at lanes*(packed offset of f): 1 blob of
                              ceil(N/lanes)*lanes*S */
    LLAMA_SPLIT = 5,       /* two of the other kinds over two parts of the record (sec. 3.7
                              Split); see llama_split_desc */
    LLAMA_ONE = 6,         /* every array coordinate at the same single record, packed: 1 blob
                              of S (sec. 3.7 One).  A copy reads it as a broadcast, element-wise;
                              it is never a copy's destination (LLAMA_E_UNSUPPORTED) */
    LLAMA_SOA_ALIGNED = 7  /* SoA in 1 blob whose sub-arrays start at multiples of `lanes` bytes
                              (a power of two up to 2^20; 0 means 256): leaf f's N values start
                              at the first multiple at or after the end of leaf f-1's, the bytes
                              between sub-arrays are padding (zero in a destination, or kept
                              with LLAMA_COPY_PRESERVE_PADDING), and the blob ends with the last
                              sub-array.  The padded SoA that sec. 4.4 notes SoA cannot produce
                              yet; sec. 3.9 names copies between a mapping with and without such
                              padding.  Not for llama_copy_transfer (LLAMA_E_UNSUPPORTED) */
} llama_mapping_kind;

/* A Split mapping (sec. 3.7): the leaves [first_leaf, first_leaf + leaf_count)
 * of the flattened record form the selected part, mapped by kind[0] (lanes[0]);
 * the other leaves, in leaf order, form the rest, mapped by kind[1] (lanes[1]).
 * Each part is that mapping of its own sub-record (its leaves with their sizes
 * and alignments, offsets recomputed) over the same array dimensions.  The
 * parts keep separate blobs: the selected part's blobs first, then the rest's.
 * A record coordinate selects a subtree, whose leaves are such a contiguous
 * range in depth-first order.  Both parts must be non-empty.  A part of kind
 * LLAMA_SPLIT is split again by split[k], whose leaf range counts the part's
 * own leaves (the nesting of sec. 3.7's mapping listing), at most 8 levels
 * deep.  The descriptors are read during each call only. */
typedef struct llama_split_desc {
    uint32_t first_leaf;
    uint32_t leaf_count;
    uint32_t kind[2];  /* llama_mapping_kind of the selected part and of the rest */
    uint32_t lanes[2]; /* LLAMA_AOSOA parts: lanes per block, a power of two */
    const struct llama_split_desc* split[2]; /* LLAMA_SPLIT parts: their split; else ignored */
} llama_split_desc;

#define LLAMA_MAX_RANK 8

/* Linearizers: how an array coordinate becomes the linear index i that a
 * mapping lays out (sec. 3.7 lists linearizers among the building blocks of
 * mappings; sec. 2 names other storage orders and space-filling curves).  In
 * rank 1 all three are the identity. */
typedef enum {
    LLAMA_ROW_MAJOR = 0, /* last index fastest (sec. 3.6, Listing 4) */
    LLAMA_COL_MAJOR = 1, /* first index fastest */
    LLAMA_MORTON = 2     /* Z-order: bit j of coordinate d is bit j*rank + (rank-1-d) of i, with as
                            many bits per coordinate as the largest extent needs; the mapping lays
                            out indices up to the last coordinate's, and the indices that no
                            coordinate reaches are padding */
} llama_linearizer;

/* A mapping of the data space: record dimension, kind and array dimensions. */
typedef struct {
    const llama_record_desc* record;
    uint32_t kind;                    /* llama_mapping_kind */
    uint32_t rank;                    /* 1 .. LLAMA_MAX_RANK */
    uint64_t extents[LLAMA_MAX_RANK]; /* extents[0 .. rank-1]; zero extents allowed */
    uint32_t lanes;                   /* LLAMA_AOSOA: lanes per block, a power of two; LLAMA_SOA_ALIGNED:
                                         the sub-array alignment in bytes; else ignored */
    uint32_t linearizer;              /* llama_linearizer (0: row-major); Split and its parts: row-major
                                         only; One: ignored */
    const llama_split_desc* split;    /* LLAMA_SPLIT: the split (required); else ignored */
} llama_mapping_desc;

/* Number of blobs the mapping needs (the paper's compile-time blobCount). */
int llama_mapping_blob_count(const llama_mapping_desc* mapping, uint32_t* count);

/* Bytes blob `blob` needs (the paper's blobSize). */
int llama_mapping_blob_size(const llama_mapping_desc* mapping, uint32_t blob, uint64_t* size);

/* Host-side blobNrAndOffset (sec. 3.7): where leaf `leaf` of the record at
 * array coordinate coord[0 .. rank-1] lives.  Coordinates must be in range. */
int llama_mapping_offset(const llama_mapping_desc* mapping, const uint64_t* coord, uint32_t leaf,
                         uint32_t* blob, uint64_t* offset);

/* ------------------------------------------------------------------------ */
/* Blobs (sec. 3.8) and the copy (sec. 3.9)                                 */
/* ------------------------------------------------------------------------ */

/* A contiguous byte range in device memory (any alignment).  `size` may
 * exceed what the mapping needs; bytes past the mapping's blob size are never
 * read or written. */
typedef struct {
    void* ptr;
    uint64_t size;
} llama_blob;

/* Copies the view (src, src_blobs) into the view (dst, dst_blobs).
 *  - src and dst must flatten to the same leaves (same sizes and alignments
 *    in the same order) and have the same rank and extents.
 *  - Their linearizers may differ: every coordinate's record moves from its
 *    source index to its destination index (the box kernel runs such
 *    copies, and Morton copies whose indices have holes; the other paths
 *    work on equal linear indices).
 *  - src_blobs / dst_blobs hold blob_count entries of their mapping.
 *  - No source range may overlap a destination range.
 *  - Every byte of every destination blob up to the mapping's blob size is
 *    written exactly once (a Split destination part fed by several copies
 *    excepted, see below): leaf values from the source, and zero for
 *    the destination's padding (alignment gaps of aligned AoS, lanes past the
 *    last record in the last AoSoA block, Morton indices that no coordinate
 *    reaches).  llama_copy_heatmap counts it.
 *  - A data space with zero records enqueues nothing and returns LLAMA_OK.
 *  - A Split on either side runs as a few tile copies, in order on `stream`
 *    (llama_plan_copy lists them):
 *     - a destination part fed by several source parts is one copy whose
 *       source gathers those parts, when the record-major ones share one
 *       lane count and every chunk (a part block, or that many values of an
 *       SoA leaf) is whole 16-byte granules at a 16-byte aligned address, or
 *       when all are SoA (LLAMA_PLAN_GATHERED_SOURCE);
 *     - a source part feeding several destination parts (each taking all its
 *       leaves from it, or SoA) is one copy whose stores scatter over those
 *       parts, when the record-major ones are AoSoA parts of one lane count
 *       with runs of 128 bytes or more at 16-byte aligned addresses, or all
 *       are SoA (LLAMA_PLAN_SCATTERED_DESTINATION);
 *     - every other pair of parts that share leaves is one copy.  Into a
 *       record-major destination part (AoS, AoSoA) fed by several such
 *       copies, the one with the most bytes writes whole records first (the
 *       other leaves' bytes as zeros, or kept with
 *       LLAMA_COPY_PRESERVE_PADDING); each later copy into an AoS part
 *       without padding reads the part's records into LDS, replaces its own
 *       leaves and stores the records back whole
 *       (LLAMA_PLAN_KEEPS_DESTINATION), so those bytes are written more than
 *       once and nothing else may write the destination while the copy
 *       runs.  A later copy into another record-major part stores only its
 *       own leaves (a direct-store tile, else the element-wise path).
 *    Batches and the batched server policy take a Split item as one copy per
 *    pair of parts, side by side, unless one of them writes part of the
 *    records of a record-major destination part or reads a One part
 *    (LLAMA_E_UNSUPPORTED); the other server policies run its copies in
 *    order.  llama_plan, autotuning and servers with an executor take plain
 *    mappings only (LLAMA_E_UNSUPPORTED). */
int llama_copy(const llama_mapping_desc* src, const llama_blob* src_blobs, const llama_mapping_desc* dst,
               const llama_blob* dst_blobs, void* stream);

/* The plain element-wise copy on the GPU: one thread per record, looping over
 * the leaves, each leaf located through the run-time mapping arithmetic and
 * moved at its own width (the naive copy of sec. 4.2, on the GPU).  Same
 * contract and same result as llama_copy; it exists as the baseline. */
int llama_copy_naive(const llama_mapping_desc* src, const llama_blob* src_blobs, const llama_mapping_desc* dst,
                     const llama_blob* dst_blobs, void* stream);

/* Copy strategies (llama_plan_info.path, llama_copy_options.path). */
typedef enum {
    LLAMA_PATH_AUTO = 0,   /* options only: let the planner choose */
    LLAMA_PATH_STREAM = 1, /* contiguous runs copied with wide vector accesses (includes identical layouts) */
    LLAMA_PATH_TILE = 2,   /* record tiles staged through LDS, transposed, stored coalesced */
    LLAMA_PATH_NAIVE = 3,  /* the element-wise baseline kernel */
    LLAMA_PATH_EMPTY = 4,  /* plan only: nothing to do (no records) */
    LLAMA_PATH_BOX = 5     /* tiles of coordinates whose records sit at different linear indices on the
                              two sides (box copies, differing linearizers), staged through LDS */
} llama_path;

/* Kernel parameters.  Zero in any field means "the library's choice". */
typedef struct {
    uint32_t path;         /* llama_path */
    uint32_t tile_records; /* TILE: records per tile, a power of two (16 .. 4096) */
    uint32_t threads;      /* threads per workgroup, a multiple of 64 in 64 .. 1024 */
    uint32_t wg_per_cu;    /* TILE: 0 launches one workgroup per tile; 1 .. 16 launches a
                              persistent grid of that many workgroups per compute unit */
    uint32_t flags;        /* LLAMA_COPY_* bits */
} llama_copy_options;

/* TILE: always stage the destination through LDS (LLAMA_TILE_STAGED).  By
 * default the planner takes, where the layouts allow it, a mode that skips
 * one of the two LDS regions: LLAMA_TILE_DIRECT_STORE, LLAMA_TILE_GATHER_STORE
 * or LLAMA_TILE_DIRECT_LOAD. */
#define LLAMA_COPY_NO_DIRECT 1u

/* TILE: move a misaligned value byte by byte (by default a 2-, 4- or 8-byte
 * value of a packed record of odd size is read whole from the words that hold
 * it and written in pieces of the destination's alignment), and take neither
 * the direct store of such values from their aligned words nor the direct
 * load that writes them (or 1- and 2-byte leaves) into the region in pieces:
 * those pairs stage both regions. */
#define LLAMA_COPY_NO_SPLIT 2u

/* Keep the destination's padding bytes (aligned-AoS gaps and record tails,
 * AoSoA lanes past the last record) as they were, instead of writing zeros
 * there.  Field-major destinations are written value by value as before; the
 * tiles of a record-major destination with padding are read, their values
 * replaced, and written back whole, so such a copy also reads the
 * destination, and nothing else may write the destination's padding while it
 * runs.  Without padding in the destination the flag changes nothing. */
#define LLAMA_COPY_PRESERVE_PADDING 4u

/* TILE: do not take LLAMA_TILE_GATHER_STORE.  Where the gather store would
 * apply, the planner tries the direct load, else stages both regions.  Only the
 * speed changes; llama_autotune tries it per copy class. */
#define LLAMA_COPY_NO_GATHER 8u

/* llama_copy with explicit kernel parameters.  The result does not depend on
 * the options; only the speed does. */
int llama_copy_ex(const llama_mapping_desc* src, const llama_blob* src_blobs, const llama_mapping_desc* dst,
                  const llama_blob* dst_blobs, const llama_copy_options* options, void* stream);

/* Copies a box of the array dimensions between two views whose extents may
 * differ (sec. 3.2: a VirtualView shows a sub-box of a view, shifted by an
 * offset; sec. 3.9 names copies between views of different size or shape):
 * for every coordinate c with 0 <= c[d] < box[d], the record at
 * src_offset + c of the source moves to dst_offset + c of the destination.
 *  - src and dst flatten to the same leaves and have the same rank; extents,
 *    kinds and linearizers may differ.  The box must lie inside both views
 *    (LLAMA_E_EXTENT_MISMATCH otherwise).
 *  - Destination records outside the box keep every byte (AoSoA lanes past
 *    the last record included).  The alignment gaps of the box's records in
 *    an aligned-AoS destination become zero, or keep their bytes with
 *    LLAMA_COPY_PRESERVE_PADDING (then the destination records are read and
 *    stored back whole).
 *  - Mappings: plain kinds; the source may be One (broadcast), the
 *    destination not; no Split (LLAMA_E_UNSUPPORTED).
 *  - Options: path AUTO or BOX runs the tiled box kernel, NAIVE its
 *    element-wise baseline (one thread per record of the box); tile_records
 *    sets the records per tile (a power of two, 16 .. 4096), threads the
 *    workgroup size; the result does not depend on them.
 *  - A box with a zero extent enqueues nothing.  No source blob may overlap
 *    a destination blob.  Asynchronous like llama_copy. */
int llama_copy_box(const llama_mapping_desc* src, const llama_blob* src_blobs, const uint64_t* src_offset,
                   const llama_mapping_desc* dst, const llama_blob* dst_blobs, const uint64_t* dst_offset,
                   const uint64_t* box, const llama_copy_options* options, void* stream);

/* Where a view's blobs live (llama_copy_transfer). */
typedef enum {
    LLAMA_MEMORY_DEVICE = 0, /* device memory of the current device */
    LLAMA_MEMORY_HOST = 1    /* host memory; pinned (hipHostMalloc, torch pin_memory) for the transfers to
                                overlap the layout changes, pageable works but serialises them */
} llama_memory;

/* Copies a view between host and device memory, changing the mapping on the
 * way (sec. 3.9: copies between address spaces shuffle a chunk into the
 * other mapping in a small intermediate view and transfer it, overlapping
 * shuffles and transfers; sec. 1 names copies between devices).  The records
 * are cut into chunks of whole AoSoA blocks of both sides, about chunk_bytes
 * each (0: 64 MiB).  Host to device: each chunk is transferred in the
 * source's layout into a device staging view, whose layout the GPU then
 * changes into the destination; device to host: the GPU changes the layout of
 * a chunk into the staging view, which is then transferred.  Two staging
 * buffers alternate, so the transfer of one chunk overlaps the layout change
 * of the next on a second stream of the library.
 *  - One of src_memory / dst_memory is LLAMA_MEMORY_HOST, the other
 *    LLAMA_MEMORY_DEVICE (LLAMA_E_INVALID_ARG otherwise).
 *  - The result equals llama_copy's: same records, extents and linearizer on
 *    both sides (LLAMA_E_UNSUPPORTED for differing linear indices, Split and
 *    a One source); padding zeroed.
 *  - Asynchronous: returns after enqueueing; the work on `stream` completes
 *    after the whole copy.  Host blobs must stay valid (and, for a device to
 *    host copy, unread) until then.
 *  - The library keeps two staging buffers per device (allocated, or grown,
 *    on a call that needs more) and runs one transfer per device at a time: a
 *    call first waits for the previous transfer on the device to finish. */
int llama_copy_transfer(const llama_mapping_desc* src, const llama_blob* src_blobs, uint32_t src_memory,
                        const llama_mapping_desc* dst, const llama_blob* dst_blobs, uint32_t dst_memory,
                        uint64_t chunk_bytes, void* stream);

/* Marks a destination leaf that takes no source leaf (llama_copy_leaves). */
#define LLAMA_NO_LEAF 0xFFFFFFFFu

/* Copies between views whose records differ (sec. 3.9: a field missing on one
 * side).  Destination leaf k takes source leaf src_leaf[k] (src_leaf holds one
 * entry per flattened destination leaf), which must have the same size; a
 * destination leaf with LLAMA_NO_LEAF keeps all its bytes, unused AoSoA lanes
 * included.  The destination's padding (alignment gaps, and the unused AoSoA
 * lanes of the leaves that take a value) becomes zero, or keeps its bytes with
 * LLAMA_COPY_PRESERVE_PADDING.  A source leaf may feed several destination
 * leaves.  Mappings: not Split; the source may be One, the destination not
 * (LLAMA_E_UNSUPPORTED).  Errors: LLAMA_E_INVALID_ARG for a leaf index out of
 * range or no destination leaf with a source, LLAMA_E_RECORD_MISMATCH for
 * leaves of different sizes, and llama_copy's others.  When some destination
 * leaves keep their bytes, a packed AoS destination is written by a tile
 * that loads the destination records into LDS, replaces the leaves that
 * take a value and stores the records back whole: the kept leaves' bytes
 * are read and written back unchanged, so nothing else may write that
 * destination while the copy runs.  Another record-major destination is
 * written by a direct-store tile plan if one applies (only the leaves that
 * take a value), else element-wise; options as for llama_copy_ex. */
int llama_copy_leaves(const llama_mapping_desc* src, const llama_blob* src_blobs, const llama_mapping_desc* dst,
                      const llama_blob* dst_blobs, const uint32_t* src_leaf, const llama_copy_options* options,
                      void* stream);


/* ------------------------------------------------------------------------ */
/* Heatmap and Trace (sec. 3.7): access counters around a copy              */
/* ------------------------------------------------------------------------ */

/* Per-byte counters of a Heatmap copy.  Each array has one entry per blob of
 * its mapping (an entry, or the array itself, may be NULL: not counted); an
 * entry is a device array of 32-bit counters, one per byte of the mapping's
 * blob size, which the copy adds to (the caller zeroes it first). */
typedef struct {
    uint32_t* const* src_reads;  /* source blobs: bytes read */
    uint32_t* const* dst_writes; /* destination blobs: bytes written */
    uint32_t* const* dst_reads;  /* destination blobs: bytes read (kept padding, kept-gap tiles) */
} llama_heatmap;

/* The Heatmap of sec. 3.7, for the library's own copies: runs the copy that
 * llama_copy_ex (src_leaf == NULL) or llama_copy_leaves (src_leaf != NULL)
 * would run with these options -- the same plans, paths and tile modes --
 * in counted kernel variants that add one to a byte's counter for every
 * global load that reads it and every global store that writes it.  The
 * destination ends up as the plain copy leaves it.  It is a debugging and
 * analysis tool: the counted variants run many times slower, and they take
 * plain (not nontemporal) loads and stores.  At most 128 blobs per list
 * (source reads and destination reads together count as one list).  The counters live in a device global of the library: Heatmap
 * copies on one device must not overlap in time.  A copy that writes every
 * destination byte exactly once shows a destination write count of one on
 * every byte (zero on kept padding and on leaves without a source). */
int llama_copy_heatmap(const llama_mapping_desc* src, const llama_blob* src_blobs, const llama_mapping_desc* dst,
                       const llama_blob* dst_blobs, const uint32_t* src_leaf, const llama_copy_options* options,
                       const llama_heatmap* heatmap, void* stream);

/* A byte range whose accesses a Heatmap counts: `size` bytes at `ptr`
 * (device memory), one 32-bit counter per byte at `counters`. */
typedef struct {
    const void* ptr;
    uint64_t size;
    uint32_t* counters;
} llama_count_range;

/* The Heatmap around any of this thread's copies: after llama_heatmap_begin,
 * llama_copy, llama_copy_ex, llama_copy_naive, llama_copy_leaves and
 * llama_copy_box on the calling thread run in their counted kernel variants
 * (the same plans), which add one to the counter of every byte of `reads`
 * that a global load reads and of every byte of `writes` that a global store
 * writes, until llama_heatmap_end.  At most 128 ranges per list
 * (LLAMA_E_UNSUPPORTED).  The list is uploaded on `stream` into a device
 * global of the library: the copies counted must run on that stream (or
 * after it), and Heatmaps on one device must not overlap in time.
 * llama_copy_heatmap is this around one copy. */
int llama_heatmap_begin(size_t nreads, const llama_count_range* reads, size_t nwrites,
                        const llama_count_range* writes, void* stream);
int llama_heatmap_end(void);

/* The Trace of sec. 3.7 (accesses per field), from a view's per-byte
 * counters (such as a llama_heatmap's): sums[f] is the sum of the counters of
 * the bytes of leaf f over all records, for each of the F leaves, and
 * sums[F] the sum over the bytes that no leaf owns (alignment gaps, AoSoA
 * lanes past the last record).  counters holds one device array of 32-bit
 * counters per blob of the mapping.  Not for One mappings
 * (LLAMA_E_UNSUPPORTED).  Synchronous: runs on `stream` and waits for it. */
int llama_trace_leaves(const llama_mapping_desc* mapping, uint32_t* const* counters, uint64_t* sums, void* stream);

/* How a TILE copy moves one tile (llama_plan_info.tile_mode). */
typedef enum {
    LLAMA_TILE_STAGED = 1,       /* source span(s) -> LDS -> destination region in LDS -> destination span(s) */
    LLAMA_TILE_DIRECT_STORE = 2, /* field-major (or long-run AoSoA) destination: 16-byte granules of one
                                    leaf gathered from the staged source and stored from registers */
    LLAMA_TILE_DIRECT_LOAD = 3,  /* field-major (or long-run AoSoA) source: granules loaded into registers
                                    and written to the destination region in LDS */
    LLAMA_TILE_GATHER_STORE = 4  /* record-major destination of whole 4-byte words: every 16-byte granule
                                    of the destination span assembled word by word from the staged source */
} llama_tile_mode;

/* What llama_copy_ex would do for this pair with these options (NULL: the
 * defaults), without touching any blob. */
typedef struct {
    uint32_t path;          /* llama_path chosen */
    uint32_t tile_records;  /* TILE: records per tile */
    uint32_t threads;       /* threads per workgroup */
    uint32_t lds_bytes;     /* TILE: LDS bytes per workgroup */
    uint64_t workgroups;    /* workgroups launched */
    uint32_t runs;          /* STREAM: contiguous runs (zero runs included) */
    uint32_t wg_per_cu;     /* TILE: persistent workgroups per compute unit (0: one per tile) */
    uint64_t tiles;         /* TILE: tiles of tile_records records */
    uint64_t read_bytes;    /* bytes of source blobs the copy reads */
    uint64_t write_bytes;   /* bytes of destination blobs the copy writes */
    uint32_t tile_mode;     /* TILE: llama_tile_mode; 0 for the other paths */
    uint32_t cache_hints;   /* TILE and STREAM: bit 0 (LLAMA_HINT_STREAM_LOADS) when the source
                               loads carry the nontemporal hint (sources of 256 MiB or more, the
                               size of the Infinity Cache); bit 1 (LLAMA_HINT_STREAM_STORES) when
                               the destination's 16-byte stores do (TILE, destinations of 1 GiB or
                               more) */
    uint32_t plan_flags;    /* TILE: LLAMA_PLAN_* bits */
    uint32_t source_chunks; /* TILE with LLAMA_PLAN_GATHERED_SOURCE: chunks of one virtual source block */
} llama_plan_info;

#define LLAMA_HINT_STREAM_LOADS 1u
#define LLAMA_HINT_STREAM_STORES 2u

/* llama_plan_info.plan_flags */
/* The tile's source is gathered from several parts of a Split source (sec.
 * 3.7): every tile loads the records' chunks from each part (a whole AoSoA
 * or AoS block, or the values of one SoA leaf) into one staged region, so a
 * destination part fed by several source parts is written by one copy. */
#define LLAMA_PLAN_GATHERED_SOURCE 1u
/* The tile loads each destination region and stores it back whole: the
 * bytes it does not own (kept padding, leaves without a source, leaves that
 * another part copy writes) keep their values but are written again, so
 * nothing else may write that destination while the copy runs. */
#define LLAMA_PLAN_KEEPS_DESTINATION 2u
/* The tile's destination is scattered over several parts of a Split
 * destination (sec. 3.7): one source part feeding several destination parts
 * (AoSoA parts of one lane count, SoA leaves) is read once, and each leaf's
 * 16-byte granules are stored into its own part. */
#define LLAMA_PLAN_SCATTERED_DESTINATION 4u

/* What a copy of this pair with these options would launch, without blobs:
 * the plan assumes distinct blobs aligned to 256 bytes (a real copy plans for
 * its actual blob addresses, which can change alignment-dependent choices).
 * With the environment variable LLAMA_TRACE set (and not "0"), the plan is
 * also printed to stderr, as every launch's plan is. */
int llama_plan(const llama_mapping_desc* src, const llama_mapping_desc* dst, const llama_copy_options* options,
               llama_plan_info* info);

/* Every launch that llama_copy_ex (src_leaf NULL) or llama_copy_leaves
 * (src_leaf: its leaf map) would enqueue for this pair with these options, in
 * order, without blobs (distinct blobs aligned to 256 bytes are assumed, as
 * by llama_plan): a copy with a Split side lists its part copies, a box copy
 * its box launch and tail fill.  infos[0 .. *count - 1] receive the plans;
 * more launches than `capacity` fail with LLAMA_E_INVALID_ARG (*count 0).
 * Errors as the copy itself would report them for its descriptors. */
int llama_plan_copy(const llama_mapping_desc* src, const llama_mapping_desc* dst, const uint32_t* src_leaf,
                    const llama_copy_options* options, llama_plan_info* infos, uint32_t capacity, uint32_t* count);

/* ------------------------------------------------------------------------ */
/* Autotuning                                                               */
/* ------------------------------------------------------------------------ */

/* Measures kernel parameters for this copy on its own blobs: TILE with tile
 * sizes 16 .. 4096 records and 64/128/256 threads (each also with
 * LLAMA_COPY_NO_DIRECT where the plan would use a direct mode), and STREAM
 * where the pair has long runs.  Each candidate first runs on a destination filled with a
 * pattern and must produce the same bytes (compared by a 64-bit hash of the
 * destination blobs) as the default plan; then it is timed (best of `reps`
 * launches, 0: 3).  The fastest goes to the process-wide tuning cache, keyed
 * by (leaf sizes and alignments, source kind and lanes, destination kind and
 * lanes, floor(log2(record count))), and later copies of that class made with
 * default options use it (the entry of the nearest size bucket when the
 * exact one is missing).  Synchronous; the destination blobs end up holding
 * the copy.  `best` and `best_gbs` (read+write GB/s) may be NULL. */
int llama_autotune(const llama_mapping_desc* src, const llama_blob* src_blobs, const llama_mapping_desc* dst,
                   const llama_blob* dst_blobs, void* stream, uint32_t reps, llama_copy_options* best,
                   double* best_gbs);

/* The cached parameters for this pair's class; *found is 0 when there are none. */
int llama_tune_lookup(const llama_mapping_desc* src, const llama_mapping_desc* dst, llama_copy_options* options,
                      int* found);

int llama_tune_clear(void);

/* The tuning cache as a text file: one line per class, 12 fields separated
 * by blanks (leaf hash in hex, source kind, source lanes, destination kind,
 * destination lanes, size bucket, path, tile records, threads, wg_per_cu,
 * flags, measured GB/s); lines starting with '#' are comments. */
int llama_tune_save(const char* path);

/* Adds the classes of a file written by llama_tune_save; *entries (may be
 * NULL) receives how many lines were read. */
int llama_tune_load(const char* path, uint32_t* entries);

/* ------------------------------------------------------------------------ */
/* Batches: many independent copies in one launch                           */
/* ------------------------------------------------------------------------ */

/* One copy of a batch; the same contract as llama_copy's arguments. */
typedef struct {
    const llama_mapping_desc* src;
    const llama_blob* src_blobs;
    const llama_mapping_desc* dst;
    const llama_blob* dst_blobs;
} llama_copy_item;

/* A prepared batch: the items' plans in one device work table, run by one
 * kernel launch over the work units (the tiles of tiled items and the 4 KiB
 * chunks of long-run items).  Items that all fall in one LDS class (long
 * runs, or tiles of up to 1, 2, 4, ... KiB of LDS) run one workgroup per work
 * unit; a batch of several classes runs a persistent grid whose workgroups
 * take blocks of units from an atomic counter in the table.  The launch is
 * captured into a hipGraph on the first llama_batch_launch on a non-null
 * stream and replayed afterwards.  The result equals n separate llama_copy
 * calls.
 *  - Validation: every item as in llama_copy; no destination range may
 *    overlap another destination range or any source range of the batch
 *    (items run in no fixed order).
 *  - Ownership: the batch copies the descriptors and blob addresses; the
 *    blobs stay the caller's and must stay valid while launches are pending.
 *  - Options (may be NULL): tile_records (a fixed tile size for every TILE
 *    item, 0: each item's own), threads (per workgroup, for every item),
 *    wg_per_cu (1 .. 16: a persistent grid of that many workgroups per compute
 *    unit; 0: the choice above, a persistent grid taking as many as LDS and
 *    wave slots allow, at most 8); path must be 0, flags takes the
 *    LLAMA_COPY_* bits.  Every workgroup reserves
 *    the largest item's LDS, so without a fixed tile size each tiled item
 *    takes the largest tile whose plan fits 32 KB of LDS (the tuning cache,
 *    which is measured on standalone launches, is not used).
 *  - Items whose record does not fit the tiled kernel are refused with
 *    LLAMA_E_UNSUPPORTED.
 *  - A batch belongs to the device that was current at creation.
 *  - Launches of one batch must not overlap in time: they share the work
 *    counter (launch them on one stream). */
typedef struct llama_batch llama_batch;

typedef struct {
    uint64_t items;        /* non-empty items; an item with a Split side counts its part copies */
    uint64_t tile_items;   /* items copied by the tiled kernel */
    uint64_t stream_items; /* items copied as long runs */
    uint64_t work_units;   /* tiles plus run chunks */
    uint64_t read_bytes;   /* source blob bytes of all items */
    uint64_t write_bytes;  /* destination blob bytes of all items */
    uint32_t threads;      /* threads per workgroup */
    uint32_t wg_per_cu;    /* persistent grid: workgroups per compute unit; 0: one workgroup per work unit */
    uint32_t workgroups;   /* grid size (one launch per tile mode: all launches together) */
    uint32_t lds_bytes;    /* LDS per workgroup (one launch per tile mode: the largest) */
    uint32_t launches;     /* kernel launches per batch launch: 1, or one per tile mode when the
                              table is sorted by mode (each mode in its own compiled kernel) */
    uint32_t reserved;
} llama_batch_info;

int llama_batch_create(size_t n, const llama_copy_item* items, const llama_copy_options* options,
                       llama_batch** batch);

/* Enqueues one run of the whole batch on `stream`. */
int llama_batch_launch(llama_batch* batch, void* stream);

int llama_batch_get_info(const llama_batch* batch, llama_batch_info* info);

/* The batch's autotuner: measures launch parameters on the batch's own
 * blobs and re-plans the batch with the fastest.  Candidates: the LDS a tiled
 * item's plan may take (8, 16, 31 or 48 KiB: each item then takes the largest
 * tile that fits, so this sets the tile shapes and the LDS depth of every
 * workgroup), 128, 256 or 512 threads per workgroup (the waves that share a
 * tile), and the grid (the default rule, a persistent grid of 2, 4 or 8
 * workgroups per compute unit, or the table sorted by tile mode and run as
 * one launch per mode, each mode in its own compiled kernel with one
 * workgroup per work unit).  Every candidate first runs on destinations
 * filled with a pattern and must write the bytes the current plan writes
 * (compared by a 64-bit hash of every destination); then it is timed, best of
 * `reps` launches (0: 3).  A tile size fixed at creation stays fixed.
 * Synchronous: the destinations end up holding the copy, the batch's graph
 * is captured again on its next launch.  *best_gbs (may be NULL) receives the
 * winner's read+write GB/s. */
int llama_batch_autotune(llama_batch* batch, void* stream, uint32_t reps, double* best_gbs);

/* Waits for the device to finish pending work, then frees the batch. */
int llama_batch_destroy(llama_batch* batch);

/* One-shot batch: create, launch on `stream`, and release the batch once the
 * launch has finished.  Asynchronous like llama_copy. */
int llama_copy_batch(size_t n, const llama_copy_item* items, void* stream);

/* llama_copy_batch for callers that cannot allocate device memory (code under
 * stream capture, serving loops that must not call hipMalloc, harnesses that
 * forbid it): the same validation, plans, kernels and result, but the work
 * table (plans, unit prefix sums and the persistent grid's work counters)
 * goes into a static device buffer of the library, 8 MiB on every device the
 * library runs on (held until the process ends), instead of an allocation.
 * The call allocates no device memory and frees none: it uploads the table
 * into that buffer with hipMemcpyAsync on `stream` (the counters are uploaded
 * as zeros) and launches the batch kernel after it, without a graph.
 *  - A batch whose table needs more than 8 MiB fails with LLAMA_E_NO_BUDGET
 *    before anything is enqueued (a plain item takes a few hundred bytes of
 *    table: the 1,000-array batch needs about half a megabyte).
 *  - Every call on one device shares that device's buffer, which keeps the
 *    last call's table: calls whose work overlaps in time on one device race
 *    (a later upload overwrites a table still being read).  Calls in order on
 *    one stream are safe; calls on different streams must be ordered by the
 *    caller (events or synchronisation).
 *  - No batch handle, graph or host callback outlives the call. */
int llama_copy_batch_noalloc(size_t n, const llama_copy_item* items, void* stream);

/* ------------------------------------------------------------------------ */
/* Serving: continuous batching within an HBM budget                        */
/* ------------------------------------------------------------------------ */

/* How a server runs admitted requests. */
typedef enum {
    LLAMA_SERVE_BATCHED = 0,    /* every admitted group is one launch of the batch kernel (a group
                                   of one request is launched as that request's own copy) */
    LLAMA_SERVE_NAIVE = 1,      /* one element-wise (naive) kernel per request, one stream */
    LLAMA_SERVE_PER_REQUEST = 2 /* one llama_copy per request, streams round robin */
} llama_serve_policy;

typedef struct {
    uint64_t budget_bytes;   /* admission budget: source plus destination blob bytes in flight (> 0) */
    uint64_t group_bytes;    /* BATCHED: a request of this many bytes or more runs alone (its own
                                copy with its tuned plan); smaller requests queued together share
                                one launch of the batch kernel, which takes no further request once
                                its bytes reach this (0: 8 MiB) */
    uint64_t stream_bytes;   /* BATCHED: no launch joins a stream that already has this many bytes in
                                flight, and arrivals gather into larger launches meanwhile
                                (0: no limit) */
    uint32_t streams;        /* HIP streams whose launches overlap (0: 2; NAIVE: 1); at most 16 */
    uint32_t depth;          /* launches in flight per stream (0: BATCHED 64, PER_REQUEST 128,
                                NAIVE 256); at most 1024 */
    uint32_t max_batch;      /* requests per launch at most (0: 1024) */
    uint32_t queue_capacity; /* queued requests at most before submit says LLAMA_E_BUSY (0: 2^20) */
    uint32_t threads;        /* threads per workgroup (0: 256) */
    uint32_t policy;         /* llama_serve_policy */
} llama_server_config;

typedef struct {
    uint64_t submitted, completed, failed, queued;
    uint64_t launches;           /* kernel launches (batches) so far */
    uint64_t bytes_done;         /* source plus destination bytes of completed requests */
    uint64_t max_inflight_bytes; /* largest admitted total seen */
    double mean_batch;           /* requests per launch */
    double p50_latency, p99_latency, max_latency; /* seconds, submit to observed completion */
    double window;               /* seconds from the first submit to the last completion */
} llama_server_stats;

/* A server owns an engine thread, `streams` HIP streams on the current
 * device, and one preallocated work table per launch slot (streams x depth);
 * it never allocates blobs.
 *
 * Requests keep their blobs on the device (the caller's, valid until the
 * request completes).  The server's streams do not wait for the caller's
 * streams: a request's source must be complete, and nothing else may touch
 * its blobs, from submit until it completes.  The engine admits queued requests in arrival order
 * while the bytes in flight stay within budget_bytes and no destination range
 * meets a range of a request in flight; each admitted group is one launch on
 * the next free stream.  Requests that arrive while launches run join the
 * next launch as soon as a stream and budget free up.  Each result equals a
 * lone llama_copy of the request. */
typedef struct llama_server llama_server;

int llama_server_create(const llama_server_config* config, llama_server** server);

/* Validates the request (errors return here and concern this request only:
 * LLAMA_E_NO_BUDGET when it alone exceeds the budget, LLAMA_E_BUSY when the
 * queue is full), queues it and returns its ticket. */
int llama_server_submit(llama_server* server, const llama_copy_item* item, uint64_t* ticket);

/* *done = 1 and *status / *latency_s filled in when the request has finished,
 * else *done = 0.  status / latency_s may be NULL. */
int llama_server_poll(llama_server* server, uint64_t ticket, int* done, int* status, double* latency_s);

/* Blocks until the request has finished. */
int llama_server_wait(llama_server* server, uint64_t ticket, int* status, double* latency_s);

int llama_server_get_stats(llama_server* server, llama_server_stats* stats);

/* Clears the counters and latencies (queued and running requests continue). */
int llama_server_reset_stats(llama_server* server);

/* Finishes every queued and running request, then frees the server. */
int llama_server_destroy(llama_server* server);

/* An executor runs a server's launches on an engine of the caller's instead
 * of the library's HIP streams (another device runtime, a simulator, or a
 * host reference used to test the engine without a GPU).  The server keeps
 * everything else: validation, admission within the budget, range conflicts,
 * arrival order, grouping, completion and latency accounting.
 *  - start(context, launch, n, items): begin launch number `launch` (unique,
 *    increasing) copying items[0 .. n); return LLAMA_OK, or an error status
 *    that fails the launch's requests.  `items` is valid during the call;
 *    the descriptors and blob arrays it points to stay valid until poll has
 *    reported the launch finished.
 *  - poll(context, launch): 1 when the launch has finished, 0 while it runs,
 *    a negative status when it failed (its requests fail with that status).
 * Both are called from the server's engine thread only, one call at a time;
 * poll is called with the server's lock held, so neither may call any
 * llama_server_* function. */
typedef struct {
    void* context;
    int (*start)(void* context, uint64_t launch, size_t n, const llama_copy_item* items);
    int (*poll)(void* context, uint64_t launch);
} llama_executor;

/* llama_server_create on an executor (NULL: the HIP engine).  With an
 * executor the server touches no GPU: `policy` only chooses the grouping
 * (BATCHED: small requests share a launch as above; otherwise one request per
 * launch), `streams` x `depth` bounds the launches in flight, and `threads`
 * and the record's fit in the tiled kernel are not checked. */
int llama_server_create_ex(const llama_server_config* config, const llama_executor* executor,
                           llama_server** server);

#ifdef __cplusplus
}
#endif

#endif /* LLAMA_MI355X_H */
