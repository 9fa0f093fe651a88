// HIP kernels of the layout-aware copy for gfx950 (MI355X), and their launch.
//
// The copy is pure data movement: every kernel moves bytes as unsigned
// integers (never as floating point), so values survive bit for bit.
//
//  tile_kernel    records [i0, i0+T) of a tile: the source span(s) are loaded
//                 straight into LDS with 16-byte global_load_lds, the values
//                 are moved inside LDS from source to destination positions
//                 (one leaf per step, lanes over records), and the destination
//                 span(s) are written back with 16-byte coalesced stores.
//                 Three modes keep one side out of LDS: direct store and
//                 gather store build 16-byte destination granules in
//                 registers from the staged source (by leaf, or word by word
//                 through a table); direct load loads source granules into
//                 registers and writes them to the destination region.
//  stream_kernel  long contiguous runs (SoA <-> SoA, identical layouts),
//                 16-byte loads and stores, no LDS.
//  naive_kernel   the element-wise baseline: one thread per record, each leaf
//                 located with run-time '/' and '%' and moved at its own width.
#include <hip/hip_runtime.h>

#include <mutex>

#include "batch.hpp"
#include "core.hpp"
#include "serve.hpp"

// The work table of llama_copy_batch_noalloc: a static device buffer, so that
// that entry point allocates nothing.  Each device holds its own copy, at its
// own address, which host code takes from hipGetSymbolAddress (the array's
// name itself is not a device address in host code).
static __device__ __align__(256) uint8_t scratch[llama::kScratchBytes];

namespace llama {

namespace {

typedef __attribute__((address_space(3))) void lds_void_t;
#define GLOBAL __attribute__((address_space(1)))
#define CONSTANT __attribute__((address_space(4))) // read-only for the whole kernel: uniform loads become scalar

typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
typedef u32x4 u32x4_a4 __attribute__((aligned(4))); // 16 bytes at a 4-byte-aligned address

// The Heatmap counters of a counted launch (sec. 3.7 Heatmap): set with
// hipMemcpyAsync before the launch.  A counted kernel variant adds one to a
// blob's 32-bit counter of a byte for every global load that reads the byte
// (blobs in r) and every global store that writes it (blobs in w).
__device__ CountTable g_count_table;

__device__ __forceinline__ void count_range(const CountBlob* t, uint32_t nb, uint64_t a, uint32_t len)
{
    for (uint32_t k = 0; k < nb; k++) {
        const uint64_t lo = t[k].lo, hi = t[k].hi;
        if (a + len <= lo || a >= hi)
            continue;
        uint32_t* c = (uint32_t*)t[k].counters;
        for (uint64_t b = max(a, lo); b < min(a + len, hi); b++)
            atomicAdd(c + (b - lo), 1u);
    }
}

template <bool kCount>
__device__ __forceinline__ void note_read(uint64_t a, uint32_t len)
{
    if constexpr (kCount)
        count_range(g_count_table.r, g_count_table.nr, a, len);
}

template <bool kCount>
__device__ __forceinline__ void note_write(uint64_t a, uint32_t len)
{
    if constexpr (kCount)
        count_range(g_count_table.w, g_count_table.nw, a, len);
}

// A global store of one value, counted in a counted variant.
template <bool kCount, typename T>
__device__ __forceinline__ void gput(uint64_t a, T v)
{
    note_write<kCount>(a, sizeof(T));
    *(GLOBAL T*)a = v;
}

// A global load of one value, counted in a counted variant.
template <bool kCount, typename T>
__device__ __forceinline__ T gget(uint64_t a)
{
    note_read<kCount>(a, sizeof(T));
    return *(const GLOBAL T*)a;
}

__device__ __forceinline__ uint32_t wave_id()
{
    return __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
}

__device__ __forceinline__ uint32_t uniform(uint32_t x) { return __builtin_amdgcn_readfirstlane(x); }

// Copies a read-only table record word by word (scalar loads for a uniform address).
template <typename T>
__device__ __forceinline__ T load_const(const CONSTANT T* p)
{
    static_assert(sizeof(T) % 4 == 0, "table records are whole words");
    T v;
    const CONSTANT uint32_t* src = (const CONSTANT uint32_t*)p;
    uint32_t* dst = (uint32_t*)&v;
#pragma unroll
    for (uint32_t k = 0; k < sizeof(T) / 4; k++)
        dst[k] = src[k];
    return v;
}

// 16-byte loads of source bytes.  A copy reads every source byte once;
// kOnce adds the nontemporal hint, for sources larger than the 256 MB
// Infinity Cache, which streams them past the caches (a plain copy from HBM
// measured 6.19 -> 6.52 TB/s with it, reads alone 6.79 -> 7.09 TB/s; a
// 58 MB batch of frames that the cache holds lost 8% with it).
template <bool kOnce, bool kCount = false>
__device__ __forceinline__ u32x4 load_src(const GLOBAL u32x4* p)
{
    note_read<kCount>(uint64_t(p), 16);
    if constexpr (kOnce)
        return __builtin_nontemporal_load(p);
    else
        return *p;
}

// The same at a 4-byte-aligned address.
template <bool kOnce, bool kCount = false>
__device__ __forceinline__ u32x4 load_src_a4(const GLOBAL u32x4_a4* p)
{
    note_read<kCount>(uint64_t(p), 16);
    if constexpr (kOnce)
        return __builtin_nontemporal_load(p);
    else
        return *p;
}

// A 16-byte store of destination bytes; kStream marks it nontemporal, for
// destinations far larger than the 256 MB Infinity Cache (tile copies of
// 1.9 GB measured +3-5% with it; copies of a few hundred MB lose up to 9%,
// because plain stores can leave part of the writes in that cache).
template <bool kStream, bool kCount = false>
__device__ __forceinline__ void store16(GLOBAL u32x4* p, u32x4 v)
{
    note_write<kCount>(uint64_t(p), 16);
    if constexpr (kStream)
        __builtin_nontemporal_store(v, p);
    else
        *p = v;
}

// One 16-byte global load per active lane, written by the memory system
// straight into LDS at m0 + 16 * lane (global_load_lds_dwordx4).  Issued as
// inline assembly so that the compiler does not wait for these loads at every
// later barrier: the only wave that issues them waits for them itself before
// the barrier that publishes the buffer.
#pragma clang diagnostic push
#pragma clang diagnostic ignored "-Winline-asm" // m0 is written here and used by nothing else in these kernels
// kOnce: with the nontemporal hint (see load_src).
template <bool kOnce, bool kCount = false>
__device__ __forceinline__ void lds_dma16(uint64_t gaddr, uint32_t lds_addr)
{
    note_read<kCount>(gaddr, 16);
    if constexpr (kOnce)
        asm volatile("s_mov_b32 m0, %1\n\tglobal_load_lds_dwordx4 %0, off nt" : : "v"(gaddr), "s"(lds_addr)
                     : "memory", "m0");
    else
        asm volatile("s_mov_b32 m0, %1\n\tglobal_load_lds_dwordx4 %0, off" : : "v"(gaddr), "s"(lds_addr)
                     : "memory", "m0");
}
#pragma clang diagnostic pop

// Loads bytes [gstart, gstart + len) into LDS at lds_region + (gstart & 15):
// whole 16-byte granules from gstart rounded down, 64 granules (1 KiB) per
// wave instruction; chunk c of the span goes to wave (c + first_wave) mod
// nwaves.  A granule that holds a byte of the span lies in the same page as
// that byte, so the rounding never reaches an unmapped page; the extra bytes
// are never used.
template <bool kOnce, bool kCount = false>
__device__ __forceinline__ void load_span(uint64_t gstart, uint32_t len, uint32_t lds_region, uint32_t wave,
                                          uint32_t nwaves, uint32_t first_wave, uint32_t lane, uint32_t lds_base)
{
    const uint32_t shift = uint32_t(gstart) & 15u;
    const uint64_t g0 = gstart - shift;
    const uint32_t G = (shift + len + 15u) >> 4;
    const uint32_t c0 = wave >= first_wave ? wave - first_wave : wave + nwaves - first_wave;
    for (uint32_t c = c0; c * 64u < G; c += nwaves) {
        const uint32_t gi = c * 64u + lane;
        if (gi < G)
            lds_dma16<kOnce, kCount>(g0 + uint64_t(gi) * 16u, uniform(lds_base + lds_region + c * 1024u));
    }
}

// The source region of tile t gathered from several parts (kTileVirtualSrc):
// ceil(nv / L) virtual blocks of K bytes, granule by granule.  LDS granule q
// of the region lies in virtual block b = q / (K / 16); the last chunk that
// starts at or before the granule's byte in the block gives its global
// address.  A leaf chunk's granules past the tile's records with values are
// not loaded (the remap never reads those bytes), so no load reaches past the
// end of an SoA part's leaf; part blocks are whole in their blob.
template <bool kOnce, bool kCount, typename Entries>
__device__ __forceinline__ void load_virtual(const TileHeader& h, Entries ent, uint64_t t, uint32_t nv, uint32_t wave,
                                             uint32_t nwaves, uint32_t lane, uint32_t lds_base)
{
    const uint32_t gpb = uint32_t(h.src.block >> 4);
    const uint32_t L = uint32_t(h.src.lanes);
    const uint32_t nvb = (nv + L - 1u) >> h.src.log2_lanes;
    const uint32_t G = nvb * gpb;
    const uint64_t tile_blocks = uint64_t(t) << (h.log2_tile - h.src.log2_lanes);
    for (uint32_t c = wave; c * 64u < G; c += nwaves) {
        const uint32_t q = c * 64u + lane;
        const uint32_t b = __umulhi(q, h.src.pad); // q / gpb
        const uint32_t off = (q - b * gpb) * 16u;  // byte of the granule in its virtual block
        uint64_t ga = 0;
        uint32_t rel = 0, valid = 0;
        for (uint32_t k = 0; k < h.slots; k++) {
            const auto& ch = ent(h.num_entries + k);
            if (off >= ch.src_pos) {
                rel = off - ch.src_pos;
                ga = ch.src_addr + (tile_blocks + b) * ch.dst_addr + rel;
                valid = ch.move ? min(ch.size, (nv - b * L) * ch.move) : ch.size;
            }
        }
        if (q < G && rel < valid)
            lds_dma16<kOnce, kCount>(ga, uniform(lds_base + h.src.lds_base + c * 1024u));
    }
}

// Stores LDS bytes lds_region + (gstart & 15) .. into [gstart, gstart + len):
// whole granules with 16-byte stores, the partial first and last granule byte
// by byte so that no byte outside the span is written.  Granule gi goes to
// thread (gi + rot) mod nthr, so that short spans spread over the waves.
template <bool kStream, bool kCount = false>
__device__ __forceinline__ void store_span(uint64_t gstart, uint32_t len, uint32_t lds_region, uint32_t tid,
                                           uint32_t nthr, uint32_t rot, const uint8_t* lds)
{
    const uint32_t shift = uint32_t(gstart) & 15u;
    const uint64_t g0 = gstart - shift;
    const uint32_t end = shift + len;
    const uint32_t G = (end + 15u) >> 4;
    for (uint32_t gi = tid >= rot ? tid - rot : tid + nthr - rot; gi < G; gi += nthr) {
        const uint32_t lo = gi == 0 ? shift : 0u;
        const uint32_t hi = min(16u, end - gi * 16u);
        const uint8_t* lp = lds + lds_region + gi * 16u;
        if (lo == 0 && hi == 16) {
            store16<kStream, kCount>((GLOBAL u32x4*)(g0 + uint64_t(gi) * 16u), *(const u32x4*)lp);
        } else {
            const uint64_t gp = g0 + uint64_t(gi) * 16u;
            for (uint32_t b = lo; b < hi; b++)
                gput<kCount>(gp + b, lp[b]);
        }
    }
}

// Global start of the field-major span of one leaf for the records of the
// tile that starts at record i0.
__device__ __forceinline__ uint64_t field_span_start(uint64_t addr, const TileSide& s, uint64_t i0, uint32_t size)
{
    if (s.lanes == 0)
        return addr + i0 * size;
    return addr + (i0 >> s.log2_lanes) * s.block + (i0 & (s.lanes - 1)) * size;
}

// Device address of 16-byte granule g of a leaf's values in a tile, from the
// leaf's tile base; `lg` is log2 of the leaf size.  A field-major side holds
// the values as one span; an AoSoA side as lane runs of 2^(log2 L + lg - 4)
// granules, one per block (the planner ensures a run is whole granules).
template <bool kRecordMajorSide>
__device__ __forceinline__ uint64_t leaf_granule_addr(uint64_t base, const TileSide& s, uint32_t g, uint32_t lg)
{
    if constexpr (!kRecordMajorSide) {
        return base + uint64_t(g) * 16u;
    } else {
        const uint32_t run = s.log2_lanes + lg - 4u;
        return base + uint64_t(g >> run) * s.block + uint64_t(g & ((1u << run) - 1u)) * 16u;
    }
}

// Device address of a leaf's first value in tile t (records i0 ..): a
// record-major side advances by whole tiles, a field-major side by values.
template <bool kRecordMajorSide>
__device__ __forceinline__ uint64_t leaf_tile_base(uint64_t addr, const TileSide& s, uint64_t t, uint64_t i0,
                                                   uint32_t size)
{
    if constexpr (kRecordMajorSide)
        return addr + t * s.tile_bytes;
    else
        return field_span_start(addr, s, i0, size);
}

// Moves one entry of records r0, r0 + step, r0 + 2 step, r0 + 3 step inside
// LDS in words of type T; records >= nv, and gap entries, receive zeros.  The
// four loads are issued before the four stores.
template <typename T>
__device__ __forceinline__ void move4(uint8_t* lds, uint32_t sp, uint32_t dp, const TileSide& s, const TileSide& d,
                                      uint32_t size, uint32_t r0, uint32_t step, uint32_t nv, uint32_t nd, bool gap)
{
    for (uint32_t k = 0; k < size; k += sizeof(T)) {
        T v[4];
#pragma unroll
        for (uint32_t j = 0; j < 4; j++) {
            const uint32_t r = r0 + j * step;
            v[j] = T{};
            if (!gap && r < nv)
                v[j] = *(const T*)(lds + sp + (r >> s.pos_lg) * s.pos_k + (r & s.pos_m) * size + k);
        }
#pragma unroll
        for (uint32_t j = 0; j < 4; j++) {
            const uint32_t r = r0 + j * step;
            if (r < nd)
                *(T*)(lds + dp + (r >> d.pos_lg) * d.pos_k + (r & d.pos_m) * size + k) = v[j];
        }
    }
}

// A value of T (2, 4 or 8 bytes) at LDS byte p aligned to 2^rd bytes: read
// whole when rd allows, else assembled from the aligned 4-byte words that hold
// it (funnel shifts).  The words may reach up to 4 bytes past the value; in a
// staged tile the destination region follows the source region, so the read
// stays inside the workgroup's LDS, and the extra bytes are shifted out.
template <typename T>
__device__ __forceinline__ T read_split(const uint8_t* lds, uint32_t p, uint32_t rd)
{
    if ((1u << rd) >= sizeof(T))
        return *(const T*)(lds + p);
    const uint32_t* w = (const uint32_t*)(lds + (p & ~3u));
    const uint32_t sh = (p & 3u) * 8u;
    const uint32_t w0 = w[0], w1 = w[1];
    const uint32_t lo = uint32_t(((uint64_t(w1) << 32) | w0) >> sh);
    if constexpr (sizeof(T) == 8) {
        const uint32_t w2 = w[2];
        const uint32_t hi = uint32_t(((uint64_t(w2) << 32) | w1) >> sh);
        return T((uint64_t(hi) << 32) | lo);
    } else {
        return T(lo);
    }
}

// Writes a value of T at LDS byte p aligned to 2^wr bytes, in pieces of that
// alignment (at most sizeof(T)).
template <typename T>
__device__ __forceinline__ void write_split(uint8_t* lds, uint32_t p, T v, uint32_t wr)
{
    const uint64_t x = uint64_t(v);
    if ((1u << wr) >= sizeof(T)) {
        *(T*)(lds + p) = v;
    } else if (wr == 2) {
        *(uint32_t*)(lds + p) = uint32_t(x);
        *(uint32_t*)(lds + p + 4) = uint32_t(x >> 32);
    } else if (wr == 1) {
#pragma unroll
        for (uint32_t k = 0; k < sizeof(T); k += 2)
            *(uint16_t*)(lds + p + k) = uint16_t(x >> (8 * k));
    } else {
#pragma unroll
        for (uint32_t k = 0; k < sizeof(T); k++)
            lds[p + k] = uint8_t(x >> (8 * k));
    }
}

// move4 for a split entry (kMoveSplit): the values are sizeof(T) bytes, read
// at alignment 2^rd and written at alignment 2^wr.
template <typename T>
__device__ __forceinline__ void move4_split(uint8_t* lds, uint32_t sp, uint32_t dp, const TileSide& s,
                                            const TileSide& d, uint32_t r0, uint32_t step, uint32_t nv, uint32_t nd,
                                            uint32_t rd, uint32_t wr)
{
    constexpr uint32_t size = sizeof(T);
    T v[4];
#pragma unroll
    for (uint32_t j = 0; j < 4; j++) {
        const uint32_t r = r0 + j * step;
        v[j] = T{};
        if (r < nv)
            v[j] = read_split<T>(lds, sp + (r >> s.pos_lg) * s.pos_k + (r & s.pos_m) * size, rd);
    }
#pragma unroll
    for (uint32_t j = 0; j < 4; j++) {
        const uint32_t r = r0 + j * step;
        if (r < nd)
            write_split<T>(lds, dp + (r >> d.pos_lg) * d.pos_k + (r & d.pos_m) * size, v[j], wr);
    }
}

// Reads value r of an entry from the source region (ld = log2 of its size).
template <typename T>
__device__ __forceinline__ T src_value(const uint8_t* lds, uint32_t sp, const TileSide& s, uint32_t r, uint32_t size)
{
    return *(const T*)(lds + sp + (r >> s.pos_lg) * s.pos_k + (r & s.pos_m) * size);
}

// Direct store of one leaf: every 16-byte granule of the leaf's destination
// values (a field-major span, or the lane runs of an AoSoA block) gathers
// 16 / size consecutive records from the source region; records >= nv (AoSoA
// lanes past the last record) are zero.  A field-major span that starts `ph`
// values past the 16-byte grid (the granules stay on the grid) and a granule
// that passes record nd are stored value by value, only for records 0 .. nd
// - 1 of the tile.  `gdst` is the leaf's tile base on side d.
// kSplit: source values sit at positions aligned to 2^rd bytes only (a packed
// record of odd size) and are read from the aligned words that hold them.
template <typename T, bool kDstRecordMajor, bool kStream, bool kCount, bool kSplit = false>
__device__ __forceinline__ void direct_store_leaf(const uint8_t* lds, uint32_t sp, const TileSide& s,
                                                  const TileSide& d, uint64_t gdst, uint32_t nv, uint32_t nd,
                                                  uint32_t tid, uint32_t nthr, uint32_t rot, uint32_t ph,
                                                  uint32_t rd = 4)
{
    constexpr uint32_t per = 16 / sizeof(T);
    const uint32_t G = (nd + ph + per - 1) / per;
    const uint64_t gbase = gdst - uint64_t(ph) * sizeof(T); // 16-byte aligned
    for (uint32_t g = tid >= rot ? tid - rot : tid + nthr - rot; g < G; g += nthr) {
        const int32_t r0 = int32_t(g * per) - int32_t(ph); // record of the granule's first value
        union {
            u32x4 v;
            T t[per];
        } u;
#pragma unroll
        for (uint32_t j = 0; j < per; j++) {
            const int32_t r = r0 + int32_t(j);
            if constexpr (kSplit && sizeof(T) >= 2 && sizeof(T) <= 8)
                u.t[j] = r >= 0 && uint32_t(r) < nv
                             ? read_split<T>(lds, sp + (uint32_t(r) >> s.pos_lg) * s.pos_k + (uint32_t(r) & s.pos_m) * sizeof(T), rd)
                             : T{};
            else
                u.t[j] = r >= 0 && uint32_t(r) < nv ? src_value<T>(lds, sp, s, uint32_t(r), sizeof(T)) : T{};
        }
        constexpr uint32_t lg = sizeof(T) == 16 ? 4 : sizeof(T) == 8 ? 3 : sizeof(T) == 4 ? 2 : sizeof(T) == 2 ? 1 : 0;
        const uint64_t a = leaf_granule_addr<kDstRecordMajor>(gbase, d, g, lg);
        if (r0 >= 0 && uint32_t(r0) + per <= nd) {
            store16<kStream, kCount>((GLOBAL u32x4*)a, u.v);
        } else {
#pragma unroll
            for (uint32_t j = 0; j < per; j++) {
                const int32_t r = r0 + int32_t(j);
                if (r >= 0 && uint32_t(r) < nd)
                    gput<kCount>(a + j * sizeof(T), u.t[j]);
            }
        }
    }
}

// Direct store of a tile: every leaf in turn, at the width of its values.
// kVirtualDst: each leaf's runs of L values lie in its own part, e.dst_pos
// bytes apart (kTileVirtualDst).
// kSplit: leaves whose source positions are aligned below their size (bits
// 24-26 of `move`: log2 of that alignment) are read from aligned words.
template <bool kDstRecordMajor, bool kStream, bool kCount, bool kVirtualDst = false, bool kSplit = false,
          typename Entries>
__device__ __forceinline__ void direct_store_tile(const TileHeader& h, Entries ent, uint64_t t, uint64_t i0,
                                                  uint32_t nv, uint32_t nd, uint32_t tid, uint32_t nthr,
                                                  const uint8_t* lds)
{
    for (uint32_t f = 0; f < h.num_leaves; f++) {
        const auto& e = ent(f);
        TileSide d = h.dst;
        uint64_t gdst;
        uint32_t ne = nd;
        if constexpr (kVirtualDst) {
            d.block = e.dst_pos;
            gdst = e.dst_addr + t * (uint64_t(e.dst_pos) << (h.log2_tile - h.dst.log2_lanes));
            if (e.move & kMoveValuesOnly)
                ne = nv;
        } else {
            gdst = leaf_tile_base<kDstRecordMajor>(e.dst_addr, h.dst, t, i0, e.size);
        }
        const uint32_t rot = (e.move >> 8) & 4095u;
        const uint32_t ph = (e.move >> 20) & 15u;
        const uint32_t sp = e.src_pos;
        if constexpr (kSplit) {
            const uint32_t rd = (e.move >> 24) & 7u;
            switch (e.move & 7u) {
            case 4: direct_store_leaf<u32x4, kDstRecordMajor, kStream, kCount>(lds, sp, h.src, d, gdst, nv, ne, tid, nthr, rot, ph); break;
            case 3: direct_store_leaf<uint64_t, kDstRecordMajor, kStream, kCount, true>(lds, sp, h.src, d, gdst, nv, ne, tid, nthr, rot, ph, rd); break;
            case 2: direct_store_leaf<uint32_t, kDstRecordMajor, kStream, kCount, true>(lds, sp, h.src, d, gdst, nv, ne, tid, nthr, rot, ph, rd); break;
            case 1: direct_store_leaf<uint16_t, kDstRecordMajor, kStream, kCount, true>(lds, sp, h.src, d, gdst, nv, ne, tid, nthr, rot, ph, rd); break;
            default: direct_store_leaf<uint8_t, kDstRecordMajor, kStream, kCount>(lds, sp, h.src, d, gdst, nv, ne, tid, nthr, rot, ph); break;
            }
            continue;
        }
        switch (e.move & 7u) {
        case 4: direct_store_leaf<u32x4, kDstRecordMajor, kStream, kCount>(lds, sp, h.src, d, gdst, nv, ne, tid, nthr, rot, ph); break;
        case 3: direct_store_leaf<uint64_t, kDstRecordMajor, kStream, kCount>(lds, sp, h.src, d, gdst, nv, ne, tid, nthr, rot, ph); break;
        case 2: direct_store_leaf<uint32_t, kDstRecordMajor, kStream, kCount>(lds, sp, h.src, d, gdst, nv, ne, tid, nthr, rot, ph); break;
        case 1: direct_store_leaf<uint16_t, kDstRecordMajor, kStream, kCount>(lds, sp, h.src, d, gdst, nv, ne, tid, nthr, rot, ph); break;
        default: direct_store_leaf<uint8_t, kDstRecordMajor, kStream, kCount>(lds, sp, h.src, d, gdst, nv, ne, tid, nthr, rot, ph); break;
        }
    }
}

// Direct load of a tile from a field-major source (leaf sizes 4, 8 or 16
// bytes): every thread loads its slots' granules into registers (all loads in
// flight together), then writes the values to the destination region.
// Records in [nv, nd) (AoSoA lanes past the last record) and gap entries are
// zero-filled.
// kSplit (kTileSplitDst): leaves of 1 and 2 bytes too, and destination
// positions aligned below the leaf size (bits 24-26 of `move`: log2 of that
// alignment), written in pieces of that alignment.
template <bool kSrcRecordMajor, bool kOnce, bool kCount, bool kSplit = false, typename Entries>
__device__ __forceinline__ void direct_load_tile(const TileHeader& h, Entries ent, uint64_t t, uint64_t i0,
                                                 uint32_t nv, uint32_t nd, uint8_t* lds)
{
    const uint32_t tid = threadIdx.x, nthr = blockDim.x, wave = wave_id(), lane = tid & 63u;
    u32x4 v[kDirectLoadSlots];
    // slot of (wave, j): q = wave * 64 + j * nthr + lane; its leaf is uniform,
    // and the slots grow with j, so each leaf search resumes from the last
    uint32_t f = 0;
#pragma unroll
    for (uint32_t j = 0; j < kDirectLoadSlots; j++) {
        const uint32_t q0 = uniform(wave * 64u + j * nthr);
        if (q0 >= h.slots)
            break;
        while (f + 1 < h.num_leaves && ent(f + 1).src_pos <= q0)
            f++;
        const auto& e = ent(f);
        const uint32_t g = q0 + lane - e.src_pos; // granule within the leaf's values of the tile
        if (g * 16u < nv * e.size)
            v[j] = load_src<kOnce, kCount>((const GLOBAL u32x4*)leaf_granule_addr<kSrcRecordMajor>(
                leaf_tile_base<kSrcRecordMajor>(e.src_addr, h.src, t, i0, e.size), h.src, g, e.move & 7u));
    }
    f = 0;
#pragma unroll
    for (uint32_t j = 0; j < kDirectLoadSlots; j++) {
        const uint32_t q0 = uniform(wave * 64u + j * nthr);
        if (q0 >= h.slots)
            break;
        while (f + 1 < h.num_leaves && ent(f + 1).src_pos <= q0)
            f++;
        const auto& e = ent(f);
        const uint32_t g = q0 + lane - e.src_pos;
        const uint32_t size = e.size; // 4, 8 or 16
        const uint32_t r0 = g << (4u - (e.move & 7u)); // first record of the granule
        if (g * 16u >= nv * size)
            continue;
        const uint32_t d0 = e.dst_pos + (r0 >> h.dst.pos_lg) * h.dst.pos_k + (r0 & h.dst.pos_m) * size;
        if constexpr (kSplit) {
            const uint32_t wr = (e.move >> 24) & 7u;
            const uint32_t w[4] = {v[j].x, v[j].y, v[j].z, v[j].w};
            auto pos = [&](uint32_t r) { return e.dst_pos + (r >> h.dst.pos_lg) * h.dst.pos_k + (r & h.dst.pos_m) * size; };
            if (size == 16) {
                *(u32x4*)(lds + d0) = v[j];
            } else if (size == 8) {
#pragma unroll
                for (uint32_t k = 0; k < 2; k++)
                    if (r0 + k < nv)
                        write_split<uint64_t>(lds, pos(r0 + k), (uint64_t(w[2 * k + 1]) << 32) | w[2 * k], wr);
            } else if (size == 4) {
#pragma unroll
                for (uint32_t k = 0; k < 4; k++)
                    if (r0 + k < nv)
                        write_split<uint32_t>(lds, pos(r0 + k), w[k], wr);
            } else if (size == 2) {
#pragma unroll
                for (uint32_t k = 0; k < 8; k++)
                    if (r0 + k < nv)
                        write_split<uint16_t>(lds, pos(r0 + k), uint16_t(w[k >> 1] >> (16u * (k & 1u))), wr);
            } else {
#pragma unroll
                for (uint32_t k = 0; k < 16; k++)
                    if (r0 + k < nv)
                        lds[pos(r0 + k)] = uint8_t(w[k >> 2] >> (8u * (k & 3u)));
            }
            continue;
        }
        if (size == 16) {
            *(u32x4*)(lds + d0) = v[j];
        } else if (size == 8) {
            *(uint2*)(lds + d0) = uint2{v[j].x, v[j].y};
            if (r0 + 1 < nv) {
                const uint32_t r = r0 + 1;
                *(uint2*)(lds + e.dst_pos + (r >> h.dst.pos_lg) * h.dst.pos_k + (r & h.dst.pos_m) * 8u) =
                    uint2{v[j].z, v[j].w};
            }
        } else {
            const uint32_t w[4] = {v[j].x, v[j].y, v[j].z, v[j].w};
#pragma unroll
            for (uint32_t k = 0; k < 4; k++) {
                const uint32_t r = r0 + k;
                if (r < nv)
                    *(uint32_t*)(lds + e.dst_pos + (r >> h.dst.pos_lg) * h.dst.pos_k + (r & h.dst.pos_m) * 4u) = w[k];
            }
        }
    }
    // zeros: every gap entry, and every leaf for records in [nv, nd)
    for (uint32_t k = 0; k < h.num_entries; k++) {
        const auto& e = ent(k);
        const bool gap = (e.move >> 31) != 0;
        const uint32_t first = gap ? 0u : nv;
        for (uint32_t r = first + tid; r < nd; r += nthr) {
            const uint32_t dp = e.dst_pos + (r >> h.dst.pos_lg) * h.dst.pos_k + (r & h.dst.pos_m) * e.size;
            for (uint32_t b = 0; b < e.size; b++)
                lds[dp + b] = 0;
        }
    }
}

// Gather store (kTileGatherStore): copies the planner's word table into LDS
// (at dst.lds_base) once per workgroup; the first tile's barrier publishes it.
__device__ __forceinline__ void gather_table(const TileHeader& h, const TileGather& gg, const uint32_t* table,
                                             uint8_t* lds)
{
    uint32_t* tab = (uint32_t*)(lds + h.dst.lds_base);
    for (uint32_t k = threadIdx.x; k < gg.table; k += blockDim.x)
        tab[k] = table[k];
}

// One piece of a destination word (a word-table entry, or an entry of a group
// of pieces): the 4 source bytes at LDS byte p = p0 + (blk >> q) * kq +
// ((blk & (2^q - 1)) << run) in destination super-block blk, read from the two
// aligned words that hold them, with the bytes the piece does not give
// cleared.  Bits 0-17: p0 (the source byte that the word's byte 0 lines up
// with), 18-22: run, 23-26: the word bytes the piece gives.
__device__ __forceinline__ uint32_t gather_piece(uint32_t x, uint32_t bq, uint32_t bm, const uint8_t* lds)
{
    const uint32_t p = (x & 0x3FFFFu) + bq + (bm << ((x >> 18) & 31u));
    const uint32_t* wp = (const uint32_t*)(lds + (p & ~3u));
    const uint32_t v = __builtin_amdgcn_alignbyte(wp[1], wp[0], p & 3u);
    // bit k of the 4-bit byte mask to all of byte k
    const uint32_t m = ((((x >> 23) & 15u) * 0x204081u) & 0x01010101u) * 0xFFu;
    return v & m;
}

// One byte of a word of three or four pieces: the LDS byte p0 + (blk >> q) *
// kq + ((blk & (2^q - 1)) << run) (p0 in bits 0-17, run in bits 18-22), or
// zero (bit 31).
__device__ __forceinline__ uint32_t gather_byte(uint32_t b, uint32_t bq, uint32_t bm, const uint8_t* lds)
{
    const uint32_t v = lds[(b & 0x3FFFFu) + bq + (bm << ((b >> 18) & 31u))];
    return (b >> 31) ? 0u : v;
}

// Records without values in a tile's source region ([nv, nd): the tail lanes
// of the last AoSoA block) read as zero, so that the gather store needs no
// per-record test: their leaf bytes in LDS are cleared.
template <typename Entries>
__device__ __forceinline__ void zero_source_records(const TileHeader& h, Entries ent, uint32_t nv, uint32_t nd,
                                                    uint32_t tid, uint32_t nthr, uint8_t* lds)
{
    for (uint32_t f = 0; f < h.num_leaves; f++) {
        const auto& e = ent(f);
        for (uint32_t r = nv + tid; r < nd; r += nthr) {
            const uint32_t p = e.src_pos + (r >> h.src.pos_lg) * h.src.pos_k + (r & h.src.pos_m) * e.size;
            for (uint32_t b = 0; b < e.size; b++)
                lds[p + b] = 0;
        }
    }
}

// Gather store of one tile: every thread assembles 16-byte granules of the
// destination span word by word from the source region and stores them.  A
// word is one piece (its entry in the table), two or four pieces (a group of
// entries the table points to); padding bytes belong to no piece and stay
// zero, and so do records without values (cleared in the source region).
template <bool kStream, bool kOdd, bool kCount>
__device__ __forceinline__ void gather_store_tile(const TileHeader& h, const TileGather& gg, uint64_t t, uint32_t nd,
                                                  uint32_t tid, uint32_t nthr, const uint8_t* lds)
{
    const uint32_t* tab = (const uint32_t*)(lds + h.dst.lds_base);
    const uint32_t qm = (1u << gg.q) - 1u;
    // the span's bytes; a block of odd size can end it inside a word
    const uint32_t span = uint32_t(((uint64_t(nd) + h.dst.lanes - 1) >> h.dst.log2_lanes) * h.dst.block);
    const uint32_t words = (span + 3u) >> 2;
    const uint64_t gbase = h.dst.span_base + t * h.dst.tile_bytes;
    for (uint32_t u = tid * 4u; u < words; u += nthr * 4u) {
        uint32_t blk = __umulhi(u, gg.magic);
        uint32_t w = u - blk * gg.words;
        uint32_t v[4];
#pragma unroll
        for (uint32_t c = 0; c < 4; c++) {
            const uint32_t e = tab[w];
            const uint32_t bq = (blk >> gg.q) * gg.kq, bm = blk & qm;
            const uint32_t kind = e >> 30;
            uint32_t x, e1 = kind == 0u ? e : 0u;
            if (__any(kind == 1u)) {
                // a wave with words of two pieces reads two for every word
                // (a second piece of a one-piece word gives no byte), in one
                // path instead of two divergent ones
                const uint2 g = *(const uint2*)(tab + (kind == 1u ? (e & 0xFFFFu) : 0u));
                uint32_t e2 = 0u;
                if (kind == 1u) {
                    e1 = g.x;
                    e2 = g.y;
                }
                x = gather_piece(e1, bq, bm, lds) | gather_piece(e2, bq, bm, lds);
            } else {
                x = gather_piece(e1, bq, bm, lds);
            }
            if (kind == 2u) { // three or four pieces: byte by byte
                const u32x4 g = *(const u32x4*)(tab + (e & 0xFFFFu));
                x = gather_byte(g.x, bq, bm, lds) | (gather_byte(g.y, bq, bm, lds) << 8) |
                    (gather_byte(g.z, bq, bm, lds) << 16) | (gather_byte(g.w, bq, bm, lds) << 24);
            }
            v[c] = x;
            if (++w == gg.words) {
                w = 0;
                blk++;
            }
        }
        const uint64_t a = gbase + uint64_t(u) * 4u;
        if ((u + 4u) * 4u <= span) {
            store16<kStream, kCount>((GLOBAL u32x4*)a, u32x4{v[0], v[1], v[2], v[3]});
        } else if (!kOdd) { // the span's last granule: whole words (blocks of whole words)
#pragma unroll
            for (uint32_t c = 0; c < 4; c++)
                if (u + c < words)
                    gput<kCount>(a + 4u * c, v[c]);
        } else { // the span's last granule: whole words, then the bytes of a partial word
#pragma unroll
            for (uint32_t c = 0; c < 4; c++) {
                const uint32_t b = (u + c) * 4u;
                if (b + 4u <= span)
                    gput<kCount>(a + 4u * c, v[c]);
                else
                    for (uint32_t k = 0; b + k < span; k++)
                        gput<kCount>(a + 4u * c + k, uint8_t(v[c] >> (8u * k)));
            }
        }
    }
}

// One tile: every wave issues its share of the source loads straight into
// LDS, then all threads move the values to their destination positions
// inside LDS, then all threads store the destination span(s).  `ent(k)`
// returns entry k (kernel arguments for one copy, the work table for a batch).
// Kernel variants: kModeAny dispatches on the plan's flags at run time (the
// batch kernel); the single-copy kernel is compiled once per mode so that each
// mode gets its own register allocation.
enum : uint32_t {
    kModeAny = 0,
    kModeStaged = 1,
    kModeDirectStore = 2,
    kModeDirectLoad = 3,
    kModeGatherStore = 4,
    kModeGatherOdd = 5, // gather store with kTileGatherOdd
    kModeStreamUnits = 6 // the batch kernel over long-run items only
};
// added to a mode: the tile's 16-byte destination stores are nontemporal
constexpr uint32_t kModeStreamStores = 8;
// added to a mode: the tile's source loads are nontemporal
constexpr uint32_t kModeStreamLoads = 16;
// added to a mode: every global load and store is counted (Heatmap)
constexpr uint32_t kModeCount = 32;
// added to a mode: the source region is gathered from several parts
// (kTileVirtualSrc)
constexpr uint32_t kModeVirtualSrc = 64;
// added to kModeDirectStore: the destination is scattered over several parts
// (kTileVirtualDst)
constexpr uint32_t kModeVirtualDst = 128;
// added to kModeDirectStore: source values aligned below their size are read
// from aligned words (kTileSplitSrc)
constexpr uint32_t kModeSplitSrc = 256;
// added to kModeDirectLoad: leaves of 1 and 2 bytes, and destination values
// aligned below their size, written in pieces (kTileSplitDst)
constexpr uint32_t kModeSplitDst = 512;

template <uint32_t ModeBits, typename Entries>
__device__ __forceinline__ void tile_body(const TileHeader& h, Entries ent, uint64_t t, uint8_t* lds,
                                          const TileGather* gg = nullptr)
{
    constexpr uint32_t Mode = ModeBits & 7u;
    constexpr bool kStream = (ModeBits & kModeStreamStores) != 0;
    constexpr bool kOnce = (ModeBits & kModeStreamLoads) != 0;
    constexpr bool kCount = (ModeBits & kModeCount) != 0;
    constexpr bool kVirtual = (ModeBits & kModeVirtualSrc) != 0;
    constexpr bool kVirtualDst = (ModeBits & kModeVirtualDst) != 0;
    constexpr bool kSplitSrc = (ModeBits & kModeSplitSrc) != 0;
    constexpr bool kSplitDst = (ModeBits & kModeSplitDst) != 0;
    // the batch kernel (kModeAny) takes split reads and writes from the plan
    const bool split_src = kSplitSrc || (Mode == kModeAny && (h.flags & kTileSplitSrc));
    const bool split_dst = kSplitDst || (Mode == kModeAny && (h.flags & kTileSplitDst));
    const bool dload = Mode == kModeDirectLoad || (Mode == kModeAny && (h.flags & kTileDirectLoad));
    const bool dstore = Mode == kModeDirectStore || (Mode == kModeAny && (h.flags & kTileDirectStore));
    const bool gstore = Mode == kModeGatherStore || Mode == kModeGatherOdd ||
                        (Mode == kModeAny && (h.flags & kTileGatherStore));
    const uint32_t tid = threadIdx.x, nthr = blockDim.x;
    const uint32_t lane = tid & 63u, wave = wave_id(), nwaves = nthr >> 6;
    const uint32_t lds_base = uint32_t(uintptr_t((lds_void_t*)lds));
    const uint32_t T = 1u << h.log2_tile;
    const uint64_t i0 = t << h.log2_tile;
    const uint32_t nv = i0 < h.n ? uint32_t(min<uint64_t>(T, h.n - i0)) : 0u; // records with values
    const uint32_t nd = uint32_t(min<uint64_t>(T, h.npad - i0));              // records the destination spans
    // kept padding: only records with values are written (a record-major
    // destination region is loaded first and stored back whole)
    const bool preserve = (h.flags & kTilePreserve) != 0;
    const uint32_t ns = preserve ? nv : nd;

    // ---- 1. source span(s) -> LDS
    if (dload) {
        if (Mode == kModeAny && split_dst) {
            if (h.src.mode == kRecordMajor)
                direct_load_tile<true, kOnce, kCount, true>(h, ent, t, i0, nv, nd, lds);
            else
                direct_load_tile<false, kOnce, kCount, true>(h, ent, t, i0, nv, nd, lds);
        } else if (h.src.mode == kRecordMajor) {
            direct_load_tile<true, kOnce, kCount, kSplitDst>(h, ent, t, i0, nv, nd, lds);
        } else {
            direct_load_tile<false, kOnce, kCount, kSplitDst>(h, ent, t, i0, nv, nd, lds);
        }
    } else if (nv > 0) {
        if (kVirtual) {
            load_virtual<kOnce, kCount>(h, ent, t, nv, wave, nwaves, lane, lds_base);
        } else if (h.src.mode == kRecordMajor) {
            const uint32_t len = uint32_t(((uint64_t(nv) + h.src.lanes - 1) >> h.src.log2_lanes) * h.src.block);
            load_span<kOnce, kCount>(h.src.span_base + t * h.src.tile_bytes, len, h.src.lds_base, wave, nwaves, 0, lane, lds_base);
        } else {
            for (uint32_t f = 0; f < h.num_leaves; f++) {
                const auto& e = ent(f);
                load_span<kOnce, kCount>(field_span_start(e.src_addr, h.src, i0, e.size), nv * e.size, e.src_pos & ~15u, wave,
                          nwaves, (e.move >> 4) & 15u, lane, lds_base);
            }
        }
    }
    if (preserve && !dstore && h.dst.mode == kRecordMajor) {
        const uint32_t len = uint32_t(((uint64_t(nd) + h.dst.lanes - 1) >> h.dst.log2_lanes) * h.dst.block);
        load_span<false, kCount>(h.dst.span_base + t * h.dst.tile_bytes, len, h.dst.lds_base, wave, nwaves, 0, lane, lds_base);
    }
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();

    if (dload) {
        // ---- 2''. the destination region is complete: store it
        if (h.dst.mode == kRecordMajor) {
            const uint32_t len = uint32_t(((uint64_t(nd) + h.dst.lanes - 1) >> h.dst.log2_lanes) * h.dst.block);
            store_span<kStream, kCount>(h.dst.span_base + t * h.dst.tile_bytes, len, h.dst.lds_base, tid, nthr, 0, lds);
        } else {
            for (uint32_t f = 0; f < h.num_leaves; f++) {
                const auto& e = ent(f);
                store_span<kStream, kCount>(field_span_start(e.dst_addr, h.dst, i0, e.size), nd * e.size, e.dst_pos & ~15u, tid,
                           nthr, (e.move >> 8) & 4095u, lds);
            }
        }
        return;
    }

    if (gstore) {
        // ---- 2'''. assemble every destination granule word by word from
        //           the source region and store it; no destination region
        if (nv < nd) {
            zero_source_records(h, ent, nv, nd, tid, nthr, lds);
            __syncthreads();
        }
        if (Mode == kModeGatherOdd || (Mode == kModeAny && (h.flags & kTileGatherOdd)))
            gather_store_tile<kStream, true, kCount>(h, *gg, t, nd, tid, nthr, lds);
        else
            gather_store_tile<kStream, false, kCount>(h, *gg, t, nd, tid, nthr, lds);
        return;
    }

    if (dstore) {
        // ---- 2'. gather each destination granule from the source region and
        //          store it; no destination region, no second barrier
        if (kVirtualDst)
            direct_store_tile<true, kStream, kCount, true>(h, ent, t, i0, nv, ns, tid, nthr, lds);
        else if (Mode == kModeAny && split_src && h.dst.mode == kRecordMajor)
            direct_store_tile<true, kStream, kCount, false, true>(h, ent, t, i0, nv, ns, tid, nthr, lds);
        else if (Mode == kModeAny && split_src)
            direct_store_tile<false, kStream, kCount, false, true>(h, ent, t, i0, nv, ns, tid, nthr, lds);
        else if (h.dst.mode == kRecordMajor)
            direct_store_tile<true, kStream, kCount, false, kSplitSrc>(h, ent, t, i0, nv, ns, tid, nthr, lds);
        else
            direct_store_tile<false, kStream, kCount, false, kSplitSrc>(h, ent, t, i0, nv, ns, tid, nthr, lds);
        return;
    }

    // ---- 2. every value from its source to its destination position;
    //         destination padding becomes zero (or, kept, is left as loaded)
    for (uint32_t k = 0; k < h.num_entries; k++) {
        const auto& e = ent(k);
        const bool gap = (e.move >> 31) != 0;
        if (gap && preserve)
            continue;
        if (e.move & kMoveSplit) {
            const uint32_t rd = (e.move >> 20) & 7u, wr = (e.move >> 24) & 7u;
            for (uint32_t r0 = tid; r0 < ns; r0 += 4u * nthr) {
                switch (e.size) {
                case 2: move4_split<uint16_t>(lds, e.src_pos, e.dst_pos, h.src, h.dst, r0, nthr, nv, ns, rd, wr); break;
                case 4: move4_split<uint32_t>(lds, e.src_pos, e.dst_pos, h.src, h.dst, r0, nthr, nv, ns, rd, wr); break;
                default: move4_split<uint64_t>(lds, e.src_pos, e.dst_pos, h.src, h.dst, r0, nthr, nv, ns, rd, wr); break;
                }
            }
            continue;
        }
        for (uint32_t r0 = tid; r0 < ns; r0 += 4u * nthr) {
            switch (e.move & 7u) {
            case 4: move4<u32x4>(lds, e.src_pos, e.dst_pos, h.src, h.dst, e.size, r0, nthr, nv, ns, gap); break;
            case 3: move4<uint64_t>(lds, e.src_pos, e.dst_pos, h.src, h.dst, e.size, r0, nthr, nv, ns, gap); break;
            case 2: move4<uint32_t>(lds, e.src_pos, e.dst_pos, h.src, h.dst, e.size, r0, nthr, nv, ns, gap); break;
            case 1: move4<uint16_t>(lds, e.src_pos, e.dst_pos, h.src, h.dst, e.size, r0, nthr, nv, ns, gap); break;
            default: move4<uint8_t>(lds, e.src_pos, e.dst_pos, h.src, h.dst, e.size, r0, nthr, nv, ns, gap); break;
            }
        }
    }
    __syncthreads();

    // ---- 3. LDS -> destination span(s)
    if (h.dst.mode == kRecordMajor) {
        const uint32_t len = uint32_t(((uint64_t(nd) + h.dst.lanes - 1) >> h.dst.log2_lanes) * h.dst.block);
        store_span<kStream, kCount>(h.dst.span_base + t * h.dst.tile_bytes, len, h.dst.lds_base, tid, nthr, 0, lds);
    } else {
        for (uint32_t f = 0; f < h.num_leaves; f++) {
            const auto& e = ent(f);
            store_span<kStream, kCount>(field_span_start(e.dst_addr, h.dst, i0, e.size), ns * e.size, e.dst_pos & ~15u, tid, nthr,
                       (e.move >> 8) & 4095u, lds);
        }
    }
}

template <uint32_t ModeBits>
__global__ void __launch_bounds__(1024) tile_kernel(const TileArgs a)
{
    constexpr uint32_t Mode = ModeBits & 7u;
    extern __shared__ __attribute__((aligned(16))) uint8_t lds[];
    auto ent = [&](uint32_t k) -> const TileEntry& { return a.e[k]; };
    const uint64_t nt = a.h.num_tiles;
    uint64_t t = blockIdx.x, stride = gridDim.x;
    if (Mode != kModeStaged && gridDim.x == nt) {
        // one workgroup per tile: workgroups are dispatched to the 8 XCDs in
        // turn, so block b goes to XCD b mod 8; give each XCD one contiguous
        // eighth of the tiles (a bijection for any tile count).  Measured
        // +4-7% for the direct modes, -2.5% for the staged one, which keeps
        // the plain order.  One call site of tile_body: a second inlined
        // copy changed how the compiler unrolled the direct-load registers
        // and moved them to scratch.
        const uint64_t b = blockIdx.x, x = b & 7u, k = b >> 3, q = nt >> 3, rem = nt & 7u;
        t = x * q + min(x, rem) + k;
        stride = nt;
    }
    if (Mode == kModeGatherStore || Mode == kModeGatherOdd) // the word table follows the entries (and chunks)
        gather_table(a.h, a.gather,
                     reinterpret_cast<const uint32_t*>(a.e + a.h.num_entries + ((ModeBits & kModeVirtualSrc) ? a.h.slots : 0u)),
                     lds);
    for (; t < nt; t += stride) {
        tile_body<ModeBits>(a.h, ent, t, lds, &a.gather);
        if (t + stride < nt)
            __syncthreads();
    }
}

// The counted variant of tile_kernel (plain loads and stores; one workgroup
// per tile in plain order, or a grid-stride loop), for the Heatmap.
template <uint32_t Mode>
__global__ void __launch_bounds__(1024) tile_count_kernel(const TileArgs a)
{
    extern __shared__ __attribute__((aligned(16))) uint8_t lds[];
    auto ent = [&](uint32_t k) -> const TileEntry& { return a.e[k]; };
    if ((Mode & 7u) == kModeGatherStore || (Mode & 7u) == kModeGatherOdd)
        gather_table(a.h, a.gather,
                     reinterpret_cast<const uint32_t*>(a.e + a.h.num_entries + ((Mode & kModeVirtualSrc) ? a.h.slots : 0u)),
                     lds);
    for (uint64_t t = blockIdx.x; t < a.h.num_tiles; t += gridDim.x) {
        tile_body<Mode | kModeCount>(a.h, ent, t, lds, &a.gather);
        if (t + gridDim.x < a.h.num_tiles)
            __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// STREAM
// ---------------------------------------------------------------------------

// Copies [src, src + len) to [dst, dst + len) (src == 0: writes zeros);
// src and dst are congruent modulo 4.
template <bool kOnce, bool kCount = false>
__device__ __forceinline__ void copy_run_chunk(uint64_t dst, uint64_t src, uint64_t len, uint32_t tid, uint32_t nthr)
{
    const uint32_t head = uint32_t(min<uint64_t>(len, (16u - (uint32_t(dst) & 15u)) & 15u));
    const uint64_t body = (len - head) & ~uint64_t(15);
    const uint32_t tail = uint32_t(len - head - body);
    const bool zero = src == 0;
    // head and tail bytes
    if (tid < head)
        gput<kCount>(dst + tid, zero ? uint8_t(0) : gget<kCount, uint8_t>(src + tid));
    if (tid < tail) {
        const uint64_t o = head + body + tid;
        gput<kCount>(dst + o, zero ? uint8_t(0) : gget<kCount, uint8_t>(src + o));
    }
    // 16-byte granules: 4 per thread in flight
    GLOBAL u32x4* d = (GLOBAL u32x4*)(dst + head);
    const uint64_t ng = body >> 4;
    if (zero) {
        for (uint64_t g = tid; g < ng; g += nthr)
            gput<kCount>(uint64_t(d + g), u32x4{0u, 0u, 0u, 0u});
        return;
    }
    if (((src + head) & 15u) == 0) {
        const GLOBAL u32x4* s = (const GLOBAL u32x4*)(src + head);
        uint64_t g = tid;
        for (; g + 3u * nthr < ng; g += 4u * nthr) {
            u32x4 v0 = load_src<kOnce, kCount>(s + g), v1 = load_src<kOnce, kCount>(s + g + nthr),
                  v2 = load_src<kOnce, kCount>(s + g + 2u * nthr), v3 = load_src<kOnce, kCount>(s + g + 3u * nthr);
            gput<kCount>(uint64_t(d + g), v0);
            gput<kCount>(uint64_t(d + g + nthr), v1);
            gput<kCount>(uint64_t(d + g + 2u * nthr), v2);
            gput<kCount>(uint64_t(d + g + 3u * nthr), v3);
        }
        for (; g < ng; g += nthr)
            gput<kCount>(uint64_t(d + g), load_src<kOnce, kCount>(s + g));
    } else {
        const GLOBAL u32x4_a4* s = (const GLOBAL u32x4_a4*)(src + head);
        uint64_t g = tid;
        for (; g + 3u * nthr < ng; g += 4u * nthr) {
            const u32x4 v0 = load_src_a4<kOnce, kCount>(s + g), v1 = load_src_a4<kOnce, kCount>(s + g + nthr),
                        v2 = load_src_a4<kOnce, kCount>(s + g + 2u * nthr),
                        v3 = load_src_a4<kOnce, kCount>(s + g + 3u * nthr);
            gput<kCount>(uint64_t(d + g), v0);
            gput<kCount>(uint64_t(d + g + nthr), v1);
            gput<kCount>(uint64_t(d + g + 2u * nthr), v2);
            gput<kCount>(uint64_t(d + g + 3u * nthr), v3);
        }
        for (; g < ng; g += nthr)
            gput<kCount>(uint64_t(d + g), load_src_a4<kOnce, kCount>(s + g));
    }
}

// Work unit c of a run list: the run holding chunk c is the last run whose
// first chunk is <= c.  `run(k)` returns run k.
// Chunks are 2^chunk_log2 bytes.
template <bool kOnce, bool kCount, typename Runs>
__device__ __forceinline__ void stream_unit(Runs run, uint32_t num_runs, uint64_t c, uint32_t chunk_log2)
{
    uint32_t lo = 0, hi = num_runs;
    while (hi - lo > 1) {
        const uint32_t mid = (lo + hi) >> 1;
        if (run(mid).first_chunk <= c)
            lo = mid;
        else
            hi = mid;
    }
    const auto& r = run(lo);
    const uint64_t off = (c - r.first_chunk) << chunk_log2;
    const uint64_t len = min<uint64_t>(r.bytes - off, uint64_t(1) << chunk_log2);
    copy_run_chunk<kOnce, kCount>(r.dst + off, r.src ? r.src + off : 0, len, threadIdx.x, blockDim.x);
}

// kOnce: nontemporal source loads (StreamArgs.flags & kStreamLoadsOnce).
template <bool kOnce>
__global__ void __launch_bounds__(1024) stream_kernel(const StreamArgs a)
{
    auto run = [&](uint32_t k) -> const StreamRun& { return a.r[k]; };
    for (uint64_t c = blockIdx.x; c < a.num_chunks; c += gridDim.x)
        stream_unit<kOnce, false>(run, a.num_runs, c, kStreamChunkLog2);
}

// The counted variant of stream_kernel (plain loads), for the Heatmap.
__global__ void __launch_bounds__(1024) stream_count_kernel(const StreamArgs a)
{
    auto run = [&](uint32_t k) -> const StreamRun& { return a.r[k]; };
    for (uint64_t c = blockIdx.x; c < a.num_chunks; c += gridDim.x)
        stream_unit<false, true>(run, a.num_runs, c, kStreamChunkLog2);
}

// ---------------------------------------------------------------------------
// BATCH
// ---------------------------------------------------------------------------

// Persistent kernel over the work units of many copies.  Each workgroup takes
// a block of consecutive units from an atomic counter (an eighth of the
// remaining units per workgroup, between 1 and 64, so that blocks shrink
// towards the end) until the counter passes the total; the last workgroup to
// finish puts both counters back to zero, so the next launch (a graph replay
// included) starts from zero without a memset.
// Runs work unit g of item j (begin[j] <= g < begin[j + 1]).
// `table_item`: the item whose gather word table the workgroup's LDS holds
// (the table is copied when a unit of another gathering item comes).
template <bool kOnce, uint32_t Mode = kModeAny>
__device__ __forceinline__ void batch_unit(const BatchArgs& a, const CONSTANT uint64_t* begin, uint32_t j,
                                           uint64_t g, uint8_t* lds, uint32_t& table_item)
{
    const CONSTANT BatchItem* it = (const CONSTANT BatchItem*)a.items + j;
    const uint64_t u = g - begin[j];
    // a launch for one tile mode holds tile items only, a launch for
    // kModeStreamUnits long-run items only (a table sorted by mode)
    constexpr bool kGatherMode = (Mode & 7u) == kModeGatherStore || (Mode & 7u) == kModeGatherOdd;
    if (Mode != kModeStreamUnits && (Mode != kModeAny || it->kind == kItemTile)) {
        const TileHeader h = load_const(&it->h);
        const CONSTANT TileEntry* entries = (const CONSTANT TileEntry*)a.entries + it->first;
        TileGather gg{};
        if (kGatherMode || (Mode == kModeAny && (h.flags & kTileGatherStore))) {
            gg = load_const(&it->gather);
            if (table_item != j) {
                // the previous unit's barrier has ended every read of the
                // region; this unit's first barrier publishes the table
                gather_table(h, gg, (const uint32_t*)(entries + h.num_entries), lds);
                table_item = j;
            }
        } else if (h.lds_bytes > 0) {
            table_item = ~0u; // this unit's regions may cover the table
        }
        tile_body<Mode | (kOnce ? kModeStreamLoads : 0u)>(
            h, [&](uint32_t k) -> const CONSTANT TileEntry& { return entries[k]; }, u, lds, &gg);
    } else {
        const CONSTANT StreamRun* runs = (const CONSTANT StreamRun*)a.runs + it->first;
        stream_unit<kOnce, false>([&](uint32_t k) -> const CONSTANT StreamRun& { return runs[k]; }, it->count, u,
                           kBatchStreamChunkLog2);
    }
}

// The item holding unit g: the last j with begin[j] <= g.
__device__ __forceinline__ uint32_t batch_item_of(const CONSTANT uint64_t* begin, uint32_t num_items, uint64_t g)
{
    uint32_t lo = 0, hi = num_items;
    while (hi - lo > 1) {
        const uint32_t mid = (lo + hi) >> 1;
        if (begin[mid] <= g)
            lo = mid;
        else
            hi = mid;
    }
    return lo;
}

// One workgroup per work unit, the default batch launch: the dispatcher
// starts workgroups as residency allows, as for single copies, which
// measured faster than any persistent grid; unit g's item is found by binary
// search over the unit prefix sums, between the hints of g's block of units.  With as many workgroups as units, each
// XCD takes one contiguous eighth of the units (as tile_kernel does).
template <bool kOnce>
__global__ void __launch_bounds__(1024) batch_unit_kernel(const BatchArgs a)
{
    extern __shared__ __attribute__((aligned(16))) uint8_t lds[];
    const CONSTANT uint64_t* begin = (const CONSTANT uint64_t*)a.unit_begin;
    const uint64_t nt = a.total_units;
    uint64_t g = blockIdx.x, stride = gridDim.x;
    if (gridDim.x == nt) {
        const uint64_t b = blockIdx.x, x = b & 7u, k = b >> 3, q = nt >> 3, rem = nt & 7u;
        g = x * q + min(x, rem) + k;
        stride = nt;
    }
    const CONSTANT uint32_t* hint = (const CONSTANT uint32_t*)a.hint;
    uint32_t table_item = ~0u;
    for (; g < nt; g += stride) {
        // the item lies between the hints of g's block of units
        const uint64_t c = g >> kBatchHintLog2;
        uint32_t lo = hint[c], hi = min(hint[c + 1] + 1u, a.num_items);
        while (hi - lo > 1) {
            const uint32_t mid = (lo + hi) >> 1;
            if (begin[mid] <= g)
                lo = mid;
            else
                hi = mid;
        }
        batch_unit<kOnce>(a, begin, lo, g, lds, table_item);
        if (g + stride < nt)
            __syncthreads();
    }
}

// One launch per tile mode over a table sorted by mode: workgroup k runs
// unit first + k of a range whose items all take one mode (Mode, or kModeAny
// for long-run items), so each mode runs in its own compiled body and
// register allocation, with the range's own LDS reservation.
template <bool kOnce, uint32_t Mode>
__global__ void __launch_bounds__(1024) batch_mode_kernel(const BatchArgs a, uint64_t first, uint64_t count)
{
    extern __shared__ __attribute__((aligned(16))) uint8_t lds[];
    const CONSTANT uint64_t* begin = (const CONSTANT uint64_t*)a.unit_begin;
    uint64_t k = blockIdx.x, stride = gridDim.x;
    if (gridDim.x == count) { // each XCD takes one contiguous eighth of the range
        const uint64_t b = blockIdx.x, x = b & 7u, kk = b >> 3, q = count >> 3, rem = count & 7u;
        k = x * q + min(x, rem) + kk;
        stride = count;
    }
    const CONSTANT uint32_t* hint = (const CONSTANT uint32_t*)a.hint;
    uint32_t table_item = ~0u;
    for (; k < count; k += stride) {
        const uint64_t g = first + k;
        const uint64_t c = g >> kBatchHintLog2;
        uint32_t lo = hint[c], hi = min(hint[c + 1] + 1u, a.num_items);
        while (hi - lo > 1) {
            const uint32_t mid = (lo + hi) >> 1;
            if (begin[mid] <= g)
                lo = mid;
            else
                hi = mid;
        }
        batch_unit<kOnce, Mode>(a, begin, lo, g, lds, table_item);
        if (k + stride < count)
            __syncthreads();
    }
}

// kOnce: nontemporal source loads (BatchArgs.flags & kBatchLoadsOnce).
template <bool kOnce>
__global__ void __launch_bounds__(1024) batch_kernel(const BatchArgs a)
{
    extern __shared__ __attribute__((aligned(16))) uint8_t lds[];
    __shared__ unsigned long long block_first, block_count;
    const CONSTANT uint64_t* begin = (const CONSTANT uint64_t*)a.unit_begin;
    uint64_t seen = 0; // thread 0: the counter after its last block
    uint32_t table_item = ~0u;
    for (;;) {
        if (threadIdx.x == 0) {
            const uint64_t remaining = a.total_units > seen ? a.total_units - seen : 0;
            const uint64_t want = min<uint64_t>(max<uint64_t>(remaining / (8ull * gridDim.x), 1ull), 64ull);
            block_first = atomicAdd(&a.counters[0], (unsigned long long)want);
            block_count = want;
            seen = block_first + want;
        }
        __syncthreads();
        const uint64_t g0 = __builtin_amdgcn_readfirstlane(uint32_t(block_first)) |
                            (uint64_t(__builtin_amdgcn_readfirstlane(uint32_t(block_first >> 32))) << 32);
        const uint64_t g1 = min<uint64_t>(g0 + __builtin_amdgcn_readfirstlane(uint32_t(block_count)), a.total_units);
        __syncthreads();
        if (g0 >= a.total_units)
            break;
        uint32_t lo = batch_item_of(begin, a.num_items, g0);
        for (uint64_t g = g0; g < g1; g++) {
            while (begin[lo + 1] <= g)
                lo++;
            batch_unit<kOnce>(a, begin, lo, g, lds, table_item);
            __syncthreads();
        }
    }
    if (threadIdx.x == 0) {
        __threadfence();
        if (atomicAdd(&a.counters[1], 1ull) == gridDim.x - 1ull) {
            __threadfence();
            atomicExch(&a.counters[0], 0ull);
            atomicExch(&a.counters[1], 0ull);
        }
    }
}

// ---------------------------------------------------------------------------
// BOX: records at different linear indices on the two sides (sub-boxes,
// differing linearizers); see BoxArgs
// ---------------------------------------------------------------------------

// The fast dimension of an order's runs (-1: none).
__device__ __forceinline__ int box_fast(uint32_t order, uint32_t rank)
{
    return order == kOrderRow ? int(rank) - 1 : order == kOrderCol ? 0 : -1;
}

// Tile-local coordinate x of element e of run k (for row and column orders,
// e is the coordinate in the fast dimension).  The run index ravels the
// other dimensions, last fastest; a Morton run's element is the Morton index
// inside the tile's cube.
template <int R>
__device__ __forceinline__ void box_coord(const BoxHeader& h, uint32_t order, uint32_t k, uint32_t e, uint32_t* x)
{
    const uint32_t r = h.rank;
    if (order == kOrderMorton) {
#pragma unroll
        for (uint32_t d = 0; d < R; d++)
            x[d] = 0;
        for (uint32_t j = 0; j < h.qlog[0]; j++)
#pragma unroll
            for (uint32_t d = 0; d < R; d++)
                if (d < r)
                    x[d] |= ((e >> (j * r + r - 1 - d)) & 1u) << j;
        return;
    }
    const int fast = box_fast(order, r);
    uint32_t rem = k;
#pragma unroll
    for (int d = R - 1; d >= 0; d--) {
        if (d >= int(r)) {
            x[d] = 0;
        } else if (d == fast) {
            x[d] = e;
        } else {
            x[d] = rem & ((1u << h.qlog[d]) - 1u);
            rem >>= h.qlog[d];
        }
    }
}

// The inverse of box_coord: run k and element e of tile-local coordinate x.
template <int R>
__device__ __forceinline__ void box_run(const BoxHeader& h, uint32_t order, const uint32_t* x, uint32_t& k, uint32_t& e)
{
    const uint32_t r = h.rank;
    k = 0;
    e = 0;
    if (order == kOrderOne)
        return;
    if (order == kOrderMorton) {
        for (uint32_t j = 0; j < h.qlog[0]; j++)
#pragma unroll
            for (uint32_t d = 0; d < R; d++)
                if (d < r)
                    e |= ((x[d] >> j) & 1u) << (j * r + r - 1 - d);
        return;
    }
    const int fast = box_fast(order, r);
#pragma unroll
    for (int d = 0; d < R; d++) {
        if (d >= int(r))
            continue;
        if (d == fast)
            e = x[d];
        else
            k = (k << h.qlog[d]) | x[d];
    }
}

// Linear index of the absolute coordinate c on side s (its linearizer).
template <int R>
__device__ __forceinline__ uint64_t box_linear(const BoxSide& s, uint32_t r, const uint64_t* c)
{
    uint64_t i = 0;
    if (s.lin == kLinMorton) {
        for (uint32_t j = 0; j < s.morton_bits; j++)
#pragma unroll
            for (uint32_t d = 0; d < R; d++)
                if (d < r)
                    i |= ((c[d] >> j) & 1ull) << (j * r + r - 1 - d);
    } else if (s.lin == kLinCol) {
#pragma unroll
        for (int d = R - 1; d >= 0; d--)
            if (d < int(r))
                i = i * s.extent[d] + c[d];
    } else {
#pragma unroll
        for (int d = 0; d < R; d++)
            if (d < int(r))
                i = i * s.extent[d] + c[d];
    }
    return i;
}

// Records of run k whose start index is `start` (~0: an empty run): the
// clipped fast range for row and column orders, the cube up to the blob's
// end for a Morton run, one record otherwise.
__device__ __forceinline__ uint32_t box_run_len(const BoxSide& s, uint32_t Q, uint64_t start, uint32_t fast_len)
{
    if (start == ~0ull)
        return 0;
    if (s.order == kOrderRow || s.order == kOrderCol)
        return fast_len;
    if (s.order == kOrderMorton)
        return start >= s.npad ? 0u : uint32_t(min<uint64_t>(Q, s.npad - start));
    return 1;
}

// Copies `size` bytes inside LDS at the widest width both positions allow.
__device__ __forceinline__ void box_move_lds(uint8_t* lds, uint32_t sp, uint32_t dp, uint32_t size)
{
    const uint32_t al = sp | dp | size;
    if ((al & 7u) == 0) {
        for (uint32_t b = 0; b < size; b += 8)
            *(uint64_t*)(lds + dp + b) = *(const uint64_t*)(lds + sp + b);
    } else if ((al & 3u) == 0) {
        for (uint32_t b = 0; b < size; b += 4)
            *(uint32_t*)(lds + dp + b) = *(const uint32_t*)(lds + sp + b);
    } else if ((al & 1u) == 0) {
        for (uint32_t b = 0; b < size; b += 2)
            *(uint16_t*)(lds + dp + b) = *(const uint16_t*)(lds + sp + b);
    } else {
        for (uint32_t b = 0; b < size; b++)
            lds[dp + b] = lds[sp + b];
    }
}

// Writes `size` bytes from LDS (sp; zero: zeros) to global address g at the
// widest width both allow.
template <bool kCount>
__device__ __forceinline__ void box_store_value(const uint8_t* lds, uint32_t sp, uint64_t g, uint32_t size, bool zero)
{
    const uint32_t al = (zero ? 0u : sp) | uint32_t(g) | size;
    if ((al & 7u) == 0) {
        for (uint32_t b = 0; b < size; b += 8)
            gput<kCount>(g + b, zero ? uint64_t(0) : *(const uint64_t*)(lds + sp + b));
    } else if ((al & 3u) == 0) {
        for (uint32_t b = 0; b < size; b += 4)
            gput<kCount>(g + b, zero ? uint32_t(0) : *(const uint32_t*)(lds + sp + b));
    } else if ((al & 1u) == 0) {
        for (uint32_t b = 0; b < size; b += 2)
            gput<kCount>(g + b, zero ? uint16_t(0) : *(const uint16_t*)(lds + sp + b));
    } else {
        for (uint32_t b = 0; b < size; b++)
            gput<kCount>(g + b, zero ? uint8_t(0) : lds[sp + b]);
    }
}

// The byte range of run k of side X (start index `start`, w records): its
// first byte and its length.  Record-major sides span whole blocks; a One
// source is its single record.
__device__ __forceinline__ void box_span(const BoxSide& X, uint64_t start, uint32_t w, uint64_t& g0, uint32_t& len)
{
    if (X.order == kOrderOne) {
        g0 = X.blob;
        len = uint32_t(X.block);
        return;
    }
    const uint64_t b0 = start >> X.log2_lanes, b1 = (start + w - 1) >> X.log2_lanes;
    g0 = X.blob + b0 * X.block;
    len = uint32_t((b1 - b0 + 1) * X.block);
}

// Loads the spans of a group into LDS with 16-byte DMA, every lane of every
// wave on one granule: span k of the group holds `gran` granules at LDS byte
// `base` + 16 gran k (its first byte at its global address mod 16); lanes
// past a span's granules load nothing.  `span(k, g0, len)` gives span k's
// global range (len 0: no span).
template <bool kCount, typename Span>
__device__ __forceinline__ void box_load_group(uint32_t base, uint32_t nspans, uint32_t gran, uint32_t magic,
                                               uint32_t wave, uint32_t nwaves, uint32_t lane, uint32_t lds_base,
                                               Span span)
{
    const uint32_t total = nspans * gran;
    for (uint32_t c = wave; c * 64u < total; c += nwaves) {
        const uint32_t g = c * 64u + lane;
        const uint32_t k = __umulhi(g, magic);
        const uint32_t gi = g - k * gran;
        uint64_t g0 = 0;
        uint32_t len = 0;
        if (g < total)
            span(k, g0, len);
        if (len > 0 && gi < ((uint32_t(g0) & 15u) + len + 15u) >> 4)
            lds_dma16<false, kCount>((g0 & ~uint64_t(15)) + uint64_t(gi) * 16u, uniform(lds_base + base + c * 1024u));
    }
}

// Record map entries (16 bytes per record of a tile, in the destination's
// order): a = kMapSkip (no record), kMapHole (a hole of a full copy: zeros),
// or the source position: record-major source: a = LDS byte of the record's
// block plus its phase, b = its lane; field-major: a = run, b = element, c =
// the run's start index (low bits).  d: staged destination: LDS byte of the
// destination record.
constexpr uint32_t kMapSkip = 0xFFFFFFFFu, kMapHole = 0xFFFFFFFEu;

// R: the largest rank this instantiation handles (loops over dimensions are
// unrolled to R, which keeps the per-dimension values in registers)
template <int R, bool kStaged, bool kCount>
__device__ __forceinline__ void box_body(const BoxArgs& a, uint64_t u, uint8_t* lds)
{
    const BoxHeader& h = a.h;
    const BoxSide &S = a.src, &D = a.dst;
    const uint32_t r = h.rank;
    const uint32_t tid = threadIdx.x, nthr = blockDim.x, lane = tid & 63u, wave = wave_id(), nwaves = nthr >> 6;
    const uint32_t lds_base = uint32_t(uintptr_t((lds_void_t*)lds));
    const uint32_t Q = 1u << h.qlog_sum;
    const bool full = (h.flags & kBoxFull) != 0, preserve = (h.flags & kBoxPreserve) != 0;

    // ---- the tile's frame origin in box coordinates
    int64_t o[R];
    if (h.flags & kBoxUnitMorton) {
        // cube u of the destination's Morton order: deinterleave u
        uint64_t c[R] = {};
        for (uint32_t j = 0; j * r < 64; j++)
#pragma unroll
            for (uint32_t d = 0; d < R; d++)
                if (d < r && j * r + r - 1 - d < 64)
                    c[d] |= ((u >> (j * r + r - 1 - d)) & 1ull) << j;
#pragma unroll
        for (uint32_t d = 0; d < R; d++)
            o[d] = d < r ? int64_t(c[d] << h.qlog[d]) : 0;
    } else {
        // the unit count and every grid extent fit 32 bits (checked by the planner)
        uint32_t rem = uint32_t(u);
#pragma unroll
        for (int d = R - 1; d >= 0; d--) {
            o[d] = 0;
            if (d < int(r)) {
                const uint32_t g = uint32_t(h.grid[d]), q = rem / g, t = rem - q * g;
                rem = q;
                o[d] = int64_t(uint64_t(t) << h.qlog[d]) - int64_t(h.shift[d]);
            }
        }
    }
    // the clipped fast range of each side: [lo, lo + len)
    const int fs = box_fast(S.order, r), fd = box_fast(D.order, r);
    uint32_t lo_s = 0, len_s = 0, lo_d = 0, len_d = 0;
#pragma unroll
    for (int d = 0; d < R; d++) {
        if (d >= int(r))
            continue;
        const int64_t lo = max<int64_t>(0, -o[d]), hi = min<int64_t>(1ll << h.qlog[d], int64_t(h.box[d]) - o[d]);
        const uint32_t l = uint32_t(lo), n = hi > lo ? uint32_t(hi - lo) : 0u;
        if (d == fs) {
            lo_s = l;
            len_s = n;
        }
        if (d == fd) {
            lo_d = l;
            len_d = n;
        }
    }

    // ---- run tables: the start index of every run (~0: no record in the box);
    //      one side per loop, so that the side's fields stay uniform
    const uint32_t Rs = Q >> S.run_log2, Rd = Q >> D.run_log2;
    uint64_t* tab_s = (uint64_t*)(lds + S.table);
    uint64_t* tab_d = (uint64_t*)(lds + D.table);
    auto run_start = [&](const BoxSide& X, int fx, uint32_t lo, uint32_t len, uint32_t k) -> uint64_t {
        if (X.order == kOrderOne)
            return 0;
        uint32_t x[R];
        box_coord<R>(h, X.order, k, fx >= 0 ? lo : 0u, x);
        bool in = fx < 0 || len > 0;
        uint64_t c[R];
#pragma unroll
        for (uint32_t d = 0; d < R; d++) {
            c[d] = 0;
            if (d < r) {
                const int64_t b = o[d] + int64_t(x[d]);
                // a Morton run's cube may reach past the box: its records are
                // checked one by one
                if (X.order != kOrderMorton && (b < 0 || b >= int64_t(h.box[d])))
                    in = false;
                c[d] = uint64_t(int64_t(X.offset[d]) + b);
            }
        }
        return in ? box_linear<R>(X, r, c) : ~0ull;
    };
    for (uint32_t k = tid; k < Rs; k += nthr)
        tab_s[k] = run_start(S, fs, lo_s, len_s, k);
    for (uint32_t k = tid; k < Rd; k += nthr)
        tab_d[k] = (h.flags & kBoxUnitMorton) ? (u << h.qlog_sum) // the cube's first Morton index
                                              : run_start(D, fd, lo_d, len_d, k);
    __syncthreads();

    // ---- source runs -> LDS, granule by granule over all waves
    if (S.mode == kFieldMajor) {
        for (uint32_t f = 0; f < h.num_leaves; f++) {
            const BoxEntry& en = a.e[f];
            box_load_group<kCount>(S.lds_base + en.src_off, Rs, en.gran, en.magic, wave, nwaves, lane, lds_base,
                                   [&](uint32_t k, uint64_t& g0, uint32_t& len) {
                                       const uint64_t st = tab_s[k];
                                       const uint32_t w = box_run_len(S, Q, st, len_s);
                                       g0 = en.src_addr + st * en.size;
                                       len = w * en.size;
                                   });
        }
    } else {
        box_load_group<kCount>(S.lds_base, Rs, S.gran, S.magic, wave, nwaves, lane, lds_base,
                               [&](uint32_t k, uint64_t& g0, uint32_t& len) {
                                   const uint64_t st = tab_s[k];
                                   const uint32_t w = box_run_len(S, Q, st, len_s);
                                   len = 0;
                                   if (w > 0)
                                       box_span(S, st, w, g0, len);
                               });
    }
    if (kStaged && preserve) // kept padding: the destination records are loaded first
        box_load_group<kCount>(D.lds_base, Rd, D.gran, D.magic, wave, nwaves, lane, lds_base,
                               [&](uint32_t k, uint64_t& g0, uint32_t& len) {
                                   const uint64_t st = tab_d[k];
                                   const uint32_t w = box_run_len(D, Q, st, len_d);
                                   g0 = D.blob + st * D.block;
                                   len = w * uint32_t(D.block);
                               });

    // ---- the record map, in the destination's order (overlaps the loads)
    const uint32_t wlog = D.run_log2, wmask = (1u << wlog) - 1u;
    uint4* map = (uint4*)(lds + h.map);
    for (uint32_t j = tid; j < Q; j += nthr) {
        const uint32_t kd = j >> wlog, ed = j & wmask;
        const uint64_t sd = tab_d[kd];
        uint4 m{kMapSkip, 0u, 0u, 0u};
        if (ed < box_run_len(D, Q, sd, len_d)) {
            if (kStaged)
                m.w = D.lds_base + kd * (D.gran << 4) + ((uint32_t(D.blob) + uint32_t(sd) * uint32_t(D.block)) & 15u) +
                      ed * uint32_t(D.block);
            uint32_t x[R];
            box_coord<R>(h, D.order, kd, fd >= 0 ? lo_d + ed : ed, x);
            bool in = true;
#pragma unroll
            for (uint32_t d = 0; d < R; d++)
                if (d < r) {
                    const int64_t b = o[d] + int64_t(x[d]);
                    in = in && b >= 0 && b < int64_t(h.box[d]);
                }
            if (!in) {
                // a hole or tail lane of a full copy into a Morton destination
                m.x = full && !preserve ? kMapHole : kMapSkip;
            } else {
                uint32_t ks, es;
                box_run<R>(h, S.order, x, ks, es);
                if (fs >= 0)
                    es -= lo_s;
                const uint64_t ss = tab_s[ks];
                if (S.mode == kFieldMajor) {
                    m.x = ks;
                    m.y = es;
                    m.z = uint32_t(ss);
                } else if (S.order == kOrderOne) {
                    m.x = S.lds_base + (uint32_t(S.blob) & 15u);
                    m.y = 0;
                } else {
                    const uint64_t i = ss + es, b0 = ss >> S.log2_lanes;
                    m.x = S.lds_base + ks * (S.gran << 4) +
                          ((uint32_t(S.blob) + uint32_t(b0) * uint32_t(S.block)) & 15u) +
                          uint32_t((i >> S.log2_lanes) - b0) * uint32_t(S.block);
                    m.y = uint32_t(i & ((uint64_t(1) << S.log2_lanes) - 1u));
                }
            }
        }
        map[j] = m;
    }
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();

    // ---- every (entry, record) pair; the lanes of a wave hold consecutive
    //      records of one entry, whose fields then load as scalars
    const uint32_t E = h.num_entries;
    const uint64_t lmask = (uint64_t(1) << D.log2_lanes) - 1u;
    auto move = [&](const BoxEntry& en, uint32_t rec) {
        const uint4 m = map[rec];
        if (m.x == kMapSkip)
            return;
        const bool zero = en.gap || m.x == kMapHole;
        if (zero && preserve)
            return;
        uint32_t sp = 0;
        if (!zero)
            sp = S.mode == kFieldMajor
                     ? S.lds_base + en.src_off + m.x * (en.gran << 4) +
                           ((uint32_t(en.src_addr) + m.z * en.size) & 15u) + m.y * en.size
                     : m.x + en.src_off + m.y * en.size;
        if constexpr (kStaged) {
            if (zero) {
                for (uint32_t b = 0; b < en.size; b++)
                    lds[m.w + en.dst_off + b] = 0;
            } else {
                box_move_lds(lds, sp, m.w + en.dst_off, en.size);
            }
        } else {
            const uint64_t i = tab_d[rec >> wlog] + (rec & wmask);
            uint64_t g;
            if (en.gap)
                g = D.blob + i * D.block + en.dst_off; // an AoS destination (lanes 1)
            else if (D.mode == kFieldMajor)
                g = en.dst_addr + i * en.size;
            else
                g = en.dst_addr + (i >> D.log2_lanes) * D.block + (i & lmask) * en.size;
            box_store_value<kCount>(lds, sp, g, en.size, zero);
        }
    };
    if (kStaged && (h.flags & kBoxGather)) {
        // ---- AoS destination of whole words: every granule of every
        //      destination run assembled word by word, stored at once
        const uint32_t* wt = (const uint32_t*)(lds + h.wtab);
        const uint4* lf = (const uint4*)(lds + h.wtab + ((h.words * 4u + 15u) & ~15u));
        const uint32_t K = uint32_t(D.block);
        const uint32_t total = Rd * D.gran;
        for (uint32_t g = tid; g < total; g += nthr) {
            const uint32_t k = __umulhi(g, D.magic), gi = g - k * D.gran;
            const uint64_t st = tab_d[k];
            const uint32_t w = box_run_len(D, Q, st, len_d);
            if (w == 0)
                continue;
            const uint64_t g0 = D.blob + st * D.block;
            const uint32_t shift = uint32_t(g0) & 15u, end = shift + w * K;
            if (gi * 16u >= end)
                continue;
            uint32_t v[4];
#pragma unroll
            for (uint32_t c = 0; c < 4; c++) {
                v[c] = 0;
                const int32_t b = int32_t(gi * 16u + 4u * c) - int32_t(shift); // byte of the run's span
                if (b < 0 || uint32_t(b) >= w * K)
                    continue;
                const uint32_t rr = __umulhi(uint32_t(b), h.kmagic); // record of the run
                const uint32_t wi = (uint32_t(b) - rr * K) >> 2;
                const uint4 m = map[(k << wlog) + rr];
                const uint32_t e = wt[wi];
                if (m.x >= kMapHole || (e & 0xFFu) == kBoxWordZero)
                    continue; // a hole of a full copy, or a gap: zero
                const uint4 L = lf[e & 0xFFu]; // src_off, size, slot bytes, address low bits
                const uint32_t sp = S.mode == kFieldMajor
                                        ? S.lds_base + L.x + m.x * L.z + ((L.w + m.z * L.y) & 15u) + m.y * L.y
                                        : m.x + L.x + m.y * L.y;
                v[c] = *(const uint32_t*)(lds + sp + (e >> 8));
            }
            const uint64_t ga = (g0 & ~uint64_t(15)) + uint64_t(gi) * 16u;
            const uint32_t lo = gi == 0 ? shift : 0u, hi = min(16u, end - gi * 16u);
            if (lo == 0 && hi == 16) {
                store16<false, kCount>((GLOBAL u32x4*)ga, u32x4{v[0], v[1], v[2], v[3]});
            } else {
#pragma unroll
                for (uint32_t c = 0; c < 4; c++)
                    if (4u * c >= lo && 4u * c + 4u <= hi)
                        gput<kCount>(ga + 4u * c, v[c]);
            }
        }
        return;
    }
    if (h.qlog_sum >= 6) {
        // a wave's 64 consecutive pairs lie in one entry: all threads busy
        for (uint32_t j = tid; j < (E << h.qlog_sum); j += nthr)
            move(a.e[uniform(j >> h.qlog_sum)], j & (Q - 1u));
    } else {
        for (uint32_t f = 0; f < E; f++)
            for (uint32_t rec = tid; rec < Q; rec += nthr)
                move(a.e[f], rec);
    }

    if constexpr (kStaged) {
        // ---- destination runs: exact byte spans, granule by granule
        __syncthreads();
        const uint32_t total = Rd * D.gran;
        for (uint32_t g = tid; g < total; g += nthr) {
            const uint32_t k = __umulhi(g, D.magic), gi = g - k * D.gran;
            const uint64_t st = tab_d[k];
            const uint32_t w = box_run_len(D, Q, st, len_d);
            if (w == 0)
                continue;
            const uint64_t g0 = D.blob + st * D.block;
            const uint32_t shift = uint32_t(g0) & 15u, end = shift + w * uint32_t(D.block);
            if (gi * 16u >= end)
                continue;
            const uint32_t lo = gi == 0 ? shift : 0u, hi = min(16u, end - gi * 16u);
            const uint8_t* lp = lds + D.lds_base + g * 16u;
            const uint64_t ga = (g0 & ~uint64_t(15)) + uint64_t(gi) * 16u;
            if (lo == 0 && hi == 16) {
                store16<false, kCount>((GLOBAL u32x4*)ga, *(const u32x4*)lp);
            } else {
                for (uint32_t b = lo; b < hi; b++)
                    gput<kCount>(ga + b, lp[b]);
            }
        }
    }
}

template <int R, bool kStaged, bool kCount>
__global__ void __launch_bounds__(1024) box_kernel(const BoxArgs a)
{
    extern __shared__ __attribute__((aligned(16))) uint8_t lds[];
    if (kStaged && (a.h.flags & kBoxGather)) {
        // the word table, then per leaf its source fields (src_off, size,
        // slot bytes, address low bits), read by lanes of different leaves;
        // the first tile's barriers publish them
        uint32_t* t = (uint32_t*)(lds + a.h.wtab);
        for (uint32_t k = threadIdx.x; k < a.h.words; k += blockDim.x)
            t[k] = a.words[k];
        uint4* l = (uint4*)(lds + a.h.wtab + ((a.h.words * 4u + 15u) & ~15u));
        for (uint32_t f = threadIdx.x; f < a.h.num_leaves; f += blockDim.x)
            l[f] = uint4{a.e[f].src_off, a.e[f].size, a.e[f].gran << 4, uint32_t(a.e[f].src_addr)};
    }
    const uint64_t nt = a.h.num_units;
    uint64_t t = blockIdx.x, stride = gridDim.x;
    if (!kCount && gridDim.x == nt) { // each XCD one contiguous eighth of the tiles
        const uint64_t b = blockIdx.x, x = b & 7u, k = b >> 3, q = nt >> 3, rem = nt & 7u;
        t = x * q + min(x, rem) + k;
        stride = nt;
    }
    for (; t < nt; t += stride) {
        box_body<R, kStaged, kCount>(a, t, lds);
        if (t + stride < nt)
            __syncthreads();
    }
}

// The coordinate of linear index i on side s; false when no coordinate inside
// the view's extents has that index (a Morton hole, an AoSoA tail lane).
__device__ __forceinline__ bool box_delinear(const BoxSide& s, uint32_t r, uint64_t i, uint64_t* c)
{
    bool in = true;
    if (s.lin == kLinMorton) {
#pragma unroll
        for (uint32_t d = 0; d < LLAMA_MAX_RANK; d++)
            c[d] = 0;
        for (uint32_t j = 0; j < s.morton_bits; j++)
#pragma unroll
            for (uint32_t d = 0; d < LLAMA_MAX_RANK; d++)
                if (d < r)
                    c[d] |= ((i >> (j * r + r - 1 - d)) & 1ull) << j;
        if (s.morton_bits * r < 64 && (i >> (s.morton_bits * r)) != 0)
            in = false;
#pragma unroll
        for (uint32_t d = 0; d < LLAMA_MAX_RANK; d++)
            if (d < r && c[d] >= s.extent[d])
                in = false;
        return in;
    }
    uint64_t rem = i;
    if (s.lin == kLinCol) {
#pragma unroll
        for (int d = 0; d < LLAMA_MAX_RANK; d++) {
            c[d] = 0;
            if (d < int(r)) {
                c[d] = rem % s.extent[d];
                rem /= s.extent[d];
            }
        }
    } else {
#pragma unroll
        for (int d = LLAMA_MAX_RANK - 1; d >= 0; d--) {
            c[d] = 0;
            if (d < int(r)) {
                c[d] = rem % s.extent[d];
                rem /= s.extent[d];
            }
        }
    }
    return rem == 0;
}

// The element-wise baseline of a box copy: one thread per record of the box
// (row-major), both linear indices from the coordinate, every leaf moved at
// its own width, aligned-AoS gaps zeroed (kBoxPreserve: kept).  A full copy
// (kBoxFull) runs one thread per destination index instead, so that the
// indices no coordinate reaches (Morton holes, AoSoA tail lanes) get zeros.
template <bool kCount>
__global__ void __launch_bounds__(1024) box_naive_kernel(const BoxArgs a)
{
    const BoxHeader& h = a.h;
    const uint32_t r = h.rank;
    const bool full = (h.flags & kBoxFull) != 0, preserve = (h.flags & kBoxPreserve) != 0;
    uint64_t n = 1;
    if (full) {
        n = a.dst.npad;
    } else {
        for (uint32_t d = 0; d < r; d++)
            n *= h.box[d];
    }
    for (uint64_t i = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += uint64_t(gridDim.x) * blockDim.x) {
        uint64_t cs[LLAMA_MAX_RANK], cd[LLAMA_MAX_RANK], rem = i;
        bool in = true;
        uint64_t id = 0;
        if (full) {
            id = i;
            in = box_delinear(a.dst, r, i, cd);
#pragma unroll
            for (uint32_t d = 0; d < LLAMA_MAX_RANK; d++)
                cs[d] = cd[d];
        } else {
#pragma unroll
            for (int d = LLAMA_MAX_RANK - 1; d >= 0; d--) {
                cs[d] = cd[d] = 0;
                if (d < int(r)) {
                    const uint64_t c = rem % h.box[d];
                    rem /= h.box[d];
                    cs[d] = a.src.offset[d] + c;
                    cd[d] = a.dst.offset[d] + c;
                }
            }
            id = box_linear<LLAMA_MAX_RANK>(a.dst, r, cd);
        }
        const uint64_t is = (!in || a.src.order == kOrderOne) ? 0 : box_linear<LLAMA_MAX_RANK>(a.src, r, cs);
        for (uint32_t f = 0; f < h.num_entries; f++) {
            const BoxEntry& en = a.e[f];
            uint64_t gd;
            if (a.dst.mode == kFieldMajor)
                gd = en.dst_addr + id * en.size;
            else if (en.gap)
                gd = a.dst.blob + id * a.dst.block + en.dst_off;
            else
                gd = en.dst_addr + (id >> a.dst.log2_lanes) * a.dst.block +
                     (id & ((uint64_t(1) << a.dst.log2_lanes) - 1u)) * en.size;
            if (en.gap || !in) {
                if (!preserve)
                    for (uint32_t b = 0; b < en.size; b++)
                        gput<kCount>(gd + b, uint8_t(0));
                continue;
            }
            uint64_t gs;
            if (a.src.mode == kFieldMajor)
                gs = en.src_addr + is * en.size;
            else
                gs = a.src.blob + (is >> a.src.log2_lanes) * a.src.block + en.src_off +
                     (is & ((uint64_t(1) << a.src.log2_lanes) - 1u)) * en.size;
            const uint32_t al = uint32_t(gs) | uint32_t(gd) | en.size;
            if ((al & 7u) == 0)
                for (uint32_t b = 0; b < en.size; b += 8)
                    gput<kCount>(gd + b, gget<kCount, uint64_t>(gs + b));
            else if ((al & 3u) == 0)
                for (uint32_t b = 0; b < en.size; b += 4)
                    gput<kCount>(gd + b, gget<kCount, uint32_t>(gs + b));
            else
                for (uint32_t b = 0; b < en.size; b++)
                    gput<kCount>(gd + b, gget<kCount, uint8_t>(gs + b));
        }
    }
}

// ---------------------------------------------------------------------------
// NAIVE
// ---------------------------------------------------------------------------

template <typename T, bool kCount>
__device__ __forceinline__ void naive_move(uint64_t d, uint64_t s, uint32_t size, bool zero)
{
    for (uint32_t k = 0; k < size; k += sizeof(T))
        gput<kCount>(d + k, zero ? T(0) : gget<kCount, T>(s + k));
}

template <bool kCount>
__device__ __forceinline__ void naive_body(const NaiveArgs& a)
{
    const uint64_t stride = uint64_t(gridDim.x) * blockDim.x;
    for (uint64_t i = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < a.npad; i += stride) {
        for (uint32_t k = 0; k < a.num_entries; k++) {
            const NaiveEntry& e = a.e[k];
            const bool zero = e.src_addr == 0 || i >= a.n;
            if (zero && a.preserve)
                continue; // padding keeps its bytes
            const uint64_t doff = a.dst.lanes ? (i / a.dst.lanes) * a.dst.block + (i % a.dst.lanes) * e.size
                                              : i * e.size;
            uint64_t soff = 0;
            if (!zero)
                soff = a.src.lanes ? (i / a.src.lanes) * a.src.block + (i % a.src.lanes) * e.size : i * e.size;
            const uint64_t d = e.dst_addr + doff, s = e.src_addr + soff;
            switch (e.width) {
            case 8: naive_move<uint64_t, kCount>(d, s, e.size, zero); break;
            case 4: naive_move<uint32_t, kCount>(d, s, e.size, zero); break;
            case 2: naive_move<uint16_t, kCount>(d, s, e.size, zero); break;
            default: naive_move<uint8_t, kCount>(d, s, e.size, zero); break;
            }
        }
    }
}

__global__ void __launch_bounds__(1024) naive_kernel(const NaiveArgs a)
{
    naive_body<false>(a);
}

// The counted variant of naive_kernel, for the Heatmap.
__global__ void __launch_bounds__(1024) naive_count_kernel(const NaiveArgs a)
{
    naive_body<true>(a);
}

// ---------------------------------------------------------------------------
// HASH: a position-dependent 64-bit hash of a byte range, summed over
// 16-byte granules (the autotuner compares candidates' outputs with it)
// ---------------------------------------------------------------------------

__device__ __forceinline__ uint64_t mix64(uint64_t x)
{
    // the finaliser of splitmix64 (Steele, Lea and Flood, 2014)
    x ^= x >> 30;
    x *= 0xbf58476d1ce4e5b9ull;
    x ^= x >> 27;
    x *= 0x94d049bb133111ebull;
    x ^= x >> 31;
    return x;
}

__global__ void __launch_bounds__(256) hash_kernel(const uint8_t* p, uint64_t len, unsigned long long* acc)
{
    // byte k of the range contributes through the granule (k / 16) it falls in
    const uint64_t granules = (len + 15) / 16;
    uint64_t h = 0;
    for (uint64_t g = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x; g < granules;
         g += uint64_t(gridDim.x) * blockDim.x) {
        uint64_t lo = 0, hi = 0;
        const uint64_t n = min<uint64_t>(16, len - g * 16);
        for (uint64_t b = 0; b < n; b++) {
            const uint64_t v = ((const GLOBAL uint8_t*)p)[g * 16 + b];
            if (b < 8)
                lo |= v << (8 * b);
            else
                hi |= v << (8 * (b - 8));
        }
        h += mix64(lo ^ mix64(2 * g + 1)) + mix64(hi ^ mix64(2 * g + 2));
    }
    for (int off = 32; off > 0; off >>= 1)
        h += __shfl_xor(h, off);
    if ((threadIdx.x & 63) == 0)
        atomicAdd(acc, (unsigned long long)h);
}

// ---------------------------------------------------------------------------
// TRACE: per-leaf sums of a view's per-byte Heatmap counters, through the
// mapping's affine form (sec. 3.7 Trace counts accesses per field)
// ---------------------------------------------------------------------------

struct TraceLeaf {
    uint64_t counters; // device address of the counters of the leaf's blob
    uint64_t base;     // byte offset of the leaf's record 0 in that blob
    uint64_t lanes;    // L (0: unblocked)
    uint64_t block;    // K
    uint32_t size;
    uint32_t pad;
};

__global__ void __launch_bounds__(256) trace_kernel(const TraceLeaf* leaves, uint32_t nleaves, uint64_t n,
                                                    unsigned long long* out)
{
    const uint64_t stride = uint64_t(gridDim.x) * blockDim.x;
    for (uint32_t f = 0; f < nleaves; f++) {
        const TraceLeaf e = leaves[f];
        const GLOBAL uint32_t* c = (const GLOBAL uint32_t*)e.counters;
        uint64_t sum = 0;
        for (uint64_t i = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += stride) {
            const uint64_t off = e.lanes ? e.base + (i / e.lanes) * e.block + (i % e.lanes) * e.size
                                         : e.base + i * e.size;
            for (uint32_t b = 0; b < e.size; b++)
                sum += c[off + b];
        }
        for (int o = 32; o > 0; o >>= 1)
            sum += __shfl_xor(sum, o);
        if ((threadIdx.x & 63) == 0 && sum)
            atomicAdd(out + f, (unsigned long long)sum);
    }
}

__global__ void __launch_bounds__(256) counter_sum_kernel(const uint32_t* c, uint64_t len, unsigned long long* out)
{
    uint64_t sum = 0;
    for (uint64_t k = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x; k < len; k += uint64_t(gridDim.x) * blockDim.x)
        sum += ((const GLOBAL uint32_t*)c)[k];
    for (int o = 32; o > 0; o >>= 1)
        sum += __shfl_xor(sum, o);
    if ((threadIdx.x & 63) == 0 && sum)
        atomicAdd(out, (unsigned long long)sum);
}

void check_hip(hipError_t e, const char* what)
{
    if (e != hipSuccess)
        fail(LLAMA_E_HIP, std::string(what) + ": " + hipGetErrorString(e));
}

// tile_kernel variants by mode (kModeStaged .. kModeGatherOdd): plain loads
// and stores, then nontemporal loads, then nontemporal loads and stores
constexpr uint32_t kLd = kModeStreamLoads, kLdSt = kModeStreamLoads | kModeStreamStores;
constexpr uint32_t kTileModes = 5;
const void* const kTileKernels[3 * kTileModes] = {
    (const void*)tile_kernel<kModeStaged>, (const void*)tile_kernel<kModeDirectStore>,
    (const void*)tile_kernel<kModeDirectLoad>, (const void*)tile_kernel<kModeGatherStore>,
    (const void*)tile_kernel<kModeGatherOdd>,
    (const void*)tile_kernel<kModeStaged | kLd>, (const void*)tile_kernel<kModeDirectStore | kLd>,
    (const void*)tile_kernel<kModeDirectLoad | kLd>, (const void*)tile_kernel<kModeGatherStore | kLd>,
    (const void*)tile_kernel<kModeGatherOdd | kLd>,
    (const void*)tile_kernel<kModeStaged | kLdSt>, (const void*)tile_kernel<kModeDirectStore | kLdSt>,
    (const void*)tile_kernel<kModeDirectLoad | kLdSt>, (const void*)tile_kernel<kModeGatherStore | kLdSt>,
    (const void*)tile_kernel<kModeGatherOdd | kLdSt>};

const void* const kTileCountKernels[kTileModes] = {
    (const void*)tile_count_kernel<kModeStaged>, (const void*)tile_count_kernel<kModeDirectStore>,
    (const void*)tile_count_kernel<kModeDirectLoad>, (const void*)tile_count_kernel<kModeGatherStore>,
    (const void*)tile_count_kernel<kModeGatherOdd>};

// the same with the source gathered from several parts (kTileVirtualSrc);
// never with direct load
constexpr uint32_t kV = kModeVirtualSrc;
const void* const kTileVirtualKernels[3 * kTileModes] = {
    (const void*)tile_kernel<kModeStaged | kV>, (const void*)tile_kernel<kModeDirectStore | kV>, nullptr,
    (const void*)tile_kernel<kModeGatherStore | kV>, (const void*)tile_kernel<kModeGatherOdd | kV>,
    (const void*)tile_kernel<kModeStaged | kV | kLd>, (const void*)tile_kernel<kModeDirectStore | kV | kLd>, nullptr,
    (const void*)tile_kernel<kModeGatherStore | kV | kLd>, (const void*)tile_kernel<kModeGatherOdd | kV | kLd>,
    (const void*)tile_kernel<kModeStaged | kV | kLdSt>, (const void*)tile_kernel<kModeDirectStore | kV | kLdSt>, nullptr,
    (const void*)tile_kernel<kModeGatherStore | kV | kLdSt>, (const void*)tile_kernel<kModeGatherOdd | kV | kLdSt>};

// direct store into a destination scattered over several parts
// (kTileVirtualDst): plain, nontemporal loads, nontemporal loads and stores;
// then the counted variant
constexpr uint32_t kVD = kModeDirectStore | kModeVirtualDst;
const void* const kTileScatterKernels[4] = {(const void*)tile_kernel<kVD>, (const void*)tile_kernel<kVD | kLd>,
                                            (const void*)tile_kernel<kVD | kLdSt>,
                                            (const void*)tile_count_kernel<kVD>};

// direct store with split source reads (kTileSplitSrc) and direct load with
// split destination writes (kTileSplitDst): plain, nontemporal loads,
// nontemporal loads and stores; then the counted variant
constexpr uint32_t kSS = kModeDirectStore | kModeSplitSrc, kSD = kModeDirectLoad | kModeSplitDst;
const void* const kTileSplitSrcKernels[4] = {(const void*)tile_kernel<kSS>, (const void*)tile_kernel<kSS | kLd>,
                                             (const void*)tile_kernel<kSS | kLdSt>, (const void*)tile_count_kernel<kSS>};
const void* const kTileSplitDstKernels[4] = {(const void*)tile_kernel<kSD>, (const void*)tile_kernel<kSD | kLd>,
                                             (const void*)tile_kernel<kSD | kLdSt>, (const void*)tile_count_kernel<kSD>};

const void* const kTileVirtualCountKernels[kTileModes] = {
    (const void*)tile_count_kernel<kModeStaged | kV>, (const void*)tile_count_kernel<kModeDirectStore | kV>, nullptr,
    (const void*)tile_count_kernel<kModeGatherStore | kV>, (const void*)tile_count_kernel<kModeGatherOdd | kV>};

// box_kernel<R, staged, counted>: index (R == 8) * 4 + staged * 2 + counted
const void* const kBoxKernels[8] = {
    (const void*)box_kernel<4, false, false>, (const void*)box_kernel<4, false, true>,
    (const void*)box_kernel<4, true, false>,  (const void*)box_kernel<4, true, true>,
    (const void*)box_kernel<8, false, false>, (const void*)box_kernel<8, false, true>,
    (const void*)box_kernel<8, true, false>,  (const void*)box_kernel<8, true, true>};

const void* box_kernel_for(const BoxArgs& b, bool counted)
{
    return kBoxKernels[(b.h.rank > 4 ? 4 : 0) + ((b.h.flags & kBoxStaged) ? 2 : 0) + (counted ? 1 : 0)];
}

bool g_attr_set = false;

template <bool kOnce>
const void* batch_mode_kernel_for(uint32_t key);

void set_attributes()
{
    if (g_attr_set)
        return;
    for (const void* k : kTileKernels)
        check_hip(hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, int(kHardLdsBytes)),
                  "hipFuncSetAttribute(tile_kernel)");
    for (const void* k : kTileCountKernels)
        check_hip(hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, int(kHardLdsBytes)),
                  "hipFuncSetAttribute(tile_count_kernel)");
    for (const void* k : kBoxKernels)
        check_hip(hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, int(kHardLdsBytes)),
                  "hipFuncSetAttribute(box_kernel)");
    for (const void* const* table : {kTileVirtualKernels, kTileVirtualCountKernels, kTileScatterKernels,
                                     kTileSplitSrcKernels, kTileSplitDstKernels})
        for (size_t j = 0; j < (table == kTileVirtualKernels ? 3 * kTileModes : table == kTileVirtualCountKernels ? kTileModes : 4); j++)
            if (table[j])
                check_hip(hipFuncSetAttribute(table[j], hipFuncAttributeMaxDynamicSharedMemorySize, int(kHardLdsBytes)),
                          "hipFuncSetAttribute(tile_kernel variant)");
    for (uint32_t key : {uint32_t(kModeAny), uint32_t(kModeStreamUnits), uint32_t(kModeStaged), uint32_t(kModeDirectStore),
                         kModeDirectStore | kModeSplitSrc, uint32_t(kModeDirectLoad), kModeDirectLoad | kModeSplitDst,
                         uint32_t(kModeGatherStore), uint32_t(kModeGatherOdd)})
        for (const void* k : {batch_mode_kernel_for<false>(key), batch_mode_kernel_for<true>(key)})
            check_hip(hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, int(kHardLdsBytes)),
                      "hipFuncSetAttribute(batch_mode_kernel)");
    for (const void* k : {(const void*)batch_kernel<false>, (const void*)batch_kernel<true>,
                          (const void*)batch_unit_kernel<false>, (const void*)batch_unit_kernel<true>})
        check_hip(hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, int(kHardLdsBytes - 64)),
                  "hipFuncSetAttribute(batch_kernel)");
    g_attr_set = true;
}

constexpr uint64_t kMaxGrid = uint64_t(1) << 24;

} // namespace

uint32_t device_cu_count()
{
    static thread_local int cached_device = -1;
    static thread_local uint32_t cached = 0;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) {
        (void)hipGetLastError();
        return 256;
    }
    if (dev != cached_device) {
        int n = 0;
        if (hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || n <= 0) {
            (void)hipGetLastError();
            return 256;
        }
        cached_device = dev;
        cached = uint32_t(n);
    }
    return cached;
}

namespace {
thread_local bool t_counting = false; // launches on this thread take the counted variants
}

void set_counting(const CountTable* table, void* stream)
{
    if (!table) {
        t_counting = false;
        return;
    }
    void* sym = nullptr;
    check_hip(hipGetSymbolAddress(&sym, HIP_SYMBOL(g_count_table)), "hipGetSymbolAddress(g_count_table)");
    check_hip(hipMemcpyAsync(sym, table, sizeof(CountTable), hipMemcpyHostToDevice, (hipStream_t)stream),
              "hipMemcpyAsync(count table)");
    t_counting = true;
}

namespace {
void launch_one(const Plan& p, void* stream_ptr);
}

// A plan's launch, then the launches chained after it (the zero fill of an
// aligned SoA destination's padding).
void launch(const Plan& p, void* stream_ptr)
{
    for (const Plan* q = &p; q; q = q->then.get())
        launch_one(*q, stream_ptr);
}

namespace {
void launch_one(const Plan& p, void* stream_ptr)
{
    hipStream_t stream = (hipStream_t)stream_ptr;
    if (p.path == LLAMA_PATH_EMPTY || p.workgroups == 0)
        return;
    const uint32_t grid = uint32_t(std::min<uint64_t>(p.workgroups, kMaxGrid));
    if (trace_enabled())
        trace_plan(p);
    if (t_counting) {
        void* args[] = {p.path == LLAMA_PATH_TILE     ? (void*)&p.tile
                        : p.path == LLAMA_PATH_STREAM ? (void*)&p.stream
                                                      : (void*)&p.naive};
        const void* k = nullptr;
        uint32_t lds = 0;
        if (p.path == LLAMA_PATH_TILE) {
            set_attributes();
            const uint32_t f = p.tile.h.flags;
            const uint32_t mode = (f & kTileDirectLoad)    ? kModeDirectLoad
                                  : (f & kTileDirectStore) ? kModeDirectStore
                                  : (f & kTileGatherStore) ? ((f & kTileGatherOdd) ? kModeGatherOdd : kModeGatherStore)
                                                           : kModeStaged;
            k = (f & kTileVirtualSrc) ? kTileVirtualCountKernels[mode - 1] : kTileCountKernels[mode - 1];
            if (f & kTileVirtualDst)
                k = mode == kModeDirectStore && !(f & kTileVirtualSrc) ? kTileScatterKernels[3] : nullptr;
            if (f & kTileSplitSrc)
                k = mode == kModeDirectStore && !(f & (kTileVirtualSrc | kTileVirtualDst)) ? kTileSplitSrcKernels[3] : nullptr;
            if (f & kTileSplitDst)
                k = mode == kModeDirectLoad && !(f & kTileVirtualSrc) ? kTileSplitDstKernels[3] : nullptr;
            if (!k)
                fail(LLAMA_E_INVALID_ARG, "no kernel variant for this combination of gathered parts");
            lds = p.tile.h.lds_bytes;
        } else if (p.path == LLAMA_PATH_STREAM) {
            k = (const void*)stream_count_kernel;
        } else if (p.path == LLAMA_PATH_NAIVE) {
            k = (const void*)naive_count_kernel;
        } else if (p.path == LLAMA_PATH_BOX) {
            set_attributes();
            args[0] = (void*)&p.box;
            k = p.box_naive ? (const void*)box_naive_kernel<true> : box_kernel_for(p.box, true);
            lds = p.box_naive ? 0 : p.box.h.lds_bytes;
        } else {
            fail(LLAMA_E_INVALID_ARG, "unknown path");
        }
        check_hip(hipLaunchKernel(k, dim3(grid), dim3(p.threads), args, lds, stream), "hipLaunchKernel(counted)");
        check_hip(hipGetLastError(), "kernel launch");
        return;
    }
    switch (p.path) {
    case LLAMA_PATH_TILE: {
        set_attributes();
        const uint32_t f = p.tile.h.flags;
        const uint32_t mode = (f & kTileDirectLoad)    ? kModeDirectLoad
                              : (f & kTileDirectStore) ? kModeDirectStore
                              : (f & kTileGatherStore) ? ((f & kTileGatherOdd) ? kModeGatherOdd : kModeGatherStore)
                                                       : kModeStaged;
        // streaming stores come with streaming loads (a destination of 1 GiB
        // or more has a source of far more than 256 MB in every layout pair)
        const uint32_t variant = (f & kTileStreamStores) ? 2 : (f & kTileStreamLoads) ? 1 : 0;
        const void* k = ((f & kTileVirtualSrc) ? kTileVirtualKernels : kTileKernels)[(mode - 1) + kTileModes * variant];
        if (f & kTileVirtualDst)
            k = mode == kModeDirectStore && !(f & kTileVirtualSrc) ? kTileScatterKernels[variant] : nullptr;
        if (f & kTileSplitSrc)
            k = mode == kModeDirectStore && !(f & (kTileVirtualSrc | kTileVirtualDst)) ? kTileSplitSrcKernels[variant]
                                                                                     : nullptr;
        if (f & kTileSplitDst)
            k = mode == kModeDirectLoad && !(f & kTileVirtualSrc) ? kTileSplitDstKernels[variant] : nullptr;
        if (!k)
            fail(LLAMA_E_INVALID_ARG, "no kernel variant for this combination of gathered parts");
        void* args[] = {(void*)&p.tile};
        check_hip(hipLaunchKernel(k, dim3(grid), dim3(p.threads), args, p.tile.h.lds_bytes, stream),
                  "hipLaunchKernel(tile_kernel)");
        break;
    }
    case LLAMA_PATH_STREAM:
        if (p.stream.flags & kStreamLoadsOnce)
            hipLaunchKernelGGL(stream_kernel<true>, dim3(grid), dim3(p.threads), 0, stream, p.stream);
        else
            hipLaunchKernelGGL(stream_kernel<false>, dim3(grid), dim3(p.threads), 0, stream, p.stream);
        break;
    case LLAMA_PATH_NAIVE:
        hipLaunchKernelGGL(naive_kernel, dim3(grid), dim3(p.threads), 0, stream, p.naive);
        break;
    case LLAMA_PATH_BOX: {
        if (p.box_naive) {
            hipLaunchKernelGGL(box_naive_kernel<false>, dim3(grid), dim3(p.threads), 0, stream, p.box);
            break;
        }
        set_attributes();
        const void* k = box_kernel_for(p.box, false);
        void* args[] = {(void*)&p.box};
        check_hip(hipLaunchKernel(k, dim3(grid), dim3(p.threads), args, p.box.h.lds_bytes, stream),
                  "hipLaunchKernel(box_kernel)");
        break;
    }
    default:
        fail(LLAMA_E_INVALID_ARG, "unknown path");
    }
    check_hip(hipGetLastError(), "kernel launch");
}
} // namespace

void trace_leaves(const llama_mapping_desc* m, uint32_t* const* counters, uint64_t* sums, void* stream_ptr)
{
    hipStream_t stream = (hipStream_t)stream_ptr;
    const Record r = flatten(m->record);
    const Side s = make_side(m, r);
    if (s.kind == LLAMA_ONE)
        fail(LLAMA_E_UNSUPPORTED, "a One mapping puts every record at the same bytes; trace its single record");
    const uint32_t F = uint32_t(r.leaves.size());
    for (size_t b = 0; b < s.blob_size.size(); b++)
        if (!counters[b] && s.blob_size[b])
            fail(LLAMA_E_INVALID_ARG, "counters of blob " + std::to_string(b) + " are NULL");
    std::vector<TraceLeaf> leaves(F);
    for (uint32_t f = 0; f < F; f++) {
        leaves[f].counters = uint64_t(uintptr_t(counters[s.blob[f]]));
        leaves[f].base = s.base[f];
        leaves[f].lanes = s.leaf_lanes.empty() ? s.lanes : s.leaf_lanes[f];
        leaves[f].block = s.leaf_block.empty() ? s.block : s.leaf_block[f];
        leaves[f].size = r.leaves[f].size;
    }
    const size_t tbytes = F * sizeof(TraceLeaf), obytes = (F + 1) * sizeof(unsigned long long);
    void* tmp = nullptr;
    check_hip(hipMalloc(&tmp, tbytes + obytes), "hipMalloc(trace)");
    std::vector<unsigned long long> out(F + 1, 0);
    hipError_t e = hipSuccess;
    unsigned long long* dout = (unsigned long long*)((uint8_t*)tmp + tbytes);
    auto step = [&](hipError_t x) {
        if (e == hipSuccess)
            e = x;
    };
    step(hipMemcpyAsync(tmp, leaves.data(), tbytes, hipMemcpyHostToDevice, stream));
    step(hipMemcpyAsync(dout, out.data(), obytes, hipMemcpyHostToDevice, stream));
    if (e == hipSuccess && s.n > 0) {
        const uint32_t grid = uint32_t(std::min<uint64_t>((s.n + 255) / 256, 4096));
        hipLaunchKernelGGL(trace_kernel, dim3(grid), dim3(256), 0, stream, (const TraceLeaf*)tmp, F, s.n, dout);
        step(hipGetLastError());
    }
    for (size_t b = 0; b < s.blob_size.size() && e == hipSuccess; b++) {
        if (!s.blob_size[b])
            continue;
        const uint32_t grid = uint32_t(std::min<uint64_t>((s.blob_size[b] + 255) / 256, 4096));
        hipLaunchKernelGGL(counter_sum_kernel, dim3(grid), dim3(256), 0, stream, (const uint32_t*)counters[b],
                           s.blob_size[b], dout + F);
        step(hipGetLastError());
    }
    step(hipMemcpyAsync(out.data(), dout, obytes, hipMemcpyDeviceToHost, stream));
    step(hipStreamSynchronize(stream));
    (void)hipFree(tmp);
    check_hip(e, "trace");
    uint64_t leaves_total = 0;
    for (uint32_t f = 0; f < F; f++) {
        sums[f] = out[f];
        leaves_total += out[f];
    }
    sums[F] = out[F] - leaves_total; // the bytes no leaf owns
}

void launch_hash(const void* p, uint64_t len, unsigned long long* acc, void* stream)
{
    if (len == 0)
        return;
    const uint64_t granules = (len + 15) / 16;
    const uint32_t grid = uint32_t(std::min<uint64_t>((granules + 255) / 256, 4096));
    hipLaunchKernelGGL(hash_kernel, dim3(grid), dim3(256), 0, (hipStream_t)stream, (const uint8_t*)p, len, acc);
    check_hip(hipGetLastError(), "hash kernel launch");
}

void launch_batch_args(const BatchArgs& args, uint32_t grid, uint32_t threads, uint32_t lds_bytes, bool persistent,
                       void* stream)
{
    set_attributes();
    const bool once = (args.flags & kBatchLoadsOnce) != 0;
    const void* k = persistent ? (once ? (const void*)batch_kernel<true> : (const void*)batch_kernel<false>)
                               : (once ? (const void*)batch_unit_kernel<true> : (const void*)batch_unit_kernel<false>);
    void* kargs[] = {(void*)&args};
    check_hip(hipLaunchKernel(k, dim3(grid), dim3(threads), kargs, lds_bytes, (hipStream_t)stream),
              "hipLaunchKernel(batch)");
    check_hip(hipGetLastError(), "batch kernel launch");
}

namespace {
constexpr int kScratchDevices = 64;
std::mutex g_scratch_mutex;
uint64_t g_scratch_addr[kScratchDevices] = {}; // per device; 0 until resolved
} // namespace

uint64_t scratch_address()
{
    int dev = 0;
    check_hip(hipGetDevice(&dev), "hipGetDevice");
    if (dev < 0 || dev >= kScratchDevices)
        fail(LLAMA_E_UNSUPPORTED, "device " + std::to_string(dev) + " is past the static buffers' device limit");
    std::lock_guard<std::mutex> lock(g_scratch_mutex);
    if (g_scratch_addr[dev] == 0) {
        // with `dev` current: this device's copy of the array
        void* ptr = nullptr;
        check_hip(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)), "hipGetSymbolAddress(scratch)");
        if (!ptr)
            fail(LLAMA_E_HIP, "hipGetSymbolAddress(scratch) returned no address");
        g_scratch_addr[dev] = uint64_t(uintptr_t(ptr));
    }
    return g_scratch_addr[dev];
}

namespace {
// batch_mode_kernel by mode key (kModeAny for long-run items; a tile mode,
// with kModeSplitSrc or kModeSplitDst) and nontemporal loads
template <bool kOnce>
const void* batch_mode_kernel_for(uint32_t key)
{
    switch (key) {
    case kModeAny: return (const void*)batch_mode_kernel<kOnce, kModeAny>;
    case kModeStreamUnits: return (const void*)batch_mode_kernel<kOnce, kModeStreamUnits>;
    case kModeStaged: return (const void*)batch_mode_kernel<kOnce, kModeStaged>;
    case kModeDirectStore: return (const void*)batch_mode_kernel<kOnce, kModeDirectStore>;
    case kModeDirectStore | kModeSplitSrc: return (const void*)batch_mode_kernel<kOnce, kModeDirectStore | kModeSplitSrc>;
    case kModeDirectLoad: return (const void*)batch_mode_kernel<kOnce, kModeDirectLoad>;
    case kModeDirectLoad | kModeSplitDst: return (const void*)batch_mode_kernel<kOnce, kModeDirectLoad | kModeSplitDst>;
    case kModeGatherStore: return (const void*)batch_mode_kernel<kOnce, kModeGatherStore>;
    case kModeGatherOdd: return (const void*)batch_mode_kernel<kOnce, kModeGatherOdd>;
    default: return nullptr;
    }
}
} // namespace

uint32_t batch_mode_key(const BatchItem& it)
{
    if (it.kind != kItemTile)
        return kModeStreamUnits;
    const uint32_t f = it.h.flags;
    if (f & kTileDirectLoad)
        return kModeDirectLoad | ((f & kTileSplitDst) ? kModeSplitDst : 0u);
    if (f & kTileDirectStore)
        return kModeDirectStore | ((f & kTileSplitSrc) ? kModeSplitSrc : 0u);
    if (f & kTileGatherStore)
        return (f & kTileGatherOdd) ? kModeGatherOdd : kModeGatherStore;
    return kModeStaged;
}

void launch_batch_ranges(const BatchArgs& b_args, const std::vector<BatchRange>& ranges, uint32_t threads,
                         void* stream)
{
    set_attributes();
    const bool once = (b_args.flags & kBatchLoadsOnce) != 0;
    for (const BatchRange& r : ranges) {
        const void* k = once ? batch_mode_kernel_for<true>(r.key) : batch_mode_kernel_for<false>(r.key);
        if (!k)
            fail(LLAMA_E_INVALID_ARG, "no batch kernel for tile mode key " + std::to_string(r.key));
        BatchArgs args = b_args;
        uint64_t first = r.first_unit, count = r.units;
        void* kargs[] = {(void*)&args, (void*)&first, (void*)&count};
        const uint32_t grid = uint32_t(std::min<uint64_t>(count, kBatchMaxGrid));
        check_hip(hipLaunchKernel(k, dim3(grid), dim3(threads), kargs, r.lds_bytes, (hipStream_t)stream),
                  "hipLaunchKernel(batch by mode)");
        check_hip(hipGetLastError(), "batch kernel launch");
    }
}

void launch_batch_kernel(const Batch& b, void* stream)
{
    if (b.ranges.empty())
        launch_batch_args(b.args, b.grid, b.threads, b.lds_bytes, b.wg_per_cu != 0, stream);
    else
        launch_batch_ranges(b.args, b.ranges, b.threads, stream);
}

} // namespace llama
