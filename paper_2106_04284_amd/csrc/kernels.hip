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
template <bool kOnce>
__device__ __forceinline__ u32x4 load_src(const GLOBAL u32x4* p)
{
    if constexpr (kOnce)
        return __builtin_nontemporal_load(p);
    else
        return *p;
}

// The same at a 4-byte-aligned address.
template <bool kOnce>
__device__ __forceinline__ u32x4 load_src_a4(const GLOBAL u32x4_a4* p)
{
    if constexpr (kOnce)
        return __builtin_nontemporal_load(p);
    else
        return *p;
}

// A 16-byte store of destination bytes; kStream marks it nontemporal, for
// destinations far larger than the 256 MB Infinity Cache (tile copies of
// 1.9 GB measured +3-5% with it; copies of a few hundred MB lose up to 9%,
// because plain stores can leave part of the writes in that cache).
template <bool kStream>
__device__ __forceinline__ void store16(GLOBAL u32x4* p, u32x4 v)
{
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
template <bool kOnce>
__device__ __forceinline__ void lds_dma16(uint64_t gaddr, uint32_t lds_addr)
{
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
template <bool kOnce>
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
            lds_dma16<kOnce>(g0 + uint64_t(gi) * 16u, uniform(lds_base + lds_region + c * 1024u));
    }
}

// Stores LDS bytes lds_region + (gstart & 15) .. into [gstart, gstart + len):
// whole granules with 16-byte stores, the partial first and last granule byte
// by byte so that no byte outside the span is written.  Granule gi goes to
// thread (gi + rot) mod nthr, so that short spans spread over the waves.
template <bool kStream>
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
            store16<kStream>((GLOBAL u32x4*)(g0 + uint64_t(gi) * 16u), *(const u32x4*)lp);
        } else {
            GLOBAL uint8_t* gp = (GLOBAL uint8_t*)(g0 + uint64_t(gi) * 16u);
            for (uint32_t b = lo; b < hi; b++)
                gp[b] = lp[b];
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
template <typename T, bool kDstRecordMajor, bool kStream>
__device__ __forceinline__ void direct_store_leaf(const uint8_t* lds, uint32_t sp, const TileSide& s,
                                                  const TileSide& d, uint64_t gdst, uint32_t nv, uint32_t nd,
                                                  uint32_t tid, uint32_t nthr, uint32_t rot, uint32_t ph)
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
            u.t[j] = r >= 0 && uint32_t(r) < nv ? src_value<T>(lds, sp, s, uint32_t(r), sizeof(T)) : T{};
        }
        constexpr uint32_t lg = sizeof(T) == 16 ? 4 : sizeof(T) == 8 ? 3 : sizeof(T) == 4 ? 2 : sizeof(T) == 2 ? 1 : 0;
        const uint64_t a = leaf_granule_addr<kDstRecordMajor>(gbase, d, g, lg);
        if (r0 >= 0 && uint32_t(r0) + per <= nd) {
            store16<kStream>((GLOBAL u32x4*)a, u.v);
        } else {
#pragma unroll
            for (uint32_t j = 0; j < per; j++) {
                const int32_t r = r0 + int32_t(j);
                if (r >= 0 && uint32_t(r) < nd)
                    *(GLOBAL T*)(a + j * sizeof(T)) = u.t[j];
            }
        }
    }
}

// Direct store of a tile: every leaf in turn, at the width of its values.
template <bool kDstRecordMajor, bool kStream, typename Entries>
__device__ __forceinline__ void direct_store_tile(const TileHeader& h, Entries ent, uint64_t t, uint64_t i0,
                                                  uint32_t nv, uint32_t nd, uint32_t tid, uint32_t nthr,
                                                  const uint8_t* lds)
{
    for (uint32_t f = 0; f < h.num_leaves; f++) {
        const auto& e = ent(f);
        const uint64_t gdst = leaf_tile_base<kDstRecordMajor>(e.dst_addr, h.dst, t, i0, e.size);
        const uint32_t rot = (e.move >> 8) & 4095u;
        const uint32_t ph = (e.move >> 20) & 15u;
        const uint32_t sp = e.src_pos;
        switch (e.move & 7u) {
        case 4: direct_store_leaf<u32x4, kDstRecordMajor, kStream>(lds, sp, h.src, h.dst, gdst, nv, nd, tid, nthr, rot, ph); break;
        case 3: direct_store_leaf<uint64_t, kDstRecordMajor, kStream>(lds, sp, h.src, h.dst, gdst, nv, nd, tid, nthr, rot, ph); break;
        case 2: direct_store_leaf<uint32_t, kDstRecordMajor, kStream>(lds, sp, h.src, h.dst, gdst, nv, nd, tid, nthr, rot, ph); break;
        case 1: direct_store_leaf<uint16_t, kDstRecordMajor, kStream>(lds, sp, h.src, h.dst, gdst, nv, nd, tid, nthr, rot, ph); break;
        default: direct_store_leaf<uint8_t, kDstRecordMajor, kStream>(lds, sp, h.src, h.dst, gdst, nv, nd, tid, nthr, rot, ph); break;
        }
    }
}

// Direct load of a tile from a field-major source (leaf sizes 4, 8 or 16
// bytes): every thread loads its slots' granules into registers (all loads in
// flight together), then writes the values to the destination region.
// Records in [nv, nd) (AoSoA lanes past the last record) and gap entries are
// zero-filled.
template <bool kSrcRecordMajor, bool kOnce, typename Entries>
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
            v[j] = load_src<kOnce>((const GLOBAL u32x4*)leaf_granule_addr<kSrcRecordMajor>(
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

// LDS byte of a gather source (a word-table entry of a whole word, or a byte
// entry of a composite word) in destination block blk.
__device__ __forceinline__ uint32_t gather_pos(uint32_t x, uint32_t blk, const TileGather& gg)
{
    return (x & 0x3FFFFu) + (blk >> gg.q) * gg.kq + ((blk & ((1u << gg.q) - 1u)) << ((x >> 18) & 31u));
}

// Gather store of one tile: every thread assembles 16-byte granules of the
// destination span word by word from the source region and stores them;
// padding and records >= nv are zero.
template <bool kStream, bool kOdd>
__device__ __forceinline__ void gather_store_tile(const TileHeader& h, const TileGather& gg, uint64_t t, uint32_t nv,
                                                  uint32_t nd, uint32_t tid, uint32_t nthr, const uint8_t* lds)
{
    const uint32_t* tab = (const uint32_t*)(lds + h.dst.lds_base);
    const uint32_t* btab = tab + gg.words; // the byte sources of composite words
    const uint32_t lgd = gg.lg;            // records per super-block, log2
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
            uint32_t x = 0;
            if ((e >> 31) == 0) {
                if ((blk << lgd) + ((e >> 23) & 127u) < nv) {
                    const uint32_t p = gather_pos(e, blk, gg);
                    if (kOdd && (e & (1u << 30))) { // at p mod 4 = 1..3: the two aligned words that hold it
                        const uint32_t* wp = (const uint32_t*)(lds + (p & ~3u));
                        x = uint32_t(((uint64_t(wp[1]) << 32) | wp[0]) >> ((p & 3u) * 8u));
                    } else {
                        x = *(const uint32_t*)(lds + p);
                    }
                }
            } else if ((e >> 30) == 3u) {
#pragma unroll
                for (uint32_t k = 0; k < 4; k++) {
                    const uint32_t be = btab[4u * (e & 0xFFFFu) + k];
                    if ((be >> 31) == 0 && (blk << lgd) + ((be >> 23) & 127u) < nv)
                        x |= uint32_t(lds[gather_pos(be, blk, gg)]) << (8u * k);
                }
            }
            v[c] = x;
            if (++w == gg.words) {
                w = 0;
                blk++;
            }
        }
        const uint64_t a = gbase + uint64_t(u) * 4u;
        if ((u + 4u) * 4u <= span) {
            store16<kStream>((GLOBAL u32x4*)a, u32x4{v[0], v[1], v[2], v[3]});
        } else if (!kOdd) { // the span's last granule: whole words (blocks of whole words)
#pragma unroll
            for (uint32_t c = 0; c < 4; c++)
                if (u + c < words)
                    *(GLOBAL uint32_t*)(a + 4u * c) = v[c];
        } else { // the span's last granule: whole words, then the bytes of a partial word
#pragma unroll
            for (uint32_t c = 0; c < 4; c++) {
                const uint32_t b = (u + c) * 4u;
                if (b + 4u <= span)
                    *(GLOBAL uint32_t*)(a + 4u * c) = v[c];
                else
                    for (uint32_t k = 0; b + k < span; k++)
                        *(GLOBAL uint8_t*)(a + 4u * c + k) = uint8_t(v[c] >> (8u * k));
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
    kModeGatherOdd = 5 // gather store with kTileGatherOdd
};
// added to a mode: the tile's 16-byte destination stores are nontemporal
constexpr uint32_t kModeStreamStores = 8;
// added to a mode: the tile's source loads are nontemporal
constexpr uint32_t kModeStreamLoads = 16;

template <uint32_t ModeBits, typename Entries>
__device__ __forceinline__ void tile_body(const TileHeader& h, Entries ent, uint64_t t, uint8_t* lds,
                                          const TileGather* gg = nullptr)
{
    constexpr uint32_t Mode = ModeBits & 7u;
    constexpr bool kStream = (ModeBits & kModeStreamStores) != 0;
    constexpr bool kOnce = (ModeBits & kModeStreamLoads) != 0;
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
        if (h.src.mode == kRecordMajor)
            direct_load_tile<true, kOnce>(h, ent, t, i0, nv, nd, lds);
        else
            direct_load_tile<false, kOnce>(h, ent, t, i0, nv, nd, lds);
    } else if (nv > 0) {
        if (h.src.mode == kRecordMajor) {
            const uint32_t len = uint32_t(((uint64_t(nv) + h.src.lanes - 1) >> h.src.log2_lanes) * h.src.block);
            load_span<kOnce>(h.src.span_base + t * h.src.tile_bytes, len, h.src.lds_base, wave, nwaves, 0, lane, lds_base);
        } else {
            for (uint32_t f = 0; f < h.num_leaves; f++) {
                const auto& e = ent(f);
                load_span<kOnce>(field_span_start(e.src_addr, h.src, i0, e.size), nv * e.size, e.src_pos & ~15u, wave,
                          nwaves, (e.move >> 4) & 15u, lane, lds_base);
            }
        }
    }
    if (preserve && !dstore && h.dst.mode == kRecordMajor) {
        const uint32_t len = uint32_t(((uint64_t(nd) + h.dst.lanes - 1) >> h.dst.log2_lanes) * h.dst.block);
        load_span<false>(h.dst.span_base + t * h.dst.tile_bytes, len, h.dst.lds_base, wave, nwaves, 0, lane, lds_base);
    }
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();

    if (dload) {
        // ---- 2''. the destination region is complete: store it
        if (h.dst.mode == kRecordMajor) {
            const uint32_t len = uint32_t(((uint64_t(nd) + h.dst.lanes - 1) >> h.dst.log2_lanes) * h.dst.block);
            store_span<kStream>(h.dst.span_base + t * h.dst.tile_bytes, len, h.dst.lds_base, tid, nthr, 0, lds);
        } else {
            for (uint32_t f = 0; f < h.num_leaves; f++) {
                const auto& e = ent(f);
                store_span<kStream>(field_span_start(e.dst_addr, h.dst, i0, e.size), nd * e.size, e.dst_pos & ~15u, tid,
                           nthr, (e.move >> 8) & 4095u, lds);
            }
        }
        return;
    }

    if (gstore) {
        // ---- 2'''. assemble every destination granule word by word from
        //           the source region and store it; no destination region
        if (Mode == kModeGatherOdd || (Mode == kModeAny && (h.flags & kTileGatherOdd)))
            gather_store_tile<kStream, true>(h, *gg, t, nv, nd, tid, nthr, lds);
        else
            gather_store_tile<kStream, false>(h, *gg, t, nv, nd, tid, nthr, lds);
        return;
    }

    if (dstore) {
        // ---- 2'. gather each destination granule from the source region and
        //          store it; no destination region, no second barrier
        if (h.dst.mode == kRecordMajor)
            direct_store_tile<true, kStream>(h, ent, t, i0, nv, ns, tid, nthr, lds);
        else
            direct_store_tile<false, kStream>(h, ent, t, i0, nv, ns, tid, nthr, lds);
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
        store_span<kStream>(h.dst.span_base + t * h.dst.tile_bytes, len, h.dst.lds_base, tid, nthr, 0, lds);
    } else {
        for (uint32_t f = 0; f < h.num_leaves; f++) {
            const auto& e = ent(f);
            store_span<kStream>(field_span_start(e.dst_addr, h.dst, i0, e.size), ns * e.size, e.dst_pos & ~15u, tid, nthr,
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
    if (Mode == kModeGatherStore || Mode == kModeGatherOdd) // the word table follows the entries
        gather_table(a.h, a.gather, reinterpret_cast<const uint32_t*>(a.e + a.h.num_entries), lds);
    for (; t < nt; t += stride) {
        tile_body<ModeBits>(a.h, ent, t, lds, &a.gather);
        if (t + stride < nt)
            __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// STREAM
// ---------------------------------------------------------------------------

// Copies [src, src + len) to [dst, dst + len) (src == 0: writes zeros);
// src and dst are congruent modulo 4.
template <bool kOnce>
__device__ __forceinline__ void copy_run_chunk(uint64_t dst, uint64_t src, uint64_t len, uint32_t tid, uint32_t nthr)
{
    const uint32_t head = uint32_t(min<uint64_t>(len, (16u - (uint32_t(dst) & 15u)) & 15u));
    const uint64_t body = (len - head) & ~uint64_t(15);
    const uint32_t tail = uint32_t(len - head - body);
    const bool zero = src == 0;
    // head and tail bytes
    if (tid < head)
        ((GLOBAL uint8_t*)dst)[tid] = zero ? 0 : ((const GLOBAL uint8_t*)src)[tid];
    if (tid < tail) {
        const uint64_t o = head + body + tid;
        ((GLOBAL uint8_t*)dst)[o] = zero ? 0 : ((const GLOBAL uint8_t*)src)[o];
    }
    // 16-byte granules: 4 per thread in flight
    GLOBAL u32x4* d = (GLOBAL u32x4*)(dst + head);
    const uint64_t ng = body >> 4;
    if (zero) {
        for (uint64_t g = tid; g < ng; g += nthr)
            d[g] = u32x4{0u, 0u, 0u, 0u};
        return;
    }
    if (((src + head) & 15u) == 0) {
        const GLOBAL u32x4* s = (const GLOBAL u32x4*)(src + head);
        uint64_t g = tid;
        for (; g + 3u * nthr < ng; g += 4u * nthr) {
            u32x4 v0 = load_src<kOnce>(s + g), v1 = load_src<kOnce>(s + g + nthr), v2 = load_src<kOnce>(s + g + 2u * nthr),
                  v3 = load_src<kOnce>(s + g + 3u * nthr);
            d[g] = v0;
            d[g + nthr] = v1;
            d[g + 2u * nthr] = v2;
            d[g + 3u * nthr] = v3;
        }
        for (; g < ng; g += nthr)
            d[g] = load_src<kOnce>(s + g);
    } else {
        const GLOBAL u32x4_a4* s = (const GLOBAL u32x4_a4*)(src + head);
        uint64_t g = tid;
        for (; g + 3u * nthr < ng; g += 4u * nthr) {
            const u32x4 v0 = load_src_a4<kOnce>(s + g), v1 = load_src_a4<kOnce>(s + g + nthr),
                        v2 = load_src_a4<kOnce>(s + g + 2u * nthr), v3 = load_src_a4<kOnce>(s + g + 3u * nthr);
            d[g] = v0;
            d[g + nthr] = v1;
            d[g + 2u * nthr] = v2;
            d[g + 3u * nthr] = v3;
        }
        for (; g < ng; g += nthr)
            d[g] = load_src_a4<kOnce>(s + g);
    }
}

// Work unit c of a run list: the run holding chunk c is the last run whose
// first chunk is <= c.  `run(k)` returns run k.
// Chunks are 2^chunk_log2 bytes.
template <bool kOnce, typename Runs>
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
    copy_run_chunk<kOnce>(r.dst + off, r.src ? r.src + off : 0, len, threadIdx.x, blockDim.x);
}

// kOnce: nontemporal source loads (StreamArgs.flags & kStreamLoadsOnce).
template <bool kOnce>
__global__ void __launch_bounds__(1024) stream_kernel(const StreamArgs a)
{
    auto run = [&](uint32_t k) -> const StreamRun& { return a.r[k]; };
    for (uint64_t c = blockIdx.x; c < a.num_chunks; c += gridDim.x)
        stream_unit<kOnce>(run, a.num_runs, c, kStreamChunkLog2);
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
template <bool kOnce>
__device__ __forceinline__ void batch_unit(const BatchArgs& a, const CONSTANT uint64_t* begin, uint32_t j,
                                           uint64_t g, uint8_t* lds, uint32_t& table_item)
{
    const CONSTANT BatchItem* it = (const CONSTANT BatchItem*)a.items + j;
    const uint64_t u = g - begin[j];
    if (it->kind == kItemTile) {
        const TileHeader h = load_const(&it->h);
        const CONSTANT TileEntry* entries = (const CONSTANT TileEntry*)a.entries + it->first;
        TileGather gg{};
        if (h.flags & kTileGatherStore) {
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
        tile_body<kModeAny | (kOnce ? kModeStreamLoads : 0u)>(
            h, [&](uint32_t k) -> const CONSTANT TileEntry& { return entries[k]; }, u, lds, &gg);
    } else {
        const CONSTANT StreamRun* runs = (const CONSTANT StreamRun*)a.runs + it->first;
        stream_unit<kOnce>([&](uint32_t k) -> const CONSTANT StreamRun& { return runs[k]; }, it->count, u,
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
// NAIVE
// ---------------------------------------------------------------------------

template <typename T>
__device__ __forceinline__ void naive_move(uint64_t d, uint64_t s, uint32_t size, bool zero)
{
    for (uint32_t k = 0; k < size; k += sizeof(T))
        *(GLOBAL T*)(d + k) = zero ? T(0) : *(const GLOBAL T*)(s + k);
}

__global__ void __launch_bounds__(1024) naive_kernel(const NaiveArgs a)
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
            case 8: naive_move<uint64_t>(d, s, e.size, zero); break;
            case 4: naive_move<uint32_t>(d, s, e.size, zero); break;
            case 2: naive_move<uint16_t>(d, s, e.size, zero); break;
            default: naive_move<uint8_t>(d, s, e.size, zero); break;
            }
        }
    }
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

bool g_attr_set = false;

void set_attributes()
{
    if (g_attr_set)
        return;
    for (const void* k : kTileKernels)
        check_hip(hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, int(kHardLdsBytes)),
                  "hipFuncSetAttribute(tile_kernel)");
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

void launch(const Plan& p, void* stream_ptr)
{
    hipStream_t stream = (hipStream_t)stream_ptr;
    if (p.path == LLAMA_PATH_EMPTY || p.workgroups == 0)
        return;
    const uint32_t grid = uint32_t(std::min<uint64_t>(p.workgroups, kMaxGrid));
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
        const void* k = kTileKernels[(mode - 1) + kTileModes * variant];
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
    default:
        fail(LLAMA_E_INVALID_ARG, "unknown path");
    }
    check_hip(hipGetLastError(), "kernel launch");
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

void launch_batch_kernel(const Batch& b, void* stream)
{
    launch_batch_args(b.args, b.grid, b.threads, b.lds_bytes, b.wg_per_cu != 0, stream);
}

} // namespace llama
