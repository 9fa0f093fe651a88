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
//  stream_kernel  long contiguous runs (SoA <-> SoA, identical layouts),
//                 16-byte loads and stores, no LDS.
//  naive_kernel   the element-wise baseline: one thread per record, each leaf
//                 located with run-time '/' and '%' and moved at its own width.
#include <hip/hip_runtime.h>

#include "core.hpp"

namespace llama {

namespace {

typedef __attribute__((address_space(3))) void lds_void_t;
#define GLOBAL __attribute__((address_space(1)))

typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
typedef u32x4 u32x4_a4 __attribute__((aligned(4))); // 16 bytes at a 4-byte-aligned address

__device__ __forceinline__ uint32_t wave_id()
{
    return __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
}

__device__ __forceinline__ uint32_t uniform(uint32_t x) { return __builtin_amdgcn_readfirstlane(x); }

// Loads bytes [gstart, gstart + len) into LDS at lds_region + (gstart & 15):
// whole 16-byte granules from gstart rounded down.  A granule that holds a
// byte of the span lies in the same page as that byte, so the rounding never
// reaches an unmapped page; the extra bytes are never used.
__device__ __forceinline__ void load_span(uint64_t gstart, uint32_t len, uint32_t lds_region, uint32_t wave,
                                          uint32_t nwaves, uint32_t lane, uint8_t* lds)
{
    const uint32_t shift = uint32_t(gstart) & 15u;
    const uint64_t g0 = gstart - shift;
    const uint32_t G = (shift + len + 15u) >> 4;
    for (uint32_t c = wave; c * 64u < G; c += nwaves) {
        const uint32_t gi = c * 64u + lane;
        if (gi < G)
            __builtin_amdgcn_global_load_lds((const void*)(g0 + uint64_t(gi) * 16u),
                                             (lds_void_t*)(lds + lds_region + c * 1024u), 16, 0, 0);
    }
}

// Stores LDS bytes lds_region + (gstart & 15) .. into [gstart, gstart + len):
// whole granules with 16-byte stores, the partial first and last granule byte
// by byte so that no byte outside the span is written.
__device__ __forceinline__ void store_span(uint64_t gstart, uint32_t len, uint32_t lds_region, uint32_t tid,
                                           uint32_t nthr, const uint8_t* lds)
{
    const uint32_t shift = uint32_t(gstart) & 15u;
    const uint64_t g0 = gstart - shift;
    const uint32_t end = shift + len;
    const uint32_t G = (end + 15u) >> 4;
    for (uint32_t gi = tid; gi < G; gi += nthr) {
        const uint32_t lo = gi == 0 ? shift : 0u;
        const uint32_t hi = min(16u, end - gi * 16u);
        GLOBAL uint8_t* gp = (GLOBAL uint8_t*)(g0 + uint64_t(gi) * 16u);
        const uint8_t* lp = lds + lds_region + gi * 16u;
        if (lo == 0 && hi == 16) {
            *(GLOBAL u32x4*)gp = *(const u32x4*)lp;
        } else {
            for (uint32_t b = lo; b < hi; b++)
                gp[b] = lp[b];
        }
    }
}

// Position of record r of entry e inside a side's LDS region:
//   p0 + (r >> lg) * K + (r & m) * size
struct Pos {
    uint32_t p0, lg, K, m;
};

__device__ __forceinline__ uint32_t pos_of(const Pos& p, uint32_t r, uint32_t size)
{
    return p.p0 + (r >> p.lg) * p.K + (r & p.m) * size;
}

// Global start of a field-major span of records [i0, ...) of one leaf.
__device__ __forceinline__ uint64_t field_span_start(uint64_t addr, const TileSide& s, uint64_t i0, uint32_t size)
{
    if (s.lanes == 0)
        return addr + i0 * size;
    return addr + (i0 >> s.log2_lanes) * s.block + (i0 & (s.lanes - 1)) * size;
}

template <typename T>
__device__ __forceinline__ void move_values(uint8_t* lds, uint32_t dpos, uint32_t spos, uint32_t size, bool zero)
{
    for (uint32_t k = 0; k < size; k += sizeof(T)) {
        T v;
        if (zero)
            v = T{};
        else
            v = *(const T*)(lds + spos + k);
        *(T*)(lds + dpos + k) = v;
    }
}

__device__ void tile_body(const TileArgs& a, uint64_t t, uint8_t* lds)
{
    const uint32_t tid = threadIdx.x, nthr = blockDim.x;
    const uint32_t lane = tid & 63u, wave = wave_id(), nwaves = nthr >> 6;
    const uint32_t T = 1u << a.log2_tile;
    const uint64_t i0 = t << a.log2_tile;
    const uint32_t nv = i0 < a.n ? uint32_t(min<uint64_t>(T, a.n - i0)) : 0u; // records with values
    const uint32_t nd = uint32_t(min<uint64_t>(T, a.npad - i0));              // records the destination spans

    // ---- 1. source span(s) -> LDS
    if (nv > 0) {
        if (a.src.mode == kRecordMajor) {
            const uint64_t start = a.src.span_base + (i0 >> a.src.log2_lanes) * a.src.block;
            const uint32_t len = uint32_t(((uint64_t(nv) + a.src.lanes - 1) >> a.src.log2_lanes) * a.src.block);
            load_span(start, len, a.src.lds_base, wave, nwaves, lane, lds);
        } else {
            for (uint32_t f = 0; f < a.num_leaves; f++) {
                const TileEntry& e = a.e[f];
                const uint64_t start = field_span_start(e.src_addr, a.src, i0, e.size);
                load_span(start, nv * e.size, a.src.lds_base + uint32_t(e.src_lds16) * 16u, wave, nwaves, lane, lds);
            }
        }
    }
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();

    // ---- 2. move every value from its source position to its destination
    //         position inside LDS; destination padding becomes zero
    const uint64_t src_start = a.src.span_base + (i0 >> a.src.log2_lanes) * a.src.block;
    const uint64_t dst_start = a.dst.span_base + (i0 >> a.dst.log2_lanes) * a.dst.block;
    for (uint32_t k = 0; k < a.num_entries; k++) {
        const TileEntry& e = a.e[k];
        const uint32_t size = e.size;
        const bool gap = e.src_addr == 0;
        Pos sp{0, 31, 0, ~0u}, dp{0, 31, 0, ~0u};
        uint32_t align_bits = size;
        if (!gap) {
            if (a.src.mode == kRecordMajor) {
                sp.p0 = a.src.lds_base + (uint32_t(src_start) & 15u) + uint32_t(e.src_addr - a.src.span_base);
                sp.lg = a.src.log2_lanes;
                sp.K = uint32_t(a.src.block);
                sp.m = uint32_t(a.src.lanes - 1);
                align_bits |= sp.K;
            } else {
                const uint64_t s0 = field_span_start(e.src_addr, a.src, i0, size);
                sp.p0 = a.src.lds_base + uint32_t(e.src_lds16) * 16u + (uint32_t(s0) & 15u);
            }
            align_bits |= sp.p0;
        }
        if (a.dst.mode == kRecordMajor) {
            dp.p0 = a.dst.lds_base + (uint32_t(dst_start) & 15u) + uint32_t(e.dst_addr - a.dst.span_base);
            dp.lg = a.dst.log2_lanes;
            dp.K = uint32_t(a.dst.block);
            dp.m = uint32_t(a.dst.lanes - 1);
            align_bits |= dp.K;
        } else {
            const uint64_t d0 = field_span_start(e.dst_addr, a.dst, i0, size);
            dp.p0 = a.dst.lds_base + uint32_t(e.dst_lds16) * 16u + (uint32_t(d0) & 15u);
        }
        align_bits |= dp.p0;
        const uint32_t w = uniform(min(align_bits & (~align_bits + 1u), 16u));
        for (uint32_t r = tid; r < nd; r += nthr) {
            const bool zero = gap || r >= nv;
            const uint32_t dpos = pos_of(dp, r, size);
            const uint32_t spos = zero ? 0u : pos_of(sp, r, size);
            switch (w) {
            case 16: move_values<u32x4>(lds, dpos, spos, size, zero); break;
            case 8: move_values<uint64_t>(lds, dpos, spos, size, zero); break;
            case 4: move_values<uint32_t>(lds, dpos, spos, size, zero); break;
            case 2: move_values<uint16_t>(lds, dpos, spos, size, zero); break;
            default: move_values<uint8_t>(lds, dpos, spos, size, zero); break;
            }
        }
    }
    __syncthreads();

    // ---- 3. LDS -> destination span(s)
    if (a.dst.mode == kRecordMajor) {
        const uint32_t len = uint32_t(((uint64_t(nd) + a.dst.lanes - 1) >> a.dst.log2_lanes) * a.dst.block);
        store_span(dst_start, len, a.dst.lds_base, tid, nthr, lds);
    } else {
        for (uint32_t f = 0; f < a.num_leaves; f++) {
            const TileEntry& e = a.e[f];
            const uint64_t start = field_span_start(e.dst_addr, a.dst, i0, e.size);
            store_span(start, nd * e.size, a.dst.lds_base + uint32_t(e.dst_lds16) * 16u, tid, nthr, lds);
        }
    }
}

__global__ void __launch_bounds__(1024) tile_kernel(const TileArgs a)
{
    extern __shared__ __attribute__((aligned(16))) uint8_t lds[];
    for (uint64_t t = blockIdx.x; t < a.num_tiles; t += gridDim.x) {
        tile_body(a, t, lds);
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// STREAM
// ---------------------------------------------------------------------------

// Copies [src, src + len) to [dst, dst + len) (src == 0: writes zeros);
// src and dst are congruent modulo 4.
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
            u32x4 v0 = s[g], v1 = s[g + nthr], v2 = s[g + 2u * nthr], v3 = s[g + 3u * nthr];
            d[g] = v0;
            d[g + nthr] = v1;
            d[g + 2u * nthr] = v2;
            d[g + 3u * nthr] = v3;
        }
        for (; g < ng; g += nthr)
            d[g] = s[g];
    } else {
        const GLOBAL u32x4_a4* s = (const GLOBAL u32x4_a4*)(src + head);
        uint64_t g = tid;
        for (; g + 3u * nthr < ng; g += 4u * nthr) {
            const u32x4 v0 = s[g], v1 = s[g + nthr], v2 = s[g + 2u * nthr], v3 = s[g + 3u * nthr];
            d[g] = v0;
            d[g + nthr] = v1;
            d[g + 2u * nthr] = v2;
            d[g + 3u * nthr] = v3;
        }
        for (; g < ng; g += nthr)
            d[g] = s[g];
    }
}

__global__ void __launch_bounds__(1024) stream_kernel(const StreamArgs a)
{
    for (uint64_t c = blockIdx.x; c < a.num_chunks; c += gridDim.x) {
        // run holding chunk c: the last run whose first chunk is <= c
        uint32_t lo = 0, hi = a.num_runs;
        while (hi - lo > 1) {
            const uint32_t mid = (lo + hi) >> 1;
            if (a.r[mid].first_chunk <= c)
                lo = mid;
            else
                hi = mid;
        }
        const StreamRun& run = a.r[lo];
        const uint64_t off = (c - run.first_chunk) << kStreamChunkLog2;
        const uint64_t len = min<uint64_t>(run.bytes - off, uint64_t(1) << kStreamChunkLog2);
        copy_run_chunk(run.dst + off, run.src ? run.src + off : 0, len, threadIdx.x, blockDim.x);
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

void check_hip(hipError_t e, const char* what)
{
    if (e != hipSuccess)
        fail(LLAMA_E_HIP, std::string(what) + ": " + hipGetErrorString(e));
}

bool g_attr_set = false;

void set_attributes()
{
    if (g_attr_set)
        return;
    check_hip(hipFuncSetAttribute((const void*)tile_kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                                  int(kHardLdsBytes)),
              "hipFuncSetAttribute(tile_kernel)");
    g_attr_set = true;
}

constexpr uint64_t kMaxGrid = uint64_t(1) << 24;

} // namespace

void launch(const Plan& p, void* stream_ptr)
{
    hipStream_t stream = (hipStream_t)stream_ptr;
    if (p.path == LLAMA_PATH_EMPTY || p.workgroups == 0)
        return;
    const uint32_t grid = uint32_t(std::min<uint64_t>(p.workgroups, kMaxGrid));
    switch (p.path) {
    case LLAMA_PATH_TILE:
        set_attributes();
        hipLaunchKernelGGL(tile_kernel, dim3(grid), dim3(p.threads), p.tile.lds_bytes, stream, p.tile);
        break;
    case LLAMA_PATH_STREAM:
        hipLaunchKernelGGL(stream_kernel, dim3(grid), dim3(p.threads), 0, stream, p.stream);
        break;
    case LLAMA_PATH_NAIVE:
        hipLaunchKernelGGL(naive_kernel, dim3(grid), dim3(p.threads), 0, stream, p.naive);
        break;
    default:
        fail(LLAMA_E_INVALID_ARG, "unknown path");
    }
    check_hip(hipGetLastError(), "kernel launch");
}

} // namespace llama
