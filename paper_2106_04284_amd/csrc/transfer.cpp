// Copies between address spaces (host <-> device) that change the layout on
// the way, chunk by chunk, with the transfers of one chunk overlapping the
// layout change of another (sec. 3.9: a chunk is shuffled into the other
// mapping in a small intermediate view, then transferred; shuffles and
// transfers overlap).  On this hardware the layout change runs on the GPU,
// where it is far faster than on the host: a host -> device copy transfers a
// chunk in the source layout into a device staging view and changes its
// layout there; a device -> host copy changes the layout into the staging
// view and transfers that.  Either way the link moves every byte once.
#include <hip/hip_runtime_api.h>

#include <algorithm>
#include <cstring>
#include <mutex>
#include <string>

#include "core.hpp"

namespace llama {

namespace {

void check_hip(hipError_t e, const char* what)
{
    if (e != hipSuccess)
        fail(LLAMA_E_HIP, std::string(what) + ": " + hipGetErrorString(e));
}

uint64_t gcd64(uint64_t a, uint64_t b)
{
    while (b) {
        const uint64_t t = a % b;
        a = b;
        b = t;
    }
    return a;
}

// One contiguous byte range of a chunk: `off` bytes into blob `blob` of the
// full view, `stage` bytes into the staging view, `len` bytes long.
struct Span {
    uint32_t blob;
    uint64_t off, stage, len;
};

// The byte ranges of records [i0, i0 + c) of a plain mapping, and where the
// same bytes sit in a staging view of those c records (same kind; a multi-
// blob SoA stages as single-blob SoA).  i0 is a multiple of the lanes.
std::vector<Span> chunk_spans(const Side& s, const Record& r, uint64_t i0, uint64_t c)
{
    std::vector<Span> out;
    if (s.lanes >= 1) { // AoS (L = 1) or AoSoA: whole blocks, tail lanes of the last chunk included
        const uint64_t L = s.lanes;
        const uint64_t b0 = i0 / L, b1 = (i0 + c + L - 1) / L;
        out.push_back({0, b0 * s.block, 0, (b1 - b0) * s.block});
        return out;
    }
    uint64_t stage = 0;
    for (size_t f = 0; f < r.leaves.size(); f++) {
        const uint64_t sz = r.leaves[f].size;
        out.push_back({s.blob[f], s.base[f] + i0 * sz, stage, c * sz});
        stage += c * sz;
    }
    return out;
}

// A view of c records: the staging view (kind of `s`; multi-blob SoA as
// single-blob), or the window of the full device view holding records
// [i0, i0 + c) (SoA as multi-blob with one blob per leaf).
struct View {
    llama_mapping_desc m{};
    std::vector<llama_blob> blobs;
};

View staging_view(const llama_mapping_desc* full, const Side& s, uint64_t c, uint64_t ptr, uint64_t bytes)
{
    View v;
    v.m = *full;
    v.m.rank = 1;
    std::memset(v.m.extents, 0, sizeof(v.m.extents));
    v.m.extents[0] = c;
    v.m.linearizer = LLAMA_ROW_MAJOR;
    if (s.kind == LLAMA_SOA_MULTI)
        v.m.kind = LLAMA_SOA_SINGLE;
    v.blobs.push_back({(void*)uintptr_t(ptr), bytes});
    return v;
}

View window_view(const llama_mapping_desc* full, const Side& s, const Record& r, const std::vector<uint64_t>& ptr,
                 uint64_t i0, uint64_t c)
{
    View v;
    v.m = *full;
    v.m.rank = 1;
    std::memset(v.m.extents, 0, sizeof(v.m.extents));
    v.m.extents[0] = c;
    v.m.linearizer = LLAMA_ROW_MAJOR;
    if (s.lanes >= 1) {
        const uint64_t L = s.lanes;
        v.blobs.push_back({(void*)uintptr_t(ptr[0] + (i0 / L) * s.block), ((c + L - 1) / L) * s.block});
    } else {
        v.m.kind = LLAMA_SOA_MULTI;
        for (size_t f = 0; f < r.leaves.size(); f++)
            v.blobs.push_back({(void*)uintptr_t(ptr[s.blob[f]] + s.base[f] + i0 * r.leaves[f].size),
                               c * r.leaves[f].size});
    }
    return v;
}

// Per-device state: a copy stream, double-buffered staging and its events.
// Transfers on one device take turns (each waits for the previous one's
// staging to be free).
struct Engine {
    int device = -1;
    hipStream_t copy = nullptr;
    void* staging = nullptr;
    uint64_t staging_bytes = 0; // per buffer
    hipEvent_t ready[2] = {}, free_[2] = {};
    hipEvent_t done = nullptr;
    std::mutex lock;
};

std::mutex g_engines_lock;
Engine g_engines[16];

Engine& engine_for_device()
{
    int dev = 0;
    check_hip(hipGetDevice(&dev), "hipGetDevice");
    if (dev < 0 || dev >= 16)
        fail(LLAMA_E_UNSUPPORTED, "transfers run on devices 0..15");
    std::lock_guard<std::mutex> g(g_engines_lock);
    Engine& e = g_engines[dev];
    if (e.device < 0) {
        // default priority (as every stream of the library)
        check_hip(hipStreamCreateWithFlags(&e.copy, hipStreamNonBlocking), "hipStreamCreate(transfer)");
        for (int k = 0; k < 2; k++) {
            check_hip(hipEventCreateWithFlags(&e.ready[k], hipEventDisableTiming), "hipEventCreate");
            check_hip(hipEventCreateWithFlags(&e.free_[k], hipEventDisableTiming), "hipEventCreate");
        }
        check_hip(hipEventCreateWithFlags(&e.done, hipEventDisableTiming), "hipEventCreate");
        e.device = dev;
    }
    return e;
}

void check_host_blobs(const char* which, const Side& s, const llama_blob* blobs, std::vector<uint64_t>& ptrs)
{
    check_blobs(which, s, blobs, ptrs);
}

} // namespace

void copy_transfer(const llama_mapping_desc* src, const llama_blob* src_blobs, uint32_t src_memory,
                   const llama_mapping_desc* dst, const llama_blob* dst_blobs, uint32_t dst_memory,
                   uint64_t chunk_bytes, void* stream_ptr)
{
    hipStream_t stream = (hipStream_t)stream_ptr;
    if (src_memory > LLAMA_MEMORY_HOST || dst_memory > LLAMA_MEMORY_HOST)
        fail(LLAMA_E_INVALID_ARG, "memory must be LLAMA_MEMORY_DEVICE or LLAMA_MEMORY_HOST");
    if (src_memory == dst_memory)
        fail(LLAMA_E_INVALID_ARG, "one view must be in host memory and the other in device memory "
                                  "(device views: llama_copy)");
    Request rq = make_request(src, nullptr, dst, nullptr, false);
    if (src->kind == LLAMA_SPLIT || dst->kind == LLAMA_SPLIT || src->kind == LLAMA_ONE ||
        src->kind == LLAMA_SOA_ALIGNED || dst->kind == LLAMA_SOA_ALIGNED)
        fail(LLAMA_E_UNSUPPORTED, "transfers take plain mappings (no Split, no One source, no aligned SoA)");
    if (needs_box(rq))
        fail(LLAMA_E_UNSUPPORTED, "transfers take views with equal linear indices (the same linearizer)");
    check_host_blobs("source", rq.src, src_blobs, rq.src_ptr);
    check_host_blobs("destination", rq.dst, dst_blobs, rq.dst_ptr);
    const Record& r = rq.record;
    const uint64_t n = rq.src.n;
    if (n == 0)
        return;
    const bool h2d = src_memory == LLAMA_MEMORY_HOST;
    const Side& host = h2d ? rq.src : rq.dst;
    const Side& dev = h2d ? rq.dst : rq.src;
    // chunks of whole blocks on both sides
    const uint64_t Ls = std::max<uint64_t>(rq.src.lanes, 1), Ld = std::max<uint64_t>(rq.dst.lanes, 1);
    const uint64_t unit = Ls / gcd64(Ls, Ld) * Ld;
    const uint64_t per = std::max<uint64_t>(r.packed_size, r.aligned_size);
    uint64_t c = std::max<uint64_t>(chunk_bytes ? chunk_bytes : uint64_t(64) << 20, per) / per;
    c = std::max<uint64_t>(unit, c / unit * unit);
    if (c >= n)
        c = (n + unit - 1) / unit * unit;
    // staging holds one chunk of the host side's layout
    const uint64_t hostL = std::max<uint64_t>(host.lanes, 1);
    const uint64_t sbytes = host.lanes >= 1 ? ((c + hostL - 1) / hostL) * host.block : c * r.packed_size;

    Engine& e = engine_for_device();
    std::lock_guard<std::mutex> g(e.lock);
    // the previous transfer on this device has released the staging
    check_hip(hipEventSynchronize(e.done), "hipEventSynchronize(previous transfer)");
    if (e.staging_bytes < sbytes) {
        if (e.staging)
            check_hip(hipFree(e.staging), "hipFree(staging)");
        e.staging = nullptr;
        e.staging_bytes = 0;
        check_hip(hipMalloc(&e.staging, 2 * sbytes), "hipMalloc(staging)");
        e.staging_bytes = sbytes;
    }
    const uint64_t stage_ptr[2] = {uint64_t(uintptr_t(e.staging)),
                                   uint64_t(uintptr_t(e.staging)) + e.staging_bytes};
    // the copy stream starts after the work already on the caller's stream
    check_hip(hipEventRecord(e.done, stream), "hipEventRecord");
    check_hip(hipStreamWaitEvent(e.copy, e.done, 0), "hipStreamWaitEvent");
    const uint64_t chunks = (n + c - 1) / c;
    for (uint64_t k = 0; k < chunks; k++) {
        const int b = int(k & 1);
        const uint64_t i0 = k * c, cn = std::min(c, n - i0);
        const std::vector<Span> spans = chunk_spans(host, r, i0, cn);
        View stage = staging_view(h2d ? src : dst, host, cn, stage_ptr[b], e.staging_bytes);
        View win = window_view(h2d ? dst : src, dev, r, h2d ? rq.dst_ptr : rq.src_ptr, i0, cn);
        if (h2d) {
            // host -> staging on the copy stream, once the staging is free
            if (k >= 2)
                check_hip(hipStreamWaitEvent(e.copy, e.free_[b], 0), "hipStreamWaitEvent");
            for (const Span& sp : spans)
                check_hip(hipMemcpyAsync((void*)uintptr_t(stage_ptr[b] + sp.stage),
                                         (const void*)uintptr_t(rq.src_ptr[sp.blob] + sp.off), sp.len,
                                         hipMemcpyHostToDevice, e.copy),
                          "hipMemcpyAsync(host to staging)");
            check_hip(hipEventRecord(e.ready[b], e.copy), "hipEventRecord");
            // staging -> destination window, changing the layout
            check_hip(hipStreamWaitEvent(stream, e.ready[b], 0), "hipStreamWaitEvent");
            Request c_rq = make_request(&stage.m, stage.blobs.data(), &win.m, win.blobs.data(), true);
            launch(make_plan(c_rq, nullptr), stream);
            check_hip(hipEventRecord(e.free_[b], stream), "hipEventRecord");
        } else {
            // source window -> staging in the destination's layout
            if (k >= 2)
                check_hip(hipStreamWaitEvent(stream, e.free_[b], 0), "hipStreamWaitEvent");
            Request c_rq = make_request(&win.m, win.blobs.data(), &stage.m, stage.blobs.data(), true);
            launch(make_plan(c_rq, nullptr), stream);
            check_hip(hipEventRecord(e.ready[b], stream), "hipEventRecord");
            // staging -> host on the copy stream
            check_hip(hipStreamWaitEvent(e.copy, e.ready[b], 0), "hipStreamWaitEvent");
            for (const Span& sp : spans)
                check_hip(hipMemcpyAsync((void*)uintptr_t(rq.dst_ptr[sp.blob] + sp.off),
                                         (const void*)uintptr_t(stage_ptr[b] + sp.stage), sp.len,
                                         hipMemcpyDeviceToHost, e.copy),
                          "hipMemcpyAsync(staging to host)");
            check_hip(hipEventRecord(e.free_[b], e.copy), "hipEventRecord");
        }
    }
    // the caller's stream finishes after every transfer
    if (!h2d) {
        check_hip(hipEventRecord(e.done, e.copy), "hipEventRecord");
        check_hip(hipStreamWaitEvent(stream, e.done, 0), "hipStreamWaitEvent");
    }
    check_hip(hipEventRecord(e.done, stream), "hipEventRecord");
}

} // namespace llama
