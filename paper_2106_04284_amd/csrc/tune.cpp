// Autotuner: measures candidate kernel parameters of one copy on its own
// blobs, keeps only candidates whose output hashes like the default plan's,
// and caches the fastest per class of copies.
#include <hip/hip_runtime_api.h>

#include <algorithm>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <map>
#include <mutex>
#include <sstream>

#include "core.hpp"

namespace llama {

bool TuneKey::operator<(const TuneKey& o) const
{
    if (leaves != o.leaves)
        return leaves < o.leaves;
    if (src_kind != o.src_kind)
        return src_kind < o.src_kind;
    if (dst_kind != o.dst_kind)
        return dst_kind < o.dst_kind;
    if (src_lanes != o.src_lanes)
        return src_lanes < o.src_lanes;
    if (dst_lanes != o.dst_lanes)
        return dst_lanes < o.dst_lanes;
    return bucket < o.bucket;
}

namespace {

struct TuneValue {
    llama_copy_options opt;
    double gbs;
};

std::mutex g_tune_mutex;
std::map<TuneKey, TuneValue> g_tune;

void check_hip(hipError_t e, const char* what)
{
    if (e != hipSuccess)
        fail(LLAMA_E_HIP, std::string(what) + ": " + hipGetErrorString(e));
}

uint64_t fnv1a(uint64_t h, uint64_t v)
{
    for (int k = 0; k < 8; k++) {
        h ^= (v >> (8 * k)) & 0xff;
        h *= 0x100000001b3ull;
    }
    return h;
}

// per-device scratch word for the output hash
std::mutex g_acc_mutex;
std::map<int, unsigned long long*> g_acc;

unsigned long long* hash_accumulator()
{
    int dev = 0;
    check_hip(hipGetDevice(&dev), "hipGetDevice");
    std::lock_guard<std::mutex> lock(g_acc_mutex);
    auto it = g_acc.find(dev);
    if (it != g_acc.end())
        return it->second;
    void* p = nullptr;
    check_hip(hipMalloc(&p, sizeof(unsigned long long)), "hipMalloc(hash accumulator)");
    g_acc[dev] = (unsigned long long*)p;
    return (unsigned long long*)p;
}

// Fills every destination blob with `fill`, runs plan `p`, and returns the
// hash of the destination blobs (synchronous).
uint64_t run_and_hash(const Request& rq, const Plan& p, hipStream_t stream, int fill)
{
    for (size_t b = 0; b < rq.dst_ptr.size(); b++)
        check_hip(hipMemsetAsync((void*)rq.dst_ptr[b], fill, rq.dst.blob_size[b], stream), "hipMemsetAsync");
    launch(p, stream);
    unsigned long long* acc = hash_accumulator();
    check_hip(hipMemsetAsync(acc, 0, sizeof(*acc), stream), "hipMemsetAsync");
    for (size_t b = 0; b < rq.dst_ptr.size(); b++)
        launch_hash((const void*)rq.dst_ptr[b], rq.dst.blob_size[b], acc, stream);
    unsigned long long h = 0;
    check_hip(hipMemcpyAsync(&h, acc, sizeof(h), hipMemcpyDeviceToHost, stream), "hipMemcpyAsync");
    check_hip(hipStreamSynchronize(stream), "hipStreamSynchronize");
    return h;
}

// Best of `reps` timed launches, in milliseconds.
double time_plan(const Plan& p, hipStream_t stream, int reps)
{
    hipEvent_t e0, e1;
    check_hip(hipEventCreate(&e0), "hipEventCreate");
    check_hip(hipEventCreate(&e1), "hipEventCreate");
    double best = 1e30;
    try {
        launch(p, stream); // warm-up
        for (int r = 0; r < reps; r++) {
            check_hip(hipEventRecord(e0, stream), "hipEventRecord");
            launch(p, stream);
            check_hip(hipEventRecord(e1, stream), "hipEventRecord");
            check_hip(hipEventSynchronize(e1), "hipEventSynchronize");
            float ms = 0;
            check_hip(hipEventElapsedTime(&ms, e0, e1), "hipEventElapsedTime");
            best = std::min(best, double(ms));
        }
    } catch (...) {
        hipEventDestroy(e0);
        hipEventDestroy(e1);
        throw;
    }
    hipEventDestroy(e0);
    hipEventDestroy(e1);
    return best;
}

} // namespace

TuneKey tune_key(const Request& rq)
{
    TuneKey k{};
    uint64_t h = 0xcbf29ce484222325ull;
    for (const Leaf& l : rq.record.leaves)
        h = fnv1a(fnv1a(h, l.size), l.align);
    k.leaves = h;
    k.src_kind = rq.src.kind;
    k.dst_kind = rq.dst.kind;
    k.src_lanes = rq.src.kind == LLAMA_AOSOA ? rq.src.lanes : 0;
    k.dst_lanes = rq.dst.kind == LLAMA_AOSOA ? rq.dst.lanes : 0;
    uint32_t b = 0;
    while (b < 63 && (uint64_t(2) << b) <= rq.src.n)
        b++;
    k.bucket = b;
    return k;
}

// The entry of this class with the nearest size bucket (the exact bucket
// first, then the larger one of two equally near).
bool tune_lookup(const TuneKey& k, llama_copy_options& out)
{
    std::lock_guard<std::mutex> lock(g_tune_mutex);
    auto it = g_tune.find(k);
    if (it != g_tune.end()) {
        out = it->second.opt;
        return true;
    }
    TuneKey lo = k;
    lo.bucket = 0;
    const TuneValue* best = nullptr;
    uint32_t best_dist = ~0u;
    for (auto i = g_tune.lower_bound(lo); i != g_tune.end(); ++i) {
        const TuneKey& c = i->first;
        if (c.leaves != k.leaves || c.src_kind != k.src_kind || c.dst_kind != k.dst_kind ||
            c.src_lanes != k.src_lanes || c.dst_lanes != k.dst_lanes)
            break;
        uint32_t d = c.bucket > k.bucket ? c.bucket - k.bucket : k.bucket - c.bucket;
        if (d < best_dist || (d == best_dist && c.bucket > k.bucket)) {
            best_dist = d;
            best = &i->second;
        }
    }
    if (!best)
        return false;
    out = best->opt;
    return true;
}

// Tries TILE with tile sizes around the default and 64/128/256 threads (and
// STREAM when the pair allows it); every candidate's output must hash like
// the default plan's output before it is timed.
void autotune(const Request& rq, void* stream_ptr, int reps, llama_copy_options& best_opt, double& best_gbs)
{
    hipStream_t stream = (hipStream_t)stream_ptr;
    Plan ref = make_plan(rq, nullptr);
    best_opt = llama_copy_options{0, 0, 0, 0, 0};
    best_gbs = 0;
    if (ref.path == LLAMA_PATH_EMPTY)
        return;
    const double bytes = double(ref.read_bytes + ref.write_bytes);
    const uint64_t want = run_and_hash(rq, ref, stream, 0xA5);
    std::vector<llama_copy_options> cands;
    cands.push_back({LLAMA_PATH_STREAM, 0, 0, 0, 0});
    for (uint32_t T = 16; T <= 4096; T *= 2)
        for (uint32_t th : {64u, 128u, 256u})
            if (T / 4 <= 4 * th && T >= th / 4)
                for (uint32_t flags : {0u, LLAMA_COPY_NO_DIRECT, LLAMA_COPY_NO_GATHER})
                    cands.push_back({LLAMA_PATH_TILE, T, th, 0, flags});
    for (const llama_copy_options& c : cands) {
        Plan p;
        try {
            p = make_plan(rq, &c);
        } catch (const Error&) {
            continue; // candidate does not apply (no long runs, too large for LDS)
        }
        // the staged variant of a plan that uses no direct mode is the same plan
        if ((c.flags & LLAMA_COPY_NO_DIRECT) && p.path == LLAMA_PATH_TILE) {
            llama_copy_options d = c;
            d.flags = 0;
            if (!(make_plan(rq, &d).tile.h.flags & (kTileDirectStore | kTileDirectLoad | kTileGatherStore)))
                continue;
        }
        // likewise without the gather store where the default takes none
        if ((c.flags & LLAMA_COPY_NO_GATHER) && p.path == LLAMA_PATH_TILE) {
            llama_copy_options d = c;
            d.flags = 0;
            if (!(make_plan(rq, &d).tile.h.flags & kTileGatherStore))
                continue;
        }
        if (run_and_hash(rq, p, stream, 0x5A) != want)
            fail(LLAMA_E_HIP, "autotune: a candidate plan wrote different bytes than the default plan");
        const double ms = time_plan(p, stream, reps);
        const double gbs = bytes / (ms * 1e-3) / 1e9;
        if (gbs > best_gbs) {
            best_gbs = gbs;
            best_opt = c;
        }
    }
    std::lock_guard<std::mutex> lock(g_tune_mutex);
    g_tune[tune_key(rq)] = TuneValue{best_opt, best_gbs};
}

void tune_clear()
{
    std::lock_guard<std::mutex> lock(g_tune_mutex);
    g_tune.clear();
}

void tune_save(const char* path)
{
    std::lock_guard<std::mutex> lock(g_tune_mutex);
    std::ofstream f(path);
    if (!f)
        fail(LLAMA_E_INVALID_ARG, std::string("cannot write ") + path);
    f << "# llama_mi355x tuning cache: leaves src_kind src_lanes dst_kind dst_lanes bucket path tile threads "
         "wg_per_cu flags gbs\n";
    for (const auto& kv : g_tune) {
        const TuneKey& k = kv.first;
        const TuneValue& v = kv.second;
        f << std::hex << k.leaves << std::dec << ' ' << k.src_kind << ' ' << k.src_lanes << ' ' << k.dst_kind << ' '
          << k.dst_lanes << ' ' << k.bucket << ' ' << v.opt.path << ' ' << v.opt.tile_records << ' ' << v.opt.threads
          << ' ' << v.opt.wg_per_cu << ' ' << v.opt.flags << ' ' << v.gbs << '\n';
    }
    if (!f)
        fail(LLAMA_E_INVALID_ARG, std::string("cannot write ") + path);
}

uint32_t tune_load(const char* path)
{
    std::ifstream f(path);
    if (!f)
        fail(LLAMA_E_INVALID_ARG, std::string("cannot read ") + path);
    std::map<TuneKey, TuneValue> loaded;
    std::string line;
    while (std::getline(f, line)) {
        if (line.empty() || line[0] == '#')
            continue;
        {
            std::istringstream count(line);
            std::string tok;
            int fields = 0;
            while (count >> tok)
                fields++;
            if (fields != 12)
                fail(LLAMA_E_INVALID_ARG, std::string("tuning cache line needs 12 fields in ") + path + ": " + line);
        }
        std::istringstream in(line);
        TuneKey k{};
        TuneValue v{};
        in >> std::hex >> k.leaves >> std::dec >> k.src_kind >> k.src_lanes >> k.dst_kind >> k.dst_lanes >> k.bucket >>
            v.opt.path >> v.opt.tile_records >> v.opt.threads >> v.opt.wg_per_cu >> v.opt.flags >> v.gbs;
        if (!in)
            fail(LLAMA_E_INVALID_ARG, std::string("malformed tuning cache line in ") + path + ": " + line);
        if (v.opt.path > LLAMA_PATH_NAIVE || (v.opt.flags & ~kTuneFlags) || v.opt.threads % 64 ||
            v.opt.threads > 1024 || v.opt.wg_per_cu > 16 ||
            (v.opt.tile_records && (v.opt.tile_records < 16 || v.opt.tile_records > 4096 ||
                                    (v.opt.tile_records & (v.opt.tile_records - 1)))))
            fail(LLAMA_E_INVALID_ARG, std::string("invalid parameters in tuning cache line: ") + line);
        loaded[k] = v;
    }
    std::lock_guard<std::mutex> lock(g_tune_mutex);
    for (const auto& kv : loaded)
        g_tune[kv.first] = kv.second;
    return uint32_t(loaded.size());
}

uint32_t tune_size()
{
    std::lock_guard<std::mutex> lock(g_tune_mutex);
    return uint32_t(g_tune.size());
}

} // namespace llama
