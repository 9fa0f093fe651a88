// Copies whose records sit at different linear indices on the two sides: a
// box of the array dimensions between views of different extents (sec. 3.2
// VirtualView, sec. 3.9 "the size or shape of the view is different"), and
// whole copies between views whose linearizers differ (sec. 3.7 lists
// linearizers among the building blocks of mappings).  The planner here picks
// the tile shape and each side's run order for the box kernel.
#include <algorithm>
#include <cstring>
#include <string>

#include "core.hpp"

namespace llama {

namespace {

uint32_t log2u(uint64_t x)
{
    uint32_t l = 0;
    while ((uint64_t(1) << (l + 1)) <= x)
        l++;
    return l;
}

uint32_t log2_ceil(uint64_t x)
{
    uint32_t l = 0;
    while ((uint64_t(1) << l) < x)
        l++;
    return l;
}

uint32_t round16(uint64_t x)
{
    if (x > (uint64_t(1) << 30))
        fail(LLAMA_E_UNSUPPORTED, "a box tile needs more LDS than a workgroup has");
    return uint32_t((x + 15) & ~uint64_t(15));
}

struct SidePlan {
    uint32_t order;
    bool field_major;
    bool one;
};

SidePlan side_plan(const Side& s)
{
    SidePlan p{};
    p.one = s.kind == LLAMA_ONE;
    p.field_major = !p.one && s.lanes == 0;
    p.order = p.one                        ? uint32_t(kOrderOne)
              : s.lin == LLAMA_COL_MAJOR   ? uint32_t(kOrderCol)
              : s.lin == LLAMA_MORTON      ? uint32_t(kOrderMorton)
                                           : uint32_t(kOrderRow);
    return p;
}

// log2 of the records of a run of `order` for tile extents qlog
uint32_t run_log2(uint32_t order, uint32_t rank, const uint32_t* qlog, uint32_t qsum)
{
    switch (order) {
    case kOrderRow: return qlog[rank - 1];
    case kOrderCol: return qlog[0];
    case kOrderMorton:
    case kOrderOne: return qsum;
    default: return 0; // kOrderPoint
    }
}

// Tile extents (log2 per dimension) for about 2^qsum records: a Morton side
// needs a cube; otherwise each side's fast dimension gets as long runs as the
// box allows.  When the two fast dimensions differ (a transpose), each side
// first gets runs of about 256 bytes per span (a field-major side's spans are
// one leaf's values, a record-major side's whole records; unit_s and unit_d
// are those bytes per record), then the two share the rest.
void tile_shape(uint32_t rank, const uint64_t* box, const SidePlan& s, const SidePlan& d, uint32_t qsum,
                uint32_t unit_s, uint32_t unit_d, uint32_t* qlog)
{
    for (uint32_t k = 0; k < LLAMA_MAX_RANK; k++)
        qlog[k] = 0;
    if (rank == 1) {
        qlog[0] = std::min(qsum, log2_ceil(std::max<uint64_t>(box[0], 1)));
        return;
    }
    if (s.order == kOrderMorton || d.order == kOrderMorton) {
        // a cube of at least 2^qsum records, so that the other side's runs
        // stay long (the LDS budget shrinks it if needed)
        const uint32_t b = std::max<uint32_t>(1, (qsum + rank - 1) / rank);
        for (uint32_t k = 0; k < rank; k++)
            qlog[k] = b;
        return;
    }
    auto cap = [&](uint32_t k) { return log2_ceil(std::max<uint64_t>(box[k], 1)); };
    auto fast = [&](const SidePlan& x) { return x.order == kOrderCol ? 0u : rank - 1; };
    uint32_t left = qsum;
    const bool one_s = s.order == kOrderOne;
    const uint32_t fa = one_s ? fast(d) : fast(s), fb = fast(d);
    if (fa != fb) { // a transpose: both fast dimensions share the tile
        auto want = [&](uint32_t unit) { return log2_ceil((256 + unit - 1) / std::max<uint32_t>(unit, 1)); };
        qlog[fa] = std::min({cap(fa), want(unit_s), left});
        left -= qlog[fa];
        qlog[fb] = std::min({cap(fb), want(unit_d), left});
        left -= qlog[fb];
        while (left > 0 && (qlog[fa] < cap(fa) || qlog[fb] < cap(fb))) {
            // the side whose spans are shorter grows first
            const bool grow_a = qlog[fa] < cap(fa) &&
                                (qlog[fb] >= cap(fb) || (uint64_t(unit_s) << qlog[fa]) <= (uint64_t(unit_d) << qlog[fb]));
            qlog[grow_a ? fa : fb]++;
            left--;
        }
        for (int k = int(rank) - 1; k >= 0; k--) {
            if (uint32_t(k) == fa || uint32_t(k) == fb)
                continue;
            qlog[k] = std::min(cap(uint32_t(k)), left);
            left -= qlog[k];
        }
        return;
    }
    // one fast dimension: fill it, then the next slower ones
    std::vector<uint32_t> dims;
    if (fa == 0) {
        for (uint32_t k = 0; k < rank; k++)
            dims.push_back(k);
    } else {
        for (int k = int(rank) - 1; k >= 0; k--)
            dims.push_back(uint32_t(k));
    }
    for (uint32_t k : dims) {
        qlog[k] = std::min(cap(k), left);
        left -= qlog[k];
    }
}

uint32_t magic_for(uint32_t g)
{
    return uint32_t(((uint64_t(1) << 32) + g - 1) / g);
}

// Fills a BoxSide (everything but the LDS layout).
void fill_side(BoxSide& b, const Side& s, const std::vector<uint64_t>& ptr, const uint64_t* off, const SidePlan& sp,
               const Record& r)
{
    std::memset(&b, 0, sizeof(b));
    for (uint32_t k = 0; k < s.rank; k++) {
        b.offset[k] = off[k];
        b.extent[k] = s.extents[k];
    }
    b.blob = ptr.empty() ? 0 : ptr[0];
    b.npad = s.npad;
    b.lin = s.lin == LLAMA_COL_MAJOR ? kLinCol : s.lin == LLAMA_MORTON ? kLinMorton : kLinRow;
    b.order = sp.order;
    b.morton_bits = s.morton_bits;
    if (sp.one) {
        b.mode = kRecordMajor;
        b.block = r.packed_size;
        b.npad = 1;
    } else if (sp.field_major) {
        b.mode = kFieldMajor;
    } else {
        b.mode = kRecordMajor;
        b.block = s.block;
        b.log2_lanes = log2u(s.lanes);
    }
}

// Builds the box plan for 2^qsum records per tile; false when its LDS does
// not fit `budget`.
bool try_plan(const Request& rq, const uint64_t* so, const uint64_t* dof, const uint64_t* box, bool full,
              bool preserve, uint32_t qsum, uint32_t budget, Plan& p)
{
    const Side &S = rq.src, &D = rq.dst;
    const Record& r = rq.record;
    const uint32_t rank = S.rank;
    SidePlan ss = side_plan(S), ds = side_plan(D);
    BoxArgs& a = p.box;
    std::memset(&a, 0, sizeof(a));
    BoxHeader& h = a.h;
    h.rank = rank;
    uint32_t min_leaf = ~0u;
    for (const Leaf& l : r.leaves)
        min_leaf = std::min(min_leaf, l.size);
    const uint32_t unit_s = ss.field_major ? min_leaf : uint32_t(r.packed_size);
    const uint32_t unit_d = ds.field_major ? min_leaf : uint32_t(r.packed_size);
    tile_shape(rank, box, ss, ds, qsum, unit_s, unit_d, h.qlog);
    h.qlog_sum = 0;
    for (uint32_t k = 0; k < rank; k++)
        h.qlog_sum += h.qlog[k];
    // a Morton side runs its tile as one range of indices when the tile is
    // an aligned cube in its own coordinates; the tile grid is anchored on
    // the destination's cubes (else the source's), and a Morton side whose
    // cubes the anchor misses walks its tile record by record
    const SidePlan* anchor = ds.order == kOrderMorton ? &ds : ss.order == kOrderMorton ? &ss : nullptr;
    const uint64_t* aoff = anchor == &ds ? dof : so;
    for (uint32_t k = 0; k < rank; k++) {
        h.box[k] = box[k];
        const uint64_t q = uint64_t(1) << h.qlog[k];
        h.shift[k] = anchor ? aoff[k] & (q - 1) : 0;
        h.grid[k] = (box[k] + h.shift[k] + q - 1) >> h.qlog[k];
    }
    auto aligned = [&](const uint64_t* off) {
        for (uint32_t k = 0; k < rank; k++)
            if (((off[k] - h.shift[k]) & ((uint64_t(1) << h.qlog[k]) - 1)) != 0)
                return false;
        return true;
    };
    if (ss.order == kOrderMorton && !aligned(so))
        ss.order = kOrderPoint;
    if (ds.order == kOrderMorton && !aligned(dof))
        ds.order = kOrderPoint;
    fill_side(a.src, S, rq.src_ptr, so, ss, r);
    fill_side(a.dst, D, rq.dst_ptr, dof, ds, r);
    a.src.run_log2 = run_log2(ss.order, rank, h.qlog, h.qlog_sum);
    a.dst.run_log2 = run_log2(ds.order, rank, h.qlog, h.qlog_sum);

    // an AoS destination is staged in LDS and stored as exact byte spans,
    // unless its runs are Morton cubes that reach past the box (a box copy
    // must not write the records outside it): then value by value
    const bool aos_dst = !ds.field_major && D.lanes == 1;
    const bool staged = aos_dst && !(ds.order == kOrderMorton && !full);
    h.flags = (full ? kBoxFull : 0u) | (preserve ? kBoxPreserve : 0u) | (staged ? kBoxStaged : 0u);
    if (full && ds.order == kOrderMorton) {
        // units: the destination's aligned cubes in Morton order, holes and
        // lanes past the last index included
        h.flags |= kBoxUnitMorton;
        h.num_units = (D.npad + (uint64_t(1) << h.qlog_sum) - 1) >> h.qlog_sum;
    } else {
        h.num_units = 1;
        for (uint32_t k = 0; k < rank; k++)
            h.num_units *= h.grid[k];
    }
    if (h.num_units >= (uint64_t(1) << 32))
        fail(LLAMA_E_UNSUPPORTED, "a box copy of more than 2^32 tiles");

    // entries: the leaves, then (AoS destinations) the destination's gaps
    const size_t F = r.leaves.size();
    const size_t ne = F + (aos_dst ? D.gaps.size() : 0);
    if (ne > size_t(kBoxMaxEntries))
        fail(LLAMA_E_UNSUPPORTED, "the record has more leaves than the box kernel takes (" +
                                      std::to_string(kBoxMaxEntries) + ")");
    h.num_leaves = uint32_t(F);
    h.num_entries = uint32_t(ne);
    const uint64_t Ws = uint64_t(1) << a.src.run_log2, Wd = uint64_t(1) << a.dst.run_log2;
    const uint64_t Q = uint64_t(1) << h.qlog_sum;
    const uint64_t Rs = Q / Ws, Rd = Q / Wd;
    uint64_t lds = 0; // source runs first
    for (size_t f = 0; f < F; f++) {
        BoxEntry& e = a.e[f];
        const uint32_t sz = r.leaves[f].size;
        e.size = sz;
        e.dst_addr = rq.dst_ptr[D.blob[f]] + D.base[f];
        e.dst_off = uint32_t(D.base[f]);
        if (ss.field_major) {
            // leaf f's runs, one slot of `gran` granules each
            e.src_addr = rq.src_ptr[S.blob[f]] + S.base[f];
            e.src_off = uint32_t(std::min<uint64_t>(lds, ~0u));
            e.gran = round16(Ws * sz + 16) / 16;
            e.magic = magic_for(e.gran);
            lds += Rs * e.gran * 16;
        } else {
            e.src_off = uint32_t(S.base[f]);
        }
    }
    if (aos_dst)
        for (size_t g = 0; g < D.gaps.size(); g++) {
            BoxEntry& e = a.e[F + g];
            e.gap = 1;
            e.dst_off = uint32_t(D.gaps[g].first);
            e.size = uint32_t(D.gaps[g].second);
        }
    if (!ss.field_major) {
        uint64_t blocks;
        if (ss.one)
            blocks = 1;
        else if (S.lanes == 1)
            blocks = Ws;
        else
            blocks = (Ws - 1) / S.lanes + 2;
        a.src.gran = round16(blocks * a.src.block + 16) / 16;
        a.src.magic = magic_for(a.src.gran);
        lds = Rs * a.src.gran * 16;
    }
    a.src.lds_base = 0;
    // destination runs (staged), the record map, the two run tables
    a.dst.lds_base = uint32_t(std::min<uint64_t>(lds, ~0u));
    // an AoS destination of whole 4-byte words of whole 4-byte values, read
    // from 4-byte aligned source positions, gathers its granules word by word
    // (no destination region); kept padding needs the region (loaded first)
    bool gather = staged && !preserve && D.block % 4 == 0 && D.block / 4 <= uint64_t(kBoxMaxWords) &&
                  F < kBoxWordZero;
    if (gather) {
        for (size_t f = 0; f < F && gather; f++) {
            const uint32_t sz = r.leaves[f].size;
            gather = sz % 4 == 0 && D.base[f] % 4 == 0 &&
                     (ss.field_major ? (rq.src_ptr[S.blob[f]] + S.base[f]) % 4 == 0
                                     : S.base[f] % 4 == 0 && a.src.block % 4 == 0 && rq.src_ptr[0] % 4 == 0);
        }
        gather = gather && rq.dst_ptr[0] % 4 == 0;
    }
    if (staged) {
        a.dst.gran = round16(Wd * D.block + 16) / 16;
        a.dst.magic = magic_for(a.dst.gran);
        if (!gather)
            lds += Rd * a.dst.gran * 16;
    }
    if (gather) {
        h.flags |= kBoxGather;
        h.words = uint32_t(D.block / 4);
        h.kmagic = magic_for(uint32_t(D.block));
        for (uint32_t w = 0; w < h.words; w++) {
            uint32_t e = kBoxWordZero;
            for (size_t f = 0; f < F; f++)
                if (D.base[f] <= 4 * w && 4 * w < D.base[f] + r.leaves[f].size)
                    e = uint32_t(f) | (uint32_t(4 * w - D.base[f]) << 8);
            a.words[w] = e;
        }
        h.wtab = uint32_t(std::min<uint64_t>(lds, ~0u));
        lds += ((h.words * 4 + 15) & ~15u) + F * 16;
    }
    h.map = uint32_t(std::min<uint64_t>(lds, ~0u));
    lds += Q * 16;
    a.src.table = uint32_t(std::min<uint64_t>(lds, ~0u));
    lds += Rs * 8;
    a.dst.table = uint32_t(std::min<uint64_t>(lds, ~0u));
    lds += Rd * 8;
    if (lds > budget)
        return false;
    h.lds_bytes = uint32_t(lds);
    p.lds_bytes = h.lds_bytes;
    return true;
}

} // namespace

std::vector<Plan> make_box_plans(const Request& rq, const uint64_t* so, const uint64_t* dof, const uint64_t* box,
                                 bool full, const llama_copy_options* opt)
{
    const Side &S = rq.src, &D = rq.dst;
    const Record& r = rq.record;
    if (opt && (opt->flags & ~kCopyFlags) != 0)
        fail(LLAMA_E_INVALID_ARG, "unknown bits in llama_copy_options.flags");
    const uint32_t want = opt ? opt->path : uint32_t(LLAMA_PATH_AUTO);
    if (want != LLAMA_PATH_AUTO && want != LLAMA_PATH_BOX && want != LLAMA_PATH_NAIVE)
        fail(LLAMA_E_INVALID_ARG, "a copy between different linear indices takes path AUTO, BOX or NAIVE");
    const uint32_t threads = (opt && opt->threads) ? opt->threads : kDefaultThreads;
    if (threads % 64 != 0 || threads == 0 || threads > 1024)
        fail(LLAMA_E_INVALID_ARG, "threads must be a multiple of 64 in 64..1024");
    const uint32_t T = opt ? opt->tile_records : 0;
    if (T && (T < 16 || T > 4096 || (T & (T - 1))))
        fail(LLAMA_E_INVALID_ARG, "tile_records must be a power of two in 16..4096");
    if (opt && opt->wg_per_cu)
        fail(LLAMA_E_INVALID_ARG, "box copies launch one workgroup per tile (wg_per_cu must be 0)");
    const bool preserve = opt && (opt->flags & LLAMA_COPY_PRESERVE_PADDING);
    uint64_t nbox = 1;
    for (uint32_t k = 0; k < S.rank; k++)
        nbox *= box[k];
    std::vector<Plan> plans;
    if (nbox == 0 && (!full || D.npad == 0))
        return plans;

    Plan p;
    p.path = LLAMA_PATH_BOX;
    p.threads = threads;
    p.flags_in = opt ? opt->flags : 0;
    const uint64_t dst_rec = D.lanes == 1 ? D.block : r.packed_size;
    p.read_bytes = nbox * r.packed_size;
    p.write_bytes = full ? [&] {
        uint64_t t = 0;
        for (uint64_t b : D.blob_size)
            t += b;
        return t;
    }() : nbox * dst_rec;
    if (want == LLAMA_PATH_NAIVE) {
        // the element-wise baseline: the same descriptors, one thread per
        // record (of the box, or of the destination's indices)
        if (!try_plan(rq, so, dof, box, full, preserve, 4, ~0u, p))
            fail(LLAMA_E_UNSUPPORTED, "box plan");
        p.box_naive = true;
        p.lds_bytes = 0;
        const uint64_t items = full ? D.npad : nbox;
        p.workgroups = (items + threads - 1) / threads;
        plans.push_back(p);
        return plans;
    }
    // records per tile: about 16 KiB of source values, at least 64
    uint32_t qsum = T ? log2u(T) : std::min<uint32_t>(12, std::max<uint32_t>(6, log2u(24576 / std::max<uint64_t>(r.packed_size, 1))));
    const uint32_t budget = 64 * 1024;
    while (!try_plan(rq, so, dof, box, full, preserve, qsum, budget, p)) {
        if (qsum <= 1)
            fail(LLAMA_E_UNSUPPORTED, "the record does not fit a box tile's LDS");
        qsum--;
    }
    p.workgroups = p.box.h.num_units;
    p.tiles = p.box.h.num_units;
    plans.push_back(p);

    // a full copy into AoSoA walked by rows or columns: the lanes past the
    // last index become zero
    if (full && !preserve && !(p.box.h.flags & kBoxUnitMorton) && D.lanes > 1 && D.npad > D.n) {
        Plan z;
        z.path = LLAMA_PATH_STREAM;
        z.threads = kDefaultThreads;
        uint64_t chunks = 0;
        const uint64_t base = rq.dst_ptr[0] + (D.n / D.lanes) * D.block;
        const uint64_t tail = D.n % D.lanes;
        for (size_t f = 0; f < r.leaves.size(); f++) {
            StreamRun& run = z.stream.r[z.stream.num_runs++];
            run.src = 0;
            run.dst = base + D.base[f] + tail * r.leaves[f].size;
            run.bytes = (D.lanes - tail) * r.leaves[f].size;
            run.first_chunk = chunks;
            chunks += (run.bytes + (uint64_t(1) << kStreamChunkLog2) - 1) >> kStreamChunkLog2;
        }
        z.stream.num_chunks = chunks;
        z.workgroups = chunks;
        z.write_bytes = (D.npad - D.n) * r.packed_size;
        plans.push_back(z);
    }
    return plans;
}

void copy_box(const llama_mapping_desc* src, const llama_blob* src_blobs, const uint64_t* src_offset,
              const llama_mapping_desc* dst, const llama_blob* dst_blobs, const uint64_t* dst_offset,
              const uint64_t* box, const llama_copy_options* options, void* stream)
{
    if (!src || !dst)
        fail(LLAMA_E_INVALID_ARG, "mapping descriptor is NULL");
    if (!src_offset || !dst_offset || !box)
        fail(LLAMA_E_INVALID_ARG, "box offsets or extents are NULL");
    if (src->kind == LLAMA_SPLIT || dst->kind == LLAMA_SPLIT)
        fail(LLAMA_E_UNSUPPORTED, "box copies take plain mappings (no Split)");
    // the same validation as a copy, with the destination's extents on both
    // sides; then the source's own side
    llama_mapping_desc same = *src;
    for (uint32_t k = 0; k < LLAMA_MAX_RANK; k++)
        same.extents[k] = k < dst->rank ? dst->extents[k] : 0;
    if (src->rank != dst->rank)
        fail(LLAMA_E_EXTENT_MISMATCH, "source and destination ranks differ");
    Request rq = make_request(&same, nullptr, dst, nullptr, false);
    rq.src = make_side(src, rq.record);
    check_blobs("source", rq.src, src_blobs, rq.src_ptr);
    check_blobs("destination", rq.dst, dst_blobs, rq.dst_ptr);
    for (size_t a = 0; a < rq.dst_ptr.size(); a++)
        for (size_t b = 0; b < rq.src_ptr.size(); b++) {
            const uint64_t d0 = rq.dst_ptr[a], dn = rq.dst.blob_size[a], s0 = rq.src_ptr[b], sn = rq.src.blob_size[b];
            if (dn > 0 && sn > 0 && d0 < s0 + sn && s0 < d0 + dn)
                fail(LLAMA_E_OVERLAP, "destination blob " + std::to_string(a) + " overlaps source blob " +
                                          std::to_string(b));
        }
    for (size_t a = 0; a < rq.dst_ptr.size(); a++)
        for (size_t b = a + 1; b < rq.dst_ptr.size(); b++) {
            const uint64_t x0 = rq.dst_ptr[a], xn = rq.dst.blob_size[a], y0 = rq.dst_ptr[b], yn = rq.dst.blob_size[b];
            if (xn > 0 && yn > 0 && x0 < y0 + yn && y0 < x0 + xn)
                fail(LLAMA_E_OVERLAP, "destination blobs " + std::to_string(a) + " and " + std::to_string(b) +
                                          " overlap");
        }
    for (uint32_t k = 0; k < src->rank; k++) {
        const bool one = src->kind == LLAMA_ONE;
        if ((!one && (src_offset[k] > src->extents[k] || box[k] > src->extents[k] - src_offset[k])) ||
            dst_offset[k] > dst->extents[k] || box[k] > dst->extents[k] - dst_offset[k])
            fail(LLAMA_E_EXTENT_MISMATCH, "the box does not lie inside both views in dimension " + std::to_string(k));
    }
    const std::vector<Plan> plans = make_box_plans(rq, src_offset, dst_offset, box, false, options);
    for (const Plan& p : plans)
        launch(p, stream);
}

} // namespace llama
