// Copies between views whose records differ (sec. 3.9: a field missing on one
// side): each destination leaf takes a chosen source leaf of the same size, or
// keeps its bytes.
#include "core.hpp"

#include <algorithm>

namespace llama {

namespace {

void blob_ptrs(const char* which, const Side& s, const llama_blob* blobs, std::vector<uint64_t>& ptrs)
{
    if (!blobs)
        fail(LLAMA_E_INVALID_ARG, std::string(which) + " blob array is NULL");
    ptrs.resize(s.blob_size.size());
    for (size_t b = 0; b < s.blob_size.size(); b++) {
        if (blobs[b].size < s.blob_size[b])
            fail(LLAMA_E_BLOB_TOO_SMALL, std::string(which) + " blob " + std::to_string(b) + " holds " +
                                             std::to_string(blobs[b].size) + " bytes, the mapping needs " +
                                             std::to_string(s.blob_size[b]));
        if (!blobs[b].ptr && s.blob_size[b] != 0)
            fail(LLAMA_E_INVALID_ARG, std::string(which) + " blob " + std::to_string(b) + " is NULL");
        ptrs[b] = uint64_t(uintptr_t(blobs[b].ptr));
    }
}

bool overlap(uint64_t a, uint64_t an, uint64_t b, uint64_t bn)
{
    return an != 0 && bn != 0 && a < b + bn && b < a + an;
}

} // namespace

std::vector<Plan> leaves_plans(const llama_mapping_desc* src, const llama_blob* src_blobs,
                               const llama_mapping_desc* dst, const llama_blob* dst_blobs, const uint32_t* src_leaf,
                               const llama_copy_options* options, bool need_blobs)
{
    if (!src || !dst)
        fail(LLAMA_E_INVALID_ARG, "mapping descriptor is NULL");
    if (!src_leaf)
        fail(LLAMA_E_INVALID_ARG, "src_leaf is NULL");
    if (src->kind == LLAMA_SPLIT || dst->kind == LLAMA_SPLIT)
        fail(LLAMA_E_UNSUPPORTED, "llama_copy_leaves takes mappings that are not Split");
    if (dst->kind == LLAMA_ONE)
        fail(LLAMA_E_UNSUPPORTED, "a One mapping holds a single record and cannot receive a copy of many");
    const Record rs = flatten(src->record), rd = flatten(dst->record);
    const Side ss = make_side(src, rs), sd = make_side(dst, rd);
    if (src->rank != dst->rank)
        fail(LLAMA_E_EXTENT_MISMATCH, "source and destination ranks differ");
    for (uint32_t d = 0; d < src->rank; d++)
        if (src->extents[d] != dst->extents[d])
            fail(LLAMA_E_EXTENT_MISMATCH, "source and destination extents differ in dimension " + std::to_string(d));
    // the destination leaves that take a value, and their source leaves
    std::vector<uint32_t> to, from;
    for (size_t k = 0; k < rd.leaves.size(); k++) {
        const uint32_t f = src_leaf[k];
        if (f == LLAMA_NO_LEAF)
            continue;
        if (f >= rs.leaves.size())
            fail(LLAMA_E_INVALID_ARG, "src_leaf[" + std::to_string(k) + "] = " + std::to_string(f) +
                                          " is not a source leaf");
        if (rs.leaves[f].size != rd.leaves[k].size)
            fail(LLAMA_E_RECORD_MISMATCH, "destination leaf " + std::to_string(k) + " has " +
                                              std::to_string(rd.leaves[k].size) + " bytes, source leaf " +
                                              std::to_string(f) + " has " + std::to_string(rs.leaves[f].size));
        to.push_back(uint32_t(k));
        from.push_back(f);
    }
    if (to.empty())
        fail(LLAMA_E_INVALID_ARG, "no destination leaf takes a source leaf");

    Request rq;
    rq.record = sub_record(rd, to);
    rq.src = ss;
    rq.src.blob.clear();
    rq.src.base.clear();
    for (uint32_t f : from) {
        rq.src.blob.push_back(ss.blob[f]);
        rq.src.base.push_back(ss.base[f]);
    }
    bool identity = from.size() == rs.leaves.size();
    for (size_t j = 0; identity && j < from.size(); j++)
        identity = from[j] == j;
    rq.src.partial = !identity;
    rq.dst = sd;
    rq.dst.blob.clear();
    rq.dst.base.clear();
    for (uint32_t k : to) {
        rq.dst.blob.push_back(sd.blob[k]);
        rq.dst.base.push_back(sd.base[k]);
    }
    rq.dst.partial = to.size() != rd.leaves.size();
    if (need_blobs) {
        blob_ptrs("source", ss, src_blobs, rq.src_ptr);
        blob_ptrs("destination", sd, dst_blobs, rq.dst_ptr);
    } else {
        // plans only: distinct blobs aligned to 256 bytes, as llama_plan assumes
        for (size_t b = 0; b < ss.blob_size.size(); b++)
            rq.src_ptr.push_back((uint64_t(b) + 1) << 40);
        for (size_t b = 0; b < sd.blob_size.size(); b++)
            rq.dst_ptr.push_back((uint64_t(b) + 1 + 4096) << 40);
    }
    for (size_t a = 0; a < rq.dst_ptr.size(); a++) {
        for (size_t b = 0; b < rq.src_ptr.size(); b++)
            if (overlap(rq.dst_ptr[a], sd.blob_size[a], rq.src_ptr[b], ss.blob_size[b]))
                fail(LLAMA_E_OVERLAP, "destination blob " + std::to_string(a) + " overlaps source blob " +
                                          std::to_string(b));
        for (size_t b = a + 1; b < rq.dst_ptr.size(); b++)
            if (overlap(rq.dst_ptr[a], sd.blob_size[a], rq.dst_ptr[b], sd.blob_size[b]))
                fail(LLAMA_E_OVERLAP, "destination blobs " + std::to_string(a) + " and " + std::to_string(b) +
                                          " overlap");
    }

    if (rq.dst.partial && sd.lanes == 1 && sd.gaps.empty() && sd.npad == sd.n) {
        // records without padding written in part (packed AoS): the bytes of
        // the leaves without a source are gaps whose bytes the tile keeps, by
        // loading each destination region and storing it back whole
        Request kept = rq;
        std::vector<std::pair<uint64_t, uint64_t>> cover;
        for (size_t j = 0; j < to.size(); j++)
            cover.push_back({kept.dst.base[j], rd.leaves[to[j]].size});
        std::sort(cover.begin(), cover.end());
        uint64_t cur = 0;
        for (const auto& c : cover) {
            if (c.first > cur)
                kept.dst.gaps.push_back({cur, c.first - cur});
            cur = std::max(cur, c.first + c.second);
        }
        if (sd.block > cur)
            kept.dst.gaps.push_back({cur, sd.block - cur});
        kept.dst.partial = false;
        llama_copy_options o = options ? *options : llama_copy_options{0, 0, 0, 0, 0};
        o.flags |= LLAMA_COPY_PRESERVE_PADDING;
        Plan t;
        bool planned = false;
        try {
            t = make_plan(kept, &o);
            planned = true;
        } catch (const Error&) {
            // too many gap entries for this build's kernels: go on below
        }
        if (planned)
            return {t};
    }
    if (rq.dst.partial && sd.lanes >= 1) {
        // a record-major destination written in part: only a direct store
        // (granules of its own leaves, no padding gaps) or the element-wise
        // kernel leaves the other leaves' bytes alone
        Plan t;
        bool direct = false;
        try {
            t = make_plan(rq, options);
            direct = t.path == LLAMA_PATH_TILE && (t.tile.h.flags & kTileDirectStore) && rq.dst.gaps.empty();
        } catch (const Error&) {
            // the caller's path or tile size does not fit; go element-wise
        }
        if (direct)
            return {t};
        llama_copy_options o = options ? *options : llama_copy_options{0, 0, 0, 0, 0};
        o.path = LLAMA_PATH_NAIVE;
        o.tile_records = 0;
        return {make_plan(rq, &o)};
    }
    return {make_plan(rq, options)};
}

void copy_leaves(const llama_mapping_desc* src, const llama_blob* src_blobs, const llama_mapping_desc* dst,
                 const llama_blob* dst_blobs, const uint32_t* src_leaf, const llama_copy_options* options,
                 void* stream)
{
    for (const Plan& p : leaves_plans(src, src_blobs, dst, dst_blobs, src_leaf, options, true))
        launch(p, stream);
}

} // namespace llama
