// Host-side core: record flattening, affine mappings, validation, planning.
#include "core.hpp"

#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <iterator>

namespace llama {

void fail(int status, const std::string& message)
{
    throw Error{status, message};
}

namespace {

bool is_pow2(uint64_t x) { return x != 0 && (x & (x - 1)) == 0; }

uint64_t lowbit(uint64_t x) { return x & (~x + 1); }

uint32_t log2_exact(uint64_t x)
{
    uint32_t l = 0;
    while ((uint64_t(1) << l) < x)
        l++;
    return l;
}

uint64_t mul(uint64_t a, uint64_t b, const char* what)
{
    uint64_t r;
    if (__builtin_mul_overflow(a, b, &r))
        fail(LLAMA_E_OVERFLOW, std::string(what) + " overflows 64 bits");
    return r;
}

uint64_t add(uint64_t a, uint64_t b, const char* what)
{
    uint64_t r;
    if (__builtin_add_overflow(a, b, &r))
        fail(LLAMA_E_OVERFLOW, std::string(what) + " overflows 64 bits");
    return r;
}

uint64_t round_up(uint64_t x, uint64_t a) { return add(x, a - 1, "offset") / a * a; }

constexpr size_t kMaxLeaves = 1u << 16;

// Parses the subtree of nodes[idx] and appends its leaves; returns the index
// after the subtree.
uint32_t parse_node(const llama_record_desc* d, uint32_t idx, uint32_t depth, std::vector<Leaf>& out)
{
    if (idx >= d->num_nodes)
        fail(LLAMA_E_INVALID_ARG, "record: a nested record has fewer child nodes than it declares");
    if (depth > 64)
        fail(LLAMA_E_INVALID_ARG, "record: nesting deeper than 64 levels");
    const llama_field& n = d->nodes[idx];
    if (n.count == 0)
        fail(LLAMA_E_INVALID_ARG, "record: node " + std::to_string(idx) + " has count 0");
    size_t first = out.size();
    uint32_t next;
    if (n.size > 0) {
        if (n.children != 0)
            fail(LLAMA_E_INVALID_ARG, "record: leaf node " + std::to_string(idx) + " declares children");
        uint32_t a = n.align ? n.align : uint32_t(std::min<uint64_t>(lowbit(n.size), 16));
        if (!is_pow2(a) || a > 4096)
            fail(LLAMA_E_INVALID_ARG, "record: leaf node " + std::to_string(idx) + " alignment is not a power of two");
        if (n.size > 4096)
            fail(LLAMA_E_INVALID_ARG, "record: leaf node " + std::to_string(idx) + " is larger than 4096 bytes");
        out.push_back(Leaf{n.size, a, 0, 0});
        next = idx + 1;
    } else {
        if (n.children == 0)
            fail(LLAMA_E_INVALID_ARG, "record: node " + std::to_string(idx) + " is neither a leaf nor a record");
        next = idx + 1;
        for (uint32_t c = 0; c < n.children; c++)
            next = parse_node(d, next, depth + 1, out);
    }
    size_t one = out.size() - first;
    if (uint64_t(one) * n.count > kMaxLeaves || out.size() + one * (n.count - 1) > kMaxLeaves)
        fail(LLAMA_E_INVALID_ARG, "record: more than 65536 leaves");
    for (uint32_t c = 1; c < n.count; c++)
        for (size_t k = 0; k < one; k++)
            out.push_back(out[first + k]);
    return next;
}

} // namespace

namespace {

// packed and aligned offsets and the record sizes from the leaf sizes
void lay_out(Record& r)
{
    r.max_align = 1;
    uint64_t packed = 0, aligned = 0;
    for (Leaf& l : r.leaves) {
        l.packed_offset = packed;
        packed = add(packed, l.size, "record size");
        aligned = round_up(aligned, l.align);
        l.aligned_offset = aligned;
        aligned = add(aligned, l.size, "record size");
        r.max_align = std::max(r.max_align, l.align);
    }
    r.packed_size = packed;
    r.aligned_size = round_up(aligned, r.max_align);
}

} // namespace

Record flatten(const llama_record_desc* d)
{
    if (!d)
        fail(LLAMA_E_INVALID_ARG, "record descriptor is NULL");
    if (d->num_nodes == 0 || !d->nodes)
        fail(LLAMA_E_INVALID_ARG, "record has no nodes");
    Record r;
    uint32_t idx = 0;
    while (idx < d->num_nodes)
        idx = parse_node(d, idx, 0, r.leaves);
    lay_out(r);
    if (r.aligned_size > (uint64_t(1) << 32))
        fail(LLAMA_E_INVALID_ARG, "record larger than 4 GiB");
    return r;
}

Record sub_record(const Record& r, const std::vector<uint32_t>& pick)
{
    Record s;
    for (uint32_t f : pick)
        s.leaves.push_back(r.leaves[f]);
    lay_out(s);
    return s;
}

bool same_leaves(const Record& a, const Record& b)
{
    if (a.leaves.size() != b.leaves.size())
        return false;
    for (size_t f = 0; f < a.leaves.size(); f++)
        if (a.leaves[f].size != b.leaves[f].size || a.leaves[f].align != b.leaves[f].align)
            return false;
    return true;
}

namespace {

// One part of a mapping: a plain mapping of the sub-record of `leaves`, whose
// blobs start at blob `first_blob` of the whole mapping.
struct Part {
    std::vector<uint32_t> leaves;
    Record sub;
    Side side;
    uint32_t first_blob = 0;
};

// The parts of a mapping: a Split's (sec. 3.7: the selected leaf range, then
// the other leaves; a part that is a Split again gives its own parts, in
// order), a plain mapping's one.
std::vector<Part> parts_of(const llama_mapping_desc* m, const Record& r, int depth = 0)
{
    const size_t F = r.leaves.size();
    std::vector<Part> parts;
    if (m->kind != LLAMA_SPLIT) {
        Part p;
        for (size_t f = 0; f < F; f++)
            p.leaves.push_back(uint32_t(f));
        p.sub = r;
        p.side = make_side(m, r);
        parts.push_back(std::move(p));
        return parts;
    }
    const llama_split_desc* sd = m->split;
    if (!sd)
        fail(LLAMA_E_INVALID_ARG, "LLAMA_SPLIT mapping without a split descriptor");
    if (depth >= 8)
        fail(LLAMA_E_INVALID_ARG, "split: nested more than 8 levels deep");
    if (sd->leaf_count == 0 || sd->leaf_count >= F || sd->first_leaf > F - sd->leaf_count)
        fail(LLAMA_E_INVALID_ARG, "split: the selected leaves [" + std::to_string(sd->first_leaf) + ", +" +
                                      std::to_string(sd->leaf_count) + ") must be a non-empty proper range of the " +
                                      std::to_string(F) + " leaves");
    uint32_t first_blob = 0;
    for (int k = 0; k < 2; k++) {
        if (sd->kind[k] > LLAMA_SOA_ALIGNED)
            fail(LLAMA_E_INVALID_ARG, "split: part " + std::to_string(k) + " has no valid mapping kind");
        std::vector<uint32_t> leaves;
        for (size_t f = 0; f < F; f++) {
            const bool sel = f >= sd->first_leaf && f < size_t(sd->first_leaf) + sd->leaf_count;
            if (sel == (k == 0))
                leaves.push_back(uint32_t(f));
        }
        const Record sub = sub_record(r, leaves);
        llama_mapping_desc inner = *m;
        inner.kind = sd->kind[k];
        inner.lanes = sd->lanes[k];
        inner.linearizer = 0;
        inner.split = sd->kind[k] == LLAMA_SPLIT ? sd->split[k] : nullptr;
        if (sd->kind[k] == LLAMA_SPLIT) {
            // the inner split's parts, their leaves renumbered in this record
            for (Part& q : parts_of(&inner, sub, depth + 1)) {
                for (uint32_t& f : q.leaves)
                    f = leaves[f];
                q.first_blob += first_blob;
                parts.push_back(std::move(q));
            }
            first_blob = parts.back().first_blob + uint32_t(parts.back().side.blob_size.size());
            continue;
        }
        Part p;
        p.leaves = leaves;
        p.sub = sub;
        p.side = make_side(&inner, p.sub);
        p.first_blob = first_blob;
        first_blob += uint32_t(p.side.blob_size.size());
        parts.push_back(std::move(p));
    }
    return parts;
}

// A Split side: every leaf at its part's place, with its part's L and K; the
// blobs of the selected part, then those of the rest.
Side split_side(const llama_mapping_desc* m, const Record& r)
{
    const std::vector<Part> parts = parts_of(m, r);
    const size_t F = r.leaves.size();
    Side s = parts[0].side;
    s.kind = LLAMA_SPLIT;
    s.lanes = 0;
    s.block = 0;
    s.npad = s.n;
    s.gaps.clear();
    s.blob.assign(F, 0);
    s.base.assign(F, 0);
    s.leaf_lanes.assign(F, 0);
    s.leaf_block.assign(F, 0);
    s.blob_size.clear();
    for (const Part& p : parts) {
        for (size_t k = 0; k < p.leaves.size(); k++) {
            const uint32_t f = p.leaves[k];
            s.blob[f] = p.first_blob + p.side.blob[k];
            s.base[f] = p.side.base[k];
            s.leaf_lanes[f] = p.side.lanes;
            s.leaf_block[f] = p.side.block;
        }
        s.blob_size.insert(s.blob_size.end(), p.side.blob_size.begin(), p.side.blob_size.end());
        for (Side::BlobGap g : p.side.blob_gaps) {
            g.blob += p.first_blob;
            s.blob_gaps.push_back(g);
        }
    }
    return s;
}

} // namespace

Side make_side(const llama_mapping_desc* m, const Record& r)
{
    if (!m)
        fail(LLAMA_E_INVALID_ARG, "mapping descriptor is NULL");
    if (m->kind > LLAMA_SOA_ALIGNED)
        fail(LLAMA_E_INVALID_ARG, "mapping kind " + std::to_string(m->kind) + " is not a llama_mapping_kind");
    if (m->rank < 1 || m->rank > LLAMA_MAX_RANK)
        fail(LLAMA_E_INVALID_ARG, "mapping rank must be 1..8");
    if (m->linearizer > LLAMA_MORTON)
        fail(LLAMA_E_INVALID_ARG, "mapping linearizer " + std::to_string(m->linearizer) + " is not a llama_linearizer");
    if (m->kind == LLAMA_SPLIT) {
        if (m->linearizer != LLAMA_ROW_MAJOR)
            fail(LLAMA_E_UNSUPPORTED, "Split mappings take the row-major linearizer only");
        return split_side(m, r);
    }
    Side s;
    s.kind = m->kind;
    s.rank = m->rank;
    // rank 1 and One: every linearizer is the identity
    s.lin = (m->rank == 1 || m->kind == LLAMA_ONE) ? uint32_t(LLAMA_ROW_MAJOR) : m->linearizer;
    uint64_t n = 1, largest = 0;
    for (uint32_t d = 0; d < m->rank; d++) {
        s.extents[d] = m->extents[d];
        n = mul(n, m->extents[d], "record count");
        largest = std::max(largest, m->extents[d]);
    }
    s.records = n;
    if (s.lin == LLAMA_MORTON) {
        while ((uint64_t(1) << s.morton_bits) < largest)
            s.morton_bits++;
        if (uint64_t(s.morton_bits) * m->rank > 63)
            fail(LLAMA_E_OVERFLOW, "the Morton index of these extents does not fit 63 bits");
        if (n > 0) { // indices up to the last coordinate's
            uint64_t last[LLAMA_MAX_RANK] = {};
            for (uint32_t d = 0; d < m->rank; d++)
                last[d] = m->extents[d] - 1;
            n = linearize(s, last) + 1;
        }
    }
    s.n = n;
    s.npad = n;
    const size_t F = r.leaves.size();
    s.blob.assign(F, 0);
    s.base.assign(F, 0);
    const uint64_t S = r.packed_size, R = r.aligned_size;
    switch (m->kind) {
    case LLAMA_AOS_PACKED:
        s.lanes = 1;
        s.block = S;
        for (size_t f = 0; f < F; f++)
            s.base[f] = r.leaves[f].packed_offset;
        s.blob_size = {mul(n, S, "blob size")};
        break;
    case LLAMA_AOS_ALIGNED: {
        s.lanes = 1;
        s.block = R;
        uint64_t cur = 0;
        for (size_t f = 0; f < F; f++) {
            s.base[f] = r.leaves[f].aligned_offset;
            if (s.base[f] > cur)
                s.gaps.push_back({cur, s.base[f] - cur});
            cur = s.base[f] + r.leaves[f].size;
        }
        if (R > cur)
            s.gaps.push_back({cur, R - cur});
        s.blob_size = {mul(n, R, "blob size")};
        break;
    }
    case LLAMA_SOA_SINGLE:
        s.lanes = 0;
        for (size_t f = 0; f < F; f++)
            s.base[f] = mul(n, r.leaves[f].packed_offset, "SoA sub-array offset");
        s.blob_size = {mul(n, S, "blob size")};
        break;
    case LLAMA_SOA_MULTI:
        s.lanes = 0;
        for (size_t f = 0; f < F; f++) {
            s.blob[f] = uint32_t(f);
            s.blob_size.push_back(mul(n, r.leaves[f].size, "blob size"));
        }
        break;
    case LLAMA_SOA_ALIGNED: {
        // each sub-array at the first multiple of the alignment at or after
        // the end of the one before; the bytes between them are padding
        const uint64_t a = m->lanes ? m->lanes : 256;
        if (!is_pow2(a) || a > (uint64_t(1) << 20))
            fail(LLAMA_E_INVALID_ARG, "aligned SoA: the sub-array alignment must be a power of two up to 2^20, got " +
                                          std::to_string(m->lanes));
        s.lanes = 0;
        uint64_t cur = 0;
        for (size_t f = 0; f < F; f++) {
            if (f > 0) {
                const uint64_t start = round_up(cur, a);
                if (start > cur)
                    s.blob_gaps.push_back({0, cur, start - cur});
                cur = start;
            }
            s.base[f] = cur;
            cur = add(cur, mul(n, r.leaves[f].size, "SoA sub-array size"), "blob size");
        }
        s.blob_size = {cur};
        break;
    }
    case LLAMA_ONE:
        // blocked with L = 1 and K = 0: every record at the one packed record
        s.lanes = 1;
        s.block = 0;
        for (size_t f = 0; f < F; f++)
            s.base[f] = r.leaves[f].packed_offset;
        s.blob_size = {S};
        break;
    case LLAMA_AOSOA: {
        if (!is_pow2(m->lanes))
            fail(LLAMA_E_INVALID_ARG, "AoSoA lanes must be a power of two, got " + std::to_string(m->lanes));
        uint64_t L = m->lanes;
        s.lanes = L;
        s.block = mul(L, S, "AoSoA block size");
        for (size_t f = 0; f < F; f++)
            s.base[f] = mul(L, r.leaves[f].packed_offset, "AoSoA chunk offset");
        uint64_t blocks = n / L + (n % L != 0);
        s.npad = mul(blocks, L, "AoSoA record count");
        s.blob_size = {mul(blocks, s.block, "blob size")};
        break;
    }
    }
    return s;
}

uint64_t linearize(const Side& s, const uint64_t* c)
{
    uint64_t i = 0;
    if (s.lin == LLAMA_MORTON) {
        for (uint32_t j = 0; j < s.morton_bits; j++)
            for (uint32_t d = 0; d < s.rank; d++)
                i |= ((c[d] >> j) & 1u) << (j * s.rank + (s.rank - 1 - d));
    } else if (s.lin == LLAMA_COL_MAJOR) {
        for (int d = int(s.rank) - 1; d >= 0; d--)
            i = i * s.extents[d] + c[d];
    } else {
        for (uint32_t d = 0; d < s.rank; d++)
            i = i * s.extents[d] + c[d];
    }
    return i;
}

bool needs_box(const Request& rq)
{
    return rq.src.lin != rq.dst.lin || rq.src.n != rq.src.records || rq.dst.n != rq.dst.records;
}

void check_blobs(const char* which, const Side& s, const llama_blob* blobs, std::vector<uint64_t>& ptrs)
{
    if (!blobs)
        fail(LLAMA_E_INVALID_ARG, std::string(which) + " blob array is NULL");
    ptrs.resize(s.blob_size.size());
    for (size_t b = 0; b < s.blob_size.size(); b++) {
        if (blobs[b].size < s.blob_size[b])
            fail(LLAMA_E_BLOB_TOO_SMALL, std::string(which) + " blob " + std::to_string(b) + " holds " +
                                             std::to_string(blobs[b].size) + " bytes, the mapping needs " +
                                             std::to_string(s.blob_size[b]));
        if (s.blob_size[b] > 0 && !blobs[b].ptr)
            fail(LLAMA_E_INVALID_ARG, std::string(which) + " blob " + std::to_string(b) + " is NULL");
        uint64_t p = uint64_t(uintptr_t(blobs[b].ptr));
        add(p, s.blob_size[b], "blob end address");
        ptrs[b] = p;
    }
}

namespace {

bool overlaps(uint64_t a, uint64_t an, uint64_t b, uint64_t bn)
{
    return an > 0 && bn > 0 && a < b + bn && b < a + an;
}

} // namespace

Request make_request(const llama_mapping_desc* src, const llama_blob* src_blobs, const llama_mapping_desc* dst,
                     const llama_blob* dst_blobs, bool need_blobs, bool allow_split)
{
    if (!src || !dst)
        fail(LLAMA_E_INVALID_ARG, "mapping descriptor is NULL");
    Request rq;
    rq.record = flatten(src->record);
    if (dst->record != src->record) {
        Record other = flatten(dst->record);
        if (!same_leaves(rq.record, other))
            fail(LLAMA_E_RECORD_MISMATCH, "source and destination records flatten to different leaves");
    }
    rq.src = make_side(src, rq.record);
    rq.dst = make_side(dst, rq.record);
    if (!allow_split && (src->kind == LLAMA_SPLIT || dst->kind == LLAMA_SPLIT))
        fail(LLAMA_E_UNSUPPORTED, "Split mappings are copied by llama_copy, llama_copy_ex and llama_copy_naive only");
    if (dst->kind == LLAMA_ONE)
        fail(LLAMA_E_UNSUPPORTED, "a One mapping holds a single record and cannot receive a copy of many");
    if (src->rank != dst->rank)
        fail(LLAMA_E_EXTENT_MISMATCH, "source and destination ranks differ");
    for (uint32_t d = 0; d < src->rank; d++)
        if (src->extents[d] != dst->extents[d])
            fail(LLAMA_E_EXTENT_MISMATCH, "source and destination extents differ in dimension " + std::to_string(d));
    if (need_blobs) {
        check_blobs("source", rq.src, src_blobs, rq.src_ptr);
        check_blobs("destination", rq.dst, dst_blobs, rq.dst_ptr);
        for (size_t a = 0; a < rq.dst_ptr.size(); a++) {
            for (size_t b = 0; b < rq.src_ptr.size(); b++)
                if (overlaps(rq.dst_ptr[a], rq.dst.blob_size[a], rq.src_ptr[b], rq.src.blob_size[b]))
                    fail(LLAMA_E_OVERLAP, "destination blob " + std::to_string(a) + " overlaps source blob " +
                                              std::to_string(b));
            for (size_t b = a + 1; b < rq.dst_ptr.size(); b++)
                if (overlaps(rq.dst_ptr[a], rq.dst.blob_size[a], rq.dst_ptr[b], rq.dst.blob_size[b]))
                    fail(LLAMA_E_OVERLAP, "destination blobs " + std::to_string(a) + " and " + std::to_string(b) +
                                              " overlap");
        }
    } else {
        // a plan without blobs assumes distinct, 256-byte aligned blobs (1 TiB
        // apart), so that runs of different blobs never look contiguous
        for (size_t b = 0; b < rq.src.blob_size.size(); b++)
            rq.src_ptr.push_back((uint64_t(b) + 1) << 40);
        for (size_t b = 0; b < rq.dst.blob_size.size(); b++)
            rq.dst_ptr.push_back((uint64_t(b) + 1 + 4096) << 40);
    }
    return rq;
}

namespace {

// lanes as far as the copy can tell: a side whose single block holds every
// record behaves as unblocked
uint64_t effective_lanes(const Side& s)
{
    return (s.lanes == 0 || s.lanes >= s.n) ? 0 : s.lanes;
}

// the side of part `p` that holds only leaves `pick` (a subset of p.leaves,
// both in leaf order)
Side restrict_side(const Part& p, const std::vector<uint32_t>& pick)
{
    Side s = p.side;
    s.blob.clear();
    s.base.clear();
    size_t k = 0;
    for (uint32_t f : pick) {
        while (p.leaves[k] != f)
            k++;
        s.blob.push_back(p.side.blob[k]);
        s.base.push_back(p.side.base[k]);
    }
    s.partial = pick.size() != p.leaves.size();
    return s;
}

using PartLeaves = std::vector<std::pair<const Part*, std::vector<uint32_t>>>;

// One copy into destination part P from all the source parts that feed it
// (`from`, each with the leaves it gives).  When every source part is
// field-major (SoA), the source is one plain field-major side over their
// blobs, planned like any copy.  When the record-major source parts share
// one lane count L, the source is a side of virtual blocks of L records,
// each assembled from the parts' chunks (a whole part block, or L values of
// an SoA leaf), which only the tile kernel reads (kTileVirtualSrc); chunks
// must be whole 16-byte granules at 16-byte aligned addresses.  Returns false
// (and the part copies run one source part at a time) when neither applies
// or no plan fits `opt`.
bool gathered_copy(const PartLeaves& from, const Part& P, const Request& whole, const llama_copy_options* opt,
                   SubCopy& out)
{
    // the leaves the parts give P: all of P's, or (a field-major part that
    // another copy also feeds) some
    std::vector<uint32_t> given;
    for (const auto& fq : from)
        given.insert(given.end(), fq.second.begin(), fq.second.end());
    std::sort(given.begin(), given.end());
    Request rq;
    rq.record = sub_record(whole.record, given);
    rq.dst = restrict_side(P, given);
    if (rq.dst.partial && effective_lanes(P.side) != 0)
        return false;
    rq.dst_ptr.assign(whole.dst_ptr.begin() + P.first_blob,
                      whole.dst_ptr.begin() + P.first_blob + P.side.blob_size.size());
    uint64_t L = 0;
    for (const auto& fq : from) {
        if (fq.first->side.kind == LLAMA_ONE)
            return false; // a broadcast part: element-wise only
        const uint64_t l = effective_lanes(fq.first->side);
        if (l != 0 && L != 0 && l != L)
            return false;
        if (l != 0)
            L = l;
    }
    const size_t F = given.size();
    std::vector<uint32_t> blob_of(whole.record.leaves.size(), 0);
    std::vector<uint64_t> base_of(whole.record.leaves.size(), 0);
    Side s = from[0].first->side;
    s.partial = false;
    s.gaps.clear();
    s.blob_gaps.clear();
    s.leaf_lanes.clear();
    s.leaf_block.clear();
    s.blob_size.clear();
    if (L == 0) {
        // every part field-major: their leaf spans as one SoA side
        s.kind = LLAMA_SOA_MULTI;
        s.lanes = 0;
        s.block = 0;
        s.npad = s.n;
        for (const auto& fq : from) {
            const Part& Q = *fq.first;
            for (uint32_t f : fq.second) {
                const size_t k = size_t(std::find(Q.leaves.begin(), Q.leaves.end(), f) - Q.leaves.begin());
                blob_of[f] = uint32_t(rq.src_ptr.size());
                base_of[f] = Q.side.base[k];
                rq.src_ptr.push_back(whole.src_ptr[Q.first_blob + Q.side.blob[k]]);
                s.blob_size.push_back(Q.side.blob_size[Q.side.blob[k]]);
            }
        }
    } else {
        uint64_t off = 0;
        for (const auto& fq : from) {
            const Part& Q = *fq.first;
            if (effective_lanes(Q.side) != 0) {
                // a record-major part: its whole block (one blob)
                const uint64_t addr = whole.src_ptr[Q.first_blob];
                if (Q.side.block % 16 != 0 || addr % 16 != 0 || Q.side.block > UINT32_MAX)
                    return false;
                rq.chunks.push_back(SrcChunk{addr, Q.side.block, uint32_t(off), uint32_t(Q.side.block), 0});
                s.blob_size.push_back(Q.side.blob_size[0]);
                for (uint32_t f : fq.second) {
                    const size_t k = size_t(std::find(Q.leaves.begin(), Q.leaves.end(), f) - Q.leaves.begin());
                    base_of[f] = off + Q.side.base[k];
                }
                off += Q.side.block;
            } else {
                // a field-major part: L values of each leaf
                for (uint32_t f : fq.second) {
                    const size_t k = size_t(std::find(Q.leaves.begin(), Q.leaves.end(), f) - Q.leaves.begin());
                    const uint32_t size = whole.record.leaves[f].size;
                    const uint64_t addr = whole.src_ptr[Q.first_blob + Q.side.blob[k]] + Q.side.base[k];
                    const uint64_t bytes = L * size;
                    if (bytes % 16 != 0 || addr % 16 != 0 || bytes > UINT32_MAX)
                        return false;
                    rq.chunks.push_back(SrcChunk{addr, bytes, uint32_t(off), uint32_t(bytes), size});
                    s.blob_size.push_back(Q.side.n * size);
                    base_of[f] = off;
                    off += bytes;
                }
            }
            if (off > UINT32_MAX || rq.chunks.size() > size_t(kTileMaxChunks))
                return false;
        }
        s.kind = LLAMA_AOSOA;
        s.lanes = L;
        s.block = off;
        s.npad = (s.n + L - 1) / L * L;
        rq.src_ptr.assign(1, 0);
    }
    s.blob.assign(F, 0);
    s.base.assign(F, 0);
    for (size_t j = 0; j < F; j++) {
        s.blob[j] = blob_of[given[j]];
        s.base[j] = base_of[given[j]];
    }
    rq.src = s;
    try {
        if (!rq.chunks.empty() && opt && opt->path != LLAMA_PATH_AUTO && opt->path != LLAMA_PATH_TILE)
            return false;
        out.plan = std::make_shared<Plan>(make_plan(rq, opt));
    } catch (const Error&) {
        return false;
    }
    out.rq = std::move(rq);
    out.gathered = true;
    out.naive = false;
    return true;
}

// One copy from source part Q into several destination parts (`to`: each
// with the leaves Q gives it; a record-major part takes all its leaves from
// Q, a field-major part may take only some).  When every such part is
// field-major, the destination is one plain field-major side over their
// blobs, planned like any copy.  When the record-major ones share one lane
// count L, the destination is scattered: each leaf's runs of L values go to
// its own part (a direct-store tile, kTileVirtualDst), which needs runs of at
// least 128 bytes (whole 16-byte granules) at 16-byte aligned addresses and
// no padding gaps.  Returns false (and the part copies run one destination
// part at a time) when neither applies or no plan fits `opt`.
bool scattered_copy(const Part& Q, const PartLeaves& to, const Request& whole, const llama_copy_options* opt,
                    SubCopy& out)
{
    uint64_t L = 0;
    std::vector<uint32_t> leaves;
    for (const auto& pl : to) {
        const Part* P = pl.first;
        const uint64_t l = effective_lanes(P->side);
        // a part taken as field-major must have no tail lanes to fill (an
        // AoSoA part whose one block outlasts the records has them)
        if (P->side.kind == LLAMA_ONE || !P->side.gaps.empty() || !P->side.blob_gaps.empty() ||
            (l != 0 && L != 0 && l != L) || (l == 0 && P->side.npad != P->side.n))
            return false;
        if (l != 0)
            L = l;
        leaves.insert(leaves.end(), pl.second.begin(), pl.second.end());
    }
    std::sort(leaves.begin(), leaves.end());
    Request rq;
    rq.record = sub_record(whole.record, leaves);
    rq.src = restrict_side(Q, leaves);
    rq.src_ptr.assign(whole.src_ptr.begin() + Q.first_blob, whole.src_ptr.begin() + Q.first_blob + Q.side.blob_size.size());
    Side d = to[0].first->side;
    d.partial = false;
    d.gaps.clear();
    d.blob_gaps.clear();
    d.leaf_lanes.clear();
    d.leaf_block.clear();
    d.blob_size.clear();
    d.blob.assign(leaves.size(), 0);
    d.base.assign(leaves.size(), 0);
    if (L != 0) {
        rq.dst_stride.assign(leaves.size(), 0);
        rq.dst_values_only.assign(leaves.size(), 0);
    }
    uint64_t run_bytes = 0;
    for (const auto& pl : to) {
        const Part* P = pl.first;
        const uint32_t first = uint32_t(rq.dst_ptr.size());
        for (size_t b = 0; b < P->side.blob_size.size(); b++) {
            rq.dst_ptr.push_back(whole.dst_ptr[P->first_blob + b]);
            d.blob_size.push_back(P->side.blob_size[b]);
        }
        const bool field = effective_lanes(P->side) == 0;
        for (uint32_t f : pl.second) {
            const size_t k = size_t(std::find(P->leaves.begin(), P->leaves.end(), f) - P->leaves.begin());
            const size_t j = size_t(std::lower_bound(leaves.begin(), leaves.end(), f) - leaves.begin());
            d.blob[j] = first + P->side.blob[k];
            d.base[j] = P->side.base[k];
            if (L == 0)
                continue;
            const uint32_t size = whole.record.leaves[f].size;
            const uint64_t stride = field ? L * size : P->side.block;
            if ((L * size) % 16 != 0 || L * size < 128 || stride % 16 != 0 || stride > UINT32_MAX ||
                (rq.dst_ptr[d.blob[j]] + d.base[j]) % 16 != 0)
                return false;
            rq.dst_stride[j] = uint32_t(stride);
            rq.dst_values_only[j] = field ? 1 : 0;
            run_bytes += L * size;
        }
    }
    if (L == 0) {
        // every part field-major: their leaf spans as one SoA side
        d.kind = LLAMA_SOA_MULTI;
        d.lanes = 0;
        d.block = 0;
        d.npad = d.n;
    } else {
        d.kind = LLAMA_AOSOA;
        d.lanes = L;
        d.block = (run_bytes + 15) / 16 * 16; // the bytes of L records, as a staged region would hold them
        d.npad = (d.n + L - 1) / L * L;
        if (opt && opt->path != LLAMA_PATH_AUTO && opt->path != LLAMA_PATH_TILE)
            return false;
    }
    rq.dst = d;
    try {
        out.plan = std::make_shared<Plan>(make_plan(rq, opt));
    } catch (const Error&) {
        return false;
    }
    out.rq = std::move(rq);
    out.gathered = true;
    out.naive = false;
    return true;
}

} // namespace

std::vector<SubCopy> split_copies(const llama_mapping_desc* src, const llama_mapping_desc* dst, const Request& whole,
                                  bool gather, const llama_copy_options* options)
{
    const std::vector<Part> sp = parts_of(src, whole.record);
    const std::vector<Part> dp = parts_of(dst, whole.record);
    std::vector<SubCopy> out;
    // per destination part, the source parts that share leaves with it, with
    // those leaves
    std::vector<PartLeaves> feeds(dp.size());
    for (size_t p = 0; p < dp.size(); p++) {
        const Part& P = dp[p];
        if (P.side.kind == LLAMA_ONE)
            fail(LLAMA_E_UNSUPPORTED, "a One part holds a single record and cannot receive a copy of many");
        for (const Part& Q : sp) {
            std::vector<uint32_t> both;
            std::set_intersection(P.leaves.begin(), P.leaves.end(), Q.leaves.begin(), Q.leaves.end(),
                                  std::back_inserter(both));
            if (!both.empty())
                feeds[p].emplace_back(&Q, std::move(both));
        }
    }
    // a source part that feeds several destination parts: one copy into all
    // the record-major ones it alone feeds and the field-major ones it feeds
    // (it then reads its blobs once); those feeds are done
    if (gather) {
        for (const Part& Q : sp) {
            PartLeaves to;
            std::vector<size_t> idx;
            for (size_t p = 0; p < dp.size(); p++)
                for (const auto& fq : feeds[p])
                    if (fq.first == &Q && (feeds[p].size() == 1 || effective_lanes(dp[p].side) == 0)) {
                        to.emplace_back(&dp[p], fq.second);
                        idx.push_back(p);
                    }
            SubCopy g;
            if (to.size() > 1 && scattered_copy(Q, to, whole, options, g)) {
                out.push_back(std::move(g));
                for (size_t p : idx)
                    feeds[p].erase(std::find_if(feeds[p].begin(), feeds[p].end(),
                                                [&](const auto& fq) { return fq.first == &Q; }));
            }
        }
    }
    for (size_t p = 0; p < dp.size(); p++) {
        if (feeds[p].empty())
            continue;
        const Part& P = dp[p];
        PartLeaves from = feeds[p];
        if (gather && from.size() > 1) {
            SubCopy g;
            if (gathered_copy(from, P, whole, options, g)) {
                out.push_back(std::move(g));
                continue;
            }
        }
        // An AoS part fed by several source parts: the copy with the most
        // bytes goes first and writes whole records, taking every byte its
        // leaves do not cover as padding (zero, or kept); the others then
        // write only their own leaves over it.
        const bool whole_first = from.size() > 1 && P.side.lanes == 1 &&
                                 P.leaves.size() + P.side.gaps.size() + 1 <= size_t(kTileMaxEntries);
        if (whole_first) {
            auto bytes = [&](const std::vector<uint32_t>& g) {
                uint64_t b = 0;
                for (uint32_t f : g)
                    b += whole.record.leaves[f].size;
                return b;
            };
            std::stable_sort(from.begin(), from.end(),
                             [&](const auto& x, const auto& y) { return bytes(x.second) > bytes(y.second); });
        }
        bool padding_written = false;
        for (const auto& fq : from) {
            const Part& Q = *fq.first;
            const std::vector<uint32_t>& both = fq.second;
            SubCopy c;
            c.rq.record = sub_record(whole.record, both);
            c.rq.src = restrict_side(Q, both);
            c.rq.dst = restrict_side(P, both);
            if (padding_written) {
                // the alignment gaps of this destination part are written once
                c.rq.dst.gaps.clear();
                c.rq.dst.blob_gaps.clear();
            } else if (whole_first) {
                // every byte of the record outside these leaves becomes a gap
                std::vector<std::pair<uint64_t, uint64_t>> cover;
                for (size_t k = 0; k < both.size(); k++)
                    cover.push_back({c.rq.dst.base[k], whole.record.leaves[both[k]].size});
                std::sort(cover.begin(), cover.end());
                c.rq.dst.gaps.clear();
                uint64_t cur = 0;
                for (const auto& cv : cover) {
                    if (cv.first > cur)
                        c.rq.dst.gaps.push_back({cur, cv.first - cur});
                    cur = std::max(cur, cv.first + cv.second);
                }
                if (P.side.block > cur)
                    c.rq.dst.gaps.push_back({cur, P.side.block - cur});
                c.rq.dst.partial = false;
            }
            const bool wrote_whole = whole_first && !padding_written;
            padding_written = true;
            c.naive = c.rq.dst.partial && P.side.lanes >= 1 && !wrote_whole;
            c.rq.src_ptr.assign(whole.src_ptr.begin() + Q.first_blob,
                                whole.src_ptr.begin() + Q.first_blob + Q.side.blob_size.size());
            c.rq.dst_ptr.assign(whole.dst_ptr.begin() + P.first_blob,
                                whole.dst_ptr.begin() + P.first_blob + P.side.blob_size.size());
            out.push_back(std::move(c));
        }
    }
    return out;
}

// ---------------------------------------------------------------------------
// Planning
// ---------------------------------------------------------------------------

namespace {

bool same_placement(const Side& a, const Side& b)
{
    if (a.partial || b.partial)
        return false;
    if (effective_lanes(a) != effective_lanes(b) || a.blob_size != b.blob_size || a.blob != b.blob ||
        a.base != b.base || a.npad != b.npad || a.gaps != b.gaps || a.blob_gaps != b.blob_gaps)
        return false;
    return effective_lanes(a) == 0 || a.block == b.block;
}

struct RunList {
    std::vector<StreamRun> runs;
    void add(uint64_t src, uint64_t dst, uint64_t bytes)
    {
        if (bytes == 0)
            return;
        if (!runs.empty()) {
            StreamRun& l = runs.back();
            bool both_zero = (l.src == 0 && src == 0);
            bool both_data = (l.src != 0 && src != 0 && l.src + l.bytes == src);
            if ((both_zero || both_data) && l.dst + l.bytes == dst) {
                l.bytes += bytes;
                return;
            }
        }
        runs.push_back(StreamRun{src, dst, bytes, 0});
    }
};

// Contiguous-chunk analysis (the run-time analysis of sec. 3.9, done on the
// affine form): returns false when the copy does not reduce to a few long
// runs.
// Contiguous runs of a pair; zero runs (src 0) fill AoSoA tail lanes unless
// `preserve` keeps the destination's padding.
bool stream_runs(const Request& rq, RunList& out, bool preserve)
{
    const Side &s = rq.src, &d = rq.dst;
    const Record& r = rq.record;
    const size_t F = r.leaves.size();
    if (!d.gaps.empty())
        return false;
    if (same_placement(s, d) && d.blob_gaps.empty()) {
        // identical layouts: whole blobs, except the lanes past the last
        // record of an AoSoA block, which become zero runs
        uint64_t L = d.lanes;
        if (d.npad == d.n) {
            for (size_t b = 0; b < d.blob_size.size(); b++)
                out.add(rq.src_ptr[b], rq.dst_ptr[b], d.blob_size[b]);
            return true;
        }
        uint64_t full = d.n / L;
        uint64_t tail = d.n % L;
        out.add(rq.src_ptr[0], rq.dst_ptr[0], full * d.block);
        for (size_t f = 0; f < F; f++) {
            uint64_t off = full * d.block + d.base[f];
            out.add(rq.src_ptr[0] + off, rq.dst_ptr[0] + off, tail * r.leaves[f].size);
            if (!preserve)
                out.add(0, rq.dst_ptr[0] + off + tail * r.leaves[f].size, (L - tail) * r.leaves[f].size);
        }
        return true;
    }
    if (effective_lanes(s) != 0 || effective_lanes(d) != 0)
        return false;
    // every leaf is one contiguous array on both sides
    for (size_t f = 0; f < F; f++) {
        uint64_t sz = r.leaves[f].size;
        uint64_t sa = rq.src_ptr[s.blob[f]] + s.base[f];
        uint64_t da = rq.dst_ptr[d.blob[f]] + d.base[f];
        out.add(sa, da, s.n * sz);
        if (!preserve)
            out.add(0, da + d.n * sz, (d.npad - d.n) * sz);
    }
    // the padding between aligned SoA sub-arrays
    if (!preserve)
        for (const Side::BlobGap& g : d.blob_gaps)
            out.add(0, rq.dst_ptr[g.blob] + g.offset, g.length);
    return true;
}

// LLAMA_COPY_PRESERVE_PADDING, where the destination has padding to keep
bool preserve_padding(const Request& rq, const Plan& p)
{
    return (p.flags_in & kPlanPreserve) && rq.dst.has_padding();
}

uint64_t total_bytes(const std::vector<uint64_t>& v)
{
    uint64_t t = 0;
    for (uint64_t x : v)
        t += x;
    return t;
}

bool fill_stream(const Request& rq, Plan& p)
{
    RunList rl;
    if (!stream_runs(rq, rl, preserve_padding(rq, p)))
        return false;
    if (rl.runs.size() > size_t(kStreamMaxRuns))
        return false;
    uint64_t chunks = 0;
    for (StreamRun& run : rl.runs) {
        if (run.src != 0 && ((run.src ^ run.dst) & 3) != 0)
            return false; // source and destination not congruent modulo 4
        run.first_chunk = chunks;
        chunks += (run.bytes + (uint64_t(1) << kStreamChunkLog2) - 1) >> kStreamChunkLog2;
    }
    p.path = LLAMA_PATH_STREAM;
    std::memset(&p.stream, 0, sizeof(p.stream));
    p.stream.num_runs = uint32_t(rl.runs.size());
    p.stream.flags = total_bytes(rq.src.blob_size) >= kStreamLoadBytes ? kStreamLoadsOnce : 0u;
    p.stream.num_chunks = chunks;
    for (size_t k = 0; k < rl.runs.size(); k++)
        p.stream.r[k] = rl.runs[k];
    p.workgroups = chunks;
    return true;
}

uint32_t tile_side(const Side& s, const Record& r, uint32_t T, TileSide& out, std::vector<uint32_t>& leaf_lds)
{
    const size_t F = r.leaves.size();
    leaf_lds.assign(F, 0);
    out.lanes = s.lanes;
    out.block = s.block;
    out.log2_lanes = s.lanes ? log2_exact(s.lanes) : 0;
    if (s.lanes >= 1 && s.lanes <= T) {
        out.mode = kRecordMajor;
        out.tile_bytes = (uint64_t(T) >> out.log2_lanes) * s.block;
        out.pos_lg = out.log2_lanes;
        out.pos_k = uint32_t(std::min<uint64_t>(s.block, UINT32_MAX));
        out.pos_m = uint32_t(s.lanes - 1);
        return uint32_t(std::min<uint64_t>((out.tile_bytes + 15 + 15) / 16 * 16, uint64_t(1) << 31));
    }
    out.mode = kFieldMajor;
    out.tile_bytes = 0;
    out.pos_lg = 31;
    out.pos_k = 0;
    out.pos_m = ~0u;
    uint64_t total = 0;
    for (size_t f = 0; f < F; f++) {
        leaf_lds[f] = uint32_t(std::min<uint64_t>(total, uint64_t(1) << 31));
        total += (uint64_t(T) * r.leaves[f].size + 15 + 15) / 16 * 16;
    }
    return uint32_t(std::min<uint64_t>(total, uint64_t(1) << 31));
}

uint32_t log2_move(uint64_t bits)
{
    uint64_t w = std::min<uint64_t>(lowbit(bits | 16), 16);
    return log2_exact(w);
}

bool fill_tile(const Request& rq, uint32_t T, uint32_t lds_limit, Plan& p)
{
    const Record& r = rq.record;
    const size_t F = r.leaves.size();
    const size_t C = rq.chunks.size(); // a source gathered from several parts
    if (F + rq.dst.gaps.size() + C > size_t(kTileMaxEntries))
        return false;
    if (C && (rq.src.lanes > T || rq.src.block % 16 != 0))
        return false;
    TileArgs& ta = p.tile;
    std::memset(&ta, 0, sizeof(ta));
    TileHeader& a = ta.h;
    std::vector<uint32_t> src_lds, dst_lds;
    uint32_t sb = tile_side(rq.src, r, T, a.src, src_lds);
    uint32_t db = tile_side(rq.dst, r, T, a.dst, dst_lds);
    uint64_t total = uint64_t(sb) + db;
    if (total > lds_limit || total > kHardLdsBytes)
        return false;
    a.src.lds_base = 0;
    a.src.lds_bytes = sb;
    a.dst.lds_base = sb;
    a.dst.lds_bytes = db;
    a.src.span_base = rq.src_ptr[0];
    a.dst.span_base = rq.dst_ptr[0];
    a.n = rq.src.n;
    a.npad = rq.dst.npad;
    a.log2_tile = log2_exact(T);
    a.num_tiles = (a.npad + T - 1) / T;
    a.num_leaves = uint32_t(F);
    a.lds_bytes = uint32_t(total);
    // T >= 16 makes every tile stride a multiple of 16, so a span's offset
    // modulo 16 is that of its first tile
    const uint64_t src_rm_bits = a.src.mode == kRecordMajor ? rq.src.block : 0;
    const uint64_t dst_rm_bits = a.dst.mode == kRecordMajor ? rq.dst.block : 0;
    for (size_t f = 0; f < F; f++) {
        TileEntry& e = ta.e[f];
        e.src_addr = rq.src_ptr[rq.src.blob[f]] + rq.src.base[f];
        e.dst_addr = rq.dst_ptr[rq.dst.blob[f]] + rq.dst.base[f];
        e.size = r.leaves[f].size;
        e.src_pos = a.src.mode == kRecordMajor
                        ? a.src.lds_base + uint32_t(rq.src_ptr[0] & 15) + uint32_t(rq.src.base[f])
                        : a.src.lds_base + src_lds[f] + uint32_t(e.src_addr & 15);
        e.dst_pos = a.dst.mode == kRecordMajor
                        ? a.dst.lds_base + uint32_t(rq.dst_ptr[0] & 15) + uint32_t(rq.dst.base[f])
                        : a.dst.lds_base + dst_lds[f] + uint32_t(e.dst_addr & 15);
        e.move = log2_move(uint64_t(e.src_pos) | e.dst_pos | e.size | src_rm_bits | dst_rm_bits);
        const uint32_t rd = log2_move(uint64_t(e.src_pos) | e.size | src_rm_bits);
        const uint32_t wr = log2_move(uint64_t(e.dst_pos) | e.size | dst_rm_bits);
        if ((e.size == 2 || e.size == 4 || e.size == 8) && (e.move & 7u) < 2 && !(p.flags_in & kPlanNoSplit))
            e.move |= kMoveSplit | (rd << 20) | (wr << 24);
    }
    size_t k = F;
    for (const auto& g : rq.dst.gaps) { // only record-major (aligned AoS) destinations have gaps
        TileEntry& e = ta.e[k++];
        e.src_addr = 0;
        e.dst_addr = rq.dst_ptr[0] + g.first;
        e.size = uint32_t(g.second);
        e.src_pos = 0;
        e.dst_pos = a.dst.lds_base + uint32_t(rq.dst_ptr[0] & 15) + uint32_t(g.first);
        e.move = log2_move(uint64_t(e.dst_pos) | e.size | dst_rm_bits) | (1u << 31);
    }
    a.num_entries = uint32_t(k);
    if (C) {
        // the chunks of a virtual source block follow the entries and gaps
        const uint64_t gpb = rq.src.block / 16;
        if ((uint64_t(T) / rq.src.lanes) * gpb * gpb >= (uint64_t(1) << 32))
            return false; // mulhi division exact only below this
        for (size_t c = 0; c < C; c++) {
            const SrcChunk& ch = rq.chunks[c];
            TileEntry& e = ta.e[k + c];
            e.src_addr = ch.addr;
            e.dst_addr = ch.block_stride;
            e.src_pos = ch.offset;
            e.dst_pos = 0;
            e.size = ch.bytes;
            e.move = ch.per_record;
        }
        a.slots = uint32_t(C);
        a.flags |= kTileVirtualSrc;
        a.src.pad = uint32_t(((uint64_t(1) << 32) + gpb - 1) / gpb);
    }
    // Lane runs: on a field-major side every leaf's values of a tile are one
    // span; on an AoSoA side whose blocks are multiples of 16 bytes they are
    // runs of L values, and when L * size is a multiple of 16 no 16-byte
    // granule of a leaf crosses a run.  Either way a granule holds 16 / size
    // consecutive records of one leaf.  Runs shorter than a 128-byte cache
    // line are left to the staged path: scattered 32-byte runs (AoSoA8 of
    // 4-byte leaves) measured 22% slower directly than staged.
    auto granule_runs = [](const TileSide& side, uint32_t sz) {
        return side.mode == kFieldMajor || (side.lanes >= 1 && side.block % 16 == 0 && side.lanes * sz >= 128 &&
                                            (side.lanes * sz) % 16 == 0);
    };
    // direct store: destination leaf values in 16-byte granules of one leaf,
    // with leaf sizes 1..16 (powers of two) read at their own width; an AoSoA
    // destination's lane runs start 16-byte aligned, a field-major leaf span
    // may start at any multiple of its size (its phase in the granule grid:
    // the partial first and last granules are written value by value)
    // A source value aligned below its size (a packed record of odd size) is
    // read from the aligned words that hold it (kTileSplitSrc), for leaves of
    // 2, 4 and 8 bytes, unless LLAMA_COPY_NO_SPLIT; a scattered destination
    // keeps aligned reads.
    const bool split_ok = !(p.flags_in & kPlanNoSplit) && rq.dst_stride.empty();
    bool direct = rq.dst.gaps.empty() && !(p.flags_in & kPlanNoDirect);
    bool split_src = false;
    for (size_t f = 0; f < F && direct; f++) {
        const TileEntry& e = ta.e[f];
        const uint32_t sz = e.size;
        const uint64_t src_bits = uint64_t(e.src_pos) | sz | src_rm_bits;
        const bool aligned = lowbit(src_bits | 16) >= sz;
        direct = sz <= 16 && (sz & (sz - 1)) == 0 && granule_runs(a.dst, sz) &&
                 (a.dst.mode == kFieldMajor ? e.dst_addr % sz == 0 : (e.dst_addr & 15) == 0) &&
                 (aligned || (split_ok && sz >= 2 && sz <= 8));
        split_src = split_src || !aligned;
    }
    if (!rq.dst_stride.empty() && (!direct || a.dst.mode != kRecordMajor))
        return false; // a scattered destination is stored by the direct-store tile only
    if (direct) {
        a.flags |= kTileDirectStore;
        a.dst.lds_bytes = 0;
        a.lds_bytes = sb;
        if (split_src)
            a.flags |= kTileSplitSrc;
        for (size_t f = 0; f < F; f++) { // the width is the leaf size; the phase replaces the split bits
            TileEntry& e = ta.e[f];
            const uint32_t phase = a.dst.mode == kFieldMajor ? uint32_t((e.dst_addr & 15) / e.size) : 0u;
            // the source alignment (kTileSplitSrc)
            const uint32_t rd = log2_move(uint64_t(e.src_pos) | e.size | src_rm_bits);
            e.move = (e.move & ~(7u | kMoveSplit | (0xFFu << 20))) | log2_exact(e.size) | (phase << 20) |
                     (split_src ? std::min<uint32_t>(rd, 7u) << 24 : 0u);
            if (!rq.dst_stride.empty()) {
                // the leaf's runs in its own part
                e.dst_pos = rq.dst_stride[f];
                if (rq.dst_values_only[f])
                    e.move |= kMoveValuesOnly;
            }
        }
        if (!rq.dst_stride.empty())
            a.flags |= kTileVirtualDst;
    }
    const bool preserve = preserve_padding(rq, p);
    // gather store: a record-major destination, every tile span 16-byte
    // aligned, planned over a super-block of gb = 1, 2 or 4 destination
    // blocks: the fewest whose bytes, and the source bytes that its records
    // advance by, are whole 4-byte words (4 records of a 49-byte packed
    // record); a source with more lanes per block than the super-block has
    // records needs leaf sizes that are powers of two (its lane runs then
    // advance by shifts)
    const uint64_t Ld = rq.dst.lanes;
    auto src_advance = [&](uint64_t recs) -> uint64_t { // source bytes per super-block, 0: by shifts
        if (a.src.mode == kFieldMajor || rq.src.lanes > recs)
            return 0;
        return (recs >> a.src.log2_lanes) * rq.src.block;
    };
    uint64_t gb = 1;
    while (gb < 4 && ((gb * rq.dst.block) % 4 != 0 || src_advance(gb * Ld) % 4 != 0))
        gb *= 2;
    const uint64_t recs = gb * Ld; // records per super-block
    const uint64_t gwords = gb * rq.dst.block / 4;
    const bool more_lanes = src_advance(recs) == 0;
    bool gather = !direct && !preserve && !(p.flags_in & kPlanNoDirect) && a.dst.mode == kRecordMajor &&
                  recs <= kGatherMaxLanes && recs <= T && (gb * rq.dst.block) % 4 == 0 && gwords >= 2 &&
                  gwords <= kGatherMaxWords && rq.dst_ptr[0] % 16 == 0 && a.dst.tile_bytes % 16 == 0 &&
                  (a.dst.tile_bytes / 4) * gwords < (uint64_t(1) << 32);
    for (size_t f = 0; f < F && gather; f++)
        gather = !more_lanes || is_pow2(r.leaves[f].size);
    if (gather) {
        TileGather g{};
        g.words = uint32_t(gwords);
        g.magic = uint32_t(((uint64_t(1) << 32) + gwords - 1) / gwords);
        g.lg = log2_exact(recs);
        if (!more_lanes) { // super-block b starts recs / L_s source blocks further
            g.q = 0;
            g.kq = uint32_t(src_advance(recs));
        } else if (a.src.mode == kFieldMajor) { // super-block b starts b * recs values further in each leaf span
            g.q = 31;
            g.kq = 0;
        } else {
            g.q = a.src.log2_lanes - g.lg;
            g.kq = uint32_t(rq.src.block);
        }
        // the source of every byte of destination super-block 0 (LDS byte
        // for super-block 0, log2 of the bytes of recs values, record; bit
        // 31: padding), from which each word's pieces follow
        std::vector<uint32_t> src_of(gwords * 4, 1u << 31);
        for (size_t f = 0; f < F; f++) {
            const TileEntry& e = ta.e[f];
            const uint32_t run = log2_exact(recs * e.size);
            for (uint32_t jj = 0; jj < recs; jj++)
                for (uint32_t k = 0; k < e.size; k++) {
                    const uint32_t p0 = e.src_pos + (jj >> a.src.pos_lg) * a.src.pos_k + (jj & a.src.pos_m) * e.size + k;
                    const uint64_t b = (jj / Ld) * rq.dst.block + rq.dst.base[f] + (jj % Ld) * e.size + k;
                    src_of[b] = p0 | (run << 18) | (jj << 23);
                }
        }
        // Every destination word becomes pieces: the bytes that read as one
        // 4-byte window of the source region in every super-block (consecutive
        // source bytes of one run shift, or of any leaf when q = 0, where
        // every byte of super-block b lies kq * b past its place in
        // super-block 0).  A piece is one entry: p0, the source byte that the
        // word's byte 0 lines up with, its run and the word bytes it gives.
        // A word of one piece (or none: padding) is its own table entry; a
        // word of two pieces points to a pair of entries; a word of three or
        // four to the sources of its 4 bytes, placed after the word entries.
        std::vector<uint32_t> table(gwords), quads, pairs;
        bool pieces_ok = true;
        for (uint64_t w = 0; w < gwords && pieces_ok; w++) {
            const uint32_t* x = &src_of[4 * w];
            uint32_t piece[4], n = 0;
            for (uint32_t k = 0; k < 4; k++) {
                if (x[k] >> 31) // padding: no piece, the byte stays zero
                    continue;
                const uint32_t pos = x[k] & 0x3FFFFu, run = g.q == 0 ? 0u : (x[k] >> 18) & 31u;
                if (pos < k || pos - k >= (1u << 18)) {
                    pieces_ok = false; // the window would start before the region
                    break;
                }
                const uint32_t key = (pos - k) | (run << 18);
                uint32_t j = 0;
                while (j < n && (piece[j] & 0x7FFFFFu) != key)
                    j++;
                if (j == n)
                    piece[n++] = key;
                piece[j] |= 1u << (23 + k);
            }
            if (!pieces_ok)
                break;
            if (n <= 1) {
                table[w] = n ? piece[0] : 0u;
            } else if (n == 2) {
                table[w] = (1u << 30) | uint32_t(pairs.size());
                pairs.insert(pairs.end(), piece, piece + 2);
            } else { // byte by byte: the source byte of each (bit 31: a zero byte)
                table[w] = (2u << 30) | uint32_t(quads.size());
                for (uint32_t k = 0; k < 4; k++)
                    quads.push_back((x[k] >> 31) ? 1u << 31
                                                 : (x[k] & 0x3FFFFu) | ((g.q == 0 ? 0u : (x[k] >> 18) & 31u) << 18));
            }
        }
        // groups of four at a 16-byte boundary, then the pairs; a group's
        // entry holds its index in the table
        const uint32_t quads_at = uint32_t((gwords + 3) & ~uint64_t(3));
        const uint32_t pairs_at = quads_at + uint32_t(quads.size());
        for (uint64_t w = 0; w < gwords; w++)
            if ((table[w] >> 30) == 1u)
                table[w] += pairs_at;
            else if ((table[w] >> 30) == 2u)
                table[w] += quads_at;
        table.resize(quads_at, 0u);
        table.insert(table.end(), quads.begin(), quads.end());
        table.insert(table.end(), pairs.begin(), pairs.end());
        g.table = uint32_t(table.size());
        // a word of two pieces costs about two reads of one, of four about
        // four; the gather store takes the tile while the table fits the
        // argument block and LDS and its words average at most
        // kGatherMaxReadsPct / 100 reads
        const uint64_t cost = gwords + pairs.size() / 2 + 3 * (quads.size() / 4);
        const uint64_t base = (uint64_t(sb) + 15) & ~uint64_t(15); // the table, 16-byte aligned
        const uint64_t table_bytes = (table.size() * 4 + 15) / 16 * 16;
        const uint64_t room = uint64_t(kTileMaxEntries - a.num_entries - C) * (sizeof(TileEntry) / 4);
        if (pieces_ok && !(p.flags_in & kPlanNoGather) && cost * 100 <= gwords * kGatherMaxReadsPct &&
            table.size() <= room && table.size() < (1u << 16) &&
            base + table_bytes <= std::min<uint64_t>(lds_limit, kHardLdsBytes)) {
            a.flags |= kTileGatherStore;
            if (rq.dst.block % 4 != 0)
                a.flags |= kTileGatherOdd;
            a.dst.lds_base = uint32_t(base);
            a.dst.lds_bytes = uint32_t(table_bytes);
            a.lds_bytes = uint32_t(base + table_bytes);
            ta.gather = g;
            std::memcpy(&ta.e[a.num_entries + C], table.data(), table.size() * 4);
            for (size_t f = 0; f < F; f++)
                ta.e[f].dst_pos = uint32_t(rq.dst.base[f]); // the value of lane 0 in a destination block
        }
    }
    // direct load: source leaf values in 16-byte granules of one leaf,
    // starting 16-byte aligned, leaf sizes 4, 8 or 16, destination positions
    // aligned to the leaf size, and at most kDirectLoadSlots granule slots
    // per thread
    // (a kept destination padding needs the destination region loaded first)
    if (preserve)
        a.flags |= kTilePreserve;
    // (leaves of 1 or 2 bytes, and destination values aligned below their
    // size, are written into the region in pieces: kTileSplitDst, unless
    // LLAMA_COPY_NO_SPLIT)
    bool dload = !direct && !(a.flags & kTileGatherStore) && !preserve && !(p.flags_in & kPlanNoDirect) && C == 0;
    bool split_dst = false;
    uint32_t slots = 0;
    std::vector<uint32_t> first(F, 0), wr_of(F, 0);
    for (size_t f = 0; f < F && dload; f++) {
        const TileEntry& e = ta.e[f];
        const uint32_t sz = e.size;
        const uint64_t dst_bits = uint64_t(e.dst_pos) | (a.dst.mode == kRecordMajor ? rq.dst.block : 0);
        const bool aligned = lowbit(dst_bits | 16) >= sz;
        const bool whole = sz == 4 || sz == 8 || sz == 16;
        // (a 1- or 2-byte leaf, a small share of a record, also loads from
        // AoSoA lane runs of 32 bytes and more)
        const bool runs = granule_runs(a.src, sz) ||
                          (sz <= 2 && a.src.mode == kRecordMajor && rq.src.block % 16 == 0 &&
                           rq.src.lanes * sz >= 32 && (rq.src.lanes * sz) % 16 == 0);
        dload = (sz == 1 || sz == 2 || whole) && runs && (e.src_addr & 15) == 0 &&
                ((aligned && whole) || (!(p.flags_in & kPlanNoSplit) && (sz <= 8 || aligned)));
        split_dst = split_dst || !aligned || !whole;
        wr_of[f] = std::min<uint32_t>(log2_move(dst_bits | sz), 7u);
        first[f] = slots;
        const uint32_t granules = uint32_t((uint64_t(T) * sz + 15) / 16);
        slots += (granules + 63) / 64 * 64;
    }
    if (dload && slots <= kDirectLoadSlots * p.threads && p.threads % 64 == 0) {
        a.flags |= kTileDirectLoad | (split_dst ? kTileSplitDst : 0u);
        a.slots = slots;
        for (size_t f = 0; f < k; f++) {
            TileEntry& e = ta.e[f];
            e.dst_pos -= sb; // the destination region moves to the start of LDS
            if (f < F) {
                e.src_pos = first[f];
                e.move = log2_exact(e.size) | (e.move & ~(7u | kMoveSplit | (7u << 24))) |
                         (split_dst ? wr_of[f] << 24 : 0u);
            }
        }
        a.src.lds_bytes = 0;
        a.dst.lds_base = 0;
        a.lds_bytes = db;
    }
    // field-major spans are short: rotate the first loading wave and the
    // first storing thread from leaf to leaf so that every wave takes a share
    const uint32_t nwaves = p.threads / 64;
    uint32_t first_wave = 0, first_thread = 0;
    for (size_t f = 0; f < F; f++) {
        TileEntry& e = ta.e[f];
        e.move |= (first_wave << 4) | (first_thread << 8);
        uint64_t granules = (uint64_t(T) * e.size + 30) / 16;
        if (a.flags & kTileDirectStore)
            granules = (uint64_t(T) * e.size + 15) / 16;
        first_wave = uint32_t((first_wave + (granules + 63) / 64) % nwaves);
        first_thread = uint32_t((first_thread + granules) % p.threads);
    }
    if (total_bytes(rq.dst.blob_size) >= kStreamStoreBytes)
        a.flags |= kTileStreamStores;
    if (total_bytes(rq.src.blob_size) >= kStreamLoadBytes)
        a.flags |= kTileStreamLoads;
    p.path = LLAMA_PATH_TILE;
    p.lds_bytes = a.lds_bytes;
    p.tiles = a.num_tiles;
    return true;
}

// Grid: by default one workgroup per tile (the hardware keeps as many
// resident as LDS and wave slots allow); with wg_per_cu set, a persistent
// grid of that many workgroups per compute unit loops over the tiles.
void tile_grid(Plan& p, uint32_t wg_per_cu)
{
    p.wg_per_cu = wg_per_cu;
    p.workgroups = wg_per_cu ? std::min<uint64_t>(p.tiles, uint64_t(device_cu_count()) * wg_per_cu) : p.tiles;
}

// The default tile: the largest power of two with T * S <= 16 KiB, but at
// least 128 records while T * S stays within 32 KiB, so that a large record
// (the 156-byte lattice-Boltzmann cell) still gets 1 KiB per f64 leaf span.
uint32_t default_tile(const Request& rq)
{
    uint64_t rec = std::max<uint64_t>(rq.record.packed_size, 1);
    uint64_t T = 16;
    while ((T * 2 * rec <= kDefaultTileBytes || (T < 128 && T * 2 * rec <= 2 * kDefaultTileBytes)) && T < 4096)
        T *= 2;
    return uint32_t(T);
}

// Default threads of a tile: about 112 source bytes per thread (128 threads
// for a 14 KiB particle tile), a multiple of 64 in 64 .. 256.
uint32_t default_threads(const Request& rq, uint32_t T)
{
    const uint64_t bytes = uint64_t(T) * std::max<uint64_t>(rq.record.packed_size, 1);
    const uint64_t th = (bytes / 112 + 63) / 64 * 64;
    return uint32_t(std::min<uint64_t>(std::max<uint64_t>(th, 64), kDefaultThreads));
}

void fill_naive(const Request& rq, Plan& p)
{
    const Record& r = rq.record;
    const size_t F = r.leaves.size();
    if (F + rq.dst.gaps.size() > size_t(kNaiveMaxEntries))
        fail(LLAMA_E_UNSUPPORTED, "record has more than " + std::to_string(kNaiveMaxEntries) +
                                      " leaves and padding gaps; this build cannot copy it");
    NaiveArgs& a = p.naive;
    std::memset(&a, 0, sizeof(a));
    a.n = rq.src.n;
    a.npad = rq.dst.npad;
    a.src.lanes = rq.src.lanes;
    a.src.block = rq.src.block;
    a.dst.lanes = rq.dst.lanes;
    a.dst.block = rq.dst.block;
    a.num_leaves = uint32_t(F);
    auto width = [](uint64_t addr, uint64_t size, const Side& s) {
        uint64_t w = addr | size;
        if (s.lanes >= 1 && s.npad > s.lanes)
            w |= s.block;
        return uint32_t(std::min<uint64_t>(lowbit(w | 8), 8));
    };
    for (size_t f = 0; f < F; f++) {
        NaiveEntry& e = a.e[f];
        e.src_addr = rq.src_ptr[rq.src.blob[f]] + rq.src.base[f];
        e.dst_addr = rq.dst_ptr[rq.dst.blob[f]] + rq.dst.base[f];
        e.size = r.leaves[f].size;
        e.width = std::min(width(e.src_addr, e.size, rq.src), width(e.dst_addr, e.size, rq.dst));
    }
    size_t k = F;
    for (const auto& g : rq.dst.gaps) {
        NaiveEntry& e = a.e[k++];
        e.src_addr = 0;
        e.dst_addr = rq.dst_ptr[0] + g.first;
        e.size = uint32_t(g.second);
        e.width = width(e.dst_addr, e.size, rq.dst);
    }
    a.num_entries = uint32_t(k);
    a.preserve = preserve_padding(rq, p) ? 1u : 0u;
    p.path = LLAMA_PATH_NAIVE;
    p.workgroups = (a.npad + p.threads - 1) / p.threads;
}

} // namespace

namespace {
Plan make_plan_raw(const Request& rq, const llama_copy_options* opt);
}

namespace {
Plan make_plan_tuned(const Request& rq, const llama_copy_options* opt);
}

// The zero fill of the padding between a destination's aligned SoA
// sub-arrays: STREAM plans of zero runs, chained through `then` when there
// are more runs than one launch takes.
Plan zero_fill_plan(const Request& rq)
{
    RunList rl;
    for (const Side::BlobGap& g : rq.dst.blob_gaps)
        rl.add(0, rq.dst_ptr[g.blob] + g.offset, g.length);
    Plan first;
    Plan* cur = &first;
    for (size_t k0 = 0; k0 < rl.runs.size(); k0 += size_t(kStreamMaxRuns)) {
        if (k0) {
            cur->then = std::make_shared<Plan>();
            cur = cur->then.get();
        }
        const size_t k1 = std::min(rl.runs.size(), k0 + size_t(kStreamMaxRuns));
        cur->path = LLAMA_PATH_STREAM;
        cur->threads = kDefaultThreads;
        std::memset(&cur->stream, 0, sizeof(cur->stream));
        uint64_t chunks = 0;
        for (size_t k = k0; k < k1; k++) {
            StreamRun run = rl.runs[k];
            run.first_chunk = chunks;
            chunks += (run.bytes + (uint64_t(1) << kStreamChunkLog2) - 1) >> kStreamChunkLog2;
            cur->stream.r[k - k0] = run;
            cur->write_bytes += run.bytes;
        }
        cur->stream.num_runs = uint32_t(k1 - k0);
        cur->stream.num_chunks = chunks;
        cur->workgroups = chunks;
    }
    return first;
}

// The plan for `opt` (and, into an aligned SoA destination whose path does
// not zero its padding itself, the zero fill after it).
Plan make_plan(const Request& rq, const llama_copy_options* opt)
{
    Plan p = make_plan_tuned(rq, opt);
    if (!rq.dst.blob_gaps.empty() && p.path != LLAMA_PATH_EMPTY && p.path != LLAMA_PATH_STREAM &&
        !(p.flags_in & kPlanPreserve))
        p.then = std::make_shared<Plan>(zero_fill_plan(rq));
    return p;
}

namespace {

// When the caller leaves the path and tile size to the library, a
// tuning-cache entry for this class of copies supplies them (the caller's
// threads and wg_per_cu still win).
Plan make_plan_tuned(const Request& rq, const llama_copy_options* opt)
{
    if (needs_box(rq))
        fail(LLAMA_E_UNSUPPORTED, "the two views place records at different linear indices (differing "
                                  "linearizers, or Morton holes): copy them with llama_copy or llama_copy_box");
    if (rq.chunks.empty() && rq.dst_stride.empty() && (!opt || (opt->path == LLAMA_PATH_AUTO && opt->tile_records == 0))) {
        llama_copy_options tuned;
        if (tune_lookup(tune_key(rq), tuned)) {
            if (opt && opt->threads)
                tuned.threads = opt->threads;
            if (opt && opt->wg_per_cu)
                tuned.wg_per_cu = opt->wg_per_cu;
            tuned.flags = (tuned.flags & kTuneFlags) | (opt ? opt->flags : 0u);
            try {
                return make_plan_raw(rq, &tuned);
            } catch (const Error&) {
                // the cached parameters do not apply here; plan from scratch
            }
        }
    }
    return make_plan_raw(rq, opt);
}

Plan make_plan_raw(const Request& rq, const llama_copy_options* opt)
{
    Plan p;
    p.read_bytes = total_bytes(rq.src.blob_size);
    p.write_bytes = total_bytes(rq.dst.blob_size);
    uint32_t want = opt ? opt->path : uint32_t(LLAMA_PATH_AUTO);
    if (opt && (opt->flags & ~kCopyFlags) != 0)
        fail(LLAMA_E_INVALID_ARG, "unknown bits in llama_copy_options.flags");
    p.flags_in = opt ? opt->flags : 0;
    if (want > LLAMA_PATH_NAIVE)
        fail(LLAMA_E_INVALID_ARG, "llama_copy_options.path is not a llama_path");
    uint32_t threads = (opt && opt->threads) ? opt->threads : 0;
    if (threads && (threads % 64 != 0 || threads > 1024))
        fail(LLAMA_E_INVALID_ARG, "threads must be a multiple of 64 in 64..1024");
    uint32_t T = (opt && opt->tile_records) ? opt->tile_records : 0;
    if (T && (!is_pow2(T) || T < 16 || T > 4096))
        fail(LLAMA_E_INVALID_ARG, "tile_records must be a power of two in 16..4096");
    uint32_t wg_per_cu = opt ? opt->wg_per_cu : 0;
    if (wg_per_cu > 16)
        fail(LLAMA_E_INVALID_ARG, "wg_per_cu must be 0..16");
    if (rq.dst.npad == 0) {
        p.path = LLAMA_PATH_EMPTY;
        return p;
    }
    p.threads = threads ? threads : kDefaultThreads;
    if (rq.src.kind == LLAMA_ONE) {
        // a broadcast: every record reads the same bytes, which only the
        // element-wise kernel's per-record arithmetic expresses (K = 0)
        if (want != LLAMA_PATH_AUTO && want != LLAMA_PATH_NAIVE)
            fail(LLAMA_E_UNSUPPORTED, "a One source is copied element-wise only");
        fill_naive(rq, p);
        return p;
    }
    if (!rq.chunks.empty() || !rq.dst_stride.empty()) {
        // a gathered source or scattered destination exists only for the tile kernel
        if (want != LLAMA_PATH_AUTO && want != LLAMA_PATH_TILE)
            fail(LLAMA_E_UNSUPPORTED, "copies gathered from or scattered to several parts take the TILE path only");
        if (!rq.chunks.empty() && !rq.dst_stride.empty())
            fail(LLAMA_E_UNSUPPORTED, "a copy gathers several source parts or scatters to several destination "
                                      "parts, not both");
        want = LLAMA_PATH_TILE;
    }
    if (want == LLAMA_PATH_AUTO || want == LLAMA_PATH_STREAM) {
        if (fill_stream(rq, p))
            return p;
        if (want == LLAMA_PATH_STREAM)
            fail(LLAMA_E_UNSUPPORTED, "the STREAM path needs long runs congruent modulo 4 on both sides");
    }
    if (want == LLAMA_PATH_AUTO || want == LLAMA_PATH_TILE) {
        // four records per thread in the LDS remap
        auto nthreads = [&](uint32_t t) { return default_threads(rq, t); };
        uint32_t t = T ? T : default_tile(rq);
        p.threads = threads ? threads : nthreads(t);
        bool ok = fill_tile(rq, t, T ? kHardLdsBytes : kMaxLdsBytes, p);
        while (!ok && !T && t > 16) {
            t /= 2;
            p.threads = threads ? threads : nthreads(t);
            ok = fill_tile(rq, t, kMaxLdsBytes, p);
        }
        if (ok && !threads && !(p.tile.h.flags & (kTileDirectLoad | kTileDirectStore))) {
            // a source in granules of one leaf loads directly when every
            // thread holds at most kDirectLoadSlots of them: try enough
            // threads for that
            uint32_t slots = 0;
            for (const Leaf& l : rq.record.leaves)
                slots += uint32_t((uint64_t(t) * l.size / 16 + 63) / 64 * 64);
            uint32_t want = (slots + kDirectLoadSlots * 64 - 1) / (kDirectLoadSlots * 64) * 64;
            if (want > p.threads && want <= 1024) {
                Plan q = p;
                q.threads = want;
                if (fill_tile(rq, t, kMaxLdsBytes, q) && (q.tile.h.flags & kTileDirectLoad))
                    p = q;
            }
        }
        if (ok && (p.tile.h.flags & kTileGatherStore) && rq.dst.lanes >= 32 && p.tile.h.src.mode == kFieldMajor) {
            // into AoSoA lane runs of 32 records or more from a field-major
            // source, loading the source granules into registers beats reading
            // them word by word (the mixed record from SoA into AoSoA32 and
            // AoSoA64: 5-11%)
            Plan q = p;
            q.flags_in |= kPlanNoGather;
            uint32_t slots = 0;
            for (const Leaf& l : rq.record.leaves)
                slots += uint32_t((uint64_t(t) * l.size / 16 + 63) / 64 * 64);
            q.threads = threads ? threads
                                : std::max(nthreads(t), (slots + kDirectLoadSlots * 64 - 1) / (kDirectLoadSlots * 64) * 64);
            if (q.threads <= 1024 && fill_tile(rq, t, T ? kHardLdsBytes : kMaxLdsBytes, q) &&
                (q.tile.h.flags & kTileDirectLoad)) {
                q.flags_in = p.flags_in;
                p = q;
            }
        }
        if (ok && !threads && (p.tile.h.flags & kTileGatherStore) && p.threads < 256 &&
            (p.threads < 192 || p.tile.h.src.mode == kRecordMajor)) {
            // a gathering tile assembles every destination word on its own:
            // 256 threads (particle pairs: -2% over 128), except that a
            // field-major source the default gives 192 keeps them (the
            // lattice-Boltzmann cell from SoA multi-blob: 7% faster than
            // 256; from AoSoA32, 4% slower)
            Plan q = p;
            q.threads = 256;
            if (fill_tile(rq, t, T ? kHardLdsBytes : kMaxLdsBytes, q) && (q.tile.h.flags & kTileGatherStore))
                p = q;
        }
        if (ok && !T && !threads && (p.tile.h.flags & kTileDirectStore) && p.tile.h.src.mode == kRecordMajor) {
            // direct store of a small record (at most 32 bytes) from a
            // record-major source runs fastest with tiles of about 4 KiB and
            // one wave per workgroup (+2-5% on the particle pairs; a
            // field-major source loses as much, its leaf spans being short),
            // as long as every leaf span keeps 256 bytes
            uint64_t t2 = t;
            while (t2 > 128 && t2 * std::max<uint64_t>(rq.record.packed_size, 1) > 4096)
                t2 /= 2;
            uint32_t smin = ~0u;
            for (const Leaf& l : rq.record.leaves)
                smin = std::min(smin, l.size);
            if (t2 < t && t2 * std::max<uint64_t>(rq.record.packed_size, 1) <= 4096 && t2 * smin >= 256) {
                Plan q = p;
                q.threads = 64;
                if (fill_tile(rq, uint32_t(t2), kMaxLdsBytes, q) && (q.tile.h.flags & kTileDirectStore))
                    p = q;
            }
        }
        if (ok && !T && !threads && (p.tile.h.flags & kTileDirectStore) && p.tile.h.src.mode == kFieldMajor) {
            // direct store from a field-major source reads one span per leaf:
            // where the widest leaf's span is under 2 KiB (the 156-byte
            // lattice-Boltzmann cell at 128 records), twice the records
            // (SoA multi-blob to AoSoA32 at 128^3: -14%)
            uint32_t smax = 0;
            for (const Leaf& l : rq.record.leaves)
                smax = std::max(smax, l.size);
            if (uint64_t(t) * smax < 2048 && t < 4096) {
                Plan q = p;
                q.threads = nthreads(2 * t);
                // the staged twin of the doubled tile may exceed the default
                // LDS budget; the direct store itself must not
                if (fill_tile(rq, 2 * t, kHardLdsBytes, q) && (q.tile.h.flags & kTileDirectStore) &&
                    q.lds_bytes <= kMaxLdsBytes)
                    p = q;
            }
        }
        if (ok) {
            tile_grid(p, wg_per_cu);
            return p;
        }
        if (want == LLAMA_PATH_TILE)
            fail(LLAMA_E_UNSUPPORTED, "the TILE path does not fit this record in LDS with these options");
    }
    p.threads = threads ? threads : kDefaultThreads;
    fill_naive(rq, p);
    return p;
}

} // namespace

bool trace_enabled()
{
    static const bool on = [] {
        const char* v = std::getenv("LLAMA_TRACE");
        return v && *v && std::string(v) != "0";
    }();
    return on;
}

void trace_plan(const Plan& p)
{
    static const char* const paths[] = {"auto", "stream", "tile", "naive", "empty"};
    std::string mode;
    if (p.path == LLAMA_PATH_TILE) {
        const uint32_t f = p.tile.h.flags;
        mode = (f & kTileDirectLoad)    ? " mode=direct_load"
               : (f & kTileDirectStore) ? " mode=direct_store"
               : (f & kTileGatherStore) ? ((f & kTileGatherOdd) ? " mode=gather_odd" : " mode=gather_store")
                                        : " mode=staged";
        mode += " tile=" + std::to_string(1u << p.tile.h.log2_tile) + " entries=" +
                std::to_string(p.tile.h.num_entries) + " lds=" + std::to_string(p.tile.h.lds_bytes);
        if (f & kTileGatherStore) { // words per super-block, and their reads of one piece each
            const uint32_t chunks = (f & kTileVirtualSrc) ? p.tile.h.slots : 0u;
            const uint32_t* tab = reinterpret_cast<const uint32_t*>(&p.tile.e[p.tile.h.num_entries + chunks]);
            uint64_t cost = 0;
            for (uint32_t w = 0; w < p.tile.gather.words; w++)
                cost += (tab[w] >> 30) == 0u ? 1u : (tab[w] >> 30) == 1u ? 2u : 4u;
            mode += " words=" + std::to_string(p.tile.gather.words) + " reads=" + std::to_string(cost);
        }
        if (f & kTilePreserve)
            mode += " keep_padding";
        if (f & kTileStreamLoads)
            mode += " nt_loads";
        if (f & kTileStreamStores)
            mode += " nt_stores";
    } else if (p.path == LLAMA_PATH_STREAM) {
        mode = " runs=" + std::to_string(p.stream.num_runs) + " chunks=" + std::to_string(p.stream.num_chunks);
        if (p.stream.flags & kStreamLoadsOnce)
            mode += " nt_loads";
    }
    std::fprintf(stderr, "[llama] path=%s%s threads=%u workgroups=%llu wg_per_cu=%u read=%llu write=%llu\n",
                 paths[p.path < 5 ? p.path : 0], mode.c_str(), p.threads, (unsigned long long)p.workgroups,
                 p.wg_per_cu, (unsigned long long)p.read_bytes, (unsigned long long)p.write_bytes);
}

} // namespace llama
