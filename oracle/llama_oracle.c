/*
 * llama_oracle.c -- CPU oracle for the layout-aware copy.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the plain, slow reference that the
 * GPU library is checked against.  Only the test suite, the smoke check and the
 * CPU-baseline leg of the benchmark load it; the library never does.  It shares
 * no code, header, table or helper with the GPU path: it has its own record
 * parser, its own flattening and its own mapping formulas.
 *
 * What it computes (LLAMA paper, section 3 "Design" and section 4.2):
 *
 *  - Record dimension (sec. 3.3 "Describing a data structure", Listings 1-2):
 *    a nested record of fields; a field is an elemental type or another
 *    record; a field of static array type T[n] is a record of n fields of T.
 *    Leaves are enumerated depth first in declaration order, which is the order
 *    forEachLeaf visits record coordinates (sec. 3.6 "C++ integration").
 *
 *  - Array dimensions: N-D extents; coordinates are visited in row-major order,
 *    last index fastest (ArrayDimsIndexRange, sec. 3.6), and a coordinate is
 *    linearised row-major (the index linearisation in Listing 4).
 *
 *  - Mappings (sec. 3.7 "Mappings"), each a function
 *    (array coordinate, leaf) -> (blob number, byte offset):
 *      AoS      fields one after another, repeated once per record; the fields
 *               either tightly packed or each padded to its type's alignment.
 *      SoA      per field, all records' values contiguous; either one blob per
 *               field (multi-blob) or all fields in one blob (single-blob),
 *               without padding between the sub-arrays (sec. 4.4 notes that
 *               SoA inserts no padding between its sub-arrays).
 *      SoA, aligned sub-arrays
 *               single-blob SoA whose every sub-array starts at a multiple of
 *               A bytes (`lanes` holds A, 0 meaning 256), the bytes between
 *               them being padding: the "with padding" SoA that sec. 4.4
 *               notes LLAMA's SoA cannot yet produce, and that sec. 3.9
 *               names as the other side of a copy between related mappings.
 *      AoSoA L  like AoS but each field repeated L times before the next
 *               field; the linear index i splits as (i / L, i mod L)
 *               (sec. 4.1).
 *      One      every coordinate maps to the same single record, packed:
 *               the array dimensions collapse to one element.
 *      Split    a selected part of the record dimension mapped by one of the
 *               mappings above, the remaining leaves by another; each part
 *               is that mapping of its own sub-record (the selected leaves,
 *               or the others in their order) and owns its blobs, the
 *               selected part's first.
 *
 *  - Copy (sec. 3.9 "Copying between views", sec. 4.2 "Layout changing
 *    copying"): the naive copy, nested loops over the array dimensions (outer)
 *    and the record leaves (inner), copying field by field through both
 *    mappings.  Bytes are copied verbatim, never as typed values.
 *
 * Readings where the paper is silent (each is listed with its reason in the
 * design notes of the repository):
 *   - aligned AoS follows the C struct rule on the flattened leaves: each leaf
 *     offset rounds up to the leaf's alignment, and the record stride rounds up
 *     to the largest leaf alignment (Listings 1 and 2 are declared equivalent);
 *     nested records add no padding of their own;
 *   - AoSoA blocks are packed: the chunk of leaf f starts at L * (packed offset
 *     of f), a block is L * (packed record size) bytes, the blob holds
 *     ceil(N / L) blocks;
 *   - multi-blob SoA has one blob per leaf, in leaf order;
 *   - Split selects a contiguous range of leaves (a record coordinate
 *     selects a subtree, whose leaves are contiguous in depth-first order),
 *     the two parts keep separate blobs, and a part may itself be a Split
 *     over its own leaves (the nesting of sec. 3.7's mapping listing);
 *   - aligned SoA: leaf f's sub-array starts at the first multiple of A at or
 *     after the end of leaf f - 1's; the blob ends with the last sub-array;
 *   - destination bytes that no (coordinate, leaf) pair maps to (alignment gaps
 *     of aligned AoS, unused lanes of the last AoSoA block, the padding between
 *     aligned SoA sub-arrays) are set to zero.
 *
 * Arithmetic: plain unsigned 64-bit integers, plain '/' and '%'.  No shifts,
 * masks, tiling, blocking or reordering.  The one exception is
 * orc_copy_threads, which runs the same loop over contiguous pieces of the
 * coordinate order on several host threads, to time the oracle on all cores;
 * its result is the serial copy's byte for byte.
 */
#include <stdint.h>
#include <stddef.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_MAX_RANK 8

/* mapping kinds */
#define ORC_AOS_PACKED 0
#define ORC_AOS_ALIGNED 1
#define ORC_SOA_SINGLE 2
#define ORC_SOA_MULTI 3
#define ORC_AOSOA 4
#define ORC_SPLIT 5
#define ORC_ONE 6
#define ORC_SOA_ALIGNED 7

/* most leaves a record mapped by Split may have */
#define ORC_SPLIT_MAX_LEAVES 1024

/* error codes */
#define ORC_OK 0
#define ORC_E_PARSE -1
#define ORC_E_TOO_MANY -2
#define ORC_E_ARG -3

typedef struct {
    int32_t nleaves;
    const uint64_t* size;  /* bytes of each leaf, in leaf order */
    const uint64_t* align; /* alignment of each leaf */
} orc_record;

typedef struct orc_mapping_s {
    int32_t kind;
    int32_t rank;
    uint64_t extents[ORC_MAX_RANK];
    uint64_t lanes; /* AoSoA: lanes L; aligned SoA: sub-array alignment A (0: 256) */
    /* Split only: leaves [first, first + count) form the selected part,
     * mapped by part_kind[0] (lanes part_lanes[0]); the other leaves by
     * part_kind[1] (lanes part_lanes[1]); a part of kind Split takes its
     * split from part_split[k] (over the part's own leaves) */
    int32_t first, count;
    int32_t part_kind[2];
    uint64_t part_lanes[2];
    const struct orc_mapping_s* part_split[2];
    /* how a coordinate becomes the linear index the mapping lays out: row-major
     * (ORC_ROW_MAJOR, the default), column-major or Morton order */
    int32_t linearizer;
} orc_mapping;

/* linearizers (sec. 3.7 lists them among the building blocks of mappings;
 * sec. 2 names other storage orders and space-filling curves) */
#define ORC_ROW_MAJOR 0
#define ORC_COL_MAJOR 1
#define ORC_MORTON 2

/* ---------------------------------------------------------------------------
 * Record parsing and flattening (sec. 3.3, Listings 1-2).
 *
 * Grammar:  record := '{' member (',' member)* '}'
 *           member := (type | record) ('[' count ']')?
 * type names: u8 i8 bool  (1 byte)   u16 i16 f16 bf16 (2 bytes)
 *             u32 i32 f32 (4 bytes)  u64 i64 f64      (8 bytes);
 * every elemental type is aligned to its own size.
 * ------------------------------------------------------------------------- */

typedef struct {
    const char* p;
    uint64_t* size;
    uint64_t* align;
    int max;
    int n;
    int err;
} orc_parser;

static void skip_space(orc_parser* ps)
{
    while (*ps->p == ' ' || *ps->p == '\t' || *ps->p == '\n')
        ps->p++;
}

static int elemental_size(const char* name, size_t len, uint64_t* out)
{
    static const struct { const char* name; uint64_t size; } types[] = {
        {"u8", 1},  {"i8", 1},  {"bool", 1}, {"u16", 2}, {"i16", 2},
        {"f16", 2}, {"bf16", 2}, {"u32", 4}, {"i32", 4}, {"f32", 4},
        {"u64", 8}, {"i64", 8}, {"f64", 8},
    };
    for (size_t k = 0; k < sizeof(types) / sizeof(types[0]); k++) {
        if (strlen(types[k].name) == len && strncmp(types[k].name, name, len) == 0) {
            *out = types[k].size;
            return 1;
        }
    }
    return 0;
}

static void parse_record(orc_parser* ps);

/* Parses one member and appends its leaves; a trailing [n] repeats them n
 * times (a static array becomes a record of n fields, sec. 3.3). */
static void parse_member(orc_parser* ps)
{
    skip_space(ps);
    int first = ps->n;
    if (*ps->p == '{') {
        parse_record(ps);
    } else {
        const char* start = ps->p;
        while ((*ps->p >= 'a' && *ps->p <= 'z') || (*ps->p >= '0' && *ps->p <= '9'))
            ps->p++;
        uint64_t s;
        if (!elemental_size(start, (size_t)(ps->p - start), &s)) {
            ps->err = ORC_E_PARSE;
            return;
        }
        if (ps->n >= ps->max) {
            ps->err = ORC_E_TOO_MANY;
            return;
        }
        ps->size[ps->n] = s;
        ps->align[ps->n] = s;
        ps->n++;
    }
    if (ps->err)
        return;
    skip_space(ps);
    if (*ps->p == '[') {
        ps->p++;
        uint64_t count = 0;
        int digits = 0;
        while (*ps->p >= '0' && *ps->p <= '9') {
            count = count * 10 + (uint64_t)(*ps->p - '0');
            ps->p++;
            digits++;
        }
        skip_space(ps);
        if (!digits || count == 0 || *ps->p != ']') {
            ps->err = ORC_E_PARSE;
            return;
        }
        ps->p++;
        int one = ps->n - first; /* leaves of a single element */
        for (uint64_t c = 1; c < count; c++) {
            for (int k = 0; k < one; k++) {
                if (ps->n >= ps->max) {
                    ps->err = ORC_E_TOO_MANY;
                    return;
                }
                ps->size[ps->n] = ps->size[first + k];
                ps->align[ps->n] = ps->align[first + k];
                ps->n++;
            }
        }
    }
}

static void parse_record(orc_parser* ps)
{
    skip_space(ps);
    if (*ps->p != '{') {
        ps->err = ORC_E_PARSE;
        return;
    }
    ps->p++;
    for (;;) {
        parse_member(ps);
        if (ps->err)
            return;
        skip_space(ps);
        if (*ps->p == ',') {
            ps->p++;
            continue;
        }
        if (*ps->p == '}') {
            ps->p++;
            return;
        }
        ps->err = ORC_E_PARSE;
        return;
    }
}

/* Flattens a record spec into leaf sizes and alignments in depth-first
 * declaration order.  Returns the leaf count, or a negative error. */
int orc_parse_record(const char* spec, uint64_t* size, uint64_t* align, int max_leaves)
{
    orc_parser ps = {spec, size, align, max_leaves, 0, 0};
    parse_record(&ps);
    if (ps.err)
        return ps.err;
    skip_space(&ps);
    if (*ps.p != '\0')
        return ORC_E_PARSE;
    return ps.n;
}

/* ---------------------------------------------------------------------------
 * Record-dimension sizes and offsets (sec. 3.7: "computing sizes and offsets
 * in the record dimension").
 * ------------------------------------------------------------------------- */

static uint64_t round_up(uint64_t x, uint64_t a)
{
    return (x + a - 1) / a * a;
}

/* packed offset of leaf f: the sum of the sizes of the leaves before it */
uint64_t orc_packed_offset(const orc_record* r, int f)
{
    uint64_t off = 0;
    for (int g = 0; g < f; g++)
        off += r->size[g];
    return off;
}

/* packed record size: the sum of all leaf sizes */
uint64_t orc_packed_size(const orc_record* r)
{
    return orc_packed_offset(r, r->nleaves);
}

/* aligned offset of leaf f: each leaf starts at the next multiple of its own
 * alignment after the end of the previous leaf */
uint64_t orc_aligned_offset(const orc_record* r, int f)
{
    uint64_t off = 0;
    for (int g = 0; g <= f; g++) {
        off = round_up(off, r->align[g]);
        if (g < f)
            off += r->size[g];
    }
    return off;
}

/* aligned record stride: end of the last leaf rounded up to the largest
 * alignment, so that the next record is aligned as well */
uint64_t orc_aligned_size(const orc_record* r)
{
    uint64_t max_align = 1;
    for (int g = 0; g < r->nleaves; g++)
        if (r->align[g] > max_align)
            max_align = r->align[g];
    if (r->nleaves == 0)
        return 0;
    uint64_t end = orc_aligned_offset(r, r->nleaves - 1) + r->size[r->nleaves - 1];
    return round_up(end, max_align);
}

/* ---------------------------------------------------------------------------
 * Array dimensions (sec. 3.6 ArrayDimsIndexRange; Listing 4 linearisation).
 * ------------------------------------------------------------------------- */

uint64_t orc_record_count(const orc_mapping* m)
{
    uint64_t n = 1;
    for (int d = 0; d < m->rank; d++)
        n *= m->extents[d];
    return n;
}

/* bits of the Morton index per dimension: enough for the largest extent */
static int morton_bits(const orc_mapping* m)
{
    uint64_t largest = 0;
    for (int d = 0; d < m->rank; d++)
        if (m->extents[d] > largest)
            largest = m->extents[d];
    int b = 0;
    while (b < 64 && ((uint64_t)1 << b) < largest)
        b++;
    return b;
}

/* The linear index of a coordinate.
 *  - row-major: last index fastest, i = (..((c0) * e1 + c1) * e2 + ..) + c(r-1)
 *    (the linearisation of Listing 4);
 *  - column-major: first index fastest, the same with the dimensions reversed;
 *  - Morton (Z-order): bit j of coordinate d becomes bit j * r + (r - 1 - d)
 *    of the index, so that within each group of r bits the last dimension
 *    is the least significant, as in row-major order. */
uint64_t orc_linearize(const orc_mapping* m, const uint64_t* coord)
{
    uint64_t i = 0;
    if (m->linearizer == ORC_COL_MAJOR) {
        for (int d = m->rank - 1; d >= 0; d--)
            i = i * m->extents[d] + coord[d];
        return i;
    }
    if (m->linearizer == ORC_MORTON) {
        int b = morton_bits(m);
        for (int j = 0; j < b; j++)
            for (int d = 0; d < m->rank; d++)
                if ((coord[d] / ((uint64_t)1 << j)) % 2 == 1)
                    i += (uint64_t)1 << (j * m->rank + (m->rank - 1 - d));
        return i;
    }
    for (int d = 0; d < m->rank; d++)
        i = i * m->extents[d] + coord[d];
    return i;
}

/* How many linear indices the mapping lays out: the record count for the
 * row- and column-major orders; for Morton order one more than the index of
 * the last coordinate (the index grows with every coordinate), so indices
 * that no coordinate reaches lie between them and are padding. */
uint64_t orc_linear_size(const orc_mapping* m)
{
    uint64_t n = orc_record_count(m);
    if (m->linearizer != ORC_MORTON || n == 0)
        return n;
    uint64_t last[ORC_MAX_RANK];
    for (int d = 0; d < m->rank; d++)
        last[d] = m->extents[d] - 1;
    return orc_linearize(m, last) + 1;
}

/* advances a coordinate to the next one in row-major order; returns 0 after
 * the last coordinate */
static int next_coord(const orc_mapping* m, uint64_t* coord)
{
    for (int d = m->rank - 1; d >= 0; d--) {
        coord[d]++;
        if (coord[d] < m->extents[d])
            return 1;
        coord[d] = 0;
    }
    return 0;
}

/* ---------------------------------------------------------------------------
 * Mappings (sec. 3.7): blob count, blob sizes, blobNrAndOffset.
 * ------------------------------------------------------------------------- */

/* one part of a Split: its plain mapping and its sub-record */
typedef struct {
    orc_mapping m;
    orc_record r;
    uint64_t size[ORC_SPLIT_MAX_LEAVES];
    uint64_t align[ORC_SPLIT_MAX_LEAVES];
} orc_part;

static int in_selection(const orc_mapping* m, int f) { return f >= m->first && f < m->first + m->count; }

/* part 0 holds the selected leaves, part 1 the others, each in leaf order */
static void split_part(const orc_mapping* m, const orc_record* r, int part, orc_part* out)
{
    if (m->part_kind[part] == ORC_SPLIT && m->part_split[part]) {
        out->m = *m->part_split[part]; /* a nested split over the part's leaves */
        out->m.rank = m->rank;
        for (int d = 0; d < ORC_MAX_RANK; d++)
            out->m.extents[d] = m->extents[d];
    } else {
        out->m = *m;
        out->m.kind = m->part_kind[part];
        out->m.lanes = m->part_lanes[part];
    }
    int n = 0;
    for (int f = 0; f < r->nleaves && n < ORC_SPLIT_MAX_LEAVES; f++)
        if (in_selection(m, f) == (part == 0)) {
            out->size[n] = r->size[f];
            out->align[n] = r->align[f];
            n++;
        }
    out->r.nleaves = n;
    out->r.size = out->size;
    out->r.align = out->align;
}

/* which part leaf f is in, and its index inside that part's sub-record */
static int split_leaf(const orc_mapping* m, int f, int* part)
{
    if (in_selection(m, f)) {
        *part = 0;
        return f - m->first;
    }
    *part = 1;
    return f < m->first ? f : f - m->count;
}

/* aligned SoA: where leaf f's sub-array starts, n records per sub-array;
 * each sub-array starts at the first multiple of A at or after the end of the
 * one before it */
static uint64_t soa_aligned_start(const orc_mapping* m, const orc_record* r, uint64_t n, int f)
{
    uint64_t a = m->lanes ? m->lanes : 256;
    uint64_t start = 0;
    for (int g = 1; g <= f; g++) /* after the sub-array of leaf g - 1 */
        start = round_up(start + n * r->size[g - 1], a);
    return start;
}

int orc_blob_count(const orc_mapping* m, const orc_record* r)
{
    if (m->kind == ORC_SPLIT) {
        orc_part p0, p1;
        split_part(m, r, 0, &p0);
        split_part(m, r, 1, &p1);
        return orc_blob_count(&p0.m, &p0.r) + orc_blob_count(&p1.m, &p1.r);
    }
    if (m->kind == ORC_SOA_MULTI)
        return r->nleaves;
    return 1; /* AoS, SoA single-blob, AoSoA, One */
}

uint64_t orc_blob_size(const orc_mapping* m, const orc_record* r, int blob)
{
    uint64_t n = orc_linear_size(m);
    if (m->kind == ORC_SPLIT) {
        orc_part p;
        split_part(m, r, 0, &p);
        int b0 = orc_blob_count(&p.m, &p.r);
        if (blob >= b0) {
            split_part(m, r, 1, &p);
            blob -= b0;
        }
        return orc_blob_size(&p.m, &p.r, blob);
    }
    switch (m->kind) {
    case ORC_AOS_PACKED:
        return n * orc_packed_size(r);
    case ORC_AOS_ALIGNED:
        return n * orc_aligned_size(r);
    case ORC_SOA_SINGLE:
        return n * orc_packed_size(r);
    case ORC_SOA_MULTI:
        return n * r->size[blob];
    case ORC_SOA_ALIGNED: /* up to the end of the last sub-array */
        return soa_aligned_start(m, r, n, r->nleaves - 1) + n * r->size[r->nleaves - 1];
    case ORC_AOSOA: {
        uint64_t blocks = (n + m->lanes - 1) / m->lanes;
        return blocks * m->lanes * orc_packed_size(r);
    }
    case ORC_ONE: /* a single packed record, whatever the extents */
        return orc_packed_size(r);
    }
    return 0;
}

/* The mapping function: where leaf f of the record at `coord` lives. */
int orc_blob_nr_and_offset(const orc_mapping* m, const orc_record* r, const uint64_t* coord,
                           int f, uint64_t* blob, uint64_t* offset)
{
    if (f < 0 || f >= r->nleaves)
        return ORC_E_ARG;
    if (m->kind == ORC_SPLIT) { /* the part's own mapping of its sub-record */
        orc_part p;
        int part;
        int g = split_leaf(m, f, &part);
        uint64_t first_blob = 0;
        if (part == 1) {
            split_part(m, r, 0, &p);
            first_blob = (uint64_t)orc_blob_count(&p.m, &p.r);
        }
        split_part(m, r, part, &p);
        int rc = orc_blob_nr_and_offset(&p.m, &p.r, coord, g, blob, offset);
        *blob += first_blob;
        return rc;
    }
    uint64_t n = orc_linear_size(m);
    uint64_t i = orc_linearize(m, coord);
    switch (m->kind) {
    case ORC_AOS_PACKED: /* record i at i * S, leaf f at its packed offset */
        *blob = 0;
        *offset = i * orc_packed_size(r) + orc_packed_offset(r, f);
        return ORC_OK;
    case ORC_AOS_ALIGNED: /* record i at i * R, leaf f at its aligned offset */
        *blob = 0;
        *offset = i * orc_aligned_size(r) + orc_aligned_offset(r, f);
        return ORC_OK;
    case ORC_SOA_SINGLE: /* sub-array of leaf f after the sub-arrays of 0..f-1 */
        *blob = 0;
        *offset = n * orc_packed_offset(r, f) + i * r->size[f];
        return ORC_OK;
    case ORC_SOA_MULTI: /* sub-array of leaf f in blob f */
        *blob = (uint64_t)f;
        *offset = i * r->size[f];
        return ORC_OK;
    case ORC_SOA_ALIGNED: /* sub-array of leaf f at its aligned start */
        *blob = 0;
        *offset = soa_aligned_start(m, r, n, f) + i * r->size[f];
        return ORC_OK;
    case ORC_AOSOA: { /* block i / L; inside it leaf f's L values, lane i mod L */
        uint64_t L = m->lanes;
        uint64_t block = i / L;
        uint64_t lane = i % L;
        *blob = 0;
        *offset = block * (L * orc_packed_size(r)) + L * orc_packed_offset(r, f) + lane * r->size[f];
        return ORC_OK;
    }
    case ORC_ONE: /* the one record, whatever the coordinate */
        (void)i;
        *blob = 0;
        *offset = orc_packed_offset(r, f);
        return ORC_OK;
    }
    return ORC_E_ARG;
}

/* ---------------------------------------------------------------------------
 * Validation shared by the entry points below.
 * ------------------------------------------------------------------------- */

static int valid_mapping(const orc_mapping* m, const orc_record* r);

static int valid_plain(int32_t kind, uint64_t lanes)
{
    if (kind == ORC_ONE)
        return 1;
    if (kind == ORC_SOA_ALIGNED) /* an alignment of 1 .. 2^20 bytes, a power of two, or 0 */
        return lanes <= ((uint64_t)1 << 20) && (lanes & (lanes - 1)) == 0;
    if (kind < ORC_AOS_PACKED || kind > ORC_AOSOA)
        return 0;
    return kind != ORC_AOSOA || lanes != 0;
}

static int valid_mapping(const orc_mapping* m, const orc_record* r)
{
    if (m->rank < 1 || m->rank > ORC_MAX_RANK)
        return 0;
    if (m->linearizer < ORC_ROW_MAJOR || m->linearizer > ORC_MORTON ||
        (m->linearizer == ORC_MORTON && morton_bits(m) * m->rank > 64))
        return 0;
    if (m->kind == ORC_SPLIT) {
        if (!(r->nleaves <= ORC_SPLIT_MAX_LEAVES && m->first >= 0 && m->count >= 1 && m->count < r->nleaves &&
              m->first + m->count <= r->nleaves))
            return 0;
        for (int k = 0; k < 2; k++) {
            if (m->part_kind[k] == ORC_SPLIT) {
                orc_part p;
                if (!m->part_split[k] || m->part_split[k]->kind != ORC_SPLIT)
                    return 0;
                split_part(m, r, k, &p);
                if (!valid_mapping(&p.m, &p.r))
                    return 0;
            } else if (!valid_plain(m->part_kind[k], m->part_lanes[k])) {
                return 0;
            }
        }
        return 1;
    }
    return valid_plain(m->kind, m->lanes);
}

static int same_extents(const orc_mapping* a, const orc_mapping* b)
{
    if (a->rank != b->rank)
        return 0;
    for (int d = 0; d < a->rank; d++)
        if (a->extents[d] != b->extents[d])
            return 0;
    return 1;
}

/* ---------------------------------------------------------------------------
 * The copy (sec. 3.9, sec. 4.2 naive copy).
 * ------------------------------------------------------------------------- */

/* Copies every (coordinate, leaf) value of the source view into the
 * destination view.  Destination bytes that no value maps to are zero. */
int orc_copy(const orc_record* r, const orc_mapping* src, uint8_t* const* src_blobs,
             const orc_mapping* dst, uint8_t* const* dst_blobs)
{
    if (!valid_mapping(src, r) || !valid_mapping(dst, r) || !same_extents(src, dst))
        return ORC_E_ARG;
    /* padding policy: the whole destination starts at zero */
    for (int b = 0; b < orc_blob_count(dst, r); b++)
        memset(dst_blobs[b], 0, (size_t)orc_blob_size(dst, r, b));
    if (orc_record_count(src) == 0)
        return ORC_OK;
    uint64_t coord[ORC_MAX_RANK] = {0};
    do {
        for (int f = 0; f < r->nleaves; f++) {
            uint64_t bs, os, bd, od;
            orc_blob_nr_and_offset(src, r, coord, f, &bs, &os);
            orc_blob_nr_and_offset(dst, r, coord, f, &bd, &od);
            memcpy(dst_blobs[bd] + od, src_blobs[bs] + os, (size_t)r->size[f]);
        }
    } while (next_coord(src, coord));
    return ORC_OK;
}

/* The same copy with the other padding reading, which the library offers as
 * an option: destination bytes that no value maps to keep whatever they held
 * before the copy (nothing is zeroed). */
int orc_copy_keep(const orc_record* r, const orc_mapping* src, uint8_t* const* src_blobs,
                  const orc_mapping* dst, uint8_t* const* dst_blobs)
{
    if (!valid_mapping(src, r) || !valid_mapping(dst, r) || !same_extents(src, dst))
        return ORC_E_ARG;
    if (orc_record_count(src) == 0)
        return ORC_OK;
    uint64_t coord[ORC_MAX_RANK] = {0};
    do {
        for (int f = 0; f < r->nleaves; f++) {
            uint64_t bs, os, bd, od;
            orc_blob_nr_and_offset(src, r, coord, f, &bs, &os);
            orc_blob_nr_and_offset(dst, r, coord, f, &bd, &od);
            memcpy(dst_blobs[bd] + od, src_blobs[bs] + os, (size_t)r->size[f]);
        }
    } while (next_coord(src, coord));
    return ORC_OK;
}

/* The copy of a box of the array dimensions (sec. 3.2: a VirtualView is a
 * view onto a sub-box of another view's array dimensions, shifted by an
 * offset; sec. 3.9 names copies between views of different size or shape).
 * Source and destination share the record dimension and the rank; their
 * extents may differ.  For every coordinate c of the box, in row-major order,
 * and every leaf, the value at src_offset + c is copied to dst_offset + c.
 * Destination records outside the box keep every byte.  The alignment gaps of
 * the box's records in an aligned-AoS destination become zero, or keep their
 * bytes with `keep`.  Both mappings are plain (not Split); the source may be
 * One.  The box must lie inside both views. */
int orc_copy_box(const orc_record* r, const orc_mapping* src, uint8_t* const* src_blobs, const uint64_t* src_offset,
                 const orc_mapping* dst, uint8_t* const* dst_blobs, const uint64_t* dst_offset, const uint64_t* box,
                 int keep)
{
    if (!valid_mapping(src, r) || !valid_mapping(dst, r) || src->rank != dst->rank || src->kind == ORC_SPLIT ||
        dst->kind == ORC_SPLIT || dst->kind == ORC_ONE)
        return ORC_E_ARG;
    orc_mapping b = *src; /* iterates the box's coordinates */
    for (int d = 0; d < src->rank; d++) {
        if (src_offset[d] + box[d] > src->extents[d] || dst_offset[d] + box[d] > dst->extents[d] ||
            src_offset[d] + box[d] < box[d] || dst_offset[d] + box[d] < box[d])
            return ORC_E_ARG;
        b.extents[d] = box[d];
    }
    if (orc_record_count(&b) == 0)
        return ORC_OK;
    uint64_t c[ORC_MAX_RANK] = {0};
    do {
        uint64_t sc[ORC_MAX_RANK], dc[ORC_MAX_RANK];
        for (int d = 0; d < src->rank; d++) {
            sc[d] = src_offset[d] + c[d];
            dc[d] = dst_offset[d] + c[d];
        }
        if (!keep && dst->kind == ORC_AOS_ALIGNED) {
            /* the record's bytes start at zero, so its gaps end up zero */
            uint64_t R = orc_aligned_size(r);
            memset(dst_blobs[0] + orc_linearize(dst, dc) * R, 0, (size_t)R);
        }
        for (int f = 0; f < r->nleaves; f++) {
            uint64_t bs, os, bd, od;
            orc_blob_nr_and_offset(src, r, sc, f, &bs, &os);
            orc_blob_nr_and_offset(dst, r, dc, f, &bd, &od);
            memcpy(dst_blobs[bd] + od, src_blobs[bs] + os, (size_t)r->size[f]);
        }
    } while (next_coord(&b, c));
    return ORC_OK;
}

/* The copy between views whose records differ (sec. 3.9: a field missing on
 * one side).  Destination leaf k takes source leaf from[k], whose size must be
 * the same; a leaf with from[k] < 0 keeps all its bytes, unused AoSoA lanes
 * included.  The destination's padding (alignment gaps, and the unused AoSoA
 * lanes of the leaves that take a value) becomes zero, or keeps its bytes
 * with `keep`.  Both mappings are plain (not Split); the source may be One. */
int orc_copy_leaves(const orc_record* rs, const orc_mapping* src, uint8_t* const* src_blobs, const orc_record* rd,
                    const orc_mapping* dst, uint8_t* const* dst_blobs, const int32_t* from, int keep)
{
    if (!valid_mapping(src, rs) || !valid_mapping(dst, rd) || !same_extents(src, dst) || src->kind == ORC_SPLIT ||
        dst->kind == ORC_SPLIT || dst->kind == ORC_ONE || src->linearizer != ORC_ROW_MAJOR ||
        dst->linearizer != ORC_ROW_MAJOR)
        return ORC_E_ARG;
    for (int k = 0; k < rd->nleaves; k++)
        if (from[k] >= rs->nleaves || (from[k] >= 0 && rs->size[from[k]] != rd->size[k]))
            return ORC_E_ARG;
    uint64_t n = orc_record_count(dst);
    if (!keep) {
        /* mark every byte a leaf owns: values of all records, and for the
         * leaves that keep their bytes, their unused AoSoA lanes too */
        int nb = orc_blob_count(dst, rd);
        uint8_t* owned[ORC_SPLIT_MAX_LEAVES];
        if (nb > ORC_SPLIT_MAX_LEAVES)
            return ORC_E_ARG;
        for (int b = 0; b < nb; b++)
            owned[b] = (uint8_t*)calloc((size_t)orc_blob_size(dst, rd, b) + 1, 1);
        uint64_t coord[ORC_MAX_RANK] = {0};
        if (n > 0)
            do {
                for (int k = 0; k < rd->nleaves; k++) {
                    uint64_t b, o;
                    orc_blob_nr_and_offset(dst, rd, coord, k, &b, &o);
                    memset(owned[b] + o, 1, (size_t)rd->size[k]);
                }
            } while (next_coord(dst, coord));
        if (dst->kind == ORC_AOSOA) {
            uint64_t L = dst->lanes;
            for (uint64_t i = n; i < (n + L - 1) / L * L; i++)
                for (int k = 0; k < rd->nleaves; k++)
                    if (from[k] < 0)
                        memset(owned[0] + (i / L) * (L * orc_packed_size(rd)) + L * orc_packed_offset(rd, k) +
                                   (i % L) * rd->size[k],
                               1, (size_t)rd->size[k]);
        }
        for (int b = 0; b < nb; b++) {
            uint64_t sz = orc_blob_size(dst, rd, b);
            for (uint64_t o = 0; o < sz; o++)
                if (!owned[b][o])
                    dst_blobs[b][o] = 0;
            free(owned[b]);
        }
    }
    if (n == 0)
        return ORC_OK;
    uint64_t coord[ORC_MAX_RANK] = {0};
    do {
        for (int k = 0; k < rd->nleaves; k++) {
            if (from[k] < 0)
                continue;
            uint64_t bs, os, bd, od;
            orc_blob_nr_and_offset(src, rs, coord, from[k], &bs, &os);
            orc_blob_nr_and_offset(dst, rd, coord, k, &bd, &od);
            memcpy(dst_blobs[bd] + od, src_blobs[bs] + os, (size_t)rd->size[k]);
        }
    } while (next_coord(dst, coord));
    return ORC_OK;
}

/* Adds one to counts[b][o] for every byte o of blob b that a (coordinate, leaf)
 * value maps to.  Used to check that a mapping is injective and which of its
 * bytes are padding. */
int orc_write_counts(const orc_record* r, const orc_mapping* m, uint32_t* const* counts)
{
    if (!valid_mapping(m, r))
        return ORC_E_ARG;
    if (orc_record_count(m) == 0)
        return ORC_OK;
    uint64_t coord[ORC_MAX_RANK] = {0};
    do {
        for (int f = 0; f < r->nleaves; f++) {
            uint64_t b, o;
            orc_blob_nr_and_offset(m, r, coord, f, &b, &o);
            for (uint64_t k = 0; k < r->size[f]; k++)
                counts[b][o + k]++;
        }
    } while (next_coord(m, coord));
    return ORC_OK;
}

/* The writes that the copy's definition makes into the destination, as
 * per-byte counts (the Heatmap of sec. 3.7 applied to the definition of sec.
 * 3.9): one for every byte a value is copied to, and one for every byte of
 * the zero fill.  from == NULL: the plain copy, every leaf takes a value;
 * otherwise destination leaf k takes a value when from[k] >= 0, as in
 * orc_copy_leaves, whose zero fill covers the bytes no leaf owns and the
 * unused AoSoA lanes of the leaves that take a value.  keep: no zero fill.
 * counts[b] holds blob_size(b) counters and is added to. */
int orc_copy_writes(const orc_record* r, const orc_mapping* dst, const int32_t* from, int keep,
                    uint32_t* const* counts)
{
    if (!valid_mapping(dst, r) || dst->kind == ORC_ONE)
        return ORC_E_ARG;
    int nb = orc_blob_count(dst, r);
    if (nb > ORC_SPLIT_MAX_LEAVES)
        return ORC_E_ARG;
    /* owned[b][o]: 1 when a value of a leaf maps to byte o, 2 when it is an
     * unused AoSoA lane of a leaf that keeps its bytes */
    uint8_t* owned[ORC_SPLIT_MAX_LEAVES];
    for (int b = 0; b < nb; b++)
        owned[b] = (uint8_t*)calloc((size_t)orc_blob_size(dst, r, b) + 1, 1);
    uint64_t n = orc_record_count(dst);
    uint64_t coord[ORC_MAX_RANK] = {0};
    if (n > 0)
        do {
            for (int f = 0; f < r->nleaves; f++) {
                uint64_t b, o;
                orc_blob_nr_and_offset(dst, r, coord, f, &b, &o);
                for (uint64_t k = 0; k < r->size[f]; k++) {
                    owned[b][o + k] = 1;
                    if (!from || from[f] >= 0)
                        counts[b][o + k]++;
                }
            }
        } while (next_coord(dst, coord));
    if (from && dst->kind == ORC_AOSOA) {
        uint64_t L = dst->lanes;
        for (uint64_t i = n; i < (n + L - 1) / L * L; i++)
            for (int f = 0; f < r->nleaves; f++)
                if (from[f] < 0)
                    memset(owned[0] + (i / L) * (L * orc_packed_size(r)) + L * orc_packed_offset(r, f) +
                               (i % L) * r->size[f],
                           2, (size_t)r->size[f]);
    }
    for (int b = 0; b < nb; b++) {
        uint64_t sz = orc_blob_size(dst, r, b);
        if (!keep)
            for (uint64_t o = 0; o < sz; o++)
                if (!owned[b][o])
                    counts[b][o]++;
        free(owned[b]);
    }
    return ORC_OK;
}

/* Checks sampled values of a finished copy one by one: for each sample
 * (linear index idx[k], leaf leaf[k]) the destination bytes must equal the
 * source bytes, both located through the mappings.  Returns the number of
 * mismatching samples; the first mismatch index goes to *first_bad. */
int64_t orc_check_samples(const orc_record* r, const orc_mapping* src, uint8_t* const* src_blobs,
                          const orc_mapping* dst, uint8_t* const* dst_blobs, const uint64_t* idx,
                          const int32_t* leaf, int64_t nsamples, int64_t* first_bad)
{
    int64_t bad = 0;
    *first_bad = -1;
    for (int64_t k = 0; k < nsamples; k++) {
        /* the coordinate of linear index idx[k], row-major */
        uint64_t coord[ORC_MAX_RANK];
        uint64_t rest = idx[k];
        for (int d = src->rank - 1; d >= 0; d--) {
            coord[d] = rest % src->extents[d];
            rest /= src->extents[d];
        }
        uint64_t bs, os, bd, od;
        if (orc_blob_nr_and_offset(src, r, coord, leaf[k], &bs, &os) != ORC_OK ||
            orc_blob_nr_and_offset(dst, r, coord, leaf[k], &bd, &od) != ORC_OK)
            return -1;
        if (memcmp(dst_blobs[bd] + od, src_blobs[bs] + os, (size_t)r->size[leaf[k]]) != 0) {
            if (*first_bad < 0)
                *first_bad = k;
            bad++;
        }
    }
    return bad;
}

/* ---------------------------------------------------------------------------
 * The same copy on several host threads (the paper times its copies with one
 * thread per physical core, sec. 4).  The coordinate range is cut into
 * contiguous pieces of the row-major order; each thread runs the loop of
 * orc_copy over its piece, starting from the coordinate of its first linear
 * index.  Values of different coordinates occupy different destination bytes
 * (a mapping that is a valid destination maps distinct values to distinct
 * bytes), so the result does not depend on the number of threads.  A
 * destination holding a One part (every coordinate at the same bytes) is copied
 * on one thread, so that the last coordinate's value wins as in orc_copy.
 * ------------------------------------------------------------------------- */

static int has_one(const orc_mapping* m)
{
    if (m->kind == ORC_ONE)
        return 1;
    if (m->kind != ORC_SPLIT)
        return 0;
    for (int k = 0; k < 2; k++) {
        if (m->part_kind[k] == ORC_ONE)
            return 1;
        if (m->part_kind[k] == ORC_SPLIT && m->part_split[k] && has_one(m->part_split[k]))
            return 1;
    }
    return 0;
}

/* the row-major coordinate of linear index i */
static void delinearize(const orc_mapping* m, uint64_t i, uint64_t* coord)
{
    for (int d = m->rank - 1; d >= 0; d--) {
        coord[d] = i % m->extents[d];
        i /= m->extents[d];
    }
}

/* orc_copy (keep == 0) or orc_copy_keep (keep != 0) on `threads` threads
 * (<= 0: the OpenMP default).  Built without OpenMP it runs on one thread. */
int orc_copy_threads(const orc_record* r, const orc_mapping* src, uint8_t* const* src_blobs,
                     const orc_mapping* dst, uint8_t* const* dst_blobs, int keep, int threads)
{
    if (!valid_mapping(src, r) || !valid_mapping(dst, r) || !same_extents(src, dst))
        return ORC_E_ARG;
    if (has_one(dst))
        return keep ? orc_copy_keep(r, src, src_blobs, dst, dst_blobs) : orc_copy(r, src, src_blobs, dst, dst_blobs);
#ifdef _OPENMP
    if (threads <= 0)
        threads = omp_get_max_threads();
#else
    threads = 1;
#endif
    int64_t pieces = (int64_t)threads * 16;
    if (!keep) {
        /* padding policy: the whole destination starts at zero */
        for (int b = 0; b < orc_blob_count(dst, r); b++) {
            uint64_t size = orc_blob_size(dst, r, b);
            uint8_t* base = dst_blobs[b];
#ifdef _OPENMP
#pragma omp parallel for num_threads(threads) schedule(static)
#endif
            for (int64_t k = 0; k < pieces; k++) {
                uint64_t lo = size / (uint64_t)pieces * (uint64_t)k;
                uint64_t hi = k + 1 == pieces ? size : size / (uint64_t)pieces * (uint64_t)(k + 1);
                memset(base + lo, 0, (size_t)(hi - lo));
            }
        }
    }
    uint64_t n = orc_record_count(src);
    if (n == 0)
        return ORC_OK;
#ifdef _OPENMP
#pragma omp parallel for num_threads(threads) schedule(dynamic, 1)
#endif
    for (int64_t k = 0; k < pieces; k++) {
        uint64_t lo = n / (uint64_t)pieces * (uint64_t)k;
        uint64_t hi = k + 1 == pieces ? n : n / (uint64_t)pieces * (uint64_t)(k + 1);
        if (lo == hi)
            continue;
        uint64_t coord[ORC_MAX_RANK] = {0};
        delinearize(src, lo, coord);
        for (uint64_t i = lo; i < hi; i++) {
            for (int f = 0; f < r->nleaves; f++) {
                uint64_t bs, os, bd, od;
                orc_blob_nr_and_offset(src, r, coord, f, &bs, &os);
                orc_blob_nr_and_offset(dst, r, coord, f, &bd, &od);
                memcpy(dst_blobs[bd] + od, src_blobs[bs] + os, (size_t)r->size[f]);
            }
            next_coord(src, coord);
        }
    }
    return ORC_OK;
}

/* Host memcpy of `bytes` bytes on `threads` threads, each taking one
 * contiguous piece: the reference the paper sets beside its copies
 * (sec. 4.2).  Returns the number of threads used. */
int orc_memcpy_threads(uint8_t* dst, const uint8_t* src, uint64_t bytes, int threads)
{
#ifdef _OPENMP
    if (threads <= 0)
        threads = omp_get_max_threads();
#else
    threads = 1;
#endif
    int used = 1;
#ifdef _OPENMP
#pragma omp parallel num_threads(threads)
    {
        int t = omp_get_thread_num(), nt = omp_get_num_threads();
        uint64_t lo = bytes / (uint64_t)nt * (uint64_t)t;
        uint64_t hi = t + 1 == nt ? bytes : bytes / (uint64_t)nt * (uint64_t)(t + 1);
        memcpy(dst + lo, src + lo, (size_t)(hi - lo));
        if (t == 0)
            used = nt;
    }
#else
    memcpy(dst, src, (size_t)bytes);
#endif
    return used;
}

/* Threads an OpenMP region of this library gets by default (1 without
 * OpenMP). */
int orc_max_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
