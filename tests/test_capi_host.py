"""Host-side tests of the C ABI (no GPU): the library loads and exports every
entry point of include/llama_mi355x.h, its host mapping arithmetic agrees with
the oracle, the planner picks the expected path, and invalid requests fail with
the documented status before anything would be enqueued."""
import ctypes
import os
import random
import re
import subprocess
import sys

import numpy as np
import pytest

from paper_2106_04284_amd import llama as L
from paper_2106_04284_amd import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LAYOUTS = W.LAYOUTS + [("aosoa", 1), ("aosoa", 2), ("aosoa", 4)]


def _declared_functions():
    names = set()
    inc = os.path.join(ROOT, "include")
    for fn in os.listdir(inc):
        if fn.endswith(".h"):
            text = open(os.path.join(inc, fn)).read()
            text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
            names |= set(re.findall(r"\b(llama_[a-z0-9_]+)\s*\(", text))
    return sorted(names)


def test_library_exports_every_declared_function():
    lib = ctypes.CDLL(L.LIB_PATH)
    names = _declared_functions()
    assert "llama_copy" in names
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing


@pytest.mark.parametrize("name", ["particle", "lbm", "mixed", "listing1"])
def test_record_info_matches_oracle(orc, name):
    r = L.Record(W.RECORDS[name])
    o = orc.Record(W.RECORDS[name])
    assert r.info() == (o.nleaves, o.packed_size, o.aligned_size)
    for f in range(o.nleaves):
        leaf = r.leaf(f)
        assert leaf["size"] == o.sizes[f]
        assert leaf["align"] == o.aligns[f]
        assert leaf["packed_offset"] == o.packed_offset(f)
        assert leaf["aligned_offset"] == o.aligned_offset(f)


def _random_record(g, depth=0):
    types = ["u8", "u16", "u32", "f64", "bool", "f32", "i64"]
    out = []
    for _ in range(g.randint(1, 4)):
        if depth < 2 and g.random() < 0.3:
            m = _random_record(g, depth + 1)
        else:
            m = g.choice(types)
        if g.random() < 0.2:
            m = (m, g.randint(1, 3))
        out.append(m)
    return out


@pytest.mark.parametrize("seed", range(12))
def test_mapping_arithmetic_matches_oracle(orc, seed):
    g = random.Random(seed)
    rec = _random_record(g) if seed >= 4 else W.RECORDS[["particle", "lbm", "mixed", "listing1"][seed]]
    r, o = L.Record(rec), orc.Record(rec)
    ext = [g.randint(1, 6) for _ in range(g.randint(1, 3))]
    for kind, lanes in LAYOUTS:
        m = L.Mapping(r, kind, ext, lanes)
        mo = orc.Mapping(o, kind, ext, lanes)
        assert m.blob_sizes() == mo.blob_sizes(), (kind, lanes)
        for _ in range(40):
            c = [g.randrange(e) for e in ext]
            f = g.randrange(o.nleaves)
            assert m.offset(c, f) == mo.blob_nr_and_offset(c, f), (kind, lanes, c, f)


@pytest.mark.parametrize("lin", ["col", "morton"])
@pytest.mark.parametrize("seed", range(4))
def test_linearizer_offsets_match_oracle(orc, lin, seed):
    """Blob sizes and every offset of column-major and Morton mappings equal
    the oracle's (Morton extents of any size: the holes in its indices are
    padding, so blob sizes follow the last coordinate's index)."""
    g = random.Random(seed)
    name = ["particle", "lbm", "mixed", "listing1"][seed]
    r, o = L.Record(W.RECORDS[name]), orc.Record(W.RECORDS[name])
    ext = [g.randint(1, 9) for _ in range(g.randint(2, 4))]
    for kind, lanes in LAYOUTS:
        m = L.Mapping(r, kind, ext, lanes, linearizer=lin)
        mo = orc.Mapping(o, kind, ext, lanes, linearizer=lin)
        assert m.blob_sizes() == mo.blob_sizes(), (kind, lanes, ext)
        for _ in range(40):
            c = [g.randrange(e) for e in ext]
            f = g.randrange(o.nleaves)
            assert m.offset(c, f) == mo.blob_nr_and_offset(c, f), (kind, lanes, c, f)


def test_box_plans_host():
    """Copies between linearizers plan the box kernel: tiles within the LDS
    budget, a bad linearizer and Split with a linearizer refused."""
    r = L.Record(W.RECORDS["lbm"])
    for a, b in [("row", "col"), ("col", "morton"), ("morton", "row"), ("morton", "morton")]:
        for kind, lanes in LAYOUTS:
            ext = [100, 60, 7] if b != "morton" or a != "morton" else [100, 60, 7]
            p = L.plan(L.Mapping(r, "aos_aligned", ext, linearizer=a), L.Mapping(r, kind, ext, lanes, linearizer=b))
            assert p["path"] == "box", (a, b, kind)
            assert 0 < p["lds_bytes"] <= 64 * 1024 and p["tile_records"] >= 16
    m = L.Mapping(r, "aos_packed", [4, 4])
    m.desc.linearizer = 3
    with pytest.raises(L.LlamaError) as e:
        m.blob_sizes()
    assert e.value.status == L.E_INVALID_ARG
    with pytest.raises(L.LlamaError) as e:
        L.Mapping(r, "split", [4, 4], split=(0, 3, ("soa_multi", 0), ("aos_packed", 0)), linearizer="col").blob_sizes()
    assert e.value.status == L.E_UNSUPPORTED


def test_planner_paths_for_particle_pairs():
    r = L.Record(W.PARTICLE)
    n = 1 << 26
    seen = {}
    for a in W.LAYOUTS:
        for b in W.LAYOUTS:
            if a == b:
                continue
            p = L.plan(L.Mapping(r, a[0], [n], a[1]), L.Mapping(r, b[0], [n], b[1]))
            seen[(a, b)] = p["path"]
            assert p["read_bytes"] == p["write_bytes"] == n * 28
    aos = {("aos_packed", 0), ("aos_aligned", 0)}
    soa = {("soa_single", 0), ("soa_multi", 0)}
    for (a, b), path in seen.items():
        if {a, b} <= aos or {a, b} <= soa:
            assert path == "stream", (a, b)  # identical bytes, or one long run per leaf
        else:
            assert path == "tile", (a, b)


SOA_KINDS = {"soa_single", "soa_multi"}


@pytest.mark.parametrize("name", ["particle", "mixed", "lbm", "listing1"])
@pytest.mark.parametrize("n", [1000, 1024])
def test_planner_classification_all_pairs(orc, name, n):
    """All 49 ordered pairs (identity included): a long-run copy only where
    every byte moves in whole runs (identical placement without destination
    gaps, or SoA <-> SoA, one run per leaf); the tiled transpose otherwise.
    A different mapping never becomes a whole-blob memcpy (sec. 3.9)."""
    r = L.Record(W.RECORDS[name])
    ro = orc.Record(W.RECORDS[name])
    gaps = ro.aligned_size != ro.packed_size
    for a in W.LAYOUTS:
        for b in W.LAYOUTS:
            ma, mb = L.Mapping(r, a[0], [n], a[1]), L.Mapping(r, b[0], [n], b[1])
            p = L.plan(ma, mb)
            same_bytes = a == b or (not gaps and {a[0], b[0]} == {"aos_packed", "aos_aligned"})
            if same_bytes and not (b[0] == "aos_aligned" and gaps):
                assert p["path"] == "stream", (a, b)
                # a partial last AoSoA block: whole blocks, then per leaf its
                # values and its zero lanes (leaf 0's values continue the
                # whole blocks: one run)
                tail = b[0] == "aosoa" and n % b[1] != 0
                assert p["runs"] == (mb.blob_count if not tail else 2 * ro.nleaves), (a, b)
            elif a[0] in SOA_KINDS and b[0] in SOA_KINDS:
                assert p["path"] == "stream" and p["runs"] == ro.nleaves, (a, b)
            else:
                assert p["path"] == "tile", (a, b)


def test_default_tile_sizes():
    """Default tile records and threads: about 16 KiB of source per tile and
    112 source bytes per thread; at least 256 threads for a gathering tile
    unless a field-major source gets 192; a small record stored directly
    from a record-major source in tiles of 4 KiB and one wave; a direct
    store from a field-major source whose widest leaf span is under 2 KiB
    at twice the records."""
    def plan(name, a, b, n):
        r = L.Record(W.RECORDS[name])
        p = L.plan(L.Mapping(r, a[0], [n], a[1]), L.Mapping(r, b[0], [n], b[1]))
        return p["tile_mode"], p["tile_records"], p["threads"]

    AA, M, S, Q32 = ("aos_aligned", 0), ("soa_multi", 0), ("soa_single", 0), ("aosoa", 32)
    A, Q8 = ("aos_packed", 0), ("aosoa", 8)
    n = 128 ** 3
    # lattice-Boltzmann cell, 156 bytes packed: 128-record tiles, 192 threads
    assert plan("lbm", AA, M, n) == ("direct_store", 128, 192)
    assert plan("lbm", Q32, M, n) == ("direct_store", 128, 192)
    assert plan("lbm", M, AA, n) == ("gather_store", 128, 192)
    assert plan("lbm", Q32, AA, n) == ("gather_store", 128, 256)
    assert plan("lbm", M, Q32, n) == ("direct_store", 256, 256)
    # particle, 28 bytes: 512-record tiles; 4 KiB and one wave from a
    # record-major source; the 2 KiB leaf spans from SoA are not doubled
    n = 1 << 26
    assert plan("particle", S, A, n) == ("gather_store", 512, 256)
    assert plan("particle", A, Q8, n) == ("gather_store", 512, 256)
    assert plan("particle", A, M, n) == ("direct_store", 128, 64)
    assert plan("particle", M, Q32, n) == ("direct_store", 512, 128)


def test_tile_modes():
    """The tile mode the planner takes: a destination in 16-byte granules of
    one leaf stores from registers; a record-major destination in 4-byte
    words gathers word by word from the staged source (each word read as the
    pieces of it that are one 4-byte window of the source, at most 1.45 reads
    per word on average); a source in granules of one leaf loads into
    registers; anything else stages both sides.  LLAMA_COPY_NO_DIRECT stages every tile, and a destination whose
    padding is kept never gathers."""
    def plan(name, a, b, n=1 << 20, **kw):
        r = L.Record(W.RECORDS[name])
        return L.plan(L.Mapping(r, a[0], [n], a[1]), L.Mapping(r, b[0], [n], b[1]), **kw)

    def mode(*args, **kw):
        return plan(*args, **kw)["tile_mode"]
    A, AA, S, M = ("aos_packed", 0), ("aos_aligned", 0), ("soa_single", 0), ("soa_multi", 0)
    Q8, Q32 = ("aosoa", 8), ("aosoa", 32)
    # particle, 4-byte leaves: AoSoA32 lane runs are 128 bytes (one cache
    # line), AoSoA8 runs 32 bytes
    assert mode("particle", A, S) == "direct_store"
    assert mode("particle", A, Q32) == "direct_store"
    assert mode("particle", A, Q8) == "gather_store"
    assert mode("particle", Q8, AA) == "gather_store"
    assert mode("particle", S, A) == "gather_store"
    # lbm: 8-byte leaves and a 4-byte flag word in a 160-byte aligned cell
    assert mode("lbm", M, AA) == "gather_store"
    assert mode("lbm", Q32, AA) == "gather_store"
    assert mode("lbm", AA, M) == "direct_store"
    # an odd record count puts single-blob SoA leaf spans off the 16-byte
    # grid (4 N f bytes in): still stored directly, the partial granules at
    # the span ends value by value
    assert mode("particle", A, S, n=1000003) == "direct_store"
    assert mode("mixed", AA, S, n=1000003) == "direct_store"
    # a u8 leaf (mixed) or u16 / bool leaves (listing1) share words with
    # other leaves or padding: those words read two or four pieces
    assert mode("mixed", M, AA) == "gather_store"
    assert mode("mixed", AA, Q8) == "gather_store"
    assert mode("listing1", M, AA) == "gather_store"
    # the 49-byte packed mixed record: 4 records are whole words.  A word
    # across two of its values is one piece where the source keeps the bytes
    # in order (AoS), so both directions between AoS and AoSoA gather; from
    # SoA or AoSoA most of its words read two pieces (1.65 reads per word):
    # SoA and AoSoA32 load directly (the u8 leaf from lane runs of 32
    # bytes), AoSoA8 (8-byte u8 runs) stages
    assert mode("mixed", AA, A) == "gather_store"
    assert mode("mixed", A, AA) == "gather_store"
    assert mode("mixed", A, Q32) == "gather_store"
    assert mode("mixed", A, Q8) == "gather_store"
    assert mode("mixed", Q8, A) == "staged"
    assert mode("mixed", Q32, A) == "direct_load"
    # from SoA the source loads into registers and each value is written into
    # the packed region in pieces of its alignment (the u8 leaf byte by byte);
    # into SoA each value is read from the aligned words that hold it
    assert mode("mixed", M, A) == "direct_load"
    assert mode("mixed", A, M) == "direct_store"
    assert mode("mixed", M, A, flags=L.COPY_NO_SPLIT) == "staged"
    assert mode("mixed", A, M, flags=L.COPY_NO_SPLIT) == "staged"
    # into AoSoA from AoS, listing 1's u16 and bool lanes make words of two
    # and four pieces (1.52 reads per word): staged; from SoA every lane run
    # is one piece: gather into AoSoA8, and into lane runs of 32 records or
    # more the source loads directly
    assert mode("listing1", AA, Q32) == "staged"
    assert mode("listing1", A, Q8) == "staged"
    assert mode("listing1", M, Q8) == "gather_store"
    assert mode("listing1", M, ("aosoa", 64)) == "direct_load"
    assert mode("mixed", M, Q32) == "direct_load"
    assert mode("mixed", M, Q32, flags=L.COPY_NO_GATHER) == "direct_load"
    assert mode("mixed", M, Q8, flags=L.COPY_NO_GATHER) == "direct_load"
    assert mode("mixed", Q32, AA, flags=L.COPY_NO_GATHER) == "direct_load"
    assert mode("mixed", Q8, AA, flags=L.COPY_NO_GATHER) == "staged"
    # LDS of a gathering tile: the source region (leaf spans of 256 records)
    # plus the word table of a 56-byte aligned record (14 word entries, padded
    # to 16: 12 whole words, the u8 word one piece with its padding, one
    # padding word)
    p = plan("mixed", M, AA)
    spans = 3 * ((256 * 8 + 30) // 16 * 16) + 6 * ((256 * 4 + 30) // 16 * 16) + (256 + 30) // 16 * 16
    assert p["tile_records"] == 256 and p["lds_bytes"] == spans + 16 * 4
    assert mode("particle", A, Q8, flags=L.COPY_NO_DIRECT) == "staged"
    assert mode("lbm", M, AA, flags=L.COPY_PRESERVE_PADDING) == "staged"
    assert mode("particle", A, Q8, n=1031, flags=L.COPY_PRESERVE_PADDING) == "staged"  # 1031 = 128 * 8 + 7
    assert mode("particle", A, Q8, flags=L.COPY_PRESERVE_PADDING) == "gather_store"  # no padding to keep
    assert plan("particle", A, S)["tile_mode"] == "direct_store"
    assert plan("particle", A, A)["tile_mode"] is None  # identical layouts: no tiles
    # nontemporal destination stores from 1 GiB of destination up: the
    # particle at 2^26 records (1.88 GB per layout), not the 128^3
    # lattice-Boltzmann grid (336 MB aligned)
    assert plan("particle", A, Q8, n=1 << 26)["stream_stores"]
    assert plan("particle", A, S, n=1 << 26)["stream_stores"]
    assert not plan("particle", A, Q8, n=(1 << 30) // 28 - 1000)["stream_stores"]
    assert plan("particle", A, Q8, n=(1 << 30) // 28 + 1000)["stream_stores"]
    assert not plan("lbm", M, AA, n=128 ** 3)["stream_stores"]
    assert not plan("particle", A, A, n=1 << 26)["stream_stores"]  # STREAM path: plain stores
    # nontemporal loads from 256 MiB of source up (the Infinity Cache): the
    # 128^3 lattice-Boltzmann grid (336 MB), not a 58 MB batch of frames
    assert plan("lbm", M, AA, n=128 ** 3)["stream_loads"]
    assert plan("particle", A, A, n=1 << 26)["stream_loads"]  # STREAM path too
    assert not plan("particle", S, Q32, n=4096 * 256)["stream_loads"]
    assert not plan("particle", A, Q8, n=(256 << 20) // 28 - 1000)["stream_loads"]
    assert plan("particle", A, Q8, n=(256 << 20) // 28 + 1000)["stream_loads"]
    # LDS of a gathering tile: the source region (512 records of 28 bytes and
    # room for the 16-byte phase) plus the word table of one destination
    # block (8 records of 28 bytes: 56 words), and no destination region
    p = plan("particle", A, Q8)
    assert p["tile_records"] == 512
    assert p["lds_bytes"] == (512 * 28 + 30) // 16 * 16 + 8 * 28


_GATHER_READS = r"""
import sys
from paper_2106_04284_amd import llama as L, workloads as W
for name, a, b in [("particle", ("aos_packed", 0), ("aosoa", 8)), ("mixed", ("soa_multi", 0), ("aos_aligned", 0)),
                   ("mixed", ("aos_packed", 0), ("aosoa", 8)), ("listing1", ("soa_multi", 0), ("aos_aligned", 0))]:
    r = L.Record(W.RECORDS[name])
    print("PAIR", name, a[0], a[1], b[0], b[1], file=sys.stderr, flush=True)
    L.plan(L.Mapping(r, a[0], [1 << 20], a[1]), L.Mapping(r, b[0], [1 << 20], b[1]))
"""


def test_gather_piece_reads():
    """The gather store's cost model, read from the plan log: every word of a
    destination super-block reads one piece, two (a word across two values
    or records) or four bytes one by one (three or four pieces).  Counted by
    hand from the layouts: AoSoA8 particles from packed AoS, 56 words of one
    piece each (each lane run's words are one value's bytes); the mixed
    record's 56-byte aligned record from SoA, 14 words of one piece (its u8
    word is one piece and three padding bytes); the mixed record's AoSoA8
    from packed AoS, 98 words of which the two u8-lane words take 4 bytes
    from 4 records (98 + 2 x 3 reads); listing 1's 32-byte aligned record
    from SoA, 8 words of which the three bools share one (8 + 3 reads)."""
    env = dict(os.environ, LLAMA_TRACE="1")
    out = subprocess.run([sys.executable, "-c", _GATHER_READS], env=env, capture_output=True, text=True,
                         cwd=os.path.dirname(os.path.dirname(os.path.abspath(__file__))), check=True).stderr
    got = re.findall(r"mode=gather_\w+ .*?words=(\d+) reads=(\d+)", out)
    assert [(int(w), int(r)) for w, r in got] == [(56, 56), (14, 14), (98, 104), (8, 11)], out


@pytest.mark.parametrize("name", ["particle", "mixed", "lbm", "listing1"])
def test_byte_accounting(orc, name):
    """The bytes a plan reports (and the benchmark counts) are the blob bytes
    the mappings span, padding included, each read or written once; the
    payload 2 N S is at most that, and equal without padding."""
    r, ro = L.Record(W.RECORDS[name]), orc.Record(W.RECORDS[name])
    n = 1031
    for a in W.LAYOUTS:
        for b in W.LAYOUTS:
            ma, mb = L.Mapping(r, a[0], [n], a[1]), L.Mapping(r, b[0], [n], b[1])
            oa, ob = orc.Mapping(ro, a[0], [n], a[1]), orc.Mapping(ro, b[0], [n], b[1])
            p = L.plan(ma, mb)
            assert p["read_bytes"] == sum(oa.blob_sizes()) and p["write_bytes"] == sum(ob.blob_sizes())
            payload = 2 * n * ro.packed_size
            pad = sum(int(m.sum()) for m in orc.padding_masks(oa)) + sum(int(m.sum()) for m in orc.padding_masks(ob))
            assert p["read_bytes"] + p["write_bytes"] == payload + pad


def test_planner_identity_and_padding():
    r = L.Record(W.MIXED)
    # identical aligned AoS with gaps: padding must be rewritten as zeros, so
    # this is not a plain memcpy
    m = L.Mapping(r, "aos_aligned", [1000])
    assert L.plan(m, L.Mapping(r, "aos_aligned", [1000]))["path"] == "tile"
    # identical AoSoA with a partial last block: runs plus zero runs
    a = L.Mapping(r, "aosoa", [1000], 64)
    p = L.plan(a, L.Mapping(r, "aosoa", [1000], 64))
    assert p["path"] == "stream" and p["runs"] > 1
    # SoA single-blob is AoSoA with N lanes (sec. 4.2): identical placement
    s = L.Mapping(r, "soa_single", [1024])
    p = L.plan(s, L.Mapping(r, "aosoa", [1024], 1024))
    assert p["path"] == "stream" and p["runs"] == 1
    # empty data space
    e = L.Mapping(r, "aos_packed", [0])
    assert L.plan(e, L.Mapping(r, "soa_multi", [0]))["path"] == "empty"


def test_forced_paths_and_options():
    r = L.Record(W.LBM)
    a = L.Mapping(r, "aos_aligned", [128, 128, 128])
    b = L.Mapping(r, "soa_multi", [128, 128, 128])
    assert L.plan(a, b)["path"] == "tile"
    assert L.plan(a, b, path="naive")["path"] == "naive"
    with pytest.raises(L.LlamaError) as e:
        L.plan(a, b, path="stream")
    assert e.value.status == L.E_UNSUPPORTED
    p = L.plan(a, b, path="tile", tile_records=64, threads=128)
    assert (p["tile_records"], p["threads"]) == (64, 128)
    for bad in ({"tile_records": 3}, {"tile_records": 8192}, {"threads": 96}, {"threads": 2048}):
        with pytest.raises(L.LlamaError) as e:
            L.plan(a, b, path="tile", **bad)
        assert e.value.status == L.E_INVALID_ARG


def _copy_status(src, sblobs, dst, dblobs):
    try:
        L.copy(src, sblobs, dst, dblobs, stream=0)
    except L.LlamaError as e:
        return e.status
    return L.OK


def test_validation_errors():
    """Every one of these fails validation, so no kernel is ever launched."""
    p, m = L.Record(W.PARTICLE), L.Record(W.MIXED)
    n = 100
    src = L.Mapping(p, "aos_packed", [n])
    dst = L.Mapping(p, "soa_multi", [n])
    sb = [(0x10000, n * 28)]
    db = [(0x100000 + k * 4096, n * 4) for k in range(7)]
    assert _copy_status(src, sb, L.Mapping(m, "soa_multi", [n]), db) == L.E_RECORD_MISMATCH
    assert _copy_status(src, sb, L.Mapping(p, "soa_multi", [n + 1]), db) == L.E_EXTENT_MISMATCH
    assert _copy_status(src, sb, L.Mapping(p, "soa_multi", [10, 10]), db) == L.E_EXTENT_MISMATCH
    assert _copy_status(src, [(0x10000, n * 28 - 1)], dst, db) == L.E_BLOB_TOO_SMALL
    assert _copy_status(src, [(0, n * 28)], dst, db) == L.E_INVALID_ARG
    overlap = list(db)
    overlap[3] = (0x10000 + 8, n * 4)
    assert _copy_status(src, sb, dst, overlap) == L.E_OVERLAP
    self_overlap = list(db)
    self_overlap[5] = (db[4][0] + 4, n * 4)
    assert _copy_status(src, sb, dst, self_overlap) == L.E_OVERLAP
    assert _copy_status(src, sb, L.Mapping(p, "aosoa", [n], 12), [(0x100000, 4096)]) == L.E_INVALID_ARG
    bad_kind = L.Mapping(p, "aos_packed", [n])
    bad_kind.desc.kind = 9
    assert _copy_status(bad_kind, sb, dst, db) == L.E_INVALID_ARG
    bad_rank = L.Mapping(p, "aos_packed", [n])
    bad_rank.desc.rank = 0
    assert _copy_status(bad_rank, sb, dst, db) == L.E_INVALID_ARG
    huge = L.Mapping(p, "aos_packed", [1 << 40, 1 << 30])
    assert _copy_status(huge, sb, L.Mapping(p, "soa_multi", [1 << 40, 1 << 30]), db) == L.E_OVERFLOW
    assert "overflows" in L.lib().llama_last_error().decode()


def test_record_descriptor_errors():
    def status(nodes):
        arr = (L.Field * max(len(nodes), 1))(*[L.Field(*x) for x in nodes])
        desc = L.RecordDesc(len(nodes), ctypes.cast(arr, ctypes.POINTER(L.Field)))
        n = ctypes.c_uint32()
        return L.lib().llama_record_info(ctypes.byref(desc), ctypes.byref(n), None, None), n.value

    assert status([(4, 4, 1, 0)]) == (L.OK, 1)
    assert status([(0, 0, 2, 2), (4, 4, 1, 0), (1, 1, 3, 0)]) == (L.OK, 8)
    assert status([])[0] == L.E_INVALID_ARG
    assert status([(4, 4, 0, 0)])[0] == L.E_INVALID_ARG         # count 0
    assert status([(4, 3, 1, 0)])[0] == L.E_INVALID_ARG         # alignment not a power of two
    assert status([(4, 4, 1, 2)])[0] == L.E_INVALID_ARG         # leaf with children
    assert status([(0, 0, 1, 0)])[0] == L.E_INVALID_ARG         # record without children
    assert status([(0, 0, 1, 3), (4, 4, 1, 0)])[0] == L.E_INVALID_ARG  # missing children


def test_empty_copy_is_a_no_op():
    r = L.Record(W.PARTICLE)
    a = L.Mapping(r, "aos_packed", [0])
    b = L.Mapping(r, "aosoa", [0], 32)
    # zero-sized blobs may be NULL; nothing is enqueued, so no GPU is needed
    assert _copy_status(a, [(0, 0)], b, [(0, 0)]) == L.OK


def test_status_strings():
    assert L.status_string(L.E_OVERLAP) == "LLAMA_E_OVERLAP"
    assert L.status_string(12345) == "LLAMA_E_UNKNOWN"


def test_tuning_cache_file_round_trip(tmp_path):
    """The tuning cache saves and loads as text; an entry whose leaf hash
    matches no record leaves plans unchanged; malformed or invalid lines are
    refused.  (Tuning itself, and its effect on plans, is tested on the GPU.)"""
    L.tune_clear()
    r = L.Record(W.PARTICLE)
    a = L.Mapping(r, "aos_packed", [1 << 20])
    b = L.Mapping(r, "soa_multi", [1 << 20])
    assert L.tune_lookup(a, b) is None
    default = L.plan(a, b)
    path = tmp_path / "tune.txt"
    L.tune_save(str(path))
    assert [ln for ln in path.read_text().splitlines() if not ln.startswith("#")] == []
    probe = tmp_path / "probe.txt"
    probe.write_text("0 0 0 3 0 20 2 64 192 0 1 1.0\n")
    assert L.tune_load(str(probe)) == 1
    L.tune_save(str(path))
    assert "0 0 0 3 0 20 2 64 192 0 1 1" in path.read_text()
    assert L.plan(a, b) == default and L.tune_lookup(a, b) is None
    L.tune_clear()
    for bad in ("garbage\n", "0 0 0 3 0 20 2 63 192 0 0 1.0\n", "0 0 0 3 0 20 2 64 100 0 0 1.0\n",
                "0 0 0 3 0 20 9 64 192 0 0 1.0\n", "0 0 0 3 0 20 2 64 192 0 4 1.0\n",
                "0 0 0 3 0 20 2 64 192 0 1.0\n"):
        probe.write_text(bad)
        with pytest.raises(L.LlamaError):
            L.tune_load(str(probe))
    with pytest.raises(L.LlamaError):
        L.tune_load(str(tmp_path / "missing.txt"))


def test_build_refuses_kernels_with_scratch():
    """A kernel that spills to scratch memory runs many times slower: the
    build parses hipcc's resource remarks and the device assembly, and
    refuses a kernel with a private segment that its code loads or stores; a
    reserved slot that no instruction touches is accepted."""
    from paper_2106_04284_amd import build as B
    ok = ("k.hip:1:1: remark: Function Name: _Zgood [-Rpass-analysis=kernel-resource-usage]\n"
          "k.hip:1:1: remark:     ScratchSize [bytes/lane]: 0 [-Rpass-analysis=kernel-resource-usage]\n")
    asm = "_Zgood:\n\tglobal_load_dword v0, v[0:1], off\n\ts_endpgm\n"
    B._check_no_scratch(ok, asm)
    slot = ok + ("k.hip:3:1: remark: Function Name: _Zslot [-Rpass-analysis=kernel-resource-usage]\n"
                 "k.hip:3:1: remark:     ScratchSize [bytes/lane]: 36 [-Rpass-analysis=kernel-resource-usage]\n")
    B._check_no_scratch(slot, asm + "_Zslot:\n\tv_writelane_b32 v1, s4, 0\n\ts_endpgm\n")
    bad = ok + ("k.hip:2:1: remark: Function Name: _Zspills [-Rpass-analysis=kernel-resource-usage]\n"
                "k.hip:2:1: remark:     ScratchSize [bytes/lane]: 3960 [-Rpass-analysis=kernel-resource-usage]\n")
    with pytest.raises(RuntimeError, match="_Zspills: 3960"):
        B._check_no_scratch(bad, asm + "_Zspills:\n\tscratch_store_dword off, v3, s0 offset:16\n\ts_endpgm\n")
    with pytest.raises(RuntimeError, match="_Zspills: 3960"):  # no assembly for it: refused
        B._check_no_scratch(bad, asm)


def test_split_mapping_host(orc):
    """Split mappings (sec. 3.7) through the C ABI: blob counts, sizes and
    every offset equal the oracle's; malformed splits are rejected; plans,
    batches and tuning take plain mappings only."""
    import random
    rng = random.Random(5)
    plain = [("aos_packed", 0), ("aos_aligned", 0), ("soa_single", 0), ("soa_multi", 0), ("aosoa", 4), ("aosoa", 32)]
    for name in ("particle", "mixed", "listing1", "lbm"):
        rec = W.RECORDS[name]
        rg, ro = L.Record(rec), orc.Record(rec)
        F = ro.nleaves
        for first, count in [(0, 1), (0, F - 1), (1, F - 1), (F // 2, 1)]:
            for _ in range(3):
                sp = (first, count, rng.choice(plain), rng.choice(plain))
                for ext in ([1], [45], [3, 5]):
                    m = L.Mapping(rg, "split", ext, split=sp)
                    o = orc.Mapping(ro, "split", ext, split=sp)
                    assert m.blob_sizes() == o.blob_sizes(), (name, sp, ext)
                    n = int(np.prod(ext))
                    for i in sorted({0, n // 2, n - 1}):
                        coord = list(np.unravel_index(i, ext))
                        for f in range(F):
                            assert m.offset(coord, f) == o.blob_nr_and_offset(coord, f), (name, sp, ext, i, f)
    rg = L.Record(W.PARTICLE)
    ok = ("soa_multi", 0), ("aos_packed", 0)
    for bad in [(0, 7, *ok), (5, 3, *ok), (0, 0, *ok), (1, 2, (8, 0), ok[1]), (1, 2, ("aosoa", 3), ok[1]),
                (1, 2, ("soa_aligned", 3), ok[1]),
                (1, 2, ("split", (0, 2, *ok)), ok[1])]:
        with pytest.raises(L.LlamaError) as e:
            L.Mapping(rg, "split", [10], split=bad).blob_sizes()
        assert e.value.status == L.E_INVALID_ARG
    s = L.Mapping(rg, "split", [10], split=(0, 3, *ok))
    a = L.Mapping(rg, "aos_packed", [10])
    for call in (lambda: L.plan(s, a), lambda: L.plan(a, s)):
        with pytest.raises(L.LlamaError) as e:
            call()
        assert e.value.status == L.E_UNSUPPORTED
    desc = L.MappingDesc()
    ctypes.memmove(ctypes.byref(desc), ctypes.byref(s.desc), ctypes.sizeof(desc))
    desc.split = None
    cnt = ctypes.c_uint32()
    assert L.lib().llama_mapping_blob_count(ctypes.byref(desc), ctypes.byref(cnt)) == L.E_INVALID_ARG


def test_one_mapping_host(orc):
    """One (sec. 3.7): one packed record whatever the extents, offsets equal the
    oracle's, alone and as a Split part; never a copy's destination, and a
    One source is planned element-wise."""
    for name in ("particle", "mixed"):
        rec = W.RECORDS[name]
        rg, ro = L.Record(rec), orc.Record(rec)
        F = ro.nleaves
        for ext in ([1], [33], [2, 7]):
            m, o = L.Mapping(rg, "one", ext), orc.Mapping(ro, "one", ext)
            assert m.blob_sizes() == o.blob_sizes() == [rg.info()[1]]
            sp = (F - 1, 1, ("one", 0), ("aosoa", 8))
            ms, os_ = L.Mapping(rg, "split", ext, split=sp), orc.Mapping(ro, "split", ext, split=sp)
            assert ms.blob_sizes() == os_.blob_sizes()
            n = int(np.prod(ext))
            for i in (0, n - 1):
                coord = list(np.unravel_index(i, ext))
                for f in range(F):
                    assert m.offset(coord, f) == o.blob_nr_and_offset(coord, f)
                    assert ms.offset(coord, f) == os_.blob_nr_and_offset(coord, f)
    rg = L.Record(W.PARTICLE)
    one, aos = L.Mapping(rg, "one", [10]), L.Mapping(rg, "aos_packed", [10])
    assert L.plan(one, aos)["path"] == "naive"
    with pytest.raises(L.LlamaError) as e:
        L.plan(one, aos, path="tile")
    assert e.value.status == L.E_UNSUPPORTED
    with pytest.raises(L.LlamaError) as e:
        L.plan(aos, one)
    assert e.value.status == L.E_UNSUPPORTED
    # into a One part of a Split: refused before anything is enqueued
    bufs = [ctypes.create_string_buffer(s) for s in (28 * 10, 28)]
    blob = lambda b: L.Blob(ctypes.cast(b, ctypes.c_void_p), len(b))  # noqa: E731
    dst = L.Mapping(rg, "split", [10], split=(0, 6, ("aos_packed", 0), ("one", 0)))
    src_b = (L.Blob * 1)(blob(bufs[0]))
    dst_bufs = [ctypes.create_string_buffer(s) for s in dst.blob_sizes()]
    dst_b = (L.Blob * 2)(*[blob(b) for b in dst_bufs])
    rc = L.lib().llama_copy(ctypes.byref(aos.desc), src_b, ctypes.byref(dst.desc), dst_b, None)
    assert rc == L.E_UNSUPPORTED


def test_nested_split_descriptors(orc):
    """Nested splits (sec. 3.7's mapping listing): offsets and blob sizes equal
    the oracle's; a Split part without its descriptor and a descriptor that
    contains itself are rejected."""
    rg, ro = L.Record(W.PARTICLE), orc.Record(W.PARTICLE)
    specs = [(3, 3, ("soa_multi", 0), ("split", (3, 1, ("one", 0), ("aos_aligned", 0)))),
             (0, 3, ("split", (1, 1, ("aosoa", 8), ("soa_single", 0))), ("split", (0, 2, ("aos_packed", 0), ("aosoa", 4)))),
             (6, 1, ("aos_packed", 0), ("split", (2, 3, ("soa_multi", 0),
                                                  ("split", (0, 1, ("aosoa", 32), ("aos_aligned", 0))))))]
    for sp in specs:
        for ext in ([1], [45], [3, 5]):
            m, o = L.Mapping(rg, "split", ext, split=sp), orc.Mapping(ro, "split", ext, split=sp)
            assert m.blob_sizes() == o.blob_sizes()
            n = int(np.prod(ext))
            for i in (0, n - 1):
                coord = list(np.unravel_index(i, ext))
                for f in range(7):
                    assert m.offset(coord, f) == o.blob_nr_and_offset(coord, f), (sp, ext, i, f)
    m = L.Mapping(rg, "split", [10], split=(0, 3, ("soa_multi", 0), ("split", (0, 2, ("aos_packed", 0), ("one", 0)))))
    inner = ctypes.cast(m.desc.split.contents.split[1], ctypes.c_void_p).value  # the address, not a view of the slot
    m.desc.split.contents.split[1] = ctypes.POINTER(L.SplitDesc)()  # a Split part with no descriptor
    with pytest.raises(L.LlamaError) as e:
        m.blob_sizes()
    assert e.value.status == L.E_INVALID_ARG
    m.desc.split.contents.split[1] = m.desc.split  # contains itself
    with pytest.raises(L.LlamaError) as e:
        m.blob_sizes()
    assert e.value.status == L.E_INVALID_ARG
    m.desc.split.contents.split[1] = ctypes.cast(inner, ctypes.POINTER(L.SplitDesc))
    assert m.blob_sizes() == [40, 40, 40, 80, 8]  # pos as SoA; vel.x, vel.y packed; vel.z, mass in One


def test_header_is_c99_and_matches_the_binding(tmp_path):
    """The header compiles as C99, and the binding's structures have the C
    layout: sizes and the offsets of the fields added for Split."""
    inc = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include")
    src = tmp_path / "abi.c"
    src.write_text(
        '#include <stddef.h>\n#include <stdio.h>\n#include "llama_mi355x.h"\n'
        "int main(void) {\n"
        '  printf("%zu %zu %zu %zu %zu %zu %zu\\n", sizeof(llama_mapping_desc), offsetof(llama_mapping_desc, split),\n'
        "         sizeof(llama_split_desc), offsetof(llama_split_desc, split), sizeof(llama_copy_options),\n"
        "         sizeof(llama_plan_info), sizeof(llama_copy_item));\n"
        "  return 0;\n}\n")
    exe = tmp_path / "abi"
    subprocess.check_call(["gcc", "-std=c99", "-Wall", "-Wextra", "-Werror", "-I", inc, str(src), "-o", str(exe)])
    got = [int(x) for x in subprocess.check_output([str(exe)]).split()]
    want = [ctypes.sizeof(L.MappingDesc), L.MappingDesc.split.offset, ctypes.sizeof(L.SplitDesc),
            L.SplitDesc.split.offset, ctypes.sizeof(L.CopyOptions), ctypes.sizeof(L.PlanInfo),
            ctypes.sizeof(L.CopyItem)]
    assert got == want


def test_copy_leaves_validation():
    """llama_copy_leaves rejects bad leaf maps before anything is enqueued."""
    r7, r6 = L.Record(W.PARTICLE), L.Record([["f32", "f32", "f32"], ["f32", "f32", "f32"]])
    a, b = L.Mapping(r7, "aos_packed", [10]), L.Mapping(r6, "soa_multi", [10])
    bufs = [ctypes.create_string_buffer(x) for x in a.blob_sizes() + b.blob_sizes()]
    blob = lambda x: L.Blob(ctypes.cast(x, ctypes.c_void_p), len(x))  # noqa: E731
    sb = (L.Blob * 1)(blob(bufs[0]))
    db = (L.Blob * 6)(*[blob(x) for x in bufs[1:]])

    def rc(m_src, s_b, m_dst, d_b, leaves):
        arr = (ctypes.c_uint32 * len(leaves))(*leaves)
        return L.lib().llama_copy_leaves(ctypes.byref(m_src.desc), s_b, ctypes.byref(m_dst.desc), d_b, arr, None, None)

    assert rc(a, sb, b, db, [0, 1, 2, 3, 4, 7]) == L.E_INVALID_ARG           # no source leaf 7
    assert rc(a, sb, b, db, [L.NO_LEAF] * 6) == L.E_INVALID_ARG             # nothing to copy
    rm = L.Record([["f32", "f32", "f32"], ["f32", "f32", "f64"]])
    c = L.Mapping(rm, "soa_multi", [10])
    cb = [ctypes.create_string_buffer(x) for x in c.blob_sizes()]
    cbb = (L.Blob * 6)(*[blob(x) for x in cb])
    assert rc(a, sb, c, cbb, [0, 1, 2, 3, 4, 5]) == L.E_RECORD_MISMATCH     # 4 bytes into 8
    one = L.Mapping(r6, "one", [10])
    ob = (L.Blob * 1)(blob(ctypes.create_string_buffer(24)))
    assert rc(a, sb, one, ob, list(range(6))) == L.E_UNSUPPORTED            # into One
    s = L.Mapping(r6, "split", [10], split=(0, 3, ("soa_multi", 0), ("aos_packed", 0)))
    assert rc(a, sb, s, db, list(range(6))) == L.E_UNSUPPORTED              # Split
    small = (L.Blob * 6)(*[L.Blob(ctypes.cast(x, ctypes.c_void_p), 4) for x in bufs[1:]])
    assert rc(a, sb, b, small, list(range(6))) == L.E_BLOB_TOO_SMALL
    assert rc(a, sb, b, (L.Blob * 6)(*([blob(bufs[0])] * 6)), list(range(6))) == L.E_OVERLAP


def test_plan_copy_lists_every_launch():
    """llama_plan_copy: the launches of a copy in order, without blobs.  A
    plain pair is one launch equal to llama_plan's; a Split destination part
    fed by an AoSoA32 part and SoA leaves is one tile copy with a gathered
    source (sec. 3.7), and by SoA parts one copy from a merged field-major
    side; an AoS part and 4-byte SoA leaves cannot be gathered and take a
    kept-gap tile after the first part copy; a copy between differing
    records into packed AoS that keeps a leaf takes the kept-gap tile too;
    too small a capacity is an error."""
    rg = L.Record(W.PARTICLE)
    n = 1 << 20
    aos = L.Mapping(rg, "aos_packed", [n])
    soa = L.Mapping(rg, "soa_multi", [n])
    q32 = L.Mapping(rg, "aosoa", [n], 32)
    one = L.plan_copy(aos, soa)
    assert len(one) == 1 and one[0] == L.plan(aos, soa)
    s1 = L.Mapping(rg, "split", [n], split=(0, 3, ("aosoa", 32), ("soa_multi", 0)))
    g = L.plan_copy(s1, aos)
    assert len(g) == 1 and g[0]["path"] == "tile" and g[0]["gathered_source"] and g[0]["source_chunks"] == 5
    assert not g[0]["keeps_destination"]
    assert g[0]["read_bytes"] == n * 28 and g[0]["write_bytes"] == n * 28
    # a tile smaller than the 32-record virtual block: part copies again
    small = L.plan_copy(s1, aos, tile_records=16)
    assert len(small) == 2 and not any(p["gathered_source"] for p in small) and small[1]["keeps_destination"]
    # SoA parts: one copy from one field-major side
    s3 = L.Mapping(rg, "split", [n], split=(0, 3, ("soa_multi", 0), ("soa_single", 0)))
    m = L.plan_copy(s3, aos)
    assert len(m) == 1 and not m[0]["gathered_source"] and m[0]["path"] == "tile"
    # an aligned AoS part (one-record blocks) with 4-byte SoA leaves: not gathered
    s4 = L.Mapping(rg, "split", [n], split=(0, 3, ("aos_aligned", 0), ("soa_multi", 0)))
    k = L.plan_copy(s4, aos)
    assert len(k) == 2 and not k[0]["keeps_destination"] and k[1]["keeps_destination"]
    # a Split destination fed by one source part: one copy scattering into
    # both parts; from a plain AoSoA32 source as well
    d = L.plan_copy(aos, s1)
    assert len(d) == 1 and d[0]["scattered_destination"] and d[0]["tile_mode"] == "direct_store"
    assert len(L.plan_copy(q32, s1)) == 1
    # an aligned AoS part feeding AoSoA32 positions and an SoA mass, its SoA
    # velocities feeding the SoA velocities: one scattered copy, one stream
    s2 = L.Mapping(rg, "split", [n], split=(3, 3, ("soa_multi", 0), ("aos_aligned", 0)))
    d2 = L.plan_copy(s2, s1)
    assert len(d2) == 2 and d2[0]["scattered_destination"] and d2[1]["path"] == "stream"
    assert d2[0]["read_bytes"] == n * 16
    # without direct store there is no scattered copy
    assert not any(p["scattered_destination"] for p in L.plan_copy(aos, s1, flags=L.COPY_NO_DIRECT))
    # differing records: keep the mass of a packed AoS destination
    rs = L.Record(W.PARTICLE[:2])
    lv = L.plan_copy(L.Mapping(rs, "soa_multi", [n]), aos, src_leaf=[0, 1, 2, 3, 4, 5, None])
    assert len(lv) == 1 and lv[0]["tile_mode"] == "staged" and lv[0]["keeps_destination"]
    with pytest.raises(L.LlamaError) as e:
        L.plan_copy(s1, aos, capacity=0)
    assert e.value.status == L.E_INVALID_ARG
    with pytest.raises(L.LlamaError) as e:
        L.plan_copy(s1, aos, path=L.PATH_STREAM)
    assert e.value.status == L.E_UNSUPPORTED


def test_aligned_soa_host(orc):
    """LLAMA_SOA_ALIGNED: blob sizes and every offset equal the oracle's for
    four records, alignments 1..4096 (0: 256) and ragged counts; a bad
    alignment is rejected; a copy into it whose path does not zero the padding
    (a tile copy) is followed by a zero-fill launch of one run per gap (none
    with kept padding), while a long-run copy zeroes the gaps in its own runs;
    transfers refuse it."""
    for name in ("particle", "mixed", "lbm", "listing1"):
        rec = W.RECORDS[name]
        rg, ro = L.Record(rec), orc.Record(rec)
        for n in (0, 1, 77, 1000003):
            for a in (0, 1, 2, 16, 256, 4096):
                m, o = L.Mapping(rg, "soa_aligned", [n], a), orc.Mapping(ro, "soa_aligned", [n], a)
                assert m.blob_sizes() == o.blob_sizes(), (name, n, a)
                for i in sorted({0, n // 2, n - 1}) if n else []:
                    for f in range(ro.nleaves):
                        assert m.offset([i], f) == o.blob_nr_and_offset([i], f), (name, n, a, i, f)
    rg = L.Record(W.MIXED)
    for bad in (3, 1 << 21):
        with pytest.raises(L.LlamaError) as e:
            L.Mapping(rg, "soa_aligned", [10], bad).blob_sizes()
        assert e.value.status == L.E_INVALID_ARG
    n = 1000003
    aos, q = L.Mapping(rg, "aos_packed", [n]), L.Mapping(rg, "soa_aligned", [n], 256)
    ps = L.plan_copy(aos, q)
    gaps = 9  # between the 10 sub-arrays, none of which ends on a 256-byte boundary at this count
    assert [p["path"] for p in ps] == ["tile", "stream"] and ps[1]["runs"] == gaps
    assert ps[1]["write_bytes"] == q.blob_size(0) - n * 49
    assert len(L.plan_copy(aos, q, flags=L.COPY_PRESERVE_PADDING)) == 1
    s = L.plan_copy(L.Mapping(rg, "soa_single", [n]), q)
    assert len(s) == 1 and s[0]["path"] == "stream" and s[0]["runs"] == 10 + gaps
    assert L.plan_copy(q, aos)[0]["path"] == "tile" and len(L.plan_copy(q, aos)) == 1
    # transfers refuse it (before touching any blob)
    with pytest.raises(L.LlamaError) as e:
        L.copy_transfer(aos, [(1 << 40, aos.blob_size(0))], q, [(2 << 40, q.blob_size(0))], True, stream=0)
    assert e.value.status == L.E_UNSUPPORTED
