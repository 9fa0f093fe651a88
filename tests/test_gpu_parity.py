"""GPU parity: the HIP copy through the C ABI against the CPU oracle, byte for
byte, on seeded inputs.

Sources hold random bytes everywhere, padding included; destinations start
filled with a canary and sit between guard bytes.  A case passes only if every
destination blob equals the oracle's (values moved, padding zero) and no byte
outside the destination blobs changed.
"""
import random

import numpy as np
import pytest

from paper_2106_04284_amd import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

GUARD = 64
L_NO_DIRECT = 1  # LLAMA_COPY_NO_DIRECT
LAYOUTS = W.LAYOUTS
PAIRS = [(a, b) for a in LAYOUTS for b in LAYOUTS]


@pytest.fixture(scope="module")
def L():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2106_04284_amd import llama
    llama.lib()
    return llama


def _name(layout):
    kind, lanes = layout
    return f"{kind}{lanes}" if kind == "aosoa" else kind


def _device_blobs(blobs, offset=0, fill=None, sizes=None):
    """Each blob as a view at byte `offset` inside a guarded device buffer."""
    views, bufs = [], []
    for k, s in enumerate(sizes if sizes is not None else [b.size for b in blobs]):
        buf = torch.empty(s + offset + GUARD, dtype=torch.uint8, device="cuda")
        buf.fill_(0xA5 if fill is None else fill)
        if blobs is not None:
            buf[offset:offset + s].copy_(torch.from_numpy(blobs[k]))
        bufs.append(buf)
        views.append(buf[offset:offset + s])
    return views, bufs


def run_case(L, orc, rec, src_layout, dst_layout, extents, seed, src_off=0, dst_off=0, fill=0xCD,
             extra_dst=0, keep=False, **opts):
    """keep: LLAMA_COPY_PRESERVE_PADDING; the destination's padding must keep
    the canary `fill` (the oracle's keep-padding copy over canary blobs)."""
    ro, rg = orc.Record(rec), L.Record(rec)
    ms_o = orc.Mapping(ro, src_layout[0], extents, src_layout[1])
    md_o = orc.Mapping(ro, dst_layout[0], extents, dst_layout[1])
    ms = L.Mapping(rg, src_layout[0], extents, src_layout[1])
    md = L.Mapping(rg, dst_layout[0], extents, dst_layout[1])
    assert ms.blob_sizes() == ms_o.blob_sizes() and md.blob_sizes() == md_o.blob_sizes()
    src = [W.random_bytes(s, seed * 131 + k) for k, s in enumerate(ms_o.blob_sizes())]
    if keep:
        opts["flags"] = opts.get("flags", 0) | L.COPY_PRESERVE_PADDING
        want = orc.copy(ms_o, src, md_o, [np.full(s, fill, np.uint8) for s in md_o.blob_sizes()],
                        keep_padding=True)
    else:
        want = orc.copy(ms_o, src, md_o)
    s_views, _ = _device_blobs(src, src_off)
    dsizes = [s + extra_dst for s in md_o.blob_sizes()]
    d_views, d_bufs = _device_blobs(None, dst_off, fill=fill, sizes=dsizes)
    L.copy(ms, s_views, md, d_views, **opts)
    torch.cuda.synchronize()
    for k, (buf, w) in enumerate(zip(d_bufs, want)):
        host = buf.cpu().numpy()
        got = host[dst_off:dst_off + w.size]
        if not np.array_equal(got, w):
            bad = np.flatnonzero(got != w)
            raise AssertionError(f"blob {k}: {bad.size} bytes differ, first at {bad[0]} "
                                 f"(got {got[bad[0]]:#x}, want {w[bad[0]]:#x})")
        untouched = np.concatenate([host[:dst_off], host[dst_off + w.size:]])
        assert (untouched == fill).all(), f"blob {k}: bytes outside the mapping's blob changed"
    return want


# --------------------------------------------------------------------------
# config 1: the n-body particle, packed AoS -> SoA single-blob -> packed AoS
# --------------------------------------------------------------------------

def test_particle_roundtrip_65536(L, orc):
    n = 65536
    vals = W.particle_values(n, W.BASE_SEED + 1)
    ro = orc.Record(W.PARTICLE)
    mb = orc.Mapping(ro, "soa_multi", [n])
    aos_o = orc.Mapping(ro, "aos_packed", [n])
    soa_o = orc.Mapping(ro, "soa_single", [n])
    aos_host = orc.copy(mb, [v.view(np.uint8) for v in vals], aos_o)
    soa_want = orc.copy(aos_o, aos_host, soa_o)
    rg = L.Record(W.PARTICLE)
    aos = L.Mapping(rg, "aos_packed", [n])
    soa = L.Mapping(rg, "soa_single", [n])
    a_dev = torch.from_numpy(aos_host[0]).cuda()
    s_dev = torch.empty(soa.blob_size(0), dtype=torch.uint8, device="cuda")
    back = torch.empty_like(a_dev)
    L.copy(aos, [a_dev], soa, [s_dev])
    L.copy(soa, [s_dev], aos, [back])
    torch.cuda.synchronize()
    assert np.array_equal(s_dev.cpu().numpy(), soa_want[0])
    assert torch.equal(back, a_dev)
    # the SoA blob is the per-field arrays one after another
    assert np.array_equal(s_dev.cpu().numpy(), np.concatenate([v.view(np.uint8) for v in vals]))


# --------------------------------------------------------------------------
# every ordered layout pair (identity included), several records and sizes
# --------------------------------------------------------------------------

@pytest.mark.parametrize("pair", PAIRS, ids=[f"{_name(a)}-{_name(b)}" for a, b in PAIRS])
@pytest.mark.parametrize("n", [1, 1000, 4099])
def test_particle_pairs(L, orc, pair, n):
    run_case(L, orc, W.PARTICLE, pair[0], pair[1], [n], seed=n)


@pytest.mark.parametrize("pair", PAIRS, ids=[f"{_name(a)}-{_name(b)}" for a, b in PAIRS])
@pytest.mark.parametrize("name", ["mixed", "lbm", "listing1"])
def test_record_pairs(L, orc, pair, name):
    run_case(L, orc, W.RECORDS[name], pair[0], pair[1], [777], seed=7)


@pytest.mark.parametrize("pair", [(("aos_packed", 0), ("soa_multi", 0)), (("aosoa", 8), ("aos_aligned", 0)),
                                  (("soa_single", 0), ("aosoa", 64)), (("aos_aligned", 0), ("aosoa", 32))])
@pytest.mark.parametrize("offsets", [(1, 0), (0, 3), (5, 7), (12, 9)])
@pytest.mark.parametrize("name", ["particle", "mixed", "listing1"])
def test_misaligned_blobs(L, orc, pair, offsets, name):
    run_case(L, orc, W.RECORDS[name], pair[0], pair[1], [1031], seed=3, src_off=offsets[0],
             dst_off=offsets[1])


@pytest.mark.parametrize("extents", [[0], [1, 0, 5], [2], [3, 5, 7], [17, 1, 13], [64, 64]])
@pytest.mark.parametrize("pair", [(("aos_aligned", 0), ("aosoa", 32)), (("soa_multi", 0), ("aos_packed", 0)),
                                  (("aosoa", 64), ("soa_single", 0)), (("aosoa", 8), ("aosoa", 64))])
def test_extents_and_empty(L, orc, extents, pair):
    run_case(L, orc, W.MIXED, pair[0], pair[1], extents, seed=11)


def test_oversized_destination_blobs_keep_their_tail(L, orc):
    run_case(L, orc, W.MIXED, ("aos_packed", 0), ("soa_multi", 0), [513], seed=5, extra_dst=100)
    run_case(L, orc, W.LBM, ("soa_multi", 0), ("aosoa", 32), [100], seed=5, extra_dst=37)


@pytest.mark.parametrize("opts", [dict(path="tile", tile_records=t, threads=th, wg_per_cu=w, flags=fl)
                                  for t in (16, 64, 256, 1024) for th in (64, 192, 1024) for w in (0, 1, 3)
                                  for fl in (0, 1)]
                         + [dict(path="naive"), dict(path="naive", threads=64)])
@pytest.mark.parametrize("pair", [(("aos_packed", 0), ("soa_single", 0)), (("aosoa", 32), ("soa_multi", 0)),
                                  (("aos_aligned", 0), ("aosoa", 8)), (("soa_multi", 0), ("soa_single", 0)),
                                  (("soa_multi", 0), ("aos_aligned", 0)), (("soa_single", 0), ("aosoa", 64))])
def test_kernel_options(L, orc, opts, pair):
    """The result is the same whatever tile, workgroup size or path is used."""
    for name, n in (("particle", 3001), ("mixed", 1500), ("lbm", 300)):
        r = L.Record(W.RECORDS[name])
        try:
            L.plan(L.Mapping(r, pair[0][0], [n], pair[0][1]), L.Mapping(r, pair[1][0], [n], pair[1][1]), **opts)
        except L.LlamaError as e:  # a tile too large for LDS is refused up front
            assert e.status == L.E_UNSUPPORTED and opts.get("tile_records", 0) >= 512
            continue
        run_case(L, orc, W.RECORDS[name], pair[0], pair[1], [n], seed=n, **opts)


@pytest.mark.parametrize("pair", PAIRS, ids=[f"{_name(a)}-{_name(b)}" for a, b in PAIRS])
@pytest.mark.parametrize("name", ["mixed", "lbm", "listing1"])
def test_preserve_padding(L, orc, pair, name):
    """LLAMA_COPY_PRESERVE_PADDING: aligned-AoS gaps and AoSoA tail lanes keep
    the destination's canary bytes, every value lands as in the default copy
    (1,031 records: a partial AoSoA block and several tiles)."""
    run_case(L, orc, W.RECORDS[name], pair[0], pair[1], [1031], seed=29, keep=True)


@pytest.mark.parametrize("opts", [dict(flags=L_NO_DIRECT), dict(path="naive"), dict(path="tile", tile_records=16),
                                  dict(path="tile", tile_records=256, threads=64, wg_per_cu=2)])
@pytest.mark.parametrize("pair", [(("soa_multi", 0), ("aos_aligned", 0)), (("aosoa", 8), ("aosoa", 64)),
                                  (("aos_packed", 0), ("aosoa", 32)), (("aosoa", 64), ("soa_single", 0)),
                                  (("aos_aligned", 0), ("aos_aligned", 0))])
def test_preserve_padding_options(L, orc, opts, pair):
    for name, n in (("mixed", 1031), ("lbm", 333), ("listing1", 77)):
        run_case(L, orc, W.RECORDS[name], pair[0], pair[1], [n], seed=n, keep=True, dst_off=3, **opts)


SPLIT_PAIRS = [(("aos_packed", 0), b) for b in LAYOUTS if b[0] != "aos_packed"] + \
              [(a, ("aos_packed", 0)) for a in LAYOUTS if a[0] != "aos_packed"]


@pytest.mark.parametrize("pair", SPLIT_PAIRS, ids=[f"{_name(a)}-{_name(b)}" for a, b in SPLIT_PAIRS])
@pytest.mark.parametrize("offsets", [(0, 0), (1, 2), (3, 1), (2, 3)])
@pytest.mark.parametrize("flags", [0, 1, 2])
@pytest.mark.parametrize("name", ["mixed", "listing1"])
def test_odd_record_sizes(L, orc, pair, offsets, flags, name):
    """Packed records of odd size (49 and 21 bytes) put 2-, 4- and 8-byte
    values at every alignment: the split move (reads assembled from aligned
    words, writes in pieces), the byte-wise move (flags 2) and the staged path
    (flags 1) give the oracle's bytes at every blob offset."""
    run_case(L, orc, W.RECORDS[name], pair[0], pair[1], [1031], seed=17, src_off=offsets[0],
             dst_off=offsets[1], flags=flags)


# record-major destinations in 4-byte words: the gather-store tile mode, over
# tile sizes, thread counts, a persistent grid (several tiles per workgroup,
# one word table), ragged record counts and source blobs at every 4-byte
# phase; destinations 16-byte aligned (dst offset 16), and at offset 4, where
# the planner falls back to the staged mode
GATHER_CASES = [("particle", ("aos_packed", 0), ("aosoa", 8)), ("particle", ("aosoa", 8), ("aos_aligned", 0)),
                ("particle", ("soa_multi", 0), ("aos_packed", 0)), ("particle", ("aosoa", 64), ("aosoa", 8)),
                ("lbm", ("soa_multi", 0), ("aos_aligned", 0)), ("lbm", ("aosoa", 32), ("aos_aligned", 0)),
                ("lbm", ("aos_aligned", 0), ("aosoa", 8)), ("lbm", ("aosoa", 64), ("aosoa", 8)),
                # 1- and 2-byte leaves: composite words assembled byte by byte
                ("mixed", ("aos_aligned", 0), ("aosoa", 8)), ("mixed", ("soa_multi", 0), ("aos_aligned", 0)),
                ("mixed", ("aosoa", 32), ("aos_aligned", 0)), ("mixed", ("soa_single", 0), ("aosoa", 8)),
                ("listing1", ("aosoa", 64), ("aos_aligned", 0)), ("listing1", ("soa_multi", 0), ("aos_aligned", 0)),
                # packed records of odd size: super-blocks of 4 records, whole
                # words at odd positions read funnel-shifted, a span that ends
                # inside a word
                ("mixed", ("aos_packed", 0), ("aos_aligned", 0)), ("mixed", ("aos_aligned", 0), ("aos_packed", 0)),
                ("listing1", ("aos_packed", 0), ("aos_aligned", 0))]
GATHER_RUNS = [(77, {}), (1031, {}), (4099, {"tile_records": 16}), (5000, {"tile_records": 64, "threads": 64}),
               (20000, {"tile_records": 256, "threads": 1024}), (30011, {"tile_records": 16, "wg_per_cu": 1})]


@pytest.mark.parametrize("case", GATHER_CASES, ids=[f"{c[0]}-{_name(c[1])}-{_name(c[2])}" for c in GATHER_CASES])
@pytest.mark.parametrize("run", GATHER_RUNS, ids=[f"n{n}-{'-'.join(f'{k}{v}' for k, v in o.items())}"
                                                  for n, o in GATHER_RUNS])
@pytest.mark.parametrize("offsets", [(0, 0), (4, 16), (8, 0), (12, 4)])
def test_gather_store(L, orc, case, run, offsets):
    name, a, b = case
    n, opts = run
    r = L.Record(W.RECORDS[name])
    assert L.plan(L.Mapping(r, a[0], [n], a[1]), L.Mapping(r, b[0], [n], b[1]), **opts)["tile_mode"] == \
        "gather_store"
    run_case(L, orc, W.RECORDS[name], a, b, [n], seed=n + offsets[0], src_off=offsets[0], dst_off=offsets[1],
             **opts)


# values aligned below their size: the direct store reads them from the
# aligned LDS words that hold them (a packed record of odd size into SoA or
# long-run AoSoA), the direct load writes them into the packed region in
# pieces (and 1- and 2-byte leaves byte or half by half), from SoA or
# long-run AoSoA
SPLIT_DIRECT_CASES = [("mixed", ("aos_packed", 0), ("soa_single", 0), "direct_store"),
                      ("mixed", ("aos_packed", 0), ("soa_multi", 0), "direct_store"),
                      ("listing1", ("aos_packed", 0), ("soa_multi", 0), "direct_store"),
                      ("mixed", ("soa_multi", 0), ("aos_packed", 0), "direct_load"),
                      ("mixed", ("soa_single", 0), ("aos_packed", 0), "direct_load"),
                      ("listing1", ("soa_multi", 0), ("aos_packed", 0), "direct_load"),
                      ("listing1", ("soa_multi", 0), ("aosoa", 32), "direct_load"),
                      ("listing1", ("soa_single", 0), ("aosoa", 64), "direct_load")]
SPLIT_DIRECT_RUNS = [(1, {}), (77, {}), (1031, {}), (4099, {"tile_records": 16}), (20000, {"threads": 1024}),
                     (30011, {"tile_records": 64, "wg_per_cu": 1})]


@pytest.mark.parametrize("case", SPLIT_DIRECT_CASES,
                         ids=[f"{c[0]}-{_name(c[1])}-{_name(c[2])}" for c in SPLIT_DIRECT_CASES])
@pytest.mark.parametrize("run", SPLIT_DIRECT_RUNS, ids=[f"n{n}-{'-'.join(f'{k}{v}' for k, v in o.items())}"
                                                        for n, o in SPLIT_DIRECT_RUNS])
@pytest.mark.parametrize("offsets", [(0, 0), (16, 32), (0, 5)])
def test_split_direct_modes(L, orc, case, run, offsets):
    name, a, b, mode = case
    n, opts = run
    r = L.Record(W.RECORDS[name])
    if offsets == (0, 0) and n % 16 == 0:  # (odd counts put single-blob SoA spans off the granule grid)
        assert L.plan(L.Mapping(r, a[0], [n], a[1]), L.Mapping(r, b[0], [n], b[1]), **opts)["tile_mode"] == mode
    run_case(L, orc, W.RECORDS[name], a, b, [n], seed=n + offsets[1], src_off=offsets[0], dst_off=offsets[1],
             **opts)


# field-major destinations whose leaf spans start off the 16-byte grid (an
# odd record count in a single-blob SoA, or a blob 4, 8 or 12 bytes in): the
# direct store writes the partial first and last granules of every span value
# by value, and must touch no byte outside the spans
PHASE_PAIRS = [(("aos_packed", 0), ("soa_single", 0)), (("aosoa", 8), ("soa_single", 0)),
               (("aos_aligned", 0), ("soa_multi", 0)), (("aosoa", 32), ("soa_multi", 0))]


@pytest.mark.parametrize("pair", PHASE_PAIRS, ids=[f"{_name(a)}-{_name(b)}" for a, b in PHASE_PAIRS])
@pytest.mark.parametrize("name", ["particle", "mixed", "lbm"])
@pytest.mark.parametrize("n", [1, 3, 17, 777, 4099])
@pytest.mark.parametrize("dst_off", [0, 4, 8, 12])
def test_direct_store_off_grid(L, orc, pair, name, n, dst_off):
    run_case(L, orc, W.RECORDS[name], pair[0], pair[1], [n], seed=n + dst_off, dst_off=dst_off)


@pytest.mark.parametrize("seed", range(24))
def test_random_records(L, orc, seed):
    g = random.Random(seed)

    def rec(depth=0):
        out = []
        for _ in range(g.randint(1, 4)):
            m = rec(depth + 1) if depth < 2 and g.random() < 0.3 else g.choice(
                ["u8", "u16", "u32", "f64", "bool", "f32", "i64"])
            if g.random() < 0.2:
                m = (m, g.randint(1, 3))
            out.append(m)
        return out

    r = rec()
    layouts = LAYOUTS + [("aosoa", 1), ("aosoa", 2), ("aosoa", 16), ("aosoa", 128)]
    for _ in range(6):
        a, b = g.choice(layouts), g.choice(layouts)
        run_case(L, orc, r, a, b, [g.randint(1, 3000)], seed=seed, src_off=g.choice([0, 0, 1, 4]),
                 dst_off=g.choice([0, 0, 2, 8]))


def test_special_float_patterns_survive(L, orc):
    """NaN payloads (signalling and quiet), -0, subnormals and infinities move
    bit for bit."""
    n = 4096
    ro, rg = orc.Record(W.PARTICLE), L.Record(W.PARTICLE)
    vals = W.raw_u32_values(7, n, W.BASE_SEED + 2)
    mb = [torch.from_numpy(v.view(np.uint8)).cuda() for v in vals]
    for a, b in [(("soa_multi", 0), ("aosoa", 32)), (("soa_multi", 0), ("aos_packed", 0))]:
        mid = L.Mapping(rg, b[0], [n], b[1]).alloc()
        L.copy(L.Mapping(rg, "soa_multi", [n]), mb, L.Mapping(rg, b[0], [n], b[1]), mid)
        back = L.Mapping(rg, "soa_multi", [n]).alloc()
        L.copy(L.Mapping(rg, b[0], [n], b[1]), mid, L.Mapping(rg, "soa_multi", [n]), back)
        torch.cuda.synchronize()
        for v, t in zip(vals, back):
            assert np.array_equal(t.cpu().numpy().view(np.uint32), v)
        for special in W.SPECIAL_U32:
            assert any((t.cpu().numpy().view(np.uint32) == special).any() for t in back)


# --------------------------------------------------------------------------
# SoA with aligned sub-arrays (the padded SoA of sec. 4.4; sec. 3.9 names
# copies between a mapping with and without that padding): against every
# other layout both ways, alignments of 16 bytes, 256 (the default) and
# 4096, record counts that leave padding between the sub-arrays, blobs at
# odd offsets, kept padding and the option sets
# --------------------------------------------------------------------------

ALIGNED = [("soa_aligned", 16), ("soa_aligned", 0), ("soa_aligned", 4096)]
ALIGNED_PAIRS = ([(a, b) for a in ALIGNED for b in LAYOUTS] + [(b, a) for a in ALIGNED for b in LAYOUTS] +
                 [(a, b) for a in ALIGNED for b in ALIGNED])


@pytest.mark.parametrize("pair", ALIGNED_PAIRS, ids=[f"{_name(a)}{a[1] if a[0] == 'soa_aligned' else ''}-"
                                                     f"{_name(b)}{b[1] if b[0] == 'soa_aligned' else ''}"
                                                     for a, b in ALIGNED_PAIRS])
@pytest.mark.parametrize("name", ["particle", "mixed", "lbm", "listing1"])
def test_aligned_soa_pairs(L, orc, pair, name):
    n = {"particle": 4099, "mixed": 777, "lbm": 301, "listing1": 1031}[name]
    print(f"aligned soa {name} {pair} n={n}", flush=True)
    run_case(L, orc, W.RECORDS[name], pair[0], pair[1], [n], seed=n + 3)


@pytest.mark.parametrize("case", [dict(keep=True), dict(flags=L_NO_DIRECT), dict(path=2, tile_records=16),
                                  dict(path=3), dict(threads=1024), dict(src_off=5, dst_off=3),
                                  dict(src_off=16, dst_off=4)],
                         ids=["keep", "no_direct", "T16", "naive", "t1024", "off5-3", "off16-4"])
def test_aligned_soa_options(L, orc, case):
    """The padding between sub-arrays is zero after every path (tile, then the
    zero-fill launch; stream runs; the element-wise kernel, then the zero
    fill), and keeps its bytes with LLAMA_COPY_PRESERVE_PADDING."""
    case = dict(case)
    offs = dict(src_off=case.pop("src_off", 0), dst_off=case.pop("dst_off", 0))
    for k, (rec, a, b, n) in enumerate([(W.MIXED, ("aos_packed", 0), ("soa_aligned", 64), 2001),
                                        (W.PARTICLE, ("soa_aligned", 256), ("aosoa", 32), 5003),
                                        (W.LBM, ("soa_multi", 0), ("soa_aligned", 4096), 333),
                                        (W.LISTING1, ("soa_aligned", 16), ("soa_aligned", 1024), 999)]):
        print(f"aligned soa options {case} {offs} pair {k}", flush=True)
        run_case(L, orc, rec, a, b, [n], seed=40 + k, **offs, **case)


def test_aligned_soa_extents_and_linearizers(L, orc):
    """Rank 3 and a column-major view: the box kernel copies the records and
    the zero fill follows it for the aligned SoA destination."""
    ro, rg = orc.Record(W.MIXED), L.Record(W.MIXED)
    ext = [7, 5, 9]
    for lin_s, lin_d in (("row", "row"), ("col", "row"), ("row", "morton")):
        ms_o = orc.Mapping(ro, "aos_aligned", ext, 0, linearizer=lin_s)
        md_o = orc.Mapping(ro, "soa_aligned", ext, 128, linearizer=lin_d)
        ms = L.Mapping(rg, "aos_aligned", ext, 0, linearizer=lin_s)
        md = L.Mapping(rg, "soa_aligned", ext, 128, linearizer=lin_d)
        src = [W.random_bytes(s, 91) for s in ms_o.blob_sizes()]
        want = orc.copy(ms_o, src, md_o)
        sd = [torch.from_numpy(x).cuda() for x in src]
        dd = md.alloc(fill=0xCD)
        L.copy(ms, sd, md, dd)
        torch.cuda.synchronize()
        for g, w in zip(dd, want):
            assert np.array_equal(g.cpu().numpy(), w), (lin_s, lin_d)
