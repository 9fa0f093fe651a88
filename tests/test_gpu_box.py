"""GPU parity of copies whose records sit at different linear indices on the
two sides, against the oracle:

 - box copies (sec. 3.2 VirtualView: a sub-box of a view at an offset; sec.
   3.9: views of different size or shape), llama_copy_box;
 - whole copies between views whose linearizers differ (row-major,
   column-major, Morton order; sec. 3.7 lists linearizers among the building
   blocks of mappings), and Morton views whose indices have holes, through
   llama_copy.

Destinations start as a canary; the oracle runs on the same canary, so bytes
outside the box must keep it.  Every comparison is byte for byte."""
import random

import numpy as np
import pytest

from paper_2106_04284_amd import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

LAYOUTS = W.LAYOUTS + [("aosoa", 4), ("aosoa", 16)]
LINS = ["row", "col", "morton"]


@pytest.fixture(scope="module")
def L():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2106_04284_amd import llama
    llama.lib()
    return llama


def _maps(L, orc, name, layout, extents, lin):
    rec = W.RECORDS[name]
    ro, rg = orc.Record(rec), L.Record(rec)
    return (orc.Mapping(ro, layout[0], extents, layout[1], linearizer=lin),
            L.Mapping(rg, layout[0], extents, layout[1], linearizer=lin))


def _check(dd, want, what):
    for j, (got, w) in enumerate(zip(dd, want)):
        g = got.cpu().numpy()
        if not np.array_equal(g, w):
            bad = np.flatnonzero(g != w)
            raise AssertionError(f"{what}: blob {j}: {bad.size} bytes differ, first at {bad[0]}")


def _box_case(L, orc, name, a, b, sext, dext, so, do, box, lin_s, lin_d, seed, **opts):
    ms_o, ms = _maps(L, orc, name, a, sext, lin_s)
    md_o, md = _maps(L, orc, name, b, dext, lin_d)
    src = [W.random_bytes(s, seed + j) for j, s in enumerate(ms_o.blob_sizes())]
    canary = [W.random_bytes(s, seed + 100 + j) for j, s in enumerate(md_o.blob_sizes())]
    keep = bool(opts.get("flags", 0) & L.COPY_PRESERVE_PADDING)
    want = orc.copy_box(ms_o, src, so, md_o, [c.copy() for c in canary], do, box, keep_padding=keep)
    sd = [torch.from_numpy(x).cuda() for x in src]
    dd = [torch.from_numpy(c.copy()).cuda() for c in canary]
    L.copy_box(ms, sd, so, md, dd, do, box, **opts)
    torch.cuda.synchronize()
    _check(dd, want, f"{name} {a}{lin_s}{sext}@{so} -> {b}{lin_d}{dext}@{do} box {box} {opts}")


def _random_box(g, rank, big=False):
    hi = {1: 9000 if big else 3000, 2: 90 if big else 60, 3: 24 if big else 18}.get(rank, 6)
    box = [g.randint(1, hi) for _ in range(rank)]
    sext = [x + g.randint(0, 9) for x in box]
    dext = [x + g.randint(0, 9) for x in box]
    so = [g.randint(0, s - x) for s, x in zip(sext, box)]
    do = [g.randint(0, d - x) for d, x in zip(dext, box)]
    return sext, dext, so, do, box


@pytest.mark.parametrize("name", ["particle", "mixed", "lbm", "listing1"])
@pytest.mark.parametrize("rank", [1, 2, 3])
def test_box_row_major(L, orc, name, rank):
    """Sub-boxes between row-major views of different extents, random layout
    pairs, offsets and ragged box extents."""
    g = random.Random(hash((name, rank)) & 0xFFFF)
    for k in range(10):
        sext, dext, so, do, box = _random_box(g, rank)
        a, b = g.choice(LAYOUTS), g.choice(LAYOUTS)
        _box_case(L, orc, name, a, b, sext, dext, so, do, box, "row", "row", 31 * k + rank)


@pytest.mark.parametrize("name", ["particle", "mixed"])
def test_box_all_layout_pairs(L, orc, name):
    """Every ordered layout pair once, 2-D boxes with odd offsets."""
    g = random.Random(5)
    for a in LAYOUTS:
        for b in LAYOUTS:
            sext, dext, so, do, box = _random_box(g, 2)
            _box_case(L, orc, name, a, b, sext, dext, so, do, box, "row", "row", 7)


@pytest.mark.parametrize("lin_s", LINS)
@pytest.mark.parametrize("lin_d", LINS)
def test_box_linearizers(L, orc, lin_s, lin_d):
    """Boxes between views of every pair of linearizers, including Morton
    offsets that do not fall on the tile grid."""
    g = random.Random(LINS.index(lin_s) * 3 + LINS.index(lin_d))
    for k in range(8):
        rank = g.choice([2, 3])
        sext, dext, so, do, box = _random_box(g, rank)
        name = g.choice(["particle", "mixed", "lbm"])
        a, b = g.choice(LAYOUTS), g.choice(LAYOUTS)
        _box_case(L, orc, name, a, b, sext, dext, so, do, box, lin_s, lin_d, 11 * k)


@pytest.mark.parametrize("opts", [dict(flags=4), dict(path="naive"), dict(tile_records=16), dict(tile_records=4096),
                                  dict(threads=64), dict(threads=1024), dict(path="box", threads=128)])
def test_box_options(L, orc, opts):
    """Kept padding, the element-wise baseline and tile and workgroup sizes
    give the same bytes."""
    g = random.Random(17)
    for k in range(8):
        rank = g.choice([1, 2, 3])
        sext, dext, so, do, box = _random_box(g, rank)
        name = g.choice(["particle", "mixed", "listing1", "lbm"])
        a, b = g.choice(LAYOUTS), g.choice([("aos_aligned", 0), ("aosoa", 8), ("soa_multi", 0), ("aos_packed", 0)])
        lin_s, lin_d = g.choice(LINS), g.choice(LINS)
        _box_case(L, orc, name, a, b, sext, dext, so, do, box, lin_s, lin_d, 3 * k, **opts)


def test_box_one_source(L, orc):
    """A One source broadcast into a box of the destination."""
    g = random.Random(2)
    for k in range(6):
        rank = g.choice([1, 2, 3])
        sext, dext, so, do, box = _random_box(g, rank)
        b = g.choice(LAYOUTS)
        _box_case(L, orc, g.choice(["particle", "mixed"]), ("one", 0), b, sext, dext, [0] * rank, do, box, "row",
                  g.choice(LINS), 9 * k)


def test_box_edges(L, orc):
    """An empty box writes nothing; a box of the whole views; a single
    record at the far corner; eight dimensions."""
    _box_case(L, orc, "particle", ("aos_packed", 0), ("soa_single", 0), [7, 9], [5, 9], [3, 0], [0, 2], [0, 7],
              "row", "row", 1)
    _box_case(L, orc, "mixed", ("aosoa", 8), ("aos_aligned", 0), [33, 17], [33, 17], [0, 0], [0, 0], [33, 17],
              "row", "col", 2)
    _box_case(L, orc, "lbm", ("soa_multi", 0), ("aosoa", 32), [40, 41], [50, 3], [39, 40], [49, 2], [1, 1],
              "morton", "row", 3)
    ext = [3, 2, 2, 3, 2, 2, 3, 2]
    _box_case(L, orc, "particle", ("aos_packed", 0), ("aosoa", 8), ext, ext, [1, 0, 1, 0, 0, 1, 1, 0],
              [0, 1, 0, 1, 1, 0, 0, 1], [2, 1, 1, 2, 1, 1, 2, 1], "row", "row", 4)
    _box_case(L, orc, "particle", ("aos_aligned", 0), ("soa_multi", 0), ext, ext, [0] * 8, [0] * 8, ext,
              "col", "morton", 5)


@pytest.mark.parametrize("lin_s", LINS)
@pytest.mark.parametrize("lin_d", LINS)
def test_full_copy_between_linearizers(L, orc, lin_s, lin_d):
    """llama_copy between views whose linearizers differ (and Morton views
    with holes in their indices): every destination byte as the oracle's
    copy, padding, holes and AoSoA lanes past the last index zero."""
    g = random.Random(100 + LINS.index(lin_s) * 3 + LINS.index(lin_d))
    for k in range(10):
        rank = g.choice([2, 2, 3])
        ext = [g.randint(1, 70 if rank == 2 else 17) for _ in range(rank)]
        name = g.choice(["particle", "mixed", "lbm", "listing1"])
        a, b = g.choice(LAYOUTS), g.choice(LAYOUTS)
        ms_o, ms = _maps(L, orc, name, a, ext, lin_s)
        md_o, md = _maps(L, orc, name, b, ext, lin_d)
        src = [W.random_bytes(s, 7 * k + j) for j, s in enumerate(ms_o.blob_sizes())]
        want = orc.copy(ms_o, src, md_o)
        sd = [torch.from_numpy(x).cuda() for x in src]
        for opts in ({}, {"path": "naive"}):
            dd = md.alloc(fill=0xCD)
            L.copy(ms, sd, md, dd, **opts)
            torch.cuda.synchronize()
            _check(dd, want, f"{name} {a}{lin_s} -> {b}{lin_d} {ext} {opts}")


def test_full_copy_keep_padding(L, orc):
    g = random.Random(8)
    for k in range(12):
        rank = g.choice([2, 3])
        ext = [g.randint(1, 40 if rank == 2 else 12) for _ in range(rank)]
        name = g.choice(["mixed", "lbm", "listing1"])
        a, b = g.choice(LAYOUTS), g.choice(LAYOUTS)
        lin_s, lin_d = g.sample(LINS, 2)
        ms_o, ms = _maps(L, orc, name, a, ext, lin_s)
        md_o, md = _maps(L, orc, name, b, ext, lin_d)
        src = [W.random_bytes(s, k + j) for j, s in enumerate(ms_o.blob_sizes())]
        canary = [W.random_bytes(s, 50 + k + j) for j, s in enumerate(md_o.blob_sizes())]
        want = orc.copy(ms_o, src, md_o, [c.copy() for c in canary], keep_padding=True)
        sd = [torch.from_numpy(x).cuda() for x in src]
        dd = [torch.from_numpy(c.copy()).cuda() for c in canary]
        L.copy(ms, sd, md, dd, flags=L.COPY_PRESERVE_PADDING)
        torch.cuda.synchronize()
        _check(dd, want, f"keep {name} {a}{lin_s} -> {b}{lin_d} {ext}")


def test_box_heatmap_exactly_once(L, orc):
    """The box kernel's Heatmap: every byte the box copy defines is written
    once (values and the gaps of the box's records), every other destination
    byte is not written, except where a kept-padding region is read and stored
    back whole."""
    g = random.Random(23)
    for k in range(16):
        rank = g.choice([1, 2, 3])
        sext, dext, so, do, box = _random_box(g, rank)
        name = g.choice(["particle", "mixed", "lbm"])
        a, b = g.choice(LAYOUTS), g.choice(LAYOUTS)
        lin_s, lin_d = g.choice(LINS), g.choice(LINS)
        ms_o, ms = _maps(L, orc, name, a, sext, lin_s)
        md_o, md = _maps(L, orc, name, b, dext, lin_d)
        src = [W.random_bytes(s, k + j) for j, s in enumerate(ms_o.blob_sizes())]
        keep = k % 4 == 3
        # the bytes the definition writes: equal after copies into two fills
        x0 = orc.copy_box(ms_o, src, so, md_o, [np.zeros(s, np.uint8) for s in md_o.blob_sizes()], do, box,
                          keep_padding=keep)
        x1 = orc.copy_box(ms_o, src, so, md_o, [np.full(s, 0xFF, np.uint8) for s in md_o.blob_sizes()], do, box,
                          keep_padding=keep)
        sd = [torch.from_numpy(x).cuda() for x in src]
        dd = md.alloc(fill=0)
        writes = [torch.zeros(s, dtype=torch.int32, device="cuda") for s in md.blob_sizes()]
        reads = [torch.zeros(s, dtype=torch.int32, device="cuda") for s in md.blob_sizes()]
        opts = {"flags": L.COPY_PRESERVE_PADDING} if keep else {}
        with L.heatmap(reads=list(zip(dd, reads)), writes=list(zip(dd, writes))):
            L.copy_box(ms, sd, so, md, dd, do, box, **opts)
        torch.cuda.synchronize()
        _check(dd, x0, f"heatmap box {name} {a}->{b}")
        for j, (w, rd, p0, p1) in enumerate(zip(writes, reads, x0, x1)):
            w, rd = w.cpu().numpy(), rd.cpu().numpy()
            defined = p0 == p1
            assert bool((w[defined] == 1).all()), f"box heatmap {name} {a}->{b} {box}: a defined byte not written once"
            other = ~defined
            assert bool((w[other] <= rd[other]).all()) and int(w[other].max(initial=0)) <= 1, \
                f"box heatmap {name} {a}->{b} {box}: a byte outside the box written"


def test_box_errors(L):
    rg = L.Record(W.PARTICLE)
    a = L.Mapping(rg, "aos_packed", [10, 10])
    b = L.Mapping(rg, "soa_multi", [8, 12])
    sa, db = a.alloc(fill=1), b.alloc(fill=0)
    with pytest.raises(L.LlamaError) as e:
        L.copy_box(a, sa, [3, 0], b, db, [0, 0], [8, 5])  # 3 + 8 > 10
    assert e.value.status == L.E_EXTENT_MISMATCH
    with pytest.raises(L.LlamaError) as e:
        L.copy_box(a, sa, [0, 0], b, db, [1, 0], [8, 5])  # 1 + 8 > 8
    assert e.value.status == L.E_EXTENT_MISMATCH
    c = L.Mapping(rg, "aos_packed", [10])
    with pytest.raises(L.LlamaError) as e:
        L.copy_box(c, c.alloc(), [0], b, db, [0], [1])
    assert e.value.status == L.E_EXTENT_MISMATCH
    one = L.Mapping(rg, "one", [8, 12])
    with pytest.raises(L.LlamaError) as e:
        L.copy_box(a, sa, [0, 0], one, one.alloc(), [0, 0], [1, 1])
    assert e.value.status == L.E_UNSUPPORTED
    with pytest.raises(L.LlamaError) as e:
        L.copy_box(a, sa, [0, 0], a, sa, [0, 0], [1, 1])
    assert e.value.status == L.E_OVERLAP
    with pytest.raises(L.LlamaError) as e:
        L.copy_box(a, sa, [0, 0], b, db, [0, 0], [2, 2], path="tile")
    assert e.value.status == L.E_INVALID_ARG
    # a whole copy between linearizers is not a batch item
    d = L.Mapping(rg, "soa_multi", [10, 10], linearizer="col")
    with pytest.raises(L.LlamaError) as e:
        L.Batch([(a, sa, d, d.alloc())])
    assert e.value.status == L.E_UNSUPPORTED
