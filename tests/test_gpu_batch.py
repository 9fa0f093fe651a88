"""GPU parity of batched copies: one persistent launch (replayed from a
hipGraph) must leave every item's destination exactly as the oracle's copy of
that item, and exactly as a lone llama_copy of it."""
import random

import numpy as np
import pytest

from paper_2106_04284_amd import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def L():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2106_04284_amd import llama
    llama.lib()
    return llama


def make_items(L, orc, seed, count, nmax, records=("particle", "mixed"), layouts=None, keep=False):
    """Random batch items: record, size, layout pair; source bytes random, the
    oracle's expected destination computed on the host (keep: padding keeps
    the destination's 0xCD canary)."""
    g = random.Random(seed)
    layouts = layouts or (W.LAYOUTS + [("aosoa", 16)])
    items, want = [], []
    for k in range(count):
        name = g.choice(records)
        rec = W.RECORDS[name]
        n = g.randint(0, nmax) if k % 7 else g.randint(1, 3)
        a, b = g.choice(layouts), g.choice(layouts)
        ro, rg = orc.Record(rec), L.Record(rec)
        ms_o, md_o = orc.Mapping(ro, a[0], [n], a[1]), orc.Mapping(ro, b[0], [n], b[1])
        src = [W.random_bytes(s, seed * 7919 + k * 31 + j) for j, s in enumerate(ms_o.blob_sizes())]
        if keep:
            want.append(orc.copy(ms_o, src, md_o, [np.full(x, 0xCD, np.uint8) for x in md_o.blob_sizes()],
                                 keep_padding=True))
        else:
            want.append(orc.copy(ms_o, src, md_o))
        ms, md = L.Mapping(rg, a[0], [n], a[1]), L.Mapping(rg, b[0], [n], b[1])
        sd = [torch.from_numpy(x).cuda() for x in src]
        dd = md.alloc(fill=0xCD)
        items.append((ms, sd, md, dd))
    return items, want


def check(items, want):
    for k, ((_, _, _, dd), w) in enumerate(zip(items, want)):
        for j, (t, x) in enumerate(zip(dd, w)):
            got = t.cpu().numpy()
            if not np.array_equal(got, x):
                bad = np.flatnonzero(got != x)
                raise AssertionError(f"item {k} blob {j}: {bad.size} bytes differ, first at {bad[0]}")


def refill(items, value):
    for _, _, _, dd in items:
        for t in dd:
            t.fill_(value)


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_batch_matches_oracle_and_replays(L, orc, seed):
    items, want = make_items(L, orc, seed, count=40, nmax=20000)
    b = L.Batch(items)
    info = b.info()
    assert info["work_units"] > 0 and info["items"] <= len(items)
    stream = torch.cuda.Stream()
    for rep in range(3):
        refill(items, 0xCD if rep % 2 == 0 else 0x00)  # eager work between graph replays
        torch.cuda.synchronize()
        with torch.cuda.stream(stream):
            b.launch()
        stream.synchronize()
        check(items, want)
    b.close()


def test_batch_equals_lone_copies(L, orc):
    items, want = make_items(L, orc, 9, count=30, nmax=5000, records=("particle", "mixed", "lbm", "listing1"))
    lone = []
    for ms, sd, md, _ in items:
        out = md.alloc(fill=0x11)
        L.copy(ms, sd, md, out)
        lone.append(out)
    b = L.Batch(items)
    b.launch()
    torch.cuda.synchronize()
    for (_, _, _, dd), lo in zip(items, lone):
        for x, y in zip(dd, lo):
            assert torch.equal(x, y)
    check(items, want)


@pytest.mark.parametrize("opts", [dict(threads=64), dict(threads=512), dict(wg_per_cu=1), dict(wg_per_cu=5),
                                  dict(wg_per_cu=16), dict(wg_per_cu=2, tile_records=16),
                                  dict(tile_records=64, threads=128), dict(tile_records=16)])
def test_batch_options(L, orc, opts):
    items, want = make_items(L, orc, 5, count=20, nmax=8000)
    b = L.Batch(items, **opts)
    info = b.info()
    cus = torch.cuda.get_device_properties(0).multi_processor_count
    if opts.get("wg_per_cu"):  # a persistent grid of that many workgroups per compute unit
        assert info["wg_per_cu"] == opts["wg_per_cu"]
    elif info["wg_per_cu"]:  # items of several LDS classes: as many as fit LDS and wave slots
        w = min(160 * 1024 // (info["lds_bytes"] + 64), 32 // (info["threads"] // 64), 8)
        assert info["wg_per_cu"] == max(1, w)
    if info["wg_per_cu"]:
        assert info["workgroups"] == min(info["work_units"], cus * info["wg_per_cu"])
    else:  # one workgroup per work unit
        assert info["workgroups"] == info["work_units"]
    if not opts.get("tile_records"):
        assert info["lds_bytes"] <= 160 * 1024 // 5 - 64
    torch.cuda.synchronize()  # inputs were written on the default stream
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        b.launch()
        b.launch()  # a second run over the same destinations gives the same bytes
    stream.synchronize()
    check(items, want)


ONE_CLASS = [("particle", ("soa_single", 0), ("aosoa", 32)), ("particle", ("aos_packed", 0), ("aosoa", 8)),
             ("particle", ("soa_multi", 0), ("soa_single", 0)), ("mixed", ("aos_aligned", 0), ("aosoa", 64))]


@pytest.mark.parametrize("case", ONE_CLASS, ids=[f"{c[0]}-{c[1][0]}{c[1][1] or ''}-{c[2][0]}{c[2][1] or ''}"
                                                 for c in ONE_CLASS])
def test_one_class_batch_runs_one_workgroup_per_unit(L, orc, case):
    """Items of one layout pair (one tile mode) run one launch, one workgroup
    per work unit; a batch with items of several tile modes sorts its table
    by mode and runs one launch per mode, and with a persistent grid
    (wg_per_cu) one launch of the dispatching kernel.  All leave the oracle's
    bytes, over graph replays."""
    name, a, b = case
    items, want = make_items_pair(L, orc, 41, 30, 5000, name, a, b)
    bt = L.Batch(items)
    info = bt.info()
    assert info["wg_per_cu"] == 0 and info["workgroups"] == info["work_units"] and info["launches"] == 1
    torch.cuda.synchronize()
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        bt.launch()
        bt.launch()
    stream.synchronize()
    check(items, want)
    # adding items of other modes: one launch per mode, or one persistent launch
    more, more_want = make_items(L, orc, 43, count=12, nmax=5000)
    mixed_batch = L.Batch(items + more)
    assert mixed_batch.info()["launches"] > 1 and mixed_batch.info()["wg_per_cu"] == 0
    persistent = L.Batch(items + more, wg_per_cu=4)
    assert persistent.info()["launches"] == 1 and persistent.info()["wg_per_cu"] == 4
    for bt2, fill in ((mixed_batch, 0x11), (persistent, 0x22), (mixed_batch, 0x33)):
        refill(items + more, fill)
        torch.cuda.synchronize()
        with torch.cuda.stream(stream):
            bt2.launch()
        stream.synchronize()
        check(items + more, want + more_want)


def make_items_pair(L, orc, seed, count, nmax, name, a, b):
    """Items of one record and one layout pair, random sizes (at least 100
    records, so that every item is tiled the same way)."""
    g = random.Random(seed)
    rec = W.RECORDS[name]
    items, want = [], []
    for k in range(count):
        n = g.randint(100, nmax)
        ro, rg = orc.Record(rec), L.Record(rec)
        ms_o, md_o = orc.Mapping(ro, a[0], [n], a[1]), orc.Mapping(ro, b[0], [n], b[1])
        src = [W.random_bytes(s, seed * 7919 + k * 31 + j) for j, s in enumerate(ms_o.blob_sizes())]
        want.append(orc.copy(ms_o, src, md_o))
        ms, md = L.Mapping(rg, a[0], [n], a[1]), L.Mapping(rg, b[0], [n], b[1])
        items.append((ms, [torch.from_numpy(x).cuda() for x in src], md, md.alloc(fill=0xCD)))
    return items, want


def test_one_shot_batch_and_null_stream(L, orc):
    items, want = make_items(L, orc, 12, count=25, nmax=3000)
    L.copy_batch(items)
    torch.cuda.synchronize()
    check(items, want)
    refill(items, 0x5A)
    b = L.Batch(items)
    b.launch(stream=0)  # the null stream is not captured; the kernel is launched directly
    torch.cuda.synchronize()
    check(items, want)


def test_batch_preserve_padding(L, orc):
    """LLAMA_COPY_PRESERVE_PADDING in a batch: padding keeps its canary in
    tiled items and in long-run items (AoSoA tail lanes)."""
    items, want = make_items(L, orc, 17, count=30, nmax=5000, records=("particle", "mixed", "lbm"), keep=True)
    b = L.Batch(items, flags=L.COPY_PRESERVE_PADDING)
    torch.cuda.synchronize()
    b.launch()
    torch.cuda.synchronize()
    check(items, want)


def test_batch_rejects_overlap(L):
    r = L.Record(W.PARTICLE)
    a, s = L.Mapping(r, "aos_packed", [1000]), L.Mapping(r, "soa_single", [1000])
    src = torch.empty(28000, dtype=torch.uint8, device="cuda")
    dst = torch.empty(28000 * 2, dtype=torch.uint8, device="cuda")
    with pytest.raises(L.LlamaError) as e:
        L.Batch([(a, [src], s, [dst[:28000]]), (a, [src], s, [dst[100:28100]])])
    assert e.value.status == L.E_OVERLAP
    with pytest.raises(L.LlamaError) as e:
        L.Batch([(a, [src], s, [dst[:28000]]), (a, [dst[:28000]], s, [dst[28000:]])])
    assert e.value.status == L.E_OVERLAP


def test_autotune_caches_a_bit_exact_plan(L, orc, tmp_path):
    """Autotuning picks a plan, every candidate having matched the default
    plan's bytes; later default copies of the class use it and stay exact."""
    L.tune_clear()
    rg = L.Record(W.MIXED)
    n = 150000
    a, b = L.Mapping(rg, "aos_aligned", [n]), L.Mapping(rg, "aosoa", [n], 32)
    ro = orc.Record(W.MIXED)
    src = [W.random_bytes(s, 77) for s in orc.Mapping(ro, "aos_aligned", [n]).blob_sizes()]
    expect = orc.copy(orc.Mapping(ro, "aos_aligned", [n]), src, orc.Mapping(ro, "aosoa", [n], 32))
    sd = [torch.from_numpy(x).cuda() for x in src]
    dd = b.alloc(fill=0)
    best, gbs = L.autotune(a, sd, b, dd)
    assert gbs > 0 and best["path"] in ("tile", "stream")
    assert L.tune_lookup(a, b) == best
    p = L.plan(a, b)
    if best["path"] == "tile":
        assert (p["tile_records"], p["threads"]) == (best["tile_records"], best["threads"])
    for t in dd:
        t.fill_(0xEE)
    L.copy(a, sd, b, dd)
    torch.cuda.synchronize()
    assert np.array_equal(dd[0].cpu().numpy(), expect[0])
    path = str(tmp_path / "tune.txt")
    L.tune_save(path)
    L.tune_clear()
    assert L.tune_lookup(a, b) is None
    assert L.tune_load(path) == 1 and L.tune_lookup(a, b) == best
    L.tune_clear()


def _split_map(mod, rec, layout, n):
    if layout[0] == "split":
        return mod.Mapping(rec, "split", [n], split=layout[1])
    return mod.Mapping(rec, layout[0], [n], layout[1])


def test_batch_with_split_items(L, orc):
    """Items with a Split side (sec. 3.7) run as their part copies, side by
    side with plain items, over two graph replays; an item whose part copies
    would write parts of the records of a record-major destination part in
    turn is refused."""
    g = random.Random(44)
    s1 = ("split", (0, 3, ("aosoa", 32), ("soa_multi", 0)))
    s2 = ("split", (3, 3, ("soa_multi", 0), ("aos_aligned", 0)))
    s3 = ("split", (0, 3, ("aos_packed", 0), ("aosoa", 8)))
    pairs = [(("aos_packed", 0), s1), (s1, ("soa_multi", 0)), (s2, ("soa_single", 0)), (s1, s3), (s3, s1),
             (("aosoa", 64), s2), (("aos_aligned", 0), ("aosoa", 16))]
    ro, rg = orc.Record(W.PARTICLE), L.Record(W.PARTICLE)
    items, want = [], []
    for k in range(21):
        a, b = pairs[k % len(pairs)]
        n = g.choice([1, 77, 4099, 30011])
        ms_o, md_o = _split_map(orc, ro, a, n), _split_map(orc, ro, b, n)
        src = [W.random_bytes(x, 500 + k * 13 + j) for j, x in enumerate(ms_o.blob_sizes())]
        want.append(orc.copy(ms_o, src, md_o))
        ms, md = _split_map(L, rg, a, n), _split_map(L, rg, b, n)
        items.append((ms, [torch.from_numpy(x).cuda() for x in src], md, md.alloc(fill=0xCD)))
    print("split batch: 21 items", flush=True)
    b = L.Batch(items)
    for rep in range(2):
        refill(items, 0xCD if rep == 0 else 0x00)
        torch.cuda.synchronize()
        b.launch()
        torch.cuda.synchronize()
        check(items, want)
    b.close()
    # into packed AoS from both parts of s1: the part copies depend on their order
    n = 100
    ms, md = _split_map(L, rg, s1, n), L.Mapping(rg, "aos_packed", [n])
    bad = [(ms, [t.cuda() for t in (torch.zeros(x, dtype=torch.uint8) for x in ms.blob_sizes())], md, md.alloc())]
    with pytest.raises(L.LlamaError) as e:
        L.Batch(bad)
    assert e.value.status == L.E_UNSUPPORTED


def test_batch_with_aligned_soa_items(L, orc):
    """Items into and out of SoA with aligned sub-arrays: a tiled item's zero
    fill of the padding between sub-arrays joins the batch as an item of its
    own; over two graph replays the destinations equal the oracle's, padding
    zero."""
    g = random.Random(46)
    lay = [("aos_packed", 0), ("aos_aligned", 0), ("soa_multi", 0), ("aosoa", 32), ("soa_aligned", 64),
           ("soa_aligned", 0)]
    items, want = [], []
    for k in range(18):
        name = g.choice(["particle", "mixed"])
        a, b = g.choice(lay), g.choice(lay)
        if a[0] != "soa_aligned" and b[0] != "soa_aligned":
            b = ("soa_aligned", 256)
        n = g.choice([1, 77, 4099, 30011])
        ro, rg = orc.Record(W.RECORDS[name]), L.Record(W.RECORDS[name])
        ms_o, md_o = orc.Mapping(ro, a[0], [n], a[1]), orc.Mapping(ro, b[0], [n], b[1])
        src = [W.random_bytes(x, 700 + k * 13 + j) for j, x in enumerate(ms_o.blob_sizes())]
        want.append(orc.copy(ms_o, src, md_o))
        ms, md = L.Mapping(rg, a[0], [n], a[1]), L.Mapping(rg, b[0], [n], b[1])
        items.append((ms, [torch.from_numpy(x).cuda() for x in src], md, md.alloc(fill=0xCD)))
    print("aligned soa batch: 18 items", flush=True)
    b = L.Batch(items)
    for rep in range(2):
        refill(items, 0xCD if rep == 0 else 0x77)
        torch.cuda.synchronize()
        b.launch()
        torch.cuda.synchronize()
        check(items, want)
    b.close()


def test_batch_autotune_keeps_result(L, orc):
    """llama_batch_autotune re-plans the batch (LDS budget, threads, grid);
    every candidate must write the same bytes, and the tuned batch, replayed
    from its graph, still equals the oracle."""
    items, want = make_items(L, orc, 41, count=25, nmax=30000)
    b = L.Batch(items)
    gbs = b.autotune(reps=1)
    assert gbs > 0
    info = b.info()
    assert info["threads"] in (128, 256, 512)
    check(items, want)
    stream = torch.cuda.Stream()
    for rep in range(2):
        refill(items, 0x33 + rep)
        torch.cuda.synchronize()
        with torch.cuda.stream(stream):
            b.launch()
        stream.synchronize()
        check(items, want)
    b.close()

