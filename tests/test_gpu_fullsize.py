"""Parity at the benchmark's full sizes, in the launch configuration bench.py
times (default plans; the batch with the benchmark's thread counts).

  * particle record, 2^26 records, every ordered layout pair: the oracle builds
    all seven layouts from the benchmark's raw 32-bit values (NaN payloads,
    -0, subnormals and infinities planted); each is uploaded and copied into
    every other layout, whose every byte must equal the oracle's layout;
  * lattice-Boltzmann cells, 128^3, aligned AoS <-> multi-blob SoA <-> AoSoA32:
    the whole destination against the oracle's full copy;
  * the 1,000-array batch: the two launches (graph capture, replay) agree
    byte for byte, and every item's destination equals the oracle's copy in
    full.
"""

import numpy as np
import pytest

from paper_2106_04284_amd import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

PAIRS = [(a, b) for a in W.LAYOUTS for b in W.LAYOUTS if a != b]


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


def _random_blob(nbytes, seed, plant=True):
    g = torch.Generator(device="cuda")
    g.manual_seed(seed)
    t = torch.randint(0, 256, (nbytes,), dtype=torch.uint8, device="cuda", generator=g)
    if plant and nbytes >= 4 * 4096:
        # special 32-bit patterns at fixed word offsets (the particle's values
        # are 4-byte words in every layout)
        words = t[: nbytes // 4 * 4].view(torch.int32)
        special = torch.from_numpy(W.SPECIAL_U32.view(np.int32).copy()).cuda()
        for k in range(len(special)):
            idx = torch.arange(k, words.numel(), 1009 * (k + 1), device="cuda")
            words[idx] = special[k]
    return t


def _samples(n, nleaves, count, seed):
    g = np.random.default_rng(seed)
    idx = g.integers(0, n, size=count, dtype=np.uint64)
    idx[:16] = np.arange(16, dtype=np.uint64)  # the first and last records
    idx[16:32] = np.arange(n - 16, n, dtype=np.uint64)
    leaf = g.integers(0, nleaves, size=count, dtype=np.int32)
    return idx, leaf


@pytest.fixture(scope="module")
def particle_2e26_layouts(L, orc):
    """The seven particle layouts at 2^26 records, each built by the oracle
    from the benchmark's raw 32-bit values (NaN payloads, -0, subnormals and
    infinities planted), then uploaded: the expected bytes of every copy."""
    n = 1 << 26
    ro = orc.Record(W.PARTICLE)
    values = W.raw_u32_values(7, n, W.BASE_SEED + 2)
    mb = orc.Mapping(ro, "soa_multi", [n])
    mb_blobs = [v.view(np.uint8).reshape(-1) for v in values]
    out = {}
    for lay in W.LAYOUTS:
        if lay == ("soa_multi", 0):
            host = mb_blobs
        else:
            host = orc.copy_threads(mb, mb_blobs, orc.Mapping(ro, lay[0], [n], lay[1]))
        out[lay] = [torch.from_numpy(h).cuda() for h in host]
        del host
    del values, mb_blobs
    torch.cuda.synchronize()
    return n, out


@pytest.mark.parametrize("src", W.LAYOUTS, ids=[_name(a) for a in W.LAYOUTS])
def test_particle_2e26_full(L, particle_2e26_layouts, src):
    """Every destination byte of the six copies out of `src` at 2^26 records
    equals the oracle's layout (the benchmark's pairs, default plans)."""
    n, want = particle_2e26_layouts
    rg = L.Record(W.PARTICLE)
    ms = L.Mapping(rg, src[0], [n], src[1])
    bad = []
    for dst in W.LAYOUTS:
        if dst == src:
            continue
        md = L.Mapping(rg, dst[0], [n], dst[1])
        out = md.alloc(fill=0xA5)
        L.copy(ms, want[src], md, out)
        torch.cuda.synchronize()
        for k, (x, y) in enumerate(zip(out, want[dst])):
            if not torch.equal(x, y):
                diff = torch.nonzero(x != y).flatten()
                bad.append(f"{_name(src)} -> {_name(dst)} blob {k}: {diff.numel()} bytes differ, first at "
                           f"{int(diff[0])}; plan {L.plan(ms, md)}")
        del out
    assert not bad, "\n".join(bad)


# destinations of 1 GiB or more take nontemporal stores; the particle pairs
# above run them in the direct-store and gather-store modes, these cases in
# the staged mode (from AoSoA8 into the packed 49-byte mixed record, most
# words straddle two values), the direct-load mode writing that packed record
# in pieces from SoA (its u8 leaf and values at odd positions), the
# direct-store mode reading it from aligned words into SoA, the gather-store
# mode from that packed record (whole words at odd positions read
# funnel-shifted), with composite words (the mixed record's u8 leaf shares
# words with other lanes or padding) and the direct-load mode (a destination
# 4 bytes past 16-byte alignment cannot gather: a field-major source then
# loads into registers; the plan without blobs, which assumes aligned blobs,
# gathers)
STREAM_STORE_CASES = [("mixed", 1 << 25, ("aosoa", 8), ("aos_packed", 0), 0, "staged"),
                      ("mixed", 1 << 25, ("soa_multi", 0), ("aos_packed", 0), 0, "direct_load"),
                      ("mixed", 1 << 25, ("aos_packed", 0), ("soa_single", 0), 0, "direct_store"),
                      ("mixed", 1 << 25, ("aos_packed", 0), ("aosoa", 64), 0, "gather_store"),
                      ("mixed", 1 << 25, ("aosoa", 8), ("aos_aligned", 0), 0, "gather_store"),
                      ("mixed", 1 << 25, ("soa_multi", 0), ("aosoa", 32), 0, "direct_load"),
                      ("mixed", 1 << 25, ("aosoa", 32), ("aosoa", 8), 0, "gather_store"),
                      ("mixed", 1 << 25, ("aos_aligned", 0), ("aos_packed", 0), 0, "gather_store"),
                      ("particle", 1 << 26, ("soa_multi", 0), ("aos_packed", 0), 4, "gather_store")]


@pytest.mark.parametrize("case", STREAM_STORE_CASES,
                         ids=[f"{c[0]}-{_name(c[2])}-{_name(c[3])}-off{c[4]}" for c in STREAM_STORE_CASES])
def test_stream_store_modes_sampled(L, orc, case):
    name, n, a, b, off, mode = case
    ro, rg = orc.Record(W.RECORDS[name]), L.Record(W.RECORDS[name])
    ms_o, md_o = orc.Mapping(ro, a[0], [n], a[1]), orc.Mapping(ro, b[0], [n], b[1])
    ms, md = L.Mapping(rg, a[0], [n], a[1]), L.Mapping(rg, b[0], [n], b[1])
    p = L.plan(ms, md)
    assert p["path"] == "tile" and p["stream_stores"] and p["tile_mode"] == mode
    src = [_random_blob(sz, 2000 + k, plant=False) for k, sz in enumerate(ms.blob_sizes())]
    outs = []
    for fill in (0x00, 0xFF):
        views = []
        for sz in md.blob_sizes():
            buf = torch.full((sz + off + 64,), fill, dtype=torch.uint8, device="cuda")
            views.append((buf, buf[off:off + sz]))
        L.copy(ms, src, md, [v for _, v in views])
        outs.append(views)
    torch.cuda.synchronize()
    for (b0, v0), (b1, v1) in zip(*outs):
        assert torch.equal(v0, v1)  # every destination byte written
        assert (b0[:off] == 0x00).all() and (b0[off + v0.numel():] == 0x00).all()  # nothing outside
        assert (b1[:off] == 0xFF).all() and (b1[off + v1.numel():] == 0xFF).all()
    src_h = [t.cpu().numpy() for t in src]
    dst_h = [v.cpu().numpy() for _, v in outs[0]]
    idx, leaf = _samples(n, ro.nleaves, 1 << 20, 11)
    bad, first = orc.check_samples(ms_o, src_h, md_o, dst_h, idx, leaf)
    assert bad == 0, f"{bad} sampled values differ, first sample {first}"
    if b[0] not in ("soa_single", "soa_multi"):
        # padding is zero: a record-major blob of n records is n / 64 copies
        # of the structure of a 64-record blob, whose padding the oracle marks
        small = orc.Mapping(ro, b[0], [64], b[1])
        for blob, pad, sz in zip(dst_h, orc.padding_masks(small), small.blob_sizes()):
            assert not blob.reshape(-1, sz)[:, pad].any()


# the Split pairs the benchmark times (particle, 2^26 records): positions as
# AoSoA32 with velocities and mass as multi-blob SoA, and velocities as
# multi-blob SoA with positions and mass as aligned AoS
_S1 = ("split", (0, 3, ("aosoa", 32), ("soa_multi", 0)))
_S2 = ("split", (3, 3, ("soa_multi", 0), ("aos_aligned", 0)))
SPLIT_PAIRS = [(("aos_packed", 0), _S1), (_S1, ("aos_packed", 0)), (("soa_multi", 0), _S2), (_S2, ("aosoa", 32)),
               (_S1, _S2), (_S2, _S1)]


def _mk(mod, rec, layout, ext):
    if layout[0] == "split":
        return mod.Mapping(rec, "split", ext, split=layout[1])
    return mod.Mapping(rec, layout[0], ext, layout[1])


@pytest.mark.parametrize("pair", SPLIT_PAIRS, ids=["A-S1", "S1-A", "M-S2", "S2-Q32", "S1-S2", "S2-S1"])
def test_split_2e26_sampled(L, orc, pair):
    """Every destination byte written (two fills agree) and 2^20 sampled
    values equal the oracle's, at the benchmark's size."""
    n = 1 << 26
    a, b = pair
    ro, rg = orc.Record(W.PARTICLE), L.Record(W.PARTICLE)
    ms_o, md_o = _mk(orc, ro, a, [n]), _mk(orc, ro, b, [n])
    ms, md = _mk(L, rg, a, [n]), _mk(L, rg, b, [n])
    assert ms.blob_sizes() == ms_o.blob_sizes() and md.blob_sizes() == md_o.blob_sizes()
    src = [_random_blob(s, 2000 + k) for k, s in enumerate(ms.blob_sizes())]
    d0 = md.alloc(fill=0x00)
    d1 = md.alloc(fill=0xFF)
    L.copy(ms, src, md, d0)
    L.copy(ms, src, md, d1)
    torch.cuda.synchronize()
    for x, y in zip(d0, d1):
        assert torch.equal(x, y)
    src_h = [t.cpu().numpy() for t in src]
    dst_h = [t.cpu().numpy() for t in d0]
    idx, leaf = _samples(n, 7, 1 << 20, 9)
    bad, first = orc.check_samples(ms_o, src_h, md_o, dst_h, idx, leaf)
    assert bad == 0, f"{bad} sampled values differ, first sample {first}"


def test_copy_leaves_2e26_kept_mass_full(L, orc):
    """The benchmark's copy into packed AoS that keeps a leaf (the particle's
    mass has no source): the kept-gap tile path, with streaming loads and
    stores at this size.  The destination starts as random bytes; every byte
    must equal the oracle's copy_leaves of the same start (the kept mass
    included)."""
    n = 1 << 26
    no_mass = W.PARTICLE[:2]  # {pos, vel}: the particle without its mass
    rs_o, rd_o = orc.Record(no_mass), orc.Record(W.PARTICLE)
    rs, rd = L.Record(no_mass), L.Record(W.PARTICLE)
    ms_o, md_o = orc.Mapping(rs_o, "soa_multi", [n]), orc.Mapping(rd_o, "aos_packed", [n])
    ms, md = L.Mapping(rs, "soa_multi", [n]), L.Mapping(rd, "aos_packed", [n])
    frm = [0, 1, 2, 3, 4, 5, None]
    src = [_random_blob(s, 3000 + k) for k, s in enumerate(ms.blob_sizes())]
    dst = [_random_blob(s, 3100 + k) for k, s in enumerate(md.blob_sizes())]
    start = [t.cpu().numpy() for t in dst]
    L.copy_leaves(ms, src, md, dst, frm)
    torch.cuda.synchronize()
    want = orc.copy_leaves(ms_o, [t.cpu().numpy() for t in src], md_o, start, frm)
    for j, (got, w) in enumerate(zip(dst, want)):
        g = got.cpu().numpy()
        if not np.array_equal(g, w):
            bad = np.flatnonzero(g != w)
            raise AssertionError(f"blob {j}: {bad.size} bytes differ, first at {bad[0]}")


LBM_LAYOUTS = [("aos_aligned", 0), ("soa_multi", 0), ("aosoa", 32)]
LBM_PAIRS = [(a, b) for a in LBM_LAYOUTS for b in LBM_LAYOUTS if a != b]


@pytest.mark.parametrize("pair", LBM_PAIRS, ids=[f"{_name(a)}-{_name(b)}" for a, b in LBM_PAIRS])
def test_lbm_128cubed_full(L, orc, pair):
    ext = [128, 128, 128]
    a, b = pair
    ro, rg = orc.Record(W.LBM), L.Record(W.LBM)
    ms_o, md_o = orc.Mapping(ro, a[0], ext, a[1]), orc.Mapping(ro, b[0], ext, b[1])
    ms, md = L.Mapping(rg, a[0], ext, a[1]), L.Mapping(rg, b[0], ext, b[1])
    vals = W.lbm_values(128 ** 3, W.BASE_SEED + 3)
    mb = orc.Mapping(ro, "soa_multi", ext)
    src_h = orc.copy(mb, [np.ascontiguousarray(v).view(np.uint8).reshape(-1) for v in vals], ms_o)
    # the source's own padding holds random bytes, not zeros
    for blob, pad in zip(src_h, orc.padding_masks(ms_o)):
        blob[pad] = np.random.default_rng(5).integers(0, 256, int(pad.sum()), dtype=np.uint8)
    want = orc.copy(ms_o, src_h, md_o)
    src = [torch.from_numpy(x).cuda() for x in src_h]
    dst = md.alloc(fill=0xCD)
    L.copy(ms, src, md, dst)
    torch.cuda.synchronize()
    for t, w in zip(dst, want):
        assert np.array_equal(t.cpu().numpy(), w)


@pytest.mark.parametrize("threads", [128, 256])
def test_batch_1000_arrays(L, orc, threads):
    items_spec = W.batch_items()
    cache, items = {}, []
    for k, it in enumerate(items_spec):
        rg = cache.setdefault(it["record"], L.Record(W.RECORDS[it["record"]]))
        ms = L.Mapping(rg, it["src"][0], [it["n"]], it["src"][1])
        md = L.Mapping(rg, it["dst"][0], [it["n"]], it["dst"][1])
        sb = [_random_blob(s, 5000 + 3 * k + j, plant=False) for j, s in enumerate(ms.blob_sizes())]
        items.append((ms, sb, md, md.alloc(fill=0x00)))
    b = L.Batch(items, threads=threads)
    stream = torch.cuda.Stream()
    b.launch(stream)  # captured into a hipGraph and launched
    torch.cuda.synchronize()
    first = [[t.clone() for t in it[3]] for it in items]
    for it in items:
        for t in it[3]:
            t.fill_(0xFF)
    torch.cuda.synchronize()  # the fills run on the default stream, the batch on `stream`
    b.launch(stream)  # graph replay
    torch.cuda.synchronize()
    bad_items = []
    for k, (f, it) in enumerate(zip(first, items)):
        for j, (x, y) in enumerate(zip(f, it[3])):
            if not torch.equal(x, y):
                diff = torch.nonzero(x != y).flatten()
                bad_items.append(f"item {k} {items_spec[k]} blob {j}: {diff.numel()} of {x.numel()} bytes differ "
                                 f"between the runs, first at {int(diff[0])} (run 1 {int(x[diff[0]])}, run 2 "
                                 f"{int(y[diff[0]])}); plan {L.plan(it[0], it[2], threads=threads)}")
    assert not bad_items, "\n".join(bad_items[:10])
    del first
    # every item in full against the oracle's copy of its source
    mismatched = []
    for k, (it, spec) in enumerate(zip(items, items_spec)):
        ro = orc.Record(W.RECORDS[spec["record"]])
        ms_o = orc.Mapping(ro, spec["src"][0], [spec["n"]], spec["src"][1])
        md_o = orc.Mapping(ro, spec["dst"][0], [spec["n"]], spec["dst"][1])
        want = orc.copy_threads(ms_o, [t.cpu().numpy() for t in it[1]], md_o)
        for j, (t, w) in enumerate(zip(it[3], want)):
            got = t.cpu().numpy()
            if not np.array_equal(got, w):
                mismatched.append(f"item {k} {spec} blob {j}: {int((got != w).sum())} bytes differ")
    assert not mismatched, "\n".join(mismatched[:10])


BIG_PAIRS = [(("aos_packed", 0), ("soa_single", 0)), (("aosoa", 32), ("aos_aligned", 0)),
             (("soa_single", 0), ("soa_multi", 0))]


@pytest.mark.parametrize("pair", BIG_PAIRS, ids=[f"{_name(a)}-{_name(b)}" for a, b in BIG_PAIRS])
def test_particle_2e28_blobs_past_4gib(L, orc, pair):
    """Blobs of 7.5 GB (2^28 particle records): byte offsets past 2^32 in the
    tile, direct-store and stream paths; the whole destination equals the
    oracle's copy."""
    n = 1 << 28
    a, b = pair
    ro, rg = orc.Record(W.PARTICLE), L.Record(W.PARTICLE)
    ms_o, md_o = orc.Mapping(ro, a[0], [n], a[1]), orc.Mapping(ro, b[0], [n], b[1])
    ms, md = L.Mapping(rg, a[0], [n], a[1]), L.Mapping(rg, b[0], [n], b[1])
    assert max(ms.blob_sizes() + md.blob_sizes()) > (1 << 32)
    src = [_random_blob(s, 3000 + k) for k, s in enumerate(ms.blob_sizes())]
    out = md.alloc(fill=0xA5)
    L.copy(ms, src, md, out)
    torch.cuda.synchronize()
    src_h = [t.cpu().numpy() for t in src]
    del src
    want = orc.copy_threads(ms_o, src_h, md_o)
    del src_h
    for k, (t, w) in enumerate(zip(out, want)):
        got = t.cpu().numpy()
        assert np.array_equal(got, w), f"blob {k}: {int((got != w).sum())} bytes differ"
