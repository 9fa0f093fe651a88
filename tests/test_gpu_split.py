"""GPU parity of copies with a Split mapping (sec. 3.7) on either side: the
HIP copy through the C ABI against the CPU oracle, byte for byte, with the
destination's padding and the bytes around every destination blob checked.
A Split copy runs as one copy per pair of parts sharing leaves."""
import random

import numpy as np
import pytest

from paper_2106_04284_amd import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

GUARD = 64
PLAIN = [("aos_packed", 0), ("aos_aligned", 0), ("soa_single", 0), ("soa_multi", 0), ("aosoa", 4),
         ("aosoa", 8), ("aosoa", 32), ("aosoa", 64)]


@pytest.fixture(scope="module")
def L():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2106_04284_amd import llama
    llama.lib()
    return llama


def _maps(L, orc, rec, layout, extents):
    kind, arg = layout
    ro, rg = orc.Record(rec), L.Record(rec)
    if kind == "split":
        return orc.Mapping(ro, "split", extents, split=arg), L.Mapping(rg, "split", extents, split=arg)
    return orc.Mapping(ro, kind, extents, arg), L.Mapping(rg, kind, extents, arg)


def _cases():
    rng = random.Random(2106)
    out = []
    for name in ("particle", "mixed", "listing1", "lbm"):
        F = len(W.leaf_types(W.RECORDS[name]))
        ranges = sorted({(0, 1), (0, F - 1), (1, F - 1), (F // 2, 1), (1, max(1, F // 2)), (F - 1, 1)})

        def split():
            first, count = rng.choice(ranges)
            return ("split", (first, count, rng.choice(PLAIN), rng.choice(PLAIN)))

        for _ in range(10):
            n = rng.choice([1, 63, 777, 4099, 20011])
            ext = [n] if rng.random() < 0.8 else [13, 17]
            s = split()
            kind = rng.randrange(4)
            if kind == 0:
                pair = (rng.choice(PLAIN), s)
            elif kind == 1:
                pair = (s, rng.choice(PLAIN))
            elif kind == 2:  # the same selection on both sides, other inner mappings
                f, c = s[1][0], s[1][1]
                pair = (s, ("split", (f, c, rng.choice(PLAIN), rng.choice(PLAIN))))
            else:
                pair = (s, split())
            out.append((name, pair[0], pair[1], ext))
    return out


CASES = _cases()


def _id(c):
    def lay(x):
        if x[0] == "split":
            f, n, a, b = x[1]
            return f"split{f}+{n}[{a[0]}{a[1] or ''},{b[0]}{b[1] or ''}]"
        return f"{x[0]}{x[1] or ''}"
    return f"{c[0]}-{lay(c[1])}-{lay(c[2])}-{'x'.join(map(str, c[3]))}"


def _run(L, orc, rec, src_l, dst_l, extents, seed, fill=0xCD, keep=False, src_off=0, dst_off=0, **opts):
    ms_o, ms = _maps(L, orc, rec, src_l, extents)
    md_o, md = _maps(L, orc, rec, dst_l, extents)
    assert ms.blob_sizes() == ms_o.blob_sizes() and md.blob_sizes() == md_o.blob_sizes()
    src = [W.random_bytes(s, seed * 131 + k) for k, s in enumerate(ms_o.blob_sizes())]
    if keep:
        opts["flags"] = opts.get("flags", 0) | L.COPY_PRESERVE_PADDING
        want = orc.copy(ms_o, src, md_o, [np.full(s, fill, np.uint8) for s in md_o.blob_sizes()], keep_padding=True)
    else:
        want = orc.copy(ms_o, src, md_o)
    s_dev = []
    for b in src:  # each source blob at byte `src_off` of its own buffer
        sbuf = torch.empty(b.size + src_off, dtype=torch.uint8, device="cuda")
        sbuf[src_off:].copy_(torch.from_numpy(b))
        s_dev.append(sbuf[src_off:])
    bufs = []
    for s in md_o.blob_sizes():
        buf = torch.full((s + 2 * GUARD + dst_off,), fill, dtype=torch.uint8, device="cuda")
        bufs.append(buf)
    lo = GUARD + dst_off
    L.copy(ms, s_dev, md, [b[lo:b.numel() - GUARD] for b in bufs], **opts)
    torch.cuda.synchronize()
    for k, (buf, w) in enumerate(zip(bufs, want)):
        host = buf.cpu().numpy()
        got = host[lo:lo + w.size]
        if not np.array_equal(got, w):
            bad = np.flatnonzero(got != w)
            raise AssertionError(f"blob {k}: {bad.size} bytes differ, first at {bad[0]} "
                                 f"(got {got[bad[0]]:#x}, want {w[bad[0]]:#x})")
        assert (host[:lo] == fill).all() and (host[lo + w.size:] == fill).all(), \
            f"blob {k}: bytes outside the blob changed"


@pytest.mark.parametrize("case", CASES, ids=_id)
def test_split_copy(L, orc, case):
    name, src_l, dst_l, ext = case
    print(f"split case {_id(case)}", flush=True)
    _run(L, orc, W.RECORDS[name], src_l, dst_l, ext, seed=len(_id(case)))


@pytest.mark.parametrize("opts", [dict(flags=1), dict(path="naive"), dict(keep=True), dict(threads=64),
                                  dict(tile_records=16)], ids=["no_direct", "naive", "keep", "t64", "T16"])
def test_split_copy_options(L, orc, opts):
    """Options reach every part-to-part copy; the element-wise path and kept
    padding give the oracle's bytes too."""
    opts = dict(opts)
    keep = opts.pop("keep", False)
    if opts.get("path") == "naive":
        opts["path"] = L.PATH_NAIVE
    rec = W.MIXED
    a = ("split", (2, 5, ("aos_aligned", 0), ("aosoa", 8)))
    b = ("split", (0, 4, ("aosoa", 32), ("aos_aligned", 0)))
    for k, (s, d) in enumerate([(a, b), (("aos_aligned", 0), a), (b, ("aosoa", 64))]):
        print(f"split options {opts} keep={keep} pair {k}", flush=True)
        _run(L, orc, rec, s, d, [3001], seed=70 + k, keep=keep, **opts)


def test_split_copy_zero_records(L, orc):
    rg = L.Record(W.PARTICLE)
    s = L.Mapping(rg, "split", [0], split=(0, 3, ("soa_multi", 0), ("aos_aligned", 0)))
    d = L.Mapping(rg, "aosoa", [0], 8)
    L.copy(s, [torch.empty(0, dtype=torch.uint8, device="cuda")] * 5, d,
           [torch.empty(0, dtype=torch.uint8, device="cuda")])
    torch.cuda.synchronize()


AOS_FED_BY_TWO = [(name, first, count, part, dst, keep)
                  for name in ("particle", "mixed", "listing1", "lbm")
                  for first, count in ((0, 1), (1, 2))
                  for part in (("aosoa", 8), ("soa_single", 0))
                  for dst in (("aos_packed", 0), ("aos_aligned", 0), ("aosoa", 1))
                  for keep in (False, True)]


@pytest.mark.parametrize("case", AOS_FED_BY_TWO, ids=lambda c: "-".join(map(str, c)))
def test_split_into_aos_from_two_parts(L, orc, case):
    """An AoS destination fed by two source parts: the larger part copy writes
    whole records (every other byte as padding), the smaller one then writes
    its own leaves over it."""
    name, first, count, part, dst, keep = case
    src = ("split", (first, count, part, ("soa_multi", 0)))
    print(f"split into aos {case}", flush=True)
    _run(L, orc, W.RECORDS[name], src, dst, [1031], seed=first * 7 + count, keep=keep)


@pytest.mark.parametrize("offs", [(1, 0), (0, 3), (4, 8), (7, 13)], ids=lambda o: f"src{o[0]}-dst{o[1]}")
def test_split_copy_misaligned_blobs(L, orc, offs):
    """Blobs at any byte offset: every part copy plans for the addresses its
    part's blobs really have."""
    src_off, dst_off = offs
    a = ("split", (0, 3, ("aosoa", 32), ("soa_multi", 0)))
    b = ("split", (3, 3, ("soa_multi", 0), ("aos_aligned", 0)))
    for k, (s, d) in enumerate([(("aos_packed", 0), a), (a, ("aos_packed", 0)), (a, b), (b, ("aosoa", 8))]):
        print(f"split misaligned {offs} pair {k}", flush=True)
        _run(L, orc, W.PARTICLE, s, d, [5003], seed=90 + k, src_off=src_off, dst_off=dst_off)


GATHERED = [(name, split, dst, n) for name in ("particle", "mixed", "lbm")
            for split in (("split", (0, 3, ("aosoa", 32), ("soa_multi", 0))),
                          ("split", (1, 2, ("aosoa", 8), ("soa_multi", 0))),
                          ("split", (0, 1, ("aosoa", 64), ("aosoa", 64))),
                          ("split", (0, 2, ("soa_multi", 0), ("soa_single", 0))))
            for dst in (("aos_packed", 0), ("aos_aligned", 0), ("aosoa", 8), ("aosoa", 32))
            for n in (1, 31, 33, 4099)]


@pytest.mark.parametrize("case", GATHERED, ids=lambda c: f"{c[0]}-{_id(('', c[1], c[2], [c[3]]))}")
def test_split_source_gathered(L, orc, case):
    """A destination part fed by several source parts, copied by one tile
    copy whose source gathers the parts (AoSoA parts of one lane count and SoA
    leaves as chunks of a virtual block, or SoA parts as one field-major side)
    where the layouts allow it, else part by part: the oracle's bytes either
    way, at record counts below, at and past one virtual block."""
    name, split, dst, n = case
    print(f"split gathered {case}", flush=True)
    _run(L, orc, W.RECORDS[name], split, dst, [n], seed=n + 3)


@pytest.mark.parametrize("opts", [dict(flags=1), dict(keep=True), dict(threads=64), dict(tile_records=16),
                                  dict(tile_records=4096), dict(wg_per_cu=2)],
                         ids=["no_direct", "keep", "t64", "T16", "T4096", "persistent"])
def test_split_source_gathered_options(L, orc, opts):
    """Options reach the gathered copy (a tile smaller than a virtual block
    falls back to part copies); kept padding keeps the destination's gaps."""
    opts = dict(opts)
    keep = opts.pop("keep", False)
    src = ("split", (0, 3, ("aosoa", 32), ("soa_multi", 0)))
    for k, (rec, dst, n) in enumerate([(W.PARTICLE, ("aos_packed", 0), 5003), (W.MIXED, ("aos_aligned", 0), 2049),
                                       (W.LBM, ("aosoa", 16), 777)]):
        print(f"split gathered options {opts} keep={keep} case {k}", flush=True)
        _run(L, orc, rec, src, dst, [n], seed=50 + k, keep=keep, **opts)


SCATTERED = [(name, src, split, n) for name in ("particle", "mixed", "lbm")
             for src in (("aos_packed", 0), ("aos_aligned", 0), ("aosoa", 8), ("soa_single", 0),
                         ("split", (3, 3, ("soa_multi", 0), ("aos_aligned", 0))))
             for split in (("split", (0, 3, ("aosoa", 32), ("soa_multi", 0))),
                           ("split", (1, 2, ("soa_single", 0), ("aosoa", 64))),
                           ("split", (0, 2, ("soa_multi", 0), ("soa_single", 0))))
             for n in (1, 33, 4099)]


@pytest.mark.parametrize("case", SCATTERED, ids=lambda c: f"{c[0]}-{_id(('', c[1], c[2], [c[3]]))}")
def test_split_destination_scattered(L, orc, case):
    """A source part feeding several destination parts, copied by one tile
    copy whose stores scatter each leaf's granules into its own part (AoSoA
    parts of one lane count, SoA leaves), or into one field-major side (SoA
    parts), where the layouts allow it, else part by part: the oracle's
    bytes either way, AoSoA tail lanes zero and nothing past an SoA leaf's
    last record written."""
    name, src, split, n = case
    print(f"split scattered {case}", flush=True)
    _run(L, orc, W.RECORDS[name], src, split, [n], seed=n + 5)


@pytest.mark.parametrize("opts", [dict(flags=1), dict(keep=True), dict(threads=256), dict(tile_records=16),
                                  dict(tile_records=2048), dict(wg_per_cu=3)],
                         ids=["no_direct", "keep", "t256", "T16", "T2048", "persistent"])
def test_split_destination_scattered_options(L, orc, opts):
    """Options reach the scattered copy (no direct store, or a tile smaller
    than the destination's lanes, falls back to part copies)."""
    opts = dict(opts)
    keep = opts.pop("keep", False)
    dst = ("split", (0, 3, ("aosoa", 32), ("soa_multi", 0)))
    for k, (rec, src, n) in enumerate([(W.PARTICLE, ("aos_packed", 0), 5003), (W.MIXED, ("aos_aligned", 0), 2049),
                                       (W.LBM, ("split", (3, 3, ("soa_multi", 0), ("aos_aligned", 0))), 777)]):
        print(f"split scattered options {opts} keep={keep} case {k}", flush=True)
        _run(L, orc, rec, src, dst, [n], seed=60 + k, keep=keep, **opts)


ONE_CASES = [(name, dst, n) for name in ("particle", "mixed", "lbm", "listing1")
             for dst in PLAIN for n in (1, 3001)]


@pytest.mark.parametrize("case", ONE_CASES, ids=lambda c: f"{c[0]}-{c[1][0]}{c[1][1] or ''}-{c[2]}")
def test_one_broadcast_copy(L, orc, case):
    """A One source (sec. 3.7) broadcast into every plain layout."""
    name, dst, n = case
    print(f"one case {case}", flush=True)
    _run(L, orc, W.RECORDS[name], ("one", 0), dst, [n], seed=n + len(name))


@pytest.mark.parametrize("dst", [("aos_aligned", 0), ("soa_multi", 0), ("aosoa", 32),
                                 ("split", (3, 3, ("soa_multi", 0), ("aos_aligned", 0)))],
                         ids=["aos_aligned", "soa_multi", "aosoa32", "split"])
def test_split_with_one_part(L, orc, dst):
    """The particle with its mass through One and the rest as multi-blob SoA
    (a one-level form of the nested mapping in sec. 3.7's listing)."""
    src = ("split", (6, 1, ("one", 0), ("soa_multi", 0)))
    for n, ext in ((1, [1]), (4099, [4099]), (391, [17, 23])):
        print(f"split with one -> {dst} n={n}", flush=True)
        _run(L, orc, W.PARTICLE, src, dst, ext, seed=n)


# the nesting of sec. 3.7's mapping listing: velocities as multi-blob SoA, the
# rest split again into mass through One and positions as aligned AoS
LISTING_C = ("split", (3, 3, ("soa_multi", 0), ("split", (3, 1, ("one", 0), ("aos_aligned", 0)))))
NESTED_A = ("split", (0, 3, ("split", (1, 1, ("aosoa", 8), ("soa_single", 0))),
                      ("split", (0, 2, ("aos_packed", 0), ("aosoa", 4)))))
NESTED_B = ("split", (6, 1, ("aos_packed", 0), ("split", (2, 3, ("soa_multi", 0),
                                                         ("split", (0, 1, ("aosoa", 32), ("aos_aligned", 0)))))))
NESTED_PAIRS = [(LISTING_C, ("aos_packed", 0)), (LISTING_C, ("soa_multi", 0)), (LISTING_C, ("aosoa", 32)),
                (LISTING_C, NESTED_A), (("aos_aligned", 0), NESTED_A), (NESTED_A, NESTED_B), (NESTED_B, NESTED_A),
                (NESTED_B, ("aosoa", 8)), (("soa_single", 0), NESTED_B)]


@pytest.mark.parametrize("k", range(len(NESTED_PAIRS)))
def test_nested_split_copy(L, orc, k):
    src, dst = NESTED_PAIRS[k]
    for ext in ([1], [2053], [9, 31]):
        print(f"nested split pair {k} ext {ext}", flush=True)
        _run(L, orc, W.PARTICLE, src, dst, ext, seed=k * 10 + len(ext))
