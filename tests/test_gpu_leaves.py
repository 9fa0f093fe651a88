"""GPU parity of copies between differing records (sec. 3.9: a field missing
on one side), llama_copy_leaves against the CPU oracle byte for byte, guard
bytes included: leaves without a source keep their canary bytes."""
import random

import numpy as np
import pytest

from paper_2106_04284_amd import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

GUARD = 64
PLAIN = [("aos_packed", 0), ("aos_aligned", 0), ("soa_single", 0), ("soa_multi", 0), ("aosoa", 4),
         ("aosoa", 8), ("aosoa", 32), ("aosoa", 64)]
NO_MASS = [["f32", "f32", "f32"], ["f32", "f32", "f32"]]
RECORDS = {"particle": W.PARTICLE, "no_mass": NO_MASS, "mixed": W.MIXED, "listing1": W.RECORDS["listing1"]}


@pytest.fixture(scope="module")
def L():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2106_04284_amd import llama
    llama.lib()
    return llama


def _cases():
    g = random.Random(2021)
    pairs = [("particle", "no_mass"), ("no_mass", "particle"), ("particle", "particle"), ("mixed", "mixed"),
             ("listing1", "listing1"), ("mixed", "particle")]
    out = []
    for k in range(48):
        rs, rd = pairs[k % len(pairs)]
        out.append((rs, rd, g.choice(PLAIN if k % 8 else [("one", 0)]), g.choice(PLAIN),
                    g.choice([1, 77, 4099]), k % 5 == 4, g.randrange(1 << 30)))
    return out


def _leaf_map(orc, rs, rd, seed):
    """Per destination leaf a random source leaf of the same size, or None."""
    g = random.Random(seed)
    s, d = orc.Record(RECORDS[rs]), orc.Record(RECORDS[rd])
    out = []
    for k in range(d.nleaves):
        same = [f for f in range(s.nleaves) if s.sizes[f] == d.sizes[k]]
        out.append(g.choice(same) if same and g.random() < 0.8 else None)
    if all(x is None for x in out):
        k = next(k for k in range(d.nleaves) if any(s.sizes[f] == d.sizes[k] for f in range(s.nleaves)))
        out[k] = next(f for f in range(s.nleaves) if s.sizes[f] == d.sizes[k])
    return out


@pytest.mark.parametrize("case", _cases(), ids=lambda c: f"{c[0]}-{c[1]}-{c[2][0]}{c[2][1] or ''}-"
                                                          f"{c[3][0]}{c[3][1] or ''}-{c[4]}{'-keep' if c[5] else ''}")
def test_copy_leaves(L, orc, case):
    rs, rd, a, b, n, keep, seed = case
    leaves = _leaf_map(orc, rs, rd, seed)
    print(f"copy_leaves {case} map {leaves}", flush=True)
    ros, rod = orc.Record(RECORDS[rs]), orc.Record(RECORDS[rd])
    rgs, rgd = L.Record(RECORDS[rs]), L.Record(RECORDS[rd])
    ms_o, md_o = orc.Mapping(ros, a[0], [n], a[1]), orc.Mapping(rod, b[0], [n], b[1])
    ms, md = L.Mapping(rgs, a[0], [n], a[1]), L.Mapping(rgd, b[0], [n], b[1])
    assert ms.blob_sizes() == ms_o.blob_sizes() and md.blob_sizes() == md_o.blob_sizes()
    src = [W.random_bytes(x, seed % 1000 + j) for j, x in enumerate(ms_o.blob_sizes())]
    fill = 0xCD
    want = orc.copy_leaves(ms_o, src, md_o, [np.full(x, fill, np.uint8) for x in md_o.blob_sizes()], leaves,
                           keep_padding=keep)
    s_dev = [torch.from_numpy(x).cuda() for x in src]
    bufs = [torch.full((x + 2 * GUARD,), fill, dtype=torch.uint8, device="cuda") for x in md_o.blob_sizes()]
    L.copy_leaves(ms, s_dev, md, [t[GUARD:t.numel() - GUARD] for t in bufs], leaves,
                  flags=L.COPY_PRESERVE_PADDING if keep else 0)
    torch.cuda.synchronize()
    for k, (buf, w) in enumerate(zip(bufs, want)):
        host = buf.cpu().numpy()
        got = host[GUARD:GUARD + w.size]
        if not np.array_equal(got, w):
            bad = np.flatnonzero(got != w)
            raise AssertionError(f"blob {k}: {bad.size} bytes differ, first at {bad[0]} "
                                 f"(got {got[bad[0]]:#x}, want {w[bad[0]]:#x})")
        assert (host[:GUARD] == fill).all() and (host[GUARD + w.size:] == fill).all()


@pytest.mark.parametrize("case", [("mixed", ("soa_multi", 0), [0, None, 2, 3, None, 5, 6, 7, None, 9], False),
                                  ("mixed", ("aosoa", 8), [None, 1, 2, None, 4, 5, 6, None, 8, 9], True),
                                  ("listing1", ("soa_single", 0), [0, 1, 2, None, 4, 5, None], False),
                                  ("particle", ("aosoa", 32), [6, 5, 4, 3, 2, 1, None], False)],
                         ids=["mixed-soa_multi", "mixed-aosoa8-keep", "listing1-soa_single", "particle-reversed"])
def test_copy_leaves_into_packed_aos_in_part(L, orc, case):
    """Packed AoS written in part: the leaves without a source keep their
    bytes through a tile that stores whole regions back."""
    name, a, leaves, keep = case
    rec = W.RECORDS[name]
    for n in (1, 1000, 20011):
        print(f"copy_leaves into packed aos {case} n={n}", flush=True)
        ro, rg = orc.Record(rec), L.Record(rec)
        ms_o, md_o = orc.Mapping(ro, a[0], [n], a[1]), orc.Mapping(ro, "aos_packed", [n])
        ms, md = L.Mapping(rg, a[0], [n], a[1]), L.Mapping(rg, "aos_packed", [n])
        src = [W.random_bytes(x, n + j) for j, x in enumerate(ms_o.blob_sizes())]
        want = orc.copy_leaves(ms_o, src, md_o, [np.full(x, 0xCD, np.uint8) for x in md_o.blob_sizes()], leaves,
                               keep_padding=keep)
        buf = torch.full((md_o.blob_size(0) + 2 * GUARD,), 0xCD, dtype=torch.uint8, device="cuda")
        L.copy_leaves(ms, [torch.from_numpy(x).cuda() for x in src], md, [buf[GUARD:buf.numel() - GUARD]], leaves,
                      flags=L.COPY_PRESERVE_PADDING if keep else 0)
        torch.cuda.synchronize()
        host = buf.cpu().numpy()
        assert np.array_equal(host[GUARD:GUARD + want[0].size], want[0])
        assert (host[:GUARD] == 0xCD).all() and (host[GUARD + want[0].size:] == 0xCD).all()
