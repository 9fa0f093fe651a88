"""GPU parity of llama_copy_transfer, the host <-> device copy that changes
the layout chunk by chunk (sec. 3.9: copies between address spaces through a
small intermediate view, transfers and shuffles overlapped).  Its result must
equal the oracle's copy byte for byte, in both directions, for chunk sizes
that leave a ragged last chunk, from pinned and from pageable host memory."""
import random

import numpy as np
import pytest

from paper_2106_04284_amd import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

LAYOUTS = W.LAYOUTS + [("aosoa", 16)]


@pytest.fixture(scope="module")
def L():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2106_04284_amd import llama
    llama.lib()
    return llama


def _host(x, pinned):
    t = torch.from_numpy(x.copy())
    return t.pin_memory() if pinned else t


def _case(L, orc, name, a, b, ext, chunk, h2d, pinned, seed):
    rec = W.RECORDS[name]
    ro, rg = orc.Record(rec), L.Record(rec)
    ms_o, md_o = orc.Mapping(ro, a[0], ext, a[1]), orc.Mapping(ro, b[0], ext, b[1])
    ms, md = L.Mapping(rg, a[0], ext, a[1]), L.Mapping(rg, b[0], ext, b[1])
    src = [W.random_bytes(s, seed + j) for j, s in enumerate(ms_o.blob_sizes())]
    want = orc.copy(ms_o, src, md_o)
    if h2d:
        sb = [_host(x, pinned) for x in src]
        db = md.alloc(fill=0xCD)
    else:
        sb = [torch.from_numpy(x).cuda() for x in src]
        db = [_host(np.full(s, 0xCD, np.uint8), pinned) for s in md_o.blob_sizes()]
    stream = torch.cuda.Stream()
    stream.wait_stream(torch.cuda.current_stream())
    L.copy_transfer(ms, sb, md, db, src_on_host=h2d, chunk_bytes=chunk, stream=stream)
    stream.synchronize()
    for j, (got, w) in enumerate(zip(db, want)):
        g = got.cpu().numpy()
        if not np.array_equal(g, w):
            bad = np.flatnonzero(g != w)
            raise AssertionError(f"{name} {a}->{b} {ext} chunk {chunk} h2d={h2d} pinned={pinned}: blob {j}: "
                                 f"{bad.size} bytes differ, first at {bad[0]}")


@pytest.mark.parametrize("h2d", [True, False], ids=["h2d", "d2h"])
@pytest.mark.parametrize("name", ["particle", "mixed", "lbm"])
def test_transfer_matches_oracle(L, orc, h2d, name):
    g = random.Random(hash((h2d, name)) & 0xFFFF)
    for k in range(12):
        a, b = g.choice(LAYOUTS), g.choice(LAYOUTS)
        ext = [g.randint(1, 40000)] if k % 3 else [g.randint(1, 60), g.randint(1, 90)]
        chunk = g.choice([1, 4096, 100000, 1 << 20, 0])
        _case(L, orc, name, a, b, ext, chunk, h2d, pinned=k % 4 != 0, seed=13 * k)


def test_transfer_all_pairs_particle(L, orc):
    for a in W.LAYOUTS:
        for b in W.LAYOUTS:
            for h2d in (True, False):
                _case(L, orc, "particle", a, b, [77777], 65536, h2d, pinned=True, seed=3)


def test_transfer_in_turn(L, orc):
    """Two transfers on different streams take turns on the device's staging."""
    rec = W.RECORDS["particle"]
    ro, rg = orc.Record(rec), L.Record(rec)
    n = 300000
    ms_o, md_o = orc.Mapping(ro, "aos_packed", [n]), orc.Mapping(ro, "soa_multi", [n])
    ms, md = L.Mapping(rg, "aos_packed", [n]), L.Mapping(rg, "soa_multi", [n])
    src = [W.random_bytes(s, 5) for s in ms_o.blob_sizes()]
    want = orc.copy(ms_o, src, md_o)
    sb = [_host(x, True) for x in src]
    d1, d2 = md.alloc(fill=1), md.alloc(fill=2)
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
    L.copy_transfer(ms, sb, md, d1, src_on_host=True, chunk_bytes=1 << 20, stream=s1)
    L.copy_transfer(ms, sb, md, d2, src_on_host=True, chunk_bytes=1 << 20, stream=s2)
    torch.cuda.synchronize()
    for x, y, w in zip(d1, d2, want):
        assert np.array_equal(x.cpu().numpy(), w) and np.array_equal(y.cpu().numpy(), w)


def test_transfer_errors(L):
    rg = L.Record(W.PARTICLE)
    a, b = L.Mapping(rg, "aos_packed", [10]), L.Mapping(rg, "soa_multi", [10])
    with pytest.raises(L.LlamaError) as e:  # both on the device
        L.check(L.lib().llama_copy_transfer(L.ctypes.byref(a.desc), L._blobs(a.alloc()), 0,
                                            L.ctypes.byref(b.desc), L._blobs(b.alloc()), 0, 0,
                                            L._stream(None)))
    assert e.value.status == L.E_INVALID_ARG
    c = L.Mapping(rg, "soa_multi", [2, 5], linearizer="col")
    d = L.Mapping(rg, "aos_packed", [2, 5])
    with pytest.raises(L.LlamaError) as e:
        L.copy_transfer(d, [torch.zeros(d.blob_size(0), dtype=torch.uint8)], c, c.alloc(), src_on_host=True)
    assert e.value.status == L.E_UNSUPPORTED
    z = L.Mapping(rg, "aos_packed", [0])
    L.copy_transfer(z, [torch.zeros(1, dtype=torch.uint8)], z, [torch.zeros(1, dtype=torch.uint8).cuda()],
                    src_on_host=True)
