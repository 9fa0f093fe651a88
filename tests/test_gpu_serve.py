"""GPU tests of the request server: each result is the same alone and in the
mix (byte for byte, against the oracle), admission respects the HBM budget,
and a bad request fails alone while the others complete."""
import random
import threading
import time

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


def requests(L, orc, seed, count, nmax):
    g = random.Random(seed)
    out = []
    for k in range(count):
        name = g.choice(["particle", "mixed"])
        rec = W.RECORDS[name]
        n = g.randint(1, nmax)
        a, b = g.sample(W.LAYOUTS, 2)
        ro, rg = orc.Record(rec), L.Record(rec)
        ms_o, md_o = orc.Mapping(ro, a[0], [n], a[1]), orc.Mapping(ro, b[0], [n], b[1])
        src = [W.random_bytes(s, seed * 1000 + k * 13 + j) for j, s in enumerate(ms_o.blob_sizes())]
        want = orc.copy(ms_o, src, md_o)
        ms, md = L.Mapping(rg, a[0], [n], a[1]), L.Mapping(rg, b[0], [n], b[1])
        sd = [torch.from_numpy(x).cuda() for x in src]
        dd = md.alloc(fill=0xCD)
        nbytes = sum(ms.blob_sizes()) + sum(md.blob_sizes())
        out.append({"src": ms, "sd": sd, "dst": md, "dd": dd, "want": want, "bytes": nbytes})
    return out


def check(r):
    for t, w in zip(r["dd"], r["want"]):
        assert np.array_equal(t.cpu().numpy(), w)


@pytest.mark.parametrize("policy", [0, 1, 2])
def test_mix_equals_alone(L, orc, policy):
    reqs = requests(L, orc, 3 + policy, count=60, nmax=30000)
    budget = 3 * max(r["bytes"] for r in reqs)  # forces queuing behind the budget
    srv = L.Server(budget, policy=policy)
    torch.cuda.synchronize()
    tickets = [srv.submit(r["src"], r["sd"], r["dst"], r["dd"]) for r in reqs]
    for t in tickets:
        status, lat = srv.wait(t)
        assert status == L.OK and lat >= 0
    st = srv.stats()
    assert st["completed"] == len(reqs) and st["failed"] == 0
    assert st["max_inflight_bytes"] <= budget
    assert 0 <= st["p50_latency"] <= st["p99_latency"] <= st["max_latency"]
    if policy != 0:
        assert st["launches"] == len(reqs)
    srv.close()
    for r in reqs:
        check(r)
    # each result also equals a lone copy of the request
    for r in reqs[:10]:
        out = r["dst"].alloc(fill=0x33)
        L.copy(r["src"], r["sd"], r["dst"], out)
        torch.cuda.synchronize()
        for x, y in zip(out, r["dd"]):
            assert torch.equal(x, y)


@pytest.mark.parametrize("group_bytes,depth,stream_bytes", [(1, 1, 0), (1, 3, 0), (1 << 20, 2, 0), (1 << 40, 1, 0),
                                                          (1 << 40, 4, 1), (1 << 21, 8, 1 << 22)])
def test_group_bytes_and_depth(L, orc, group_bytes, depth, stream_bytes):
    """A launch closes once its bytes reach group_bytes (one request per launch
    when that is 1 byte); any depth of launches per stream, and holding
    requests back while a stream has stream_bytes in flight, give the same
    bytes."""
    reqs = requests(L, orc, 21, count=40, nmax=20000)
    srv = L.Server(1 << 34, group_bytes=group_bytes, depth=depth, stream_bytes=stream_bytes)
    torch.cuda.synchronize()
    tickets = [srv.submit(r["src"], r["sd"], r["dst"], r["dd"]) for r in reqs]
    for t in tickets:
        assert srv.wait(t)[0] == L.OK
    st = srv.stats()
    assert st["completed"] == len(reqs)
    if group_bytes == 1:
        assert st["launches"] == len(reqs)
    srv.close()
    for r in reqs:
        check(r)


def test_concurrent_submitters_and_bad_requests(L, orc):
    reqs = requests(L, orc, 11, count=48, nmax=20000)
    srv = L.Server(1 << 34)
    torch.cuda.synchronize()
    errors, tickets = [], {}

    def worker(part):
        for k in part:
            r = reqs[k]
            tickets[k] = srv.submit(r["src"], r["sd"], r["dst"], r["dd"])
            if k % 8 == 0:  # a bad request: destination blob too small
                small = [t[: t.numel() // 2] for t in r["dst"].alloc()]
                try:
                    srv.submit(r["src"], r["sd"], r["dst"], small)
                except L.LlamaError as e:
                    errors.append(e.status)
            time.sleep(0.0005)

    threads = [threading.Thread(target=worker, args=(range(j, 48, 4),)) for j in range(4)]
    for th in threads:
        th.start()
    for th in threads:
        th.join()
    for k, t in tickets.items():
        assert srv.wait(t)[0] == L.OK
    assert errors == [L.E_BLOB_TOO_SMALL] * 6
    srv.close()
    for r in reqs:
        check(r)


def test_budget_and_dependencies(L, orc):
    r = L.Record(W.PARTICLE)
    n = 10000
    a, b, c = (L.Mapping(r, k, [n], l) for k, l in (("aos_packed", 0), ("aosoa", 32), ("soa_single", 0)))
    x = torch.randint(0, 255, (n * 28,), dtype=torch.uint8, device="cuda")
    y = b.alloc(fill=0)
    z = c.alloc(fill=0)
    torch.cuda.synchronize()  # the server's streams do not wait for the default stream
    srv = L.Server(4 * n * 28)
    with pytest.raises(L.LlamaError) as e:
        L.Server(100).submit(a, [x], b, y)
    assert e.value.status == L.E_NO_BUDGET
    # B reads what A writes: the server must not run them together
    ta = srv.submit(a, [x], b, y)
    tb = srv.submit(b, y, c, z)
    assert srv.wait(ta)[0] == L.OK and srv.wait(tb)[0] == L.OK
    want = c.alloc(fill=1)
    L.copy(a, [x], c, want)
    torch.cuda.synchronize()
    assert torch.equal(z[0], want[0])
    srv.close()


def _smap(mod, rec, layout, n):
    if layout[0] == "split":
        return mod.Mapping(rec, "split", [n], split=layout[1])
    return mod.Mapping(rec, layout[0], [n], layout[1])


@pytest.mark.parametrize("policy", [0, 1, 2])
def test_split_requests(L, orc, policy):
    """Requests with a Split side (sec. 3.7) among plain ones: their part
    copies go into the group's launch side by side (batched), or run in order
    (per request, element-wise); all equal the oracle.  The batched server
    refuses a request whose part copies must run in order."""
    s1 = ("split", (0, 3, ("aosoa", 32), ("soa_multi", 0)))
    s2 = ("split", (3, 3, ("soa_multi", 0), ("aos_aligned", 0)))
    s3 = ("split", (0, 3, ("aos_packed", 0), ("aosoa", 8)))
    pairs = [(("aos_packed", 0), s1), (s1, ("soa_multi", 0)), (s1, s3), (s3, s1), (("aosoa", 64), s2),
             (("aos_aligned", 0), ("soa_single", 0))]
    if policy != 0:  # part copies in order: into AoS from two parts, and a One source
        pairs += [(s1, ("aos_packed", 0)), (s2, ("aosoa", 32)),
                  (("split", (6, 1, ("one", 0), ("soa_multi", 0))), ("aos_aligned", 0))]
    g = random.Random(60 + policy)
    ro, rg = orc.Record(W.PARTICLE), L.Record(W.PARTICLE)
    reqs = []
    for k in range(3 * len(pairs)):
        a, b = pairs[k % len(pairs)]
        n = g.choice([1, 500, 20011])
        ms_o, md_o = _smap(orc, ro, a, n), _smap(orc, ro, b, n)
        src = [W.random_bytes(x, 900 + k * 7 + j) for j, x in enumerate(ms_o.blob_sizes())]
        ms, md = _smap(L, rg, a, n), _smap(L, rg, b, n)
        reqs.append({"src": ms, "sd": [torch.from_numpy(x).cuda() for x in src], "dst": md,
                     "dd": md.alloc(fill=0xCD), "want": orc.copy(ms_o, src, md_o)})
    srv = L.Server(1 << 33, policy=policy)
    torch.cuda.synchronize()
    print(f"split requests, policy {policy}: {len(reqs)}", flush=True)
    tickets = [srv.submit(r["src"], r["sd"], r["dst"], r["dd"]) for r in reqs]
    for t in tickets:
        assert srv.wait(t)[0] == L.OK
    if policy == 0:
        n = 100
        ms, md = _smap(L, rg, s1, n), L.Mapping(rg, "aos_packed", [n])
        with pytest.raises(L.LlamaError) as e:
            srv.submit(ms, ms.alloc(), md, md.alloc())
        assert e.value.status == L.E_UNSUPPORTED
    srv.close()
    for r in reqs:
        check(r)


@pytest.mark.parametrize("policy", [0, 2])
def test_bench_size_requests_in_full(L, orc, policy):
    """Requests of the serving benchmark's sizes (payloads of 256 MB to 1 GB
    beside small ones) in one mix under its 64 GB budget: every destination
    byte equals the oracle's copy."""
    g = random.Random(41 + policy)
    reqs = []
    for k in range(10):
        name = g.choice(["particle", "mixed"])
        ro, rg = orc.Record(W.RECORDS[name]), L.Record(W.RECORDS[name])
        payload = g.uniform(256e6, 1e9) if k % 2 == 0 else g.uniform(64e3, 8e6)
        n = int(payload // ro.packed_size)
        a, b = g.sample(W.LAYOUTS, 2)
        ms_o, md_o = orc.Mapping(ro, a[0], [n], a[1]), orc.Mapping(ro, b[0], [n], b[1])
        src = [W.random_bytes(s, 9000 + k * 13 + j) for j, s in enumerate(ms_o.blob_sizes())]
        want = orc.copy_threads(ms_o, src, md_o)
        ms, md = L.Mapping(rg, a[0], [n], a[1]), L.Mapping(rg, b[0], [n], b[1])
        reqs.append({"src": ms, "sd": [torch.from_numpy(x).cuda() for x in src], "dst": md,
                     "dd": md.alloc(fill=0xCD), "want": want})
        del src
    srv = L.Server(64 << 30, policy=policy)
    torch.cuda.synchronize()
    tickets = [srv.submit(r["src"], r["sd"], r["dst"], r["dd"]) for r in reqs]
    for t in tickets:
        assert srv.wait(t)[0] == L.OK
    assert srv.stats()["completed"] == len(reqs)
    srv.close()
    for r in reqs:
        check(r)
