"""The request server's engine on the CPU (no GPU): the server runs on an
executor (llama_server_create_ex) whose launches are carried out here, on
host buffers, by the oracle.  This checks what the engine decides, apart from
the kernels: results, grouping, admission within the budget, arrival order,
range conflicts, error isolation and latency bookkeeping.  The oracle is used
by this test only; the library's own engine runs launches with its kernels."""
import threading
import time

import numpy as np
import pytest

from paper_2106_04284_amd import llama as L
from paper_2106_04284_amd import workloads as W


class OracleExecutor:
    """Runs each launch with the oracle.  A launch finishes when the test
    releases it (hold=True), or `delay` seconds after it started."""

    def __init__(self, orc, hold=False, delay=0.0, fail_start=(), fail_poll=()):
        self.orc, self.hold, self.delay = orc, hold, delay
        self.fail_start, self.fail_poll = set(fail_start), set(fail_poll)
        self.lock = threading.Lock()
        self.requests = {}      # dst blob pointer -> request record
        self.active = {}        # launch -> (start time, [requests])
        self.released = set()
        self.log = []           # (launch, [request ids]) in start order
        self.max_active_bytes = 0
        self.conflicts = []

    def register(self, req):
        self.requests[req["dst_ptrs"][0]] = req

    def _ranges(self, req):
        return [(p, p + s, False) for p, s in zip(req["src_ptrs"], req["src_sizes"])] + \
               [(p, p + s, True) for p, s in zip(req["dst_ptrs"], req["dst_sizes"])]

    def start(self, launch, items):
        reqs = [self.requests[int(it.dst_blobs[0].ptr)] for it in items]
        for it, req in zip(items, reqs):  # the engine hands over the submitted descriptors
            assert it.src.contents.kind == L.KINDS[req["src_layout"][0]]
            assert it.dst.contents.kind == L.KINDS[req["dst_layout"][0]]
            assert it.src.contents.extents[0] == req["n"]
            assert it.src.contents.record.contents.num_nodes == req["nodes"]
        with self.lock:
            mine = [r for req in reqs for r in self._ranges(req)]
            for other, (_, oreqs) in self.active.items():
                theirs = [r for q in oreqs for r in self._ranges(q)]
                for a in mine:
                    for b in theirs:
                        if (a[2] or b[2]) and a[0] < b[1] and b[0] < a[1]:
                            self.conflicts.append((launch, other))
            self.log.append((launch, [r["id"] for r in reqs]))
            if any(r["id"] in self.fail_start for r in reqs):
                return L.E_HIP
            self.active[launch] = (time.monotonic(), reqs)
            self.max_active_bytes = max(self.max_active_bytes,
                                        sum(q["bytes"] for _, qs in self.active.values() for q in qs))
        for req in reqs:  # the copy itself, on the host buffers
            out = self.orc.copy(req["ms_o"], req["src"], req["md_o"])
            for d, o in zip(req["dst"], out):
                np.copyto(d, o)
        return L.OK

    def poll(self, launch):
        with self.lock:
            t0, reqs = self.active[launch]
            if self.hold and launch not in self.released:
                return 0
            if time.monotonic() - t0 < self.delay:
                return 0
            del self.active[launch]
        if any(r["id"] in self.fail_poll for r in reqs):
            return L.E_HIP
        return 1

    def release_all(self):
        with self.lock:
            self.released |= set(self.active)


def make_requests(orc, count, seed, nmax=3000, chain=False):
    g = np.random.default_rng(seed)
    out = []
    for k in range(count):
        name = ["particle", "mixed", "listing1"][k % 3]
        rec = W.RECORDS[name]
        n = int(g.integers(1, nmax))
        a, b = [W.LAYOUTS[i] for i in g.choice(len(W.LAYOUTS), 2, replace=False)]
        if chain and out:  # this request reads the previous one's destination
            prev = out[-1]
            name, rec, n, a = prev["name"], prev["rec"], prev["n"], prev["dst_layout"]
        ro, rg = orc.Record(rec), L.Record(rec)
        ms_o, md_o = orc.Mapping(ro, a[0], [n], a[1]), orc.Mapping(ro, b[0], [n], b[1])
        if chain and out:
            src = out[-1]["dst"]
        else:
            src = [W.random_bytes(s, seed * 1000 + k * 7 + j) for j, s in enumerate(ms_o.blob_sizes())]
        dst = [np.full(s, 0xCD, dtype=np.uint8) for s in md_o.blob_sizes()]
        ms, md = L.Mapping(rg, a[0], [n], a[1]), L.Mapping(rg, b[0], [n], b[1])
        out.append({"id": k, "name": name, "rec": rec, "n": n, "src_layout": a, "dst_layout": b,
                    "ms_o": ms_o, "md_o": md_o, "ms": ms, "md": md, "src": src, "dst": dst,
                    "nodes": len(ms.record.nodes),
                    "src_ptrs": [x.ctypes.data for x in src], "src_sizes": [x.nbytes for x in src],
                    "dst_ptrs": [x.ctypes.data for x in dst], "dst_sizes": [x.nbytes for x in dst],
                    "bytes": sum(x.nbytes for x in src) + sum(x.nbytes for x in dst)})
    return out


def submit(srv, req):
    return srv.submit(req["ms"], [(p, s) for p, s in zip(req["src_ptrs"], req["src_sizes"])],
                      req["md"], [(p, s) for p, s in zip(req["dst_ptrs"], req["dst_sizes"])])


def expected(orc, req, src=None):
    return orc.copy(req["ms_o"], src if src is not None else req["src"], req["md_o"])


def test_results_and_grouping(orc):
    ex = OracleExecutor(orc)
    reqs = make_requests(orc, 30, seed=1)
    for r in reqs:
        ex.register(r)
    wants = [expected(orc, r) for r in reqs]
    srv = L.Server(1 << 40, group_bytes=1 << 30, max_batch=8, executor=ex)
    tickets = [submit(srv, r) for r in reqs]
    for t in tickets:
        assert srv.wait(t)[0] == L.OK
    st = srv.stats()
    srv.close()
    for r, w in zip(reqs, wants):
        for d, x in zip(r["dst"], w):
            assert np.array_equal(d, x)
    assert st["completed"] == 30 and st["failed"] == 0
    assert all(len(ids) <= 8 for _, ids in ex.log)
    # every request ran exactly once, and queued small requests shared launches
    assert sorted(i for _, ids in ex.log for i in ids) == list(range(30))
    assert st["launches"] == len(ex.log) < 30


def test_large_requests_run_alone(orc):
    ex = OracleExecutor(orc, hold=True)
    reqs = make_requests(orc, 12, seed=2)
    for r in reqs:
        ex.register(r)
    cut = sorted(r["bytes"] for r in reqs)[6]  # about half the requests are "large"
    srv = L.Server(1 << 40, group_bytes=cut, streams=1, depth=1, executor=ex)
    tickets = [submit(srv, r) for r in reqs]
    while any(srv.poll(t) is None for t in tickets):
        ex.release_all()
        time.sleep(0.002)
    srv.close()
    for _, ids in ex.log:
        big = [i for i in ids if reqs[i]["bytes"] >= cut]
        assert not big or len(ids) == 1, ids  # a large request never shares a launch
        assert sum(reqs[i]["bytes"] for i in ids[:-1]) < cut  # a group closes once it reaches group_bytes


def test_budget_and_arrival_order(orc):
    ex = OracleExecutor(orc, hold=True)
    reqs = make_requests(orc, 24, seed=3)
    for r in reqs:
        ex.register(r)
    budget = 3 * max(r["bytes"] for r in reqs)
    srv = L.Server(budget, group_bytes=1, executor=ex)  # one request per launch
    tickets = [submit(srv, r) for r in reqs]
    time.sleep(0.05)
    with ex.lock:
        assert ex.active, "nothing admitted"
        held = sum(q["bytes"] for _, qs in ex.active.values() for q in qs)
    assert held <= budget
    assert srv.stats()["queued"] > 0  # the rest wait for budget
    while any(srv.poll(t) is None for t in tickets):
        ex.release_all()
        time.sleep(0.002)
    st = srv.stats()
    srv.close()
    assert ex.max_active_bytes <= budget and st["max_inflight_bytes"] <= budget
    started = [i for _, ids in ex.log for i in ids]
    assert started == sorted(started)  # admitted in arrival order


def test_dependent_requests_never_overlap(orc):
    ex = OracleExecutor(orc, delay=0.01)
    reqs = make_requests(orc, 10, seed=4, chain=True)  # each reads the previous destination
    for r in reqs:
        ex.register(r)
    srv = L.Server(1 << 40, group_bytes=1 << 30, executor=ex)
    tickets = [submit(srv, r) for r in reqs]
    for t in tickets:
        assert srv.wait(t)[0] == L.OK
    srv.close()
    assert ex.conflicts == []
    # the chain composes: the last destination equals the oracle's copy
    # chain from the first source
    cur = reqs[0]["src"]
    for r in reqs:
        cur = expected(orc, r, cur)
    for d, x in zip(reqs[-1]["dst"], cur):
        assert np.array_equal(d, x)


def test_failures_stay_with_their_requests(orc):
    ex = OracleExecutor(orc, fail_start=[3], fail_poll=[7])
    reqs = make_requests(orc, 12, seed=5)
    for r in reqs:
        ex.register(r)
    srv = L.Server(1 << 40, group_bytes=1, executor=ex)
    tickets = [submit(srv, r) for r in reqs]
    status = [srv.wait(t)[0] for t in tickets]
    st = srv.stats()
    srv.close()
    assert status[3] == L.E_HIP and status[7] == L.E_HIP
    assert all(s == L.OK for k, s in enumerate(status) if k not in (3, 7))
    assert st["failed"] == 2 and st["completed"] == 10


def test_latency_bookkeeping(orc):
    ex = OracleExecutor(orc, delay=0.02)
    reqs = make_requests(orc, 6, seed=6)
    for r in reqs:
        ex.register(r)
    srv = L.Server(1 << 40, group_bytes=1, executor=ex)
    tickets = [submit(srv, r) for r in reqs]
    lat = [srv.wait(t)[1] for t in tickets]
    st = srv.stats()
    assert all(x >= 0.02 for x in lat)  # submit to observed completion
    assert 0.02 <= st["p50_latency"] <= st["p99_latency"] <= st["max_latency"] == pytest.approx(max(lat))
    assert st["window"] >= 0.02 and st["bytes_done"] == sum(r["bytes"] for r in reqs)
    srv.reset_stats()
    st = srv.stats()
    assert st["completed"] == 0 and st["p99_latency"] == 0
    srv.close()


def test_submit_errors(orc):
    ex = OracleExecutor(orc, hold=True)
    reqs = make_requests(orc, 4, seed=7)
    for r in reqs:
        ex.register(r)
    with pytest.raises(L.LlamaError) as e:  # a request larger than the whole budget
        submit(L.Server(reqs[0]["bytes"] - 1, executor=ex), reqs[0])
    assert e.value.status == L.E_NO_BUDGET
    srv = L.Server(1 << 40, group_bytes=1, streams=1, depth=1, queue_capacity=2, executor=ex)
    t0 = submit(srv, reqs[0])
    time.sleep(0.05)  # admitted and held: the queue is empty again
    t1, t2 = submit(srv, reqs[1]), submit(srv, reqs[2])
    with pytest.raises(L.LlamaError) as e:
        submit(srv, reqs[3])
    assert e.value.status == L.E_BUSY
    while any(srv.poll(t) is None for t in (t0, t1, t2)):
        ex.release_all()
        time.sleep(0.002)
    srv.close()
