#!/usr/bin/env python3
"""Benchmark of the MI355X layout-aware copy.

Default workload: the n-body particle record {pos{x,y,z}, vel{x,y,z}, mass}
(7 x float32, LLAMA sec. 4.1/4.2) with 2^26 records, copied between every
ordered pair of the seven layouts packed AoS, aligned AoS, SoA single-blob,
SoA multi-blob, AoSoA8, AoSoA32 and AoSoA64 (42 pairs).  One step is one pass
over the 42 copies; every copy reads a 1.879 GB source layout and writes a
1.879 GB destination layout, with all seven layouts resident in HBM.

Prints one JSON line: whole-job throughput in GB/s (bytes read plus bytes
written, 1 GB = 1e9 B), the roofline of the dominant kernel (the TILE kernel,
timed per launch with HIP events on the launch stream), the CPU oracle
timed on a bounded sample of the same workload, and, under
extras.batch_1000_arrays, the batching workload below (one graph-captured
launch against 1,000 naive and 1,000 llama_copy launches on the same GPU).

Other workloads (--workload):
  pairs  the 42 layout pairs of one record (--record, --records; per-pair
         figures with --details);
  lbm    128^3 cells of 19 f64 + u32, aligned AoS <-> SoA multi-blob <->
         AoSoA32, each copy started cold (1 GiB read before it);
  batch  1,000 arrays of log-uniform size and mixed record types as one
         hipGraph-captured launch, against 1,000 naive and 1,000 llama_copy
         launches;
  serve  a Poisson trace of copy requests against the request server at
         offered loads of 0.5 and 0.8 of the batch's GB/s (p50/p99 latency);
  pic    4,096 particle-in-cell frames of 256 records, SoA <-> AoSoA32, as
         one batch launch per direction against per-frame launches;
  box    sub-box copies: the 256^3 interior of a 258^3 lattice-Boltzmann
         grid into a 256^3 grid of another layout (sec. 3.2 VirtualView);
  linearize  2^26 particles on an 8192 x 8192 grid between row-major,
         column-major and Morton views (sec. 3.7 linearizers);
  transfer   host <-> device copies with a layout change, chunked and
         overlapped (sec. 3.9), against unchunked and raw memcpy.
"""
from __future__ import annotations

import argparse
import collections
import hashlib
import json
import os
import statistics
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)
# CPUs this process may run on, read before any OpenMP runtime pins the thread
START_CPUS = os.sched_getaffinity(0)
AFFINITY_CPUS = len(START_CPUS)
# the threaded CPU oracle runs one thread per core, each pinned (sec. 4 setup);
# OpenMP reads these when it starts
os.environ.setdefault("OMP_PROC_BIND", "close")
os.environ.setdefault("OMP_PLACES", "cores")

from paper_2106_04284_amd import workloads as W  # noqa: E402

METRIC = "layout-copy GB/s (rd+wr) & % HBM peak; batched vs naive per-array; p99 latency"
HBM_PEAK_GBS = 8000.0
PROFILE_COUNTERS = os.path.join(ROOT, "profiles", "tile_kernel_particle_2e26_counters.json")


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def _name(layout):
    if layout[0] == "split":
        f, c, a, b = layout[1]
        return f"split[{f},{f + c})({_name(a)},{_name(b)})"
    kind, lanes = layout
    return f"{kind}{lanes}" if kind == "aosoa" else kind


def kernel_source_sha() -> str:
    h = hashlib.sha256()
    for fn in ("kernels.hip", "kernel_args.hpp", "core.cpp"):
        with open(os.path.join(ROOT, "paper_2106_04284_amd", "csrc", fn), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def measured_traffic():
    """HBM bytes per TILE launch from committed rocprofv3 counter runs, if they
    were taken on the current kernel source."""
    try:
        with open(PROFILE_COUNTERS) as f:
            c = json.load(f)
    except (OSError, ValueError):
        return None
    if c.get("kernel_source_sha") != kernel_source_sha():
        return None
    return c.get("hbm_bytes_per_launch")


# --------------------------------------------------------------------------
# CPU baseline: the oracle on a bounded sample of the same workload
# --------------------------------------------------------------------------

def make_mapping(mod, rec, layout, extents):
    """A mapping of `mod` (the library binding or the oracle): layout is
    (kind, lanes), or ("split", (first, count, (kind, lanes), (kind, lanes)))."""
    if layout[0] == "split":
        return mod.Mapping(rec, "split", extents, split=layout[1])
    return mod.Mapping(rec, layout[0], extents, layout[1])


def host_info():
    """The host's CPU model and core counts, for the CPU baseline."""
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"cpu_model": model, "nproc": os.cpu_count(), "affinity_cpus": AFFINITY_CPUS,
            "omp_num_threads": os.environ.get("OMP_NUM_THREADS")}


def cpu_baseline(record, layouts, pairs, n_single, n_full, budget_single_s=6.0, budget_all_s=12.0):
    """The oracle on the host: one thread over the pairs at n_single records,
    then the threaded oracle on every core it may use (pinned, one thread per
    core) over pairs at the full n_full records, and host memcpy of one full
    layout at 1 and at all threads (the reference line of sec. 4.2)."""
    from oracle import oracle as orc
    # the calling thread is the OpenMP team's first thread: it takes the
    # first core, the others one core each
    os.sched_setaffinity(0, {min(START_CPUS)})
    ro = orc.Record(record)
    threads = orc.max_threads()

    def run(n, todo, nthreads, budget):
        maps = {l: make_mapping(orc, ro, l, [n]) for l in layouts}
        size = max(sum(m.blob_sizes()) for m in maps.values())
        pool = W.random_bytes(size, 99)
        out = np.zeros(size, dtype=np.uint8)  # pages touched before timing

        def views(buf, m):
            offs = np.cumsum([0] + m.blob_sizes())
            return [buf[offs[k]:offs[k + 1]] for k in range(m.blob_count)]

        nbytes, elapsed, done = 0, 0.0, 0
        for a, b in todo:
            src, dst = views(pool, maps[a]), views(out, maps[b])
            t0 = time.perf_counter()
            orc.copy_threads(maps[a], src, maps[b], dst, threads=nthreads)
            elapsed += time.perf_counter() - t0
            nbytes += sum(maps[a].blob_sizes()) + sum(maps[b].blob_sizes())
            done += 1
            if elapsed > budget:
                break
        return nbytes, elapsed, done, pool, out

    nb1, t1, done1, _, _ = run(n_single, pairs, 1, budget_single_s)
    spread = pairs[::7] + [p for k, p in enumerate(pairs) if k % 7]
    nba, ta, donea, pool, out = run(n_full, spread, threads, budget_all_s)
    mem = {}
    for nt in (1, threads):
        orc.memcpy_threads(out, pool, nt)
        t0 = time.perf_counter()
        used = orc.memcpy_threads(out, pool, nt)
        mem[used] = 2 * pool.nbytes / (time.perf_counter() - t0) / 1e9
    del pool, out
    host = host_info()
    return {"value": round(nba / ta / 1e9, 3), "unit": "GB/s", "cores": threads, "kind": "oracle",
            "sample": f"threaded oracle, {threads} threads pinned one per core, {donea} of the {len(pairs)} layout "
                      f"pairs at the full {n_full} records ({nba / 1e9:.2f} GB read+written in {ta:.1f} s); "
                      f"one thread: {done1} pairs at {n_single} records ({nb1 / 1e9:.2f} GB in {t1:.1f} s)",
            "single_thread_gbs": round(nb1 / t1 / 1e9, 3),
            "host_memcpy_gbs": {str(k): round(v, 1) for k, v in mem.items()},
            "host": host}


# --------------------------------------------------------------------------
# GPU workloads
# --------------------------------------------------------------------------

def setup_layouts(L, torch, record, extents, layouts, values):
    """Uploads the per-leaf values as multi-blob SoA and fills every other
    layout from it on the GPU (untimed)."""
    rg = L.Record(record)
    maps = {l: make_mapping(L, rg, l, extents) for l in layouts}
    mb_layout = ("soa_multi", 0)
    blobs = {mb_layout: [torch.from_numpy(np.ascontiguousarray(v).view(np.uint8).reshape(-1)).cuda()
                         for v in values]}
    for l in layouts:
        if l != mb_layout:
            blobs[l] = maps[l].alloc()
            L.copy(maps[mb_layout], blobs[mb_layout], maps[l], blobs[l])
    torch.cuda.synchronize()
    return maps, blobs


def time_pairs(L, torch, maps, blobs, pairs, steps, warmup, stream, flush=None):
    """Times every pair `steps` times with HIP events around each copy.  With
    `flush` (a device buffer larger than the 256 MB Infinity Cache), the
    buffer is read before each copy, outside its events, so that every copy
    starts cold."""
    plans = {p: (L.plan(maps[p[0]], maps[p[1]]) if "split" not in (p[0][0], p[1][0]) else {"path": "split"})
             for p in pairs}
    for _ in range(warmup):
        for a, b in pairs:
            L.copy(maps[a], blobs[a], maps[b], blobs[b], stream=stream)
    torch.cuda.synchronize()
    ev = {p: [] for p in pairs}
    # every event exists before the clock starts: creating one is host work
    # that, between two copies, can leave the GPU idle
    pending = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
               for _ in range(steps * len(pairs))]
    for e0, e1 in pending:  # the runtime creates an event at its first record
        e0.record(stream)
        e1.record(stream)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    start = torch.cuda.Event(enable_timing=True)
    end = torch.cuda.Event(enable_timing=True)
    start.record(stream)
    for k in range(steps):
        for a, b in pairs:
            e0, e1 = pending.pop()
            if flush is not None:
                with torch.cuda.stream(stream):
                    flush.sum(dtype=torch.int64)  # reads it: evicts without leaving dirty lines
            e0.record(stream)
            L.copy(maps[a], blobs[a], maps[b], blobs[b], stream=stream)
            e1.record(stream)
            ev[(a, b)].append((e0, e1))
    end.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    total_ms = start.elapsed_time(end)
    per_pair = {}
    for p, lst in ev.items():
        ms = [e0.elapsed_time(e1) for e0, e1 in lst]
        nb = sum(maps[p[0]].blob_sizes()) + sum(maps[p[1]].blob_sizes())
        per_pair[p] = {"path": plans[p]["path"], "bytes": nb, "ms_median": statistics.median(ms),
                       "ms_min": min(ms), "ms_mean": statistics.mean(ms),
                       "gbs_median": nb / (statistics.median(ms) * 1e-3) / 1e9}
    copies_ms = sum(sum(e0.elapsed_time(e1) for e0, e1 in lst) for lst in ev.values())
    return wall, (copies_ms if flush is not None else total_ms), per_pair, plans


def naive_reference(L, torch, maps, blobs, pairs, stream, reps=3):
    """The element-wise baseline kernel on the same pairs (median GB/s)."""
    out = {}
    for a, b in pairs:
        L.copy_naive(maps[a], blobs[a], maps[b], blobs[b], stream=stream)
        ms = []
        for _ in range(reps):
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            L.copy_naive(maps[a], blobs[a], maps[b], blobs[b], stream=stream)
            e1.record(stream)
            e1.synchronize()
            ms.append(e0.elapsed_time(e1))
        nb = sum(maps[a].blob_sizes()) + sum(maps[b].blob_sizes())
        out[(a, b)] = nb / (statistics.median(ms) * 1e-3) / 1e9
    return out


def d2d_reference(torch, nbytes, stream, reps=5):
    """Device-to-device memcpy of the same byte count (GB/s, read+write)."""
    import ctypes
    src = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    dst = torch.empty_like(src)
    hip = ctypes.CDLL("libamdhip64.so")
    hip.hipMemcpyAsync.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int, ctypes.c_void_p]
    ms = []
    for k in range(reps + 1):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        rc = hip.hipMemcpyAsync(ctypes.c_void_p(dst.data_ptr()), ctypes.c_void_p(src.data_ptr()), nbytes, 3,
                                ctypes.c_void_p(stream.cuda_stream))
        e1.record(stream)
        e1.synchronize()
        if rc != 0:
            return None
        if k:
            ms.append(e0.elapsed_time(e1))
    del src, dst
    return 2 * nbytes / (statistics.median(ms) * 1e-3) / 1e9


# --------------------------------------------------------------------------
# batching (1,000 arrays) and serving (Poisson requests)
# --------------------------------------------------------------------------

def _layout_maps(L, rec_name, n, src, dst, cache):
    rg = cache.setdefault(("rec", rec_name), L.Record(W.RECORDS[rec_name]))
    return L.Mapping(rg, src[0], [n], src[1]), L.Mapping(rg, dst[0], [n], dst[1])


TUNE_CACHE = None  # --tune-cache: a tuning-cache file read before and written after class tuning


def _tune_classes(L, torch, classes, stream):
    """Autotunes each (record, layout pair) class once at 2^20 records (a
    class already in the tuning cache is kept)."""
    cache, tuned = {}, 0
    if TUNE_CACHE and os.path.exists(TUNE_CACHE):
        L.tune_load(TUNE_CACHE)
    for rec_name, src, dst in sorted(classes):
        ms, md = _layout_maps(L, rec_name, 1 << 20, src, dst, cache)
        if L.tune_lookup(ms, md) is not None:
            continue
        sb = [torch.empty(s, dtype=torch.uint8, device="cuda").random_(0, 255) for s in ms.blob_sizes()]
        db = md.alloc()
        torch.cuda.synchronize()  # the fills ran on torch's stream
        L.autotune(ms, sb, md, db, stream=stream, reps=2)
        tuned += 1
        del sb, db
    if TUNE_CACHE:
        L.tune_save(TUNE_CACHE)
    return tuned


def _batch_items(L, torch, stream):
    """The 1,000 arrays of the batching workload, sources filled with random
    bytes, and the autotuned record/pair classes."""
    items_spec = W.batch_items()
    log(f"batch: allocating {len(items_spec)} arrays")
    cache, items = {}, []
    for it in items_spec:
        ms, md = _layout_maps(L, it["record"], it["n"], it["src"], it["dst"], cache)
        sb = [torch.empty(s, dtype=torch.uint8, device="cuda") for s in ms.blob_sizes()]
        for t in sb:
            t.random_(0, 255)
        items.append((ms, sb, md, md.alloc()))
    total = sum(sum(i[0].blob_sizes()) + sum(i[2].blob_sizes()) for i in items)
    torch.cuda.synchronize()
    log(f"batch: {total / 1e9:.1f} GB read+written per pass; autotuning the record/pair classes")
    tuned = _tune_classes(L, torch, {(it["record"], it["src"], it["dst"]) for it in items_spec}, stream)
    return items, total, tuned


def _timed(torch, stream, fn, reps):
    """Median and minimum milliseconds of `fn` over `reps` runs after one
    warm-up, with HIP events on `stream`."""
    fn()
    torch.cuda.synchronize()
    ms = []
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        fn()
        e1.record(stream)
        e1.synchronize()
        ms.append(e0.elapsed_time(e1))
    return statistics.median(ms), min(ms)


def batch_measure(L, torch, args, stream, naive=True):
    """The 1,000-array batch: the default plan, then the batch's autotuner,
    then (with `naive`) the same arrays as 1,000 naive and as 1,000
    llama_copy launches.  Returns the figures and releases the arrays."""
    items, total, tuned = _batch_items(L, torch, stream)

    def timed(fn, reps):
        return _timed(torch, stream, fn, reps)

    # the default plan (largest tile in 31 KiB of LDS, 256 threads), then the
    # batch's autotuner choosing LDS budget, threads and grid on these arrays
    b = L.Batch(items)
    heur_med, _ = timed(lambda: b.launch(stream), 3)
    heur_gbs = total / (heur_med * 1e-3) / 1e9
    log(f"batch: default plan {heur_gbs:.1f} GB/s; autotuning the batch")
    if not args.no_batch_autotune:
        b.autotune(stream=stream, reps=2)
    info = b.info()
    log(f"batch: plan of {info['threads']} threads, {info['lds_bytes']} B of LDS")
    med, mn = timed(lambda: b.launch(stream), args.steps)
    out = {"bytes": total, "arrays": len(items), "tuned_classes": tuned, "info": info, "ms": med, "ms_min": mn,
           "gbs": total / (med * 1e-3) / 1e9, "default_gbs": heur_gbs, "default_ms": heur_med}
    if naive:
        log("batch: timing 1,000 per-array naive launches and 1,000 per-array llama_copy launches")
        out["naive_ms"], _ = timed(lambda: [L.copy_naive(i[0], i[1], i[2], i[3], stream=stream) for i in items], 2)
        out["lone_ms"], _ = timed(lambda: [L.copy(i[0], i[1], i[2], i[3], stream=stream) for i in items], 2)
    b.close()
    del items, b
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    return out


def batch_extras(m):
    """The batch figures as they appear in a bench line."""
    gbs = lambda ms: round(m["bytes"] / (ms * 1e-3) / 1e9, 1)  # noqa: E731
    ex = {"batched_gbs": round(m["gbs"], 1), "batched_ms": round(m["ms"], 3), "batched_ms_min": round(m["ms_min"], 3),
          "hbm_peak_frac": round(m["gbs"] / HBM_PEAK_GBS, 4), "default_plan_gbs": round(m["default_gbs"], 1),
          "autotuned_vs_default": round(m["default_ms"] / m["ms"], 3)}
    if "naive_ms" in m:
        ex.update({"naive_per_array_gbs": gbs(m["naive_ms"]), "llama_copy_per_array_gbs": gbs(m["lone_ms"]),
                   "batched_vs_naive": round(m["naive_ms"] / m["ms"], 2),
                   "batched_vs_per_array_copy": round(m["lone_ms"] / m["ms"], 2)})
    return ex


BATCH_WORKLOAD = ("batching: 1,000 arrays, record counts log-uniform 1e3..1e7, particle or mixed "
                  "{f64[3],f32[4],i32[2],u8} record, random ordered layout pair of 42; one hipGraph-captured launch")


def bench_batch(L, torch, args, dev, stream):
    m = batch_measure(L, torch, args, stream, naive=not args.no_naive)
    info = m["info"]
    return {"metric": METRIC, "value": round(m["gbs"], 1), "unit": "GB/s", "n_gpus": 1, "steps": args.steps,
            "warmup": 1, "ms_per_step": round(m["ms"], 3), "higher_is_better": True, "scaling": "weak",
            "vs_baseline": None, "dtype": "u32", "data": "synthetic",
            "config": {"workload": BATCH_WORKLOAD,
                       "bytes_per_step": m["bytes"], "arrays": m["arrays"], "threads": info["threads"],
                       "work_units": info["work_units"], "workgroups": info["workgroups"],
                       "wg_per_cu": info["wg_per_cu"], "lds_bytes": info["lds_bytes"], "launches": info["launches"],
                       "tuned_classes": m["tuned_classes"]},
            "hbm_peak_frac": round(m["gbs"] / HBM_PEAK_GBS, 4),
            "extras": batch_extras(m),
            "device": dev.name}


def bench_pic(L, torch, args, dev, stream):
    """Particle-in-cell-shaped batch: 4,096 frames of 256 particle records,
    single-blob SoA -> AoSoA32 and back, each direction as one batch launch,
    against one naive launch and one llama_copy per frame."""
    frames, per = 4096, 256
    r = L.Record(W.PARTICLE)
    soa, aosoa = L.Mapping(r, "soa_single", [per]), L.Mapping(r, "aosoa", [per], 32)
    g = torch.Generator(device="cuda")
    g.manual_seed(W.BASE_SEED + 6)
    a = [torch.randint(0, 256, (soa.blob_size(0),), dtype=torch.uint8, device="cuda", generator=g)
         for _ in range(frames)]
    b = [aosoa.alloc()[0] for _ in range(frames)]
    fwd = [(soa, [x], aosoa, [y]) for x, y in zip(a, b)]
    back = [(aosoa, [y], soa, [x]) for x, y in zip(a, b)]
    total = frames * (soa.blob_size(0) + aosoa.blob_size(0))
    torch.cuda.synchronize()
    res = {}
    for name, items in (("soa_to_aosoa32", fwd), ("aosoa32_to_soa", back)):
        bt = L.Batch(items)
        med, mn = _timed(torch, stream, lambda: bt.launch(stream), args.steps)
        naive, _ = _timed(torch, stream, lambda: [L.copy_naive(*it, stream=stream) for it in items], 3)
        lone, _ = _timed(torch, stream, lambda: [L.copy(*it, stream=stream) for it in items], 3)
        res[name] = {"batched_ms": round(med, 4), "batched_gbs": round(total / (med * 1e-3) / 1e9, 1),
                     "naive_per_frame_gbs": round(total / (naive * 1e-3) / 1e9, 1),
                     "llama_copy_per_frame_gbs": round(total / (lone * 1e-3) / 1e9, 1),
                     "batched_vs_naive": round(naive / med, 2), "batched_vs_per_frame_copy": round(lone / med, 2)}
        bt.close()
    gbs = res["soa_to_aosoa32"]["batched_gbs"]
    return {"metric": METRIC, "value": gbs, "unit": "GB/s", "n_gpus": 1, "steps": args.steps, "warmup": 1,
            "ms_per_step": res["soa_to_aosoa32"]["batched_ms"], "higher_is_better": True, "scaling": "weak",
            "vs_baseline": None, "dtype": "u32", "data": "synthetic",
            "config": {"workload": "particle-in-cell frames: 4,096 frames of 256 particle records (7xf32), "
                                   "single-blob SoA <-> AoSoA32, one hipGraph-captured batch launch per direction",
                       "bytes_per_step": total, "frames": frames, "records_per_frame": per,
                       "cache": "58.7 MB per launch: mostly resident in the 256 MB Infinity Cache"},
            "hbm_peak_frac": round(gbs / HBM_PEAK_GBS, 4), "extras": res, "device": dev.name}


def bench_leaves(L, torch, args, dev, stream):
    """Copies between records that differ (sec. 3.9): the particle with and
    without its mass, 2^26 records, three layout pairs each way.  Into the
    record without mass the mass is dropped; into the record with mass the
    mass keeps its bytes.  Bytes are the values moved (read + written)."""
    n = 1 << 26
    no_mass = [["f32", "f32", "f32"], ["f32", "f32", "f32"]]
    r7, r6 = L.Record(W.PARTICLE), L.Record(no_mass)
    lay = [("aos_packed", 0), ("soa_multi", 0), ("aosoa", 32)]
    m7 = {l: L.Mapping(r7, l[0], [n], l[1]) for l in lay}
    m6 = {l: L.Mapping(r6, l[0], [n], l[1]) for l in lay}
    g = torch.Generator(device="cuda")
    g.manual_seed(W.BASE_SEED + 7)
    b7 = {l: [torch.randint(0, 256, (s,), dtype=torch.uint8, device="cuda", generator=g) for s in m.blob_sizes()]
          for l, m in m7.items()}
    b6 = {l: [torch.randint(0, 256, (s,), dtype=torch.uint8, device="cuda", generator=g) for s in m.blob_sizes()]
          for l, m in m6.items()}
    drop, keep = list(range(6)), list(range(6)) + [None]
    cases = [(f"{_name(a)}->{_name(b)}-without-mass", m7[a], b7[a], m6[b], b6[b], drop)
             for a, b in ((lay[0], lay[1]), (lay[1], lay[2]), (lay[2], lay[0]))]
    cases += [(f"{_name(a)}-without-mass->{_name(b)}", m6[a], b6[a], m7[b], b7[b], keep)
              for a, b in ((lay[1], lay[0]), (lay[0], lay[2]), (lay[2], lay[1]))]
    moved = 2 * n * 24  # six 4-byte leaves read and written per record
    torch.cuda.synchronize()
    per, total_ms = {}, 0.0
    for name, ms, sb, md, db, lv in cases:
        med, mn = _timed(torch, stream, lambda: L.copy_leaves(ms, sb, md, db, lv, stream=stream), args.steps)
        per[name] = {"ms_median": round(med, 4), "gbs": round(moved / (med * 1e-3) / 1e9, 1)}
        total_ms += med
    value = round(moved * len(cases) / (total_ms * 1e-3) / 1e9, 1)
    cpu = None
    if not args.no_cpu_baseline:
        from oracle import oracle as orc
        ns = 1 << 19
        o7, o6 = orc.Record(W.PARTICLE), orc.Record(no_mass)
        t = 0.0
        for k, (a, b, lv, rs, rd) in enumerate([(lay[0], lay[1], drop, o7, o6), (lay[1], lay[0], keep, o6, o7)]):
            ms = orc.Mapping(rs, a[0], [ns], a[1])
            md = orc.Mapping(rd, b[0], [ns], b[1])
            src = [W.random_bytes(x, 70 + k + j) for j, x in enumerate(ms.blob_sizes())]
            dst = md.alloc()
            t0 = time.perf_counter()
            orc.copy_leaves(ms, src, md, dst, lv)
            t += time.perf_counter() - t0
        cpu = {"value": 2 * 2 * ns * 24 / t / 1e9, "unit": "GB/s", "cores": 1, "kind": "oracle",
               "sample": f"2 of the 6 pairs (one each way) at {ns} records ({t:.1f} s, single thread)"}
    return {"metric": METRIC, "value": value, "unit": "GB/s", "n_gpus": 1, "steps": args.steps, "warmup": 1,
            "ms_per_step": round(total_ms, 3), "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
            "dtype": "u32", "data": "synthetic",
            "config": {"workload": "particle 7xf32 and the particle without mass (6xf32), 2^26 records, "
                                   "copies between the two records over packed AoS, SoA multi-blob and AoSoA32, "
                                   "3 pairs each way", "records": n, "pairs": len(cases),
                       "bytes_per_step": moved * len(cases), "parallelism": "single GPU"},
            "roofline": {"bound": "hbm", "achieved": value, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                         "frac": round(value / HBM_PEAK_GBS, 4), "traffic": None,
                         "kernel": "llama_copy_leaves (tile, stream or naive kernel)"},
            "cpu_baseline": cpu, "hbm_peak_frac": round(value / HBM_PEAK_GBS, 4), "extras": per,
            "device": dev.name}


def _serve_setup(L, torch, count, warm=200):
    """The serving trace: warm + count requests whose blobs lie in one device
    arena used as a ring (132 GB), and the autotuned record/pair classes."""
    budget = 64 * 10**9
    trace = W.poisson_trace(W.BASE_SEED + 5, 1000.0, warm + count)
    S = {"particle": 28, "mixed": 49}
    arena_bytes = 2 * budget + 4 * 10**9
    arena = torch.empty(arena_bytes, dtype=torch.uint8, device="cuda")
    arena.random_(0, 255)
    cache, reqs, off, lap = {}, [], 0, 0
    for r in trace:
        n = max(1, int(r["payload"] // S[r["record"]]))
        ms, md = _layout_maps(L, r["record"], n, r["src"], r["dst"], cache)
        need = sum(ms.blob_sizes()) + sum(md.blob_sizes()) + 256 * (ms.blob_count + md.blob_count)
        if off + need > arena_bytes:
            off, lap = 0, lap + 1
        blobs, o = [], off
        for s in ms.blob_sizes() + md.blob_sizes():
            blobs.append((arena.data_ptr() + o, s))
            o += (s + 255) // 256 * 256
        sb, db = blobs[:ms.blob_count], blobs[ms.blob_count:]
        # the request's C structures are built here, outside the replay: the
        # client then submits at several times the offered rate
        reqs.append({"ms": ms, "md": md, "sb": sb, "db": db, "lo": off, "hi": o, "lap": lap,
                     "bytes": sum(ms.blob_sizes()) + sum(md.blob_sizes()), "c": L.Server.prepare(ms, sb, md, db)})
        off = o
    torch.cuda.synchronize()
    log(f"serve: {len(reqs)} requests, {sum(r['bytes'] for r in reqs) / 1e9:.0f} GB in total")
    _tune_classes(L, torch, {(r["record"], r["src"], r["dst"]) for r in trace}, torch.cuda.current_stream())

    return {"reqs": reqs, "trace": trace, "warm": warm, "budget": budget, "arena": arena}


def _serve_run(L, setup, policy, rate, **server_options):
    """Replays the trace against a new server at `rate` requests per second."""
    import time as _t
    reqs, trace, warm, budget = setup["reqs"], setup["trace"], setup["warm"], setup["budget"]
    srv = L.Server(budget, policy=policy, **server_options)
    # the server's streams take their first launches before the clock starts
    # (a new stream's first launch can stall for milliseconds, and a backlog
    # that early outlasts a short trace at a high load)
    for t in [srv.submit_prepared(r["c"]) for r in reqs[:16]]:
        srv.wait(t)
    srv.reset_stats()
    tickets, done = [], {}
    t0 = _t.perf_counter()
    base = trace[0]["t"]
    # arena regions in allocation order: the ring reuses the oldest first;
    # a region of the previous lap is retired when the new one overlaps
    # it, anything older at once
    users = collections.deque()
    for k, r in enumerate(reqs):
        due = t0 + (trace[k]["t"] - base) * (1000.0 / rate)
        while _t.perf_counter() < due:
            pass
        while users and (users[0][3] < r["lap"] - 1 or (users[0][1] < r["hi"] and r["lo"] < users[0][2])):
            j = users.popleft()[0]
            if j not in done:
                done[j] = srv.wait(tickets[j])
        tickets.append(srv.submit_prepared(r["c"]))
        users.append((k, r["lo"], r["hi"], r["lap"]))
        if k == warm - 1:
            t_meas = _t.perf_counter()
    for j, t in enumerate(tickets):
        if j not in done:
            done[j] = srv.wait(t)
    t_end = _t.perf_counter()
    st = srv.stats()
    srv.close()
    lat = sorted(done[j][1] for j in range(warm, len(reqs)))
    measured = sum(reqs[j]["bytes"] for j in range(warm, len(reqs)))
    return {"gbs": round(measured / (t_end - t_meas) / 1e9, 1),
            "p50_ms": round(1e3 * lat[len(lat) // 2], 3),
            "p99_ms": round(1e3 * lat[min(len(lat) - 1, int(0.99 * len(lat)))], 3),
            "launches": st["launches"], "mean_batch": round(st["mean_batch"], 2),
            "max_inflight_gb": round(st["max_inflight_bytes"] / 1e9, 2),
            "failed": st["failed"]}


def bench_serve(L, torch, args, dev):
    """Poisson requests replayed against the server with three policies:
    continuous batching, one naive kernel per request, one llama_copy per
    request.  Arrival rate: rho (0.5 and 0.8) times the service capacity, the
    GB/s of the batched server at saturation (every request submitted at
    once), measured first in the same process.  (Taken from the batching
    workload's single launch instead, the offered load followed a 3-launch
    median that varied by 5% from run to run, and at 80% the latency with
    it: p50 0.4 or 3 ms on one box.)"""
    import time as _t
    stream = torch.cuda.current_stream()
    items, total, _ = _batch_items(L, torch, stream)
    b = L.Batch(items)
    med, _ = _timed(torch, stream, lambda: b.launch(stream), 3)
    batch_gbs = total / (med * 1e-3) / 1e9
    b.close()
    del items, b
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    log(f"serve: batching workload runs at {batch_gbs:.1f} GB/s")
    setup = _serve_setup(L, torch, args.requests)
    reqs, warm, count = setup["reqs"], setup["warm"], args.requests

    def run(policy, rate):
        return _serve_run(L, setup, policy, rate)

    # saturation: everything submitted at once measures the server's capacity
    capacity = run(0, 1e9)
    total_bytes = sum(r["bytes"] for r in reqs[warm:])
    mean_bytes = total_bytes / count
    log(f"serve: batched server at saturation {capacity['gbs']} GB/s")
    capacity_per_request = run(2, 1e9)
    log(f"serve: per-request llama_copy at saturation {capacity_per_request['gbs']} GB/s")
    by_rho = {}
    policies = [("batched", 0), ("naive", 1), ("per_request", 2)]
    service_gbs = capacity["gbs"]
    for n_rho, rho in enumerate(sorted({0.5, args.rho})):
        rate = rho * service_gbs * 1e9 / mean_bytes
        log(f"serve: offered load rho={rho} -> {rate:.0f} requests/s")
        # the policies in rotated order from one load to the next, so that no
        # policy always runs first (or right after the naive one's backlog)
        order = policies[n_rho % 3:] + policies[:n_rho % 3]
        res = {name: run(pol, rate) for name, pol in order}
        by_rho[rho] = {"rate_per_s": round(rate, 1), "offered_gbs": round(rho * service_gbs, 1),
                       "order": [name for name, _ in order], **res}
    out = by_rho[args.rho]
    return {"metric": METRIC, "value": out["batched"]["gbs"], "unit": "GB/s", "n_gpus": 1, "steps": count,
            "warmup": warm, "ms_per_step": None, "higher_is_better": True, "scaling": "weak",
            "vs_baseline": None, "dtype": "u32", "data": "synthetic",
            "config": {"workload": "serving: Poisson arrivals, payload log-uniform 64 KB..1 GB, particle or mixed "
                                   "record, random ordered layout pair of 42, HBM admission budget 64 GB",
                       "rho": args.rho, "rate_per_s": out["rate_per_s"], "requests": count, "warmup_requests": warm,
                       "mean_request_bytes": round(mean_bytes), "service_capacity_gbs": service_gbs,
                       "batching_workload_gbs": round(batch_gbs, 1)},
            "p50_ms": out["batched"]["p50_ms"], "p99_ms": out["batched"]["p99_ms"],
            "extras": {"server_saturation_gbs": capacity["gbs"], "saturation_batched": capacity,
                       "saturation_per_request": capacity_per_request,
                       **{f"rho_{rho}": v for rho, v in by_rho.items()}},
            "device": dev.name}


def _time_calls(torch, stream, calls, steps, warmup):
    """Times named calls (name, fn, bytes) `steps` times each with HIP events
    around every call; returns the whole-step milliseconds and per-call
    medians and means."""
    for _ in range(warmup):
        for _, fn, _ in calls:
            fn()
    torch.cuda.synchronize()
    ev = {name: [] for name, _, _ in calls}
    start, end = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    start.record(stream)
    for _ in range(steps):
        for name, fn, _ in calls:
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            fn()
            e1.record(stream)
            ev[name].append((e0, e1))
    end.record(stream)
    torch.cuda.synchronize()
    per = {}
    for name, _, nb in calls:
        ms = [e0.elapsed_time(e1) for e0, e1 in ev[name]]
        per[name] = {"bytes": nb, "ms_median": statistics.median(ms), "ms_mean": statistics.mean(ms),
                     "gbs_median": nb / (statistics.median(ms) * 1e-3) / 1e9}
    return start.elapsed_time(end), per


def _box_line(L, torch, args, dev, stream, workload, calls, naive_calls, record, dtype, extra_config):
    total_ms, per = _time_calls(torch, stream, calls, args.steps, args.warmup)
    step_bytes = sum(nb for _, _, nb in calls)
    value = step_bytes * args.steps / (total_ms * 1e-3) / 1e9
    box_ms = statistics.mean(v["ms_mean"] for v in per.values())
    box_bytes = statistics.mean(v["bytes"] for v in per.values())
    achieved = box_bytes / (box_ms * 1e-3) / 1e9
    extras = {"pairs": {k: round(v["gbs_median"], 1) for k, v in per.items()}}
    if naive_calls and not args.no_naive:
        log(f"{args.workload}: timing the element-wise box baseline")
        _, nper = _time_calls(torch, stream, naive_calls, 2, 1)
        nv = statistics.median(v["gbs_median"] for v in nper.values())
        extras["naive_box_kernel_gbs"] = round(nv, 1)
        extras["box_vs_naive_speedup"] = round(statistics.median(v["gbs_median"] for v in per.values()) / nv, 2)
    return {"metric": METRIC, "value": round(value, 1), "unit": "GB/s", "n_gpus": 1, "steps": args.steps,
            "warmup": args.warmup, "ms_per_step": round(total_ms / args.steps, 3), "higher_is_better": True,
            "scaling": "weak", "vs_baseline": None, "dtype": dtype, "data": "synthetic",
            "config": {"workload": workload, "pairs": len(calls), "bytes_per_step": step_bytes,
                       "parallelism": "single GPU", **extra_config},
            "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                         "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None, "kernel": "box_kernel",
                         "bytes_per_launch": int(box_bytes), "launch_ms_mean": round(box_ms, 4),
                         "launches": len(calls) * args.steps},
            "cpu_baseline": None, "hbm_peak_frac": round(value / HBM_PEAK_GBS, 4), "extras": extras,
            "device": dev.name}


def bench_box(L, torch, args, dev, stream):
    """Sub-box copies (sec. 3.2 VirtualView): the 256^3 interior of a
    lattice-Boltzmann grid with a one-cell halo (258^3 cells) into a 256^3
    grid of another layout, 6 ordered pairs."""
    rec = W.LBM
    rg = L.Record(rec)
    S, R = rg.info()[1], rg.info()[2]
    src_ext, dst_ext, box = [258] * 3, [256] * 3, [256] * 3
    layouts = [("aos_aligned", 0), ("soa_multi", 0), ("aosoa", 32)]
    pairs = [(a, b) for a in layouts for b in layouts if a != b]
    srcs, dsts = {}, {}
    for l in layouts:
        ms = L.Mapping(rg, l[0], src_ext, l[1])
        srcs[l] = (ms, [torch.empty(s, dtype=torch.uint8, device="cuda").random_(0, 255) for s in ms.blob_sizes()])
        md = L.Mapping(rg, l[0], dst_ext, l[1])
        dsts[l] = (md, md.alloc(fill=0))
    torch.cuda.synchronize()
    nbox = 256 ** 3

    def rb(l):
        return R if l == ("aos_aligned", 0) else S
    calls, naive = [], []
    for a, b in pairs:
        (ms, sb), (md, db) = srcs[a], dsts[b]
        nb = nbox * (rb(a) + rb(b))
        name = f"{_name(a)}->{_name(b)}"
        calls.append((name, lambda ms=ms, sb=sb, md=md, db=db: L.copy_box(ms, sb, [1, 1, 1], md, db, [0, 0, 0], box,
                                                                         stream=stream), nb))
        naive.append((name, lambda ms=ms, sb=sb, md=md, db=db: L.copy_box(ms, sb, [1, 1, 1], md, db, [0, 0, 0], box,
                                                                         stream=stream, path="naive"), nb))
    log(f"box: timing {len(calls)} box copies of {nbox} cells")
    return _box_line(L, torch, args, dev, stream,
                     "lattice-Boltzmann cell {f64[19], u32}: the 256^3 interior of a 258^3 grid (one-cell halo) "
                     "into a 256^3 grid, 6 ordered pairs of aligned AoS, SoA multi-blob, AoSoA32 (box copies)",
                     calls, naive, rec, "u64", {"records": nbox, "source_extents": src_ext, "box": box})


def bench_linearize(L, torch, args, dev, stream):
    """Whole copies between views whose linearizers differ (sec. 3.7): the
    particle record on an 8192 x 8192 grid (2^26 records), 6 ordered pairs
    between row-major, column-major and Morton views of different layouts."""
    rg = L.Record(W.PARTICLE)
    ext = [8192, 8192]
    A, As, M, Ss, Q = ("aos_packed", 0), ("aos_aligned", 0), ("soa_multi", 0), ("soa_single", 0), ("aosoa", 32)
    pairs = [((A, "row"), (M, "col")), ((M, "col"), (A, "row")), ((Ss, "row"), (Q, "morton")),
             ((Q, "morton"), (A, "row")), ((Q, "row"), (Q, "col")), ((M, "morton"), (As, "col"))]
    views = {}
    for v in {p for pr in pairs for p in pr}:
        m = L.Mapping(rg, v[0][0], ext, v[0][1], linearizer=v[1])
        views[v] = (m, [torch.empty(s, dtype=torch.uint8, device="cuda").random_(0, 255) for s in m.blob_sizes()])
    torch.cuda.synchronize()
    calls, naive = [], []
    for a, b in pairs:
        (ms, sb), (md, db) = views[a], views[b]
        nb = sum(ms.blob_sizes()) + sum(md.blob_sizes())
        name = f"{_name(a[0])}/{a[1]}->{_name(b[0])}/{b[1]}"
        calls.append((name, lambda ms=ms, sb=sb, md=md, db=db: L.copy(ms, sb, md, db, stream=stream), nb))
        naive.append((name, lambda ms=ms, sb=sb, md=md, db=db: L.copy(ms, sb, md, db, stream=stream, path="naive"),
                      nb))
    log(f"linearize: timing {len(calls)} copies between linearizers")
    return _box_line(L, torch, args, dev, stream,
                     "n-body particle 7xf32 on an 8192 x 8192 grid (2^26 records), 6 ordered pairs between "
                     "row-major, column-major and Morton views of packed/aligned AoS, SoA and AoSoA32",
                     calls, naive, W.PARTICLE, "u32", {"records": 1 << 26, "extents": ext})


def bench_transfer(L, torch, args, dev, stream):
    """Host <-> device copies with a layout change (sec. 3.9): 2^26 particles
    from pinned host memory as packed AoS into device SoA multi-blob, and
    back from device AoSoA32 into host packed AoS, chunked with transfers and
    layout changes overlapped, against the same transfer done in one piece
    (one memcpy of the whole view, then the layout change) and against raw
    host <-> device memcpy of the same bytes."""
    import ctypes
    rg = L.Record(W.PARTICLE)
    n = 1 << 26
    A, M, Q = ("aos_packed", 0), ("soa_multi", 0), ("aosoa", 32)
    ha = L.Mapping(rg, A[0], [n])
    dm, dq = L.Mapping(rg, M[0], [n]), L.Mapping(rg, Q[0], [n], Q[1])
    host = torch.empty(ha.blob_size(0), dtype=torch.uint8, pin_memory=True)
    host.random_(0, 255)
    back = torch.empty_like(host, pin_memory=True)
    dmb, dqb = dm.alloc(fill=0), dq.alloc(fill=0)
    staging = torch.empty(ha.blob_size(0), dtype=torch.uint8, device="cuda")
    torch.cuda.synchronize()
    hip = ctypes.CDLL("libamdhip64.so")
    hip.hipMemcpyAsync.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int, ctypes.c_void_p]
    sp = ctypes.c_void_p(stream.cuda_stream)
    nb = host.numel()
    chunk = 64 << 20

    def h2d_chunked():
        L.copy_transfer(ha, [host], dm, dmb, src_on_host=True, chunk_bytes=chunk, stream=stream)

    def h2d_whole():
        hip.hipMemcpyAsync(ctypes.c_void_p(staging.data_ptr()), ctypes.c_void_p(host.data_ptr()), nb, 1, sp)
        L.copy(ha, [staging], dm, dmb, stream=stream)

    def h2d_raw():
        hip.hipMemcpyAsync(ctypes.c_void_p(staging.data_ptr()), ctypes.c_void_p(host.data_ptr()), nb, 1, sp)

    def d2h_chunked():
        L.copy_transfer(dq, dqb, ha, [back], src_on_host=False, chunk_bytes=chunk, stream=stream)

    def d2h_whole():
        L.copy(dq, dqb, ha, [staging], stream=stream)
        hip.hipMemcpyAsync(ctypes.c_void_p(back.data_ptr()), ctypes.c_void_p(staging.data_ptr()), nb, 2, sp)

    def d2h_raw():
        hip.hipMemcpyAsync(ctypes.c_void_p(back.data_ptr()), ctypes.c_void_p(staging.data_ptr()), nb, 2, sp)

    calls = [("h2d_chunked", h2d_chunked, nb), ("d2h_chunked", d2h_chunked, nb)]
    refs = [("h2d_whole", h2d_whole, nb), ("h2d_memcpy", h2d_raw, nb), ("d2h_whole", d2h_whole, nb),
            ("d2h_memcpy", d2h_raw, nb)]
    log("transfer: timing chunked host <-> device copies")
    total_ms, per = _time_calls(torch, stream, calls, args.steps, args.warmup)
    _, rper = _time_calls(torch, stream, refs, max(2, args.steps // 2), 1)
    value = sum(v["bytes"] for v in per.values()) * args.steps / (total_ms * 1e-3) / 1e9
    ex = {k: round(v["gbs_median"], 2) for k, v in {**per, **rper}.items()}
    ex["h2d_vs_memcpy"] = round(per["h2d_chunked"]["gbs_median"] / rper["h2d_memcpy"]["gbs_median"], 3)
    ex["d2h_vs_memcpy"] = round(per["d2h_chunked"]["gbs_median"] / rper["d2h_memcpy"]["gbs_median"], 3)
    ex["h2d_vs_whole"] = round(per["h2d_chunked"]["gbs_median"] / rper["h2d_whole"]["gbs_median"], 3)
    ex["d2h_vs_whole"] = round(per["d2h_chunked"]["gbs_median"] / rper["d2h_whole"]["gbs_median"], 3)
    return {"metric": "host<->device layout-changing copy GB/s (bytes crossing the link)", "value": round(value, 2),
            "unit": "GB/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
            "ms_per_step": round(total_ms / args.steps, 3), "higher_is_better": True, "scaling": "weak",
            "vs_baseline": None, "dtype": "u32", "data": "synthetic",
            "config": {"workload": "n-body particle 7xf32, 2^26 records (1.879 GB): pinned host packed AoS -> "
                                   "device SoA multi-blob, and device AoSoA32 -> pinned host packed AoS, 64 MiB "
                                   "chunks, transfers and layout changes overlapped", "records": n,
                       "chunk_bytes": chunk, "parallelism": "single GPU"},
            "roofline": {"bound": "host link", "achieved": round(value, 2),
                         "peak": round((rper["h2d_memcpy"]["gbs_median"] + rper["d2h_memcpy"]["gbs_median"]) / 2, 2),
                         "unit": "GB/s", "frac": None, "traffic": None, "kernel": "hipMemcpyAsync + tile_kernel"},
            "cpu_baseline": None, "extras": ex, "device": dev.name}


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="particle",
                    choices=["particle", "pairs", "lbm", "split", "leaves", "batch", "serve", "pic", "box",
                             "linearize", "transfer"])
    ap.add_argument("--record", default="mixed", choices=sorted(W.RECORDS), help="pairs: the record")
    ap.add_argument("--records", type=int, default=1 << 23, help="pairs: records per layout")
    ap.add_argument("--requests", type=int, default=20000, help="serve: measured requests (after 200 warm-up)")
    ap.add_argument("--rho", type=float, default=0.8, help="serve: offered load as a fraction of batched GB/s")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-naive", action="store_true")
    ap.add_argument("--no-batch-autotune", action="store_true", help="batch: keep the default plan")
    ap.add_argument("--no-batch", action="store_true", help="particle: leave out the 1,000-array batch extras")
    ap.add_argument("--tune-cache", default=None, help="tuning-cache file: read before class tuning, written after")
    ap.add_argument("--details", default=None, help="write per-pair results to this JSON file")
    args = ap.parse_args()
    global TUNE_CACHE
    TUNE_CACHE = args.tune_cache

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU: the layout copy shards by record range with no exchange between "
              "GPUs, and this build runs and reports the single-GPU kernel only (--gpus 1).", file=sys.stderr)
        sys.exit(2)

    import torch
    # the OpenMP settings above bind the main thread to one core once torch
    # starts its OpenMP runtime; every thread started later (the HIP
    # runtime's, a server's engine thread) would inherit that one core (the
    # serving replay at 80% load: p50 2.1 instead of 0.27 ms, p99 7-9
    # instead of 1.9-2.1 ms)
    os.sched_setaffinity(0, START_CPUS)
    from paper_2106_04284_amd import llama as L
    L.lib()  # fails loudly when the HIP library has not been built
    if not torch.cuda.is_available():
        print("no GPU visible", file=sys.stderr)
        sys.exit(1)
    dev = torch.cuda.get_device_properties(0)
    stream = torch.cuda.current_stream()

    if args.workload == "batch":
        print(json.dumps(bench_batch(L, torch, args, dev, stream)), flush=True)
        return
    if args.workload == "serve":
        print(json.dumps(bench_serve(L, torch, args, dev)), flush=True)
        return
    if args.workload == "pic":
        print(json.dumps(bench_pic(L, torch, args, dev, stream)), flush=True)
        return
    if args.workload == "leaves":
        print(json.dumps(bench_leaves(L, torch, args, dev, stream)), flush=True)
        return
    if args.workload in ("box", "linearize", "transfer"):
        fn = {"box": bench_box, "linearize": bench_linearize, "transfer": bench_transfer}[args.workload]
        line = fn(L, torch, args, dev, stream)
        if line["roofline"]["frac"] is None and line["roofline"]["peak"]:
            line["roofline"]["frac"] = round(line["roofline"]["achieved"] / line["roofline"]["peak"], 4)
        print(json.dumps(line), flush=True)
        return

    if args.workload == "particle":
        n = 1 << 26
        record, extents = W.PARTICLE, [n]
        layouts = W.LAYOUTS
        pairs = [(a, b) for a in layouts for b in layouts if a != b]
        values = W.raw_u32_values(7, n, W.BASE_SEED + 2)
        workload = "n-body particle {pos{x,y,z},vel{x,y,z},mass} 7xf32, 2^26 records (1.879 GB per layout), " \
                   "42 ordered pairs of packed AoS, aligned AoS, SoA single-blob, SoA multi-blob, AoSoA8/32/64"
        dtype = "u32"
        cpu_n = 1 << 19
        cpu_full = n
    elif args.workload == "pairs":
        # every ordered pair of the seven layouts for one record at a given
        # size (per-pair figures with --details)
        n = args.records
        record, extents = W.RECORDS[args.record], [n]
        layouts = W.LAYOUTS
        pairs = [(a, b) for a in layouts for b in layouts if a != b]
        values = W.typed_random_values(W.leaf_types(record), n, W.BASE_SEED + 7)
        workload = f"{args.record} record, {n} records, 42 ordered pairs of packed AoS, aligned AoS, SoA " \
                   "single-blob, SoA multi-blob, AoSoA8/32/64"
        dtype = "u8"
        cpu_n = min(n, 1 << 17)
        cpu_full = n
    elif args.workload == "split":
        # Split mappings (sec. 3.7) of the particle: positions as AoSoA32 with
        # velocities and mass as multi-blob SoA; velocities as multi-blob SoA
        # with positions and mass as aligned AoS
        n = 1 << 26
        record, extents = W.PARTICLE, [n]
        A, M, Q32 = ("aos_packed", 0), ("soa_multi", 0), ("aosoa", 32)
        S1 = ("split", (0, 3, Q32, M))
        S2 = ("split", (3, 3, M, ("aos_aligned", 0)))
        layouts = [A, M, Q32, S1, S2]
        pairs = [(A, S1), (S1, A), (M, S2), (S2, Q32), (S1, S2), (S2, S1)]
        values = W.raw_u32_values(7, n, W.BASE_SEED + 4)
        workload = "n-body particle 7xf32, 2^26 records, 6 ordered pairs with a Split side: " \
                   "split[pos](AoSoA32, SoA multi-blob) and split[vel](SoA multi-blob, aligned AoS) against " \
                   "packed AoS, SoA multi-blob, AoSoA32 and each other"
        dtype = "u32"
        cpu_n = 1 << 19
        cpu_full = n
    else:
        record, extents = W.LBM, [128, 128, 128]
        layouts = [("aos_aligned", 0), ("soa_multi", 0), ("aosoa", 32)]
        pairs = [(a, b) for a in layouts for b in layouts if a != b]
        values = W.lbm_values(128 ** 3, W.BASE_SEED + 3)
        workload = "lattice-Boltzmann cell {f64[19], u32} on a 128^3 grid, row-major extents, " \
                   "6 ordered pairs of aligned AoS, SoA multi-blob, AoSoA32"
        dtype = "u64"
        cpu_n = 1 << 17
        cpu_full = 128 ** 3
    # the 128^3 lattice (663 MB per copy) would partly stay in the 256 MB
    # Infinity Cache between copies: read 1 GiB before each timed copy
    cold = args.workload == "lbm"

    log(f"inputs generated ({args.workload}); filling {len(layouts)} layouts on {dev.name}")
    maps, blobs = setup_layouts(L, torch, record, extents, layouts, values)
    del values
    log(f"timing {args.steps} steps of {len(pairs)} copies after {args.warmup} warm-up steps")
    flush = torch.ones(1 << 27, dtype=torch.int64, device="cuda") if cold else None
    wall, total_ms, per_pair, plans = time_pairs(L, torch, maps, blobs, pairs, args.steps, args.warmup, stream,
                                                 flush=flush)
    del flush
    log(f"timed: {total_ms / args.steps:.2f} ms per step")
    step_bytes = sum(v["bytes"] for v in per_pair.values())
    value = step_bytes * args.steps / (total_ms * 1e-3) / 1e9

    tile = [p for p in pairs if per_pair[p]["path"] == "tile"] or pairs
    kernel = "tile_kernel" if per_pair[tile[0]]["path"] == "tile" else "part copies (tile, stream, naive kernels)"
    tile_ms = statistics.mean(per_pair[p]["ms_mean"] for p in tile)
    tile_bytes = statistics.mean(per_pair[p]["bytes"] for p in tile)
    achieved = tile_bytes / (tile_ms * 1e-3) / 1e9
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4),
                "traffic": measured_traffic() if args.workload == "particle" else None,
                "kernel": kernel, "bytes_per_launch": int(tile_bytes),
                "launch_ms_mean": round(tile_ms, 4), "launches": len(tile) * args.steps}

    extras = {}
    # payload: 2 N S per copy (values only, no padding)
    rec_bytes = L.Record(record).info()[1]
    payload = 2 * int(np.prod(extents)) * rec_bytes * len(pairs) * args.steps
    extras["payload_gbs"] = round(payload / (total_ms * 1e-3) / 1e9, 1)
    nbytes_layout = sum(maps[layouts[0]].blob_sizes())
    d2d = d2d_reference(torch, nbytes_layout, stream)
    extras["d2d_memcpy_gbs"] = round(d2d, 1) if d2d else None
    stream_pairs = [p for p in pairs if per_pair[p]["path"] == "stream"]
    if stream_pairs:
        extras["stream_kernel_gbs"] = round(statistics.median(per_pair[p]["gbs_median"] for p in stream_pairs), 1)
    extras["tile_kernel_gbs_min_pair"] = round(min(per_pair[p]["gbs_median"] for p in tile), 1)
    extras["tile_kernel_gbs_max_pair"] = round(max(per_pair[p]["gbs_median"] for p in tile), 1)
    if not args.no_naive:
        log("timing the naive element-wise kernel on a subset of pairs")
        naive_pairs = tile[:: max(1, len(tile) // 6)]
        nv = naive_reference(L, torch, maps, blobs, naive_pairs, stream)
        ours = statistics.median(per_pair[p]["gbs_median"] for p in naive_pairs)
        extras["naive_kernel_gbs"] = round(statistics.median(nv.values()), 1)
        extras["tile_vs_naive_speedup"] = round(ours / statistics.median(nv.values()), 2)

    if args.workload == "particle" and not args.no_batch:
        # the batching workload (1,000 arrays, one graph-captured launch)
        # against per-array naive and llama_copy launches, on the same GPU
        del blobs
        torch.cuda.synchronize()
        torch.cuda.empty_cache()
        bm = batch_measure(L, torch, args, stream, naive=not args.no_naive)
        extras["batch_1000_arrays"] = {"workload": BATCH_WORKLOAD, "bytes_per_launch": bm["bytes"], **batch_extras(bm)}
        log(f"batch: {bm['gbs']:.1f} GB/s")

    cpu = None
    if not args.no_cpu_baseline:
        log("timing the CPU oracle on a bounded sample")
        cpu = cpu_baseline(record, layouts, pairs, cpu_n, cpu_full)

    line = {
        "metric": METRIC, "value": round(value, 1), "unit": "GB/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(total_ms / args.steps, 3), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": dtype, "data": "synthetic",
        "config": {"workload": workload, "records": int(np.prod(extents)), "pairs": len(pairs),
                   "bytes_per_step": step_bytes, "parallelism": "single GPU",
                   "cache": "cold: 1 GiB read before each timed copy" if cold else "no flush (layouts exceed "
                            "the 256 MB Infinity Cache)"},
        "roofline": roofline, "cpu_baseline": cpu,
        "hbm_peak_frac": round(value / HBM_PEAK_GBS, 4), "extras": extras,
        "device": dev.name, "wall_s": round(wall, 3),
    }
    print(json.dumps(line), flush=True)
    if args.details:
        with open(args.details, "w") as f:
            json.dump({"pairs": {f"{_name(a)}->{_name(b)}": v for (a, b), v in per_pair.items()},
                       "line": line}, f, indent=1)


if __name__ == "__main__":
    main()
