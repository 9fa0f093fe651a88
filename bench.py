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
timed per launch with HIP events on the launch stream), and the CPU oracle
timed on a bounded sample of the same workload.

Other workloads (--workload): lbm (128^3 cells of 19 f64 + u32, aligned AoS
<-> SoA multi-blob <-> AoSoA32).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import statistics
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

from paper_2106_04284_amd import workloads as W  # noqa: E402

METRIC = "layout-copy GB/s (rd+wr) & % HBM peak; batched vs naive per-array; p99 latency"
HBM_PEAK_GBS = 8000.0
PROFILE_COUNTERS = os.path.join(ROOT, "profiles", "tile_kernel_particle_2e26_counters.json")


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def _name(layout):
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

def cpu_baseline(record, layouts, pairs, n_sample, budget_s=20.0):
    from oracle import oracle as orc
    ro = orc.Record(record)
    maps = {l: orc.Mapping(ro, l[0], [n_sample], l[1]) for l in layouts}
    srcs = {l: [W.random_bytes(s, 99 + k) for k, s in enumerate(maps[l].blob_sizes())] for l in layouts}
    dsts = {l: maps[l].alloc() for l in layouts}
    nbytes, elapsed, done = 0, 0.0, 0
    for a, b in pairs:
        t0 = time.perf_counter()
        orc.copy(maps[a], srcs[a], maps[b], dsts[b])
        elapsed += time.perf_counter() - t0
        nbytes += sum(maps[a].blob_sizes()) + sum(maps[b].blob_sizes())
        done += 1
        if elapsed > budget_s:
            break
    return {"value": nbytes / elapsed / 1e9, "unit": "GB/s", "cores": 1, "kind": "oracle",
            "sample": f"{done} of the {len(pairs)} layout pairs at {n_sample} records each "
                      f"({nbytes / 1e9:.3f} GB read+written, {elapsed:.1f} s, single thread)"}


# --------------------------------------------------------------------------
# GPU workloads
# --------------------------------------------------------------------------

def setup_layouts(L, torch, record, extents, layouts, values):
    """Uploads the per-leaf values as multi-blob SoA and fills every other
    layout from it on the GPU (untimed)."""
    rg = L.Record(record)
    maps = {l: L.Mapping(rg, l[0], extents, l[1]) for l in layouts}
    mb_layout = ("soa_multi", 0)
    blobs = {mb_layout: [torch.from_numpy(np.ascontiguousarray(v).view(np.uint8).reshape(-1)).cuda()
                         for v in values]}
    for l in layouts:
        if l != mb_layout:
            blobs[l] = maps[l].alloc()
            L.copy(maps[mb_layout], blobs[mb_layout], maps[l], blobs[l])
    torch.cuda.synchronize()
    return maps, blobs


def time_pairs(L, torch, maps, blobs, pairs, steps, warmup, stream):
    plans = {p: L.plan(maps[p[0]], maps[p[1]]) for p in pairs}
    for _ in range(warmup):
        for a, b in pairs:
            L.copy(maps[a], blobs[a], maps[b], blobs[b], stream=stream)
    torch.cuda.synchronize()
    ev = {p: [] for p in pairs}
    t0 = time.perf_counter()
    start = torch.cuda.Event(enable_timing=True)
    end = torch.cuda.Event(enable_timing=True)
    start.record(stream)
    for _ in range(steps):
        for a, b in pairs:
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
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
        nb = plans[p]["read_bytes"] + plans[p]["write_bytes"]
        per_pair[p] = {"path": plans[p]["path"], "bytes": nb, "ms_median": statistics.median(ms),
                       "ms_min": min(ms), "ms_mean": statistics.mean(ms),
                       "gbs_median": nb / (statistics.median(ms) * 1e-3) / 1e9}
    return wall, total_ms, per_pair, plans


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


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="particle", choices=["particle", "lbm"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-naive", action="store_true")
    ap.add_argument("--details", default=None, help="write per-pair results to this JSON file")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU: the layout copy shards by record range with no exchange between "
              "GPUs, and this build runs and reports the single-GPU kernel only (--gpus 1).", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2106_04284_amd import llama as L
    L.lib()  # fails loudly when the HIP library has not been built
    if not torch.cuda.is_available():
        print("no GPU visible", file=sys.stderr)
        sys.exit(1)
    dev = torch.cuda.get_device_properties(0)
    stream = torch.cuda.current_stream()

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
    else:
        record, extents = W.LBM, [128, 128, 128]
        layouts = [("aos_aligned", 0), ("soa_multi", 0), ("aosoa", 32)]
        pairs = [(a, b) for a in layouts for b in layouts if a != b]
        values = W.lbm_values(128 ** 3, W.BASE_SEED + 3)
        workload = "lattice-Boltzmann cell {f64[19], u32} on a 128^3 grid, row-major extents, " \
                   "6 ordered pairs of aligned AoS, SoA multi-blob, AoSoA32"
        dtype = "u64"
        cpu_n = 1 << 17

    log(f"inputs generated ({args.workload}); filling {len(layouts)} layouts on {dev.name}")
    maps, blobs = setup_layouts(L, torch, record, extents, layouts, values)
    del values
    log(f"timing {args.steps} steps of {len(pairs)} copies after {args.warmup} warm-up steps")
    wall, total_ms, per_pair, plans = time_pairs(L, torch, maps, blobs, pairs, args.steps, args.warmup, stream)
    log(f"timed: {total_ms / args.steps:.2f} ms per step")
    step_bytes = sum(v["bytes"] for v in per_pair.values())
    value = step_bytes * args.steps / (total_ms * 1e-3) / 1e9

    tile = [p for p in pairs if per_pair[p]["path"] == "tile"]
    tile_ms = statistics.mean(per_pair[p]["ms_mean"] for p in tile)
    tile_bytes = statistics.mean(per_pair[p]["bytes"] for p in tile)
    achieved = tile_bytes / (tile_ms * 1e-3) / 1e9
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": measured_traffic(),
                "kernel": "tile_kernel", "bytes_per_launch": int(tile_bytes),
                "launch_ms_mean": round(tile_ms, 4), "launches": len(tile) * args.steps}

    extras = {}
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

    cpu = None
    if not args.no_cpu_baseline:
        log("timing the CPU oracle on a bounded sample")
        cpu = cpu_baseline(record, layouts, pairs, cpu_n)

    line = {
        "metric": METRIC, "value": round(value, 1), "unit": "GB/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(total_ms / args.steps, 3), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": dtype, "data": "synthetic",
        "config": {"workload": workload, "records": int(np.prod(extents)), "pairs": len(pairs),
                   "bytes_per_step": step_bytes, "parallelism": "single GPU"},
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
